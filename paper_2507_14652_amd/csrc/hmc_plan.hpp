// Plan structures shared by the host engine and the gfx950 kernels.
//
// Layout decisions (per chain, in device memory):
//  * weights in the product precision T, each layer twice: W_l [out_p][in_p]
//    for the forward product and W_l^T [in_p][out_p] for the adjoint product,
//    both row-major and zero-padded to the width padding of the precision;
//  * biases (and the DeepONet b0) in the accumulator precision A;
//  * activations of one row tile live in LDS, one [R][width_p + pad] slab per
//    layer; the adjoint of a layer overwrites the activation slab it no
//    longer needs.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

#define HMC_MAXL 8    // linear layers per tower
#define HMC_NT 512    // threads per workgroup of the tile kernels (8 waves)

struct TowerPlan {
    int nl;                     // linear layers
    int w[HMC_MAXL + 1];        // true widths
    int wp[HMC_MAXL + 1];       // padded widths
    int ls[HMC_MAXL + 1];       // LDS row stride (elements) of activation slab l
    int lo[HMC_MAXL + 1];       // LDS offset (elements) of activation slab l
    long long wo[HMC_MAXL];     // offset of W_l in the per-chain weight buffer
    long long wto[HMC_MAXL];    // offset of W_l^T
    long long bo[HMC_MAXL];     // offset of b_l in the per-chain bias buffer
    long long fo[HMC_MAXL];     // flat parameter index of W_l[0][0]
    int seg0;                   // first layer of this tower in the segment table
    int scr;                    // LDS byte offset of the dense weight-gradient scratch, 4096 bytes per wave
    int dwv[HMC_MAXL];          // dense weight-gradient variant of each layer (DWV_*)
    int rc1;                    // 1: slabs 1 and 3 share one LDS region (towers of 4 or more layers that
                                //   do not fit otherwise); the adjoint pass recomputes a_1 from the
                                //   input before layer 1's weight gradient, when slab 3 is no longer needed
};

// Per-chain mask tables of one tower, staged in LDS by the tile kernels
// that run the adjoint pass (HMC_META_BYTES reserved per workgroup).
struct TileMeta {
    long long o;                // offs[c]: the chain's first entry
    int n;                      // the chain's entry count
    unsigned dmask;             // bit l: dense weight-gradient product for layer l
    int seg[HMC_MAXL + 1];      // chain-local start of each layer's entries (and the end)
    int bseg[HMC_MAXL];         // chain-local start of each layer's bias entries
    int mloff[HMC_MAXL];        // offset (32-bit words) of each dense layer's selection list in ml
};
#define HMC_META_BYTES 128
static_assert(sizeof(TileMeta) <= HMC_META_BYTES, "TileMeta exceeds its LDS reservation");

// Arguments of the tile kernels (forward, loss head, adjoint, masked
// weight-gradient partials).
struct GradArgs {
    TowerPlan ta;               // MLP or branch tower
    TowerPlan tb;               // trunk tower (DeepONet)
    const void* wbuf;           // [C][wstride] T
    long long wstride;
    const void* bbuf;           // [C][bstride] A
    long long bstride;
    const void* xa;             // tower-A input rows [tiles_a * R_a][wp_a0] T
    const void* xb;             // trunk input rows [tiles_b * R_b][wp_b0] T
    const double* target;       // MLP y [N][d_out]; DeepONet v [n_u][n_q]
    int n_rows_a;               // valid rows of tower A (N or n_u)
    int n_rows_b;               // valid rows of the trunk (n_q)
    int d_out;                  // MLP output width
    int tiles_a, tiles_b;
    int tpg;                    // row tiles per workgroup of the MLP gradient kernel, whose
                                // weight-gradient terms it sums into one partial slot
    int overlap;                // adjoint pass: a layer's weight gradient beside its adjoint
                                // product's multiplies (epilogues after a barrier)
    int n_chains;               // chains of this launch: chain0 .. chain0 + n_chains - 1
    int chain0;                 // (gradient kernels; 0 elsewhere)
    const int* active;          // [C]
    const long long* offs;      // [C+1]
    const int* ecode;           // [nnz] (i << 16) | j, j = 0xFFFF for a bias
    const int* seg;             // [C][nseg] chain-local start of each layer's entries
    int nseg;
    const int* bseg;            // [C][nl_total] chain-local start of each layer's bias entries
    const int* dflag;           // [C][nl_total] 1: weight partials by a dense tile product
    int nl_total;
    const unsigned* ml;         // selection lists of the dense layers: per (chain, layer) block, a table
                                //   of 2 * units + 1 entry offsets (padded to an even length), then per
                                //   unit half its entries (chain-local entry offset from the layer's
                                //   first entry, LDS scratch slot) as uint2
    const long long* ml_off;    // [C][nl_total] word offset of a (chain, layer) block in ml (-1: none)
    void* part;                 // per-tile gradient partials, A
    long long tmax;             // partial slots per chain in the partial layout
    double* ulik;               // [C][tiles_a][8] likelihood partials (one slot per wave)
    double inv_lik_var;
    // DeepONet exchange buffers, T
    void* tm;                   // [C][nq_rows][p_p]   trunk features
    void* tt;                   // [C][p_p][nq_rows]   trunk features, transposed
    void* btr;                  // [C][p_p][nu_cols]   branch features, transposed
    void* dgt;                  // [C][nq_rows][nu_cols] output adjoint, transposed
    long long tm_stride, bt_stride, dgt_stride;
    int nq, nq_pad, nq_rows, nu_cols;
    long long b0_off;           // b0 position in the bias buffer
    int dg_off;                 // LDS offset (elements) of the [R][nq_pad + pad] output-adjoint slab
    int dg_ld;
    int red_off;                // LDS byte offset of the reduction scratch
    int bias_lds_a, bias_lds_b; // LDS byte offsets of the staged biases of towers A and B
    int y_lds;                  // LDS byte offset of the staged MLP targets of a tile [R][d_out]
    int meta_lds_a, meta_lds_b; // LDS byte offsets of the staged per-chain tables (TileMeta) of towers A and B
    int dgt_stage;              // 1: the trunk adjoint tile stages its rows of dgt in LDS (at dgt_lds, row
    int dgt_lds, dgt_lds_ld;    //   stride dgt_lds_ld elements) before the product dT = dG^T B; 0: reads them
                                //   from global memory
};

// Arguments of the per-entry kernels (reduction of partials, kicks, drifts,
// scatter into the dense weights, momentum refresh, Metropolis step).
// Most data batches of symmetric-splitting HMC (each batch's gradient is
// held in a register of the update kernel).
constexpr int HMC_SPLIT_MAX = 16;

struct StateArgs {
    int n_chains;               // chains of this launch: chain0 .. chain0 + n_chains - 1
    int chain0;                 // (k_update; 0 elsewhere)
    const int* active;
    const long long* offs;
    const int* seg;
    int nseg;
    int seg_trunk_lo, seg_trunk_hi;   // segment indices bounding the trunk entries
    int tiles_a, tiles_b;       // partial slots per chain and tower (row tiles, or tile groups)
    long long tmax;
    const void* part;
    const double* ulik;         // likelihood partials that define U, [C][ulik_tiles][8]
    int ulik_tiles;
    void* theta;                // S [nnz]
    void* mom;                  // S [nnz]
    void* grad;                 // S [nnz]
    void* theta_save;           // S [nnz]
    void* grad_save;            // S [nnz]
    const void* minv;           // S [nnz] or null (identity)
    const void* p_in;           // S [nnz] injected momentum or null
    void* p_out;                // S [nnz] momentum output (refresh preview)
    const int* dst;             // [2 * nnz] scatter destinations
    void* wbuf;
    long long wstride;
    void* wbuf32;               // shadow of wbuf for the energy pass (same offsets) or null
    int w32_f64;                // 1: that shadow holds doubles (FP64 energies), 0: floats
    void* bbuf64;               // FP64 shadow of bbuf for FP64 energies, or null
    void* bbuf;
    long long bstride;
    double* eps;                // [C] step sizes (written by the step-size adaptation)
    double* da;                 // [C][4] dual-averaging state: iterations m, H-bar, log eps-bar, mu
                                //   (calibration: count and sum of the acceptance probabilities)
    const int* adapt_on;        // device flag: 1 while the step sizes adapt, 2 while acceptance is summed
    const double* da_cfg;       // [4] target acceptance, gamma, t0, kappa
    double inv_prior_var;
    double* U;                  // [C]
    double* U_save;             // [C]
    double* H0;                 // [C]
    double* H1;                 // [C]
    unsigned long long* iter;   // [C]
    unsigned long long seed;
    unsigned long long iter_override;   // used by the momentum preview
    void* stats;                // hmc_traj_stat [C]
    long long* n_acc;           // [C]
    long long* n_div;           // [C]
    int split_n;                // symmetric splitting: data batches (0: plain leapfrog)
    int split_t[HMC_SPLIT_MAX + 1];   // partial slots of batch m: split_t[m] <= t < split_t[m + 1]
};

// UPD_KICK_DRIFT_LAST: the last kick and drift of a trajectory, which also
// writes the positions into the FP32 weight copy read by the energy pass
// (earlier drifts leave that copy alone: nothing reads it before the drift
// to theta_L).
enum { UPD_GRAD = 0, UPD_KICK_DRIFT = 1, UPD_HALF_KICK = 2, UPD_KICK_DRIFT_LAST = 3 };
// Symmetric-splitting kicks (k_update_split): SPL_FIRST, the batch half
// kicks in batch order and the first drift; SPL_STEP, the mirrored half
// kicks that end a step and the forward ones that start the next, then the
// drift (SPL_STEP_LAST: the trajectory's last drift); SPL_END, the mirrored
// half kicks that end the trajectory.
enum { SPL_FIRST = 0, SPL_STEP = 1, SPL_STEP_LAST = 2, SPL_END = 3 };
// Dense weight-gradient units: 2 x 2 or 4 x 2 blocks of 16 x 16, or the
// interleaved BF16 4 x 2 unit (rows i0 + 16 g + 4 v + bi, columns j0 + 2 li + bj).
enum { DWV_2X2 = 0, DWV_4X2 = 1, DWV_IL = 2 };
enum { END_ENERGY = 0, END_TRAJ = 1, END_METROPOLIS = 2 };
