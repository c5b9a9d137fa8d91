/*
 * hmc.h - C ABI of the masked full-batch HMC engine (gfx950 / MI355X).
 *
 * The engine draws samples of the selected parameter subset Theta_s of a
 * network while every other parameter stays at a given fixed value: the
 * conditional posterior P(Theta_s | D, Theta_~s) of Sec. 3.2 of the paper,
 * sampled by the HMC loop of Algorithm 2 (momentum refresh, leapfrog
 * integration of Hamilton's equations of Sec. 2.2, Metropolis-Hastings
 * step).  Each leapfrog step evaluates the network and its adjoint over the
 * whole training set (full batch) and the gradient of
 *
 *     U(Theta_s) = sum over rows and outputs of (F - y)^2 / (2 lik_sd^2)
 *                + sum over selected i of theta_i^2 / (2 prior_sd^2)
 *
 * with respect to the selected entries only (Gaussian prior and likelihood,
 * App. C; additive constants dropped).  Kinetic energy is p^T M^-1 p / 2
 * with a diagonal M (identity by default); the Hamiltonian, the likelihood
 * sum and the Metropolis test are evaluated in FP64.
 *
 * Conventions
 *  - Every function returns an hmc_status; a negative value is an error and
 *    hmc_last_error() describes it.  Nothing aborts or throws across the ABI.
 *  - All arguments are validated on the host before any device work, so an
 *    HMC_EINVAL return leaves the engine state unchanged.
 *  - The caller owns every input array; hmc_init copies what it needs, so the
 *    inputs may be freed when it returns.  The library owns its device
 *    buffers until hmc_destroy().
 *  - Arrays documented "host or device" may be host memory or device memory
 *    of the engine's GPU; the library copies with the unified-address copy.
 *  - The "state type" of an engine is double for HMC_FP64 and float for
 *    HMC_FP32, HMC_BF16 and HMC_BF16X3; positions, momenta and gradients cross the ABI in
 *    that type, in the CSR order of the mask (chain by chain).
 *  - Work is queued on the engine's stream.  Functions that return host
 *    results (stats, energies, copies to host) synchronise that stream.
 *  - A divergent (non-finite) trajectory is not an error: its proposal is
 *    rejected and reported with divergent = 1 (Sec. 4.2.3 reports infinite
 *    gradients in full-batch runs).
 *  - One engine must not be used from two threads at once; separate engines
 *    are independent.
 */
#ifndef HMC_H
#define HMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hmc_ctx hmc_ctx;

typedef enum {
    HMC_OK = 0,
    HMC_EINVAL = -1,        /* invalid argument; state unchanged              */
    HMC_ENOMEM = -2,        /* host or device allocation failed               */
    HMC_EDEVICE = -3,       /* HIP runtime error (message in hmc_last_error)  */
    HMC_ESTATE = -4,        /* call not valid in the engine's current state   */
    HMC_EUNSUPPORTED = -5   /* a shape or option this build does not support  */
} hmc_status;

/* Number format of the layer products.  FP64: everything in double.
 * FP32: products and states in float, energies in double.  BF16: products
 * take bfloat16 operands with float accumulation, states in float, energies
 * in double.  BF16X3: operands stay in float and each product is the sum of
 * three bfloat16 products of their high and low bfloat16 parts (about 16
 * significant bits per product, float accumulation), for BF16 matrix-core
 * throughput with trajectories close to FP32 ones; states in float,
 * energies in double.  The energies of the Metropolis test of BF16 and
 * BF16X3 engines come from a float forward pass. */
typedef enum { HMC_FP64 = 0, HMC_FP32 = 1, HMC_BF16 = 2, HMC_BF16X3 = 3 } hmc_precision;

/* Where U of the Hamiltonian (H0, H1, the Metropolis test) comes from.
 * DEFAULT: FP64 sums over the engine's own float products (FP32 engines),
 * or over a separate forward pass with float products on a float copy of
 * the weights (BF16 and BF16X3 engines); FP64 engines use their own FP64
 * pass.  FP64: a separate forward pass entirely in FP64 (FP64 copies of
 * the weights, biases and inputs, FP64 matrix cores) for FP32, BF16 and
 * BF16X3 engines, once per trajectory.  Acceptance depends on energy
 * differences of order one (Sec. 2.2); when U itself is very large (many
 * outputs with a small likelihood sd) the relative error of a float forward
 * pass, about 1e-7 of U, exceeds them. */
typedef enum { HMC_ENERGY_DEFAULT = 0, HMC_ENERGY_FP64 = 1 } hmc_energy;

/* Network family (Sec. 2 and App. A).  An MLP is one fully connected tower;
 * a DeepONet has a branch tower over input-function samples and a trunk
 * tower over query coordinates, combined by a dot product plus a scalar
 * bias b0.  Every layer is followed by tanh except the last of each tower. */
typedef enum { HMC_MLP = 0, HMC_DEEPONET = 1 } hmc_net_kind;

/* The network and the distribution.
 * widths_a: MLP widths [d_in, hidden..., d_out] or branch widths [m, ..., p].
 * widths_b: trunk widths [d_y, ..., p] for a DeepONet, else ignored.
 * theta0: the full flat parameter vector (n_params doubles).  Order: tower by
 *   tower (branch, then trunk, then b0), layer by layer, W[out][in]
 *   row-major then b[out].  Entries outside the mask stay at these values
 *   (Algorithm 2 fixes them at the VI means); selected entries start here
 *   unless hmc_mask_desc.theta_init is given.
 * inv_mass_diag: NULL for M = I, else n_params positive diagonal entries of
 *   M^-1 (only the selected ones are used).
 * energy: hmc_energy (HMC_ENERGY_DEFAULT or HMC_ENERGY_FP64).
 * Limits: 2..9 widths per tower, each width 1..4096. */
typedef struct {
    int32_t kind;
    int32_t n_widths_a;
    const int32_t* widths_a;
    int32_t n_widths_b;
    const int32_t* widths_b;
    const double* theta0;
    int64_t n_params;
    double prior_sd;
    double lik_sd;
    int32_t precision;
    const double* inv_mass_diag;
    int32_t energy;
} hmc_net_desc;

/* The selected subset Theta_s of each chain (Sec. 3.2), as CSR over chains.
 * offs[n_chains + 1] with offs[0] = 0; idx[offs[C]] flat indices, strictly
 * increasing within each chain, in [0, n_params); every chain selects at
 * least one entry.  Chains may select different subsets of different sizes.
 * theta_init: NULL (start from theta0[idx]) or offs[C] starting values. */
typedef struct {
    int32_t n_chains;
    const int64_t* offs;
    const int64_t* idx;
    const double* theta_init;
} hmc_mask_desc;

/* Training data D, host memory, row-major doubles.
 * MLP: x[n_rows][d_in], y[n_rows][d_out].
 * DeepONet: u[n_u][m] (branch inputs), yq[n_q][d_y] (trunk inputs, shared
 * by every function), v[n_u][n_q] (targets). */
typedef struct {
    const double* x;
    const double* y;
    int64_t n_rows;
    const double* u;
    const double* yq;
    const double* v;
    int64_t n_u;
    int64_t n_q;
} hmc_data_desc;

/* Outcome of one trajectory of one chain. */
typedef struct {
    double H0;          /* U(theta) + K(p) at the start                      */
    double H1;          /* U(theta*) + K(p*) at the end of the trajectory    */
    double log_u;       /* log of the Metropolis uniform                     */
    int32_t accepted;   /* 1 if log_u < H0 - H1                              */
    int32_t divergent;  /* 1 if H1 was not finite (proposal rejected)        */
} hmc_traj_stat;

typedef struct {
    int64_t n_params;
    int64_t nnz;              /* offs[n_chains]                              */
    int32_t n_chains;
    int32_t precision;
    int32_t kind;
    int32_t rows_per_tile_a;  /* rows of the MLP / branch tiles              */
    int32_t rows_per_tile_b;  /* rows of the trunk tiles (DeepONet)          */
    int32_t tiles_a;          /* row tiles of the MLP / branch tower         */
    int32_t tiles_b;
    int64_t device_bytes;     /* device memory held by the engine            */
    int32_t threads_a;        /* threads per workgroup of the MLP / branch   */
    int32_t threads_b;        /* ... and of the trunk tile kernels           */
    int32_t energy_precision; /* hmc_precision of the forward pass behind U  */
    int32_t chain_halves;     /* 1: trajectory graphs run the two halves of  */
                              /* the chains as two branches, one gradient    */
                              /* evaluation apart (plain leapfrog on grids   */
                              /* of at least eight workgroups per compute    */
                              /* unit in each half; HMC_HALVES=0|1, read at  */
                              /* set-up, overrides)                          */
} hmc_info_t;

/* Creates an engine for the sampling problem of Algorithm 2 (Sec. 3.2: the
 * network F_Theta, the fixed values mu_~s, the subset s, the Gaussian prior
 * and likelihood of App. C, the data D and a starting Theta_s per chain):
 * validates, uploads data and parameters, and evaluates U and its gradient
 * at the starting point of every chain.
 * seed keys the Philox4x64-10 streams of the momentum refresh and of the
 * Metropolis uniforms (key = (seed, chain), counter = (iteration, stream,
 * block, 0)).  hip_stream: a hipStream_t to queue work on, or NULL for a
 * stream owned by the engine.  *out is NULL on failure. */
hmc_status hmc_init(hmc_ctx** out, const hmc_net_desc* net, const hmc_mask_desc* mask,
                    const hmc_data_desc* data, uint64_t seed, void* hip_stream);

/* Launch-shape choices of the gradient kernels (an engineering option, not
 * a step of the method: every choice computes the same U and gradient up to
 * the summation order); 0 in a field keeps the
 * engine's own choice (made from the LDS footprint, the grid size and the
 * layer densities; HMC_ROWS_A, HMC_ROWS_B, HMC_THREADS and HMC_DW in the
 * environment override it when the field is 0).  FP32 MLP engines at
 * 32-row tiles on large grids also let one workgroup sum several row tiles
 * of a chain into one partial slot (HMC_TILE_GROUP = 1, 2, 4 or 8 fixes the
 * number); the result differs from one tile per workgroup only in the
 * summation order. */
typedef struct {
    int32_t rows_a;    /* rows per tile of the MLP / branch tower: 0, 16, 32 or 64       */
    int32_t rows_b;    /* rows per tile of the trunk tower: 0, 16, 32 or 64              */
    int32_t threads;   /* threads per workgroup of the tile kernels: 0, 256 or 512       */
    int32_t dw;        /* masked dW: 0 automatic, 1 per-entry sums, 2 dense tile product
                          (on every layer where the tile height allows it)              */
} hmc_tuning;

/* hmc_init with explicit launch shapes (tuning NULL: as hmc_init).  A tile
 * height that does not fit in LDS gives HMC_EUNSUPPORTED; values outside the
 * listed ones give HMC_EINVAL. */
hmc_status hmc_init_tuned(hmc_ctx** out, const hmc_net_desc* net, const hmc_mask_desc* mask,
                          const hmc_data_desc* data, uint64_t seed, void* hip_stream, const hmc_tuning* tuning);

/* Autotuner: builds an engine for every candidate launch shape that fits
 * (tile heights 16/32/64 for each tower, 256 or 512 threads, per-entry or
 * dense masked dW where the dense product applies), times one gradient
 * evaluation of all chains (hmc_time_kernels, reps launches each, HIP
 * events) and returns the fastest in *best and its milliseconds in *best_ms
 * (may be NULL).  Uses the current device and its own streams; synchronous;
 * takes seconds for large networks. */
hmc_status hmc_autotune(const hmc_net_desc* net, const hmc_mask_desc* mask, const hmc_data_desc* data,
                        int32_t reps, hmc_tuning* best, double* best_ms);

/* One iteration of the loop of Algorithm 2 (Sec. 3.2) for the listed chains: draw
 * p ~ N(0, M), integrate L leapfrog steps of size eps[i] for chain
 * chain_ids[i] (kick-drift-kick, exactly L gradient evaluations), then
 * accept or reject.  chain_ids NULL means chains 0..n_chains-1.
 * eps: host, n_chains positive finite values.  stats: host [n_chains] or
 * NULL (no synchronisation then). */
hmc_status hmc_leapfrog(hmc_ctx* ctx, int32_t n_chains, const int32_t* chain_ids,
                        const double* eps, int32_t L, hmc_traj_stat* stats);

/* n iterations of Algorithm 2 for every chain, each chain with its own step
 * size eps[c] (host, C values) and a common L.  After iteration i the
 * positions of all chains are written to samples + i * nnz (state type, host
 * or device, or NULL).  stats: host [n][C] or NULL. */
hmc_status hmc_sample(hmc_ctx* ctx, int64_t n, const double* eps, int32_t L,
                      void* samples, hmc_traj_stat* stats);

/* U (host, [C]) and the gradient of U with respect to the selected entries
 * (state type, host or device, [nnz]) at the current positions: the
 * potential of Sec. 2.2 with the prior and likelihood of App. C, and the
 * gradient that each leapfrog step of Algorithm 2 takes, for every chain. */
hmc_status hmc_grad(hmc_ctx* ctx, double* U, void* g);

/* The leapfrog integration of Hamilton's equations (Sec. 2.2) that one
 * iteration of Algorithm 2 runs, for every chain, without the Metropolis
 * step and without changing the engine state: starting from the current
 * positions with momentum p0 (state type,
 * host or device, [nnz]), run L leapfrog steps of size eps[c] (host, [C]) and
 * return the end point theta_out, p_out ([nnz], host or device, may be NULL)
 * and H0, H1 (host, [C], may be NULL). */
hmc_status hmc_trajectory(hmc_ctx* ctx, const void* p0, const double* eps, int32_t L,
                          void* theta_out, void* p_out, double* H0, double* H1);

/* Symmetric-splitting HMC, the integrator of the paper's full-HMC baseline
 * (Sec. 4.2.3, after Cobb and Jalaian): the data rows are split into
 * consecutive batches of batch_rows rows (the last one takes the rest); the
 * potential of a batch is its rows' likelihood plus 1/M of the prior (M
 * batches), and every step of hmc_leapfrog, hmc_sample, hmc_trajectory,
 * hmc_adapt and hmc_calibrate applies each batch gradient as a half kick of
 * its own, in batch order, then drifts, then applies the batch half kicks
 * in the mirrored order.  In exact arithmetic this is the leapfrog step;
 * the trajectory takes L + 1 gradient evaluations (the batch gradients at
 * the start are evaluated afresh).  batch_rows = 0 returns to plain
 * leapfrog.
 * Errors: HMC_EINVAL if batch_rows is negative, not a multiple of
 * rows_per_tile_a (hmc_get_info), or gives more than 16 batches;
 * HMC_EUNSUPPORTED for a DeepONet (its trunk gradient is reduced over every
 * input function inside a row tile) and for an MLP engine with tile groups
 * (HMC_TILE_GROUP above 1, or the automatic choice on large FP32 grids at
 * 32 rows per tile). */
hmc_status hmc_set_split(hmc_ctx* ctx, int64_t batch_rows);

/* The momentum p ~ N(0, M) that the refresh of Algorithm 2 draws at
 * iteration `iteration`, for every chain (state type, host or device,
 * [nnz]).  The engine state is unchanged. */
hmc_status hmc_momentum(hmc_ctx* ctx, uint64_t iteration, void* p_out);

/* The chain state of Algorithm 2: current positions (state type, host or
 * device, [nnz], may be NULL), U (host [C] or NULL) and per-chain iteration
 * counters (host [C] or NULL). */
hmc_status hmc_get_state(hmc_ctx* ctx, void* theta_s, double* U, uint64_t* iteration);

/* Sets the positions (state type, host or device, [nnz]) and iteration
 * counters (host [C], or NULL to keep them), and re-evaluates U and the
 * gradient.  Together with hmc_get_state this checkpoints and resumes a run:
 * the counter-based streams make the continuation identical. */
hmc_status hmc_set_state(hmc_ctx* ctx, const void* theta_s, const uint64_t* iteration);

/* Accepted and divergent trajectory counts per chain since hmc_init (host,
 * [C] each, either may be NULL): the outcomes of the Metropolis step of
 * Algorithm 2 (a divergent trajectory, Sec. 4.2.3, is a rejection). */
hmc_status hmc_counters(hmc_ctx* ctx, int64_t* accepted, int64_t* divergent);

hmc_status hmc_get_info(const hmc_ctx* ctx, hmc_info_t* info);

/* Measurement hook: launches each gradient-evaluation kernel `reps` times
 * back to back on the engine's stream between two HIP events and writes the
 * mean milliseconds per launch to ms[0..3]:
 *   ms[0] fused forward/adjoint/masked-gradient kernel (MLP or branch),
 *   ms[1] trunk forward (DeepONet, else 0), ms[2] trunk adjoint (DeepONet,
 *   else 0), ms[3] reduction of the per-tile gradient partials.
 * The engine state is unchanged. */
hmc_status hmc_time_kernels(hmc_ctx* ctx, int32_t reps, double* ms);

/* Parameter sensitivities of Sec. 3.1 (sensitivity equation): around the
 * mean parameters mu = net->theta0, with standard deviations sigma (host,
 * [n_params], finite, >= 0),
 *   s2[i] = sigma_i^2 / N_d * sum_{inputs j} sum_{outputs o} (dF_mu(x_j)_o / dtheta_i)^2.
 * MLP: the n_rows rows of data->x are the inputs, the outputs of a row its
 * output entries (y is not read).  DeepONet: the n_u functions of data->u are
 * the inputs, the n_q query points of data->yq the outputs of each (v is not
 * read).  The squared output derivatives are summed over the output entries
 * of each input (their variances add).  Every layer runs as MFMA tile
 * products on squared operands on the device, one adjoint pass per output
 * (MLP), per query point (DeepONet branch, seeded with the trunk features)
 * and per function (DeepONet trunk, seeded with the branch features); a
 * DeepONet tower with more such rows than latent features p is seeded with
 * the p or fewer vectors of a factor of the features' Gram matrix instead,
 * which gives the same sums; BF16
 * and BF16X3 networks are evaluated in FP32, FP64 networks in FP64.  s2: host
 * [n_params] FP64, written on success.  net->prior_sd and net->lik_sd must
 * be valid but are not used.  Synchronous; hip_stream as for hmc_init.
 * Errors: HMC_EINVAL (NULL pointers, sizes, negative or non-finite sigma),
 * HMC_ENOMEM, HMC_EDEVICE, HMC_EUNSUPPORTED (a tower that does not fit in
 * LDS); the message is in hmc_last_error(NULL). */
hmc_status hmc_sensitivity(const hmc_net_desc* net, const hmc_data_desc* data, const double* sigma,
                           double* s2, void* hip_stream);

/* Posterior predictive moments (the mean prediction and its spread shown in
 * the results sections) of chain `chain` over n_samples stored samples:
 * samples is laid out as hmc_sample writes it, [n_samples][nnz] in the
 * state type, host or device; sample k of the chain is
 * samples + k * nnz + offs[chain], its other parameters stay at their fixed
 * values.  New inputs (host): MLP inputs->x [n_rows][d_in] (y not read),
 * outputs [n_rows][d_out]; DeepONet inputs->u [n_u][m] and inputs->yq
 * [n_q][d_y] (v not read), outputs [n_u][n_q].  mean (host, output shape,
 * required) receives the mean of the network outputs over the samples and
 * var (host, same shape, or NULL) their variance (1/n_samples, no Bessel
 * correction), both accumulated in FP64.  BF16 and BF16X3 engines evaluate
 * through their FP32 weight shadow.  The engine's chain state is unchanged.
 * Synchronous.  Errors: HMC_EINVAL (chain, sizes, NULL pointers), HMC_ENOMEM,
 * HMC_EDEVICE. */
hmc_status hmc_predict(hmc_ctx* ctx, int32_t chain, const void* samples, int64_t n_samples,
                       const hmc_data_desc* inputs, double* mean, double* var);

/* hmc_predict for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, results and errors, but the call's device
 * buffers (the tiled new inputs, the staged sample, the FP64 moments and the
 * DeepONet tower outputs) come from a fixed 64 MiB region that the library
 * holds on every GPU it runs on, and the call makes no device allocation.
 * A request that needs more than 64 MiB of it (each buffer rounded up to 256
 * bytes) returns HMC_EUNSUPPORTED before any device work.  Every call on one
 * GPU uses the same region: calls that overlap on one GPU (from several
 * threads, or engines on different streams) race and must be serialised by
 * the caller; each call clears what it needs. */
hmc_status hmc_predict_noalloc(hmc_ctx* ctx, int32_t chain, const void* samples, int64_t n_samples,
                               const hmc_data_desc* inputs, double* mean, double* var);

/* The sensitive subset of Sec. 3.1 (threshold equation): the parameters
 * ordered from the most to the least sensitive (equal values in index
 * order), and the largest count N whose cumulative share of sum(s2) is at
 * most tau.  s2: host [n] (finite, >= 0, not all zero); tau in [0, 1].
 * idx: host [n], receives the N selected indices in increasing order (a
 * mask for hmc_init); *n_sel = N (it may be 0).  Host only. */
hmc_status hmc_select_mask(const double* s2, int64_t n, double tau, int64_t* idx, int64_t* n_sel);

/* Step-size adaptation for a target acceptance rate (Sec. 4.2.3 fixes it at
 * 80% with the dual-averaging scheme of Hoffman and Gelman, 2014): runs n
 * iterations of Algorithm 2 for every chain (they move the chains and
 * advance the iteration counters; nothing is stored), each chain starting
 * at eps0[c] (host, [C], positive finite) and updating its own step size on
 * the device after every Metropolis step from the trajectory's acceptance
 * probability min(1, exp(H0 - H1)) (0 if divergent), with gamma = 0.05,
 * t0 = 10, kappa = 0.75, mu = log(10 eps0[c]).  eps_out (host, [C]): the
 * averaged iterate eps-bar of each chain, the step size to sample with.
 * L >= 1 is the common trajectory length; target in (0, 1).  Synchronous.
 * Errors: HMC_EINVAL (state unchanged), HMC_EDEVICE. */
hmc_status hmc_adapt(hmc_ctx* ctx, int64_t n, const double* eps0, int32_t L, double target, double* eps_out);

/* Step sizes for a target acceptance rate to within the noise of a batch
 * mean (the matched 80% acceptance of Sec. 4.2.3's comparison; dual
 * averaging alone settles somewhat above its target): per chain, a
 * bisection in log eps over `rounds` rounds of `batch` iterations of
 * Algorithm 2 each (they move the chains; nothing is stored).  Each round
 * runs at the current step sizes and sums every trajectory's acceptance
 * probability min(1, exp(H0 - H1)) (0 if divergent) on the device; a chain
 * whose batch mean exceeds the target takes its step size as a lower bound,
 * otherwise as an upper bound, and moves to the midpoint of its bounds in log
 * eps (by a factor 1.25 while one bound is missing).  eps_in (host, [C]):
 * the starting step sizes (e.g. from hmc_adapt); eps_out (host, [C]): the
 * final midpoints; acc_out (host, [C], or NULL): each chain's batch mean in
 * the last round.  rounds in 1..64, batch >= 1, L >= 1, target in (0, 1).
 * Synchronous.  Errors: HMC_EINVAL (state unchanged), HMC_EDEVICE. */
hmc_status hmc_calibrate(hmc_ctx* ctx, int32_t rounds, int64_t batch, const double* eps_in, int32_t L, double target,
                         double* eps_out, double* acc_out);

/* Number of leapfrog steps from App. C: L = pi * v / (2 eps), rounded to the
 * nearest integer and at least 1, where v is the largest (mode 0) or the
 * median (mode 1) of the n posterior variances var (host, finite, >= 0;
 * App. C takes the largest VI variance for Burgers and BNN case I and the
 * median elsewhere).  The product L * eps is then a fixed integration time
 * pi * v / 2, as in the fixed simulation length of Hoffman and Gelman's HMC
 * with dual averaging.  Host only.  Errors: HMC_EINVAL (NULL pointers,
 * n < 1, bad mode, eps not positive and finite, a variance not finite or
 * negative, more than 10^6 steps); the message is in hmc_last_error(NULL). */
hmc_status hmc_trajectory_length(const double* var, int64_t n, int32_t mode, double eps, int32_t* L);

/* Waits for queued work and reports deferred device errors. */
hmc_status hmc_sync(hmc_ctx* ctx);

/* NUL-terminated description of the last error on ctx (ctx may be NULL for
 * errors of a failed hmc_init); valid until the next call on ctx. */
const char* hmc_last_error(const hmc_ctx* ctx);

void hmc_destroy(hmc_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* HMC_H */
