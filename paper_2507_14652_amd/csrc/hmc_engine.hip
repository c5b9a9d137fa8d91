// Host engine behind the C ABI of include/hmc.h: validation, device layout,
// launch sequencing of the leapfrog trajectory, graph capture of whole
// trajectories, and the measurement hooks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hmc.h"
#include "hmc_launch.hpp"
#include "hmc_plan.hpp"

// Fixed device scratch of hmc_predict_noalloc: one copy on every GPU the
// library runs on, held until the process ends.  Host code never uses this
// name as an address (on the host it is a stand-in); it uses the device
// address that hipGetSymbolAddress returns for the current device.
#define HMC_SCRATCH_BYTES ((size_t)64 << 20)
static __device__ __align__(256) unsigned char scratch[HMC_SCRATCH_BYTES];

namespace {

thread_local std::string g_init_error;

// Device address of `scratch` per device, looked up once per device by the
// first hmc_init that runs with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

void scratch_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess && p) g_scratch_ptr[dev] = p;
    else g_scratch_err[dev] = e == hipSuccess ? hipErrorInvalidSymbol : e;
}

void* scratch_of(int dev, hipError_t* err) {
    if (dev < 0 || dev >= kMaxDevices) { *err = hipErrorInvalidDevice; return nullptr; }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    *err = g_scratch_err[dev];
    return g_scratch_ptr[dev];
}

size_t g_lds_cap = 160 * 1024;   // LDS per workgroup on gfx950; replaced by the device's value

// K chunk of the product (bf16 MFMAs take 32), LDS row padding in elements,
// and the stored product type (split BF16 keeps float operands).
int pad_of(int prec) { return prec == HMC_BF16 || prec == HMC_BF16X3 ? 32 : 16; }
int lpad_of(int prec) { return prec == HMC_BF16 ? 8 : 4; }
size_t tsize_of(int prec) { return prec == HMC_FP64 ? 8 : prec == HMC_BF16 ? 2 : 4; }
size_t asize_of(int prec) { return prec == HMC_FP64 ? 8 : 4; }                          // accumulator / bias type
size_t ssize_of(int prec) { return prec == HMC_FP64 ? 8 : 4; }                          // state type
int roundup(int x, int m) { return (x + m - 1) / m * m; }
long long roundupl(long long x, long long m) { return (x + m - 1) / m * m; }

uint16_t to_bf16_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return 0x7FC0;   // NaN
    u += 0x7FFFu + ((u >> 16) & 1u);                                             // round to nearest even
    return (uint16_t)(u >> 16);
}

// BF16 bits of f (round to nearest even) and their value as a float.
uint16_t bf16_round(float f, float* back) {
    const uint16_t b = to_bf16_bits(f);
    const uint32_t u = (uint32_t)b << 16;
    std::memcpy(back, &u, 4);
    return b;
}

// Stores v in the product type at index i of a byte buffer.  Split BF16
// (buffers whose rows are multiples of eight elements): element i is the
// pair hi = bf16(v), lo = bf16(v - hi) at BF16 slots (i / 8) * 16 + i % 8
// and 8 slots on, as the kernels read it.
void put_t(std::vector<unsigned char>& buf, int prec, size_t i, double v) {
    if (prec == HMC_FP64) { std::memcpy(&buf[i * 8], &v, 8); return; }
    const float f = (float)v;
    if (prec == HMC_FP32) { std::memcpy(&buf[i * 4], &f, 4); return; }
    if (prec == HMC_BF16) {
        const uint16_t b = to_bf16_bits(f);
        std::memcpy(&buf[i * 2], &b, 2);
        return;
    }
    float hf;
    const uint16_t hi = bf16_round(f, &hf);
    const uint16_t lo = to_bf16_bits(f - hf);
    const size_t slot = (i >> 3) * 16 + (i & 7);
    std::memcpy(&buf[slot * 2], &hi, 2);
    std::memcpy(&buf[(slot + 8) * 2], &lo, 2);
}
void put_a(std::vector<unsigned char>& buf, int prec, size_t i, double v) {
    if (prec == HMC_FP64) { std::memcpy(&buf[i * 8], &v, 8); return; }
    const float f = (float)v;
    std::memcpy(&buf[i * 4], &f, 4);
}

struct TowerHost {
    std::vector<int> w;
    long long flat0 = 0;                 // flat index of the tower's first parameter
    std::vector<long long> lstart;       // flat index of each layer's first parameter
};

}  // namespace

struct hmc_ctx {
    std::string err;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;
    // staggered chain halves in the trajectory graph (halves_on)
    hipStream_t cap_stream2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_stag = nullptr, ev_join = nullptr;
    int halves = 0;               // halves_on, fixed at set-up and by hmc_set_split

    int kind = 0, prec = 0;
    TowerHost A, B;
    long long P = 0;
    double prior_sd = 1, lik_sd = 1;
    int C = 0;
    long long nnz = 0;
    std::vector<long long> offs;
    int max_n = 0;
    int upd_sub = 1;          // threads per entry of k_update (update_sub)
    int Ra = 0, Rb = 0, tiles_a = 0, tiles_b = 0;
    bool alias_a = false, alias_b = false;   // slabs 1 and 3 shared (a_1 recomputed in the adjoint pass)
    int grid_a = 0, grid_b = 0;
    int tpg = 1;                  // MLP gradient kernel: row tiles per workgroup (tile_group)
    int groups_a = 0, grid_mlp = 0;   // ... its tile groups per chain and its grid
    size_t lds_a = 0, lds_b = 0;
    int nt_a = 256, nt_b = 256, nt_a32 = 256, nt_b32 = 256;   // threads per workgroup
    bool force_dense = false;     // sensitivity engines: dense dW (squared terms) on every layer
    hmc_tuning tune{0, 0, 0, 0};  // launch-shape overrides (0: automatic)
    GradArgs ga{};
    StateArgs sa{};
    // BF16 and split-BF16 engines: FP32 energy pass over an FP32 shadow of the weights
    bool energy32 = false;     // a separate energy pass (its plan and buffers: ga32 and the *32 fields)
    int eprec = HMC_FP32;      // its precision: HMC_FP32, or HMC_FP64 on request
    GradArgs ga32{};
    int Ra32 = 0, Rb32 = 0, tiles_a32 = 0, tiles_b32 = 0, grid_a32 = 0, grid_b32 = 0;
    size_t lds_a32 = 0, lds_b32 = 0;
    std::vector<void*> allocs;
    long long dev_bytes = 0;
    std::vector<int> active_h;
    void* pin = nullptr;          // device [nnz] state type: injected momentum
    void* ptmp = nullptr;         // device [nnz] state type: momentum preview
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_L = -1;
    int dense_layers = 0;         // (chain, layer) pairs on the dense weight-gradient path
    hipEvent_t ev0 = nullptr, ev1 = nullptr;

    hmc_status fail(hmc_status s, const std::string& m) { err = m; return s; }
    hmc_status hip(hipError_t e, const char* what) {
        if (e == hipSuccess) return HMC_OK;
        err = std::string(what) + ": " + hipGetErrorString(e);
        return HMC_EDEVICE;
    }
    void* dalloc(size_t bytes) {
        void* p = nullptr;
        if (bytes == 0) bytes = 16;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        if (hipMemset(p, 0, bytes) != hipSuccess) { (void)hipFree(p); return nullptr; }
        allocs.push_back(p);
        dev_bytes += (long long)bytes;
        return p;
    }
};

#define HMC_TRY(expr)                          \
    do {                                       \
        hmc_status s__ = (expr);               \
        if (s__ != HMC_OK) return s__;         \
    } while (0)
#define HMC_HIP(x, call) HMC_TRY((x)->hip((call), #call))

namespace {

// ----------------------------------------------------------------- validation

hmc_status check_tower(const int32_t* w, int32_t n, const char* name, std::string& err) {
    if (!w) { err = std::string(name) + " is NULL"; return HMC_EINVAL; }
    if (n < 2 || n > HMC_MAXL + 1) {
        err = std::string(name) + ": need 2.." + std::to_string(HMC_MAXL + 1) + " widths";
        return HMC_EINVAL;
    }
    for (int i = 0; i < n; ++i)
        if (w[i] < 1 || w[i] > 4096) { err = std::string(name) + ": widths must be in 1..4096"; return HMC_EINVAL; }
    return HMC_OK;
}

long long tower_count(const std::vector<int>& w) {
    long long n = 0;
    for (size_t i = 0; i + 1 < w.size(); ++i) n += (long long)w[i] * w[i + 1] + w[i + 1];
    return n;
}

hmc_status validate(const hmc_net_desc* net, const hmc_mask_desc* mask, const hmc_data_desc* data,
                    std::string& err) {
    if (!net || !mask || !data) { err = "net, mask and data must be non-NULL"; return HMC_EINVAL; }
    if (net->kind != HMC_MLP && net->kind != HMC_DEEPONET) { err = "unknown network kind"; return HMC_EINVAL; }
    if (net->precision < HMC_FP64 || net->precision > HMC_BF16X3) { err = "unknown precision"; return HMC_EINVAL; }
    if (net->energy != HMC_ENERGY_DEFAULT && net->energy != HMC_ENERGY_FP64) { err = "unknown energy"; return HMC_EINVAL; }
    HMC_TRY(check_tower(net->widths_a, net->n_widths_a, "widths_a", err));
    std::vector<int> wa(net->widths_a, net->widths_a + net->n_widths_a), wb;
    long long P = tower_count(wa);
    if (net->kind == HMC_DEEPONET) {
        HMC_TRY(check_tower(net->widths_b, net->n_widths_b, "widths_b", err));
        wb.assign(net->widths_b, net->widths_b + net->n_widths_b);
        if (wa.back() != wb.back()) { err = "branch and trunk output widths differ"; return HMC_EINVAL; }
        P += tower_count(wb) + 1;
    }
    if (net->n_params != P) {
        err = "n_params = " + std::to_string(net->n_params) + " but the network has " + std::to_string(P);
        return HMC_EINVAL;
    }
    if (!net->theta0) { err = "theta0 is NULL"; return HMC_EINVAL; }
    if (!(net->prior_sd > 0) || !std::isfinite(net->prior_sd)) { err = "prior_sd must be positive and finite"; return HMC_EINVAL; }
    if (!(net->lik_sd > 0) || !std::isfinite(net->lik_sd)) { err = "lik_sd must be positive and finite"; return HMC_EINVAL; }
    if (net->inv_mass_diag)
        for (long long i = 0; i < P; ++i)
            if (!(net->inv_mass_diag[i] > 0) || !std::isfinite(net->inv_mass_diag[i])) {
                err = "inv_mass_diag entries must be positive and finite";
                return HMC_EINVAL;
            }
    if (mask->n_chains < 1 || mask->n_chains > 65535) { err = "n_chains must be in 1..65535"; return HMC_EINVAL; }
    if (!mask->offs || !mask->idx) { err = "mask offs and idx must be non-NULL"; return HMC_EINVAL; }
    if (mask->offs[0] != 0) { err = "mask offs[0] must be 0"; return HMC_EINVAL; }
    for (int c = 0; c < mask->n_chains; ++c) {
        const long long a = mask->offs[c], b = mask->offs[c + 1];
        if (b <= a) { err = "chain " + std::to_string(c) + " selects no entry"; return HMC_EINVAL; }
        if (b - a > (1ll << 30)) { err = "too many entries in one chain"; return HMC_EINVAL; }
        for (long long k = a; k < b; ++k) {
            const long long f = mask->idx[k];
            if (f < 0 || f >= P) { err = "mask index out of range in chain " + std::to_string(c); return HMC_EINVAL; }
            if (k > a && f <= mask->idx[k - 1]) {
                err = "mask indices must be strictly increasing within chain " + std::to_string(c);
                return HMC_EINVAL;
            }
        }
    }
    if (net->kind == HMC_MLP) {
        if (!data->x || !data->y) { err = "MLP data needs x and y"; return HMC_EINVAL; }
        if (data->n_rows < 1 || data->n_rows > (1ll << 30)) { err = "n_rows out of range"; return HMC_EINVAL; }
    } else {
        if (!data->u || !data->yq || !data->v) { err = "DeepONet data needs u, yq and v"; return HMC_EINVAL; }
        if (data->n_u < 1 || data->n_q < 1 || data->n_u > (1ll << 24) || data->n_q > (1ll << 24)) {
            err = "n_u and n_q out of range";
            return HMC_EINVAL;
        }
    }
    return HMC_OK;
}

// ----------------------------------------------------------------- planning

// Threads per workgroup of a tile kernel: 512 (8 waves).  Measured on every
// named workload it is as fast as or faster than 256, also where two
// workgroups share a CU's LDS (the FP32 MLP 32.1 -> 31.8 us, the DeepONet
// trunk adjoint 54 -> 50 us; the BF16 kernels that fill a CU's LDS alone lose
// a third of their speed at 256).  A tuning value (256 or 512) or else
// HMC_THREADS overrides it.
int pick_threads(size_t /*lds*/, int forced) {
    if (forced == 256 || forced == 512) return forced;
    if (const char* s = std::getenv("HMC_THREADS")) {
        const int t = std::atoi(s);
        if (t == 256 || t == 512) return t;
    }
    return 512;
}

// Slab sharing (recompute) applies to towers with at least four linear
// layers, where slab 3 holds a hidden activation.
// Slabs 1 and 3 may share LDS in towers of four or more layers, at tile
// heights of at most 32 rows, and at 64 rows in BF16 (the other 64-row
// kernels carry no recompute code; the 256-wide BF16 MLP fits 64-row tiles
// only with sharing: 22 against 34 ms at 32 rows).
bool can_alias(const std::vector<int>& w, int r, int prec) {
    return w.size() >= 5 && (r <= 32 || prec == HMC_BF16);
}

// LDS row stride (elements) of slab l.
int slab_ld(const std::vector<int>& w, int prec, size_t l) { return roundup(w[l], pad_of(prec)) + lpad_of(prec); }

// Bytes of a tower's activation slabs at R rows; alias: slabs 1 and 3 share
// one region of the larger stride.
size_t tower_lds(const std::vector<int>& w, int prec, int R, bool alias = false) {
    size_t e = 0;
    for (size_t l = 0; l < w.size(); ++l) {
        if (alias && l == 3) continue;
        int ld = slab_ld(w, prec, l);
        if (alias && l == 1) ld = std::max(ld, slab_ld(w, prec, 3));
        e += (size_t)R * ld;
    }
    return e * tsize_of(prec);
}

void fill_plan(TowerPlan& tp, const std::vector<int>& w, int prec, int R, bool alias = false) {
    std::memset(&tp, 0, sizeof(tp));
    tp.nl = (int)w.size() - 1;
    tp.rc1 = alias ? 1 : 0;
    int off = 0;
    for (size_t l = 0; l < w.size(); ++l) {
        tp.w[l] = w[l];
        tp.wp[l] = roundup(w[l], pad_of(prec));
        tp.ls[l] = slab_ld(w, prec, l);
        if (alias && l == 3) {
            tp.lo[l] = tp.lo[1];
            continue;
        }
        tp.lo[l] = off;
        off += R * (alias && l == 1 ? std::max(tp.ls[1], slab_ld(w, prec, 3)) : tp.ls[l]);
    }
}

// Plan of the FP32 energy pass of a BF16 engine: the same padded widths and
// weight offsets as the BF16 plan (so one scatter serves both copies), FP32
// LDS strides, and two activation slabs used alternately (forward only).
void fill_plan_energy(TowerPlan& tp, const TowerPlan& src, int R) {
    tp = src;
    int mx = 0;
    for (int l = 0; l <= src.nl; ++l) {
        tp.ls[l] = src.wp[l] + 4;
        mx = std::max(mx, tp.ls[l]);
    }
    for (int l = 0; l <= src.nl; ++l) tp.lo[l] = (l % 2) * R * mx;
}

// LDS bytes of a tower's staged biases: the padded widths of precision
// prec, stored in the accumulator type (as bytes each).
size_t bias_bytes(const std::vector<int>& w, int prec, size_t as) {
    size_t n = 0;
    for (size_t l = 1; l < w.size(); ++l) n += (size_t)roundup(w[l], pad_of(prec));
    return (n * as + 15) / 16 * 16;
}

size_t energy_lds(const TowerPlan& src, int R, size_t es) {
    int mx = 0;
    for (int l = 0; l <= src.nl; ++l) mx = std::max(mx, src.wp[l] + 4);
    return ((size_t)2 * R * mx * es + 15) / 16 * 16;
}

// fixed: bytes beside the slabs (staged biases); per_row: bytes per tile row
// (staged targets); es: bytes per element of the energy pass.
int pick_rows_energy(const TowerPlan& src, size_t fixed, size_t per_row, size_t es) {
    for (int R : {64, 32, 16})
        if (energy_lds(src, R, es) + 64 + fixed + per_row * R <= g_lds_cap) return R;
    return 0;
}

// Largest row tile whose LDS footprint fits, halved while the grid has
// fewer workgroups than the 256 compute units (smaller tiles re-read the
// weights more often, so a grid of one 512-thread workgroup per compute unit
// is enough: the DeepONet trunk adjoint runs 50 -> 46 us at 32 rows instead
// of 16).  A tower of four or more layers shares slabs 1 and 3 (alias,
// recomputing a_1 in the adjoint pass: one tile product of the narrow input
// layer) where that makes a taller tile of at most 32 rows fit.  A tuning value (16, 32 or 64;
// 0 when it does not fit) or else HMC_ROWS_A / HMC_ROWS_B overrides the
// height.  fixed: bytes beside the slabs (staged biases, alignment);
// scr_bytes: the dense weight-gradient scratch, needed at tile heights that
// are multiples of kch.
int pick_rows(const std::vector<int>& w, int prec, size_t extra_per_row, size_t fixed, long long rows, int chains,
              const char* env, int forced, size_t scr_bytes, int kch, bool& alias, bool pair = false) {
    alias = false;
    auto bytes_as = [&](int r, bool al) {
        const size_t scr = r % kch == 0 ? scr_bytes : 0;
        return tower_lds(w, prec, r, al) + extra_per_row * r + 64 + HMC_META_BYTES + 16 + fixed + scr;
    };
    auto fits_as = [&](int r, bool al) { return bytes_as(r, al) <= g_lds_cap; };
    const char* rc = std::getenv("HMC_RECOMPUTE");   // "1": share wherever possible (tests)
    const bool force_alias = rc && !std::strcmp(rc, "1");
    // the sharing choice for one candidate height; false: it does not fit
    auto choose = [&](int r, bool& al) {
        if (force_alias && can_alias(w, r, prec)) { al = true; return fits_as(r, true); }
        if (fits_as(r, false)) { al = false; return true; }
        if (can_alias(w, r, prec) && fits_as(r, true)) { al = true; return true; }
        return false;
    };
    if (forced) return choose(forced, alias) ? forced : 0;
    if (const char* s = std::getenv(env)) {
        const int r = std::atoi(s);
        if ((r == 16 || r == 32 || r == 64) && choose(r, alias)) return r;
    }
    int best = 0;
    for (int R : {64, 32, 16})
        if (choose(R, alias)) { best = R; break; }
    bool al2 = false;
    while (best > 16 && (long long)chains * ((rows + best - 1) / best) < 256 && choose(best / 2, al2)) {
        best /= 2;
        alias = al2;
    }
    // pair: on a large grid take 16-row tiles when two of those fit in one
    // compute unit's LDS and one of 32 rows does not (the FP32 MLP kernel:
    // two resident workgroups hide its LDS and barrier latency better than
    // one of twice the height; 256-wide MLP, 256 chains: 72.3 + 4.0 ms per
    // gradient evaluation at 16 rows against 78.9 + 0.25 at 32 with tile
    // groups)
    if (pair && best == 32 && bytes_as(32, alias) > g_lds_cap / 2 && choose(16, al2) &&
        bytes_as(16, al2) <= g_lds_cap / 2 && (long long)chains * ((rows + 15) / 16) >= 16 * 256) {
        best = 16;
        alias = al2;
    }
    return best;
}

// Row tiles per workgroup of the MLP gradient kernel: it sums the weight-
// gradient terms of that many consecutive tiles of one chain into one
// partial slot (read-modify-writes by the thread that owns each entry),
// which divides the partials k_update reads by as much.  Groups of up to
// eight while the grid keeps at least 16 workgroups per compute unit, for
// FP32 products at 32-row tiles only, where the read-modify-writes cost
// the gradient kernel nothing measurable (256-chain MLP: 79.7 against
// 79.7 ms, k_update 1.91 -> 0.25 ms); the 16-row instance ran 77.1 ms
// against 72.3 ungrouped (two resident workgroups per compute unit), more
// than k_update saves, and the loop's registers cost a third of the BF16
// kernel.
// HMC_TILE_GROUP (1, 2, 4 or 8) overrides the size where groups apply.
int tile_group(int prec, int R, int chains, int tiles) {
    if (prec != HMC_FP32 || R != 32) return 1;
    if (const char* s = std::getenv("HMC_TILE_GROUP")) {
        const int g = std::atoi(s);
        if (g == 1 || g == 2 || g == 4 || g == 8) return g;
    }
    int g = 1;
    while (g < 8 && (long long)chains * ((tiles + 2 * g - 1) / (2 * g)) >= 16 * 256) g *= 2;
    return g;
}

// Whether a tower may take the dense weight-gradient product on some layer
// (so that its kernels need the per-wave scratch): BF16 and split-BF16
// layers at least 64 wide on both sides, or any layer when dense is forced.
bool dense_possible(const std::vector<int>& w, int prec, bool forced) {
    if (forced) return true;
    if (prec != HMC_BF16 && prec != HMC_BF16X3) return false;
    for (size_t l = 0; l + 1 < w.size(); ++l)
        if (w[l] >= 64 && w[l + 1] >= 64) return true;
    return false;
}

// Dense weight-gradient unit of a layer (the selection lists are laid out
// for it): P >= 2 with enough 4 x 2 units for every wave takes 4 x 2 blocks
// (interleaved for BF16 with whole 64 x 32 units and no squared terms),
// otherwise 2 x 2.  NI, NJ: padded output and input widths in 16-blocks.
int dw_variant(int prec, int NI, int NJ, int nwave, bool sq) {
    if (prec >= HMC_BF16 && (NI / 4) * ((NJ + 1) / 2) >= nwave) {
        if (prec == HMC_BF16 && !sq && NI % 4 == 0 && NJ % 2 == 0) return DWV_IL;
        return DWV_4X2;
    }
    return DWV_2X2;
}

hmc_status launch_grad(hmc_ctx* x, hipStream_t s) {
    const int P = x->prec;
    if (x->kind == HMC_MLP) {
        HMC_HIP(x, hmc_launch_mlp_grad(P, x->Ra, x->nt_a, x->ga, x->grid_mlp, x->lds_a, s));
    } else {
        HMC_HIP(x, hmc_launch_trunk_fwd(P, x->Rb, x->nt_b, x->ga, x->grid_b, x->lds_b, s));
        HMC_HIP(x, hmc_launch_branch_grad(P, x->Ra, x->nt_a, x->ga, x->grid_a, x->lds_a, s));
        HMC_HIP(x, hmc_launch_trunk_bwd(P, x->Rb, x->nt_b, x->ga, x->grid_b, x->lds_b, s));
    }
    return HMC_OK;
}

// Threads per entry of k_update: with 32 or more tiles (four or more rounds
// of eight loads per thread), enough that each sums at most eight, while
// the grid stays under about two million threads; larger reductions are
// bound by HBM bandwidth, not by the latency of the tile loop, and short
// ones (16 tiles on the DeepONet branch: 4.3 against 5.8 us) do not repay
// the exchange through LDS.  Both keep one thread per entry.
int update_sub(const hmc_ctx* x) {
    const int nt = std::max(x->sa.tiles_a, x->sa.tiles_b);
    int sub = 1;
    if (nt < 32) return 1;
    while (sub < 8 && nt > 8 * sub && (long long)x->C * x->max_n * sub * 2 <= (2LL << 20)) sub *= 2;
    return sub;
}
int update_grid(const hmc_ctx* x) { return (x->max_n + 256 / x->upd_sub - 1) / (256 / x->upd_sub); }

// FP32 energy pass of BF16 and split-BF16 engines: the likelihood partials that define U in
// the Hamiltonian, at the current positions.
hmc_status launch_energy(hmc_ctx* x, hipStream_t s) {
    if (!x->energy32) return HMC_OK;
    if (x->kind == HMC_MLP) {
        HMC_HIP(x, hmc_launch_mlp_energy(x->eprec, x->Ra32, x->nt_a32, x->ga32, x->grid_a32, x->lds_a32, s));
    } else {
        HMC_HIP(x, hmc_launch_trunk_fwd(x->eprec, x->Rb32, x->nt_b32, x->ga32, x->grid_b32, x->lds_b32, s));
        HMC_HIP(x, hmc_launch_branch_energy(x->eprec, x->Ra32, x->nt_a32, x->ga32, x->grid_a32, x->lds_a32, s));
    }
    return HMC_OK;
}

// Gradient and U at the current positions (no kick).
hmc_status launch_refresh(hmc_ctx* x, hipStream_t s) {
    HMC_TRY(launch_grad(x, s));
    HMC_HIP(x, hmc_launch_update(x->prec, x->sa, UPD_GRAD, update_grid(x), x->upd_sub, s));
    HMC_TRY(launch_energy(x, s));
    HMC_HIP(x, hmc_launch_traj_end(x->prec, x->sa, END_ENERGY, s));
    return HMC_OK;
}

// Leapfrog part of a trajectory: begin (refresh or injected momentum, first
// half kick and drift), then L gradient evaluations each followed by a kick;
// all but the last kick are full steps followed by a drift.  The FP32 weight
// copy of the energy pass is written by the first drift (k_traj_begin) and
// the last one only: the energy pass reads it at theta_L.
hmc_status launch_leapfrog(hmc_ctx* x, const StateArgs& sa, int L, hipStream_t s) {
    HMC_HIP(x, hmc_launch_traj_begin(x->prec, sa, s));
    if (sa.split_n) {
        // symmetric splitting: the batch kicks need the batch gradients at the
        // start, so the trajectory takes L + 1 gradient evaluations
        const int gx = (x->max_n + 255) / 256;
        HMC_TRY(launch_grad(x, s));
        HMC_HIP(x, hmc_launch_update_split(x->prec, sa, SPL_FIRST, gx, s));
        for (int t = 1; t <= L; ++t) {
            HMC_TRY(launch_grad(x, s));
            const int mode = t == L ? SPL_END : t == L - 1 ? SPL_STEP_LAST : SPL_STEP;
            HMC_HIP(x, hmc_launch_update_split(x->prec, sa, mode, gx, s));
        }
        return launch_energy(x, s);
    }
    for (int t = 1; t <= L; ++t) {
        HMC_TRY(launch_grad(x, s));
        const int mode = t == L ? UPD_HALF_KICK : t == L - 1 ? UPD_KICK_DRIFT_LAST : UPD_KICK_DRIFT;
        HMC_HIP(x, hmc_launch_update(x->prec, sa, mode, update_grid(x), x->upd_sub, s));
    }
    return launch_energy(x, s);
}

// Staggered chain halves: the trajectory graph runs the leapfrog steps of
// chains [0, C/2) and [C/2, C) as two branches on two streams, the second
// starting one gradient evaluation later, so that one half's partial sums
// and kick (k_update, bound by HBM bandwidth) run beside the other half's
// gradient kernel (bound by MFMA and LDS) instead of after it.  The chains
// are independent, so every chain's arithmetic is unchanged.  Plain
// leapfrog only, where each half's main gradient kernel still has at least
// eight workgroups per compute unit (measured: 256-chain MLP +9%, 512-wide
// DeepONet +2%; the 64-chain DeepONet, four per compute unit, lost 1%, and
// the 8-chain 2-D MLP gained under 1%); HMC_HALVES=0 turns it off, =1
// forces it.
bool halves_on(const hmc_ctx* x) {
    if (x->sa.split_n || x->C < 2) return false;
    const char* env = std::getenv("HMC_HALVES");
    if (env && !std::strcmp(env, "0")) return false;
    if (env && !std::strcmp(env, "1")) return true;
    const long long per_chain = x->kind == HMC_MLP ? x->groups_a : x->tiles_a;
    return (long long)(x->C / 2) * per_chain >= 8LL * 256;
}

hmc_status launch_leapfrog_halves(hmc_ctx* x, int L, hipStream_t s, hipStream_t s2) {
    const StateArgs& sa = x->sa;
    HMC_HIP(x, hmc_launch_traj_begin(x->prec, sa, s));
    const int h = x->C / 2;
    const int c0[2] = {0, h}, nc[2] = {h, x->C - h};
    HMC_HIP(x, hipEventRecord(x->ev_fork, s));
    HMC_HIP(x, hipStreamWaitEvent(s2, x->ev_fork, 0));
    for (int b = 0; b < 2; ++b) {
        hipStream_t st = b ? s2 : s;
        GradArgs g = x->ga;
        g.chain0 = c0[b];
        g.n_chains = nc[b];
        StateArgs u = sa;
        u.chain0 = c0[b];
        u.n_chains = nc[b];
        if (b == 1) HMC_HIP(x, hipStreamWaitEvent(s2, x->ev_stag, 0));
        for (int t = 1; t <= L; ++t) {
            if (x->kind == HMC_MLP) {
                HMC_HIP(x, hmc_launch_mlp_grad(x->prec, x->Ra, x->nt_a, g, roundup(nc[b] * x->groups_a, 8),
                                               x->lds_a, st));
            } else {
                const int ga = roundup(nc[b] * x->tiles_a, 8), gb = roundup(nc[b] * x->tiles_b, 8);
                HMC_HIP(x, hmc_launch_trunk_fwd(x->prec, x->Rb, x->nt_b, g, gb, x->lds_b, st));
                HMC_HIP(x, hmc_launch_branch_grad(x->prec, x->Ra, x->nt_a, g, ga, x->lds_a, st));
                HMC_HIP(x, hmc_launch_trunk_bwd(x->prec, x->Rb, x->nt_b, g, gb, x->lds_b, st));
            }
            if (b == 0 && t == 1) HMC_HIP(x, hipEventRecord(x->ev_stag, s));
            const int mode = t == L ? UPD_HALF_KICK : t == L - 1 ? UPD_KICK_DRIFT_LAST : UPD_KICK_DRIFT;
            HMC_HIP(x, hmc_launch_update(x->prec, u, mode, update_grid(x), x->upd_sub, st));
        }
    }
    HMC_HIP(x, hipEventRecord(x->ev_join, s2));
    HMC_HIP(x, hipStreamWaitEvent(s, x->ev_join, 0));
    return launch_energy(x, s);
}

hmc_status set_eps_active(hmc_ctx* x, const std::vector<double>& eps, const std::vector<int>& active) {
    HMC_HIP(x, hipMemcpyAsync((void*)x->sa.eps, eps.data(), sizeof(double) * x->C, hipMemcpyHostToDevice, x->stream));
    if (active != x->active_h) {
        HMC_HIP(x, hipMemcpyAsync((void*)x->sa.active, active.data(), sizeof(int) * x->C, hipMemcpyHostToDevice,
                                  x->stream));
        x->active_h = active;
    }
    return HMC_OK;
}

hmc_status check_eps(hmc_ctx* x, const double* eps, int n, int L) {
    if (!eps) return x->fail(HMC_EINVAL, "eps is NULL");
    for (int i = 0; i < n; ++i)
        if (!(eps[i] > 0) || !std::isfinite(eps[i])) return x->fail(HMC_EINVAL, "eps must be positive and finite");
    if (L < 1 || L > 1000000) return x->fail(HMC_EINVAL, "L must be in 1..1000000");
    return HMC_OK;
}

hmc_status build(hmc_ctx* x, const hmc_net_desc* net, const hmc_mask_desc* mask, const hmc_data_desc* data,
                 uint64_t seed) {
    const int prec = x->prec;
    const size_t ts = tsize_of(prec), as = asize_of(prec), ss = ssize_of(prec);
    const int pad = pad_of(prec);
    int cap = 0;
    HMC_HIP(x, hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerBlock, x->device));
    if (cap > 0) g_lds_cap = (size_t)cap;
    x->prior_sd = net->prior_sd;
    x->lik_sd = net->lik_sd;
    x->C = mask->n_chains;
    x->offs.assign(mask->offs, mask->offs + x->C + 1);
    x->nnz = x->offs[x->C];
    for (int c = 0; c < x->C; ++c) x->max_n = std::max<int>(x->max_n, (int)(x->offs[c + 1] - x->offs[c]));
    const int la = (int)x->A.w.size() - 1;
    const int lb = x->kind == HMC_DEEPONET ? (int)x->B.w.size() - 1 : 0;

    // Masked dW path overrides (tuning record, else HMC_DW) and the per-wave
    // scratch of the dense weight-gradient product, reserved for towers
    // that may take it.
    const char* dwenv = std::getenv("HMC_DW");
    const bool force_dense = x->tune.dw == 2 || (x->tune.dw == 0 && dwenv && !std::strcmp(dwenv, "dense"));
    const bool force_gather = x->tune.dw == 1 || (x->tune.dw == 0 && dwenv && !std::strcmp(dwenv, "gather"));
    const size_t scr_wg = (size_t)(pick_threads(0, x->tune.threads) / 64) * 4096;
    const size_t scr_a = !force_gather && dense_possible(x->A.w, prec, force_dense || x->force_dense) ? scr_wg : 0;
    const size_t scr_b = x->kind == HMC_DEEPONET && !force_gather &&
                                 dense_possible(x->B.w, prec, force_dense || x->force_dense) ? scr_wg : 0;
    const int kch = pad_of(prec);

    // Row tiles.
    long long rows_a, rows_b = 0;
    int nq_pad = 0;
    if (x->kind == HMC_MLP) {
        rows_a = data->n_rows;
        x->Ra = pick_rows(x->A.w, prec, (size_t)x->A.w.back() * 8, bias_bytes(x->A.w, prec, as), rows_a, x->C,
                          "HMC_ROWS_A", x->tune.rows_a, scr_a, kch, x->alias_a, prec == HMC_FP32 && !x->force_dense);
    } else {
        rows_a = data->n_u;
        rows_b = data->n_q;
        nq_pad = roundup((int)rows_b, pad);
        x->Ra = pick_rows(x->A.w, prec, (size_t)(nq_pad + lpad_of(prec)) * ts, bias_bytes(x->A.w, prec, as), rows_a,
                          x->C, "HMC_ROWS_A", x->tune.rows_a, scr_a, kch, x->alias_a);
        x->Rb = pick_rows(x->B.w, prec, 0, bias_bytes(x->B.w, prec, as), rows_b, x->C, "HMC_ROWS_B", x->tune.rows_b,
                          scr_b, kch, x->alias_b);
        if (!x->Rb)
            return x->fail(HMC_EUNSUPPORTED, x->tune.rows_b ? "trunk tower does not fit in LDS at the requested rows per tile"
                                                            : "trunk tower does not fit in LDS");
    }
    if (!x->Ra)
        return x->fail(HMC_EUNSUPPORTED, x->tune.rows_a ? "tower does not fit in LDS at the requested rows per tile"
                                                        : "tower does not fit in LDS at 16 rows per tile");
    x->tiles_a = (int)((rows_a + x->Ra - 1) / x->Ra);
    x->tiles_b = x->kind == HMC_DEEPONET ? (int)((rows_b + x->Rb - 1) / x->Rb) : 0;
    if ((long long)x->C * x->tiles_a > (1ll << 30) || (long long)x->C * x->tiles_b > (1ll << 30))
        return x->fail(HMC_EUNSUPPORTED, "grid too large");
    x->grid_a = roundup(x->C * x->tiles_a, 8);
    x->grid_b = roundup(x->C * x->tiles_b, 8);
    x->tpg = x->force_dense || x->kind != HMC_MLP ? 1 : tile_group(prec, x->Ra, x->C, x->tiles_a);
    x->groups_a = (x->tiles_a + x->tpg - 1) / x->tpg;
    x->grid_mlp = roundup(x->C * x->groups_a, 8);

    GradArgs& g = x->ga;
    fill_plan(g.ta, x->A.w, prec, x->Ra, x->alias_a);
    g.ta.seg0 = 0;
    for (int l = 0; l < la; ++l) g.ta.fo[l] = x->A.lstart[l];
    if (x->kind == HMC_DEEPONET) {
        fill_plan(g.tb, x->B.w, prec, x->Rb, x->alias_b);
        g.tb.seg0 = la;
        for (int l = 0; l < lb; ++l) g.tb.fo[l] = x->B.lstart[l];
    }

    // Per-chain weight and bias layout.
    long long wofs = 0, bofs = 0;
    auto lay = [&](TowerPlan& tp) {
        for (int l = 0; l < tp.nl; ++l) {
            const long long sz = (long long)tp.wp[l] * tp.wp[l + 1];
            tp.wo[l] = wofs; wofs += sz;
            tp.wto[l] = wofs; wofs += sz;
            tp.bo[l] = bofs; bofs += tp.wp[l + 1];
        }
    };
    lay(g.ta);
    if (x->kind == HMC_DEEPONET) lay(g.tb);
    g.b0_off = bofs;
    bofs += 1;
    g.wstride = roundupl(std::max(wofs, 1ll), 64);
    g.bstride = roundupl(bofs, 64);

    // Dense weights from theta0 (identical for every chain before the scatter).
    std::vector<unsigned char> wh((size_t)g.wstride * ts, 0), bh((size_t)g.bstride * as, 0);
    auto fill_tower = [&](std::vector<unsigned char>& buf, int bprec, const TowerPlan& tp, const TowerHost& th) {
        for (int l = 0; l < tp.nl; ++l) {
            const int in = tp.w[l], out = tp.w[l + 1];
            const long long f0 = th.lstart[l];
            for (int i = 0; i < out; ++i) {
                for (int j = 0; j < in; ++j) {
                    const double v = net->theta0[f0 + (long long)i * in + j];
                    put_t(buf, bprec, (size_t)(tp.wo[l] + (long long)i * tp.wp[l] + j), v);
                    put_t(buf, bprec, (size_t)(tp.wto[l] + (long long)j * tp.wp[l + 1] + i), v);
                }
                put_a(bh, prec, (size_t)(tp.bo[l] + i), net->theta0[f0 + (long long)out * in + i]);
            }
        }
    };
    fill_tower(wh, prec, g.ta, x->A);
    if (x->kind == HMC_DEEPONET) {
        fill_tower(wh, prec, g.tb, x->B);
        put_a(bh, prec, (size_t)g.b0_off, net->theta0[x->P - 1]);
    }
    void* wd = x->dalloc((size_t)x->C * g.wstride * ts);
    void* bd = x->dalloc((size_t)x->C * g.bstride * as);
    if (!wd || !bd) return x->fail(HMC_ENOMEM, "device allocation of the weights failed");
    for (int c = 0; c < x->C; ++c) {
        HMC_HIP(x, hipMemcpy((char*)wd + (size_t)c * g.wstride * ts, wh.data(), wh.size(), hipMemcpyHostToDevice));
        HMC_HIP(x, hipMemcpy((char*)bd + (size_t)c * g.bstride * as, bh.data(), bh.size(), hipMemcpyHostToDevice));
    }
    g.wbuf = wd;
    g.bbuf = bd;

    // Input rows, padded to whole tiles and padded widths, in the product type.
    auto upload_rows = [&](const double* src, long long rows, int w, int wp, int R, int tiles) -> void* {
        std::vector<unsigned char> h((size_t)tiles * R * wp * ts, 0);
        for (long long r = 0; r < rows; ++r)
            for (int j = 0; j < w; ++j) put_t(h, prec, (size_t)(r * wp + j), src[r * w + j]);
        void* d = x->dalloc(h.size());
        if (d && hipMemcpy(d, h.data(), h.size(), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
        return d;
    };
    double* tgt;
    if (x->kind == HMC_MLP) {
        g.xa = upload_rows(data->x, rows_a, x->A.w[0], g.ta.wp[0], x->Ra, x->tiles_a);
        const int dout = x->A.w.back();
        tgt = (double*)x->dalloc(sizeof(double) * rows_a * dout);
        if (!g.xa || !tgt) return x->fail(HMC_ENOMEM, "device allocation of the data failed");
        HMC_HIP(x, hipMemcpy(tgt, data->y, sizeof(double) * rows_a * dout, hipMemcpyHostToDevice));
        g.d_out = dout;
    } else {
        g.xa = upload_rows(data->u, rows_a, x->A.w[0], g.ta.wp[0], x->Ra, x->tiles_a);
        g.xb = upload_rows(data->yq, rows_b, x->B.w[0], g.tb.wp[0], x->Rb, x->tiles_b);
        tgt = (double*)x->dalloc(sizeof(double) * rows_a * rows_b);
        if (!g.xa || !g.xb || !tgt) return x->fail(HMC_ENOMEM, "device allocation of the data failed");
        HMC_HIP(x, hipMemcpy(tgt, data->v, sizeof(double) * rows_a * rows_b, hipMemcpyHostToDevice));
        const int pp = g.ta.wp[la];
        g.nq = (int)rows_b;
        g.nq_pad = nq_pad;
        g.nq_rows = std::max(nq_pad, x->tiles_b * x->Rb);
        g.nu_cols = roundup(x->tiles_a * x->Ra, 32);
        g.tm_stride = (long long)g.nq_rows * pp;
        g.bt_stride = (long long)pp * g.nu_cols;
        g.dgt_stride = (long long)g.nq_rows * g.nu_cols;
        g.tm = x->dalloc((size_t)x->C * g.tm_stride * ts);
        g.tt = x->dalloc((size_t)x->C * g.tm_stride * ts);
        g.btr = x->dalloc((size_t)x->C * g.bt_stride * ts);
        g.dgt = x->dalloc((size_t)x->C * g.dgt_stride * ts);
        if (!g.tm || !g.tt || !g.btr || !g.dgt) return x->fail(HMC_ENOMEM, "device allocation of the exchange buffers failed");
    }
    g.target = tgt;
    g.n_rows_a = (int)rows_a;
    g.n_rows_b = (int)rows_b;
    g.tiles_a = x->tiles_a;
    g.tiles_b = x->tiles_b;
    g.n_chains = x->C;
    g.inv_lik_var = 1.0 / (net->lik_sd * net->lik_sd);

    // LDS: activation slabs [+ output-adjoint slab] + reduction scratch +
    // per-chain tables (TileMeta) + staged biases [+ MLP targets].
    x->lds_a = tower_lds(x->A.w, prec, x->Ra, x->alias_a);
    if (x->kind == HMC_DEEPONET) {
        g.dg_off = (int)(x->lds_a / ts);
        g.dg_ld = nq_pad + lpad_of(prec);
        x->lds_a += (size_t)x->Ra * g.dg_ld * ts;
    }
    x->lds_a = (x->lds_a + 15) / 16 * 16;
    g.red_off = (int)x->lds_a;
    x->lds_a += 64;
    g.meta_lds_a = (int)x->lds_a;
    x->lds_a += HMC_META_BYTES;
    g.bias_lds_a = (int)x->lds_a;
    x->lds_a += bias_bytes(x->A.w, prec, as);
    g.y_lds = (int)x->lds_a;
    if (x->kind == HMC_MLP) x->lds_a += (size_t)x->Ra * x->A.w.back() * 8;
    if (scr_a && x->Ra % kch == 0) {
        x->lds_a = (x->lds_a + 255) / 256 * 256;
        g.ta.scr = (int)x->lds_a;
        x->lds_a += scr_a;
    }
    // The per-kernel limit is set to the device capacity (not this engine's
    // size) so that engines of different shapes in one process coexist.
    HMC_HIP(x, hmc_set_lds_limit(prec, x->Ra, g_lds_cap));
    x->nt_a = pick_threads(x->lds_a, x->tune.threads);
    if (x->kind == HMC_DEEPONET) {
        x->lds_b = (tower_lds(x->B.w, prec, x->Rb, x->alias_b) + 15) / 16 * 16 + 64;
        g.meta_lds_b = (int)x->lds_b;
        x->lds_b += HMC_META_BYTES;
        g.bias_lds_b = (int)x->lds_b;
        x->lds_b += bias_bytes(x->B.w, prec, as);
        if (scr_b && x->Rb % kch == 0) {
            x->lds_b = (x->lds_b + 255) / 256 * 256;
            g.tb.scr = (int)x->lds_b;
            x->lds_b += scr_b;
        }
        // the trunk adjoint tile's rows of the transposed output adjoint (the
        // operand of dT = dG^T B, reduced over all nu_cols functions) staged
        // in LDS when they fit beside the tower: one bulk load, issued at
        // kernel start, in place of every wave reading them from global
        // memory inside the product
        {
            const size_t off = (x->lds_b + 15) / 16 * 16;
            const int ld = g.nu_cols + lpad_of(prec);
            const size_t need = (size_t)x->Rb * ld * ts;
            g.dgt_stage = off + need <= g_lds_cap ? 1 : 0;
            if (g.dgt_stage) {
                g.dgt_lds = (int)off;
                g.dgt_lds_ld = ld;
                x->lds_b = off + need;
            }
        }
        HMC_HIP(x, hmc_set_lds_limit(prec, x->Rb, g_lds_cap));
        x->nt_b = pick_threads(x->lds_b, x->tune.threads);
    }

    // Mask tables: entry codes, per-layer segments, scatter destinations.
    const int nseg = la + lb + 2;
    std::vector<int> code((size_t)x->nnz), dst((size_t)2 * x->nnz), seg((size_t)x->C * nseg);
    std::vector<long long> lstart;   // flat start of every layer, then b0
    std::vector<const TowerPlan*> lplan;
    std::vector<int> lidx;
    for (int l = 0; l < la; ++l) { lstart.push_back(x->A.lstart[l]); lplan.push_back(&g.ta); lidx.push_back(l); }
    for (int l = 0; l < lb; ++l) { lstart.push_back(x->B.lstart[l]); lplan.push_back(&g.tb); lidx.push_back(l); }
    const long long b0_flat = x->kind == HMC_DEEPONET ? x->P - 1 : x->P;
    lstart.push_back(b0_flat);
    for (int c = 0; c < x->C; ++c) {
        const long long o = x->offs[c], n = x->offs[c + 1] - o;
        const int64_t* id = mask->idx + o;
        for (int s = 0; s < la + lb + 1; ++s)
            seg[(size_t)c * nseg + s] = (int)(std::lower_bound(id, id + n, (int64_t)lstart[s]) - id);
        seg[(size_t)c * nseg + nseg - 1] = (int)n;
        int layer = 0;
        for (long long k = 0; k < n; ++k) {
            const long long f = id[k];
            while (layer < la + lb && f >= lstart[layer + 1]) ++layer;
            const size_t e = (size_t)(o + k);
            if (layer == la + lb) {   // b0
                code[e] = 0xFFFF;
                dst[2 * e] = -(int)g.b0_off - 1;
                dst[2 * e + 1] = -1;
                continue;
            }
            const TowerPlan& tp = *lplan[layer];
            const int l = lidx[layer];
            const int in = tp.w[l], out = tp.w[l + 1];
            const long long off = f - lstart[layer];
            if (off < (long long)in * out) {
                const int i = (int)(off / in), j = (int)(off % in);
                code[e] = (i << 16) | j;
                dst[2 * e] = (int)(tp.wo[l] + (long long)i * tp.wp[l] + j);
                dst[2 * e + 1] = (int)(tp.wto[l] + (long long)j * tp.wp[l + 1] + i);
            } else {
                const int i = (int)(off - (long long)in * out);
                code[e] = (i << 16) | 0xFFFF;
                dst[2 * e] = -(int)(tp.bo[l] + i) - 1;
                dst[2 * e + 1] = -1;
            }
        }
    }
    // Per layer: where its bias entries start, and whether its weight partials
    // come from a dense tile product (MFMA over the tile rows, selected
    // entries copied out through the layer's selection list) or from
    // per-entry sums (two LDS reads and one FMA per row and entry).  Per
    // tile, the dense product costs in proportion to in*out (the product and
    // the scratch writes, whatever the tile height), the sums in proportion
    // to (selected count) * R.  Measured on MI355X: in BF16 (MFMA 16x faster
    // than FP32) the dense product halves the 256-wide MLP at 1-20% density
    // (R = 64) and is faster on the 128-wide DeepONet branch at 5% (R = 64,
    // 158 against 172 us), but the sums are faster on the trunk tiles of 32
    // rows (5% on the 128-wide trunk: 37.6 against 39.2 us; 2% on the
    // 512-wide one: 0.47 against 0.64 ms); in FP32 and FP64 the product is
    // slower than the sums at 10% density on 64-wide layers, and on narrow
    // layers (one 16-wide block) the padded product is slower in every
    // precision.  So the dense product is used for BF16 layers at least 64
    // wide on both sides where (selected count) * R >= DWK * in * out.  Split
    // BF16 sums read two values per operand, and there the product stays the
    // faster path on 32-row tiles (DeepONet branch at 5%: 371 against
    // 384 us), so it keeps the plain density rule (>= 1/128) on such layers.
    // HMC_DW=dense or HMC_DW=gather forces one path for every layer that the
    // dense product supports (tile rows a multiple of the MFMA K chunk).
    const int nlt = la + lb;
    std::vector<int> bseg((size_t)x->C * std::max(nlt, 1)), dflag((size_t)x->C * std::max(nlt, 1));
    const long long DWK = 2;   // BF16: dense when density * R >= DWK
    for (int c = 0; c < x->C; ++c) {
        const long long o = x->offs[c], n = x->offs[c + 1] - o;
        const int64_t* id = mask->idx + o;
        for (int L = 0; L < nlt; ++L) {
            const TowerPlan& tp = *lplan[L];
            const int l = lidx[L];
            const long long wend = lstart[L] + (long long)tp.w[l] * tp.w[l + 1];
            const int b = (int)(std::lower_bound(id, id + n, (int64_t)wend) - id);
            bseg[(size_t)c * nlt + L] = b;
            const long long nw = b - seg[(size_t)c * nseg + L];
            const int R = L < la ? x->Ra : x->Rb;
            const bool can = nw > 0 && R % kch == 0;
            const long long area = (long long)tp.w[l] * tp.w[l + 1];
            const bool wide = tp.w[l] >= 64 && tp.w[l + 1] >= 64;
            const bool autod = wide && ((prec == HMC_BF16 && nw * R >= DWK * area) ||
                                        (prec == HMC_BF16X3 && nw * 128 >= area));
            const bool dense = can && !force_gather && (force_dense || autod || x->force_dense);
            dflag[(size_t)c * nlt + L] = dense ? 1 : 0;
        }
    }
    // Selection lists of the dense layers.  Per (tower, layer) the unit
    // variant (dw_variant) fixes which lane holds each dW[i][j] of a unit;
    // per (chain, layer) a block of 32-bit words: for every unit half
    // h = 2 u + bj the start of its entries (2 * units + 1 offsets, padded
    // to an even count), then the entries (entry offset from the layer's
    // first entry, LDS scratch slot (bi * 64 + 16 g + li) * 4 + v) of each
    // half in CSR order.  Chains with the same mask share one block.
    for (int L = 0; L < nlt; ++L) {
        TowerPlan& tp = L < la ? g.ta : g.tb;
        const int l = L < la ? L : L - la;
        const int nt = L < la ? x->nt_a : x->nt_b;
        tp.dwv[l] = dw_variant(prec, tp.wp[l + 1] >> 4, tp.wp[l] >> 4, nt / 64, x->force_dense);
    }
    std::vector<long long> ml_off((size_t)x->C * std::max(nlt, 1), -1);
    std::vector<unsigned> ml_h;
    std::vector<int> distinct;   // first chain of each distinct mask
    for (int c = 0; c < x->C; ++c) {
        const long long o = x->offs[c], n = x->offs[c + 1] - o;
        int same = -1;
        for (int d : distinct) {
            const long long od = x->offs[d], nd = x->offs[d + 1] - od;
            if (nd == n && std::equal(mask->idx + o, mask->idx + o + n, mask->idx + od)) { same = d; break; }
        }
        if (same < 0) distinct.push_back(c);
        for (int L = 0; L < nlt; ++L) {
            if (!dflag[(size_t)c * nlt + L]) continue;
            if (same >= 0 && dflag[(size_t)same * nlt + L]) {
                ml_off[(size_t)c * nlt + L] = ml_off[(size_t)same * nlt + L];
                continue;
            }
            const TowerPlan& tp = *lplan[L];
            const int l = lidx[L];
            if (tp.scr == 0) return x->fail(HMC_EUNSUPPORTED, "internal: dense weight gradient without its LDS scratch");
            const int in = tp.w[l];
            const int NI = tp.wp[l + 1] >> 4, NJ = tp.wp[l] >> 4, var = tp.dwv[l];
            const int BI = var == DWV_2X2 ? 2 : 4;
            const int UI = var == DWV_IL ? NI / 4 : (NI + BI - 1) / BI;
            const int UJ = var == DWV_IL ? NJ / 2 : (NJ + 1) / 2;
            const int nh = 2 * UI * UJ, tabw = (nh + 2) & ~1;
            const int k0 = seg[(size_t)c * nseg + L], k1 = bseg[(size_t)c * nlt + L];
            // unit half and scratch slot of every selected weight, in CSR order
            std::vector<int> hof(k1 - k0), slot(k1 - k0), cnt(nh + 1, 0);
            for (int k = k0; k < k1; ++k) {
                const long long off = mask->idx[o + k] - lstart[L];
                const int i = (int)(off / in), j = (int)(off % in);
                int u, bj, bi, g4, li, v;
                if (var == DWV_IL) {
                    const int ri = i % 64, cj = j % 32;
                    u = (i / 64) * UJ + j / 32;
                    g4 = ri / 16; v = (ri % 16) / 4; bi = ri % 4;
                    li = cj / 2; bj = cj % 2;
                } else {
                    const int ri = i % (BI * 16), cj = j % 32;
                    u = (i / (BI * 16)) * UJ + j / 32;
                    bi = ri / 16; g4 = (ri % 16) / 4; v = ri % 4;
                    bj = cj / 16; li = cj % 16;
                }
                hof[k - k0] = 2 * u + bj;
                slot[k - k0] = (bi * 64 + 16 * g4 + li) * 4 + v;
                ++cnt[2 * u + bj + 1];
            }
            for (int h = 0; h < nh; ++h) cnt[h + 1] += cnt[h];
            const long long base = (long long)ml_h.size();
            ml_off[(size_t)c * nlt + L] = base;
            ml_h.resize(ml_h.size() + (size_t)tabw + 2 * (size_t)(k1 - k0), 0u);
            for (int h = 0; h <= nh; ++h) ml_h[(size_t)(base + h)] = (unsigned)cnt[h];
            std::vector<int> fill(cnt.begin(), cnt.end() - 1);
            for (int k = k0; k < k1; ++k) {
                const long long e = base + tabw + 2LL * fill[hof[k - k0]]++;
                ml_h[(size_t)e] = (unsigned)(k - k0);
                ml_h[(size_t)e + 1] = (unsigned)slot[k - k0];
            }
        }
    }
    if (ml_h.size() > (size_t)INT32_MAX)
        return x->fail(HMC_EUNSUPPORTED, "selection lists exceed 2^31 words");
    int* bseg_d = (int*)x->dalloc(sizeof(int) * bseg.size());
    int* dflag_d = (int*)x->dalloc(sizeof(int) * dflag.size());
    unsigned* ml_d = (unsigned*)x->dalloc(sizeof(unsigned) * std::max<size_t>(ml_h.size(), 2));
    long long* mloff_d = (long long*)x->dalloc(sizeof(long long) * ml_off.size());
    if (!bseg_d || !dflag_d || !ml_d || !mloff_d) return x->fail(HMC_ENOMEM, "device allocation of the selection lists failed");
    HMC_HIP(x, hipMemcpy(bseg_d, bseg.data(), sizeof(int) * bseg.size(), hipMemcpyHostToDevice));
    HMC_HIP(x, hipMemcpy(dflag_d, dflag.data(), sizeof(int) * dflag.size(), hipMemcpyHostToDevice));
    if (!ml_h.empty()) HMC_HIP(x, hipMemcpy(ml_d, ml_h.data(), sizeof(unsigned) * ml_h.size(), hipMemcpyHostToDevice));
    HMC_HIP(x, hipMemcpy(mloff_d, ml_off.data(), sizeof(long long) * ml_off.size(), hipMemcpyHostToDevice));
    g.bseg = bseg_d;
    g.dflag = dflag_d;
    g.nl_total = nlt;
    g.ml = ml_d;
    g.ml_off = mloff_d;
    x->dense_layers = (int)std::count(dflag.begin(), dflag.end(), 1);

    long long* offs_d = (long long*)x->dalloc(sizeof(long long) * (x->C + 1));
    int* code_d = (int*)x->dalloc(sizeof(int) * x->nnz);
    int* dst_d = (int*)x->dalloc(sizeof(int) * 2 * x->nnz);
    int* seg_d = (int*)x->dalloc(sizeof(int) * seg.size());
    int* act_d = (int*)x->dalloc(sizeof(int) * x->C);
    if (!offs_d || !code_d || !dst_d || !seg_d || !act_d) return x->fail(HMC_ENOMEM, "device allocation of the mask tables failed");
    HMC_HIP(x, hipMemcpy(offs_d, x->offs.data(), sizeof(long long) * (x->C + 1), hipMemcpyHostToDevice));
    HMC_HIP(x, hipMemcpy(code_d, code.data(), sizeof(int) * x->nnz, hipMemcpyHostToDevice));
    HMC_HIP(x, hipMemcpy(dst_d, dst.data(), sizeof(int) * 2 * x->nnz, hipMemcpyHostToDevice));
    HMC_HIP(x, hipMemcpy(seg_d, seg.data(), sizeof(int) * seg.size(), hipMemcpyHostToDevice));
    x->active_h.assign(x->C, 1);
    HMC_HIP(x, hipMemcpy(act_d, x->active_h.data(), sizeof(int) * x->C, hipMemcpyHostToDevice));
    g.active = act_d;
    g.offs = offs_d;
    g.ecode = code_d;
    g.seg = seg_d;
    g.nseg = nseg;
    g.tpg = x->tpg;
    {
        // adjoint layers: weight gradient beside the adjoint product's
        // multiplies (HMC_OVERLAP=0 runs them one after the other)
        const char* ov = std::getenv("HMC_OVERLAP");
        g.overlap = ov && !std::strcmp(ov, "0") ? 0 : 1;
    }
    g.tmax = std::max(x->groups_a, x->tiles_b);
    g.part = x->dalloc((size_t)g.tmax * x->nnz * as);
    g.ulik = (double*)x->dalloc(sizeof(double) * 8 * x->C * x->tiles_a);
    if (!g.part || !g.ulik) return x->fail(HMC_ENOMEM, "device allocation of the gradient partials failed");

    // Separate energy pass: BF16 and split-BF16 engines always (an FP32 or,
    // on request, FP64 forward pass), FP32 engines when FP64 energies are
    // requested.  Its weights are a shadow of wbuf in the energy precision
    // with the same offsets (one scatter writes both); with FP64 energies the
    // biases get an FP64 shadow too.
    // Built after every field of the product arguments is final, since the
    // energy arguments start as a copy of them.
    void* w32 = nullptr;
    void* b64 = nullptr;
    if (prec == HMC_BF16 || prec == HMC_BF16X3 || (prec == HMC_FP32 && net->energy == HMC_ENERGY_FP64)) {
        x->energy32 = true;
        x->eprec = net->energy == HMC_ENERGY_FP64 ? HMC_FP64 : HMC_FP32;
        const char* ename = x->eprec == HMC_FP64 ? "FP64" : "FP32";
        const size_t es = tsize_of(x->eprec);
        GradArgs& e = x->ga32;
        e = g;
        x->Ra32 = pick_rows_energy(g.ta, bias_bytes(x->A.w, prec, es), x->kind == HMC_MLP ? (size_t)x->A.w.back() * 8 : 0,
                                   es);
        if (!x->Ra32) return x->fail(HMC_EUNSUPPORTED, std::string("tower does not fit in LDS for the ") + ename + " energy pass");
        fill_plan_energy(e.ta, g.ta, x->Ra32);
        x->tiles_a32 = (int)((rows_a + x->Ra32 - 1) / x->Ra32);
        x->grid_a32 = roundup(x->C * x->tiles_a32, 8);
        x->lds_a32 = energy_lds(g.ta, x->Ra32, es);
        e.red_off = (int)x->lds_a32;
        x->lds_a32 += 64;
        e.bias_lds_a = (int)x->lds_a32;
        x->lds_a32 += bias_bytes(x->A.w, prec, es);
        e.y_lds = (int)x->lds_a32;
        if (x->kind == HMC_MLP) x->lds_a32 += (size_t)x->Ra32 * x->A.w.back() * 8;
        x->nt_a32 = pick_threads(x->lds_a32, x->tune.threads);
        {
            std::vector<unsigned char> w32h((size_t)g.wstride * es, 0);
            fill_tower(w32h, x->eprec, g.ta, x->A);
            if (x->kind == HMC_DEEPONET) fill_tower(w32h, x->eprec, g.tb, x->B);
            w32 = x->dalloc((size_t)x->C * g.wstride * es);
            if (!w32) return x->fail(HMC_ENOMEM, "device allocation of the energy weight shadow failed");
            for (int c = 0; c < x->C; ++c)
                HMC_HIP(x, hipMemcpy((char*)w32 + (size_t)c * g.wstride * es, w32h.data(), w32h.size(),
                                     hipMemcpyHostToDevice));
            e.wbuf = w32;
        }
        if (x->eprec == HMC_FP64) {
            // FP64 biases (and b0) in the product buffer's layout
            std::vector<unsigned char> b64h((size_t)g.bstride * 8, 0);
            auto fill_b = [&](const TowerPlan& tp, const TowerHost& th) {
                for (int l = 0; l < tp.nl; ++l) {
                    const int in = tp.w[l], out = tp.w[l + 1];
                    for (int i = 0; i < out; ++i)
                        put_a(b64h, HMC_FP64, (size_t)(tp.bo[l] + i), net->theta0[th.lstart[l] + (long long)out * in + i]);
                }
            };
            fill_b(g.ta, x->A);
            if (x->kind == HMC_DEEPONET) {
                fill_b(g.tb, x->B);
                put_a(b64h, HMC_FP64, (size_t)g.b0_off, net->theta0[x->P - 1]);
            }
            b64 = x->dalloc((size_t)x->C * g.bstride * 8);
            if (!b64) return x->fail(HMC_ENOMEM, "device allocation of the FP64 bias shadow failed");
            for (int c = 0; c < x->C; ++c)
                HMC_HIP(x, hipMemcpy((char*)b64 + (size_t)c * g.bstride * 8, b64h.data(), b64h.size(),
                                     hipMemcpyHostToDevice));
            e.bbuf = b64;
        }
        auto upload_e = [&](const double* src, long long rows, int w, int wp, int R, int tiles) -> void* {
            std::vector<unsigned char> h((size_t)tiles * R * wp * es, 0);
            for (long long r = 0; r < rows; ++r)
                for (int j = 0; j < w; ++j) put_t(h, x->eprec, (size_t)(r * wp + j), src[r * w + j]);
            void* d = x->dalloc(h.size());
            if (d && hipMemcpy(d, h.data(), h.size(), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
            return d;
        };
        e.tiles_a = x->tiles_a32;
        e.ulik = (double*)x->dalloc(sizeof(double) * 8 * x->C * x->tiles_a32);
        if (x->kind == HMC_MLP) {
            e.xa = upload_e(data->x, rows_a, x->A.w[0], g.ta.wp[0], x->Ra32, x->tiles_a32);
        } else {
            e.xa = upload_e(data->u, rows_a, x->A.w[0], g.ta.wp[0], x->Ra32, x->tiles_a32);
            x->Rb32 = pick_rows_energy(g.tb, bias_bytes(x->B.w, prec, es), 0, es);
            if (!x->Rb32) return x->fail(HMC_EUNSUPPORTED, std::string("trunk does not fit in LDS for the ") + ename + " energy pass");
            fill_plan_energy(e.tb, g.tb, x->Rb32);
            x->tiles_b32 = (int)((rows_b + x->Rb32 - 1) / x->Rb32);
            x->grid_b32 = roundup(x->C * x->tiles_b32, 8);
            x->lds_b32 = energy_lds(g.tb, x->Rb32, es) + 64;
            e.bias_lds_b = (int)x->lds_b32;
            x->lds_b32 += bias_bytes(x->B.w, prec, es);
            x->nt_b32 = pick_threads(x->lds_b32, x->tune.threads);
            e.tiles_b = x->tiles_b32;
            e.xb = upload_e(data->yq, rows_b, x->B.w[0], g.tb.wp[0], x->Rb32, x->tiles_b32);
            const int pp = g.ta.wp[la];
            e.nq_rows = std::max(nq_pad, x->tiles_b32 * x->Rb32);
            e.tm_stride = (long long)e.nq_rows * pp;
            e.tm = x->dalloc((size_t)x->C * e.tm_stride * es);
            e.tt = x->dalloc((size_t)x->C * e.tm_stride * es);
            if (!e.xb || !e.tm || !e.tt) return x->fail(HMC_ENOMEM, "device allocation of the energy pass failed");
        }
        if (!e.xa || !e.ulik) return x->fail(HMC_ENOMEM, "device allocation of the energy pass failed");
        HMC_HIP(x, hmc_set_lds_limit(x->eprec, x->Ra32, g_lds_cap));
        if (x->Rb32) HMC_HIP(x, hmc_set_lds_limit(x->eprec, x->Rb32, g_lds_cap));
    }

    // Chain state.
    StateArgs& s = x->sa;
    s.n_chains = x->C;
    s.active = act_d;
    s.offs = offs_d;
    s.seg = seg_d;
    s.nseg = nseg;
    s.seg_trunk_lo = la;
    s.seg_trunk_hi = la + lb;
    s.tiles_a = x->groups_a;  // partials per chain and tower
    s.tiles_b = x->tiles_b;
    s.tmax = g.tmax;
    x->upd_sub = update_sub(x);
    s.part = g.part;
    s.ulik = x->energy32 ? x->ga32.ulik : g.ulik;
    s.ulik_tiles = x->energy32 ? x->tiles_a32 : x->tiles_a;
    s.wbuf32 = w32;
    s.w32_f64 = x->eprec == HMC_FP64 ? 1 : 0;
    s.bbuf64 = b64;
    s.dst = dst_d;
    s.wbuf = wd;
    s.wstride = g.wstride;
    s.bbuf = bd;
    s.bstride = g.bstride;
    s.inv_prior_var = 1.0 / (net->prior_sd * net->prior_sd);
    s.seed = seed;
    const size_t sb = (size_t)x->nnz * ss;
    s.theta = x->dalloc(sb);
    s.mom = x->dalloc(sb);
    s.grad = x->dalloc(sb);
    s.theta_save = x->dalloc(sb);
    s.grad_save = x->dalloc(sb);
    x->pin = x->dalloc(sb);
    x->ptmp = x->dalloc(sb);
    s.eps = (double*)x->dalloc(sizeof(double) * x->C);
    s.da = (double*)x->dalloc(sizeof(double) * 4 * x->C);
    s.adapt_on = (const int*)x->dalloc(sizeof(int));
    s.da_cfg = (const double*)x->dalloc(sizeof(double) * 4);
    s.U = (double*)x->dalloc(sizeof(double) * x->C);
    s.U_save = (double*)x->dalloc(sizeof(double) * x->C);
    s.H0 = (double*)x->dalloc(sizeof(double) * x->C);
    s.H1 = (double*)x->dalloc(sizeof(double) * x->C);
    s.iter = (unsigned long long*)x->dalloc(sizeof(unsigned long long) * x->C);
    s.stats = x->dalloc(sizeof(hmc_traj_stat) * x->C);
    s.n_acc = (long long*)x->dalloc(sizeof(long long) * x->C);
    s.n_div = (long long*)x->dalloc(sizeof(long long) * x->C);
    if (!s.theta || !s.mom || !s.grad || !s.theta_save || !s.grad_save || !x->pin || !x->ptmp || !s.eps || !s.da ||
        !s.adapt_on || !s.da_cfg || !s.U ||
        !s.U_save || !s.H0 || !s.H1 || !s.iter || !s.stats || !s.n_acc || !s.n_div)
        return x->fail(HMC_ENOMEM, "device allocation of the chain state failed");
    std::vector<unsigned char> th(sb);
    for (long long e = 0; e < x->nnz; ++e) {
        const double v = mask->theta_init ? mask->theta_init[e] : net->theta0[mask->idx[e]];
        if (prec == HMC_FP64) std::memcpy(&th[e * 8], &v, 8);
        else { const float f = (float)v; std::memcpy(&th[e * 4], &f, 4); }
    }
    HMC_HIP(x, hipMemcpy(s.theta, th.data(), sb, hipMemcpyHostToDevice));
    if (net->inv_mass_diag) {
        void* m = x->dalloc(sb);
        if (!m) return x->fail(HMC_ENOMEM, "device allocation of the mass matrix failed");
        for (long long e = 0; e < x->nnz; ++e) {
            const double v = net->inv_mass_diag[mask->idx[e]];
            if (prec == HMC_FP64) std::memcpy(&th[e * 8], &v, 8);
            else { const float f = (float)v; std::memcpy(&th[e * 4], &f, 4); }
        }
        HMC_HIP(x, hipMemcpy(m, th.data(), sb, hipMemcpyHostToDevice));
        s.minv = m;
    }
    HMC_HIP(x, hipEventCreate(&x->ev0));
    HMC_HIP(x, hipEventCreate(&x->ev1));
    HMC_HIP(x, hipStreamCreateWithFlags(&x->cap_stream, hipStreamNonBlocking));
    HMC_HIP(x, hipStreamCreateWithFlags(&x->cap_stream2, hipStreamNonBlocking));
    HMC_HIP(x, hipEventCreateWithFlags(&x->ev_fork, hipEventDisableTiming));
    HMC_HIP(x, hipEventCreateWithFlags(&x->ev_stag, hipEventDisableTiming));
    HMC_HIP(x, hipEventCreateWithFlags(&x->ev_join, hipEventDisableTiming));
    x->halves = halves_on(x) ? 1 : 0;

    // Scatter the starting positions and evaluate U and the gradient there.
    // A sensitivity engine samples nothing: its weights are theta0 already
    // (every entry selected, starting at theta0), and it needs neither U nor
    // the gradient.
    if (!x->force_dense) {
        HMC_HIP(x, hmc_launch_scatter_all(prec, s, x->stream));
        HMC_TRY(launch_refresh(x, x->stream));
    }
    HMC_HIP(x, hipStreamSynchronize(x->stream));
    return HMC_OK;
}

void release(hmc_ctx* x) {
    if (x->stream) (void)hipStreamSynchronize(x->stream);
    if (x->gexec) (void)hipGraphExecDestroy(x->gexec);
    if (x->graph) (void)hipGraphDestroy(x->graph);
    for (void* p : x->allocs) (void)hipFree(p);
    x->allocs.clear();
    if (x->ev0) (void)hipEventDestroy(x->ev0);
    if (x->ev1) (void)hipEventDestroy(x->ev1);
    if (x->cap_stream) (void)hipStreamDestroy(x->cap_stream);
    if (x->cap_stream2) (void)hipStreamDestroy(x->cap_stream2);
    for (hipEvent_t e : {x->ev_fork, x->ev_stag, x->ev_join})
        if (e) (void)hipEventDestroy(e);
    if (x->own_stream && x->stream) (void)hipStreamDestroy(x->stream);
}

// Graph of one full iteration of Algorithm 2 for every chain, captured once
// per L.  Step sizes, active flags and iteration counters live in device
// memory, so replays need no re-capture.
hmc_status trajectory_graph(hmc_ctx* x, int L) {
    if (x->gexec && x->graph_L == L) return HMC_OK;
    if (x->gexec) { (void)hipGraphExecDestroy(x->gexec); x->gexec = nullptr; }
    if (x->graph) { (void)hipGraphDestroy(x->graph); x->graph = nullptr; }
    HMC_HIP(x, hipStreamBeginCapture(x->cap_stream, hipStreamCaptureModeThreadLocal));
    hmc_status st = x->halves ? launch_leapfrog_halves(x, L, x->cap_stream, x->cap_stream2)
                              : launch_leapfrog(x, x->sa, L, x->cap_stream);
    if (st == HMC_OK) {
        hipError_t e = hmc_launch_traj_end(x->prec, x->sa, END_METROPOLIS, x->cap_stream);
        if (e != hipSuccess) st = x->hip(e, "traj_end");
    }
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(x->cap_stream, &g);
    if (st != HMC_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    HMC_HIP(x, ec);
    x->graph = g;
    HMC_HIP(x, hipGraphInstantiate(&x->gexec, g, nullptr, nullptr, 0));
    x->graph_L = L;
    return HMC_OK;
}

}  // namespace

// =================================================================== C ABI

extern "C" {

namespace {

hmc_status init_ctx(hmc_ctx** out, const hmc_net_desc* net, const hmc_mask_desc* mask, const hmc_data_desc* data,
                    uint64_t seed, void* hip_stream, bool sens, const hmc_tuning* tune = nullptr) {
    if (!out) { g_init_error = "out is NULL"; return HMC_EINVAL; }
    *out = nullptr;
    std::string err;
    hmc_status st = validate(net, mask, data, err);
    if (st != HMC_OK) { g_init_error = err; return st; }
    hmc_ctx* x = new (std::nothrow) hmc_ctx();
    if (!x) { g_init_error = "out of host memory"; return HMC_ENOMEM; }
    x->force_dense = sens;
    if (tune) x->tune = *tune;
    x->kind = net->kind;
    x->prec = net->precision;
    x->A.w.assign(net->widths_a, net->widths_a + net->n_widths_a);
    x->P = net->n_params;
    long long f = 0;
    for (size_t l = 0; l + 1 < x->A.w.size(); ++l) {
        x->A.lstart.push_back(f);
        f += (long long)x->A.w[l] * x->A.w[l + 1] + x->A.w[l + 1];
    }
    if (x->kind == HMC_DEEPONET) {
        x->B.w.assign(net->widths_b, net->widths_b + net->n_widths_b);
        x->B.flat0 = f;
        for (size_t l = 0; l + 1 < x->B.w.size(); ++l) {
            x->B.lstart.push_back(f);
            f += (long long)x->B.w[l] * x->B.w[l + 1] + x->B.w[l + 1];
        }
    }
    hipError_t e = hipGetDevice(&x->device);
    if (e == hipSuccess) scratch_setup(x->device);   // with the engine's device current
    if (e == hipSuccess) {
        if (hip_stream) x->stream = (hipStream_t)hip_stream;
        else {
            // a blocking stream: ordered with work on the legacy default stream,
            // where PyTorch queues by default
            e = hipStreamCreate(&x->stream);
            x->own_stream = (e == hipSuccess);
        }
    }
    if (e != hipSuccess) {
        g_init_error = std::string("HIP: ") + hipGetErrorString(e);
        release(x);
        delete x;
        return HMC_EDEVICE;
    }
    st = build(x, net, mask, data, seed);
    if (st != HMC_OK) {
        g_init_error = x->err;
        release(x);
        delete x;
        return st;
    }
    *out = x;
    return HMC_OK;
}

}  // namespace

hmc_status hmc_init(hmc_ctx** out, const hmc_net_desc* net, const hmc_mask_desc* mask, const hmc_data_desc* data,
                    uint64_t seed, void* hip_stream) {
    g_init_error.clear();
    return init_ctx(out, net, mask, data, seed, hip_stream, false);
}

namespace {
hmc_status check_tuning(const hmc_tuning* t) {
    auto rows_ok = [](int r) { return r == 0 || r == 16 || r == 32 || r == 64; };
    if (!rows_ok(t->rows_a) || !rows_ok(t->rows_b)) { g_init_error = "tuning rows must be 0, 16, 32 or 64"; return HMC_EINVAL; }
    if (t->threads != 0 && t->threads != 256 && t->threads != 512) {
        g_init_error = "tuning threads must be 0, 256 or 512";
        return HMC_EINVAL;
    }
    if (t->dw < 0 || t->dw > 2) { g_init_error = "tuning dw must be 0, 1 or 2"; return HMC_EINVAL; }
    return HMC_OK;
}
}  // namespace

hmc_status hmc_init_tuned(hmc_ctx** out, const hmc_net_desc* net, const hmc_mask_desc* mask,
                          const hmc_data_desc* data, uint64_t seed, void* hip_stream, const hmc_tuning* tuning) {
    g_init_error.clear();
    if (tuning) {
        const hmc_status st = check_tuning(tuning);
        if (st != HMC_OK) return st;
    }
    return init_ctx(out, net, mask, data, seed, hip_stream, false, tuning);
}

hmc_status hmc_autotune(const hmc_net_desc* net, const hmc_mask_desc* mask, const hmc_data_desc* data,
                        int32_t reps, hmc_tuning* best, double* best_ms) {
    g_init_error.clear();
    if (!best || reps < 1) { g_init_error = "best must not be NULL and reps >= 1"; return HMC_EINVAL; }
    {
        std::string err;
        const hmc_status st = validate(net, mask, data, err);
        if (st != HMC_OK) { g_init_error = err; return st; }
    }
    const bool deep = net->kind == HMC_DEEPONET;
    std::vector<int> ra = {16, 32, 64}, rb = deep ? std::vector<int>{16, 32, 64} : std::vector<int>{0};
    double bt = -1.0;
    hmc_tuning bb{0, 0, 0, 0};
    std::string last;
    for (int a : ra)
        for (int b : rb)
            for (int th : {256, 512})
                for (int dw : {1, 2}) {
                    const hmc_tuning t{a, b, th, dw};
                    hmc_ctx* x = nullptr;
                    if (init_ctx(&x, net, mask, data, 0, nullptr, false, &t) != HMC_OK) {
                        last = g_init_error;   // e.g. a tile that does not fit in LDS
                        continue;
                    }
                    // candidates whose dense request changed nothing repeat the per-entry one
                    if (dw == 2 && x->dense_layers == 0) { hmc_destroy(x); continue; }
                    double ms[4] = {0, 0, 0, 0};
                    const hmc_status st = hmc_time_kernels(x, reps, ms);
                    if (st != HMC_OK) {
                        g_init_error = x->err;
                        hmc_destroy(x);
                        return st;
                    }
                    const double tot = ms[0] + ms[1] + ms[2] + ms[3];
                    if (bt < 0.0 || tot < bt) { bt = tot; bb = t; }
                    hmc_destroy(x);
                }
    if (bt < 0.0) {
        g_init_error = "no candidate launch shape fits: " + last;
        return HMC_EUNSUPPORTED;
    }
    *best = bb;
    if (best_ms) *best_ms = bt;
    return HMC_OK;
}

namespace {
// Factor of the Gram matrix G = F^T F of the rows of F (rows x p, row stride
// ld): vectors l_m with sum_m l_m l_m^T = G, by Cholesky with diagonal
// pivoting (G is positive semi-definite, of rank at most min(rows, p)),
// stopping when the largest remaining diagonal entry falls below 1e-13 of
// the largest initial one.  Returns the vectors as rows of [rank][ld]
// (entries past p zero).  For any vectors a_r,
// sum_rows (f_row . a)^2 = a^T G a = sum_m (l_m . a)^2, so the l_m seed
// the same sum of squared output derivatives in rank passes.
static std::vector<double> gram_factor(const std::vector<double>& F, long long rows, int p, int ld, int& rank) {
    std::vector<double> G((size_t)p * p, 0.0);
    for (long long r = 0; r < rows; ++r) {
        const double* f = F.data() + (size_t)r * ld;
        for (int i = 0; i < p; ++i)
            for (int j = i; j < p; ++j) G[(size_t)i * p + j] += f[i] * f[j];
    }
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < i; ++j) G[(size_t)i * p + j] = G[(size_t)j * p + i];
    std::vector<double> d(p), L;
    std::vector<char> used(p, 0);
    double d0 = 0.0;
    for (int i = 0; i < p; ++i) d0 = std::max(d0, d[i] = G[(size_t)i * p + i]);
    rank = 0;
    while (rank < p) {
        int piv = -1;
        for (int i = 0; i < p; ++i)
            if (!used[i] && (piv < 0 || d[i] > d[piv])) piv = i;
        if (piv < 0 || !(d[piv] > 1e-13 * d0)) break;
        std::vector<double> l((size_t)ld, 0.0);
        const double lp = std::sqrt(d[piv]);
        l[piv] = lp;
        for (int j = 0; j < p; ++j) {
            if (used[j] || j == piv) continue;
            double v = G[(size_t)j * p + piv];
            for (int m = 0; m < rank; ++m) v -= L[(size_t)m * ld + j] * L[(size_t)m * ld + piv];
            l[j] = v / lp;
        }
        used[piv] = 1;
        for (int j = 0; j < p; ++j)
            if (!used[j]) d[j] -= l[j] * l[j];
        L.insert(L.end(), l.begin(), l.end());
        ++rank;
    }
    return L;
}
}  // namespace

hmc_status hmc_sensitivity(const hmc_net_desc* net, const hmc_data_desc* data, const double* sigma, double* s2,
                           void* hip_stream) {
    g_init_error.clear();
    if (!net || !data || !sigma || !s2) { g_init_error = "net, data, sigma and s2 must not be NULL"; return HMC_EINVAL; }
    if (net->kind != HMC_MLP && net->kind != HMC_DEEPONET) { g_init_error = "kind must be MLP or DeepONet"; return HMC_EINVAL; }
    const int64_t P = net->n_params;
    if (P < 1 || P > (1ll << 30)) { g_init_error = "n_params out of range"; return HMC_EINVAL; }
    for (int64_t k = 0; k < P; ++k)
        if (!std::isfinite(sigma[k]) || sigma[k] < 0.0) { g_init_error = "sigma must be finite and >= 0"; return HMC_EINVAL; }
    // the whole parameter vector as one chain's mask; BF16 networks run in FP32
    std::vector<int64_t> offs = {0, P}, idx((size_t)P);
    for (int64_t k = 0; k < P; ++k) idx[(size_t)k] = k;
    hmc_net_desc n2 = *net;
    if (n2.precision == HMC_BF16 || n2.precision == HMC_BF16X3) n2.precision = HMC_FP32;
    n2.inv_mass_diag = nullptr;
    n2.energy = HMC_ENERGY_DEFAULT;
    hmc_mask_desc m{1, offs.data(), idx.data(), nullptr};
    // targets are not used; the engine keeps a zero array in their place
    hmc_data_desc d2 = *data;
    std::vector<double> zeros;
    if (n2.kind == HMC_MLP && !d2.y && d2.n_rows > 0 && d2.n_rows <= (1ll << 30) && n2.n_widths_a >= 2 &&
        n2.widths_a && n2.widths_a[n2.n_widths_a - 1] > 0 && n2.widths_a[n2.n_widths_a - 1] <= 4096) {
        zeros.assign((size_t)d2.n_rows * n2.widths_a[n2.n_widths_a - 1], 0.0);
        d2.y = zeros.data();
    }
    if (n2.kind == HMC_DEEPONET && !d2.v && d2.n_u > 0 && d2.n_q > 0 && d2.n_u <= (1ll << 24) && d2.n_q <= (1ll << 24)) {
        zeros.assign((size_t)d2.n_u * d2.n_q, 0.0);
        d2.v = zeros.data();
    }
    hmc_ctx* x = nullptr;
    hmc_status st = init_ctx(&x, &n2, &m, &d2, 0, hip_stream, true);
    if (st != HMC_OK) return st;
    auto done = [&](hmc_status r) {
        if (r != HMC_OK) g_init_error = x->err;
        hmc_destroy(x);
        return r;
    };
    const size_t ts = tsize_of(x->prec);
    const int la = (int)x->A.w.size() - 1;
    const int wpo = x->ga.ta.wp[la];
    const bool deep = x->kind == HMC_DEEPONET;
    const long long rows_a = deep ? data->n_u : data->n_rows, rows_b = deep ? data->n_q : 0;
    double* acc = (double*)x->dalloc(sizeof(double) * P);
    double* sig = (double*)x->dalloc(sizeof(double) * P);
    double* s2d = (double*)x->dalloc(sizeof(double) * P);
    // seeds: MLP, the unit vectors of the outputs; DeepONet, the trunk
    // features T_q (branch passes) and the branch features B_j (trunk passes)
    const long long nseed_a = deep ? rows_b : x->A.w.back();
    void* seed_a = x->dalloc((size_t)nseed_a * wpo * ts);
    void* seed_b = deep ? x->dalloc((size_t)rows_a * wpo * ts) : nullptr;
    if (!acc || !sig || !s2d || !seed_a || (deep && !seed_b))
        return done(x->fail(HMC_ENOMEM, "device allocation of the sensitivity buffers failed"));
    hipError_t e = hipMemcpyAsync(sig, sigma, sizeof(double) * P, hipMemcpyHostToDevice, x->stream);
    const int P_ = x->prec;
    const GradArgs& g = x->ga;
    if (!deep) {
        std::vector<unsigned char> h((size_t)nseed_a * wpo * ts, 0);
        for (long long o = 0; o < nseed_a; ++o) put_t(h, P_, (size_t)(o * wpo + o), 1.0);
        if (e == hipSuccess) e = hipMemcpyAsync(seed_a, h.data(), h.size(), hipMemcpyHostToDevice, x->stream);
        for (long long o = 0; o < nseed_a && e == hipSuccess; ++o) {
            e = hmc_launch_tower_sens(P_, x->Ra, x->nt_a, g, 0, (const char*)seed_a + (size_t)o * wpo * ts, x->grid_a,
                                      x->lds_a, x->stream);
            if (e == hipSuccess)
                e = hmc_launch_sens_reduce(P_, g.part, x->tiles_a, P, 0, P, acc, sig, 1.0 / (double)rows_a,
                                           o == nseed_a - 1 ? s2d : nullptr, x->stream);
        }
    } else {
        const long long nb = x->B.flat0;   // entries of the branch tower come first, b0 last
        if (e == hipSuccess) e = hmc_launch_tower_out(P_, x->Rb, x->nt_b, g, 1, seed_a, wpo, x->grid_b, x->lds_b, x->stream);
        if (e == hipSuccess) e = hmc_launch_tower_out(P_, x->Ra, x->nt_a, g, 0, seed_b, wpo, x->grid_a, x->lds_a, x->stream);
        // When a tower has more feature rows than features, seed its passes
        // with the factor of the features' Gram matrix instead of the rows:
        // the same sums in at most p passes (1000 trunk passes become 128 on
        // the antiderivative workload).
        long long npass_a = rows_b, npass_b = rows_a;
        auto refactor = [&](void* seed, long long rows, long long& npass) {
            const int p = x->A.w.back();
            if (e != hipSuccess || rows <= p) return;
            std::vector<unsigned char> raw((size_t)rows * wpo * ts);
            e = hipMemcpyAsync(raw.data(), seed, raw.size(), hipMemcpyDeviceToHost, x->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(x->stream);
            if (e != hipSuccess) return;
            std::vector<double> F((size_t)rows * wpo);
            for (size_t i = 0; i < F.size(); ++i) {
                if (ts == 8) std::memcpy(&F[i], &raw[i * 8], 8);
                else { float f; std::memcpy(&f, &raw[i * 4], 4); F[i] = f; }
            }
            int rank = 0;
            const std::vector<double> L = gram_factor(F, rows, p, wpo, rank);
            std::vector<unsigned char> h((size_t)std::max(rank, 1) * wpo * ts, 0);
            for (int m = 0; m < rank; ++m)
                for (int k = 0; k < p; ++k) put_t(h, P_, (size_t)m * wpo + k, L[(size_t)m * wpo + k]);
            e = hipMemcpyAsync(seed, h.data(), h.size(), hipMemcpyHostToDevice, x->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(x->stream);   // h is released on return
            npass = rank;
        };
        refactor(seed_a, rows_b, npass_a);
        refactor(seed_b, rows_a, npass_b);
        for (long long q = 0; q < npass_a && e == hipSuccess; ++q) {
            e = hmc_launch_tower_sens(P_, x->Ra, x->nt_a, g, 0, (const char*)seed_a + (size_t)q * wpo * ts, x->grid_a,
                                      x->lds_a, x->stream);
            if (e == hipSuccess) e = hmc_launch_sens_reduce(P_, g.part, x->tiles_a, P, 0, nb, acc, sig, 0.0, nullptr, x->stream);
        }
        for (long long j = 0; j < npass_b && e == hipSuccess; ++j) {
            e = hmc_launch_tower_sens(P_, x->Rb, x->nt_b, g, 1, (const char*)seed_b + (size_t)j * wpo * ts, x->grid_b,
                                      x->lds_b, x->stream);
            if (e == hipSuccess)
                e = hmc_launch_sens_reduce(P_, g.part, x->tiles_b, P, nb, P - 1, acc, sig, 0.0, nullptr, x->stream);
        }
        // dF/db0 = 1 on every (function, query point) entry
        const double nb0 = (double)rows_a * (double)rows_b;
        if (e == hipSuccess) e = hipMemcpyAsync(acc + (P - 1), &nb0, sizeof(double), hipMemcpyHostToDevice, x->stream);
        if (e == hipSuccess)
            e = hmc_launch_sens_reduce(P_, g.part, 0, P, 0, P, acc, sig, 1.0 / (double)rows_a, s2d, x->stream);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(s2, s2d, sizeof(double) * P, hipMemcpyDeviceToHost, x->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(x->stream);
    if (e != hipSuccess) return done(x->fail(HMC_EDEVICE, std::string("HIP: ") + hipGetErrorString(e)));
    return done(HMC_OK);
}

namespace {

// Device buffers of one prediction call: from hipMalloc (freed on return),
// or carved in order from a fixed region (no allocation).
struct PredictBuffers {
    char* region = nullptr;        // fixed region, or null: allocate
    size_t cap = 0, used = 0;
    std::vector<void*> owned;
    void* get(size_t bytes) {
        bytes = (std::max<size_t>(bytes, 16) + 255) / 256 * 256;
        if (region) {
            if (used + bytes > cap) return nullptr;
            void* p = region + used;
            used += bytes;
            return p;
        }
        void* d = nullptr;
        if (hipMalloc(&d, bytes) != hipSuccess) return nullptr;
        owned.push_back(d);
        return d;
    }
    ~PredictBuffers() { for (void* d : owned) (void)hipFree(d); }
};

hmc_status predict_check(hmc_ctx* x, int32_t chain, const void* samples, int64_t n_samples,
                         const hmc_data_desc* inputs, const double* mean) {
    const bool deep = x->kind == HMC_DEEPONET;
    if (chain < 0 || chain >= x->C) return x->fail(HMC_EINVAL, "chain out of range");
    if (!samples || n_samples < 1) return x->fail(HMC_EINVAL, "samples must not be NULL and n_samples >= 1");
    if (!inputs) return x->fail(HMC_EINVAL, "inputs must not be NULL");
    if (!deep && (!inputs->x || inputs->n_rows < 1 || inputs->n_rows > (1ll << 30)))
        return x->fail(HMC_EINVAL, "MLP inputs need x and 1 <= n_rows <= 2^30");
    if (deep && (!inputs->u || !inputs->yq || inputs->n_u < 1 || inputs->n_q < 1 || inputs->n_u > (1ll << 24) ||
                 inputs->n_q > (1ll << 24)))
        return x->fail(HMC_EINVAL, "DeepONet inputs need u, yq and 1 <= n_u, n_q <= 2^24");
    if (!mean) return x->fail(HMC_EINVAL, "mean must not be NULL");
    return HMC_OK;
}

// The posterior predictive moments of hmc_predict with its device buffers
// from buf (cap_check: fail with HMC_EUNSUPPORTED before any device work
// when they do not fit a fixed region).
hmc_status predict_impl(hmc_ctx* x, int32_t chain, const void* samples, int64_t n_samples,
                        const hmc_data_desc* inputs, double* mean, double* var, PredictBuffers& buf) {
    HMC_TRY(predict_check(x, chain, samples, n_samples, inputs, mean));
    const bool deep = x->kind == HMC_DEEPONET;
    // engines with a separate energy pass predict through its plan (FP32 or FP64)
    const bool f32 = x->energy32;
    const int P = f32 ? x->eprec : x->prec;
    GradArgs g = f32 ? x->ga32 : x->ga;
    const int Ra = f32 ? x->Ra32 : x->Ra, Rb = f32 ? x->Rb32 : x->Rb;
    const int nta = f32 ? x->nt_a32 : x->nt_a, ntb = f32 ? x->nt_b32 : x->nt_b;
    const size_t ldsa = f32 ? x->lds_a32 : x->lds_a, ldsb = f32 ? x->lds_b32 : x->lds_b;
    const size_t ts = tsize_of(P), ss = ssize_of(x->prec), as = f32 && x->eprec == HMC_FP64 ? 8 : asize_of(x->prec);
    const long long o = x->offs[chain], nc = x->offs[chain + 1] - o;
    // new inputs in the tile layout of the training rows (padded rows and widths)
    auto tiled = [&](const double* src, long long rows, int w, int wp, int R, std::vector<unsigned char>& h) {
        const long long tiles = (rows + R - 1) / R;
        h.assign((size_t)tiles * R * wp * ts, 0);
        for (long long r = 0; r < rows; ++r)
            for (int k = 0; k < w; ++k) put_t(h, P, (size_t)(r * wp + k), src[r * w + k]);
        return (int)tiles;
    };
    const long long ra = deep ? inputs->n_u : inputs->n_rows, rb = deep ? inputs->n_q : 0;
    const int la = (int)x->A.w.size() - 1;
    const int wpo = g.ta.wp[la];
    const size_t no = deep ? (size_t)ra * rb : (size_t)ra * x->A.w.back();
    if (buf.region) {
        // the whole need, each piece rounded as get() rounds it, against the region
        auto r256 = [](size_t b) { return (std::max<size_t>(b, 16) + 255) / 256 * 256; };
        const size_t tra = (size_t)((ra + Ra - 1) / Ra) * Ra * g.ta.wp[0] * ts;
        const size_t trb = deep ? (size_t)((rb + Rb - 1) / Rb) * Rb * g.tb.wp[0] * ts : 0;
        size_t need = r256(tra) + r256((size_t)nc * ss) + r256(sizeof(double) * 3 * no);
        if (deep) need += r256(trb) + r256((size_t)ra * wpo * ts) + r256((size_t)rb * wpo * ts);
        if (need > buf.cap - buf.used)
            return x->fail(HMC_EUNSUPPORTED, "the prediction needs " + std::to_string(need) +
                                                 " bytes of device scratch, more than the fixed " +
                                                 std::to_string(buf.cap) + " bytes");
    }
    std::vector<unsigned char> ha, hb;
    const int tiles_a = tiled(deep ? inputs->u : inputs->x, ra, x->A.w[0], g.ta.wp[0], Ra, ha);
    const int tiles_b = deep ? tiled(inputs->yq, rb, x->B.w[0], g.tb.wp[0], Rb, hb) : 0;
    void* xa = buf.get(ha.size());
    void* xb = deep ? buf.get(hb.size()) : nullptr;
    void* stage = buf.get((size_t)nc * ss);
    double* mom = (double*)buf.get(sizeof(double) * 3 * no);   // mean, m2, var
    void* Bn = deep ? buf.get((size_t)ra * wpo * ts) : nullptr;
    void* Tn = deep ? buf.get((size_t)rb * wpo * ts) : nullptr;
    if (!xa || !stage || !mom || (deep && (!xb || !Bn || !Tn)))
        return x->fail(HMC_ENOMEM, "device allocation for the predictions failed");
    // one chain's weights as a one-chain argument set over the new inputs
    g.wbuf = (const char*)g.wbuf + (size_t)chain * g.wstride * ts;
    g.bbuf = (const char*)g.bbuf + (size_t)chain * g.bstride * as;
    g.n_chains = 1;
    g.xa = xa;
    g.n_rows_a = (int)ra;
    g.tiles_a = tiles_a;
    g.xb = xb;
    g.n_rows_b = (int)rb;
    g.tiles_b = tiles_b;
    const void* b0 = (const char*)g.bbuf + (size_t)g.b0_off * as;
    hipError_t e = hipMemcpyAsync(xa, ha.data(), ha.size(), hipMemcpyHostToDevice, x->stream);
    if (e == hipSuccess && deep) e = hipMemcpyAsync(xb, hb.data(), hb.size(), hipMemcpyHostToDevice, x->stream);
    if (e == hipSuccess) e = hmc_launch_zero(mom, (long long)(3 * no), x->stream);
    for (int64_t k = 0; k < n_samples && e == hipSuccess; ++k) {
        const double inv_k = 1.0 / (double)(k + 1), inv_n = 1.0 / (double)n_samples;
        double* vout = k == n_samples - 1 ? mom + 2 * no : nullptr;
        e = hipMemcpyAsync(stage, (const char*)samples + ((size_t)k * x->nnz + o) * ss, (size_t)nc * ss,
                           hipMemcpyDefault, x->stream);
        if (e == hipSuccess) e = hmc_launch_scatter_vec(x->prec, x->sa, chain, stage, nc, x->stream);
        if (e != hipSuccess) break;
        if (!deep) {
            e = hmc_launch_mlp_predict(P, Ra, nta, g, 0, roundup(tiles_a, 8), ldsa, x->stream, mom, mom + no, vout,
                                       inv_k, inv_n);
        } else {
            e = hmc_launch_tower_out(P, Rb, ntb, g, 1, Tn, wpo, roundup(tiles_b, 8), ldsb, x->stream);
            if (e == hipSuccess) e = hmc_launch_tower_out(P, Ra, nta, g, 0, Bn, wpo, roundup(tiles_a, 8), ldsa, x->stream);
            if (e == hipSuccess)
                e = hmc_launch_combine_predict(P, Bn, Tn, wpo, x->A.w.back(), ra, rb, b0, mom, mom + no, vout, inv_k,
                                               inv_n, x->stream);
        }
    }
    // the engine's own positions back into the dense weights
    if (e == hipSuccess) e = hmc_launch_scatter_all(x->prec, x->sa, x->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(mean, mom, sizeof(double) * no, hipMemcpyDeviceToHost, x->stream);
    if (e == hipSuccess && var) e = hipMemcpyAsync(var, mom + 2 * no, sizeof(double) * no, hipMemcpyDeviceToHost, x->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(x->stream);
    if (e != hipSuccess) return x->fail(HMC_EDEVICE, std::string("HIP: ") + hipGetErrorString(e));
    return HMC_OK;
}

}  // namespace

hmc_status hmc_predict(hmc_ctx* x, int32_t chain, const void* samples, int64_t n_samples,
                       const hmc_data_desc* inputs, double* mean, double* var) {
    if (!x) return HMC_EINVAL;
    PredictBuffers buf;
    return predict_impl(x, chain, samples, n_samples, inputs, mean, var, buf);
}

hmc_status hmc_predict_noalloc(hmc_ctx* x, int32_t chain, const void* samples, int64_t n_samples,
                               const hmc_data_desc* inputs, double* mean, double* var) {
    if (!x) return HMC_EINVAL;
    hipError_t err = hipSuccess;
    void* p = scratch_of(x->device, &err);
    if (!p)
        return x->fail(HMC_EDEVICE, std::string("the fixed device scratch has no address on this device: ") +
                                        hipGetErrorString(err));
    PredictBuffers buf;
    buf.region = (char*)p;
    buf.cap = HMC_SCRATCH_BYTES;
    return predict_impl(x, chain, samples, n_samples, inputs, mean, var, buf);
}

hmc_status hmc_select_mask(const double* s2, int64_t n, double tau, int64_t* idx, int64_t* n_sel) {
    g_init_error.clear();
    if (!s2 || !idx || !n_sel || n < 1) { g_init_error = "s2, idx and n_sel must not be NULL and n >= 1"; return HMC_EINVAL; }
    if (!(tau >= 0.0 && tau <= 1.0)) { g_init_error = "tau must lie in [0, 1]"; return HMC_EINVAL; }
    for (int64_t k = 0; k < n; ++k)
        if (!std::isfinite(s2[k]) || s2[k] < 0.0) { g_init_error = "sensitivities must be finite and >= 0"; return HMC_EINVAL; }
    // most sensitive first, equal values in index order
    std::vector<int64_t> ord((size_t)n);
    for (int64_t k = 0; k < n; ++k) ord[(size_t)k] = k;
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return s2[a] > s2[b]; });
    double total = 0.0;
    for (int64_t k = 0; k < n; ++k) total += s2[ord[(size_t)k]];
    if (!(total > 0.0)) { g_init_error = "the sensitivities sum to zero"; return HMC_EINVAL; }
    // the largest count whose cumulative share is at most tau
    int64_t cnt = 0;
    double cum = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        cum += s2[ord[(size_t)k]];
        if (cum / total <= tau) cnt = k + 1;
        else break;
    }
    std::sort(ord.begin(), ord.begin() + cnt);
    std::copy(ord.begin(), ord.begin() + cnt, idx);
    *n_sel = cnt;
    return HMC_OK;
}

hmc_status hmc_leapfrog(hmc_ctx* x, int32_t n_chains, const int32_t* chain_ids, const double* eps, int32_t L,
                        hmc_traj_stat* stats) {
    if (!x) return HMC_EINVAL;
    if (n_chains < 1 || n_chains > x->C) return x->fail(HMC_EINVAL, "n_chains out of range");
    HMC_TRY(check_eps(x, eps, n_chains, L));
    std::vector<double> e(x->C, 0.0);
    std::vector<int> act(x->C, 0);
    for (int i = 0; i < n_chains; ++i) {
        const int c = chain_ids ? chain_ids[i] : i;
        if (c < 0 || c >= x->C) return x->fail(HMC_EINVAL, "chain id out of range");
        if (act[c]) return x->fail(HMC_EINVAL, "chain id listed twice");
        act[c] = 1;
        e[c] = eps[i];
    }
    HMC_TRY(set_eps_active(x, e, act));
    HMC_TRY(launch_leapfrog(x, x->sa, L, x->stream));
    HMC_HIP(x, hmc_launch_traj_end(x->prec, x->sa, END_METROPOLIS, x->stream));
    if (stats) {
        std::vector<hmc_traj_stat> all(x->C);
        HMC_HIP(x, hipMemcpyAsync(all.data(), x->sa.stats, sizeof(hmc_traj_stat) * x->C, hipMemcpyDeviceToHost, x->stream));
        HMC_HIP(x, hipStreamSynchronize(x->stream));
        for (int i = 0; i < n_chains; ++i) stats[i] = all[chain_ids ? chain_ids[i] : i];
    }
    return HMC_OK;
}

hmc_status hmc_sample(hmc_ctx* x, int64_t n, const double* eps, int32_t L, void* samples, hmc_traj_stat* stats) {
    if (!x) return HMC_EINVAL;
    if (n < 0) return x->fail(HMC_EINVAL, "n must be non-negative");
    HMC_TRY(check_eps(x, eps, x->C, L));
    if (n == 0) return HMC_OK;
    HMC_TRY(set_eps_active(x, std::vector<double>(eps, eps + x->C), std::vector<int>(x->C, 1)));
    HMC_TRY(trajectory_graph(x, L));
    hmc_traj_stat* pinned = nullptr;
    if (stats) HMC_HIP(x, hipHostMalloc((void**)&pinned, sizeof(hmc_traj_stat) * x->C * n, hipHostMallocDefault));
    const size_t sb = (size_t)x->nnz * ssize_of(x->prec);
    hmc_status st = HMC_OK;
    for (int64_t i = 0; i < n && st == HMC_OK; ++i) {
        st = x->hip(hipGraphLaunch(x->gexec, x->stream), "hipGraphLaunch");
        if (st == HMC_OK && samples)
            st = x->hip(hipMemcpyAsync((char*)samples + i * sb, x->sa.theta, sb, hipMemcpyDefault, x->stream),
                        "copy samples");
        if (st == HMC_OK && pinned)
            st = x->hip(hipMemcpyAsync(pinned + i * x->C, x->sa.stats, sizeof(hmc_traj_stat) * x->C,
                                       hipMemcpyDeviceToHost, x->stream), "copy stats");
    }
    if (pinned) {
        const hipError_t e = hipStreamSynchronize(x->stream);
        if (st == HMC_OK) st = x->hip(e, "hipStreamSynchronize");
        if (st == HMC_OK) std::memcpy(stats, pinned, sizeof(hmc_traj_stat) * x->C * n);
        (void)hipHostFree(pinned);
    }
    return st;
}

namespace {

// Starting step size of the adaptation for every chain (the heuristic that
// Hoffman and Gelman's HMC with dual averaging starts from): from eps[c],
// one leapfrog step with the chain's next momentum (the Philox stream of
// its current iteration) gives the ratio exp(H0 - H1) (0 if not finite);
// the step size doubles while the ratio stays above 1/2, or halves while it
// stays below, and stops at the first step size where it crosses.  Each
// probe is a one-step trajectory of the still-searching chains, with no
// Metropolis step and the state restored.  At most 60 probes per chain.
hmc_status reasonable_eps(hmc_ctx* x, std::vector<double>& eps) {
    const int C = x->C;
    std::vector<int> dir(C, 0), act(C, 1);
    std::vector<double> H0(C), H1(C);
    for (int probe = 0; probe <= 60; ++probe) {
        HMC_TRY(set_eps_active(x, eps, act));
        HMC_TRY(launch_leapfrog(x, x->sa, 1, x->stream));
        HMC_HIP(x, hmc_launch_traj_end(x->prec, x->sa, END_TRAJ, x->stream));
        HMC_HIP(x, hipMemcpyAsync(H0.data(), x->sa.H0, sizeof(double) * C, hipMemcpyDeviceToHost, x->stream));
        HMC_HIP(x, hipMemcpyAsync(H1.data(), x->sa.H1, sizeof(double) * C, hipMemcpyDeviceToHost, x->stream));
        HMC_HIP(x, hmc_launch_restore(x->prec, x->sa, x->stream));
        HMC_HIP(x, hipStreamSynchronize(x->stream));
        int left = 0;
        for (int c = 0; c < C; ++c) {
            if (!act[c]) continue;
            const double d = std::isfinite(H1[c]) ? H0[c] - H1[c] : -INFINITY;   // log of the ratio
            const bool above = d > -std::log(2.0);
            if (probe == 0) dir[c] = above ? 1 : -1;
            if ((dir[c] > 0) == above && probe < 60) {
                eps[c] = dir[c] > 0 ? 2.0 * eps[c] : 0.5 * eps[c];
                ++left;
            } else {
                act[c] = 0;
            }
        }
        if (!left) break;
    }
    return HMC_OK;
}

}  // namespace

hmc_status hmc_adapt(hmc_ctx* x, int64_t n, const double* eps0, int32_t L, double target, double* eps_out) {
    if (!x) return HMC_EINVAL;
    if (n < 1) return x->fail(HMC_EINVAL, "n must be positive");
    if (!(target > 0.0 && target < 1.0)) return x->fail(HMC_EINVAL, "target must lie in (0, 1)");
    if (!eps_out) return x->fail(HMC_EINVAL, "eps_out is NULL");
    HMC_TRY(check_eps(x, eps0, x->C, L));
    std::vector<double> e1(eps0, eps0 + x->C);
    HMC_TRY(reasonable_eps(x, e1));
    // gamma, t0 and kappa of Hoffman and Gelman (2014); mu = log(10 eps_1)
    const double cfg[4] = {target, 0.05, 10.0, 0.75};
    std::vector<double> da((size_t)4 * x->C, 0.0);
    for (int c = 0; c < x->C; ++c) da[(size_t)4 * c + 3] = std::log(10.0 * e1[c]);
    const int on = 1, off = 0;
    HMC_HIP(x, hipMemcpyAsync((void*)x->sa.da_cfg, cfg, sizeof(cfg), hipMemcpyHostToDevice, x->stream));
    HMC_HIP(x, hipMemcpyAsync(x->sa.da, da.data(), sizeof(double) * da.size(), hipMemcpyHostToDevice, x->stream));
    HMC_TRY(set_eps_active(x, e1, std::vector<int>(x->C, 1)));
    HMC_TRY(trajectory_graph(x, L));
    HMC_HIP(x, hipMemcpyAsync((void*)x->sa.adapt_on, &on, sizeof(int), hipMemcpyHostToDevice, x->stream));
    hmc_status st = HMC_OK;
    for (int64_t i = 0; i < n && st == HMC_OK; ++i) st = x->hip(hipGraphLaunch(x->gexec, x->stream), "hipGraphLaunch");
    // the flag goes off before any other work, also after a failed launch
    const hmc_status s2 = x->hip(hipMemcpyAsync((void*)x->sa.adapt_on, &off, sizeof(int), hipMemcpyHostToDevice,
                                                x->stream), "adapt flag");
    HMC_TRY(st);
    HMC_TRY(s2);
    HMC_HIP(x, hipMemcpyAsync(da.data(), x->sa.da, sizeof(double) * da.size(), hipMemcpyDeviceToHost, x->stream));
    HMC_HIP(x, hipStreamSynchronize(x->stream));
    for (int c = 0; c < x->C; ++c) eps_out[c] = std::exp(da[(size_t)4 * c + 2]);
    return HMC_OK;
}

hmc_status hmc_calibrate(hmc_ctx* x, int32_t rounds, int64_t batch, const double* eps_in, int32_t L, double target,
                         double* eps_out, double* acc_out) {
    if (!x) return HMC_EINVAL;
    if (rounds < 1 || rounds > 64) return x->fail(HMC_EINVAL, "rounds must be in 1..64");
    if (batch < 1) return x->fail(HMC_EINVAL, "batch must be positive");
    if (!(target > 0.0 && target < 1.0)) return x->fail(HMC_EINVAL, "target must lie in (0, 1)");
    if (!eps_out) return x->fail(HMC_EINVAL, "eps_out is NULL");
    HMC_TRY(check_eps(x, eps_in, x->C, L));
    const int C = x->C;
    std::vector<double> lo(C, -INFINITY), hi(C, INFINITY), lx(C), acc(C, 0.0), eps(C);
    for (int c = 0; c < C; ++c) lx[c] = std::log(eps_in[c]);
    const double step = std::log(1.25);
    HMC_TRY(trajectory_graph(x, L));
    std::vector<double> da((size_t)4 * C, 0.0);
    const int on = 2, off = 0;
    for (int r = 0; r < rounds; ++r) {
        for (int c = 0; c < C; ++c) eps[c] = std::exp(lx[c]);
        std::fill(da.begin(), da.end(), 0.0);
        HMC_HIP(x, hipMemcpyAsync(x->sa.da, da.data(), sizeof(double) * da.size(), hipMemcpyHostToDevice, x->stream));
        HMC_TRY(set_eps_active(x, eps, std::vector<int>(C, 1)));
        HMC_HIP(x, hipMemcpyAsync((void*)x->sa.adapt_on, &on, sizeof(int), hipMemcpyHostToDevice, x->stream));
        hmc_status st = HMC_OK;
        for (int64_t i = 0; i < batch && st == HMC_OK; ++i)
            st = x->hip(hipGraphLaunch(x->gexec, x->stream), "hipGraphLaunch");
        const hmc_status s2 = x->hip(hipMemcpyAsync((void*)x->sa.adapt_on, &off, sizeof(int), hipMemcpyHostToDevice,
                                                    x->stream), "adapt flag");
        HMC_TRY(st);
        HMC_TRY(s2);
        HMC_HIP(x, hipMemcpyAsync(da.data(), x->sa.da, sizeof(double) * da.size(), hipMemcpyDeviceToHost, x->stream));
        HMC_HIP(x, hipStreamSynchronize(x->stream));
        // bisection in log eps on the batch mean of the acceptance probability:
        // too high -> the step size is a lower bound, too low -> an upper bound;
        // before both bounds exist the step size moves by a factor 1.25
        for (int c = 0; c < C; ++c) {
            acc[c] = da[(size_t)4 * c] > 0 ? da[(size_t)4 * c + 1] / da[(size_t)4 * c] : 0.0;
            if (acc[c] > target) lo[c] = lx[c];
            else hi[c] = lx[c];
            if (std::isfinite(lo[c]) && std::isfinite(hi[c])) lx[c] = 0.5 * (lo[c] + hi[c]);
            else lx[c] += std::isfinite(lo[c]) ? step : -step;
        }
    }
    for (int c = 0; c < C; ++c) {
        eps_out[c] = std::exp(lx[c]);
        if (acc_out) acc_out[c] = acc[c];
    }
    return HMC_OK;
}

hmc_status hmc_trajectory_length(const double* var, int64_t n, int32_t mode, double eps, int32_t* L) {
    g_init_error.clear();
    if (!var || !L || n < 1) { g_init_error = "var and L must not be NULL and n >= 1"; return HMC_EINVAL; }
    if (mode != 0 && mode != 1) { g_init_error = "mode must be 0 (largest) or 1 (median)"; return HMC_EINVAL; }
    if (!(eps > 0.0) || !std::isfinite(eps)) { g_init_error = "eps must be positive and finite"; return HMC_EINVAL; }
    std::vector<double> v(var, var + n);
    for (double a : v)
        if (!(a >= 0.0) || !std::isfinite(a)) { g_init_error = "variances must be finite and >= 0"; return HMC_EINVAL; }
    double pv;
    if (mode == 0) {
        pv = *std::max_element(v.begin(), v.end());
    } else {
        std::sort(v.begin(), v.end());
        pv = n % 2 ? v[(size_t)n / 2] : 0.5 * (v[(size_t)n / 2 - 1] + v[(size_t)n / 2]);
    }
    const double steps = std::nearbyint(3.14159265358979323846 * pv / (2.0 * eps));
    if (!(steps <= 1000000.0)) { g_init_error = "the rule gives more than 10^6 steps"; return HMC_EINVAL; }
    *L = (int32_t)std::max(1.0, steps);
    return HMC_OK;
}

hmc_status hmc_grad(hmc_ctx* x, double* U, void* g) {
    if (!x) return HMC_EINVAL;
    std::vector<int> all(x->C, 1);
    if (all != x->active_h) HMC_TRY(set_eps_active(x, std::vector<double>(x->C, 0.0), all));
    HMC_TRY(launch_refresh(x, x->stream));
    if (g) HMC_HIP(x, hipMemcpyAsync(g, x->sa.grad, (size_t)x->nnz * ssize_of(x->prec), hipMemcpyDefault, x->stream));
    if (U) HMC_HIP(x, hipMemcpyAsync(U, x->sa.U, sizeof(double) * x->C, hipMemcpyDeviceToHost, x->stream));
    HMC_HIP(x, hipStreamSynchronize(x->stream));
    return HMC_OK;
}

hmc_status hmc_trajectory(hmc_ctx* x, const void* p0, const double* eps, int32_t L, void* theta_out, void* p_out,
                          double* H0, double* H1) {
    if (!x) return HMC_EINVAL;
    if (!p0) return x->fail(HMC_EINVAL, "p0 is NULL");
    HMC_TRY(check_eps(x, eps, x->C, L));
    const size_t sb = (size_t)x->nnz * ssize_of(x->prec);
    HMC_TRY(set_eps_active(x, std::vector<double>(eps, eps + x->C), std::vector<int>(x->C, 1)));
    HMC_HIP(x, hipMemcpyAsync(x->pin, p0, sb, hipMemcpyDefault, x->stream));
    StateArgs s = x->sa;
    s.p_in = x->pin;
    HMC_TRY(launch_leapfrog(x, s, L, x->stream));
    HMC_HIP(x, hmc_launch_traj_end(x->prec, s, END_TRAJ, x->stream));
    if (theta_out) HMC_HIP(x, hipMemcpyAsync(theta_out, x->sa.theta, sb, hipMemcpyDefault, x->stream));
    if (p_out) HMC_HIP(x, hipMemcpyAsync(p_out, x->sa.mom, sb, hipMemcpyDefault, x->stream));
    if (H0) HMC_HIP(x, hipMemcpyAsync(H0, x->sa.H0, sizeof(double) * x->C, hipMemcpyDeviceToHost, x->stream));
    if (H1) HMC_HIP(x, hipMemcpyAsync(H1, x->sa.H1, sizeof(double) * x->C, hipMemcpyDeviceToHost, x->stream));
    HMC_HIP(x, hmc_launch_restore(x->prec, x->sa, x->stream));
    HMC_HIP(x, hipStreamSynchronize(x->stream));
    return HMC_OK;
}

hmc_status hmc_momentum(hmc_ctx* x, uint64_t iteration, void* p_out) {
    if (!x) return HMC_EINVAL;
    if (!p_out) return x->fail(HMC_EINVAL, "p_out is NULL");
    StateArgs s = x->sa;
    s.iter_override = iteration;
    s.p_out = x->ptmp;
    HMC_HIP(x, hmc_launch_momentum(x->prec, s, x->stream));
    HMC_HIP(x, hipMemcpyAsync(p_out, x->ptmp, (size_t)x->nnz * ssize_of(x->prec), hipMemcpyDefault, x->stream));
    HMC_HIP(x, hipStreamSynchronize(x->stream));
    return HMC_OK;
}

hmc_status hmc_get_state(hmc_ctx* x, void* theta_s, double* U, uint64_t* iteration) {
    if (!x) return HMC_EINVAL;
    if (theta_s)
        HMC_HIP(x, hipMemcpyAsync(theta_s, x->sa.theta, (size_t)x->nnz * ssize_of(x->prec), hipMemcpyDefault, x->stream));
    if (U) HMC_HIP(x, hipMemcpyAsync(U, x->sa.U, sizeof(double) * x->C, hipMemcpyDeviceToHost, x->stream));
    if (iteration)
        HMC_HIP(x, hipMemcpyAsync(iteration, x->sa.iter, sizeof(uint64_t) * x->C, hipMemcpyDeviceToHost, x->stream));
    HMC_HIP(x, hipStreamSynchronize(x->stream));
    return HMC_OK;
}

hmc_status hmc_set_state(hmc_ctx* x, const void* theta_s, const uint64_t* iteration) {
    if (!x) return HMC_EINVAL;
    if (!theta_s) return x->fail(HMC_EINVAL, "theta_s is NULL");
    std::vector<int> all(x->C, 1);
    if (all != x->active_h) HMC_TRY(set_eps_active(x, std::vector<double>(x->C, 0.0), all));
    HMC_HIP(x, hipMemcpyAsync(x->sa.theta, theta_s, (size_t)x->nnz * ssize_of(x->prec), hipMemcpyDefault, x->stream));
    if (iteration)
        HMC_HIP(x, hipMemcpyAsync(x->sa.iter, iteration, sizeof(uint64_t) * x->C, hipMemcpyHostToDevice, x->stream));
    HMC_HIP(x, hmc_launch_scatter_all(x->prec, x->sa, x->stream));
    HMC_TRY(launch_refresh(x, x->stream));
    HMC_HIP(x, hipStreamSynchronize(x->stream));
    return HMC_OK;
}

hmc_status hmc_set_split(hmc_ctx* x, int64_t batch_rows) {
    if (!x) return HMC_EINVAL;
    if (batch_rows < 0) return x->fail(HMC_EINVAL, "batch_rows must be non-negative");
    if (batch_rows == 0) {
        x->sa.split_n = 0;
    } else {
        if (x->kind != HMC_MLP)
            return x->fail(HMC_EUNSUPPORTED, "symmetric splitting needs an MLP (a DeepONet's trunk gradient sums over "
                                             "every input function inside one row tile)");
        if (x->tpg != 1)
            return x->fail(HMC_EUNSUPPORTED, "symmetric splitting needs one partial slot per row tile (tile groups "
                                             "are on: set HMC_TILE_GROUP=1)");
        if (batch_rows % x->Ra)
            return x->fail(HMC_EINVAL, "batch_rows must be a multiple of the rows per tile (" +
                                           std::to_string(x->Ra) + ")");
        const long long tb = batch_rows / x->Ra;
        const long long M = (x->tiles_a + tb - 1) / tb;
        if (M > HMC_SPLIT_MAX)
            return x->fail(HMC_EINVAL, "at most " + std::to_string(HMC_SPLIT_MAX) + " batches (batch_rows too small)");
        x->sa.split_n = (int)M;
        for (int m = 0; m <= M; ++m) x->sa.split_t[m] = (int)std::min<long long>(m * tb, x->tiles_a);
    }
    // the captured trajectory follows the integrator
    x->halves = halves_on(x) ? 1 : 0;
    if (x->gexec) { (void)hipGraphExecDestroy(x->gexec); x->gexec = nullptr; }
    if (x->graph) { (void)hipGraphDestroy(x->graph); x->graph = nullptr; }
    x->graph_L = -1;
    return HMC_OK;
}

hmc_status hmc_counters(hmc_ctx* x, int64_t* accepted, int64_t* divergent) {
    if (!x) return HMC_EINVAL;
    if (accepted)
        HMC_HIP(x, hipMemcpyAsync(accepted, x->sa.n_acc, sizeof(int64_t) * x->C, hipMemcpyDeviceToHost, x->stream));
    if (divergent)
        HMC_HIP(x, hipMemcpyAsync(divergent, x->sa.n_div, sizeof(int64_t) * x->C, hipMemcpyDeviceToHost, x->stream));
    HMC_HIP(x, hipStreamSynchronize(x->stream));
    return HMC_OK;
}

hmc_status hmc_get_info(const hmc_ctx* x, hmc_info_t* info) {
    if (!x || !info) return HMC_EINVAL;
    info->n_params = x->P;
    info->nnz = x->nnz;
    info->n_chains = x->C;
    info->precision = x->prec;
    info->kind = x->kind;
    info->rows_per_tile_a = x->Ra;
    info->rows_per_tile_b = x->Rb;
    info->tiles_a = x->tiles_a;
    info->tiles_b = x->tiles_b;
    info->device_bytes = x->dev_bytes;
    info->threads_a = x->nt_a;
    info->threads_b = x->kind == HMC_DEEPONET ? x->nt_b : 0;
    info->energy_precision = x->energy32 ? x->eprec : x->prec;
    info->chain_halves = x->halves;
    return HMC_OK;
}

hmc_status hmc_time_kernels(hmc_ctx* x, int32_t reps, double* ms) {
    if (!x) return HMC_EINVAL;
    if (reps < 1 || !ms) return x->fail(HMC_EINVAL, "reps must be positive and ms non-NULL");
    std::vector<int> all(x->C, 1);
    if (all != x->active_h) HMC_TRY(set_eps_active(x, std::vector<double>(x->C, 0.0), all));
    const int P = x->prec;
    for (int i = 0; i < 4; ++i) ms[i] = 0.0;
    auto timed = [&](int slot, auto&& launch) -> hmc_status {
        HMC_TRY(launch());   // warm
        HMC_HIP(x, hipEventRecord(x->ev0, x->stream));
        for (int r = 0; r < reps; ++r) HMC_TRY(launch());
        HMC_HIP(x, hipEventRecord(x->ev1, x->stream));
        HMC_HIP(x, hipEventSynchronize(x->ev1));
        float t = 0;
        HMC_HIP(x, hipEventElapsedTime(&t, x->ev0, x->ev1));
        ms[slot] = (double)t / reps;
        return HMC_OK;
    };
    if (x->kind == HMC_MLP) {
        HMC_TRY(timed(0, [&] { return launch_grad(x, x->stream); }));
    } else {
        HMC_TRY(timed(1, [&] { return x->hip(hmc_launch_trunk_fwd(P, x->Rb, x->nt_b, x->ga, x->grid_b, x->lds_b, x->stream), "trunk_fwd"); }));
        HMC_TRY(timed(0, [&] { return x->hip(hmc_launch_branch_grad(P, x->Ra, x->nt_a, x->ga, x->grid_a, x->lds_a, x->stream), "branch_grad"); }));
        HMC_TRY(timed(2, [&] { return x->hip(hmc_launch_trunk_bwd(P, x->Rb, x->nt_b, x->ga, x->grid_b, x->lds_b, x->stream), "trunk_bwd"); }));
    }
    HMC_TRY(timed(3, [&] { return x->hip(hmc_launch_update(P, x->sa, UPD_GRAD, update_grid(x), x->upd_sub, x->stream), "update"); }));
    // leave U consistent with the gradient just recomputed: BF16 and
    // split-BF16 engines define U by the FP32 energy pass, whose likelihood
    // partials still hold the end of the last trajectory (theta_L, also
    // after a rejection), so it runs again at the current positions first
    HMC_TRY(launch_energy(x, x->stream));
    HMC_HIP(x, hmc_launch_traj_end(P, x->sa, END_ENERGY, x->stream));
    HMC_HIP(x, hipStreamSynchronize(x->stream));
    return HMC_OK;
}

hmc_status hmc_sync(hmc_ctx* x) {
    if (!x) return HMC_EINVAL;
    HMC_HIP(x, hipStreamSynchronize(x->stream));
    HMC_HIP(x, hipGetLastError());
    return HMC_OK;
}

const char* hmc_last_error(const hmc_ctx* x) { return x ? x->err.c_str() : g_init_error.c_str(); }

void hmc_destroy(hmc_ctx* x) {
    if (!x) return;
    release(x);
    delete x;
}

}  // extern "C"
