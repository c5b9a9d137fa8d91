// gfx950 kernels of the masked full-batch HMC path.
//
// One leapfrog step of the sampler (Sec. 2.2, Algorithm 2) needs U and the
// gradient of U with respect to the selected entries Theta_s.  The tile
// kernels below compute them for one (chain, row tile) per workgroup:
//   forward pass of every layer (MFMA products with the bias and tanh fused
//   into the epilogue), the squared-error head in FP64, the adjoint pass with
//   the tanh derivative fused into its epilogue, and the per-tile partial
//   sums of only those weight-gradient entries that the mask selects.
// Activations never leave LDS.  Per-tile partials are then summed in a fixed
// order by the update kernel, which also applies the prior term, the kick,
// the drift and the scatter of the new positions into the dense weights.
//
// Product tiles use the 16x16 MFMA shapes of CDNA4: f64 16x16x4, f32 16x16x4
// and bf16 16x16x32 (f32 accumulation).  The split-BF16 precision stores
// each operand as the sum of two BF16 values and takes three bf16 MFMAs per
// product (see mma1 below).  Each lane supplies row (lane % 16)
// of the A operand and column (lane % 16) of the B operand with K-slots
// picked by lane / 16; it receives four accumulator rows of column lane % 16:
// rows 4 * (lane / 16) + v for f32 and bf16, rows lane / 16 + 4 v for f64
// (measured on gfx950; the f64 A rows are permuted to match the f32 layout).
// Split-BF16 operands are stored pre-split: each group of eight consecutive
// elements of a row takes 32 bytes, the eight high BF16 parts and then the
// eight low ones, so one 32-byte access gives a lane both halves of its
// fragment and the products need no conversion.
// Any K permutation that both
// operands share leaves the product unchanged, so a lane loads VEC
// consecutive K values per 16-byte (or 32-byte) access and feeds them to
// successive K-slots.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "hmc_launch.hpp"

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef __bf16 b4v __attribute__((ext_vector_type(4)));
typedef __bf16 b16v __attribute__((ext_vector_type(16), aligned(16)));

// Storage unit of one split-BF16 element (4 bytes).  Opaque on purpose:
// elements are read and written only through ld1/st1/ld4/st4 below.
struct sb3 { uint32_t bits; };

namespace {

constexpr int NWAVE = HMC_NT / 64;

template <int P> struct PT;
template <> struct PT<0> {
    typedef double T;  typedef double A;  typedef double S;
    typedef d4v Acc;   typedef d4v Frag;  typedef d4v O4;
    static constexpr int KCH = 16, VEC = 4;
};
template <> struct PT<1> {
    typedef float T;   typedef float A;   typedef float S;
    typedef f4v Acc;   typedef f4v Frag;  typedef f4v O4;
    static constexpr int KCH = 16, VEC = 4;
};
template <> struct PT<2> {
    typedef __bf16 T;  typedef float A;   typedef float S;
    typedef f4v Acc;   typedef b8v Frag;  typedef b4v O4;
    static constexpr int KCH = 32, VEC = 8;
};
// Split BF16: pre-split storage (sb3), K chunks of the bf16 MFMA; a
// fragment is the 32-byte group of eight elements, high parts then low.
template <> struct PT<3> {
    typedef sb3 T;     typedef float A;   typedef float S;
    typedef f4v Acc;   typedef b16v Frag; typedef f4v O4;
    static constexpr int KCH = 32, VEC = 8;
};

// Element access in the stored product type.  row: the start of a row
// (16-byte aligned); k: the element's index in the row.  Split BF16 keeps
// element k at BF16 slot (k / 8) * 16 + k % 8 (high part) and 8 slots on
// (low part); the split is hi = bf16(v), lo = bf16(v - hi), both rounded to
// nearest even.  A buffer whose row length is a multiple of eight may also
// be addressed with flat indices from its start.
template <int P>
__device__ __forceinline__ typename PT<P>::A ld1(const typename PT<P>::T* row, long long k) {
    if constexpr (P == 3) {
        const __bf16* b = reinterpret_cast<const __bf16*>(row) + (k >> 3) * 16 + (k & 7);
        return (float)b[0] + (float)b[8];
    } else {
        return (typename PT<P>::A)row[k];
    }
}
template <int P>
__device__ __forceinline__ void st1(typename PT<P>::T* row, long long k, typename PT<P>::A v) {
    if constexpr (P == 3) {
        __bf16* b = reinterpret_cast<__bf16*>(row) + (k >> 3) * 16 + (k & 7);
        const __bf16 h = (__bf16)v;
        b[0] = h;
        b[8] = (__bf16)(v - (float)h);
    } else {
        row[k] = (typename PT<P>::T)v;
    }
}
// Four consecutive elements n0 .. n0 + 3 (n0 a multiple of 4).
template <int P>
__device__ __forceinline__ void st4(typename PT<P>::T* row, int n0, const typename PT<P>::A (&v)[4]) {
    if constexpr (P == 3) {
        b4v h, l;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            h[e] = (__bf16)v[e];
            l[e] = (__bf16)(v[e] - (float)h[e]);
        }
        __bf16* b = reinterpret_cast<__bf16*>(row) + (n0 >> 3) * 16 + (n0 & 7);
        *reinterpret_cast<b4v*>(b) = h;
        *reinterpret_cast<b4v*>(b + 8) = l;
    } else {
        typename PT<P>::O4 o;
#pragma unroll
        for (int e = 0; e < 4; ++e) o[e] = (typename PT<P>::T)v[e];
        *reinterpret_cast<typename PT<P>::O4*>(row + n0) = o;
    }
}
template <int P>
__device__ __forceinline__ void ld4(const typename PT<P>::T* row, int n0, typename PT<P>::A (&v)[4]) {
    if constexpr (P == 3) {
        const __bf16* b = reinterpret_cast<const __bf16*>(row) + (n0 >> 3) * 16 + (n0 & 7);
        const b4v h = *reinterpret_cast<const b4v*>(b), l = *reinterpret_cast<const b4v*>(b + 8);
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (float)h[e] + (float)l[e];
    } else {
        const typename PT<P>::O4 o = *reinterpret_cast<const typename PT<P>::O4*>(row + n0);
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (typename PT<P>::A)o[e];
    }
}

__device__ __forceinline__ void mma(d4v& c, const d4v& a, const d4v& b) {
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[2], b[2], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[3], b[3], c, 0, 0, 0);
}
__device__ __forceinline__ void mma(f4v& c, const f4v& a, const f4v& b) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], c, 0, 0, 0);
}
__device__ __forceinline__ void mma(f4v& c, const b8v& a, const b8v& b) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// One MFMA of a chunk: element e of the lane's K values (FP64 and FP32 take
// four 16x16x4 MFMAs per 16-wide chunk, BF16 one 16x16x32).  NE<P> is the
// number of MFMAs per chunk.
template <int P> constexpr int NE = (P >= 2) ? 1 : 4;
__device__ __forceinline__ void mma1(d4v& c, const d4v& a, const d4v& b, int e) {
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[e], b[e], c, 0, 0, 0);
}
__device__ __forceinline__ void mma1(f4v& c, const f4v& a, const f4v& b, int e) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], b[e], c, 0, 0, 0);
}
__device__ __forceinline__ void mma1(f4v& c, const b8v& a, const b8v& b, int) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// Split BF16 (the "bf16x3" scheme of mixed-precision GEMM emulation): each
// operand x is stored as hi + lo with hi = bf16(x) and lo = bf16(x - hi)
// (unit roundoff 2^-8, so |x - hi - lo| <= 2^-16 |x|); the product sums
// hi*hi + hi*lo + lo*hi in FP32.  The dropped lo*lo term is at most 2^-16 of
// |a b|, so each product carries about 16 significant bits against 8 for a
// single BF16 product.  A fragment holds the eight high parts in elements
// 0..7 and the low parts in 8..15.
__device__ __forceinline__ void mma1(f4v& c, const b16v& a, const b16v& b, int) {
    const b8v ah = __builtin_shufflevector(a, a, 0, 1, 2, 3, 4, 5, 6, 7);
    const b8v al = __builtin_shufflevector(a, a, 8, 9, 10, 11, 12, 13, 14, 15);
    const b8v bh = __builtin_shufflevector(b, b, 0, 1, 2, 3, 4, 5, 6, 7);
    const b8v bl = __builtin_shufflevector(b, b, 8, 9, 10, 11, 12, 13, 14, 15);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Workgroup -> (chain, tile).  Consecutive workgroup ids are dealt round-robin
// to the 8 XCDs, each with its own L2; the remap gives every XCD a contiguous
// range of logical tiles so that the tiles of one chain share the L2 that
// holds that chain's weights.  The grid is padded to a multiple of 8.
__device__ __forceinline__ bool tile_of(int total, int per_chain, int& c, int& t) {
    const int w = blockIdx.x;
    const int per_xcd = gridDim.x >> 3;
    const int logical = (w & 7) * per_xcd + (w >> 3);
    if (logical >= total) return false;
    c = logical / per_chain;
    t = logical - c * per_chain;
    return true;
}

// Deterministic workgroup sum: fixed butterfly within each wave, then the
// wave sums in wave order (blockDim.x / 64 waves, at most NWAVE).  Every
// thread returns the same value.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    const int nw = (int)(blockDim.x >> 6);
    double s = scratch[0];
    for (int w = 1; w < nw; ++w) s += scratch[w];
    __syncthreads();
    return s;
}

// Copies R rows of a dense [rows][w] global block into an LDS slab of row
// stride ld, 16 bytes per access.
template <class T, int R>
__device__ __forceinline__ void load_rows(T* dst, int ld, const T* src, int w) {
    constexpr int E = 16 / sizeof(T);
    const int cpr = w / E;
    for (int i = threadIdx.x; i < R * cpr; i += blockDim.x) {
        const int r = i / cpr, q = i - r * cpr;
        *reinterpret_cast<uint4*>(dst + r * ld + q * E) =
            *reinterpret_cast<const uint4*>(src + (size_t)r * w + q * E);
    }
}

// ---------------------------------------------------------------------------
// Row blocks per unit: all R / 16 of them (each weight fragment reused over
// the whole tile) when the column blocks keep at least half the waves busy,
// else one (narrow outputs: every wave takes a row block).  Two variants
// only, to keep the kernels' code within the instruction cache.
template <int R>
__device__ __forceinline__ int nrb_of(int Np) {
    const int NB = Np >> 4;
    const int nwave = (int)(blockDim.x >> 6);
    return NB * 2 >= nwave ? R / 16 : 1;
}

// One group of four K chunks of a work unit: the weight fragments ac[q]
// (chunk q) times the LDS operand rows at xg (row stride ldx), MFMAs
// element-major over independent accumulators (the NRB row blocks, or with
// one row block the four chunk accumulators); the LDS fragments of chunk
// q + 1 are read while chunk q multiplies.
template <int P, int NRB, int KS>
__device__ __forceinline__ void gemm_group(typename PT<P>::Acc (&acc)[NRB][KS], const typename PT<P>::Frag (&ac)[4],
                                           const typename PT<P>::T* xg, int ldx) {
    typedef typename PT<P>::Frag Frag;
    constexpr int KCH = PT<P>::KCH;
    if constexpr (NRB == 1) {
        Frag b[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) b[q] = *reinterpret_cast<const Frag*>(xg + q * KCH);
#pragma unroll
        for (int e = 0; e < NE<P>; ++e)
#pragma unroll
            for (int q = 0; q < 4; ++q) mma1(acc[0][q], ac[q], b[q], e);
    } else {
        Frag bA[NRB], bB[NRB];
        auto loadB = [&](Frag (&b)[NRB], int q) {
#pragma unroll
            for (int i = 0; i < NRB; ++i) b[i] = *reinterpret_cast<const Frag*>(xg + (size_t)i * 16 * ldx + q * KCH);
        };
        auto mul = [&](const Frag (&b)[NRB], const Frag& aq) {
#pragma unroll
            for (int e = 0; e < NE<P>; ++e)
#pragma unroll
                for (int i = 0; i < NRB; ++i) mma1(acc[i][0], aq, b[i], e);
        };
        loadB(bA, 0);
        loadB(bB, 1);
        mul(bA, ac[0]);
        loadB(bA, 2);
        mul(bB, ac[1]);
        loadB(bB, 3);
        mul(bA, ac[2]);
        mul(bB, ac[3]);
    }
}

// The K % (4 chunks) remainder of a work unit: chunk by chunk from weight
// row wr and operand rows xr (both at the remainder's first column).
template <int P, int NRB, int KS>
__device__ __forceinline__ void gemm_rem(typename PT<P>::Acc (&acc)[NRB][KS], const typename PT<P>::T* wr,
                                         const typename PT<P>::T* xr, int ldx, int rem) {
    typedef typename PT<P>::Frag Frag;
    constexpr int KCH = PT<P>::KCH;
    for (int c = 0; c < rem; ++c) {
        const Frag a = *reinterpret_cast<const Frag*>(wr + c * KCH);
        Frag b[NRB];
#pragma unroll
        for (int i = 0; i < NRB; ++i) b[i] = *reinterpret_cast<const Frag*>(xr + (size_t)i * 16 * ldx + c * KCH);
#pragma unroll
        for (int e = 0; e < NE<P>; ++e)
#pragma unroll
            for (int i = 0; i < NRB; ++i) mma1(acc[i][0], a, b[i], e);
    }
}

// ---------------------------------------------------------------------------
// Tile product: for n in [0, Np) and r in [0, R)
//     out^T[n][r] = sum_{k < K} Wm[n][k] * X[r][k]
// Wm row stride ldw, X row stride ldx (LDS or global).  Work units are
// (16-column block of n, NRB 16-row blocks of r); the A fragment (weights)
// is loaded once per K chunk and reused over the NRB row blocks.  A wave
// walks its (unit, group) steps in one loop: the weight fragments of step
// s + 1 are loaded while step s multiplies (two fragment sets swapped each
// step, so the loop body, and the epilogue, appear once in the code).
template <int P, int R, int NRB, class Epi>
__device__ __forceinline__ void gemm_units(const typename PT<P>::T* __restrict__ Wm, int ldw, int K, int Np,
                                           const typename PT<P>::T* X, int ldx, Epi& epi) {
    typedef typename PT<P>::T T;
    typedef typename PT<P>::Acc Acc;
    typedef typename PT<P>::Frag Frag;
    constexpr int KCH = PT<P>::KCH, VEC = PT<P>::VEC;
    constexpr int GK = 4 * KCH;              // K extent of one group of four chunks
    constexpr int RG = (R / 16) / NRB;
    // With a single row block per unit the four chunks of a group feed four
    // separate accumulators (summed at the end), so consecutive MFMAs do not
    // wait on each other.
    constexpr int KS = NRB == 1 ? 4 : 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwave = (int)(blockDim.x >> 6);
    const int g = lane >> 4, li = lane & 15;
    // f64 16x16x4 returns accumulator rows g + 4v (f32 and bf16: 4g + v);
    // feeding A row 4 * (li % 4) + li / 4 from lane li makes the f64 outputs
    // land on rows 4g + v as well, so every epilogue sees the same layout.
    const int arow = (P == 0) ? (4 * (li & 3) + (li >> 2)) : li;
    const int units = (Np >> 4) * RG;
    const int my_units = units > wave ? (units - wave + nwave - 1) / nwave : 0;
    const int ng = K / GK;                   // full groups; K % GK chunks follow per unit
    const int rem = (K - ng * GK) / KCH;
    const int gpu = ng > 0 ? ng : 1;         // loop steps per unit (a unit with no full group still ends once)
    const int steps = my_units * gpu;
    auto wrow = [&](int ui) {
        const int u = wave + ui * nwave;
        return Wm + (size_t)((u / RG) * 16 + arow) * ldw + g * VEC;
    };
    Acc acc[NRB][KS];
#pragma unroll
    for (int i = 0; i < NRB; ++i)
#pragma unroll
        for (int q = 0; q < KS; ++q) acc[i][q] = Acc{};
    Frag ac[4], an[4];
    if (steps > 0 && ng > 0) {
        const T* wr = wrow(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) ac[q] = *reinterpret_cast<const Frag*>(wr + q * KCH);
    }
    for (int st = 0; st < steps; ++st) {
        const int ui = st / gpu, grp = st - ui * gpu;
        const int u = wave + ui * nwave;
        const int nb = u / RG, rg = u - nb * RG;
        const T* xr = X + (size_t)(rg * NRB * 16 + li) * ldx + g * VEC;
        if (ng > 0) {
            if (st + 1 < steps) {
                const int s1 = st + 1, u1 = s1 / gpu;
                const T* wr = wrow(u1) + (s1 - u1 * gpu) * GK;
#pragma unroll
                for (int q = 0; q < 4; ++q) an[q] = *reinterpret_cast<const Frag*>(wr + q * KCH);
            }
            gemm_group<P, NRB, KS>(acc, ac, xr + grp * GK, ldx);
#pragma unroll
            for (int q = 0; q < 4; ++q) ac[q] = an[q];
        }
        if (grp == gpu - 1) {
            // remaining K % GK chunks of the unit, then its epilogue
            if (rem) gemm_rem<P, NRB, KS>(acc, wrow(ui) + ng * GK, xr + ng * GK, ldx, rem);
#pragma unroll
            for (int i = 0; i < NRB; ++i) {
                Acc t = acc[i][0];
#pragma unroll
                for (int q = 1; q < KS; ++q) t += acc[i][q];
                epi((rg * NRB + i) * 16 + li, nb * 16 + 4 * g, t);
#pragma unroll
                for (int q = 0; q < KS; ++q) acc[i][q] = Acc{};
            }
        }
    }
}

template <int P, int R, class Epi>
__device__ __forceinline__ void gemm(const typename PT<P>::T* Wm, int ldw, int K, int Np,
                                     const typename PT<P>::T* X, int ldx, Epi& epi) {
    constexpr int RB = R / 16;
    if constexpr (RB > 1) {
        if (nrb_of<R>(Np) == RB) {
            gemm_units<P, R, RB>(Wm, ldw, K, Np, X, ldx, epi);
            return;
        }
    }
    gemm_units<P, R, 1>(Wm, ldw, K, Np, X, ldx, epi);
}

// Deferred tile product: the wave's work units (at most MAXU of them, the
// caller checks) multiplied into dacc with the arithmetic of gemm_units in
// the same order, the epilogues later (gemm_deferred_epi), so that other
// work can run between the two.  NRB as gemm() picks it.
template <int P, int R, int NRB>
__device__ __forceinline__ int deferred_units(int Np) {
    constexpr int RG = (R / 16) / NRB;
    const int wave = (int)(threadIdx.x >> 6), nwave = (int)(blockDim.x >> 6);
    const int units = (Np >> 4) * RG;
    return units > wave ? (units - wave + nwave - 1) / nwave : 0;
}
// ... and the most any wave of the workgroup takes (wave 0's count): the
// same in every wave, so a branch on it keeps the workgroup together
template <int P, int R, int NRB>
__device__ __forceinline__ int deferred_units_max(int Np) {
    constexpr int RG = (R / 16) / NRB;
    const int nwave = (int)(blockDim.x >> 6);
    return ((Np >> 4) * RG + nwave - 1) / nwave;
}
template <int P, int R, int NRB, int MAXU>
__device__ __forceinline__ void gemm_deferred(const typename PT<P>::T* __restrict__ Wm, int ldw, int K, int Np,
                                              const typename PT<P>::T* X, int ldx,
                                              typename PT<P>::Acc (&dacc)[MAXU][NRB]) {
    typedef typename PT<P>::T T;
    typedef typename PT<P>::Acc Acc;
    typedef typename PT<P>::Frag Frag;
    constexpr int KCH = PT<P>::KCH, VEC = PT<P>::VEC;
    constexpr int GK = 4 * KCH;
    constexpr int RG = (R / 16) / NRB;
    constexpr int KS = NRB == 1 ? 4 : 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwave = (int)(blockDim.x >> 6);
    const int g = lane >> 4, li = lane & 15;
    const int arow = (P == 0) ? (4 * (li & 3) + (li >> 2)) : li;
    const int my_units = deferred_units<P, R, NRB>(Np);
    const int ng = K / GK;
    const int rem = (K - ng * GK) / KCH;
#pragma unroll
    for (int ui = 0; ui < MAXU; ++ui) {
        if (ui < my_units) {
            const int u = wave + ui * nwave;
            const int nb = u / RG, rg = u - nb * RG;
            const T* wr = Wm + (size_t)(nb * 16 + arow) * ldw + g * VEC;
            const T* xr = X + (size_t)(rg * NRB * 16 + li) * ldx + g * VEC;
            Acc acc[NRB][KS];
#pragma unroll
            for (int i = 0; i < NRB; ++i)
#pragma unroll
                for (int q = 0; q < KS; ++q) acc[i][q] = Acc{};
            Frag ac[4], an[4];
            if (ng > 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) ac[q] = *reinterpret_cast<const Frag*>(wr + q * KCH);
            }
            for (int grp = 0; grp < ng; ++grp) {
                if (grp + 1 < ng) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) an[q] = *reinterpret_cast<const Frag*>(wr + (grp + 1) * GK + q * KCH);
                }
                gemm_group<P, NRB, KS>(acc, ac, xr + grp * GK, ldx);
#pragma unroll
                for (int q = 0; q < 4; ++q) ac[q] = an[q];
            }
            if (rem) gemm_rem<P, NRB, KS>(acc, wr + ng * GK, xr + ng * GK, ldx, rem);
#pragma unroll
            for (int i = 0; i < NRB; ++i) {
                Acc t = acc[i][0];
#pragma unroll
                for (int q = 1; q < KS; ++q) t += acc[i][q];
                dacc[ui][i] = t;
            }
        }
    }
}
template <int P, int R, int NRB, int MAXU, class Epi>
__device__ __forceinline__ void gemm_deferred_epi(int Np, const typename PT<P>::Acc (&dacc)[MAXU][NRB], Epi& epi) {
    constexpr int RG = (R / 16) / NRB;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwave = (int)(blockDim.x >> 6);
    const int g = lane >> 4, li = lane & 15;
    const int my_units = deferred_units<P, R, NRB>(Np);
#pragma unroll
    for (int ui = 0; ui < MAXU; ++ui) {
        if (ui < my_units) {
            const int u = wave + ui * nwave;
            const int nb = u / RG, rg = u - nb * RG;
#pragma unroll
            for (int i = 0; i < NRB; ++i) epi((rg * NRB + i) * 16 + li, nb * 16 + 4 * g, dacc[ui][i]);
        }
    }
}

// ---------------------------------------------------------------------------
// Epilogues.  Each receives the output row r of the tile, the first of four
// consecutive output columns n0 and the four accumulators.

// Hidden layer: a = tanh(z + b), stored in the product precision.
// Single-precision tanh as 1 - 2 / (e^{2x} + 1) with the hardware exponential
// and reciprocal: five instructions, since the epilogue is VALU-bound.  Its
// absolute error is below 2e-7 (the cancellation near 0 makes the relative
// error grow only for |x| < 1e-3, where the values, and what they contribute
// downstream, are as small): on the FP32 parity workloads the gradient moves
// by under 1e-7 relative against FP64 tanh, below the FP32 rounding of the
// products, and far below BF16 rounding.  The limits come out right: e^{2x}
// overflows to inf (result 1) or underflows to 0 (result -1).  FP64 keeps the
// library tanh.
__device__ __forceinline__ float tanh_fast(float x) {
    return 1.0f - __fdividef(2.0f, __expf(2.0f * x) + 1.0f);
}

template <int P> struct EpiTanh {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    const A* bias; T* out; int ld;
    __device__ __forceinline__ void operator()(int r, int n0, const typename PT<P>::Acc& acc) const {
        A o[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            if constexpr (P == 0) o[v] = tanh((double)acc[v] + bias[n0 + v]);
            else o[v] = tanh_fast(acc[v] + bias[n0 + v]);
        }
        st4<P>(out + r * ld, n0, o);
    }
};

// Plain store (adjoints of linear outputs).
template <int P> struct EpiStore {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    T* out; int ld;
    __device__ __forceinline__ void operator()(int r, int n0, const typename PT<P>::Acc& acc) const {
        A o[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) o[v] = (A)acc[v];
        st4<P>(out + r * ld, n0, o);
    }
};

// Adjoint through tanh: delta_in = (delta_out W) * (1 - a^2), in place over a.
template <int P> struct EpiBack {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    T* io; int ld;
    __device__ __forceinline__ void operator()(int r, int n0, const typename PT<P>::Acc& acc) const {
        A av[4], o[4];
        ld4<P>(io + r * ld, n0, av);
#pragma unroll
        for (int v = 0; v < 4; ++v) o[v] = (A)acc[v] * ((A)1 - av[v] * av[v]);
        st4<P>(io + r * ld, n0, o);
    }
};

// MLP output layer and squared-error head: F = z + b; residual in FP64;
// delta = (F - y) / lik_sd^2 replaces the output; the squared residuals of
// the valid rows accumulate per thread.  y points at the target of the
// tile's row 0 (row r of the tile at y[r * d_out]).
template <int P> struct EpiMlpHead {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    const A* bias; T* out; int ld;
    const double* y; int d_out; int row0; int nrows; double iv;
    double sq;
    __device__ __forceinline__ void operator()(int r, int n0, const typename PT<P>::Acc& acc) {
        A o[4];
        const int row = row0 + r;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int n = n0 + v;
            A d = (A)0;
            if (n < d_out && row < nrows) {
                const double res = ((double)acc[v] + (double)bias[n]) - y[r * d_out + n];
                sq += res * res;
                d = (A)(res * iv);
            }
            o[v] = d;
        }
        st4<P>(out + r * ld, n0, o);
    }
};

// Posterior predictive head: F = z + b for the valid rows and outputs, folded
// into FP64 running moments over the samples (Welford: after the k-th
// sample mean holds the mean of the first k outputs and m2 the sum of their
// squared deviations); the last sample also writes var = m2 / n.
template <int P> struct EpiPredict {
    typedef typename PT<P>::A A;
    const A* bias; int d_out; int row0; int nrows;
    double* mean; double* m2; double* var; double inv_k; double inv_n;
    __device__ __forceinline__ void operator()(int r, int n0, const typename PT<P>::Acc& acc) const {
        const int row = row0 + r;
        if (row >= nrows) return;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int n = n0 + v;
            if (n >= d_out) continue;
            const size_t i = (size_t)row * d_out + n;
            const double f = (double)acc[v] + (double)bias[n];
            const double mu = mean[i], d = f - mu, mu2 = mu + d * inv_k;
            const double q = m2[i] + d * (f - mu2);
            mean[i] = mu2;
            m2[i] = q;
            if (var) var[i] = q * inv_n;
        }
    }
};

// Branch output layer: B = z + b kept in LDS for the combination, and B^T
// written to global memory for the trunk adjoint (zero for padded rows).
template <int P> struct EpiBranchOut {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    const A* bias; T* out; int ld; T* bt; int bt_ld; int col0; int nvalid; bool store;
    __device__ __forceinline__ void operator()(int r, int n0, const typename PT<P>::Acc& acc) const {
        A o[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const A tv = (A)acc[v] + bias[n0 + v];
            o[v] = tv;
            if (store) st1<P>(bt + (size_t)(n0 + v) * bt_ld, col0 + r, (r < nvalid) ? tv : (A)0);
        }
        st4<P>(out + r * ld, n0, o);
    }
};

// Trunk output layer: T = z + b, written to global memory both as [q][k] and
// as [k][q] (zero for padded query rows).
template <int P> struct EpiTrunkOut {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    const A* bias; T* tm; int tm_ld; T* tt; int tt_ld; int row0; int nvalid;
    __device__ __forceinline__ void operator()(int r, int n0, const typename PT<P>::Acc& acc) const {
        A o[4];
        const bool ok = r < nvalid;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const A tv = ok ? (A)acc[v] + bias[n0 + v] : (A)0;
            o[v] = tv;
            st1<P>(tt + (size_t)(n0 + v) * tt_ld, row0 + r, tv);
        }
        st4<P>(tm + (size_t)(row0 + r) * tm_ld, n0, o);
    }
};

// DeepONet combination and head: G[a][q] = <B_a, T_q> + b0 arrives as the
// transposed tile (rows q, columns a); residual in FP64; the output adjoint
// dG = (G - v) / lik_sd^2 goes to an LDS slab [a][q] and to global [q][a];
// squared residuals and the b0 gradient accumulate per thread.
template <int P> struct EpiCombine {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    T* dg; int dg_ld; T* dgt; int dgt_ld; int col0;
    const double* v; int nq; int nvalid; int row0; double b0; double iv; bool store;
    double sq; double sdg;
    __device__ __forceinline__ void operator()(int r, int n0, const typename PT<P>::Acc& acc) {
        A o[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int q = n0 + w;
            A d = (A)0;
            if (q < nq && r < nvalid) {
                const double res = ((double)acc[w] + b0) - v[(size_t)(row0 + r) * nq + q];
                sq += res * res;
                const double dd = res * iv;
                sdg += dd;
                d = (A)dd;
            }
            o[w] = d;
            if (store) st1<P>(dgt + (size_t)q * dgt_ld, col0 + r, d);
        }
        if (store) st4<P>(dg + r * dg_ld, n0, o);
    }
};

// ---------------------------------------------------------------------------
// Masked weight gradient, one tile: for each selected entry k of the layer,
//   part[k] = sum_r delta[r][i_k] * a[r][j_k]     (weights)
//   part[k] = sum_r delta[r][i_k]                  (biases)
// Rows past the data hold delta = 0 and contribute nothing.  A layer with
// few entries gives each entry LPE adjacent lanes (rows r = sub mod LPE,
// then a fixed butterfly over the LPE lanes), so that short segments do not
// leave most of the workgroup idle behind one R-long chain per entry.
// SQ: the sums of squared per-row terms, delta^2 a^2 and delta^2 (the
// Jacobian square sums of the sensitivity pass).
template <bool SQ, class V> __device__ __forceinline__ V sq_if(V v) {
    if constexpr (SQ) return v * v;
    else return v;
}

// K slot e of a fragment from element k of a row (the dense weight-gradient
// operands are read one element per tile row).
template <int P, bool SQ>
__device__ __forceinline__ void frag_put(typename PT<P>::Frag& f, int e, const typename PT<P>::T* row, int k) {
    if constexpr (P == 3) {
        static_assert(!SQ, "squared terms are formed in FP32 and FP64 only");
        const __bf16* b = reinterpret_cast<const __bf16*>(row) + (k >> 3) * 16 + (k & 7);
        f[e] = b[0];
        f[e + 8] = b[8];
    } else {
        f[e] = sq_if<SQ>(row[k]);
    }
}

template <int P, int R, bool SQ = false, bool RMW = false>
__device__ __forceinline__ void dw_partials(const int* __restrict__ code, int k0, int k1,
                                            const typename PT<P>::T* D, int ld,
                                            const typename PT<P>::T* X, int lx,
                                            typename PT<P>::A* __restrict__ part, bool accum_) {
    const bool accum = RMW && accum_;   // RMW false: the accumulate paths compile out
    typedef typename PT<P>::A A;
    const int n = k1 - k0;
    if (n <= 0) return;
    const int nthr = (int)blockDim.x;
    int lpe = 1;
    while (lpe < 16 && 2 * lpe <= R && n * 2 * lpe <= nthr) lpe *= 2;
    if (lpe == 1) {
        if constexpr (RMW) {
            if (accum) {
                // adding to the running sums of the workgroup's earlier tiles
                // (this thread wrote them): four of the thread's entries at a
                // time, their codes and running sums loaded together, so that
                // the latency of those loads (from L2 or memory) is paid once
                // per four entries
                for (int kb = k0 + (int)threadIdx.x; kb < k1; kb += 4 * nthr) {
                    int cd[4];
                    A s[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int k = kb + q * nthr;
                        cd[q] = k < k1 ? code[k] : 0;
                        s[q] = k < k1 ? part[k] : (A)0;
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int k = kb + q * nthr;
                        if (k < k1) {
                            const int i = cd[q] >> 16, j = cd[q] & 0xFFFF;
                            if (j == 0xFFFF) {
#pragma unroll 8
                                for (int r = 0; r < R; ++r) s[q] += sq_if<SQ>(ld1<P>(D + r * ld, i));
                            } else {
#pragma unroll 8
                                for (int r = 0; r < R; ++r)
                                    s[q] = fma(sq_if<SQ>(ld1<P>(D + r * ld, i)), sq_if<SQ>(ld1<P>(X + r * lx, j)),
                                               s[q]);
                            }
                            part[k] = s[q];
                        }
                    }
                }
                return;
            }
        }
        // the code of the thread's next entry is loaded while this one sums,
        // so that its global latency is paid once, not once per pass
        int cn = k0 + (int)threadIdx.x < k1 ? code[k0 + threadIdx.x] : 0;
        for (int k = k0 + (int)threadIdx.x; k < k1; k += nthr) {
            const int cd = cn;
            if (k + nthr < k1) cn = code[k + nthr];
            const int i = cd >> 16, j = cd & 0xFFFF;
            A s = (A)0;
            if (j == 0xFFFF) {
#pragma unroll 8
                for (int r = 0; r < R; ++r) s += sq_if<SQ>(ld1<P>(D + r * ld, i));
            } else {
#pragma unroll 8
                for (int r = 0; r < R; ++r)
                    s = fma(sq_if<SQ>(ld1<P>(D + r * ld, i)), sq_if<SQ>(ld1<P>(X + r * lx, j)), s);
            }
            part[k] = s;
        }
        return;
    }
    // n * lpe <= nthr: one pass; every lane of a wave takes part in the
    // shuffles (lanes past the last entry sum nothing)
    const int e = (int)threadIdx.x / lpe, sub = (int)threadIdx.x - e * lpe;
    A s = (A)0;
    if (e < n) {
        const int cd = code[k0 + e];
        const int i = cd >> 16, j = cd & 0xFFFF;
        if (j == 0xFFFF) {
            for (int r = sub; r < R; r += lpe) s += sq_if<SQ>(ld1<P>(D + r * ld, i));
        } else {
            for (int r = sub; r < R; r += lpe)
                s = fma(sq_if<SQ>(ld1<P>(D + r * ld, i)), sq_if<SQ>(ld1<P>(X + r * lx, j)), s);
        }
    }
    for (int o = 1; o < lpe; o <<= 1) s += __shfl_xor(s, o, 64);
    if (e < n && sub == 0) {
        if constexpr (RMW) part[k0 + e] = accum ? part[k0 + e] + s : s;
        else part[k0 + e] = s;
    }
}

// Selection-list entries of one dense weight-gradient unit, loaded before
// its product so that their latency overlaps the MFMAs: the unit halves'
// entry ranges and each lane's first D entries of each half.  Four for the
// BF16 types; one for FP32 and FP64, whose dense path is taken only on
// request and whose registers the FP32 kernels need for their occupancy.
template <int P> constexpr int DWP = P >= 2 ? 4 : 1;
template <int D>
struct DwPre {
    int e0[2], e1[2];
    uint2 en[2][D];
};
template <int DWP>
__device__ __forceinline__ DwPre<DWP> dw_prefetch(const unsigned* __restrict__ tab, const uint2* __restrict__ ent,
                                                  int u) {
    const int lane = threadIdx.x & 63;
    DwPre<DWP> p;
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        p.e0[bj] = (int)tab[2 * u + bj];
        p.e1[bj] = (int)tab[2 * u + bj + 1];
#pragma unroll
        for (int q = 0; q < DWP; ++q) {
            const int e = p.e0[bj] + lane + 64 * q;
            p.en[bj][q] = e < p.e1[bj] ? ent[e] : make_uint2(0u, 0u);
        }
    }
    return p;
}

// Selected entries of a dense weight-gradient unit (BI x 2 blocks of 16 x 16
// accumulators per lane: acc[bi][bj][v]).  For each column half bj the
// lane's 4 BI values go to the wave's LDS scratch, value v of block row bi
// at slot (bi * 64 + lane) * 4 + v, and then the unit half's entries of the
// selection list (chain-local entry offset from kbase, scratch slot; built
// on the host in the lane layout of the unit's variant; the first DWP per
// lane prefetched) are copied from the scratch to the tile's partials: work
// in proportion to the selected entries, not to the unit's BI * 2048
// candidates.  LDS operations of one wave complete in order, so the reads
// see the wave's own writes, and the next half's writes follow the reads.
template <class A, class Acc, int BI, int DWP, bool RMW = false>
__device__ __forceinline__ void dw_select(const Acc (&acc)[BI][2], A* scr, const DwPre<DWP>& pf,
                                          const uint2* __restrict__ ent, int kbase, A* __restrict__ part,
                                          bool accum_) {
    const bool accum = RMW && accum_;   // RMW false: the accumulate paths compile out
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
#pragma unroll
        for (int bi = 0; bi < BI; ++bi)
#pragma unroll
            for (int v = 0; v < 4; ++v) scr[(bi * 64 + lane) * 4 + v] = (A)acc[bi][bj][v];
        __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): the half is in LDS
        __builtin_amdgcn_wave_barrier();
        const int e0 = pf.e0[bj], e1 = pf.e1[bj];
#pragma unroll
        for (int q = 0; q < DWP; ++q)
            if (e0 + lane + 64 * q < e1) {
                if constexpr (RMW) {
                    A* dst = part + kbase + (int)pf.en[bj][q].x;
                    *dst = accum ? *dst + scr[pf.en[bj][q].y] : scr[pf.en[bj][q].y];
                } else {
                    part[kbase + (int)pf.en[bj][q].x] = scr[pf.en[bj][q].y];
                }
            }
        for (int e = e0 + lane + 64 * DWP; e < e1; e += 64) {
            const uint2 en = ent[e];
            if constexpr (RMW) {
                A* dst = part + kbase + (int)en.x;
                *dst = accum ? *dst + scr[en.y] : scr[en.y];
            } else {
                part[kbase + (int)en.x] = scr[en.y];
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Dense weight-gradient tile, selected entries kept: for output rows i and
// input columns j of a layer,
//   dW[i][j] = sum_r delta[r][i] * a[r][j]
// as an MFMA product whose K dimension runs over the tile rows, then the
// selected entries through the unit's selection list (dw_select).  The
// operands sit row-major in LDS, so each lane reads its K values (one per
// tile row) one scalar at a time; BI x 2 blocks per wave reuse them.  Unit u
// covers rows ui * BI * 16 .. and columns uj * 32 .. (u = ui * UJ + uj);
// lane (g, li) holds rows 4 g + v of block bi and column li of block bj.
template <int P, int R, int BI, int BJ, bool SQ = false, bool RMW = false>
__device__ __forceinline__ void dw_dense_units(const typename PT<P>::T* D, int ld, const typename PT<P>::T* X,
                                               int lx, int NI, int NJ, const unsigned* __restrict__ lst,
                                               typename PT<P>::A* scr, int kbase,
                                               typename PT<P>::A* __restrict__ part, bool accum) {
    typedef typename PT<P>::A A;
    typedef typename PT<P>::Acc Acc;
    typedef typename PT<P>::Frag Frag;
    constexpr int KCH = PT<P>::KCH, VEC = PT<P>::VEC;
    static_assert(BJ == 2, "units of two column blocks");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, li = lane & 15;
    const int arow = (P == 0) ? (4 * (li & 3) + (li >> 2)) : li;
    const int UI = (NI + BI - 1) / BI, UJ = (NJ + BJ - 1) / BJ;
    const int imax = NI * 16 - 1, jmax = NJ * 16 - 1;
    const int nwave = (int)(blockDim.x >> 6);
    const unsigned* tab = lst;
    const uint2* ent = reinterpret_cast<const uint2*>(lst + ((2 * UI * UJ + 2) & ~1));
    for (int u = wave; u < UI * UJ; u += nwave) {
        const int ui = u / UJ, uj = u - ui * UJ;
        const auto pf = dw_prefetch<DWP<P>>(tab, ent, u);
        Acc acc[BI][BJ];
        int ic[BI], jc[BJ];
#pragma unroll
        for (int bi = 0; bi < BI; ++bi) {
            ic[bi] = min((ui * BI + bi) * 16 + arow, imax);
#pragma unroll
            for (int bj = 0; bj < BJ; ++bj) acc[bi][bj] = Acc{};
        }
#pragma unroll
        for (int bj = 0; bj < BJ; ++bj) jc[bj] = min((uj * BJ + bj) * 16 + li, jmax);
#pragma unroll
        for (int k0 = 0; k0 < R; k0 += KCH) {
            const int r0 = k0 + g * VEC;
            Frag a[BI], b[BJ];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
#pragma unroll
                for (int bi = 0; bi < BI; ++bi) frag_put<P, SQ>(a[bi], e, D + (r0 + e) * ld, ic[bi]);
#pragma unroll
                for (int bj = 0; bj < BJ; ++bj) frag_put<P, SQ>(b[bj], e, X + (r0 + e) * lx, jc[bj]);
            }
#pragma unroll
            for (int e = 0; e < NE<P>; ++e)
#pragma unroll
                for (int bi = 0; bi < BI; ++bi)
#pragma unroll
                    for (int bj = 0; bj < BJ; ++bj) mma1(acc[bi][bj], a[bi], b[bj], e);
        }
        dw_select<A, Acc, BI, DWP<P>, RMW>(acc, scr, pf, ent, kbase, part, accum);
    }
}

// Dense weight-gradient tile for BF16 operands with interleaved blocks, so
// that a lane's K values (one per tile row) come from vector reads.  A unit
// covers output rows i0 .. i0 + 63 and input columns j0 .. j0 + 31 as 4 x 2
// MFMA blocks; block (bi, bj) holds rows i0 + 4 m + bi and columns
// j0 + 2 n + bj (m, n < 16).  For each of its eight K slots r lane (g, li)
// then needs delta[r][i0 + 4 li .. i0 + 4 li + 3] (one 8-byte read serves
// the four row blocks) and a[r][j0 + 2 li, j0 + 2 li + 1] (one 4-byte read
// serves the two column blocks): two LDS reads per K slot for eight blocks,
// against six scalar reads for the non-interleaved 4 x 2 tile.  Output
// layout: lane (g, li) holds rows m = 4 g + v of column n = li, i.e. entry
// (i0 + 16 g + 4 v + bi, j0 + 2 li + bj); unit u = (i0 / 64) * NJ32 + j0 / 32.
// Requires the padded output width to be a multiple of 64 and R a multiple
// of 32 (the padded input width is a multiple of 32 for BF16).
template <int R, bool RMW = false>
__device__ __forceinline__ void dw_dense_il(const __bf16* D, int ld, const __bf16* X, int lx, int NI64, int NJ32,
                                            const unsigned* __restrict__ lst, float* scr, int kbase,
                                            float* __restrict__ part, bool accum) {
    typedef __bf16 b2v __attribute__((ext_vector_type(2)));
    static_assert(R % 32 == 0, "K chunks of 32 tile rows");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, li = lane & 15;
    const int nwave = (int)(blockDim.x >> 6);
    const unsigned* tab = lst;
    const uint2* ent = reinterpret_cast<const uint2*>(lst + ((2 * NI64 * NJ32 + 2) & ~1));
    for (int u = wave; u < NI64 * NJ32; u += nwave) {
        const int ui = u / NJ32, w = u - ui * NJ32;
        const int i0 = ui * 64, j0 = w * 32;
        const auto pf = dw_prefetch<DWP<2>>(tab, ent, u);
        f4v acc[4][2];
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) acc[bi][0] = acc[bi][1] = f4v{};
#pragma unroll
        for (int k0 = 0; k0 < R; k0 += 32) {
            const int r0 = k0 + g * 8;
            b4v dv[8];
            b2v xv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                dv[e] = *reinterpret_cast<const b4v*>(D + (r0 + e) * ld + i0 + 4 * li);
                xv[e] = *reinterpret_cast<const b2v*>(X + (r0 + e) * lx + j0 + 2 * li);
            }
            b8v fa[4], fb[2];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
#pragma unroll
                for (int bi = 0; bi < 4; ++bi) fa[bi][e] = dv[e][bi];
                fb[0][e] = xv[e][0];
                fb[1][e] = xv[e][1];
            }
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) mma1(acc[bi][bj], fa[bi], fb[bj], 0);
        }
        dw_select<float, f4v, 4, DWP<2>, RMW>(acc, scr, pf, ent, kbase, part, accum);
    }
}

// Dense weight-gradient product of one layer in the variant the host chose
// (its selection list is laid out for it): 2 x 2 blocks per unit, 4 x 2
// blocks (BF16 and split BF16 layers wide enough for every wave), or the
// interleaved 4 x 2 BF16 unit.
template <int P, int R, bool SQ = false, bool RMW = false>
__device__ __forceinline__ void dw_dense(const typename PT<P>::T* D, int ld, const typename PT<P>::T* X, int lx,
                                         int NI, int NJ, int variant, const unsigned* lst, typename PT<P>::A* scr,
                                         int kbase, typename PT<P>::A* part, bool accum) {
    if constexpr (R % PT<P>::KCH == 0) {
        if constexpr (P >= 2) {
            if (variant == DWV_IL) {
                if constexpr (P == 2 && !SQ)
                    dw_dense_il<R, RMW>(D, ld, X, lx, NI / 4, NJ / 2, lst, scr, kbase, part, accum);
                return;
            }
            if (variant == DWV_4X2) {
                dw_dense_units<P, R, 4, 2, SQ, RMW>(D, ld, X, lx, NI, NJ, lst, scr, kbase, part, accum);
                return;
            }
        }
        dw_dense_units<P, R, 2, 2, SQ, RMW>(D, ld, X, lx, NI, NJ, lst, scr, kbase, part, accum);
    }
}

// Chain c's mask tables of one tower into LDS.  Called by every thread at
// kernel start; the kernel's first barrier publishes them, so the adjoint
// pass reads them from LDS instead of waiting on dependent global loads
// between its phases.
__device__ __forceinline__ void stage_meta(const GradArgs& a, const TowerPlan& tp, int c, TileMeta* m) {
    const int t = (int)threadIdx.x;
    const size_t lb = (size_t)c * a.nl_total + tp.seg0;
    if (t <= tp.nl) m->seg[t] = a.seg[(size_t)c * a.nseg + tp.seg0 + t];
    if (t < tp.nl) {
        m->bseg[t] = a.bseg[lb + t];
        m->mloff[t] = (int)a.ml_off[lb + t];
    }
    if (t == 0) {
        m->o = a.offs[c];
        m->n = (int)(a.offs[c + 1] - a.offs[c]);
        unsigned d = 0;
        for (int l = 0; l < tp.nl; ++l) d |= a.dflag[lb + l] ? 1u << l : 0u;
        m->dmask = d;
    }
}

// Lowest layer of the tower with selected entries (nl: none).
__device__ __forceinline__ int lowest_layer(const TowerPlan& tp, const TileMeta* m) {
    for (int l = 0; l < tp.nl; ++l)
        if (m->seg[l + 1] > m->seg[l]) return l;
    return tp.nl;
}

// Hidden layers; B points at the tower's biases (staged in LDS).
template <int P, int R>
__device__ __forceinline__ void tower_hidden_forward(const TowerPlan& tp, const typename PT<P>::T* W,
                                                     const typename PT<P>::A* B, typename PT<P>::T* sm) {
    for (int l = 0; l < tp.nl - 1; ++l) {
        EpiTanh<P> e{B + tp.bo[l], sm + tp.lo[l + 1], tp.ls[l + 1]};
        gemm<P, R>(W + tp.wo[l], tp.wp[l], tp.wp[l], tp.wp[l + 1], sm + tp.lo[l], tp.ls[l], e);
        __syncthreads();
    }
}

// Copies n values into LDS (biases, targets); the caller synchronises.
template <class V>
__device__ __forceinline__ void stage(V* dst, const V* src, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// Likelihood partial of one tile, one slot per wave (the wave's lanes summed
// by a fixed butterfly); slots of absent waves stay zero.
__device__ __forceinline__ void ulik_store(double* slot8, double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) slot8[threadIdx.x >> 6] = v;
}

// A layer of the adjoint pass with its weight-gradient terms (dw) and the
// multiplies of its adjoint product in one phase: the product's epilogue,
// which overwrites the layer input's slab with its adjoint, waits for a
// barrier, so that neither needs the other's result and the waves of a
// workgroup interleave the two (even waves multiply first, odd waves start
// with dw), the product on the matrix cores while dw reads LDS.  The
// arithmetic of both is that of the sequential order.  Returns false,
// having done nothing, when a wave would hold more than two units'
// accumulators (one with four row blocks; then the caller runs the two one
// after the other).
template <int P, int R, class DW>
__device__ __forceinline__ bool back_overlap(const GradArgs& a, const TowerPlan& tp, const typename PT<P>::T* W,
                                             typename PT<P>::T* sm, int l, DW& dw) {
    typedef typename PT<P>::Acc Acc;
    constexpr int RB = R / 16;
    const int Np = tp.wp[l], K = tp.wp[l + 1];
    const typename PT<P>::T* Wt = W + tp.wto[l];
    const typename PT<P>::T* Xd = sm + tp.lo[l + 1];
    const int ldx = tp.ls[l + 1];
    const int odd = (int)(threadIdx.x >> 6) & 1;
    EpiBack<P> e{sm + tp.lo[l], tp.ls[l]};
    auto run = [&](auto nrb) -> bool {
        constexpr int NRB = decltype(nrb)::value;
        constexpr int MAXU = NRB >= 4 ? 1 : 2;
        if (deferred_units_max<P, R, NRB>(Np) > MAXU) return false;   // the same in every wave
        Acc dacc[MAXU][NRB];
        if (odd) {
            dw();
            gemm_deferred<P, R, NRB, MAXU>(Wt, K, K, Np, Xd, ldx, dacc);
        } else {
            gemm_deferred<P, R, NRB, MAXU>(Wt, K, K, Np, Xd, ldx, dacc);
            dw();
        }
        __syncthreads();
        gemm_deferred_epi<P, R, NRB, MAXU>(Np, dacc, e);
        __syncthreads();
        return true;
    };
    if constexpr (RB > 1) {
        if (nrb_of<R>(Np) == RB) return run(std::integral_constant<int, RB>{});
    }
    return run(std::integral_constant<int, 1>{});
}

// Adjoint pass of one tower from the output adjoint held in slab nl: for each
// layer from the top, the selected weight-gradient partials, then (while a
// lower layer still has selected entries) the adjoint of the layer input;
// with a.overlap, at tiles of up to 32 rows, the two in one phase
// (back_overlap).
// m: the chain's tables (stage_meta, published); lowest: lowest_layer() of
// the chain; B: the tower's biases (staged).  SQ: squared weight-gradient
// terms (sensitivity pass).  With tp.rc1 slab 1 shares its LDS with slab 3,
// which the forward pass wrote later, so a_1 is recomputed from the input
// (layer 0's tile product and tanh) once layer 2's adjoint no longer needs
// slab 3.  slot: the partial slot of the tile (its row tile, or the
// workgroup's tile group); accum: add to what the slot holds (a later tile
// of the group; each entry's slot is read and written by the same thread
// in every tile) instead of overwriting it, in instances with RMW (without
// it the accumulating paths compile out).
template <int P, int R, bool SQ = false, bool RMW = false>
__device__ __forceinline__ void tower_backward(const GradArgs& a, const TowerPlan& tp, const TileMeta* m, int slot,
                                               const typename PT<P>::T* W, const typename PT<P>::A* B,
                                               typename PT<P>::T* sm, int lowest, bool accum = false) {
    typedef typename PT<P>::A A;
    const long long o = m->o;
    const int n = m->n;
    const int* code = a.ecode + o;
    const int* seg = m->seg;
    A* part = reinterpret_cast<A*>(a.part) + a.tmax * o + (long long)slot * n;
    const int* bseg = m->bseg;
    const unsigned dmask = m->dmask;
    for (int l = tp.nl - 1; l >= lowest; --l) {
        // (slab sharing is planned for tiles of at most 32 rows, and for
        // BF16 at 64 rows, so the other 64-row instances carry no recompute
        // code and its registers)
        if constexpr (R <= 32 || P == 2) {
            if (l == 1 && tp.rc1) {
                // the barrier that ended layer 2's adjoint product has
                // retired every read of slab 3 (delta_3)
                EpiTanh<P> e{B + tp.bo[0], sm + tp.lo[1], tp.ls[1]};
                gemm<P, R>(W + tp.wo[0], tp.wp[0], tp.wp[0], tp.wp[1], sm + tp.lo[0], tp.ls[0], e);
                __syncthreads();
            }
        }
        // this layer's weight-gradient terms: dense product or per-entry sums
        auto weight_gradient = [&]() {
            if (dmask & (1u << l)) {
                A* scr = reinterpret_cast<A*>(reinterpret_cast<unsigned char*>(sm) + tp.scr + (threadIdx.x >> 6) * 4096);
                dw_dense<P, R, SQ, RMW>(sm + tp.lo[l + 1], tp.ls[l + 1], sm + tp.lo[l], tp.ls[l], tp.wp[l + 1] >> 4,
                                   tp.wp[l] >> 4, tp.dwv[l], a.ml + m->mloff[l], scr, seg[l], part, accum);
                dw_partials<P, R, SQ, RMW>(code, bseg[l], seg[l + 1], sm + tp.lo[l + 1], tp.ls[l + 1], sm + tp.lo[l],
                                           tp.ls[l], part, accum);
            } else {
                dw_partials<P, R, SQ, RMW>(code, seg[l], seg[l + 1], sm + tp.lo[l + 1], tp.ls[l + 1], sm + tp.lo[l],
                                           tp.ls[l], part, accum);
            }
        };
        // (64-row tiles run the two one after the other: holding the deferred
        // accumulators beside their four row blocks spills the FP32 kernel
        // that must stay within 128 registers, 33.4 -> 34.9 us on the 2-D MLP)
        if constexpr (R <= 32) {
            if (l > lowest && a.overlap && back_overlap<P, R>(a, tp, W, sm, l, weight_gradient)) continue;
        }
        weight_gradient();
        if (l > lowest) {
            __syncthreads();
            EpiBack<P> e{sm + tp.lo[l], tp.ls[l]};
            gemm<P, R>(W + tp.wto[l], tp.wp[l + 1], tp.wp[l + 1], tp.wp[l], sm + tp.lo[l + 1], tp.ls[l + 1], e);
            __syncthreads();
        }
    }
}

// MLP output layer and head in FP64 for FP32 and split-BF16 products with
// few outputs: F = W_L a + b as FP64 dot products of the stored activations
// and weights (eight lanes per (row, output), then a butterfly), residual,
// squared residuals and delta = (F - y) / lik_sd^2 into slab L + 1 (zero for
// padded outputs and rows past the data).  Near the mode the residual is a
// small difference of values of order one, and an FP32 accumulation of the
// product would put most of its error there (2e-4 of the residual on the
// 256-wide MLP), and so into U, the output adjoint and the gradient.
// Returns the thread's sum of squared residuals.
template <int P, int R>
__device__ __forceinline__ double head_fp64(const GradArgs& a, const TowerPlan& tp, const typename PT<P>::T* W,
                                            const typename PT<P>::A* B, typename PT<P>::T* sm, const double* ys,
                                            int t) {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    const int L = tp.nl - 1;
    const T* X = sm + tp.lo[L];
    const T* Wl = W + tp.wo[L];
    T* D = sm + tp.lo[L + 1];
    const int K = tp.wp[L], NP = tp.wp[L + 1], ldx = tp.ls[L], ldd = tp.ls[L + 1], d_out = a.d_out;
    const A* bias = B + tp.bo[L];
    for (int i = threadIdx.x; i < R * NP; i += blockDim.x) {
        const int r = i / NP, n = i - r * NP;
        if (n >= d_out) st1<P>(D + r * ldd, n, (A)0);
    }
    double sq = 0.0;
    const int sub = (int)threadIdx.x & 7, groups = (int)blockDim.x >> 3;
    // every lane runs the same number of iterations, so the butterflies see
    // all eight lanes of each group
    for (int base = 0; base < R * d_out; base += groups) {
        const int pr = base + ((int)threadIdx.x >> 3);
        const int r = pr / d_out, n = pr - r * d_out;
        const bool in = pr < R * d_out;
        double acc = 0.0;
        if (in)
            for (int k = sub; k < K; k += 8)
                acc = fma((double)ld1<P>(X + r * ldx, k), (double)ld1<P>(Wl + (size_t)n * K, k), acc);
        acc += __shfl_xor(acc, 1, 64);
        acc += __shfl_xor(acc, 2, 64);
        acc += __shfl_xor(acc, 4, 64);
        if (in && sub == 0) {
            A d = (A)0;
            if (t * R + r < a.n_rows_a) {
                const double res = (acc + (double)bias[n]) - ys[r * d_out + n];
                sq += res * res;
                d = (A)(res * a.inv_lik_var);
            }
            st1<P>(D + r * ldd, n, d);
        }
    }
    return sq;
}

// Waves per SIMD the register allocation must leave room for: four (two
// 512-thread workgroups per compute unit, at most 128 VGPRs) for the FP32
// MLP kernels of 64-row tiles, whose LDS footprint on narrow layers admits
// a second workgroup; otherwise no constraint beyond one workgroup.
template <int P, int R> constexpr int MLP_WAVES = (P == 1 && R == 64) ? 4 : 1;

// ---------------------------------------------------------------------------
// MLP: forward, head and adjoint of one (chain, row tile).
// FWD = true: forward pass and likelihood partials only (the energy pass),
// with activation slabs that may alias (ping-pong plans).  The biases and
// the chain's tables are staged and published by the caller's first
// barrier; slot and accum as in tower_backward.
template <int P, int R, bool FWD, bool GROUP>
__device__ __forceinline__ void mlp_tile(const GradArgs& a, int c, int t, int slot, bool accum,
                                         const typename PT<P>::T* W, const typename PT<P>::A* B,
                                         const TileMeta* meta, typename PT<P>::T* sm, double* ys) {
    typedef typename PT<P>::T T;
    const TowerPlan& tp = a.ta;
    const int L = tp.nl - 1;
    {
        const int nv = max(0, min(R, a.n_rows_a - t * R)) * a.d_out;
        const double* yg = a.target + (size_t)t * R * a.d_out;
        for (int i = threadIdx.x; i < R * a.d_out; i += blockDim.x) ys[i] = i < nv ? yg[i] : 0.0;
    }
    load_rows<T, R>(sm + tp.lo[0], tp.ls[0], reinterpret_cast<const T*>(a.xa) + (size_t)t * R * tp.wp[0], tp.wp[0]);
    __syncthreads();
    const int lowest = FWD ? tp.nl : lowest_layer(tp, meta);
    tower_hidden_forward<P, R>(tp, W, B, sm);
    double sq = 0.0;
    bool head_done = false;
    if constexpr (P == 1 || P == 3) {
        if (a.d_out <= 4) {
            sq = head_fp64<P, R>(a, tp, W, B, sm, ys, t);
            head_done = true;
        }
    }
    if (!head_done) {
        EpiMlpHead<P> h{B + tp.bo[L], sm + tp.lo[L + 1], tp.ls[L + 1], ys, a.d_out, t * R, a.n_rows_a,
                        a.inv_lik_var, 0.0};
        gemm<P, R>(W + tp.wo[L], tp.wp[L], tp.wp[L], tp.wp[L + 1], sm + tp.lo[L], tp.ls[L], h);
        sq = h.sq;
    }
    ulik_store(a.ulik + ((size_t)c * a.tiles_a + t) * 8, 0.5 * a.inv_lik_var * sq);
    if constexpr (!FWD) {
        __syncthreads();
        tower_backward<P, R, false, GROUP>(a, tp, meta, slot, W, B, sm, lowest, accum);
    }
}

// One (chain, row tile) per workgroup; GROUP: a workgroup takes a.tpg
// consecutive row tiles of one chain and sums their weight-gradient terms
// in tile order into one partial slot (each entry's slot read and written
// by the thread that owns the entry), so that k_update reads a.tpg times
// fewer partials.  The loop keeps more values live, so it is a separate
// instance, used where it pays (the engine decides; tile_group).
template <int P, int R, bool FWD, bool GROUP = false>
__global__ __launch_bounds__(HMC_NT) __attribute__((amdgpu_waves_per_eu(MLP_WAVES<P, R>))) void k_mlp_grad(
    const GradArgs a) {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    extern __shared__ __align__(16) unsigned char smem[];
    T* sm = reinterpret_cast<T*>(smem);
    const int tpg = GROUP ? a.tpg : 1;
    const int groups = GROUP ? (a.tiles_a + tpg - 1) / tpg : a.tiles_a;
    int c, grp;
    if (!tile_of(a.n_chains * groups, groups, c, grp)) return;
    c += a.chain0;
    if (!a.active[c]) return;
    const TowerPlan& tp = a.ta;
    const T* W = reinterpret_cast<const T*>(a.wbuf) + c * a.wstride;
    const A* Bg = reinterpret_cast<const A*>(a.bbuf) + c * a.bstride;
    const int L = tp.nl - 1;
    // biases into LDS beside the input rows (the tile's targets: mlp_tile)
    A* Bs = reinterpret_cast<A*>(smem + a.bias_lds_a);
    stage(Bs, Bg + tp.bo[0], (int)(tp.bo[L] + tp.wp[L + 1] - tp.bo[0]));
    double* ys = reinterpret_cast<double*>(smem + a.y_lds);
    const A* B = Bs - tp.bo[0];
    TileMeta* meta = reinterpret_cast<TileMeta*>(smem + a.meta_lds_a);
    if constexpr (!FWD) stage_meta(a, tp, c, meta);
    if constexpr (GROUP) {
        const int t0 = grp * tpg, t1 = min(a.tiles_a, t0 + tpg);
        for (int t = t0; t < t1; ++t) {
            mlp_tile<P, R, FWD, true>(a, c, t, grp, t > t0, W, B, meta, sm, ys);
            // every read of this tile's slabs and targets is done before
            // the next tile's rows and targets overwrite them
            if (t + 1 < t1) __syncthreads();
        }
    } else {
        mlp_tile<P, R, FWD, false>(a, c, grp, grp, false, W, B, meta, sm, ys);
    }
}

// Sensitivity tile of one tower (Sec. 3.1): the forward pass at the mean
// parameters through the hidden layers, then the output adjoint set to the
// same seed vector on every valid row of the tile (its other rows zero), and
// the adjoint pass with squared weight-gradient terms on every layer:
//   part[k] = sum_{tile rows} (seed . dout/dtheta_k)^2,
// since per row dF/dW_l[i][j] = delta_l[i] a_{l-1}[j] and dF/db_l[i] =
// delta_l[i] for the output F = seed . out.  MLP: seed e_o for output o.
// DeepONet: F_jq = <B_j, T_q> + b0, so the branch tower with seed T_q gives
// the terms of query point q and the trunk tower with seed B_j those of
// function j.  tower 0: the MLP or branch tower (a.ta, a.xa), 1: the trunk
// (a.tb, a.xb).  seed: product type, [wp_out], device.
template <int P, int R>
__global__ __launch_bounds__(HMC_NT) __attribute__((amdgpu_waves_per_eu(MLP_WAVES<P, R>))) void k_tower_sens(
    const GradArgs a, int tower, const void* seed) {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    extern __shared__ __align__(16) unsigned char smem[];
    T* sm = reinterpret_cast<T*>(smem);
    const int tiles = tower ? a.tiles_b : a.tiles_a;
    int c, t;
    if (!tile_of(a.n_chains * tiles, tiles, c, t)) return;
    const TowerPlan& tp = tower ? a.tb : a.ta;
    const T* W = reinterpret_cast<const T*>(a.wbuf) + c * a.wstride;
    const A* Bg = reinterpret_cast<const A*>(a.bbuf) + c * a.bstride;
    const int L = tp.nl - 1;
    A* Bs = reinterpret_cast<A*>(smem + (tower ? a.bias_lds_b : a.bias_lds_a));
    stage(Bs, Bg + tp.bo[0], (int)(tp.bo[L] + tp.wp[L + 1] - tp.bo[0]));
    const A* B = Bs - tp.bo[0];
    const T* xin = reinterpret_cast<const T*>(tower ? a.xb : a.xa);
    TileMeta* meta = reinterpret_cast<TileMeta*>(smem + (tower ? a.meta_lds_b : a.meta_lds_a));
    stage_meta(a, tp, c, meta);
    load_rows<T, R>(sm + tp.lo[0], tp.ls[0], xin + (size_t)t * R * tp.wp[0], tp.wp[0]);
    __syncthreads();
    tower_hidden_forward<P, R>(tp, W, B, sm);
    T* so = sm + tp.lo[L + 1];
    const T* sv = reinterpret_cast<const T*>(seed);
    const int wpo = tp.wp[L + 1], nv = min(R, (tower ? a.n_rows_b : a.n_rows_a) - t * R);
    for (int i = threadIdx.x; i < R * wpo; i += blockDim.x) {
        const int r = i / wpo, col = i - r * wpo;
        so[r * tp.ls[L + 1] + col] = r < nv ? sv[col] : (T)0;
    }
    __syncthreads();
    tower_backward<P, R, true>(a, tp, meta, t, W, B, sm, 0);
}

// Output of one tower at the current weights for the rows of its tile,
// out[row][n] = (W_L a_{L-1} + b_L)[n] for the valid rows (product type,
// row stride ld): the DeepONet features that seed the sensitivity passes.
template <int P> struct EpiRowsOut {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    const A* bias; T* out; int ld; int row0; int nrows;
    __device__ __forceinline__ void operator()(int r, int n0, const typename PT<P>::Acc& acc) const {
        if (row0 + r >= nrows) return;
        A o[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) o[v] = (A)acc[v] + bias[n0 + v];
        st4<P>(out + (size_t)(row0 + r) * ld, n0, o);
    }
};

template <int P, int R>
__global__ __launch_bounds__(HMC_NT) void k_tower_out(const GradArgs a, int tower, void* out, int ld) {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    extern __shared__ __align__(16) unsigned char smem[];
    T* sm = reinterpret_cast<T*>(smem);
    const int tiles = tower ? a.tiles_b : a.tiles_a;
    int c, t;
    if (!tile_of(a.n_chains * tiles, tiles, c, t)) return;
    const TowerPlan& tp = tower ? a.tb : a.ta;
    const T* W = reinterpret_cast<const T*>(a.wbuf) + c * a.wstride;
    const A* Bg = reinterpret_cast<const A*>(a.bbuf) + c * a.bstride;
    const int L = tp.nl - 1;
    A* Bs = reinterpret_cast<A*>(smem + (tower ? a.bias_lds_b : a.bias_lds_a));
    stage(Bs, Bg + tp.bo[0], (int)(tp.bo[L] + tp.wp[L + 1] - tp.bo[0]));
    const A* B = Bs - tp.bo[0];
    const T* xin = reinterpret_cast<const T*>(tower ? a.xb : a.xa);
    load_rows<T, R>(sm + tp.lo[0], tp.ls[0], xin + (size_t)t * R * tp.wp[0], tp.wp[0]);
    __syncthreads();
    tower_hidden_forward<P, R>(tp, W, B, sm);
    EpiRowsOut<P> e{B + tp.bo[L], reinterpret_cast<T*>(out), ld, t * R, tower ? a.n_rows_b : a.n_rows_a};
    gemm<P, R>(W + tp.wo[L], tp.wp[L], tp.wp[L], tp.wp[L + 1], sm + tp.lo[L], tp.ls[L], e);
}

// Sum of the sensitivity partials of entries [k0, k1) over the row tiles,
// in tile order, into an FP64 accumulator (one pass per seed); a pass with
// s2 set also writes S^2[k] = sigma_k^2 * acc[k] / n_d.
template <int P>
__global__ __launch_bounds__(256) void k_sens_reduce(const void* part, int tiles, long long n, long long k0,
                                                     long long k1, double* acc, const double* sigma, double inv_nd,
                                                     double* s2) {
    typedef typename PT<P>::A A;
    const long long k = k0 + (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= k1) return;
    const A* pp = reinterpret_cast<const A*>(part) + k;
    // eight independent sums (tiles t = j mod 8) combined in a fixed order
    double q[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int t = 0;
    for (; t + 8 <= tiles; t += 8) {
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) q[jj] += (double)pp[(size_t)(t + jj) * n];
    }
    for (int jj = 0; t < tiles; ++t, ++jj) q[jj] += (double)pp[(size_t)t * n];
    const double sum = ((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]));
    const double v = acc[k] + sum;
    acc[k] = v;
    if (s2) s2[k] = sigma[k] * sigma[k] * v * inv_nd;
}

// Posterior predictive tile: the forward pass of chain c's current dense
// weights over one tile of new input rows, and the running moments of the
// outputs (EpiPredict).  a.xa, a.n_rows_a and a.tiles_a describe the new
// inputs; activation slabs may alias (ping-pong plans).
template <int P, int R>
__global__ __launch_bounds__(HMC_NT) void k_mlp_predict(const GradArgs a, int c, double* mean, double* m2,
                                                        double* var, double inv_k, double inv_n) {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    extern __shared__ __align__(16) unsigned char smem[];
    T* sm = reinterpret_cast<T*>(smem);
    int c0, t;
    if (!tile_of(a.tiles_a, a.tiles_a, c0, t)) return;
    const TowerPlan& tp = a.ta;
    const T* W = reinterpret_cast<const T*>(a.wbuf) + c * a.wstride;
    const A* Bg = reinterpret_cast<const A*>(a.bbuf) + c * a.bstride;
    const int L = tp.nl - 1;
    A* Bs = reinterpret_cast<A*>(smem + a.bias_lds_a);
    stage(Bs, Bg + tp.bo[0], (int)(tp.bo[L] + tp.wp[L + 1] - tp.bo[0]));
    const A* B = Bs - tp.bo[0];
    load_rows<T, R>(sm + tp.lo[0], tp.ls[0], reinterpret_cast<const T*>(a.xa) + (size_t)t * R * tp.wp[0], tp.wp[0]);
    __syncthreads();
    tower_hidden_forward<P, R>(tp, W, B, sm);
    EpiPredict<P> e{B + tp.bo[L], a.d_out, t * R, a.n_rows_a, mean, m2, var, inv_k, inv_n};
    gemm<P, R>(W + tp.wo[L], tp.wp[L], tp.wp[L], tp.wp[L + 1], sm + tp.lo[L], tp.ls[L], e);
}


// DeepONet trunk forward: T = trunk(y_q) for one (chain, query tile).
template <int P, int R>
__global__ __launch_bounds__(HMC_NT) void k_trunk_fwd(const GradArgs a) {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    extern __shared__ __align__(16) unsigned char smem[];
    T* sm = reinterpret_cast<T*>(smem);
    int c, t;
    if (!tile_of(a.n_chains * a.tiles_b, a.tiles_b, c, t)) return;
    c += a.chain0;
    if (!a.active[c]) return;
    const TowerPlan& tp = a.tb;
    const T* W = reinterpret_cast<const T*>(a.wbuf) + c * a.wstride;
    const A* Bg = reinterpret_cast<const A*>(a.bbuf) + c * a.bstride;
    const int L = tp.nl - 1;
    A* Bs = reinterpret_cast<A*>(smem + a.bias_lds_b);
    stage(Bs, Bg + tp.bo[0], (int)(tp.bo[L] + tp.wp[L + 1] - tp.bo[0]));
    const A* B = Bs - tp.bo[0];
    load_rows<T, R>(sm + tp.lo[0], tp.ls[0], reinterpret_cast<const T*>(a.xb) + (size_t)t * R * tp.wp[0], tp.wp[0]);
    __syncthreads();
    tower_hidden_forward<P, R>(tp, W, B, sm);
    const int nvalid = a.n_rows_b - t * R;
    EpiTrunkOut<P> e{B + tp.bo[L], reinterpret_cast<T*>(a.tm) + c * a.tm_stride, tp.wp[L + 1],
                     reinterpret_cast<T*>(a.tt) + c * a.tm_stride, a.nq_rows, t * R, nvalid};
    gemm<P, R>(W + tp.wo[L], tp.wp[L], tp.wp[L], tp.wp[L + 1], sm + tp.lo[L], tp.ls[L], e);
}

// DeepONet branch tile: branch forward, combination with the trunk features,
// FP64 head, adjoint of the branch output, branch adjoint pass.
template <int P, int R, bool FWD>
__global__ __launch_bounds__(HMC_NT) void k_branch_grad(const GradArgs a) {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    extern __shared__ __align__(16) unsigned char smem[];
    T* sm = reinterpret_cast<T*>(smem);
    double* red = reinterpret_cast<double*>(smem + a.red_off);
    int c, t;
    if (!tile_of(a.n_chains * a.tiles_a, a.tiles_a, c, t)) return;
    c += a.chain0;
    if (!a.active[c]) return;
    const TowerPlan& tp = a.ta;
    const T* W = reinterpret_cast<const T*>(a.wbuf) + c * a.wstride;
    const A* Bg = reinterpret_cast<const A*>(a.bbuf) + c * a.bstride;
    const int L = tp.nl - 1;
    const int pp = tp.wp[L + 1];
    const double b0 = (double)Bg[a.b0_off];
    A* Bs = reinterpret_cast<A*>(smem + a.bias_lds_a);
    stage(Bs, Bg + tp.bo[0], (int)(tp.bo[L] + tp.wp[L + 1] - tp.bo[0]));
    const A* B = Bs - tp.bo[0];
    TileMeta* meta = reinterpret_cast<TileMeta*>(smem + a.meta_lds_a);
    if constexpr (!FWD) stage_meta(a, tp, c, meta);
    load_rows<T, R>(sm + tp.lo[0], tp.ls[0], reinterpret_cast<const T*>(a.xa) + (size_t)t * R * tp.wp[0], tp.wp[0]);
    __syncthreads();
    const int lowest = FWD ? tp.nl : lowest_layer(tp, meta);
    tower_hidden_forward<P, R>(tp, W, B, sm);
    const int nvalid = a.n_rows_a - t * R;
    const T* tmc = reinterpret_cast<const T*>(a.tm) + c * a.tm_stride;
    const T* ttc = reinterpret_cast<const T*>(a.tt) + c * a.tm_stride;
    EpiBranchOut<P> eo{B + tp.bo[L], sm + tp.lo[L + 1], tp.ls[L + 1],
                       reinterpret_cast<T*>(a.btr) + c * a.bt_stride, a.nu_cols, t * R, nvalid, !FWD};
    gemm<P, R>(W + tp.wo[L], tp.wp[L], tp.wp[L], pp, sm + tp.lo[L], tp.ls[L], eo);
    __syncthreads();
    EpiCombine<P> ec{sm + a.dg_off, a.dg_ld, reinterpret_cast<T*>(a.dgt) + c * a.dgt_stride, a.nu_cols, t * R,
                     a.target, a.nq, nvalid, t * R, b0, a.inv_lik_var, !FWD, 0.0, 0.0};
    gemm<P, R>(tmc, pp, pp, a.nq_pad, sm + tp.lo[L + 1], tp.ls[L + 1], ec);
    // likelihood partials one per wave (summed in a fixed order with the
    // tile's other slots when the trajectory step ends)
    ulik_store(a.ulik + ((size_t)c * a.tiles_a + t) * 8, 0.5 * a.inv_lik_var * ec.sq);
    if constexpr (FWD) return;
    const double sdg = block_sum(ec.sdg, red);
    if (threadIdx.x == 0) {
        const long long o = a.offs[c];
        const int n = (int)(a.offs[c + 1] - o);
        const int* seg = a.seg + (size_t)c * a.nseg;
        const int kb0 = seg[a.nseg - 2];
        if (seg[a.nseg - 1] > kb0)
            reinterpret_cast<A*>(a.part)[a.tmax * o + (long long)t * n + kb0] = (A)sdg;
    }
    // adjoint of the branch output: dB = dG T, into the slab that held B
    EpiStore<P> es{sm + tp.lo[L + 1], tp.ls[L + 1]};
    gemm<P, R>(ttc, a.nq_rows, a.nq_pad, pp, sm + a.dg_off, a.dg_ld, es);
    __syncthreads();
    tower_backward<P, R>(a, tp, meta, t, W, B, sm, lowest);
}

// DeepONet trunk adjoint tile: recompute the trunk forward for the tile's
// query rows, form dT = dG^T B for those rows (reduction over all
// functions), then the trunk adjoint pass.
template <int P, int R>
__global__ __launch_bounds__(HMC_NT) void k_trunk_bwd(const GradArgs a) {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    extern __shared__ __align__(16) unsigned char smem[];
    T* sm = reinterpret_cast<T*>(smem);
    int c, t;
    if (!tile_of(a.n_chains * a.tiles_b, a.tiles_b, c, t)) return;
    c += a.chain0;
    if (!a.active[c]) return;
    const TowerPlan& tp = a.tb;
    const T* W = reinterpret_cast<const T*>(a.wbuf) + c * a.wstride;
    const A* Bg = reinterpret_cast<const A*>(a.bbuf) + c * a.bstride;
    const int L = tp.nl - 1;
    A* Bs = reinterpret_cast<A*>(smem + a.bias_lds_b);
    stage(Bs, Bg + tp.bo[0], (int)(tp.bo[L] + tp.wp[L + 1] - tp.bo[0]));
    const A* B = Bs - tp.bo[0];
    TileMeta* meta = reinterpret_cast<TileMeta*>(smem + a.meta_lds_b);
    stage_meta(a, tp, c, meta);
    load_rows<T, R>(sm + tp.lo[0], tp.ls[0], reinterpret_cast<const T*>(a.xb) + (size_t)t * R * tp.wp[0], tp.wp[0]);
    __syncthreads();
    const int lowest = lowest_layer(tp, meta);
    const T* btc = reinterpret_cast<const T*>(a.btr) + c * a.bt_stride;
    // The tile's R rows of dG^T, a contiguous block of R * nu_cols values:
    // with dgt_stage, the first XPRE 16-byte chunks of each thread are loaded
    // now, so that their latency overlaps the forward recompute, and stored
    // to LDS (rows padded to dgt_lds_ld) after it; the rest is copied there.
    const T* dgt_tile = reinterpret_cast<const T*>(a.dgt) + c * a.dgt_stride + (size_t)t * R * a.nu_cols;
    constexpr int XPRE = 8;
    const int nthr = (int)blockDim.x;
    const int rowc = a.nu_cols * (int)sizeof(T) / 16;     // 16-byte chunks per row
    const int nch = R * rowc;
    u4v xr[XPRE];
    if (a.dgt_stage) {
#pragma unroll
        for (int j = 0; j < XPRE; ++j) {
            const int e = (int)threadIdx.x + j * nthr;
            if (e < nch) xr[j] = reinterpret_cast<const u4v*>(dgt_tile)[e];
        }
    }
    tower_hidden_forward<P, R>(tp, W, B, sm);
    const T* X = dgt_tile;
    int ldx = a.nu_cols;
    if (a.dgt_stage) {
        unsigned char* xl = smem + a.dgt_lds;
        const int ldb = a.dgt_lds_ld * (int)sizeof(T);
#pragma unroll
        for (int j = 0; j < XPRE; ++j) {
            const int e = (int)threadIdx.x + j * nthr;
            if (e < nch) {
                const int r = e / rowc;
                *reinterpret_cast<u4v*>(xl + r * ldb + (e - r * rowc) * 16) = xr[j];
            }
        }
        for (int e = (int)threadIdx.x + XPRE * nthr; e < nch; e += nthr) {
            const int r = e / rowc;
            *reinterpret_cast<u4v*>(xl + r * ldb + (e - r * rowc) * 16) = reinterpret_cast<const u4v*>(dgt_tile)[e];
        }
        __syncthreads();
        X = reinterpret_cast<const T*>(xl);
        ldx = a.dgt_lds_ld;
    }
    EpiStore<P> es{sm + tp.lo[L + 1], tp.ls[L + 1]};
    gemm<P, R>(btc, a.nu_cols, a.nu_cols, tp.wp[L + 1], X, ldx, es);
    __syncthreads();
    tower_backward<P, R>(a, tp, meta, t, W, B, sm, lowest);
}

// ---------------------------------------------------------------------------
// Per-entry state kernels.

// w32: also into the weight (and bias) shadows of the energy pass, when
// there are any.  d0, d1: the entry's destinations s.dst[2e], s.dst[2e + 1].
template <int P>
__device__ __forceinline__ void scatter_to(const StateArgs& s, int c, int d0, int d1, typename PT<P>::S x,
                                           bool w32) {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    if (d0 >= 0) {
        T* W = reinterpret_cast<T*>(s.wbuf) + c * s.wstride;   // rows of multiples of 32: flat indices
        st1<P>(W, d0, (A)x);
        st1<P>(W, d1, (A)x);
        if (w32 && s.wbuf32) {   // the energy pass's weights: FP32 or FP64
            if (s.w32_f64) {
                double* W64 = reinterpret_cast<double*>(s.wbuf32) + c * s.wstride;
                W64[d0] = (double)x;
                W64[d1] = (double)x;
            } else {
                float* W32 = reinterpret_cast<float*>(s.wbuf32) + c * s.wstride;
                W32[d0] = (float)x;
                W32[d1] = (float)x;
            }
        }
    } else {
        reinterpret_cast<A*>(s.bbuf)[c * s.bstride + (-d0 - 1)] = (A)x;
        if (w32 && s.bbuf64) reinterpret_cast<double*>(s.bbuf64)[c * s.bstride + (-d0 - 1)] = (double)x;
    }
}
template <int P>
__device__ __forceinline__ void scatter(const StateArgs& s, int c, long long e, typename PT<P>::S x,
                                        bool w32 = true) {
    scatter_to<P>(s, c, s.dst[2 * e], s.dst[2 * e + 1], x, w32);
}

// Sum of the per-tile partials, plus the prior term, then the kick (and
// drift + scatter) of the leapfrog step.  sub (a power of two, at
// most 8) threads per entry: thread sl of an entry sums the tiles
// t = sl (mod sub) with eight independent partial sums (so eight loads are
// in flight), and with sub > 1 the sub-lane sums meet in LDS and are added
// in sub-lane order.  Every order is fixed, so the result does not depend
// on timing.  More sub-lanes serve small grids, where the tile loop's load
// latency, not bandwidth, sets the time.
template <int P>
__global__ __launch_bounds__(256) void k_update(const StateArgs s, int mode, int sub) {
    typedef typename PT<P>::A A; typedef typename PT<P>::S S;
    __shared__ A red[256];
    const int c = (int)blockIdx.y + s.chain0;
    if (!s.active[c]) return;
    const long long o = s.offs[c];
    const int n = (int)(s.offs[c + 1] - o);
    const int epb = 256 / sub;
    const int kl = (int)threadIdx.x % epb, sl = (int)threadIdx.x / epb;
    const int k = blockIdx.x * epb + kl;
    if (sub == 1 && k >= n) return;
    // the owning thread's state and scatter destinations, loaded before the
    // tile sums so that their latency overlaps them
    const bool own = k < n && sl == 0;
    const bool drift = mode == UPD_KICK_DRIFT || mode == UPD_KICK_DRIFT_LAST;
    S* th = reinterpret_cast<S*>(s.theta) + o;
    S* mo = reinterpret_cast<S*>(s.mom) + o;
    S x = (S)0, p = (S)0;
    int d0 = 0, d1 = 0;
    if (own) {
        x = th[k];
        if (mode != UPD_GRAD) p = mo[k];
        if (drift) {
            d0 = s.dst[2 * (o + k)];
            d1 = s.dst[2 * (o + k) + 1];
        }
    }
    A part = (A)0;
    if (k < n) {
        const int* seg = s.seg + (size_t)c * s.nseg;
        const int nt = (k >= seg[s.seg_trunk_lo] && k < seg[s.seg_trunk_hi]) ? s.tiles_b : s.tiles_a;
        const A* pp = reinterpret_cast<const A*>(s.part) + s.tmax * o + k;
        A q[8] = {(A)0, (A)0, (A)0, (A)0, (A)0, (A)0, (A)0, (A)0};
        const size_t stride = (size_t)sub * n;
        int t = sl;
        for (; t + 7 * sub < nt; t += 8 * sub) {
#pragma unroll
            for (int j = 0; j < 8; ++j) q[j] += pp[(size_t)t * n + j * stride];
        }
        for (int j = 0; t < nt; t += sub, ++j) q[j] += pp[(size_t)t * n];
        part = ((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]));
    }
    A acc = part;
    if (sub > 1) {
        red[threadIdx.x] = part;
        __syncthreads();
        if (sl != 0 || k >= n) return;
        acc = red[kl];
        for (int j = 1; j < sub; ++j) acc += red[j * epb + kl];
    }
    const S g = (S)acc + x * (S)s.inv_prior_var;
    reinterpret_cast<S*>(s.grad)[o + k] = g;
    if (mode == UPD_GRAD) return;
    const S e = (S)s.eps[c];
    if (mode == UPD_HALF_KICK) {
        mo[k] = p - (S)0.5 * e * g;
        return;
    }
    p = p - e * g;
    mo[k] = p;
    const S m = s.minv ? reinterpret_cast<const S*>(s.minv)[o + k] : (S)1;
    x = x + e * m * p;
    th[k] = x;
    scatter_to<P>(s, c, d0, d1, x, mode == UPD_KICK_DRIFT_LAST);
}

// Symmetric-splitting kicks (the full-HMC baseline integrator of Sec. 4.2.3,
// after Cobb and Jalaian): the data rows form M consecutive batches of row
// tiles, the potential of batch m is its rows' likelihood plus 1/M of the
// prior, and each batch gradient reaches p as a half kick of its own, in
// batch order before a drift and in the mirrored order after it.  One
// thread per entry: it sums each batch's tile partials in tile order (eight
// independent sums, combined in a fixed tree), keeps the M batch gradients
// in registers and applies the kicks of `mode` (SPL_*).  The stored
// gradient is the batch gradients added in batch order.
template <int P>
__global__ __launch_bounds__(256) void k_update_split(const StateArgs s, int mode) {
    typedef typename PT<P>::A A; typedef typename PT<P>::S S;
    const int c = blockIdx.y;
    if (!s.active[c]) return;
    const long long o = s.offs[c];
    const int n = (int)(s.offs[c + 1] - o);
    const int k = blockIdx.x * 256 + (int)threadIdx.x;
    if (k >= n) return;
    const int M = s.split_n;
    S* th = reinterpret_cast<S*>(s.theta) + o;
    S* mo = reinterpret_cast<S*>(s.mom) + o;
    S x = th[k], p = mo[k];
    const bool drift = mode != SPL_END;
    int d0 = 0, d1 = 0;
    if (drift) {
        d0 = s.dst[2 * (o + k)];
        d1 = s.dst[2 * (o + k) + 1];
    }
    const A* pp = reinterpret_cast<const A*>(s.part) + s.tmax * o + k;
    const S prior = x * (S)(s.inv_prior_var / M);
    S gb[HMC_SPLIT_MAX];
    S gsum = (S)0;
#pragma unroll
    for (int m = 0; m < HMC_SPLIT_MAX; ++m) {
        gb[m] = (S)0;
        if (m >= M) continue;
        A q[8] = {(A)0, (A)0, (A)0, (A)0, (A)0, (A)0, (A)0, (A)0};
        int t = s.split_t[m];
        const int t1 = s.split_t[m + 1];
        for (; t + 7 < t1; t += 8) {
#pragma unroll
            for (int j = 0; j < 8; ++j) q[j] += pp[(size_t)(t + j) * n];
        }
        for (int j = 0; t < t1; ++t, ++j) q[j] += pp[(size_t)t * n];
        gb[m] = (S)(((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]))) + prior;
        gsum += gb[m];
    }
    reinterpret_cast<S*>(s.grad)[o + k] = gsum;
    const S h = (S)0.5 * (S)s.eps[c];
    if (mode != SPL_FIRST) {   // the mirrored half kicks closing a step
#pragma unroll
        for (int m = HMC_SPLIT_MAX - 1; m >= 0; --m)
            if (m < M) p = p - h * gb[m];
    }
    if (mode != SPL_END) {     // the half kicks in batch order opening a step
#pragma unroll
        for (int m = 0; m < HMC_SPLIT_MAX; ++m)
            if (m < M) p = p - h * gb[m];
    }
    mo[k] = p;
    if (!drift) return;
    const S mi = s.minv ? reinterpret_cast<const S*>(s.minv)[o + k] : (S)1;
    x = x + (S)2 * h * mi * p;
    th[k] = x;
    scatter_to<P>(s, c, d0, d1, x, mode != SPL_STEP);
}

__device__ __forceinline__ void philox4x64_10(unsigned long long c[4], unsigned long long k0, unsigned long long k1) {
    const unsigned long long M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const unsigned long long W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += W0; k1 += W1; }
        const unsigned long long hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const unsigned long long hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const unsigned long long n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
}

__device__ __forceinline__ double u01(unsigned long long w) { return ((double)(w >> 12) + 0.5) * 0x1p-52; }

// Four standard normals of Philox block `blk` of the momentum stream.
__device__ __forceinline__ void normals4(unsigned long long seed, int chain, unsigned long long it,
                                         unsigned long long blk, double z[4]) {
    unsigned long long c[4] = {it, 0ull, blk, 0ull};
    philox4x64_10(c, seed, (unsigned long long)chain);
    const double two_pi = 6.283185307179586;
    const double r0 = sqrt(-2.0 * log(u01(c[0]))), r1 = sqrt(-2.0 * log(u01(c[2])));
    const double t0 = two_pi * u01(c[1]), t1 = two_pi * u01(c[3]);
    z[0] = r0 * cos(t0); z[1] = r0 * sin(t0);
    z[2] = r1 * cos(t1); z[3] = r1 * sin(t1);
}

__device__ __forceinline__ double metropolis_u(unsigned long long seed, int chain, unsigned long long it) {
    unsigned long long c[4] = {it, 1ull, 0ull, 0ull};
    philox4x64_10(c, seed, (unsigned long long)chain);
    return u01(c[0]);
}

// Start of a trajectory (one workgroup per chain): momentum refresh (or the
// injected momentum), save of the current state, kinetic energy and H0 in
// FP64, first half kick with the cached gradient, first drift and scatter.
template <int P>
__global__ __launch_bounds__(256) void k_traj_begin(const StateArgs s) {
    typedef typename PT<P>::S S;
    __shared__ double red[NWAVE];
    const int c = blockIdx.x;
    if (!s.active[c]) return;
    const long long o = s.offs[c];
    const int n = (int)(s.offs[c + 1] - o);
    const S e = (S)s.eps[c];
    const unsigned long long it = s.iter[c];
    S* th = reinterpret_cast<S*>(s.theta) + o;
    S* gr = reinterpret_cast<S*>(s.grad) + o;
    S* mo = reinterpret_cast<S*>(s.mom) + o;
    S* ths = reinterpret_cast<S*>(s.theta_save) + o;
    S* grs = reinterpret_cast<S*>(s.grad_save) + o;
    const S* minv = s.minv ? reinterpret_cast<const S*>(s.minv) + o : nullptr;
    const S* pin = s.p_in ? reinterpret_cast<const S*>(s.p_in) + o : nullptr;
    double kin = 0.0;
    for (int b = threadIdx.x; 4 * b < n; b += 256) {
        double z[4] = {0.0, 0.0, 0.0, 0.0};
        if (!pin) normals4(s.seed, c, it, (unsigned long long)b, z);
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * b + j;
            if (k >= n) break;
            const S m = minv ? minv[k] : (S)1;
            S p = pin ? pin[k] : (S)(z[j] / sqrt((double)m));
            S x = th[k];
            const S g = gr[k];
            ths[k] = x;
            grs[k] = g;
            kin += 0.5 * (double)m * (double)p * (double)p;
            if (s.split_n) {   // symmetric splitting: the batch kicks follow a fresh gradient
                mo[k] = p;
                continue;
            }
            p = p - (S)0.5 * e * g;
            x = x + e * m * p;
            mo[k] = p;
            th[k] = x;
            scatter<P>(s, c, o + k, x);
        }
    }
    kin = block_sum(kin, red);
    if (threadIdx.x == 0) {
        s.H0[c] = s.U[c] + kin;
        s.U_save[c] = s.U[c];
    }
}

struct DevStat { double H0, H1, log_u; int accepted, divergent; };

// End of a trajectory (one workgroup per chain).  END_ENERGY: U = likelihood
// partials + prior, stored as the current U.  END_TRAJ: also the kinetic
// energy and H1, state untouched.  END_METROPOLIS: accept iff
// log u < H0 - H1 with H1 finite; on rejection restore position, gradient
// and U; record the outcome and advance the iteration counter.
template <int P>
__global__ __launch_bounds__(256) void k_traj_end(const StateArgs s, int mode) {
    typedef typename PT<P>::S S;
    __shared__ double red[NWAVE];
    const int c = blockIdx.x;
    if (!s.active[c]) return;
    const long long o = s.offs[c];
    const int n = (int)(s.offs[c + 1] - o);
    S* th = reinterpret_cast<S*>(s.theta) + o;
    const S* mo = reinterpret_cast<const S*>(s.mom) + o;
    const S* minv = s.minv ? reinterpret_cast<const S*>(s.minv) + o : nullptr;
    double pri = 0.0, kin = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) {
        const double x = (double)th[k];
        pri += x * x;
        if (mode != END_ENERGY) {
            const double p = (double)mo[k];
            kin += (minv ? (double)minv[k] : 1.0) * p * p;
        }
    }
    pri = 0.5 * s.inv_prior_var * block_sum(pri, red);
    kin = 0.5 * block_sum(kin, red);
    double ul = 0.0;
    const int nsl = s.ulik_tiles * 8;   // eight per-wave slots per tile
    for (int t = threadIdx.x; t < nsl; t += 256) ul += s.ulik[(size_t)c * nsl + t];
    ul = block_sum(ul, red);
    const double U1 = ul + pri;
    if (mode == END_ENERGY) {
        if (threadIdx.x == 0) s.U[c] = U1;
        return;
    }
    const double H1 = U1 + kin;
    if (mode == END_TRAJ) {
        if (threadIdx.x == 0) s.H1[c] = H1;
        return;
    }
    const double H0 = s.H0[c];
    const unsigned long long it = s.iter[c];
    const double lu = log(metropolis_u(s.seed, c, it));
    const bool fin = isfinite(H1);
    const bool acc = fin && (lu < H0 - H1);
    if (!acc) {
        S* gr = reinterpret_cast<S*>(s.grad) + o;
        const S* ths = reinterpret_cast<const S*>(s.theta_save) + o;
        const S* grs = reinterpret_cast<const S*>(s.grad_save) + o;
        for (int k = threadIdx.x; k < n; k += 256) {
            const S x = ths[k];
            th[k] = x;
            gr[k] = grs[k];
            scatter<P>(s, c, o + k, x);
        }
    }
    if (threadIdx.x == 0) {
        s.U[c] = acc ? U1 : s.U_save[c];
        s.H1[c] = H1;
        DevStat st{H0, H1, lu, acc ? 1 : 0, fin ? 0 : 1};
        reinterpret_cast<DevStat*>(s.stats)[c] = st;
        s.n_acc[c] += acc ? 1 : 0;
        s.n_div[c] += fin ? 0 : 1;
        s.iter[c] = it + 1;
        const int adapt = *s.adapt_on;
        if (adapt == 2) {
            // calibration: count and sum of the acceptance probabilities
            double* d = s.da + 4 * c;
            d[0] += 1.0;
            d[1] += fin ? fmin(1.0, exp(H0 - H1)) : 0.0;
        } else if (adapt == 1) {
            // Dual averaging of the step size toward a target acceptance
            // statistic (Hoffman and Gelman 2014, HMC with dual averaging,
            // the scheme Sec. 4.2.3 uses for its 80% runs): with alpha the
            // Metropolis acceptance probability of this trajectory (0 when
            // divergent), after iteration m
            //   H-bar_m = (1 - 1/(m + t0)) H-bar_{m-1} + (target - alpha)/(m + t0)
            //   log eps_{m+1} = mu - sqrt(m)/gamma * H-bar_m
            //   log eps-bar_{m+1} = m^-kappa log eps_{m+1} + (1 - m^-kappa) log eps-bar_m
            // and the next trajectory takes eps_{m+1}.
            double* d = s.da + 4 * c;
            const double target = s.da_cfg[0], gamma = s.da_cfg[1], t0 = s.da_cfg[2], kappa = s.da_cfg[3];
            const double alpha = fin ? fmin(1.0, exp(H0 - H1)) : 0.0;
            const double m = d[0] + 1.0;
            const double w = 1.0 / (m + t0);
            const double hbar = (1.0 - w) * d[1] + w * (target - alpha);
            const double log_eps = d[3] - sqrt(m) / gamma * hbar;
            const double eta = pow(m, -kappa);
            d[0] = m;
            d[1] = hbar;
            d[2] = eta * log_eps + (1.0 - eta) * d[2];
            s.eps[c] = exp(log_eps);
        }
    }
}

// The momentum that iteration `iter_override` would draw (no state change).
template <int P>
__global__ __launch_bounds__(256) void k_momentum(const StateArgs s) {
    typedef typename PT<P>::S S;
    const int c = blockIdx.x;
    const long long o = s.offs[c];
    const int n = (int)(s.offs[c + 1] - o);
    S* out = reinterpret_cast<S*>(s.p_out) + o;
    const S* minv = s.minv ? reinterpret_cast<const S*>(s.minv) + o : nullptr;
    for (int b = threadIdx.x; 4 * b < n; b += 256) {
        double z[4];
        normals4(s.seed, c, s.iter_override, (unsigned long long)b, z);
        for (int j = 0; j < 4 && 4 * b + j < n; ++j) {
            const int k = 4 * b + j;
            const double m = minv ? (double)minv[k] : 1.0;
            out[k] = (S)(z[j] / sqrt(m));
        }
    }
}

// Puts back the state saved at the start of a trajectory.
template <int P>
__global__ __launch_bounds__(256) void k_restore(const StateArgs s) {
    typedef typename PT<P>::S S;
    const int c = blockIdx.x;
    if (!s.active[c]) return;
    const long long o = s.offs[c];
    const int n = (int)(s.offs[c + 1] - o);
    for (int k = threadIdx.x; k < n; k += 256) {
        const S x = reinterpret_cast<const S*>(s.theta_save)[o + k];
        reinterpret_cast<S*>(s.theta)[o + k] = x;
        reinterpret_cast<S*>(s.grad)[o + k] = reinterpret_cast<const S*>(s.grad_save)[o + k];
        scatter<P>(s, c, o + k, x);
    }
    if (threadIdx.x == 0) s.U[c] = s.U_save[c];
}

// Writes every chain's current positions into its dense weights.
template <int P>
__global__ __launch_bounds__(256) void k_scatter_all(const StateArgs s) {
    typedef typename PT<P>::S S;
    const int c = blockIdx.x;
    const long long o = s.offs[c];
    const int n = (int)(s.offs[c + 1] - o);
    for (int k = threadIdx.x; k < n; k += 256)
        scatter<P>(s, c, o + k, reinterpret_cast<const S*>(s.theta)[o + k]);
}

// DeepONet posterior predictive combination: G[j][q] = <B_j, T_q> + b0 from
// the tower outputs of the new functions (Bn, [n_u][ld]) and query points
// (Tn, [n_q][ld]), products accumulated in the accumulator type, folded into
// the FP64 running moments as EpiPredict does.  One thread per (j, q).
template <int P>
__global__ __launch_bounds__(256) void k_combine_predict(const void* Bn, const void* Tn, int ld, int p, long long nu,
                                                         long long nq, const void* b0, double* mean, double* m2,
                                                         double* var, double inv_k, double inv_n) {
    typedef typename PT<P>::T T; typedef typename PT<P>::A A;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= nu * nq) return;
    const long long j = i / nq, q = i - j * nq;
    const T* b = reinterpret_cast<const T*>(Bn) + (size_t)j * ld;
    const T* t = reinterpret_cast<const T*>(Tn) + (size_t)q * ld;
    A s = (A)0;
    for (int k = 0; k < p; ++k) s = fma((A)b[k], (A)t[k], s);
    const double f = (double)s + (double)*reinterpret_cast<const A*>(b0);
    const double mu = mean[i], d = f - mu, mu2 = mu + d * inv_k;
    const double qq = m2[i] + d * (f - mu2);
    mean[i] = mu2;
    m2[i] = qq;
    if (var) var[i] = qq * inv_n;
}

// Writes a given position vector of chain c (state type, [n_c]) into the
// chain's dense weights and biases (all copies), as the drift's scatter does.
template <int P>
__global__ __launch_bounds__(256) void k_scatter_vec(const StateArgs s, int c, const void* vec) {
    typedef typename PT<P>::S S;
    const long long o = s.offs[c];
    const long long n = s.offs[c + 1] - o;
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    scatter<P>(s, c, o + k, reinterpret_cast<const S*>(vec)[k]);
}

template <int P, int R>
hipError_t set_lds(size_t lds) {
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void*)k_mlp_grad<P, R, false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds))) return e;
    if constexpr (P == 1 && R == 32) {   // the tile-group instance
        if ((e = hipFuncSetAttribute((const void*)k_mlp_grad<1, R, false, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds))) return e;
    }
    if ((e = hipFuncSetAttribute((const void*)k_trunk_fwd<P, R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds))) return e;
    if ((e = hipFuncSetAttribute((const void*)k_branch_grad<P, R, false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds))) return e;
    if ((e = hipFuncSetAttribute((const void*)k_trunk_bwd<P, R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds))) return e;
    if constexpr (P < 2) {
        if ((e = hipFuncSetAttribute((const void*)k_tower_sens<P, R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds))) return e;
        if ((e = hipFuncSetAttribute((const void*)k_tower_out<P, R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds))) return e;
        if ((e = hipFuncSetAttribute((const void*)k_mlp_predict<P, R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds))) return e;
    }
    if constexpr (P < 2) {   // the energy passes (FP32 or FP64)
        if ((e = hipFuncSetAttribute((const void*)k_mlp_grad<P, R, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds))) return e;
        if ((e = hipFuncSetAttribute((const void*)k_branch_grad<P, R, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds))) return e;
    }
    return hipSuccess;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.

#define HMC_DISPATCH_PR(P, R, CALL)                                            \
    switch ((P) * 100 + (R)) {                                                 \
        case 16: CALL(0, 16); case 32: CALL(0, 32); case 64: CALL(0, 64);     \
        case 116: CALL(1, 16); case 132: CALL(1, 32); case 164: CALL(1, 64);  \
        case 216: CALL(2, 16); case 232: CALL(2, 32); case 264: CALL(2, 64);  \
        case 316: CALL(3, 16); case 332: CALL(3, 32); case 364: CALL(3, 64);  \
        default: return hipErrorInvalidValue;                                  \
    }

#define HMC_DISPATCH_P(P, CALL)                                                \
    switch (P) {                                                               \
        case 0: CALL(0); case 1: CALL(1); case 2: CALL(2); case 3: CALL(3);    \
        default: return hipErrorInvalidValue;                                  \
    }

hipError_t hmc_launch_tower_sens(int P, int R, int nt, const GradArgs& a, int tower, const void* seed, int grid,
                                 size_t lds, hipStream_t s) {
#define C_(p, r) hipLaunchKernelGGL((k_tower_sens<p, r>), dim3(grid), dim3(nt), lds, s, a, tower, seed); \
    return hipGetLastError()
    switch (P * 100 + R) {
        case 16: C_(0, 16); case 32: C_(0, 32); case 64: C_(0, 64);
        case 116: C_(1, 16); case 132: C_(1, 32); case 164: C_(1, 64);
        default: return hipErrorInvalidValue;
    }
#undef C_
}

hipError_t hmc_launch_tower_out(int P, int R, int nt, const GradArgs& a, int tower, void* out, int ld, int grid,
                                size_t lds, hipStream_t s) {
#define C_(p, r) hipLaunchKernelGGL((k_tower_out<p, r>), dim3(grid), dim3(nt), lds, s, a, tower, out, ld); \
    return hipGetLastError()
    switch (P * 100 + R) {
        case 16: C_(0, 16); case 32: C_(0, 32); case 64: C_(0, 64);
        case 116: C_(1, 16); case 132: C_(1, 32); case 164: C_(1, 64);
        default: return hipErrorInvalidValue;
    }
#undef C_
}

hipError_t hmc_launch_sens_reduce(int P, const void* part, int tiles, long long n, long long k0, long long k1,
                                  double* acc, const double* sigma, double inv_nd, double* s2, hipStream_t s) {
    const unsigned g = (unsigned)((k1 - k0 + 255) / 256);
    if (g == 0) return hipSuccess;
    if (P == 0)
        hipLaunchKernelGGL((k_sens_reduce<0>), dim3(g), dim3(256), 0, s, part, tiles, n, k0, k1, acc, sigma, inv_nd, s2);
    else if (P == 1)
        hipLaunchKernelGGL((k_sens_reduce<1>), dim3(g), dim3(256), 0, s, part, tiles, n, k0, k1, acc, sigma, inv_nd, s2);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t hmc_launch_mlp_predict(int P, int R, int nt, const GradArgs& a, int c, int grid, size_t lds,
                                  hipStream_t s, double* mean, double* m2, double* var, double inv_k, double inv_n) {
#define C_(p, r) hipLaunchKernelGGL((k_mlp_predict<p, r>), dim3(grid), dim3(nt), lds, s, a, c, mean, m2, var, inv_k, \
                                   inv_n); return hipGetLastError()
    switch (P * 100 + R) {
        case 16: C_(0, 16); case 32: C_(0, 32); case 64: C_(0, 64);
        case 116: C_(1, 16); case 132: C_(1, 32); case 164: C_(1, 64);
        default: return hipErrorInvalidValue;
    }
#undef C_
}

hipError_t hmc_launch_combine_predict(int P, const void* Bn, const void* Tn, int ld, int p, long long nu, long long nq,
                                     const void* b0, double* mean, double* m2, double* var, double inv_k,
                                     double inv_n, hipStream_t s) {
    const unsigned g = (unsigned)((nu * nq + 255) / 256);
    if (P == 0)
        hipLaunchKernelGGL((k_combine_predict<0>), dim3(g), dim3(256), 0, s, Bn, Tn, ld, p, nu, nq, b0, mean, m2, var,
                           inv_k, inv_n);
    else if (P == 1)
        hipLaunchKernelGGL((k_combine_predict<1>), dim3(g), dim3(256), 0, s, Bn, Tn, ld, p, nu, nq, b0, mean, m2, var,
                           inv_k, inv_n);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// Zero fill of n doubles (a kernel rather than a memset, so that callers
// may capture it in a graph).
__global__ __launch_bounds__(256) void k_zero_f64(double* p, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

hipError_t hmc_launch_zero(double* p, long long n, hipStream_t s) {
    const unsigned g = (unsigned)((n + 255) / 256);
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_f64, dim3(g), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t hmc_launch_scatter_vec(int P, const StateArgs& sa, int c, const void* vec, long long n, hipStream_t s) {
    const unsigned g = (unsigned)((n + 255) / 256);
    if (g == 0) return hipSuccess;
    switch (P) {
        case 0: hipLaunchKernelGGL((k_scatter_vec<0>), dim3(g), dim3(256), 0, s, sa, c, vec); break;
        case 1: hipLaunchKernelGGL((k_scatter_vec<1>), dim3(g), dim3(256), 0, s, sa, c, vec); break;
        case 2: hipLaunchKernelGGL((k_scatter_vec<2>), dim3(g), dim3(256), 0, s, sa, c, vec); break;
        case 3: hipLaunchKernelGGL((k_scatter_vec<3>), dim3(g), dim3(256), 0, s, sa, c, vec); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t hmc_set_lds_limit(int P, int R, size_t lds) {
#define C_(p, r) return set_lds<p, r>(lds)
    HMC_DISPATCH_PR(P, R, C_)
#undef C_
}

#define HMC_TILE_CALL_k_mlp_grad(p, r) \
    hipLaunchKernelGGL((k_mlp_grad<p, r, false>), dim3(grid), dim3(nt), lds, s, a); return hipGetLastError()
#define HMC_TILE_CALL_k_trunk_fwd(p, r) \
    hipLaunchKernelGGL((k_trunk_fwd<p, r>), dim3(grid), dim3(nt), lds, s, a); return hipGetLastError()
#define HMC_TILE_CALL_k_branch_grad(p, r) \
    hipLaunchKernelGGL((k_branch_grad<p, r, false>), dim3(grid), dim3(nt), lds, s, a); return hipGetLastError()
#define HMC_TILE_CALL_k_trunk_bwd(p, r) \
    hipLaunchKernelGGL((k_trunk_bwd<p, r>), dim3(grid), dim3(nt), lds, s, a); return hipGetLastError()

// nt: threads per workgroup, 256 or 512 (the tile kernels are written for
// any multiple of 64 up to HMC_NT).
hipError_t hmc_launch_mlp_grad(int P, int R, int nt, const GradArgs& a, int grid, size_t lds, hipStream_t s) {
    if (a.tpg > 1) {   // tile groups: instantiated for FP32 products at 32 rows (tile_group)
        if (P != 1 || R != 32) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_mlp_grad<1, 32, false, true>), dim3(grid), dim3(nt), lds, s, a);
        return hipGetLastError();
    }
    HMC_DISPATCH_PR(P, R, HMC_TILE_CALL_k_mlp_grad)
}
hipError_t hmc_launch_trunk_fwd(int P, int R, int nt, const GradArgs& a, int grid, size_t lds, hipStream_t s) {
    HMC_DISPATCH_PR(P, R, HMC_TILE_CALL_k_trunk_fwd)
}
hipError_t hmc_launch_branch_grad(int P, int R, int nt, const GradArgs& a, int grid, size_t lds, hipStream_t s) {
    HMC_DISPATCH_PR(P, R, HMC_TILE_CALL_k_branch_grad)
}
hipError_t hmc_launch_trunk_bwd(int P, int R, int nt, const GradArgs& a, int grid, size_t lds, hipStream_t s) {
    HMC_DISPATCH_PR(P, R, HMC_TILE_CALL_k_trunk_bwd)
}

// FP32 energy pass (forward and likelihood partials only).
// Energy passes (forward and likelihood partials only) in FP32 (P = 1) or
// FP64 (P = 0).
template <int P>
hipError_t launch_energy_mlp(int R, int nt, const GradArgs& a, int grid, size_t lds, hipStream_t s) {
    switch (R) {
        case 16: hipLaunchKernelGGL((k_mlp_grad<P, 16, true>), dim3(grid), dim3(nt), lds, s, a); break;
        case 32: hipLaunchKernelGGL((k_mlp_grad<P, 32, true>), dim3(grid), dim3(nt), lds, s, a); break;
        case 64: hipLaunchKernelGGL((k_mlp_grad<P, 64, true>), dim3(grid), dim3(nt), lds, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template <int P>
hipError_t launch_energy_branch(int R, int nt, const GradArgs& a, int grid, size_t lds, hipStream_t s) {
    switch (R) {
        case 16: hipLaunchKernelGGL((k_branch_grad<P, 16, true>), dim3(grid), dim3(nt), lds, s, a); break;
        case 32: hipLaunchKernelGGL((k_branch_grad<P, 32, true>), dim3(grid), dim3(nt), lds, s, a); break;
        case 64: hipLaunchKernelGGL((k_branch_grad<P, 64, true>), dim3(grid), dim3(nt), lds, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
hipError_t hmc_launch_mlp_energy(int P, int R, int nt, const GradArgs& a, int grid, size_t lds, hipStream_t s) {
    if (P == 0) return launch_energy_mlp<0>(R, nt, a, grid, lds, s);
    if (P == 1) return launch_energy_mlp<1>(R, nt, a, grid, lds, s);
    return hipErrorInvalidValue;
}
hipError_t hmc_launch_branch_energy(int P, int R, int nt, const GradArgs& a, int grid, size_t lds, hipStream_t s) {
    if (P == 0) return launch_energy_branch<0>(R, nt, a, grid, lds, s);
    if (P == 1) return launch_energy_branch<1>(R, nt, a, grid, lds, s);
    return hipErrorInvalidValue;
}

hipError_t hmc_launch_update(int P, const StateArgs& s, int mode, int gx, int sub, hipStream_t st) {
#define C_(p) hipLaunchKernelGGL((k_update<p>), dim3(gx, s.n_chains), dim3(256), 0, st, s, mode, sub); return hipGetLastError()
    HMC_DISPATCH_P(P, C_)
#undef C_
}
hipError_t hmc_launch_update_split(int P, const StateArgs& s, int mode, int gx, hipStream_t st) {
#define C_(p) hipLaunchKernelGGL((k_update_split<p>), dim3(gx, s.n_chains), dim3(256), 0, st, s, mode); return hipGetLastError()
    HMC_DISPATCH_P(P, C_)
#undef C_
}

hipError_t hmc_launch_traj_begin(int P, const StateArgs& s, hipStream_t st) {
#define C_(p) hipLaunchKernelGGL((k_traj_begin<p>), dim3(s.n_chains), dim3(256), 0, st, s); return hipGetLastError()
    HMC_DISPATCH_P(P, C_)
#undef C_
}
hipError_t hmc_launch_traj_end(int P, const StateArgs& s, int mode, hipStream_t st) {
#define C_(p) hipLaunchKernelGGL((k_traj_end<p>), dim3(s.n_chains), dim3(256), 0, st, s, mode); return hipGetLastError()
    HMC_DISPATCH_P(P, C_)
#undef C_
}
hipError_t hmc_launch_momentum(int P, const StateArgs& s, hipStream_t st) {
#define C_(p) hipLaunchKernelGGL((k_momentum<p>), dim3(s.n_chains), dim3(256), 0, st, s); return hipGetLastError()
    HMC_DISPATCH_P(P, C_)
#undef C_
}
hipError_t hmc_launch_restore(int P, const StateArgs& s, hipStream_t st) {
#define C_(p) hipLaunchKernelGGL((k_restore<p>), dim3(s.n_chains), dim3(256), 0, st, s); return hipGetLastError()
    HMC_DISPATCH_P(P, C_)
#undef C_
}
hipError_t hmc_launch_scatter_all(int P, const StateArgs& s, hipStream_t st) {
#define C_(p) hipLaunchKernelGGL((k_scatter_all<p>), dim3(s.n_chains), dim3(256), 0, st, s); return hipGetLastError()
    HMC_DISPATCH_P(P, C_)
#undef C_
}
