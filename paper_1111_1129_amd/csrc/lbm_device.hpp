// lbm_device.hpp -- device-side building blocks of the gfx950 library:
// the D3Q19 velocity set, storage traits, the TRT collision of one cell, and
// launch helpers.  Included by every .hip translation unit of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "lbm.h"

namespace lbm {

// ---------------------------------------------------------------------------
// D3Q19.  Populations come in opposite pairs (2k-1, 2k), k = 1..9; the odd
// member's velocity is listed, the even member is its negative.
// ---------------------------------------------------------------------------
constexpr int Q = 19;
constexpr int NPAIR = 9;
// velocity of the odd member 2k-1 of pair k (index k-1)
constexpr int PCX[NPAIR] = {1, 0, 0, 1, 1, 1, 1, 0, 0};
constexpr int PCY[NPAIR] = {0, 1, 0, 1, -1, 0, 0, 1, 1};
constexpr int PCZ[NPAIR] = {0, 0, 1, 0, 0, 1, -1, 1, -1};
// 1/18 for the three axis pairs, 1/36 for the six diagonal pairs
__host__ __device__ constexpr double pair_weight(int k) { return k < 3 ? 1.0 / 18.0 : 1.0 / 36.0; }
constexpr double W0 = 1.0 / 3.0;

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr int vel_x(int i) { return i == 0 ? 0 : ((i & 1) ? PCX[(i - 1) / 2] : -PCX[(i - 1) / 2]); }
__host__ __device__ constexpr int vel_y(int i) { return i == 0 ? 0 : ((i & 1) ? PCY[(i - 1) / 2] : -PCY[(i - 1) / 2]); }
__host__ __device__ constexpr int vel_z(int i) { return i == 0 ? 0 : ((i & 1) ? PCZ[(i - 1) / 2] : -PCZ[(i - 1) / 2]); }
__host__ __device__ constexpr double weight(int i) { return i == 0 ? W0 : pair_weight((i - 1) / 2); }

// ---------------------------------------------------------------------------
// Storage traits: element type T in memory, arithmetic type A, shift flag.
// ---------------------------------------------------------------------------
template <int ST> struct Storage;
template <> struct Storage<LBM_F64> { using T = double; using A = double; static constexpr bool shifted = false; };
template <> struct Storage<LBM_F64_SHIFTED> { using T = double; using A = double; static constexpr bool shifted = true; };
template <> struct Storage<LBM_F32> { using T = float; using A = float; static constexpr bool shifted = false; };
template <> struct Storage<LBM_F32_SHIFTED> { using T = float; using A = float; static constexpr bool shifted = true; };
template <> struct Storage<LBM_F16_SHIFTED> { using T = _Float16; using A = float; static constexpr bool shifted = true; };

// FP16 holding 2^12 x the value (LBM_F16_SHIFTED_SCALED).  Scaling by a power
// of two is exact in FP32, so loading and storing round exactly as the
// unscaled FP16 form does, only in a range shifted down by 12 binades.
struct Half12 {
    _Float16 bits;
    static constexpr float kUp = 4096.0f, kDown = 1.0f / 4096.0f;
    __host__ __device__ explicit operator float() const { return static_cast<float>(bits) * kDown; }
    __host__ __device__ explicit operator double() const {
        return static_cast<double>(static_cast<float>(bits) * kDown);
    }
};
template <> struct Storage<LBM_F16_SHIFTED_SCALED> { using T = Half12; using A = float; static constexpr bool shifted = true; };

template <class T, class A> __device__ __forceinline__ A ld(const T* p) { return static_cast<A>(*p); }
// Read-once streams (adjacency rows, adjacency codes): nontemporal loads keep
// them from displacing the PDF lines whose partial reuse by neighbouring
// cells the caches serve (measured: 2 % faster sweep over codes in FP64).
template <class T> __device__ __forceinline__ T ld_stream(const T* p) {
    return __builtin_nontemporal_load(p);
}
__device__ __forceinline__ Half12 ld_stream(const Half12* p) {
    return Half12{__builtin_nontemporal_load(&p->bits)};
}
// FP32 -> FP16 conversion rounds to nearest even (IEEE default mode).  The
// value is first rounded to A: device code is built without contraction, so
// no fused product-sum exists that the conversion could absorb, and the empty
// asm hides how the value was computed, so no mixed-precision instruction can
// round an unrounded result straight to FP16 (with contraction on, the
// compiler once did so in one kernel and not in another, and their results
// differed in the last bit).
template <class T, class A, bool NT> __device__ __forceinline__ void st(T* p, A v) {
    if constexpr (!std::is_same_v<T, A>) asm("" : "+v"(v));
    if constexpr (std::is_same_v<T, Half12>) {
        const _Float16 b = static_cast<_Float16>(v * Half12::kUp);  // exact scaling, one rounding
        if constexpr (NT)
            __builtin_nontemporal_store(b, &p->bits);
        else
            p->bits = b;
    } else if constexpr (NT) {
        __builtin_nontemporal_store(static_cast<T>(v), p);
    } else {
        *p = static_cast<T>(v);
    }
}

inline size_t storage_bytes(int st) {
    switch (st) {
    case LBM_F64: case LBM_F64_SHIFTED: return 8;
    case LBM_F32: case LBM_F32_SHIFTED: return 4;
    case LBM_F16_SHIFTED: case LBM_F16_SHIFTED_SCALED: return 2;
    default: return 0;
    }
}

// 16-bit adjacency codes (lbm_compress_adjacency): tiles of 256 list cells,
// one record of 20 int32 words per tile (18 direction offsets, the number of
// escape codes in the tile, the narrow flag of lbm_narrow_codes); reserved
// code values.
constexpr int kCodeTile = 256;
constexpr int kCodeRec = 20;
constexpr int16_t kCodeBounce = -32768;
constexpr int16_t kCodeEscape = -32767;
constexpr int32_t kCodeMin = -32766;
constexpr int32_t kCodeMax = 32767;
// 8-bit form of a tile's codes (lbm_narrow_codes): the same code in one byte,
// bounce-back as -128.
constexpr int8_t kCode8Bounce = -128;
constexpr int32_t kCode8Max = 127;

// ---------------------------------------------------------------------------
// TRT constants of one launch (host-computed in FP64).
// ---------------------------------------------------------------------------
struct TrtConst {
    double sp, sm;       // s+ = 1/tau+, s- = 1/tau-
    double G[3];         // body force
    double F[NPAIR];     // 3 w c.G for the odd member of each pair
};

inline TrtConst make_trt_const(const lbm_params& p) {
    TrtConst c;
    double tau_minus = 0.5 + p.magic / (p.tau_plus - 0.5);
    c.sp = 1.0 / p.tau_plus;
    c.sm = 1.0 / tau_minus;
    for (int d = 0; d < 3; ++d) c.G[d] = p.force[d];
    for (int k = 0; k < NPAIR; ++k)
        c.F[k] = 3.0 * pair_weight(k) * (PCX[k] * p.force[0] + PCY[k] * p.force[1] + PCZ[k] * p.force[2]);
    return c;
}

// ---------------------------------------------------------------------------
// One cell's TRT collision.  g[19] are the gathered populations (pre-collision),
// in the arithmetic type A.  Writes the post-collision f*[19] into out[] and,
// if PBB, blends with the bounce-back g_opp.  rho/j are returned for callers
// that need them (the adjoint).
// ---------------------------------------------------------------------------
template <class A>
struct CellMoments {
    A rho, jx, jy, jz;
};

template <class A>
__device__ __forceinline__ CellMoments<A> cell_moments(const A* g) {
    CellMoments<A> m;
    A rho = g[0];
    A d[NPAIR];
#pragma unroll
    for (int k = 0; k < NPAIR; ++k) {
        rho += g[2 * k + 1] + g[2 * k + 2];
        d[k] = g[2 * k + 1] - g[2 * k + 2];
    }
    m.rho = rho;
    // j = sum over pairs of c_odd * (g_odd - g_even)
    m.jx = d[0] + d[3] + d[4] + d[5] + d[6];
    m.jy = d[1] + d[3] - d[4] + d[7] + d[8];
    m.jz = d[2] + d[5] - d[6] + d[7] - d[8];
    return m;
}

template <class A, bool PBB>
__device__ __forceinline__ void trt_collide(const A* g, A* out, const TrtConst& c, A ns) {
    const CellMoments<A> m = cell_moments(g);
    const A sp = static_cast<A>(c.sp), sm = static_cast<A>(c.sm);
    const A jj = m.jx * m.jx + m.jy * m.jy + m.jz * m.jz;
    const A base = m.rho - A(1.5) * jj;  // rho - 3/2 |j|^2
    // rest population: g+ = g0, g- = 0, e+ = w0 (rho - 3/2 |j|^2)
    A f0 = g[0] - sp * (g[0] - static_cast<A>(W0) * base);
    if constexpr (PBB) f0 = (A(1) - ns) * f0 + ns * g[0];
    out[0] = f0;
#pragma unroll
    for (int k = 0; k < NPAIR; ++k) {
        const int a = 2 * k + 1, b = 2 * k + 2;
        const A w = static_cast<A>(pair_weight(k));
        const A cu = A(PCX[k]) * m.jx + A(PCY[k]) * m.jy + A(PCZ[k]) * m.jz;
        const A ep = w * (base + A(4.5) * cu * cu);
        const A em = A(3) * w * cu;
        const A gp = A(0.5) * (g[a] + g[b]);
        const A gm = A(0.5) * (g[a] - g[b]);
        const A rp = sp * (gp - ep);
        const A rm = sm * (gm - em);
        const A F = static_cast<A>(c.F[k]);
        A fa = g[a] - rp - rm + F;
        A fb = g[b] - rp + rm - F;
        if constexpr (PBB) {
            fa = (A(1) - ns) * fa + ns * g[b];
            fb = (A(1) - ns) * fb + ns * g[a];
        }
        out[a] = fa;
        out[b] = fb;
    }
}

// ---------------------------------------------------------------------------
// One cell update of the pull sweep: gather the 18 upstream populations
// through adj (plus the own rest population), collide, store the 19 results
// to the cell's own column of the destination rows.
// ---------------------------------------------------------------------------
template <int ST, bool PBB, bool NT>
__device__ __forceinline__ void update_cell(const typename Storage<ST>::T* __restrict__ src,
                                            typename Storage<ST>::T* __restrict__ dst,
                                            const uint32_t* __restrict__ adj,
                                            const double* __restrict__ ns, int64_t m,
                                            int64_t stride, const TrtConst& c) {
    using T = typename Storage<ST>::T;
    using A = typename Storage<ST>::A;
    uint32_t a[Q - 1];
    const uint32_t* ap = adj + m;
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) a[k] = ld_stream(ap + k * stride);
    A g[Q];
    g[0] = ld<T, A>(src + m);
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) g[k + 1] = ld<T, A>(src + a[k]);
    A s = A(0);
    if constexpr (PBB) s = static_cast<A>(ns[m]);
    A out[Q];
    trt_collide<A, PBB>(g, out, c, s);
    T* dp = dst + m;
#pragma unroll
    for (int i = 0; i < Q; ++i) st<T, A, NT>(dp + i * stride, out[i]);
}

// One cell update of an escape-free tile, the slots rebuilt from the 16-bit
// (CT = int16_t) or 8-bit (int8_t) codes in 32-bit arithmetic (every slot is
// below 19 * stride < 2^32).  The per-tile part i * stride + tile * 256 + toff
// is uniform (scalar); per lane it adds the lane and the code.
template <int ST, bool PBB, bool NT, class CT>
__device__ __forceinline__ void update_cell_coded(const typename Storage<ST>::T* __restrict__ src,
                                                  typename Storage<ST>::T* __restrict__ dst,
                                                  const CT* __restrict__ codes,
                                                  const int32_t* __restrict__ rec,
                                                  const double* __restrict__ ns, int64_t m,
                                                  int64_t stride, const TrtConst& c) {
    using T = typename Storage<ST>::T;
    using A = typename Storage<ST>::A;
    constexpr int32_t bounce = std::is_same_v<CT, int8_t> ? int32_t(kCode8Bounce)
                                                          : int32_t(kCodeBounce);
    int32_t cd[Q - 1];
    const CT* cp = codes + m;
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) cd[k] = ld_stream(cp + k * stride);
    const uint32_t S = uint32_t(stride);
    const uint32_t mm = uint32_t(m);
    A g[Q];
    g[0] = ld<T, A>(src + m);
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) {
        const uint32_t i = k + 1;
        const uint32_t streamed = i * S + uint32_t(rec[k]) + mm + uint32_t(cd[k]);
        const uint32_t bounced = uint32_t(opp(int(i))) * S + mm;
        g[i] = ld<T, A>(src + (cd[k] == bounce ? bounced : streamed));
    }
    A sf = A(0);
    if constexpr (PBB) sf = static_cast<A>(ns[m]);
    A out[Q];
    trt_collide<A, PBB>(g, out, c, sf);
    T* dp = dst + m;
#pragma unroll
    for (int i = 0; i < Q; ++i) st<T, A, NT>(dp + i * stride, out[i]);
}

// ---------------------------------------------------------------------------
// Launch geometry.  Workgroups are handed to the 8 XCDs of the MI355X round
// robin (workgroup w runs on XCD w % 8; checked on the device through the
// XCC_ID hardware register), and each XCD has its own L2.  The sweep relabels
// workgroups so that each XCD takes `chunk` consecutive list tiles at a time:
// the gathers of neighbouring tiles share cache lines at tile edges, which
// then stay in one L2, while all XCDs still sweep nearby parts of the list
// (DRAM page locality).  chunk = grid/8 gives each XCD one contiguous eighth;
// chunk = 1 is the hardware order.
// ---------------------------------------------------------------------------
constexpr int NXCD = 8;

// chunk_shift = log2(chunk); the grid is a multiple of NXCD << chunk_shift.
__device__ __forceinline__ int64_t logical_block(int chunk_shift) {
    const int64_t b = blockIdx.x;
    const int64_t super = b >> (3 + chunk_shift);        // group of NXCD * chunk workgroups
    const int64_t xcd = b & (NXCD - 1);
    const int64_t within = (b >> 3) & ((int64_t(1) << chunk_shift) - 1);
    return (super << (3 + chunk_shift)) + (xcd << chunk_shift) + within;
}

// Grid for n cells in blocks of `block`, padded to a multiple of NXCD << shift.
inline int64_t grid_blocks(int64_t n, int block, int chunk_shift) {
    const int64_t g = (n + block - 1) / block;
    const int64_t q = int64_t(NXCD) << chunk_shift;
    return std::max<int64_t>(q, (g + q - 1) / q * q);
}

// log2 of the XCD chunk for n cells from the LBM_FLAG_XCD_CHUNK bits.
inline int chunk_shift_for(int32_t flags, int64_t n, int block) {
    const int64_t k = (flags & LBM_FLAG_XCD_CHUNK_MASK) >> LBM_FLAG_XCD_CHUNK_SHIFT;
    int64_t chunk = k;
    if (k == 0) chunk = ((n + block - 1) / block + NXCD - 1) / NXCD;  // one eighth each
    int s = 0;
    while ((int64_t(1) << (s + 1)) <= chunk && s < 24) ++s;  // largest power of two <= chunk
    return s;
}

}  // namespace lbm
