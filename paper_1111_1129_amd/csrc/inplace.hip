// inplace.hip -- the pull sweep with one PDF array instead of two
// (lbm_step_inplace).
//
// The two-array sweep keeps the post-collision state f*_i(x) in slot (i, x)
// ("layout P") and needs a second array to write into.  Here two kinds of
// step alternate on one array, so PDF memory halves (19 instead of 38 values
// per cell):
//  * gather-scatter step, layout P -> Q: cell x gathers g_i from slot adj(i, x)
//    exactly like the two-array sweep, collides, and writes out_i into the
//    slot it gathered direction opp(i) from, adj(opp(i), x).  That slot is
//    (opp(i), x + c_i) when x + c_i is fluid -- where x + c_i will look for
//    its incoming population i -- and (i, x) otherwise (bounce-back).  So
//    after the step slot (opp(i), y) holds the incoming f_i(y) ("layout Q").
//  * local step, layout Q -> P: cell x reads g_i from (opp(i), x), collides
//    and writes out_i to (i, x).  No adjacency is read.
// Every cell reads and writes the same 19 slots within a step and no other
// cell touches them (the pull adjacency is a permutation of the slots), so
// each thread loads all its slots before storing and steps need no other
// synchronisation than the launch boundary.  The collision sees exactly the
// values the two-array sweep sees, so after an even number of steps the
// array is bitwise the two-array result; the gather-scatter step can read
// the 16-bit codes of lbm_compress_adjacency instead of adj, and the 8-bit
// codes of lbm_narrow_codes in the tiles that have them.
// Per two steps a cell moves 2 x 19 x 2 PDFs and the adjacency once: 340
// bytes per FP64 update on average (322 with 16-bit codes, 313 with 8-bit
// codes in every tile) instead of 376.
#include <algorithm>

#include "lbm_device.hpp"
#include "lbm_host.hpp"

namespace lbm {

constexpr int kIBlock = kCodeTile;  // a workgroup is one tile of the codes

// Where the gather-scatter step finds a cell's slots.
enum SlotSource { kFromAdj = 0, kFrom16 = 1, kFrom8 = 2 };

// Slots rebuilt from the 16-bit (SRC = kFrom16) or 8-bit (kFrom8) codes of
// the cell's tile: s[k] = adj(k + 1, m).
template <int SRC, class CT>
__device__ __forceinline__ void slots_from_codes(uint32_t* s, const CT* __restrict__ codes,
                                                 const int32_t* __restrict__ rec, int64_t m,
                                                 int64_t stride) {
    constexpr int32_t bounce = SRC == kFrom8 ? int32_t(kCode8Bounce) : int32_t(kCodeBounce);
    const CT* cp = codes + m;
    int32_t cd[Q - 1];
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) cd[k] = ld_stream(cp + k * stride);
    const uint32_t S = uint32_t(stride), mm = uint32_t(m);
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) {
        const uint32_t i = k + 1;
        const uint32_t streamed = i * S + uint32_t(rec[k]) + mm + uint32_t(cd[k]);
        const uint32_t bounced = uint32_t(opp(int(i))) * S + mm;
        s[k] = cd[k] == bounce ? bounced : streamed;
    }
}

// Slots of the gather-scatter step for one cell: s[k] = adj(k + 1, m).
template <int SRC>
__device__ __forceinline__ void gather_slots(uint32_t* s, const uint32_t* __restrict__ adj,
                                             const int16_t* __restrict__ codes,
                                             const int8_t* __restrict__ codes8,
                                             const int32_t* __restrict__ rec, int64_t m,
                                             int64_t stride) {
    if constexpr (SRC == kFromAdj) {
        const uint32_t* ap = adj + m;
#pragma unroll
        for (int k = 0; k < Q - 1; ++k) s[k] = ld_stream(ap + k * stride);
    } else if constexpr (SRC == kFrom16) {
        slots_from_codes<kFrom16>(s, codes, rec, m, stride);
    } else {
        slots_from_codes<kFrom8>(s, codes8, rec, m, stride);
    }
}

template <int ST, bool PBB, bool NT, int SRC>
__device__ __forceinline__ void gather_scatter_cell(typename Storage<ST>::T* f,
                                                    const uint32_t* __restrict__ adj,
                                                    const int16_t* __restrict__ codes,
                                                    const int8_t* __restrict__ codes8,
                                                    const int32_t* __restrict__ rec,
                                                    const double* __restrict__ ns, int64_t m,
                                                    int64_t stride, const TrtConst& c) {
    using T = typename Storage<ST>::T;
    using A = typename Storage<ST>::A;
    uint32_t s[Q - 1];
    gather_slots<SRC>(s, adj, codes, codes8, rec, m, stride);
    A g[Q];
    g[0] = ld<T, A>(f + m);
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) g[k + 1] = ld<T, A>(f + s[k]);
    A sf = A(0);
    if constexpr (PBB) sf = static_cast<A>(ns[m]);
    A out[Q];
    trt_collide<A, PBB>(g, out, c, sf);
    st<T, A, NT>(f + m, out[0]);
    // out_i goes where direction opp(i) was gathered from
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) st<T, A, NT>(f + s[k], out[opp(k + 1)]);
}

// SRC: the narrowest code form the launch may use; each tile then takes what
// its record allows (a workgroup-uniform choice): 8-bit codes in a narrow
// tile (kFrom8 only), the full list in a tile with escapes, else 16-bit codes.
template <int ST, bool PBB, bool NT, int SRC>
__global__ __launch_bounds__(kIBlock) void k_gather_scatter(typename Storage<ST>::T* f,
                                                            const uint32_t* __restrict__ adj,
                                                            const int16_t* __restrict__ codes,
                                                            const int8_t* __restrict__ codes8,
                                                            const int32_t* __restrict__ tile_rec,
                                                            const double* __restrict__ ns,
                                                            int64_t n, int64_t stride, TrtConst c,
                                                            int chunk_shift) {
    const int64_t tile = logical_block(chunk_shift);
    const int64_t m = tile * kIBlock + threadIdx.x;
    if (m >= n) return;
    if constexpr (SRC == kFromAdj) {
        gather_scatter_cell<ST, PBB, NT, kFromAdj>(f, adj, codes, codes8, nullptr, ns, m, stride, c);
    } else {
        const int32_t* rec = tile_rec + tile * kCodeRec;  // uniform over the workgroup
        if (SRC == kFrom8 && rec[Q] != 0)
            gather_scatter_cell<ST, PBB, NT, kFrom8>(f, adj, codes, codes8, rec, ns, m, stride, c);
        else if (rec[Q - 1] != 0)  // the tile has escape codes: use the full list
            gather_scatter_cell<ST, PBB, NT, kFromAdj>(f, adj, codes, codes8, rec, ns, m, stride, c);
        else
            gather_scatter_cell<ST, PBB, NT, kFrom16>(f, adj, codes, codes8, rec, ns, m, stride, c);
    }
}

template <int ST, bool PBB, bool NT>
__global__ __launch_bounds__(kIBlock) void k_local(typename Storage<ST>::T* f,
                                                   const double* __restrict__ ns, int64_t n,
                                                   int64_t stride, TrtConst c, int chunk_shift) {
    using T = typename Storage<ST>::T;
    using A = typename Storage<ST>::A;
    const int64_t tile = logical_block(chunk_shift);
    const int64_t m = tile * kIBlock + threadIdx.x;
    if (m >= n) return;
    T* fp = f + m;
    A g[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) g[i] = static_cast<A>(ld_stream(fp + opp(i) * stride));  // own column only
    A sf = A(0);
    if constexpr (PBB) sf = static_cast<A>(ns[m]);
    A out[Q];
    trt_collide<A, PBB>(g, out, c, sf);
#pragma unroll
    for (int i = 0; i < Q; ++i) st<T, A, NT>(fp + i * stride, out[i]);
}

template <int ST, bool PBB, bool NT>
lbm_status launch_inplace(const TrtConst& c, int cs, int64_t n, int64_t stride,
                          const uint32_t* adj, const int16_t* codes, const int8_t* codes8,
                          const int32_t* rec, const double* ns, void* fv, int phase, int n_steps,
                          hipStream_t s) {
    using T = typename Storage<ST>::T;
    T* f = static_cast<T*>(fv);
    const int64_t grid = grid_blocks(n, kIBlock, cs);
    const dim3 g{unsigned(grid)}, b{unsigned(kIBlock)};
    for (int k = 0; k < n_steps; ++k) {
        if (((phase + k) & 1) == 0) {
            if (codes8)
                k_gather_scatter<ST, PBB, NT, kFrom8><<<g, b, 0, s>>>(f, adj, codes, codes8, rec, ns, n, stride, c, cs);
            else if (codes)
                k_gather_scatter<ST, PBB, NT, kFrom16><<<g, b, 0, s>>>(f, adj, codes, codes8, rec, ns, n, stride, c, cs);
            else
                k_gather_scatter<ST, PBB, NT, kFromAdj><<<g, b, 0, s>>>(f, adj, codes, codes8, rec, ns, n, stride, c, cs);
        } else {
            k_local<ST, PBB, NT><<<g, b, 0, s>>>(f, ns, n, stride, c, cs);
        }
        if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    }
    return LBM_OK;
}

template <int ST>
lbm_status dispatch_inplace(const lbm_params& p, int64_t n, int64_t stride, const uint32_t* adj,
                            const int16_t* codes, const int8_t* codes8, const int32_t* rec,
                            const double* ns, void* f, int phase, int n_steps, hipStream_t s) {
    const TrtConst c = make_trt_const(p);
    const int cs = chunk_shift_for(p.flags, n, kIBlock);
    const bool nt = p.flags & LBM_FLAG_NONTEMPORAL;
    if (ns)
        return nt ? launch_inplace<ST, true, true>(c, cs, n, stride, adj, codes, codes8, rec, ns, f, phase, n_steps, s)
                  : launch_inplace<ST, true, false>(c, cs, n, stride, adj, codes, codes8, rec, ns, f, phase, n_steps, s);
    return nt ? launch_inplace<ST, false, true>(c, cs, n, stride, adj, codes, codes8, rec, ns, f, phase, n_steps, s)
              : launch_inplace<ST, false, false>(c, cs, n, stride, adj, codes, codes8, rec, ns, f, phase, n_steps, s);
}

lbm_status step_inplace(const lbm_params& p, int64_t n, int64_t stride, const uint32_t* adj,
                        const int16_t* codes, const int8_t* codes8, const int32_t* rec,
                        const double* ns, void* f, int phase, int n_steps, hipStream_t s) {
    switch (p.storage) {
    case LBM_F64: return dispatch_inplace<LBM_F64>(p, n, stride, adj, codes, codes8, rec, ns, f, phase, n_steps, s);
    case LBM_F64_SHIFTED: return dispatch_inplace<LBM_F64_SHIFTED>(p, n, stride, adj, codes, codes8, rec, ns, f, phase, n_steps, s);
    case LBM_F32: return dispatch_inplace<LBM_F32>(p, n, stride, adj, codes, codes8, rec, ns, f, phase, n_steps, s);
    case LBM_F32_SHIFTED: return dispatch_inplace<LBM_F32_SHIFTED>(p, n, stride, adj, codes, codes8, rec, ns, f, phase, n_steps, s);
    case LBM_F16_SHIFTED: return dispatch_inplace<LBM_F16_SHIFTED>(p, n, stride, adj, codes, codes8, rec, ns, f, phase, n_steps, s);
    case LBM_F16_SHIFTED_SCALED: return dispatch_inplace<LBM_F16_SHIFTED_SCALED>(p, n, stride, adj, codes, codes8, rec, ns, f, phase, n_steps, s);
    default: return LBM_EINVAL;
    }
}

}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_step_inplace(const lbm_params* p, int64_t n, int64_t stride,
                                       const uint32_t* adj, const int16_t* codes,
                                       const int32_t* tile_records, const double* ns, void* f,
                                       int32_t phase, int32_t n_steps, void* stream) {
    if (!valid_params(p) || !adj || !f || n_steps < 0 || (phase != 0 && phase != 1))
        return LBM_EINVAL;
    if ((codes == nullptr) != (tile_records == nullptr)) return LBM_EINVAL;
    if (lbm_status st = check_layout(n, stride); st != LBM_OK) return st;
    if (n == 0 || n_steps == 0) return LBM_OK;
    return step_inplace(*p, n, stride, adj, codes, nullptr, tile_records, ns, f, phase, n_steps,
                        as_stream(stream));
}

extern "C" lbm_status lbm_step_inplace_c8(const lbm_params* p, int64_t n, int64_t stride,
                                          const uint32_t* adj, const int8_t* codes8,
                                          const int16_t* codes, const int32_t* tile_records,
                                          const double* ns, void* f, int32_t phase,
                                          int32_t n_steps, void* stream) {
    if (!valid_params(p) || !adj || !codes8 || !codes || !tile_records || !f || n_steps < 0 ||
        (phase != 0 && phase != 1))
        return LBM_EINVAL;
    if (lbm_status st = check_layout(n, stride); st != LBM_OK) return st;
    if (n == 0 || n_steps == 0) return LBM_OK;
    return step_inplace(*p, n, stride, adj, codes, codes8, tile_records, ns, f, phase, n_steps,
                        as_stream(stream));
}
