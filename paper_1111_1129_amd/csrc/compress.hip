// compress.hip -- 16-bit and 8-bit adjacency codes and the sweeps that read
// them (lbm_compress_adjacency, lbm_step_c16, lbm_narrow_codes, lbm_step_c8).
//
// The adjacency list is 72 of the 376 bytes a FP64 cell update moves (49 %
// of the 148 bytes in shifted FP16).  In a locality-preserving ordering the
// 256 cells of a tile pull a given direction from a nearby run of cells, so
// each entry is stored as
//   code  = src - m - toff[tile][k]   (-32766..32767) for a streaming entry,
//   code  = BOUNCE (-32768)           for the implicit bounce-back,
//   code  = ESCAPE (-32767)           if the difference does not fit,
// with one int32 offset toff per tile and direction (the midpoint of the
// tile's smallest and largest src - m).  A tile record holds the 18 offsets,
// the number of escapes in the tile and a flag word, 0 until lbm_narrow_codes
// sets it (80 bytes, two scalar loads).  The sweep rebuilds the exact slot i*stride + src from the codes
// (bounce-back: opp(i)*stride + m) in a tile without escapes, and reads the
// full list in a tile with any: the choice is uniform over the workgroup, so
// neither path branches per lane and every gather of a cell is in flight at
// once.  Results are bit-identical to the uncompressed sweep; the adjacency
// traffic of an escape-free tile drops from 72 to 36.3 bytes per cell.
//
// 8-bit codes (lbm_narrow_codes, lbm_step_c8): in a tile whose 16-bit codes
// all lie in -127..127 or are bounce-backs (most tiles of a lexicographic
// order: the offsets of a tile spread over little more than the fluid count
// of one row) the same codes fit one byte each, with -128 for bounce-back.
// Word 19 of the tile record marks such a tile; the sweep then reads 18 bytes
// of codes per cell instead of 36, and the other tiles as before.
#include <algorithm>
#include <type_traits>

#include "lbm_device.hpp"
#include "lbm_host.hpp"

namespace lbm {

constexpr int kCTile = kCodeTile;  // cells per tile = workgroup size of the sweep
constexpr int kRec = kCodeRec;

// One workgroup per tile.  Every thread stores its 18 offsets (int32: an
// offset is below stride < 2^32 / 19 in magnitude) to LDS; after one barrier
// each wave reduces the smallest and largest offset of every fourth
// direction (4 values per lane, then shuffles), and after a second barrier
// every thread encodes its entries against the 18 bases.
__global__ __launch_bounds__(kCTile) void k_compress(const uint32_t* __restrict__ adj, int64_t n,
                                                     int64_t stride, int16_t* __restrict__ codes,
                                                     int32_t* __restrict__ rec) {
    constexpr int kWaves = kCTile / 64;
    __shared__ int32_t lo_s[Q - 1][kCTile], hi_s[Q - 1][kCTile];
    __shared__ int32_t base_s[Q - 1];
    __shared__ unsigned int tile_esc;
    const int64_t tile = blockIdx.x;
    const int64_t m = tile * kCTile + threadIdx.x;
    const bool live = m < n;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (threadIdx.x == 0) tile_esc = 0;
    int32_t d[Q - 1];
    uint32_t streams = 0;  // bit k: entry k streams (is not a bounce-back)
    // lanes past the list read cell 0 (n > 0) and are ignored: no branch
    // around the loads, so all 18 are in flight at once
    const int64_t mc = live ? m : 0;
    uint32_t slot32[Q - 1];
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) slot32[k] = adj[k * stride + mc];
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) {
        const int64_t i = k + 1;
        const int64_t slot = slot32[k];
        // streaming entries lie in row i (a range test: no 64-bit division)
        if (live && slot >= i * stride && slot < (i + 1) * stride) streams |= 1u << k;
        d[k] = int32_t(slot - i * stride - mc);
        const bool st_k = (streams >> k) & 1u;
        lo_s[k][threadIdx.x] = st_k ? d[k] : INT32_MAX;
        hi_s[k][threadIdx.x] = st_k ? d[k] : INT32_MIN;
    }
    __syncthreads();
    for (int k = wave; k < Q - 1; k += kWaves) {
        int32_t lo = lo_s[k][lane], hi = hi_s[k][lane];
        for (int j = 1; j < kWaves; ++j) {
            lo = min(lo, lo_s[k][lane + 64 * j]);
            hi = max(hi, hi_s[k][lane + 64 * j]);
        }
        for (int off = 32; off > 0; off >>= 1) {
            lo = min(lo, __shfl_xor(lo, off));
            hi = max(hi, __shfl_xor(hi, off));
        }
        // midpoint of the tile's range (0 if nothing streams)
        if (lane == 0) base_s[k] = (lo <= hi) ? int32_t(lo + (int64_t(hi) - lo) / 2) : 0;
    }
    __syncthreads();
    unsigned int esc = 0;
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) {
        const int32_t base = base_s[k];
        if (threadIdx.x == 0) rec[tile * kRec + k] = base;
        if (live) {
            const int64_t r = int64_t(d[k]) - base;
            int16_t c;
            if (!((streams >> k) & 1u)) {
                c = kCodeBounce;
            } else if (r >= kCodeMin && r <= kCodeMax) {
                c = int16_t(r);
            } else {
                c = kCodeEscape;
                ++esc;
            }
            codes[k * stride + m] = c;
        }
    }
    if (esc) atomicAdd(&tile_esc, esc);
    __syncthreads();
    if (threadIdx.x == 0) {
        rec[tile * kRec + Q - 1] = int32_t(tile_esc);
        rec[tile * kRec + Q] = 0;
    }
}

// Sum of one word over all tile records in two passes: up to kSumParts
// workgroups each total a strided share of the tiles, then one workgroup adds
// the partial sums (the per-tile counts are totalled here rather than by a
// global atomic per tile, which the 8 XCDs would serialise on one address).
constexpr int kSumBlock = 256;
constexpr int kSumParts = 256;
constexpr size_t kSumWorkspace = (kSumParts + 1) * sizeof(unsigned long long);

__device__ __forceinline__ unsigned long long block_sum(unsigned long long v) {
    __shared__ unsigned long long part[kSumBlock / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (threadIdx.x % 64 == 0) part[threadIdx.x / 64] = v;
    __syncthreads();
    unsigned long long total = 0;
    for (int w = 0; w < kSumBlock / 64; ++w) total += part[w];
    return total;
}

__global__ __launch_bounds__(kSumBlock) void k_sum_records(const int32_t* __restrict__ rec,
                                                           int64_t tiles, int word,
                                                           unsigned long long* __restrict__ parts) {
    unsigned long long s = 0;
    const int64_t step = int64_t(gridDim.x) * kSumBlock;
    for (int64_t t = int64_t(blockIdx.x) * kSumBlock + threadIdx.x; t < tiles; t += step)
        s += uint32_t(rec[t * kRec + word]);
    const unsigned long long total = block_sum(s);
    if (threadIdx.x == 0) parts[blockIdx.x] = total;
}

__global__ __launch_bounds__(kSumBlock) void k_sum_parts(const unsigned long long* __restrict__ parts,
                                                         int n_parts,
                                                         unsigned long long* __restrict__ out) {
    const unsigned long long total = block_sum(threadIdx.x < n_parts ? parts[threadIdx.x] : 0ull);
    if (threadIdx.x == 0) *out = total;
}

// Launches the two passes; the total lands in ws[kSumParts].
lbm_status sum_records(const int32_t* rec, int64_t tiles, int word, unsigned long long* ws,
                       hipStream_t s) {
    const int parts = int(std::min<int64_t>(kSumParts, (tiles + kSumBlock - 1) / kSumBlock));
    k_sum_records<<<parts, kSumBlock, 0, s>>>(rec, tiles, word, ws);
    if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    k_sum_parts<<<1, kSumBlock, 0, s>>>(ws, parts, ws + kSumParts);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EHIP;
}

// One workgroup per tile: the tile is narrow if every live cell's 18 codes
// fit (a tile with escapes never does).  Codes of a wide tile are stored as 0.
__global__ __launch_bounds__(kCTile) void k_narrow(const int16_t* __restrict__ codes, int64_t n,
                                                   int64_t stride, int32_t* __restrict__ rec,
                                                   int8_t* __restrict__ codes8) {
    const int64_t tile = blockIdx.x;
    const int64_t m = tile * kCTile + threadIdx.x;
    const bool live = m < n;
    const int64_t mc = live ? m : 0;  // lanes past the list read cell 0 and are ignored
    int32_t cd[Q - 1];
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) cd[k] = codes[k * stride + mc];
    bool fits = true;
#pragma unroll
    for (int k = 0; k < Q - 1; ++k)
        fits = fits && (cd[k] == kCodeBounce || (cd[k] >= -kCode8Max && cd[k] <= kCode8Max));
    const bool narrow = __syncthreads_and(!live || fits) != 0;  // every thread takes part
    if (live) {
#pragma unroll
        for (int k = 0; k < Q - 1; ++k)
            codes8[k * stride + m] =
                narrow ? (cd[k] == kCodeBounce ? kCode8Bounce : int8_t(cd[k])) : int8_t(0);
    }
    if (threadIdx.x == 0) rec[tile * kRec + Q] = narrow ? 1 : 0;
}

template <int ST, bool PBB, bool NT>
__global__ __launch_bounds__(kCTile) void k_trt_c16(const typename Storage<ST>::T* __restrict__ src,
                                                    typename Storage<ST>::T* __restrict__ dst,
                                                    const int16_t* __restrict__ codes,
                                                    const int32_t* __restrict__ tile_rec,
                                                    const uint32_t* __restrict__ adj,
                                                    const double* __restrict__ ns, int64_t n,
                                                    int64_t stride, TrtConst c, int chunk_shift) {
    const int64_t tile = logical_block(chunk_shift);
    const int64_t m = tile * kCTile + threadIdx.x;
    if (m >= n) return;
    const int32_t* rec = tile_rec + tile * kRec;  // uniform over the workgroup
    if (rec[Q - 1] != 0)
        update_cell<ST, PBB, NT>(src, dst, adj, ns, m, stride, c);
    else
        update_cell_coded<ST, PBB, NT, int16_t>(src, dst, codes, rec, ns, m, stride, c);
}

// Three-way, uniform over the workgroup: narrow tile -> 8-bit codes, tile
// with escapes -> full list, otherwise 16-bit codes.
template <int ST, bool PBB, bool NT>
__global__ __launch_bounds__(kCTile) void k_trt_c8(const typename Storage<ST>::T* __restrict__ src,
                                                   typename Storage<ST>::T* __restrict__ dst,
                                                   const int8_t* __restrict__ codes8,
                                                   const int16_t* __restrict__ codes,
                                                   const int32_t* __restrict__ tile_rec,
                                                   const uint32_t* __restrict__ adj,
                                                   const double* __restrict__ ns, int64_t n,
                                                   int64_t stride, TrtConst c, int chunk_shift) {
    const int64_t tile = logical_block(chunk_shift);
    const int64_t m = tile * kCTile + threadIdx.x;
    if (m >= n) return;
    const int32_t* rec = tile_rec + tile * kRec;
    if (rec[Q] != 0)
        update_cell_coded<ST, PBB, NT, int8_t>(src, dst, codes8, rec, ns, m, stride, c);
    else if (rec[Q - 1] != 0)
        update_cell<ST, PBB, NT>(src, dst, adj, ns, m, stride, c);
    else
        update_cell_coded<ST, PBB, NT, int16_t>(src, dst, codes, rec, ns, m, stride, c);
}

// codes8 == nullptr: the 16-bit sweep (k_trt_c16); else the 8-bit one.
template <int ST, bool PBB, bool NT>
lbm_status launch_coded(const TrtConst& c, int cs, int64_t n, int64_t stride,
                        const int8_t* codes8, const int16_t* codes, const int32_t* toff,
                        const uint32_t* adj, const double* ns, void* fa, void* fb, int n_steps,
                        hipStream_t s) {
    using T = typename Storage<ST>::T;
    T* a = static_cast<T*>(fa);
    T* b = static_cast<T*>(fb);
    const dim3 g{unsigned(grid_blocks(n, kCTile, cs))}, blk{unsigned(kCTile)};
    for (int k = 0; k < n_steps; ++k) {
        const T* src = (k & 1) ? b : a;
        T* dst = (k & 1) ? a : b;
        if (codes8)
            k_trt_c8<ST, PBB, NT><<<g, blk, 0, s>>>(src, dst, codes8, codes, toff, adj, ns, n, stride, c, cs);
        else
            k_trt_c16<ST, PBB, NT><<<g, blk, 0, s>>>(src, dst, codes, toff, adj, ns, n, stride, c, cs);
        if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    }
    return LBM_OK;
}

template <int ST>
lbm_status dispatch_coded(const lbm_params& p, int64_t n, int64_t stride, const int8_t* codes8,
                          const int16_t* codes, const int32_t* toff, const uint32_t* adj,
                          const double* ns, void* fa, void* fb, int n_steps, hipStream_t s) {
    const TrtConst c = make_trt_const(p);
    const int cs = chunk_shift_for(p.flags, n, kCTile);
    const bool nt = p.flags & LBM_FLAG_NONTEMPORAL;
    if (ns)
        return nt ? launch_coded<ST, true, true>(c, cs, n, stride, codes8, codes, toff, adj, ns, fa, fb, n_steps, s)
                  : launch_coded<ST, true, false>(c, cs, n, stride, codes8, codes, toff, adj, ns, fa, fb, n_steps, s);
    return nt ? launch_coded<ST, false, true>(c, cs, n, stride, codes8, codes, toff, adj, ns, fa, fb, n_steps, s)
              : launch_coded<ST, false, false>(c, cs, n, stride, codes8, codes, toff, adj, ns, fa, fb, n_steps, s);
}

lbm_status step_coded(const lbm_params& p, int64_t n, int64_t stride, const int8_t* codes8,
                      const int16_t* codes, const int32_t* toff, const uint32_t* adj,
                      const double* ns, void* fa, void* fb, int n_steps, hipStream_t s) {
    switch (p.storage) {
    case LBM_F64: return dispatch_coded<LBM_F64>(p, n, stride, codes8, codes, toff, adj, ns, fa, fb, n_steps, s);
    case LBM_F64_SHIFTED: return dispatch_coded<LBM_F64_SHIFTED>(p, n, stride, codes8, codes, toff, adj, ns, fa, fb, n_steps, s);
    case LBM_F32: return dispatch_coded<LBM_F32>(p, n, stride, codes8, codes, toff, adj, ns, fa, fb, n_steps, s);
    case LBM_F32_SHIFTED: return dispatch_coded<LBM_F32_SHIFTED>(p, n, stride, codes8, codes, toff, adj, ns, fa, fb, n_steps, s);
    case LBM_F16_SHIFTED: return dispatch_coded<LBM_F16_SHIFTED>(p, n, stride, codes8, codes, toff, adj, ns, fa, fb, n_steps, s);
    case LBM_F16_SHIFTED_SCALED: return dispatch_coded<LBM_F16_SHIFTED_SCALED>(p, n, stride, codes8, codes, toff, adj, ns, fa, fb, n_steps, s);
    default: return LBM_EINVAL;
    }
}

}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_compress_adjacency(int64_t n, int64_t stride, const uint32_t* adj,
                                             int16_t* codes, int32_t* tile_records,
                                             int64_t* n_escapes, void* workspace,
                                             size_t* ws_bytes, void* stream) {
    if (!ws_bytes) return LBM_EINVAL;
    if (!workspace) {
        *ws_bytes = kSumWorkspace;
        return LBM_OK;
    }
    if (*ws_bytes < kSumWorkspace) return LBM_EWORKSPACE;
    if (lbm_status st = check_layout(n, stride); st != LBM_OK) return st;
    if (!adj || !codes || !tile_records || !n_escapes || n <= 0) return LBM_EINVAL;
    hipStream_t s = as_stream(stream);
    auto* ws = static_cast<unsigned long long*>(workspace);
    const int64_t tiles = (n + kCTile - 1) / kCTile;
    k_compress<<<dim3(unsigned(tiles)), kCTile, 0, s>>>(adj, n, stride, codes, tile_records);
    if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    if (lbm_status st = sum_records(tile_records, tiles, Q - 1, ws, s); st != LBM_OK) return st;
    unsigned long long e = 0;
    LBM_TRY_HIP(hipMemcpyAsync(&e, ws + kSumParts, sizeof(e), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    *n_escapes = int64_t(e);
    return LBM_OK;
}

extern "C" lbm_status lbm_step_c16(const lbm_params* p, int64_t n, int64_t stride,
                                   const int16_t* codes, const int32_t* tile_records,
                                   const uint32_t* adj, const double* ns, void* f_a, void* f_b,
                                   int32_t n_steps, void* stream) {
    if (!valid_params(p) || !codes || !tile_records || !adj || !f_a || !f_b || n_steps < 0)
        return LBM_EINVAL;
    if (f_a == f_b) return LBM_EINVAL;
    if (lbm_status st = check_layout(n, stride); st != LBM_OK) return st;
    if (n == 0 || n_steps == 0) return LBM_OK;
    return step_coded(*p, n, stride, nullptr, codes, tile_records, adj, ns, f_a, f_b, n_steps,
                      as_stream(stream));
}

extern "C" lbm_status lbm_narrow_codes(int64_t n, int64_t stride, const int16_t* codes,
                                       int32_t* tile_records, int8_t* codes8,
                                       int64_t* n_narrow_tiles, void* workspace,
                                       size_t* ws_bytes, void* stream) {
    if (!ws_bytes) return LBM_EINVAL;
    if (!workspace) {
        *ws_bytes = kSumWorkspace;
        return LBM_OK;
    }
    if (*ws_bytes < kSumWorkspace) return LBM_EWORKSPACE;
    if (lbm_status st = check_layout(n, stride); st != LBM_OK) return st;
    if (!codes || !tile_records || !codes8 || !n_narrow_tiles || n <= 0) return LBM_EINVAL;
    hipStream_t s = as_stream(stream);
    auto* ws = static_cast<unsigned long long*>(workspace);
    const int64_t tiles = (n + kCTile - 1) / kCTile;
    k_narrow<<<dim3(unsigned(tiles)), kCTile, 0, s>>>(codes, n, stride, tile_records, codes8);
    if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    if (lbm_status st = sum_records(tile_records, tiles, Q, ws, s); st != LBM_OK) return st;
    unsigned long long t = 0;
    LBM_TRY_HIP(hipMemcpyAsync(&t, ws + kSumParts, sizeof(t), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    *n_narrow_tiles = int64_t(t);
    return LBM_OK;
}

extern "C" lbm_status lbm_step_c8(const lbm_params* p, int64_t n, int64_t stride,
                                  const int8_t* codes8, const int16_t* codes,
                                  const int32_t* tile_records, const uint32_t* adj,
                                  const double* ns, void* f_a, void* f_b, int32_t n_steps,
                                  void* stream) {
    if (!valid_params(p) || !codes8 || !codes || !tile_records || !adj || !f_a || !f_b ||
        n_steps < 0)
        return LBM_EINVAL;
    if (f_a == f_b) return LBM_EINVAL;
    if (lbm_status st = check_layout(n, stride); st != LBM_OK) return st;
    if (n == 0 || n_steps == 0) return LBM_OK;
    return step_coded(*p, n, stride, codes8, codes, tile_records, adj, ns, f_a, f_b, n_steps,
                      as_stream(stream));
}
