// moments.hip -- macroscopic fields and FP64 totals (lbm_moments).
//
// Per cell the gathered populations give rho and u = j + G/2 (always in
// FP64, whatever the storage).  Totals per segment are reduced in two fixed
// passes (per-workgroup partials, then one workgroup over the partials) with
// double-double (TwoSum) accumulation, so they are reproducible bit for bit
// and accurate to about 1e-30 relative before the final rounding.
#include <algorithm>
#include <mutex>

#include "lbm_device.hpp"
#include "lbm_host.hpp"

namespace lbm {

constexpr int kMomBlock = 256;
constexpr int kRedThreads = 256;

struct DD {
    double hi, lo;
};

// Knuth's TwoSum, then renormalise: (a.hi + a.lo) + (b.hi + b.lo) in DD.
__device__ __forceinline__ DD dd_add(DD a, DD b) {
    const double s = a.hi + b.hi;
    const double bp = s - a.hi;
    double e = (a.hi - (s - bp)) + (b.hi - bp);
    e += a.lo + b.lo;
    const double hi = s + e;
    return DD{hi, e - (hi - s)};
}

// Fixed-shape tree reduction of 4 DD values over a workgroup.
__device__ void block_reduce4(DD v[4], DD (*sh)[4]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) sh[t][q] = v[q];
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (t < off) {
#pragma unroll
            for (int q = 0; q < 4; ++q) sh[t][q] = dd_add(sh[t][q], sh[t + off][q]);
        }
        __syncthreads();
    }
}

template <int ST>
__global__ __launch_bounds__(kMomBlock) void k_moments(const typename Storage<ST>::T* __restrict__ f,
                                                       const uint32_t* __restrict__ adj, int64_t n0,
                                                       int64_t cnt, int64_t stride, double gx,
                                                       double gy, double gz, double* __restrict__ rho,
                                                       double* __restrict__ u, int64_t ld,
                                                       double* __restrict__ partial) {
    using T = typename Storage<ST>::T;
    __shared__ DD sh[kMomBlock][4];
    const int64_t local = int64_t(blockIdx.x) * kMomBlock + threadIdx.x;
    DD v[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    if (local < cnt) {
        const int64_t m = n0 + local;
        // the 18 adjacency rows first, then the 18 gathers: both batches in
        // flight at once
        uint32_t a[Q - 1];
#pragma unroll
        for (int k = 0; k < Q - 1; ++k) a[k] = ld_stream(adj + k * stride + m);
        double g[Q];
        g[0] = static_cast<double>(f[m]);
#pragma unroll
        for (int k = 0; k < Q - 1; ++k) g[k + 1] = static_cast<double>(f[a[k]]);
        const CellMoments<double> cm = cell_moments(g);
        const double r = Storage<ST>::shifted ? 1.0 + cm.rho : cm.rho;
        const double ux = cm.jx + 0.5 * gx, uy = cm.jy + 0.5 * gy, uz = cm.jz + 0.5 * gz;
        if (rho) rho[m] = r;
        if (u) {
            u[m] = ux;
            u[ld + m] = uy;
            u[2 * ld + m] = uz;
        }
        v[0].hi = r;
        v[1].hi = ux;
        v[2].hi = uy;
        v[3].hi = uz;
    }
    if (!partial) return;
    block_reduce4(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            partial[(int64_t(blockIdx.x) * 4 + q) * 2] = sh[0][q].hi;
            partial[(int64_t(blockIdx.x) * 4 + q) * 2 + 1] = sh[0][q].lo;
        }
    }
}

// k_moments with `per_block` cells per workgroup (a multiple of kMomBlock):
// each thread accumulates its cells in double-double before the workgroup
// reduction, so the number of partial sums stays bounded however large the
// segment is (lbm_moments_noalloc).  Fields are those of k_moments.
template <int ST>
__global__ __launch_bounds__(kMomBlock) void k_moments_strided(
    const typename Storage<ST>::T* __restrict__ f, const uint32_t* __restrict__ adj, int64_t n0,
    int64_t cnt, int64_t per_block, int64_t stride, double gx, double gy, double gz,
    double* __restrict__ rho, double* __restrict__ u, int64_t ld, double* __restrict__ partial) {
    __shared__ DD sh[kMomBlock][4];
    DD v[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    const int64_t begin = int64_t(blockIdx.x) * per_block;
    const int64_t end = std::min(cnt, begin + per_block);
    for (int64_t local = begin + threadIdx.x; local < end; local += kMomBlock) {
        const int64_t m = n0 + local;
        uint32_t a[Q - 1];
#pragma unroll
        for (int k = 0; k < Q - 1; ++k) a[k] = ld_stream(adj + k * stride + m);
        double g[Q];
        g[0] = static_cast<double>(f[m]);
#pragma unroll
        for (int k = 0; k < Q - 1; ++k) g[k + 1] = static_cast<double>(f[a[k]]);
        const CellMoments<double> cm = cell_moments(g);
        const double r = Storage<ST>::shifted ? 1.0 + cm.rho : cm.rho;
        const double ux = cm.jx + 0.5 * gx, uy = cm.jy + 0.5 * gy, uz = cm.jz + 0.5 * gz;
        if (rho) rho[m] = r;
        if (u) {
            u[m] = ux;
            u[ld + m] = uy;
            u[2 * ld + m] = uz;
        }
        v[0] = dd_add(v[0], DD{r, 0.0});
        v[1] = dd_add(v[1], DD{ux, 0.0});
        v[2] = dd_add(v[2], DD{uy, 0.0});
        v[3] = dd_add(v[3], DD{uz, 0.0});
    }
    if (!partial) return;
    block_reduce4(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            partial[(int64_t(blockIdx.x) * 4 + q) * 2] = sh[0][q].hi;
            partial[(int64_t(blockIdx.x) * 4 + q) * 2 + 1] = sh[0][q].lo;
        }
    }
}

// totals (4 values) and/or the objective (the x total divided by `count`)
__global__ __launch_bounds__(kRedThreads) void k_reduce_partials(const double* __restrict__ partial,
                                                                 int64_t nblocks,
                                                                 double* __restrict__ totals,
                                                                 double* __restrict__ objective,
                                                                 double count) {
    __shared__ DD sh[kRedThreads][4];
    DD v[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    // thread t sums blocks t, t + T, t + 2T, ... in order
    for (int64_t b = threadIdx.x; b < nblocks; b += kRedThreads) {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = dd_add(v[q], DD{partial[(b * 4 + q) * 2], partial[(b * 4 + q) * 2 + 1]});
    }
    block_reduce4(v, sh);
    if (threadIdx.x == 0) {
        if (totals) {
#pragma unroll
            for (int q = 0; q < 4; ++q) totals[q] = sh[0][q].hi + sh[0][q].lo;
        }
        if (objective) objective[0] = (sh[0][1].hi + sh[0][1].lo) / count;
    }
}

template <int ST>
lbm_status launch_moments(const lbm_params* p, int64_t n, int64_t stride, const uint32_t* adj,
                          const void* f, double* rho, double* u, const lbm_segment* seg,
                          int32_t n_seg, double* totals, double* objective, double* partial,
                          hipStream_t s) {
    lbm_segment whole{0, n, 0, 0};
    if (!seg || n_seg == 0) {
        seg = &whole;
        n_seg = 1;
    }
    const bool reduce = totals || objective;
    for (int32_t k = 0; k < n_seg; ++k) {
        const int64_t cnt = seg[k].n;
        const lbm_params& pk = p[seg[k].param_index];
        const int64_t blocks = std::max<int64_t>(1, (cnt + kMomBlock - 1) / kMomBlock);
        k_moments<ST><<<dim3(unsigned(blocks)), dim3(kMomBlock), 0, s>>>(
            static_cast<const typename Storage<ST>::T*>(f), adj, seg[k].base, cnt, stride,
            pk.force[0], pk.force[1], pk.force[2], rho, u, n, reduce ? partial : nullptr);
        if (hipGetLastError() != hipSuccess) return LBM_EHIP;
        if (reduce) {
            k_reduce_partials<<<1, kRedThreads, 0, s>>>(partial, blocks, totals ? totals + 4 * k : nullptr,
                                                        objective ? objective + k : nullptr,
                                                        double(cnt));
            if (hipGetLastError() != hipSuccess) return LBM_EHIP;
        }
    }
    return LBM_OK;
}

// Reads `count` totals back in fixed-size pieces (no allocation) after the
// stream has produced them: LBM_ENONFINITE if one is NaN or infinite.
lbm_status check_totals_finite(const double* totals, int64_t count, hipStream_t s) {
    double buf[64];
    bool finite = true;
    for (int64_t i0 = 0; i0 < count; i0 += 64) {
        const int64_t c = std::min<int64_t>(64, count - i0);
        LBM_TRY_HIP(hipMemcpyAsync(buf, totals + i0, size_t(c) * sizeof(double), hipMemcpyDeviceToHost, s));
        LBM_TRY_HIP(hipStreamSynchronize(s));
        for (int64_t i = 0; i < c; ++i) finite = finite && std::isfinite(buf[i]);
    }
    return finite ? LBM_OK : LBM_ENONFINITE;
}

// Shared by lbm_moments and lbm_objective.
lbm_status moments_call(const lbm_params* p, int32_t n_params, int64_t n, int64_t stride,
                        const uint32_t* adj, const void* f, double* rho, double* u,
                        const lbm_segment* seg, int32_t n_seg, double* totals, double* objective,
                        void* workspace, size_t* ws_bytes, void* stream) {
    if (!p || n_params < 1 || n_params > kMaxParamSets) return LBM_EINVAL;
    if (lbm_status st = check_layout(n, stride); st != LBM_OK) return st;
    if (!valid_segments(seg, n_seg, n, n_params)) return LBM_EINVAL;
    int64_t largest = (seg && n_seg > 0) ? 0 : n;
    for (int32_t k = 0; seg && k < n_seg; ++k) largest = std::max(largest, seg[k].n);
    const bool reduce = totals || objective;
    const size_t need = reduce ? align_up(size_t(std::max<int64_t>(1, (largest + kMomBlock - 1) / kMomBlock)) * 8 * sizeof(double), 256) : 0;
    if (reduce && !workspace) {
        if (!ws_bytes) return LBM_EINVAL;
        *ws_bytes = need;
        return LBM_OK;
    }
    if (reduce && (!ws_bytes || *ws_bytes < need)) return LBM_EWORKSPACE;
    if (!adj || !f) return LBM_EINVAL;
    for (int32_t k = 0; k < n_params; ++k) {
        if (!valid_storage(p[k].storage) || p[k].storage != p[0].storage) return LBM_EINVAL;
        for (int d = 0; d < 3; ++d)
            if (!std::isfinite(p[k].force[d])) return LBM_EINVAL;
    }
    hipStream_t s = as_stream(stream);
    double* partial = static_cast<double*>(workspace);
    lbm_status st;
    switch (p[0].storage) {
    case LBM_F64: st = launch_moments<LBM_F64>(p, n, stride, adj, f, rho, u, seg, n_seg, totals, objective, partial, s); break;
    case LBM_F64_SHIFTED: st = launch_moments<LBM_F64_SHIFTED>(p, n, stride, adj, f, rho, u, seg, n_seg, totals, objective, partial, s); break;
    case LBM_F32: st = launch_moments<LBM_F32>(p, n, stride, adj, f, rho, u, seg, n_seg, totals, objective, partial, s); break;
    case LBM_F32_SHIFTED: st = launch_moments<LBM_F32_SHIFTED>(p, n, stride, adj, f, rho, u, seg, n_seg, totals, objective, partial, s); break;
    case LBM_F16_SHIFTED: st = launch_moments<LBM_F16_SHIFTED>(p, n, stride, adj, f, rho, u, seg, n_seg, totals, objective, partial, s); break;
    case LBM_F16_SHIFTED_SCALED: st = launch_moments<LBM_F16_SHIFTED_SCALED>(p, n, stride, adj, f, rho, u, seg, n_seg, totals, objective, partial, s); break;
    default: return LBM_EINVAL;
    }
    if (st != LBM_OK || !totals || !(p[0].flags & LBM_FLAG_CHECK_FINITE)) return st;
    return check_totals_finite(totals, 4 * int64_t(std::max<int32_t>(n_seg, 1)), s);
}

// ---------------------------------------------------------------------------
// lbm_moments_noalloc: the partial sums of the totals live in `scratch`, a
// fixed device array of the library (one copy per GPU, held until the
// process ends), instead of a caller workspace.  Host code never passes the
// array's name to a kernel: it takes the device address from
// hipGetSymbolAddress once per device, with that device current, and uses it.
// ---------------------------------------------------------------------------
constexpr int64_t kNoAllocParts = 4096;  // partial sums per segment, 4 double-doubles each
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kNoAllocParts * 8];  // 256 KiB

std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's scratch (looked up on the first call on it).
lbm_status device_scratch(double** out) {
    int dev = -1;
    LBM_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return LBM_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LBM_EHIP;
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

template <int ST>
lbm_status launch_moments_noalloc(const lbm_params* p, int64_t n, int64_t stride,
                                  const uint32_t* adj, const void* f, double* rho, double* u,
                                  const lbm_segment* seg, int32_t n_seg, double* totals,
                                  double* partial, hipStream_t s) {
    lbm_segment whole{0, n, 0, 0};
    if (!seg || n_seg == 0) {
        seg = &whole;
        n_seg = 1;
    }
    for (int32_t k = 0; k < n_seg; ++k) {
        const int64_t cnt = seg[k].n;
        const lbm_params& pk = p[seg[k].param_index];
        // cells per workgroup: whole tiles, as few as keep the partials within scratch
        const int64_t tiles = std::max<int64_t>(1, (cnt + kMomBlock - 1) / kMomBlock);
        const int64_t per_block = (tiles + kNoAllocParts - 1) / kNoAllocParts * kMomBlock;
        const int64_t blocks = std::max<int64_t>(1, (cnt + per_block - 1) / per_block);
        if (blocks > kNoAllocParts) return LBM_ECAPACITY;  // cannot happen: per_block grows with cnt
        k_moments_strided<ST><<<dim3(unsigned(blocks)), dim3(kMomBlock), 0, s>>>(
            static_cast<const typename Storage<ST>::T*>(f), adj, seg[k].base, cnt, per_block, stride,
            pk.force[0], pk.force[1], pk.force[2], rho, u, n, totals ? partial : nullptr);
        if (hipGetLastError() != hipSuccess) return LBM_EHIP;
        if (totals) {
            // the segments run one after another on the stream, so they reuse the partials
            k_reduce_partials<<<1, kRedThreads, 0, s>>>(partial, blocks, totals + 4 * k, nullptr,
                                                        double(cnt));
            if (hipGetLastError() != hipSuccess) return LBM_EHIP;
        }
    }
    return LBM_OK;
}

}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_moments(const lbm_params* p, int32_t n_params, int64_t n,
                                  int64_t stride, const uint32_t* adj, const void* f, double* rho,
                                  double* u, const lbm_segment* seg, int32_t n_seg, double* totals,
                                  void* workspace, size_t* ws_bytes, void* stream) {
    return moments_call(p, n_params, n, stride, adj, f, rho, u, seg, n_seg, totals, nullptr,
                        workspace, ws_bytes, stream);
}

extern "C" lbm_status lbm_objective(const lbm_params* p, int32_t n_params, int64_t n,
                                    int64_t stride, const uint32_t* adj, const void* f,
                                    const lbm_segment* seg, int32_t n_seg, double* J,
                                    void* workspace, size_t* ws_bytes, void* stream) {
    if (!J) return LBM_EINVAL;
    return moments_call(p, n_params, n, stride, adj, f, nullptr, nullptr, seg, n_seg, nullptr, J,
                        workspace, ws_bytes, stream);
}

extern "C" lbm_status lbm_moments_noalloc(const lbm_params* p, int32_t n_params, int64_t n,
                                          int64_t stride, const uint32_t* adj, const void* f,
                                          double* rho, double* u, const lbm_segment* seg,
                                          int32_t n_seg, double* totals, void* stream) {
    if (!p || n_params < 1 || n_params > kMaxParamSets || !adj || !f) return LBM_EINVAL;
    if (lbm_status st = check_layout(n, stride); st != LBM_OK) return st;
    if (!valid_segments(seg, n_seg, n, n_params)) return LBM_EINVAL;
    for (int32_t k = 0; k < n_params; ++k) {
        if (!valid_storage(p[k].storage) || p[k].storage != p[0].storage) return LBM_EINVAL;
        for (int d = 0; d < 3; ++d)
            if (!std::isfinite(p[k].force[d])) return LBM_EINVAL;
    }
    double* partial = nullptr;
    if (totals) {
        if (lbm_status st = device_scratch(&partial); st != LBM_OK) return st;
    }
    hipStream_t s = as_stream(stream);
    lbm_status st;
    switch (p[0].storage) {
    case LBM_F64: st = launch_moments_noalloc<LBM_F64>(p, n, stride, adj, f, rho, u, seg, n_seg, totals, partial, s); break;
    case LBM_F64_SHIFTED: st = launch_moments_noalloc<LBM_F64_SHIFTED>(p, n, stride, adj, f, rho, u, seg, n_seg, totals, partial, s); break;
    case LBM_F32: st = launch_moments_noalloc<LBM_F32>(p, n, stride, adj, f, rho, u, seg, n_seg, totals, partial, s); break;
    case LBM_F32_SHIFTED: st = launch_moments_noalloc<LBM_F32_SHIFTED>(p, n, stride, adj, f, rho, u, seg, n_seg, totals, partial, s); break;
    case LBM_F16_SHIFTED: st = launch_moments_noalloc<LBM_F16_SHIFTED>(p, n, stride, adj, f, rho, u, seg, n_seg, totals, partial, s); break;
    case LBM_F16_SHIFTED_SCALED: st = launch_moments_noalloc<LBM_F16_SHIFTED_SCALED>(p, n, stride, adj, f, rho, u, seg, n_seg, totals, partial, s); break;
    default: return LBM_EINVAL;
    }
    if (st != LBM_OK || !totals || !(p[0].flags & LBM_FLAG_CHECK_FINITE)) return st;
    return check_totals_finite(totals, 4 * int64_t(std::max<int32_t>(n_seg, 1)), s);
}
