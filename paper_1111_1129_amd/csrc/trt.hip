// trt.hip -- equilibrium initialisation and the D3Q19 TRT pull sweep
// (lbm_init, lbm_step).
//
// The sweep is bandwidth-bound (about 200 flop against 376 bytes per fluid
// cell update in FP64), so the kernel is organised around memory traffic:
//  * one thread per list cell, 256-thread workgroups (4 waves of 64);
//  * the 18 adjacency entries of a cell are read as 18 coalesced rows of
//    the [18][stride] adjacency list, then the 18 gathers are issued back to
//    back so their latencies overlap;
//  * the 19 results are written to the cell's own column of each
//    destination row -- fully coalesced, optionally nontemporal (the paper's
//    solver uses nontemporal stores for the destination grid);
//  * workgroups are remapped so that each XCD (own L2) sweeps a contiguous
//    eighth of the list: the neighbours a pull reads are nearby list entries,
//    so their cache lines are shared within one L2.
// No MFMA: there is no dense contraction here.
#include <algorithm>

#include "lbm_device.hpp"
#include "lbm_host.hpp"

namespace lbm {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// init
// ---------------------------------------------------------------------------
struct EqValues {
    double v[Q];
};

template <int ST>
__global__ __launch_bounds__(kBlock) void k_init(typename Storage<ST>::T* __restrict__ f, int64_t n,
                                                 int64_t stride, EqValues e) {
    using T = typename Storage<ST>::T;
    const int64_t m = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (m >= n) return;
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i * stride + m] = static_cast<T>(static_cast<typename Storage<ST>::A>(e.v[i]));
}

// ---------------------------------------------------------------------------
// one cell update: gather through adj, collide, store to own column
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
    for (int k = 0; k < Q - 1; ++k) a[k] = ap[k * stride];
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

template <int ST, bool PBB, bool NT, bool REMAP>
__global__ __launch_bounds__(kBlock) void k_trt(const typename Storage<ST>::T* __restrict__ src,
                                                typename Storage<ST>::T* __restrict__ dst,
                                                const uint32_t* __restrict__ adj,
                                                const double* __restrict__ ns, int64_t n,
                                                int64_t stride, TrtConst c) {
    const int64_t m = logical_block(REMAP) * kBlock + threadIdx.x;
    if (m >= n) return;
    update_cell<ST, PBB, NT>(src, dst, adj, ns, m, stride, c);
}

// ---------------------------------------------------------------------------
// persistent launch: all steps in one cooperative grid, a grid-wide barrier
// between steps.  Each XCD sweeps a contiguous share of the tiles.
// ---------------------------------------------------------------------------
struct Barrier {
    unsigned int* count;  // monotone arrival counter
    int* error;           // set when a wait exceeds the spin limit
};

constexpr long kSpinLimit = 1L << 24;  // ~ seconds of s_sleep; far above any step time

// Returns false (and raises the error flag) if the wait timed out or another
// workgroup already raised it; every workgroup then leaves the kernel.
__device__ bool grid_barrier(Barrier b, unsigned int& target) {
    __shared__ int ok;
    __syncthreads();
    target += gridDim.x;
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(b.count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int good = 1;
        long spins = 0;
        while (__hip_atomic_load(b.count, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > kSpinLimit ||
                __hip_atomic_load(b.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                good = 0;
                break;
            }
        }
        if (!good) __hip_atomic_store(b.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

template <int ST, bool PBB, bool NT>
__global__ __launch_bounds__(kBlock) void k_trt_persistent(typename Storage<ST>::T* fa,
                                                           typename Storage<ST>::T* fb,
                                                           const uint32_t* __restrict__ adj,
                                                           const double* __restrict__ ns, int64_t n,
                                                           int64_t stride, TrtConst c, int n_steps,
                                                           Barrier bar) {
    const int64_t tiles = (n + kBlock - 1) / kBlock;
    const int64_t per_xcd_tiles = (tiles + NXCD - 1) / NXCD;
    const int64_t xcd = blockIdx.x % NXCD;
    const int64_t lanes = gridDim.x / NXCD;  // workgroups per XCD
    unsigned int target = 0;
    for (int step = 0; step < n_steps; ++step) {
        const auto* src = (step & 1) ? fb : fa;
        auto* dst = (step & 1) ? fa : fb;
        for (int64_t t = blockIdx.x / NXCD; t < per_xcd_tiles; t += lanes) {
            const int64_t tile = xcd * per_xcd_tiles + t;
            const int64_t m = tile * kBlock + threadIdx.x;
            if (tile < tiles && m < n) update_cell<ST, PBB, NT>(src, dst, adj, ns, m, stride, c);
        }
        if (step + 1 < n_steps && !grid_barrier(bar, target)) return;
    }
}

__global__ void k_fill_u32(unsigned int* p, int count, unsigned int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// ---------------------------------------------------------------------------
// host dispatch
// ---------------------------------------------------------------------------
template <int ST>
lbm_status launch_init(const lbm_params& p, int64_t n, int64_t stride, void* f, double rho0,
                       const double* u0, hipStream_t s) {
    EqValues e;
    const double ux = u0 ? u0[0] : 0.0, uy = u0 ? u0[1] : 0.0, uz = u0 ? u0[2] : 0.0;
    const double uu = ux * ux + uy * uy + uz * uz;
    const double r = Storage<ST>::shifted ? rho0 - 1.0 : rho0;
    for (int i = 0; i < Q; ++i) {
        const double cu = vel_x(i) * ux + vel_y(i) * uy + vel_z(i) * uz;
        e.v[i] = weight(i) * (r + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
    if (n == 0) return LBM_OK;
    const int64_t grid = (n + kBlock - 1) / kBlock;
    k_init<ST><<<dim3(unsigned(grid)), dim3(kBlock), 0, s>>>(
        static_cast<typename Storage<ST>::T*>(f), n, stride, e);
    return after_launch();
}

template <int ST, bool PBB, bool NT>
lbm_status launch_steps(const TrtConst& c, bool remap, int64_t n, int64_t stride,
                        const uint32_t* adj, const double* ns, void* fa, void* fb, int n_steps,
                        hipStream_t s) {
    using T = typename Storage<ST>::T;
    T* a = static_cast<T*>(fa);
    T* b = static_cast<T*>(fb);
    const int64_t grid = grid_blocks(n, kBlock, remap);
    for (int k = 0; k < n_steps; ++k) {
        const T* src = (k & 1) ? b : a;
        T* dst = (k & 1) ? a : b;
        if (remap)
            k_trt<ST, PBB, NT, true><<<dim3(unsigned(grid)), dim3(kBlock), 0, s>>>(src, dst, adj, ns, n, stride, c);
        else
            k_trt<ST, PBB, NT, false><<<dim3(unsigned(grid)), dim3(kBlock), 0, s>>>(src, dst, adj, ns, n, stride, c);
        if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    }
    return LBM_OK;
}

constexpr size_t kPersistentWs = 256;  // counter + error flag, 256-byte aligned block

template <int ST, bool PBB, bool NT>
lbm_status launch_persistent(const TrtConst& c, int64_t n, int64_t stride, const uint32_t* adj,
                             const double* ns, void* fa, void* fb, int n_steps, void* ws,
                             hipStream_t s) {
    using T = typename Storage<ST>::T;
    auto kern = k_trt_persistent<ST, PBB, NT>;
    int dev = 0, cus = 0, per_cu = 0, coop = 0;
    LBM_TRY_HIP(hipGetDevice(&dev));
    LBM_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    LBM_TRY_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) return LBM_EHIP;
    LBM_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), kBlock, 0));
    int64_t grid = int64_t(per_cu) * cus;
    const int64_t tiles = (n + kBlock - 1) / kBlock;
    grid = std::min<int64_t>(grid, (tiles + NXCD - 1) / NXCD * NXCD);
    grid = grid / NXCD * NXCD;
    if (grid < NXCD) return LBM_EHIP;  // the device cannot hold one workgroup per XCD

    Barrier bar;
    bar.count = static_cast<unsigned int*>(ws);
    bar.error = reinterpret_cast<int*>(static_cast<unsigned int*>(ws) + 1);
    // clear counter and flag with a kernel (no memset node if the caller captures)
    k_fill_u32<<<1, 64, 0, s>>>(bar.count, 2, 0u);
    if (hipGetLastError() != hipSuccess) return LBM_EHIP;

    T* a = static_cast<T*>(fa);
    T* b = static_cast<T*>(fb);
    int steps = n_steps;
    TrtConst cc = c;
    void* args[] = {&a, &b, const_cast<uint32_t**>(&adj), const_cast<double**>(&ns),
                    &n, &stride, &cc, &steps, &bar};
    LBM_TRY_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(unsigned(grid)),
                                           dim3(kBlock), args, 0, s));
    int err = 0;
    LBM_TRY_HIP(hipMemcpyAsync(&err, bar.error, sizeof(int), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    return err ? LBM_EBARRIER : LBM_OK;
}

template <int ST>
lbm_status dispatch_step(const lbm_params& p, int64_t n, int64_t stride, const uint32_t* adj,
                         const double* ns, void* fa, void* fb, int n_steps, int persistent,
                         void* ws, hipStream_t s) {
    const TrtConst c = make_trt_const(p);
    const bool nt = (p.flags & LBM_FLAG_NONTEMPORAL) != 0;
    const bool remap = (p.flags & LBM_FLAG_NO_XCD_REMAP) == 0;
    if (persistent) {
        if (ns) return nt ? launch_persistent<ST, true, true>(c, n, stride, adj, ns, fa, fb, n_steps, ws, s)
                          : launch_persistent<ST, true, false>(c, n, stride, adj, ns, fa, fb, n_steps, ws, s);
        return nt ? launch_persistent<ST, false, true>(c, n, stride, adj, ns, fa, fb, n_steps, ws, s)
                  : launch_persistent<ST, false, false>(c, n, stride, adj, ns, fa, fb, n_steps, ws, s);
    }
    if (ns) return nt ? launch_steps<ST, true, true>(c, remap, n, stride, adj, ns, fa, fb, n_steps, s)
                      : launch_steps<ST, true, false>(c, remap, n, stride, adj, ns, fa, fb, n_steps, s);
    return nt ? launch_steps<ST, false, true>(c, remap, n, stride, adj, ns, fa, fb, n_steps, s)
              : launch_steps<ST, false, false>(c, remap, n, stride, adj, ns, fa, fb, n_steps, s);
}

}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_init(const lbm_params* p, int64_t n, int64_t stride, void* f,
                               double rho0, const double* u0, void* stream) {
    if (!p || !f || !valid_storage(p->storage) || !std::isfinite(rho0)) return LBM_EINVAL;
    if (lbm_status st = check_layout(n, stride); st != LBM_OK) return st;
    hipStream_t s = as_stream(stream);
    switch (p->storage) {
    case LBM_F64: return launch_init<LBM_F64>(*p, n, stride, f, rho0, u0, s);
    case LBM_F64_SHIFTED: return launch_init<LBM_F64_SHIFTED>(*p, n, stride, f, rho0, u0, s);
    case LBM_F32: return launch_init<LBM_F32>(*p, n, stride, f, rho0, u0, s);
    case LBM_F32_SHIFTED: return launch_init<LBM_F32_SHIFTED>(*p, n, stride, f, rho0, u0, s);
    case LBM_F16_SHIFTED: return launch_init<LBM_F16_SHIFTED>(*p, n, stride, f, rho0, u0, s);
    default: return LBM_EINVAL;
    }
}

extern "C" lbm_status lbm_step(const lbm_params* p, int32_t n_params, const lbm_segment* seg,
                               int32_t n_seg, int64_t n, int64_t stride, const uint32_t* adj,
                               const double* ns, void* f_a, void* f_b, int32_t n_steps,
                               int32_t persistent, void* workspace, size_t* ws_bytes,
                               void* stream) {
    if (persistent && !workspace) {
        // size query
        if (!ws_bytes) return LBM_EINVAL;
        *ws_bytes = kPersistentWs;
        return LBM_OK;
    }
    if (!valid_params(p) || n_params != 1 || !adj || !f_a || !f_b || n_steps < 0) return LBM_EINVAL;
    if (f_a == f_b) return LBM_EINVAL;
    if (lbm_status st = check_layout(n, stride); st != LBM_OK) return st;
    if (!valid_segments(seg, n_seg, n)) return LBM_EINVAL;
    if (persistent && (!ws_bytes || *ws_bytes < kPersistentWs)) return LBM_EWORKSPACE;
    if (n == 0 || n_steps == 0) return LBM_OK;
    hipStream_t s = as_stream(stream);
    switch (p->storage) {
    case LBM_F64: return dispatch_step<LBM_F64>(*p, n, stride, adj, ns, f_a, f_b, n_steps, persistent, workspace, s);
    case LBM_F64_SHIFTED: return dispatch_step<LBM_F64_SHIFTED>(*p, n, stride, adj, ns, f_a, f_b, n_steps, persistent, workspace, s);
    case LBM_F32: return dispatch_step<LBM_F32>(*p, n, stride, adj, ns, f_a, f_b, n_steps, persistent, workspace, s);
    case LBM_F32_SHIFTED: return dispatch_step<LBM_F32_SHIFTED>(*p, n, stride, adj, ns, f_a, f_b, n_steps, persistent, workspace, s);
    case LBM_F16_SHIFTED: return dispatch_step<LBM_F16_SHIFTED>(*p, n, stride, adj, ns, f_a, f_b, n_steps, persistent, workspace, s);
    default: return LBM_EINVAL;
    }
}
