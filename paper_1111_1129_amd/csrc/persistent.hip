// persistent.hip -- all sweeps of a batch in one cooperative launch
// (lbm_step with persistent = 1).
//
// The grid is sized to what the device holds at once (cooperative launch
// guarantees co-residency), each workgroup walks a share of the list tiles,
// and a grid-wide barrier separates the steps.  Tiles are split into eight
// contiguous ranges, one per XCD (workgroup w runs on XCD w % 8), so each
// XCD's L2 serves the neighbour gathers of its own range.
//
// Barrier: every workgroup publishes its stores with one agent-scope release
// (an atomic add on a monotone arrival counter), then waits with relaxed
// loads and takes one acquire fence when the count is reached.  Acquire
// loads inside the spin would invalidate the L2 on every poll.  The wait is
// bounded: past the spin limit the workgroup raises an error flag and every
// workgroup leaves the kernel, so the launch always drains; the host reports
// LBM_EBARRIER.
#include <algorithm>

#include "lbm_device.hpp"
#include "lbm_host.hpp"

namespace lbm {

constexpr int kPBlock = 256;
constexpr long kSpinLimit = 1L << 24;  // polls with s_sleep; seconds, far above any step

struct Barrier {
    unsigned int* count;  // monotone arrival counter
    int* error;           // raised when a wait exceeds the spin limit
};

__device__ bool grid_barrier(Barrier b, unsigned int& target) {
    __shared__ int ok;
    __syncthreads();
    target += gridDim.x;
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(b.count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int good = 1;
        long spins = 0;
        while (__hip_atomic_load(b.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > kSpinLimit ||
                __hip_atomic_load(b.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                good = 0;
                break;
            }
        }
        if (!good) __hip_atomic_store(b.error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

template <int ST, bool PBB, bool NT>
__global__ __launch_bounds__(kPBlock) void k_trt_persistent(typename Storage<ST>::T* fa,
                                                            typename Storage<ST>::T* fb,
                                                            const uint32_t* __restrict__ adj,
                                                            const double* __restrict__ ns, int64_t n,
                                                            int64_t stride, TrtConst c, int n_steps,
                                                            Barrier bar) {
    const int64_t tiles = (n + kPBlock - 1) / kPBlock;
    const int64_t per_xcd_tiles = (tiles + NXCD - 1) / NXCD;
    const int64_t xcd = blockIdx.x % NXCD;
    const int64_t lanes = gridDim.x / NXCD;  // workgroups per XCD
    unsigned int target = 0;
    for (int step = 0; step < n_steps; ++step) {
        const auto* src = (step & 1) ? fb : fa;
        auto* dst = (step & 1) ? fa : fb;
        for (int64_t t = blockIdx.x / NXCD; t < per_xcd_tiles; t += lanes) {
            const int64_t tile = xcd * per_xcd_tiles + t;
            const int64_t m = tile * kPBlock + threadIdx.x;
            if (tile < tiles && m < n) update_cell<ST, PBB, NT>(src, dst, adj, ns, m, stride, c);
        }
        if (step + 1 < n_steps && !grid_barrier(bar, target)) return;
    }
}

__global__ void k_fill_u32(unsigned int* p, int count, unsigned int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

template <int ST, bool PBB, bool NT>
lbm_status launch_persistent_t(const TrtConst& c, int64_t n, int64_t stride, const uint32_t* adj,
                               const double* ns, void* fa, void* fb, int n_steps, void* ws,
                               hipStream_t s) {
    using T = typename Storage<ST>::T;
    auto kern = k_trt_persistent<ST, PBB, NT>;
    int dev = 0, cus = 0, per_cu = 0, coop = 0;
    LBM_TRY_HIP(hipGetDevice(&dev));
    LBM_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    LBM_TRY_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) return LBM_EHIP;
    LBM_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                             kPBlock, 0));
    // Co-residency is what the grid barrier needs.  Measured on gfx950: for
    // the FP32 instance (72 VGPRs) the query reports 7 workgroups per CU but
    // only 6 are resident at once (the arrival counter stalls after the first
    // barrier at 7, completes at 6).  So the count is also bounded by the
    // VGPR file at a 16-register granule, and by 4 workgroups per CU, which
    // keeps 4 waves per SIMD for this bandwidth-bound loop.
    hipFuncAttributes attr;
    LBM_TRY_HIP(hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(kern)));
    const int waves_per_simd = kPBlock / 64 / 4;  // one wave per SIMD per workgroup
    if (attr.numRegs > 0) {
        const int vgpr = (attr.numRegs + 15) / 16 * 16;
        per_cu = std::min(per_cu, 512 / vgpr / waves_per_simd);
    }
    per_cu = std::min(per_cu, 4);
    int64_t grid = int64_t(per_cu) * cus;
    const int64_t tiles = (n + kPBlock - 1) / kPBlock;
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
                                           dim3(kPBlock), args, 0, s));
    int err = 0;
    LBM_TRY_HIP(hipMemcpyAsync(&err, bar.error, sizeof(int), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    return err ? LBM_EBARRIER : LBM_OK;
}

template <int ST>
lbm_status launch_persistent_s(const TrtConst& c, bool nt, int64_t n, int64_t stride,
                               const uint32_t* adj, const double* ns, void* fa, void* fb,
                               int n_steps, void* ws, hipStream_t s) {
    if (ns) return nt ? launch_persistent_t<ST, true, true>(c, n, stride, adj, ns, fa, fb, n_steps, ws, s)
                      : launch_persistent_t<ST, true, false>(c, n, stride, adj, ns, fa, fb, n_steps, ws, s);
    return nt ? launch_persistent_t<ST, false, true>(c, n, stride, adj, ns, fa, fb, n_steps, ws, s)
              : launch_persistent_t<ST, false, false>(c, n, stride, adj, ns, fa, fb, n_steps, ws, s);
}

lbm_status launch_persistent(int storage, const TrtConst& c, bool nt, int64_t n, int64_t stride,
                             const uint32_t* adj, const double* ns, void* fa, void* fb,
                             int n_steps, void* ws, hipStream_t s) {
    switch (storage) {
    case LBM_F64: return launch_persistent_s<LBM_F64>(c, nt, n, stride, adj, ns, fa, fb, n_steps, ws, s);
    case LBM_F64_SHIFTED: return launch_persistent_s<LBM_F64_SHIFTED>(c, nt, n, stride, adj, ns, fa, fb, n_steps, ws, s);
    case LBM_F32: return launch_persistent_s<LBM_F32>(c, nt, n, stride, adj, ns, fa, fb, n_steps, ws, s);
    case LBM_F32_SHIFTED: return launch_persistent_s<LBM_F32_SHIFTED>(c, nt, n, stride, adj, ns, fa, fb, n_steps, ws, s);
    case LBM_F16_SHIFTED: return launch_persistent_s<LBM_F16_SHIFTED>(c, nt, n, stride, adj, ns, fa, fb, n_steps, ws, s);
    default: return LBM_EINVAL;
    }
}

}  // namespace lbm
