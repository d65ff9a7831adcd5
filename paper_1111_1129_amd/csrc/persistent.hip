// persistent.hip -- all sweeps of a batch in one cooperative launch
// (lbm_step with persistent = 1).
//
// Grid: one 256-thread workgroup per CU (co-resident by construction; the
// cooperative launch checks it), each walking list tiles in the same
// XCD-chunked order as the one-launch-per-step sweep, with a grid-wide
// barrier between steps.  Measured on gfx950 (256^3 tube, FP32): the cost of
// the barrier grows with the number of workgroups taking part, so one
// workgroup per CU (23.0 GFLUPS) beats 2, 4 and 6 per CU (20.4, 18.9,
// 17.0 GFLUPS) and 512/1024-thread workgroups; one launch per step runs at
// 24.6 GFLUPS.
//
// Barrier (two levels, every wait bounded):
//  * census at kernel start: each workgroup reads its XCD from the XCC_ID
//    hardware register and counts itself into xcd_size[xcd];
//  * per step, every thread waits for its own stores to be acknowledged by
//    the XCD's L2 (s_waitcnt 0), the workgroup arrives on xcd_count[xcd];
//    the last arrival of an XCD writes that L2 back (one agent-scope release
//    per XCD instead of one per workgroup) and increments the global count;
//    every workgroup polls the global count with relaxed loads and takes one
//    acquire fence (L1/L2 invalidate) when all XCDs have arrived.
// Past the spin limit a workgroup raises the error flag and every workgroup
// leaves the kernel, so the launch always drains; the host then reports
// LBM_EBARRIER.
#include <algorithm>

#include "lbm_device.hpp"
#include "lbm_host.hpp"

namespace lbm {

constexpr int kPBlock = 256;
constexpr long kSpinLimit = 1L << 27;  // polls of ~256 clocks: ~14 s, far above any step

// workspace layout (uint32 words): [0] global count, [1] error flag,
// [8..16) per-XCD arrivals, [16..24) per-XCD workgroup counts
struct Barrier {
    unsigned int* count;
    int* error;
    unsigned int* xcd_count;
    unsigned int* xcd_size;
};

__device__ __forceinline__ int xcc_id() {
    // hardware register XCC_ID, bits [3:0]: the XCD this wave runs on
    return int(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (NXCD - 1));
}

__device__ bool wait_at_least(unsigned int* cnt, unsigned int target, int* err) {
    long spins = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(4);  // 4 x 64 clocks between polls
        if (++spins > kSpinLimit ||
            __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    return true;
}

template <int ST, bool PBB, bool NT>
__global__ __launch_bounds__(kPBlock) void k_trt_persistent(typename Storage<ST>::T* fa,
                                                            typename Storage<ST>::T* fb,
                                                            const uint32_t* __restrict__ adj,
                                                            const double* __restrict__ ns, int64_t n,
                                                            int64_t stride, TrtConst c, int n_steps,
                                                            int chunk_shift, Barrier bar) {
    __shared__ int ok;
    __shared__ unsigned int populated;
    const int xcc = xcc_id();
    // census
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(&bar.xcd_size[xcc], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(bar.count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        ok = wait_at_least(bar.count, gridDim.x, bar.error);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        unsigned int p = 0;
        for (int x = 0; x < NXCD; ++x)
            p += __hip_atomic_load(&bar.xcd_size[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 1u : 0u;
        populated = p;
    }
    __syncthreads();
    if (!ok) return;
    const unsigned int mine =
        __hip_atomic_load(&bar.xcd_size[xcc], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

    const int64_t tiles = (n + kPBlock - 1) / kPBlock;
    const int64_t q = int64_t(NXCD) << chunk_shift;
    const int64_t vtiles = (tiles + q - 1) / q * q;  // virtual tiles, relabelled like workgroups
    unsigned int gen = 0;
    for (int step = 0; step < n_steps; ++step) {
        const auto* src = (step & 1) ? fb : fa;
        auto* dst = (step & 1) ? fa : fb;
        for (int64_t v = blockIdx.x; v < vtiles; v += gridDim.x) {
            const int64_t tile = ((v >> (3 + chunk_shift)) << (3 + chunk_shift)) +
                                 ((v & (NXCD - 1)) << chunk_shift) +
                                 ((v >> 3) & ((int64_t(1) << chunk_shift) - 1));
            const int64_t m = tile * kPBlock + threadIdx.x;
            if (tile < tiles && m < n) update_cell<ST, PBB, NT>(src, dst, adj, ns, m, stride, c);
        }
        if (step + 1 == n_steps) break;
        __builtin_amdgcn_s_waitcnt(0);  // this thread's stores acknowledged by the L2
        __syncthreads();
        ++gen;
        if (threadIdx.x == 0) {
            const unsigned int prev =
                __hip_atomic_fetch_add(&bar.xcd_count[xcc], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (prev + 1 == gen * mine) {
                // last workgroup of this XCD: write the XCD's L2 back, then arrive
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_fetch_add(bar.count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            ok = wait_at_least(bar.count, gridDim.x + gen * populated, bar.error);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (!ok) return;
    }
}

__global__ void k_fill_u32(unsigned int* p, int count, unsigned int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

template <int ST, bool PBB, bool NT>
lbm_status launch_persistent_t(const TrtConst& c, int chunk_shift, int64_t n, int64_t stride,
                               const uint32_t* adj, const double* ns, void* fa, void* fb,
                               int n_steps, void* ws, hipStream_t s) {
    using T = typename Storage<ST>::T;
    auto kern = k_trt_persistent<ST, PBB, NT>;
    int dev = 0, cus = 0, per_cu = 0, coop = 0;
    LBM_TRY_HIP(hipGetDevice(&dev));
    LBM_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    LBM_TRY_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) return LBM_EHIP;
    LBM_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                             kPBlock, 0));
    if (per_cu < 1) return LBM_EHIP;
    const int64_t tiles = (n + kPBlock - 1) / kPBlock;
    int64_t grid = std::min<int64_t>(cus, (tiles + NXCD - 1) / NXCD * NXCD);
    grid = grid / NXCD * NXCD;
    if (grid < NXCD) return LBM_EHIP;  // the device cannot hold one workgroup per XCD

    unsigned int* w = static_cast<unsigned int*>(ws);
    Barrier bar{w, reinterpret_cast<int*>(w + 1), w + 8, w + 16};
    // clear with a kernel (no memset node if the caller captures the stream)
    k_fill_u32<<<1, 64, 0, s>>>(w, 24, 0u);
    if (hipGetLastError() != hipSuccess) return LBM_EHIP;

    T* a = static_cast<T*>(fa);
    T* b = static_cast<T*>(fb);
    int steps = n_steps, cs = chunk_shift;
    TrtConst cc = c;
    void* args[] = {&a, &b, const_cast<uint32_t**>(&adj), const_cast<double**>(&ns),
                    &n, &stride, &cc, &steps, &cs, &bar};
    LBM_TRY_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(unsigned(grid)),
                                           dim3(kPBlock), args, 0, s));
    int err = 0;
    LBM_TRY_HIP(hipMemcpyAsync(&err, bar.error, sizeof(int), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    return err ? LBM_EBARRIER : LBM_OK;
}

template <int ST>
lbm_status launch_persistent_s(const TrtConst& c, bool nt, int cs, int64_t n, int64_t stride,
                               const uint32_t* adj, const double* ns, void* fa, void* fb,
                               int n_steps, void* ws, hipStream_t s) {
    if (ns) return nt ? launch_persistent_t<ST, true, true>(c, cs, n, stride, adj, ns, fa, fb, n_steps, ws, s)
                      : launch_persistent_t<ST, true, false>(c, cs, n, stride, adj, ns, fa, fb, n_steps, ws, s);
    return nt ? launch_persistent_t<ST, false, true>(c, cs, n, stride, adj, ns, fa, fb, n_steps, ws, s)
              : launch_persistent_t<ST, false, false>(c, cs, n, stride, adj, ns, fa, fb, n_steps, ws, s);
}

lbm_status launch_persistent(int storage, const TrtConst& c, bool nt, int chunk_shift, int64_t n,
                             int64_t stride, const uint32_t* adj, const double* ns, void* fa,
                             void* fb, int n_steps, void* ws, hipStream_t s) {
    switch (storage) {
    case LBM_F64: return launch_persistent_s<LBM_F64>(c, nt, chunk_shift, n, stride, adj, ns, fa, fb, n_steps, ws, s);
    case LBM_F64_SHIFTED: return launch_persistent_s<LBM_F64_SHIFTED>(c, nt, chunk_shift, n, stride, adj, ns, fa, fb, n_steps, ws, s);
    case LBM_F32: return launch_persistent_s<LBM_F32>(c, nt, chunk_shift, n, stride, adj, ns, fa, fb, n_steps, ws, s);
    case LBM_F32_SHIFTED: return launch_persistent_s<LBM_F32_SHIFTED>(c, nt, chunk_shift, n, stride, adj, ns, fa, fb, n_steps, ws, s);
    case LBM_F16_SHIFTED: return launch_persistent_s<LBM_F16_SHIFTED>(c, nt, chunk_shift, n, stride, adj, ns, fa, fb, n_steps, ws, s);
    default: return LBM_EINVAL;
    }
}

}  // namespace lbm
