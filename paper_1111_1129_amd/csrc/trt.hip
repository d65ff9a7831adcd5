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
//  * workgroups are relabelled so that each XCD (own L2) takes runs of
//    consecutive list tiles: the neighbours a pull reads are nearby list
//    entries, so their cache lines are shared within one L2 (run length set
//    by the LBM_FLAG_XCD_CHUNK bits).
// No MFMA: there is no dense contraction here.
#include <algorithm>

#include "lbm_device.hpp"
#include "lbm_host.hpp"

namespace lbm {

constexpr int kBlock = 256;

// batch.hip: sweeps with constants from a parameter table (per-segment
// parameter sets, persistent launch)
size_t step_batch_workspace(int32_t n_params, const lbm_segment* seg, int32_t n_seg, int64_t n);
lbm_status step_batch(const lbm_params* p, int32_t n_params, const lbm_segment* seg,
                      int32_t n_seg, int64_t n, int64_t stride, const int8_t* codes8,
                      const int16_t* codes, const int32_t* tile_records, const uint32_t* adj,
                      const double* ns, void* f_a, void* f_b, int32_t n_steps, bool persistent,
                      void* workspace, hipStream_t s);
// compress.hip: one launch per step over 16-bit / 8-bit codes
lbm_status step_coded(const lbm_params& p, int64_t n, int64_t stride, const int8_t* codes8,
                      const int16_t* codes, const int32_t* toff, const uint32_t* adj,
                      const double* ns, void* fa, void* fb, int n_steps, hipStream_t s);

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
    for (int i = 0; i < Q; ++i)
        st<T, typename Storage<ST>::A, false>(f + i * stride + m, static_cast<typename Storage<ST>::A>(e.v[i]));
}

template <int ST, bool PBB, bool NT>
__global__ __launch_bounds__(kBlock) void k_trt(const typename Storage<ST>::T* __restrict__ src,
                                                typename Storage<ST>::T* __restrict__ dst,
                                                const uint32_t* __restrict__ adj,
                                                const double* __restrict__ ns, int64_t n,
                                                int64_t stride, TrtConst c, int chunk_shift) {
    const int64_t m = logical_block(chunk_shift) * kBlock + threadIdx.x;
    if (m >= n) return;
    update_cell<ST, PBB, NT>(src, dst, adj, ns, m, stride, c);
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
lbm_status launch_steps(const TrtConst& c, int chunk_shift, int64_t n, int64_t stride,
                        const uint32_t* adj, const double* ns, void* fa, void* fb, int n_steps,
                        hipStream_t s) {
    using T = typename Storage<ST>::T;
    T* a = static_cast<T*>(fa);
    T* b = static_cast<T*>(fb);
    const int64_t grid = grid_blocks(n, kBlock, chunk_shift);
    for (int k = 0; k < n_steps; ++k) {
        const T* src = (k & 1) ? b : a;
        T* dst = (k & 1) ? a : b;
        k_trt<ST, PBB, NT><<<dim3(unsigned(grid)), dim3(kBlock), 0, s>>>(src, dst, adj, ns, n, stride, c,
                                                                       chunk_shift);
        if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    }
    return LBM_OK;
}

template <int ST>
lbm_status dispatch_step(const lbm_params& p, int64_t n, int64_t stride, const uint32_t* adj,
                         const double* ns, void* fa, void* fb, int n_steps, hipStream_t s) {
    const TrtConst c = make_trt_const(p);
    const bool nt = (p.flags & LBM_FLAG_NONTEMPORAL) != 0;
    const int cs = chunk_shift_for(p.flags, n, kBlock);
    if (ns) return nt ? launch_steps<ST, true, true>(c, cs, n, stride, adj, ns, fa, fb, n_steps, s)
                      : launch_steps<ST, true, false>(c, cs, n, stride, adj, ns, fa, fb, n_steps, s);
    return nt ? launch_steps<ST, false, true>(c, cs, n, stride, adj, ns, fa, fb, n_steps, s)
              : launch_steps<ST, false, false>(c, cs, n, stride, adj, ns, fa, fb, n_steps, s);
}

}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_init(const lbm_params* p, int64_t n, int64_t stride, void* f,
                               double rho0, const double* u0, void* stream) {
    if (!p || !f || !valid_storage(p->storage) || !std::isfinite(rho0)) return LBM_EINVAL;
    if (u0 && !(std::isfinite(u0[0]) && std::isfinite(u0[1]) && std::isfinite(u0[2])))
        return LBM_EINVAL;
    if (lbm_status st = check_layout(n, stride); st != LBM_OK) return st;
    hipStream_t s = as_stream(stream);
    switch (p->storage) {
    case LBM_F64: return launch_init<LBM_F64>(*p, n, stride, f, rho0, u0, s);
    case LBM_F64_SHIFTED: return launch_init<LBM_F64_SHIFTED>(*p, n, stride, f, rho0, u0, s);
    case LBM_F32: return launch_init<LBM_F32>(*p, n, stride, f, rho0, u0, s);
    case LBM_F32_SHIFTED: return launch_init<LBM_F32_SHIFTED>(*p, n, stride, f, rho0, u0, s);
    case LBM_F16_SHIFTED: return launch_init<LBM_F16_SHIFTED>(*p, n, stride, f, rho0, u0, s);
    case LBM_F16_SHIFTED_SCALED: return launch_init<LBM_F16_SHIFTED_SCALED>(*p, n, stride, f, rho0, u0, s);
    default: return LBM_EINVAL;
    }
}

extern "C" lbm_status lbm_step_batch(const lbm_params* p, int32_t n_params,
                                     const lbm_segment* seg, int32_t n_seg, int64_t n,
                                     int64_t stride, const int8_t* codes8, const int16_t* codes,
                                     const int32_t* tile_records, const uint32_t* adj,
                                     const double* ns, void* f_a, void* f_b, int32_t n_steps,
                                     int32_t persistent, void* workspace, size_t* ws_bytes,
                                     void* stream) {
    if (!p || n_params < 1 || n_params > kMaxParamSets || n_seg < 0 || (n_seg > 0 && !seg))
        return LBM_EINVAL;
    const bool table = persistent || uses_param_sets(seg, n_seg);
    if (table && !workspace) {  // size query
        if (!ws_bytes) return LBM_EINVAL;
        *ws_bytes = step_batch_workspace(n_params, seg, n_seg, std::max<int64_t>(n, 0));
        return LBM_OK;
    }
    for (int32_t k = 0; k < n_params; ++k) {
        if (!valid_params(&p[k])) return LBM_EINVAL;
        // one array type and one set of launch options for the whole launch
        if (p[k].storage != p[0].storage || p[k].flags != p[0].flags) return LBM_EINVAL;
    }
    if (!adj || !f_a || !f_b || f_a == f_b || n_steps < 0) return LBM_EINVAL;
    if ((codes8 && !codes) || ((codes != nullptr) != (tile_records != nullptr))) return LBM_EINVAL;
    if (lbm_status st = check_layout(n, stride); st != LBM_OK) return st;
    if (!valid_segments(seg, n_seg, n, n_params)) return LBM_EINVAL;
    if (table && (!ws_bytes || *ws_bytes < step_batch_workspace(n_params, seg, n_seg, n)))
        return LBM_EWORKSPACE;
    if (n == 0 || n_steps == 0) return LBM_OK;
    hipStream_t s = as_stream(stream);
    if (table)
        return step_batch(p, n_params, seg, n_seg, n, stride, codes8, codes, tile_records, adj, ns,
                          f_a, f_b, n_steps, persistent != 0, workspace, s);
    // one parameter set, one launch per step: constants as kernel arguments
    if (codes) return step_coded(*p, n, stride, codes8, codes, tile_records, adj, ns, f_a, f_b, n_steps, s);
    switch (p->storage) {
    case LBM_F64: return dispatch_step<LBM_F64>(*p, n, stride, adj, ns, f_a, f_b, n_steps, s);
    case LBM_F64_SHIFTED: return dispatch_step<LBM_F64_SHIFTED>(*p, n, stride, adj, ns, f_a, f_b, n_steps, s);
    case LBM_F32: return dispatch_step<LBM_F32>(*p, n, stride, adj, ns, f_a, f_b, n_steps, s);
    case LBM_F32_SHIFTED: return dispatch_step<LBM_F32_SHIFTED>(*p, n, stride, adj, ns, f_a, f_b, n_steps, s);
    case LBM_F16_SHIFTED: return dispatch_step<LBM_F16_SHIFTED>(*p, n, stride, adj, ns, f_a, f_b, n_steps, s);
    case LBM_F16_SHIFTED_SCALED: return dispatch_step<LBM_F16_SHIFTED_SCALED>(*p, n, stride, adj, ns, f_a, f_b, n_steps, s);
    default: return LBM_EINVAL;
    }
}

extern "C" lbm_status lbm_step(const lbm_params* p, int32_t n_params, const lbm_segment* seg,
                               int32_t n_seg, int64_t n, int64_t stride, const uint32_t* adj,
                               const double* ns, void* f_a, void* f_b, int32_t n_steps,
                               int32_t persistent, void* workspace, size_t* ws_bytes,
                               void* stream) {
    return lbm_step_batch(p, n_params, seg, n_seg, n, stride, nullptr, nullptr, nullptr, adj, ns,
                          f_a, f_b, n_steps, persistent, workspace, ws_bytes, stream);
}
