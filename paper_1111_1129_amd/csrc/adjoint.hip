// adjoint.hip -- discrete adjoint of one TRT pull step (lbm_step_adjoint).
//
// Forward step f^{t+1} = Phi(P f^t; ns): P is the pull gather through the
// adjacency (a permutation of PDF slots), Phi the per-cell collision with
// partial bounce-back.  Its transpose is applied per cell:
//   mu = lambda^{t+1}[.][m]                        (coalesced rows)
//   nu = (dPhi/dg)^T mu                            (local 19x19, in closed form)
//   lambda^t[A_k(m)] = nu_k                        (scatter through the same
//                                                   adjacency; A_0 = own slot)
// Every slot of lambda^t is written by exactly one (cell, direction) because
// P is a permutation, so the scatter needs no atomics.  The closed form:
//   with j the pre-collision momentum, m0 = sum w mu, m1 = sum w mu c,
//   m2 = sum w mu (c.j) c, mu+- = (mu_k +- mu_opp)/2:
//   nu_k = (1-ns)[mu_k - s+ mu+_k - s- mu-_k + s+ (m0 + 9 c_k.m2 - 3 m0 c_k.j)
//                 + 3 s- c_k.m1] + ns mu_opp(k)
//   grad[m] += sum_i mu_i (g_opp(i) - f*_i)
// which follows from d e+_i/d g_k = w_i [1 + 9 (c_i.j)(c_i.c_k) - 3 j.c_k] and
// d e-_i/d g_k = 3 w_i c_i.c_k.
#include "lbm_device.hpp"
#include "lbm_host.hpp"

namespace lbm {

constexpr int kAdjBlock = 256;
static_assert(kAdjBlock == kCodeTile, "a workgroup of k_adjoint_coded is one code tile");

// The adjoint of one cell m whose 19 slots A (A[0] = m, A[k+1] = the slot it
// pulls direction k + 1 from) are known.
template <bool PBB, bool NT>
__device__ __forceinline__ void adjoint_cell(const double* __restrict__ f_t, const uint32_t* A,
                                             const double* __restrict__ ns,
                                             const double* __restrict__ lam_next,
                                             double* __restrict__ lam_t,
                                             double* __restrict__ grad, int64_t m,
                                             int64_t stride, const TrtConst& c) {
    double g[Q], mu[Q], fs[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) g[k] = f_t[A[k]];
#pragma unroll
    for (int k = 0; k < Q; ++k) mu[k] = ld_stream(lam_next + k * stride + m);  // own column, read once
    trt_collide<double, false>(g, fs, c, 0.0);
    const CellMoments<double> cm = cell_moments(g);
    const double s = PBB ? ns[m] : 0.0;
    if constexpr (PBB) {
        double acc = mu[0] * (g[0] - fs[0]);
#pragma unroll
        for (int k = 0; k < NPAIR; ++k) {
            const int a = 2 * k + 1, b = 2 * k + 2;
            acc += mu[a] * (g[b] - fs[a]) + mu[b] * (g[a] - fs[b]);
        }
        if (grad) grad[m] += acc;
    }
    // moments of w mu
    double m0 = W0 * mu[0], m1x = 0, m1y = 0, m1z = 0, m2x = 0, m2y = 0, m2z = 0;
#pragma unroll
    for (int k = 0; k < NPAIR; ++k) {
        const int a = 2 * k + 1, b = 2 * k + 2;
        const double w = pair_weight(k);
        const double cj = PCX[k] * cm.jx + PCY[k] * cm.jy + PCZ[k] * cm.jz;
        const double sum = w * (mu[a] + mu[b]), dif = w * (mu[a] - mu[b]);
        m0 += sum;
        m1x += PCX[k] * dif;
        m1y += PCY[k] * dif;
        m1z += PCZ[k] * dif;
        m2x += PCX[k] * cj * sum;
        m2y += PCY[k] * cj * sum;
        m2z += PCZ[k] * cj * sum;
    }
    const double sp = c.sp, sm = c.sm;
    const double P = sp * m0;
    double nu0 = mu[0] - sp * mu[0] + P;
    if constexpr (PBB) nu0 = (1.0 - s) * nu0 + s * mu[0];
    st<double, double, NT>(lam_t + A[0], nu0);
#pragma unroll
    for (int k = 0; k < NPAIR; ++k) {
        const int a = 2 * k + 1, b = 2 * k + 2;
        const double cj = PCX[k] * cm.jx + PCY[k] * cm.jy + PCZ[k] * cm.jz;
        const double cm1 = PCX[k] * m1x + PCY[k] * m1y + PCZ[k] * m1z;
        const double cm2 = PCX[k] * m2x + PCY[k] * m2y + PCZ[k] * m2z;
        const double Qd = sp * (9.0 * cm2 - 3.0 * m0 * cj) + 3.0 * sm * cm1;
        const double mup = 0.5 * (mu[a] + mu[b]), mum = 0.5 * (mu[a] - mu[b]);
        double na = mu[a] - sp * mup - sm * mum + P + Qd;
        double nb = mu[b] - sp * mup + sm * mum + P - Qd;
        if constexpr (PBB) {
            na = (1.0 - s) * na + s * mu[b];
            nb = (1.0 - s) * nb + s * mu[a];
        }
        st<double, double, NT>(lam_t + A[a], na);
        st<double, double, NT>(lam_t + A[b], nb);
    }
}

template <bool PBB, bool NT>
__global__ __launch_bounds__(kAdjBlock) void k_adjoint(const double* __restrict__ f_t,
                                                       const uint32_t* __restrict__ adj,
                                                       const double* __restrict__ ns,
                                                       const double* __restrict__ lam_next,
                                                       double* __restrict__ lam_t,
                                                       double* __restrict__ grad, int64_t n,
                                                       int64_t stride, TrtConst c,
                                                       int chunk_shift) {
    const int64_t m = logical_block(chunk_shift) * kAdjBlock + threadIdx.x;
    if (m >= n) return;
    uint32_t A[Q];
    A[0] = uint32_t(m);
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) A[k + 1] = ld_stream(adj + k * stride + m);
    adjoint_cell<PBB, NT>(f_t, A, ns, lam_next, lam_t, grad, m, stride, c);
}

// Same, with the slots rebuilt from the adjacency codes of
// lbm_compress_adjacency (a workgroup is one 256-cell code tile): with C8 the
// 8-bit codes of a narrow tile (lbm_narrow_codes), otherwise the 16-bit codes;
// a tile with escapes reads adj.  The branch is uniform over the workgroup and
// every form rebuilds the same slots, so the result does not depend on it.
template <bool PBB, bool NT, bool C8>
__global__ __launch_bounds__(kAdjBlock) void k_adjoint_coded(const double* __restrict__ f_t,
                                                             const int8_t* __restrict__ codes8,
                                                             const int16_t* __restrict__ codes,
                                                             const int32_t* __restrict__ tile_rec,
                                                             const uint32_t* __restrict__ adj,
                                                             const double* __restrict__ ns,
                                                             const double* __restrict__ lam_next,
                                                             double* __restrict__ lam_t,
                                                             double* __restrict__ grad, int64_t n,
                                                             int64_t stride, TrtConst c,
                                                             int chunk_shift) {
    const int64_t tile = logical_block(chunk_shift);
    const int64_t m = tile * kAdjBlock + threadIdx.x;
    if (m >= n) return;
    const int32_t* rec = tile_rec + tile * kCodeRec;  // uniform over the workgroup
    uint32_t A[Q];
    A[0] = uint32_t(m);
    const uint32_t S = uint32_t(stride), mm = uint32_t(m);
    if (C8 && rec[Q] != 0) {
        int32_t cd[Q - 1];
#pragma unroll
        for (int k = 0; k < Q - 1; ++k) cd[k] = ld_stream(codes8 + k * stride + m);
#pragma unroll
        for (int k = 0; k < Q - 1; ++k) {
            const uint32_t i = k + 1;
            A[i] = cd[k] == int32_t(kCode8Bounce) ? uint32_t(opp(int(i))) * S + mm
                                                  : i * S + uint32_t(rec[k]) + mm + uint32_t(cd[k]);
        }
    } else if (rec[Q - 1] != 0) {
#pragma unroll
        for (int k = 0; k < Q - 1; ++k) A[k + 1] = ld_stream(adj + k * stride + m);
    } else {
        int32_t cd[Q - 1];
#pragma unroll
        for (int k = 0; k < Q - 1; ++k) cd[k] = ld_stream(codes + k * stride + m);
#pragma unroll
        for (int k = 0; k < Q - 1; ++k) {
            const uint32_t i = k + 1;
            A[i] = cd[k] == kCodeBounce ? uint32_t(opp(int(i))) * S + mm
                                        : i * S + uint32_t(rec[k]) + mm + uint32_t(cd[k]);
        }
    }
    adjoint_cell<PBB, NT>(f_t, A, ns, lam_next, lam_t, grad, m, stride, c);
}

// Seed lambda^T = dJ/df^T for J = (1/n) sum_m (j_x(m) + G_x/2): the slot a cell
// pulls for direction i carries c_ix / n; every other slot is 0.
__global__ __launch_bounds__(kAdjBlock) void k_adjoint_seed(const uint32_t* __restrict__ adj,
                                                            double* __restrict__ lam_t, int64_t n,
                                                            int64_t stride, double inv_n) {
    const int64_t m = int64_t(blockIdx.x) * kAdjBlock + threadIdx.x;
    if (m >= n) return;
    lam_t[m] = 0.0;
#pragma unroll
    for (int k = 0; k < Q - 1; ++k) lam_t[adj[k * stride + m]] = double(vel_x(k + 1)) * inv_n;
}

}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_step_adjoint(const lbm_params* p, int64_t n, int64_t stride,
                                       const uint32_t* adj, const void* f_t, const double* ns,
                                       const double* lam_next, double* lam_t, double* grad_ns,
                                       void* stream) {
    if (!valid_params(p) || !adj || !lam_t || n <= 0) return LBM_EINVAL;
    if (p->storage != LBM_F64 && p->storage != LBM_F64_SHIFTED) return LBM_EINVAL;
    if (lbm_status st = check_layout(n, stride); st != LBM_OK) return st;
    hipStream_t s = as_stream(stream);
    const unsigned grid = unsigned((n + kAdjBlock - 1) / kAdjBlock);
    if (!lam_next) {
        k_adjoint_seed<<<grid, kAdjBlock, 0, s>>>(adj, lam_t, n, stride, 1.0 / double(n));
        return after_launch();
    }
    if (!f_t) return LBM_EINVAL;
    const TrtConst c = make_trt_const(*p);
    const double* f = static_cast<const double*>(f_t);
    // the sweep's launch options: workgroup-to-XCD mapping, nontemporal stores
    const int cs = chunk_shift_for(p->flags, n, kAdjBlock);
    const dim3 g{unsigned(grid_blocks(n, kAdjBlock, cs))}, b{unsigned(kAdjBlock)};
    const bool nt = p->flags & LBM_FLAG_NONTEMPORAL;
    if (ns) {
        if (nt) k_adjoint<true, true><<<g, b, 0, s>>>(f, adj, ns, lam_next, lam_t, grad_ns, n, stride, c, cs);
        else k_adjoint<true, false><<<g, b, 0, s>>>(f, adj, ns, lam_next, lam_t, grad_ns, n, stride, c, cs);
    } else {
        if (nt) k_adjoint<false, true><<<g, b, 0, s>>>(f, adj, ns, lam_next, lam_t, nullptr, n, stride, c, cs);
        else k_adjoint<false, false><<<g, b, 0, s>>>(f, adj, ns, lam_next, lam_t, nullptr, n, stride, c, cs);
    }
    return after_launch();
}

namespace lbm {

template <bool C8>
lbm_status step_adjoint_coded(const lbm_params* p, int64_t n, int64_t stride,
                              const int8_t* codes8, const int16_t* codes,
                              const int32_t* tile_records, const uint32_t* adj, const void* f_t,
                              const double* ns, const double* lam_next, double* lam_t,
                              double* grad_ns, void* stream) {
    if (!valid_params(p) || (C8 && !codes8) || !codes || !tile_records || !adj || !f_t ||
        !lam_next || !lam_t || n <= 0)
        return LBM_EINVAL;
    if (p->storage != LBM_F64 && p->storage != LBM_F64_SHIFTED) return LBM_EINVAL;
    if (lbm_status st = check_layout(n, stride); st != LBM_OK) return st;
    hipStream_t s = as_stream(stream);
    const TrtConst c = make_trt_const(*p);
    const double* f = static_cast<const double*>(f_t);
    const int cs = chunk_shift_for(p->flags, n, kAdjBlock);
    const dim3 g{unsigned(grid_blocks(n, kAdjBlock, cs))}, b{unsigned(kAdjBlock)};
    const bool nt = p->flags & LBM_FLAG_NONTEMPORAL;
    if (ns) {
        if (nt) k_adjoint_coded<true, true, C8><<<g, b, 0, s>>>(f, codes8, codes, tile_records, adj, ns, lam_next, lam_t, grad_ns, n, stride, c, cs);
        else k_adjoint_coded<true, false, C8><<<g, b, 0, s>>>(f, codes8, codes, tile_records, adj, ns, lam_next, lam_t, grad_ns, n, stride, c, cs);
    } else {
        if (nt) k_adjoint_coded<false, true, C8><<<g, b, 0, s>>>(f, codes8, codes, tile_records, adj, ns, lam_next, lam_t, nullptr, n, stride, c, cs);
        else k_adjoint_coded<false, false, C8><<<g, b, 0, s>>>(f, codes8, codes, tile_records, adj, ns, lam_next, lam_t, nullptr, n, stride, c, cs);
    }
    return after_launch();
}

}  // namespace lbm

extern "C" lbm_status lbm_step_adjoint_c16(const lbm_params* p, int64_t n, int64_t stride,
                                           const int16_t* codes, const int32_t* tile_records,
                                           const uint32_t* adj, const void* f_t,
                                           const double* ns, const double* lam_next,
                                           double* lam_t, double* grad_ns, void* stream) {
    return step_adjoint_coded<false>(p, n, stride, nullptr, codes, tile_records, adj, f_t, ns,
                                     lam_next, lam_t, grad_ns, stream);
}

extern "C" lbm_status lbm_step_adjoint_c8(const lbm_params* p, int64_t n, int64_t stride,
                                          const int8_t* codes8, const int16_t* codes,
                                          const int32_t* tile_records, const uint32_t* adj,
                                          const void* f_t, const double* ns,
                                          const double* lam_next, double* lam_t,
                                          double* grad_ns, void* stream) {
    return step_adjoint_coded<true>(p, n, stride, codes8, codes, tile_records, adj, f_t, ns,
                                    lam_next, lam_t, grad_ns, stream);
}
