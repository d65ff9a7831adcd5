// lbm_host.hpp -- host-side helpers shared by the library's entry points:
// argument validation and HIP error mapping.  Nothing here allocates.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "lbm.h"

namespace lbm {

constexpr int64_t kIndexLimit = int64_t(1) << 32;  // uint32 PDF slot index
constexpr int64_t kBoxLimit = int64_t(1) << 31;    // int32 box index

#define LBM_TRY_HIP(expr)                              \
    do {                                               \
        if ((expr) != hipSuccess) return LBM_EHIP;     \
    } while (0)

inline lbm_status after_launch() {
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EHIP;
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline bool valid_storage(int st) { return st >= LBM_F64 && st <= LBM_F16_SHIFTED_SCALED; }

// TRT parameters usable for a sweep: tau+ > 1/2 and tau- > 1/2 (magic > 0),
// everything finite.
inline bool valid_params(const lbm_params* p) {
    if (!p || !valid_storage(p->storage)) return false;
    const int32_t known = LBM_FLAG_NONTEMPORAL | LBM_FLAG_CHECK_FINITE | LBM_FLAG_XCD_CHUNK_MASK;
    if (p->flags & ~known) return false;
    const int32_t chunk = (p->flags & LBM_FLAG_XCD_CHUNK_MASK) >> LBM_FLAG_XCD_CHUNK_SHIFT;
    if (chunk & (chunk - 1)) return false;  // a power of two (or 0)
    if (!std::isfinite(p->tau_plus) || !std::isfinite(p->magic)) return false;
    if (!(p->tau_plus > 0.5) || !(p->magic > 0.0)) return false;
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(p->force[d])) return false;
    return true;
}

// 19 * stride < 2^32, tested without forming the product (a caller's
// stride near INT64_MAX would overflow it).
inline bool stride_fits(int64_t stride) { return stride >= 0 && stride <= (kIndexLimit - 1) / 19; }

// Layout checks common to every call that touches [19][stride] arrays.
inline lbm_status check_layout(int64_t n, int64_t stride) {
    if (n < 0 || stride < n || stride < 0) return LBM_EINVAL;
    if (!stride_fits(stride)) return LBM_EOVERFLOW;
    return LBM_OK;
}

// Segments are ranges inside [0, n) that do not overlap, listed in increasing
// order, each naming a parameter set in [0, n_params).  When any segment
// names a set other than 0, every non-empty segment starts on a tile of
// kSegmentAlign cells, so no tile holds cells of two segments.
constexpr int64_t kSegmentAlign = 256;
constexpr int32_t kMaxParamSets = 65536;  // parameter sets of one call

inline bool uses_param_sets(const lbm_segment* seg, int32_t n_seg) {
    for (int32_t k = 0; k < n_seg; ++k)
        if (seg[k].param_index != 0) return true;
    return false;
}

inline bool valid_segments(const lbm_segment* seg, int32_t n_seg, int64_t n, int32_t n_params) {
    if (n_seg < 0 || (n_seg > 0 && !seg)) return false;
    const bool sets = uses_param_sets(seg, n_seg);
    int64_t prev_end = 0;
    for (int32_t s = 0; s < n_seg; ++s) {
        if (seg[s].n < 0 || seg[s].base < prev_end || seg[s].base > n || seg[s].n > n - seg[s].base)
            return false;
        if (seg[s].param_index < 0 || seg[s].param_index >= n_params) return false;
        if (sets && seg[s].n > 0 && seg[s].base % kSegmentAlign != 0) return false;
        prev_end = seg[s].base + seg[s].n;
    }
    return true;
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace lbm
