// abi.cpp -- host-only entry points of the C ABI.
#include "lbm.h"

extern "C" int32_t lbm_version(void) { return 1 * 10000 + 1 * 100 + 0; }

extern "C" const char* lbm_status_string(int32_t status) {
    switch (status) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ECAPACITY: return "output capacity too small";
    case LBM_EOVERFLOW: return "index overflow (19*stride >= 2^32 or box >= 2^31 cells)";
    case LBM_EWORKSPACE: return "workspace missing or too small";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_EBARRIER: return "grid barrier timed out in persistent launch";
    case LBM_ENONFINITE: return "non-finite totals (NaN or infinity in the state)";
    default: return "unknown status";
    }
}
