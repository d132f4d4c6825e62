// The dealiased form (eq. (sum) read literally) on the N = 24 grid: spectra padded to
// NI = 36, whose gain kernels keep the complex product.  A 36 x 36 x-plane takes 10.7 KB
// of LDS in FP32 (21 KB in FP64), so a workgroup holds 12 (6) of them: CH = 3 (6).
#include "dealias.hpp"

namespace dgfs {

hipError_t run_dealias_24(const dgfs_plan& outer, const dgfs_plan& inner, const void* f, void* Q, int nb, void* ws,
                          bool pairs, hipStream_t st, hipEvent_t* ev) {
    const int key = inner.geo.CH * 100 + inner.geo.CZ;
    if (outer.precision == DGFS_FP64) {
        switch (key) {
            case 604: return detail::run_dealiased<double, 24, 6, 4, false>(
                outer, inner, static_cast<const double*>(f), static_cast<double*>(Q), nb, ws, pairs, st, ev);
            default: return hipErrorInvalidValue;
        }
    }
    switch (key) {
        case 302: return detail::run_dealiased<float, 24, 3, 2, false>(
            outer, inner, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dgfs
