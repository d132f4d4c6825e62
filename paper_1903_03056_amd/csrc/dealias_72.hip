// The dealiased form (eq. (sum) read literally) on the N = 48 grid: spectra padded to
// NI = 72.  A 72 x 72 x-plane takes 42 KB of LDS in FP32 (84 KB in FP64), so a workgroup
// holds 3 (1) of them: CH = 24 (72).  The x-pass then recombines the whole pencil for
// every chunk; this grid serves accuracy studies, not throughput.
#include "dealias.hpp"

namespace dgfs {

hipError_t run_dealias_48(const dgfs_plan& outer, const dgfs_plan& inner, const void* f, void* Q, int nb, void* ws,
                          bool pairs, hipStream_t st, hipEvent_t* ev) {
    const int key = inner.geo.CH * 100 + inner.geo.CZ;
    if (outer.precision == DGFS_FP64) {
        switch (key) {
            case 7208: return detail::run_dealiased<double, 48, 72, 8, false>(
                outer, inner, static_cast<const double*>(f), static_cast<double*>(Q), nb, ws, pairs, st, ev);
            default: return hipErrorInvalidValue;
        }
    }
    switch (key) {
        case 2404: return detail::run_dealiased<float, 48, 24, 4, false>(
            outer, inner, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dgfs
