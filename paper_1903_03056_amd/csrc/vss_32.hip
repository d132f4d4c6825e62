// Gain-kernel geometries compiled for N = 32 with a VSS kernel (sigma-dependent kernel
// mode): the same tiles as the VHS family, each direction transformed as one
// complex field (the packed two-field form is not used here).
#include "gain.hpp"

namespace dgfs {

hipError_t run_vss_32(const dgfs_plan& p, const void* f, void* Q, int nb, void* ws, bool pairs, hipStream_t st,
                      hipEvent_t* ev) {
    const int key = p.geo.CH * 100 + p.geo.CZ;
    if (p.precision == DGFS_FP64) {
        switch (key) {
            case 402: return detail::run_slice<double, 32, 4, 2, false, false, true>(
                p, static_cast<const double*>(f), static_cast<double*>(Q), nb, ws, pairs, st, ev);
            default: return hipErrorInvalidValue;
        }
    }
    switch (key) {
        case 201: return detail::run_slice<float, 32, 2, 1, true, false, true>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        case 401: return detail::run_slice<float, 32, 4, 1, false, false, true>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        case 402: return detail::run_slice<float, 32, 4, 2, true, false, true>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dgfs
