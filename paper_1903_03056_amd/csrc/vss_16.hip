// Gain-kernel geometries compiled for N = 16 with a VSS kernel (sigma-dependent kernel
// mode): the same tiles as the VHS family, each direction transformed as one
// complex field (the packed two-field form is not used here).
#include "gain.hpp"

namespace dgfs {

hipError_t run_vss_16(const dgfs_plan& p, const void* f, void* Q, int nb, void* ws, bool pairs, hipStream_t st,
                      hipEvent_t* ev) {
    const int key = p.geo.CH * 100 + p.geo.CZ;
    if (p.precision == DGFS_FP64) {
        switch (key) {
            case 101: return detail::run_slice<double, 16, 1, 1, false, false, true>(
                p, static_cast<const double*>(f), static_cast<double*>(Q), nb, ws, pairs, st, ev);
            default: return hipErrorInvalidValue;
        }
    }
    switch (key) {
        case 201: return detail::run_slice<float, 16, 2, 1, false, false, true>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        case 101: return detail::run_slice<float, 16, 1, 1, false, false, true>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        case 102: return detail::run_slice<float, 16, 1, 2, false, false, true>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dgfs
