// Gain-kernel geometries compiled for N = 48 with a VSS kernel (sigma-dependent kernel
// mode): the same tiles as the VHS family, each direction transformed as one
// complex field (the packed two-field form is not used here).
#include "dealias.hpp"

namespace dgfs {

hipError_t run_vss_48(const dgfs_plan& p, const void* f, void* Q, int nb, void* ws, bool pairs, hipStream_t st,
                      hipEvent_t* ev) {
    const int key = p.geo.CH * 100 + p.geo.CZ;
    if (p.precision == DGFS_FP64) {
        switch (key) {
            case 1204: return detail::run_slice<double, 48, 12, 4, false, false, true>(
                p, static_cast<const double*>(f), static_cast<double*>(Q), nb, ws, pairs, st, ev);
            default: return hipErrorInvalidValue;
        }
    }
    switch (key) {
        case 602: return detail::run_slice<float, 48, 6, 2, true, false, true>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        case 1204: return detail::run_slice<float, 48, 12, 4, false, false, true>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        case 1202: return detail::run_slice<float, 48, 12, 2, false, false, true>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        default: return hipErrorInvalidValue;
    }
}

// The dealiased form on the N = 32 grid, its gain on this NI = 48 grid (the inner
// plan's tile geometry).
hipError_t run_dealias_32(const dgfs_plan& outer, const dgfs_plan& inner, const void* f, void* Q, int nb, void* ws,
                          bool pairs, hipStream_t st, hipEvent_t* ev) {
    const int key = inner.geo.CH * 100 + inner.geo.CZ;
    if (outer.precision == DGFS_FP64) {
        switch (key) {
            case 1204: return detail::run_dealiased<double, 32, 12, 4, false>(
                outer, inner, static_cast<const double*>(f), static_cast<double*>(Q), nb, ws, pairs, st, ev);
            default: return hipErrorInvalidValue;
        }
    }
    switch (key) {
            case 602: return detail::run_dealiased<float, 32, 6, 2, true>(
                outer, inner, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
            case 1204: return detail::run_dealiased<float, 32, 12, 4, false>(
                outer, inner, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
            case 1202: return detail::run_dealiased<float, 32, 12, 2, false>(
                outer, inner, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dgfs
