// Gain-kernel geometries compiled for N = 48: tile = (x-chunks CH, pencil groups CZ),
// whether the x-pass double-buffers its loads, and whether the two shifted fields share
// one y/z transform (packed form); both chosen per geometry by measurement.
#include "gain.hpp"

namespace dgfs {

hipError_t run_tiles_48(const dgfs_plan& p, const void* f, void* Q, int nb, void* ws, bool pairs, hipStream_t st,
                        hipEvent_t* ev) {
    const int key = p.geo.CH * 100 + p.geo.CZ;
    if (p.precision == DGFS_FP64) {
        switch (key) {
            case 1204: return detail::run_slice<double, 48, 12, 4, false, false, false>(
                p, static_cast<const double*>(f), static_cast<double*>(Q), nb, ws, pairs, st, ev);
            default: return hipErrorInvalidValue;
        }
    }
    switch (key) {
        case 602: return detail::run_slice<float, 48, 6, 2, true, true, false>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        case 1204: return detail::run_slice<float, 48, 12, 4, false, true, false>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        case 1202: return detail::run_slice<float, 48, 12, 2, false, true, false>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        case 1201: return detail::run_slice<float, 48, 12, 1, false, true, false>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        case 1203: return detail::run_slice<float, 48, 12, 3, false, true, false>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dgfs
