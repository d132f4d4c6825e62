// Gain-kernel geometries compiled for N = 24: tile = (x-chunks CH, pencil groups CZ),
// whether the x-pass double-buffers its loads, and whether the two shifted fields share
// one y/z transform (packed form); both chosen per geometry by measurement.
#include "gain.hpp"

namespace dgfs {

hipError_t run_tiles_24(const dgfs_plan& p, const void* f, void* Q, int nb, void* ws, bool pairs, hipStream_t st,
                        hipEvent_t* ev) {
    const int key = p.geo.CH * 100 + p.geo.CZ;
    if (p.precision == DGFS_FP64) {
        switch (key) {
            case 302: return detail::run_slice<double, 24, 3, 2, false, false, false>(
                p, static_cast<const double*>(f), static_cast<double*>(Q), nb, ws, pairs, st, ev);
            default: return hipErrorInvalidValue;
        }
    }
    switch (key) {
        case 301: return detail::run_slice<float, 24, 3, 1, false, false, false>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        case 302: return detail::run_slice<float, 24, 3, 2, false, false, false>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        case 304: return detail::run_slice<float, 24, 3, 4, false, false, false>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        case 303: return detail::run_slice<float, 24, 3, 3, false, false, false>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        case 101: return detail::run_slice<float, 24, 1, 1, false, false, false>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dgfs
