// Gain-kernel geometries compiled for N = 32: tile = (x-chunks CH, pencil groups CZ),
// whether the x-pass double-buffers its loads, and whether the two shifted fields share
// one y/z transform (packed form); both chosen per geometry by measurement.  (2, 0): the
// shifted fields are formed on the matrix cores (gain_mfma.hip).
#include "gain.hpp"

namespace dgfs {

hipError_t run_tiles_32(const dgfs_plan& p, const void* f, void* Q, int nb, void* ws, bool pairs, hipStream_t st,
                        hipEvent_t* ev) {
    const int key = p.geo.CH * 100 + p.geo.CZ;
    if (p.precision == DGFS_FP64) {
        switch (key) {
            case 402: return detail::run_slice<double, 32, 4, 2, false, false, false>(
                p, static_cast<const double*>(f), static_cast<double*>(Q), nb, ws, pairs, st, ev);
            default: return hipErrorInvalidValue;
        }
    }
    switch (key) {
        case 201: return detail::run_slice<float, 32, 2, 1, true, false, false>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        case 401: return detail::run_slice<float, 32, 4, 1, false, false, false>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        case 402: return detail::run_slice<float, 32, 4, 2, true, false, false>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        case 200: return detail::run_slice<float, 32, 2, 1, true, false, false, true>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dgfs
