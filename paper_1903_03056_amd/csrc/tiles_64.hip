// Gain-kernel geometries compiled for N = 64: tile = (x-chunks CH, pencil groups CZ).
// A 64 x 64 x-plane of complex values takes 33 KB of LDS in FP32 (66 KB in FP64), so a
// workgroup holds 4 (2) x-planes: CH = 16 (32), with 1024 threads in CZ = 4 (8) groups per
// y/z pencil.  The x-pass then recombines the whole pencil for every chunk, which is the
// price of the LDS capacity at this size; N = 64 serves the accuracy studies of Sec. 6.1.
#include "gain.hpp"

namespace dgfs {

hipError_t run_tiles_64(const dgfs_plan& p, const void* f, void* Q, int nb, void* ws, bool pairs, hipStream_t st,
                        hipEvent_t* ev) {
    const int key = p.geo.CH * 100 + p.geo.CZ;
    if (p.precision == DGFS_FP64) {
        switch (key) {
            case 3208: return detail::run_slice<double, 64, 32, 8, false, false, false>(
                p, static_cast<const double*>(f), static_cast<double*>(Q), nb, ws, pairs, st, ev);
            default: return hipErrorInvalidValue;
        }
    }
    switch (key) {
        case 1604: return detail::run_slice<float, 64, 16, 4, false, false, false>(
            p, static_cast<const float*>(f), static_cast<float*>(Q), nb, ws, pairs, st, ev);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dgfs
