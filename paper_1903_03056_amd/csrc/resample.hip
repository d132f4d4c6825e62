// Moving fields between species-specific velocity grids.
//
// With an independent grid per species (the remedy named in the remark after
// eq. (domain), Sec. 4) the pair (i, j) is evaluated on the wider of the two boxes.  A
// field is carried from one grid to another by its real trigonometric interpolant,
// which is a product of three one-dimensional maps T (N x N, host-built): one pass per
// axis, each output point a length-N dot product of a row of T with an input pencil.
// The passes are bandwidth-light (N^4 FMAs per field and axis) next to the collision
// operator, so they stay simple: one thread per output point, rows of T read through
// the cache.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"

namespace dgfs {
namespace {

// out[b][..a..] (+)= sum_m T[a][m] in[b][..m..] along AXIS (0 = x, 1 = y, 2 = z fastest).
template <typename T, int AXIS>
__global__ __launch_bounds__(256) void resample_pass(const T* __restrict__ in, int64_t in_stride,
                                                     T* __restrict__ out, int64_t out_stride,
                                                     const T* __restrict__ Tm, int N, int64_t nb, int accumulate) {
    const int64_t n3 = int64_t(N) * N * N;
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= nb * n3) return;
    const int64_t b = t / n3;
    const int e = int(t - b * n3);
    const int x = e / (N * N), y = (e / N) % N, z = e % N;
    const int a = AXIS == 0 ? x : (AXIS == 1 ? y : z);
    const int64_t step = AXIS == 0 ? int64_t(N) * N : (AXIS == 1 ? N : 1);
    const T* src = in + b * in_stride + (e - int64_t(a) * step);
    const T* row = Tm + int64_t(a) * N;
    T acc = T(0);
    for (int m = 0; m < N; ++m) acc = fma(row[m], src[m * step], acc);
    T* dst = out + b * out_stride + e;
    *dst = accumulate ? *dst + acc : acc;
}

template <typename T>
__global__ __launch_bounds__(256) void copy_fields(const T* __restrict__ in, int64_t in_stride, T* __restrict__ out,
                                                   int64_t out_stride, int64_t n3, int64_t nb, int accumulate) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= nb * n3) return;
    const int64_t b = t / n3, e = t - b * n3;
    const T v = in[b * in_stride + e];
    T* dst = out + b * out_stride + e;
    *dst = accumulate ? *dst + v : v;
}

template <typename T>
hipError_t move_impl(const T* in, int64_t in_stride, T* out, int64_t out_stride, const T* Tm, int N, int64_t nb,
                     bool accumulate, T* tmp, hipStream_t st) {
    const int64_t n3 = int64_t(N) * N * N;
    const dim3 grid(unsigned((nb * n3 + 255) / 256)), block(256);
    if (!Tm) {
        copy_fields<T><<<grid, block, 0, st>>>(in, in_stride, out, out_stride, n3, nb, accumulate ? 1 : 0);
        return hipGetLastError();
    }
    T* t1 = tmp;
    T* t2 = tmp + nb * n3;
    resample_pass<T, 2><<<grid, block, 0, st>>>(in, in_stride, t1, n3, Tm, N, nb, 0);
    resample_pass<T, 1><<<grid, block, 0, st>>>(t1, n3, t2, n3, Tm, N, nb, 0);
    resample_pass<T, 0><<<grid, block, 0, st>>>(t2, n3, out, out_stride, Tm, N, nb, accumulate ? 1 : 0);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_move(const dgfs_plan& p, const void* in, int64_t in_stride, void* out, int64_t out_stride,
                       const void* Tm, int64_t nb, bool accumulate, void* tmp, hipStream_t st) {
    if (nb <= 0) return hipSuccess;
    if (p.precision == DGFS_FP64)
        return move_impl<double>(static_cast<const double*>(in), in_stride, static_cast<double*>(out), out_stride,
                                 static_cast<const double*>(Tm), p.N, nb, accumulate, static_cast<double*>(tmp), st);
    return move_impl<float>(static_cast<const float*>(in), in_stride, static_cast<float*>(out), out_stride,
                            static_cast<const float*>(Tm), p.N, nb, accumulate, static_cast<float*>(tmp), st);
}

}  // namespace dgfs
