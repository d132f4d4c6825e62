// Batched 3-D FFTs of N^3 fields in global memory, one pencil per thread per pass.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft.hpp"

namespace dgfs {

// ============================================================ pencil FFT passes
// One thread transforms one pencil of a batch of N^3 fields along AXIS (0 = x,
// stride N^2; 1 = y, stride N; 2 = z, stride 1).  In place when in == out.
template <typename T, int N, int AXIS, int SIGN, bool REAL_IN>
__global__ __launch_bounds__(256) void fft_pass_kernel(const void* __restrict__ in, cx<T>* out,
                                                       int64_t npencils, T scale) {
    const int64_t pid = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (pid >= npencils) return;
    constexpr int64_t N2 = int64_t(N) * N, N3 = N2 * N;
    const int64_t field = pid / N2;
    const int r = int(pid - field * N2);
    int64_t base, stride;
    if constexpr (AXIS == 0) {
        base = field * N3 + r;
        stride = N2;
    } else if constexpr (AXIS == 1) {
        base = field * N3 + int64_t(r / N) * N2 + (r % N);
        stride = N;
    } else {
        base = field * N3 + int64_t(r) * N;
        stride = 1;
    }
    cx<T> v[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        if constexpr (REAL_IN) {
            v[k] = cx<T>{static_cast<const T*>(in)[base + k * stride], T(0)};
        } else {
            v[k] = static_cast<const cx<T>*>(in)[base + k * stride];
        }
    }
    fft<N, SIGN>(v);
#pragma unroll
    for (int k = 0; k < N; ++k) out[base + k * stride] = scale * v[k];
}

// Full 3-D transform of nfields fields in place (from real_in when sign < 0):
// sign < 0: forward (z from the real input, then y, then x with `scale`);
// sign > 0: unnormalised inverse (x, y, then z with `scale`).
template <typename T, int N>
hipError_t fft3d(cx<T>* data, const void* real_in, int64_t nfields, int sign, T scale, hipStream_t st) {
    const int64_t np = nfields * N * N;
    const dim3 grid(unsigned((np + 255) / 256)), block(256);
    if (sign < 0) {
        // forward: z (from the real input when given), y, x (with scale)
        if (real_in)
            fft_pass_kernel<T, N, 2, -1, true><<<grid, block, 0, st>>>(real_in, data, np, T(1));
        else
            fft_pass_kernel<T, N, 2, -1, false><<<grid, block, 0, st>>>(data, data, np, T(1));
        fft_pass_kernel<T, N, 1, -1, false><<<grid, block, 0, st>>>(data, data, np, T(1));
        fft_pass_kernel<T, N, 0, -1, false><<<grid, block, 0, st>>>(data, data, np, scale);
    } else {
        fft_pass_kernel<T, N, 0, +1, false><<<grid, block, 0, st>>>(data, data, np, T(1));
        fft_pass_kernel<T, N, 1, +1, false><<<grid, block, 0, st>>>(data, data, np, T(1));
        fft_pass_kernel<T, N, 2, +1, false><<<grid, block, 0, st>>>(data, data, np, scale);
    }
    return hipGetLastError();
}

}  // namespace dgfs
