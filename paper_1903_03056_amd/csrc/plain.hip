// The plain per-point FP64 path: the fast spectral method of Sec. 4 written the
// straightforward way, for comparison with the fused batched kernels.  One node at a
// time, every ordered pair (i, j) with all M directions, and for every (rho_q, sigma_p)
// separate kernel launches over global memory: phase multiply, 3-D inverse FFT of
// each shifted spectrum, product accumulation, then per rho_q the forward FFT and the
// radial weighting, then the loss convolution and the inverse transforms.  FP64 only.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft.hpp"
#include "passes.hpp"
#include "plan.hpp"

namespace dgfs {
namespace {

using C64 = cx<double>;

template <int N>
__global__ __launch_bounds__(256) void plain_phase(const C64* __restrict__ fh, C64* __restrict__ X,
                                                   const C64* __restrict__ ph) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= int64_t(N) * N * N) return;
    const int jz = int(t % N), jy = int((t / N) % N), jx = int(t / (N * N));
    X[t] = fh[t] * ph[jx] * ph[N + jy] * ph[2 * N + jz];
}

template <int N>
__global__ __launch_bounds__(256) void plain_prod(const C64* __restrict__ A, const C64* __restrict__ B,
                                                  C64* __restrict__ S, double w) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= int64_t(N) * N * N) return;
    const C64 ab = A[t] * B[t];
    S[t] = S[t] + w * ab;
}

template <int N>
__device__ __forceinline__ int mode_sq(int64_t t) {
    auto sq = [](int k) {
        const int m = k < N / 2 ? k : k - N;
        return m * m;
    };
    return sq(int(t / (N * N))) + sq(int((t / N) % N)) + sq(int(t % N));
}

template <int N>
__global__ __launch_bounds__(256) void plain_radial(const C64* __restrict__ Sh, C64* __restrict__ Qp,
                                                    const double* __restrict__ F) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= int64_t(N) * N * N) return;
    Qp[t] = Qp[t] + F[mode_sq<N>(t)] * Sh[t];
}

template <int N>
__global__ __launch_bounds__(256) void plain_loss(const C64* __restrict__ fhj, C64* __restrict__ L,
                                                  const double* __restrict__ G) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= int64_t(N) * N * N) return;
    L[t] = G[mode_sq<N>(t)] * fhj[t];
}

template <int N>
__global__ __launch_bounds__(256) void plain_zero(C64* __restrict__ X) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= int64_t(N) * N * N) return;
    X[t] = C64{0.0, 0.0};
}

template <int N>
__global__ __launch_bounds__(256) void plain_final(const C64* __restrict__ Qp, const C64* __restrict__ nu,
                                                   const double* __restrict__ fi, double* __restrict__ Qi,
                                                   int first) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= int64_t(N) * N * N) return;
    const double v = Qp[t].x - fi[t] * nu[t].x;
    Qi[t] = first ? v : Qi[t] + v;
}

template <int N>
hipError_t plain_node(const dgfs_plan& p, const double* f, double* Q, void* ws, hipStream_t st) {
    constexpr int64_t N3 = int64_t(N) * N * N;
    const dim3 grid(unsigned((N3 + 255) / 256)), block(256);
    const int s = p.s, M = p.M, nrho = p.nrho, K2 = p.K2;
    C64* fh = static_cast<C64*>(ws);
    C64* XA = fh + s * N3;
    C64* XB = XA + N3;
    C64* S = XB + N3;
    C64* Qp = S + N3;
    C64* L = Qp + N3;
    const char* dev = static_cast<const char*>(p.dev);
    const C64* ph = reinterpret_cast<const C64*>(dev + p.off_plain_ph);
    const double* F = reinterpret_cast<const double*>(dev + p.off_plain_F);
    const double* G = reinterpret_cast<const double*>(dev + p.off_G);
    const double wsig = 4.0 * 3.14159265358979323846 / M;
    hipError_t e = fft3d<double, N>(fh, f, s, -1, 1.0 / double(N3), st);
    if (e != hipSuccess) return e;
    for (int i = 0; i < s; ++i) {
        for (int j = 0; j < s; ++j) {
            const int pr = i * s + j;
            plain_zero<N><<<grid, block, 0, st>>>(Qp);
            for (int q = 0; q < nrho; ++q) {
                plain_zero<N><<<grid, block, 0, st>>>(S);
                for (int d = 0; d < M; ++d) {
                    const C64* phA = ph + ((((int64_t(pr) * nrho + q) * M + d) * 2 + 0) * 3) * N;
                    const C64* phB = ph + ((((int64_t(pr) * nrho + q) * M + d) * 2 + 1) * 3) * N;
                    plain_phase<N><<<grid, block, 0, st>>>(fh + i * N3, XA, phA);
                    if ((e = fft3d<double, N>(XA, nullptr, 1, +1, 1.0, st)) != hipSuccess) return e;
                    plain_phase<N><<<grid, block, 0, st>>>(fh + j * N3, XB, phB);
                    if ((e = fft3d<double, N>(XB, nullptr, 1, +1, 1.0, st)) != hipSuccess) return e;
                    plain_prod<N><<<grid, block, 0, st>>>(XA, XB, S, wsig);
                }
                if ((e = fft3d<double, N>(S, nullptr, 1, -1, 1.0, st)) != hipSuccess) return e;
                plain_radial<N><<<grid, block, 0, st>>>(S, Qp, F + (int64_t(pr) * nrho + q) * K2);
            }
            plain_loss<N><<<grid, block, 0, st>>>(fh + j * N3, L, G + int64_t(pr) * K2);
            if ((e = fft3d<double, N>(L, nullptr, 1, +1, 1.0, st)) != hipSuccess) return e;
            if ((e = fft3d<double, N>(Qp, nullptr, 1, +1, 1.0, st)) != hipSuccess) return e;
            plain_final<N><<<grid, block, 0, st>>>(Qp, L, f + i * N3, Q + i * N3, j == 0);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

}  // namespace

size_t plain_ws_bytes(const dgfs_plan& p) { return size_t(p.s + 5) * p.n3() * sizeof(C64); }

hipError_t launch_collide_plain(const dgfs_plan& p, const double* f, double* Q, int64_t nb, void* ws,
                                hipStream_t st) {
    const int64_t stride = int64_t(p.s) * int64_t(p.n3());
    for (int64_t b = 0; b < nb; ++b) {
        hipError_t e;
        switch (p.N) {
            case 16: e = plain_node<16>(p, f + b * stride, Q + b * stride, ws, st); break;
            case 24: e = plain_node<24>(p, f + b * stride, Q + b * stride, ws, st); break;
            case 32: e = plain_node<32>(p, f + b * stride, Q + b * stride, ws, st); break;
            case 48: e = plain_node<48>(p, f + b * stride, Q + b * stride, ws, st); break;
            default: return hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace dgfs
