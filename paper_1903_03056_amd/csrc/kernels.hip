// Device kernels of the fast spectral collision operator (Sec. 4 of the paper) for
// gfx950, and the host-side launch sequence.
//
// Pipeline for a slice of nb nodes (all fields complex, index space, z fastest):
//   1. fft_pass x3     f_hat = DFT(f) / N^3                        (per node, species)
//   2. gain_kernel     per (node, gain class, rho_q, x-chunk c):
//                        S_q = sum_p w_p A_p B_p in physical space, where
//                        A_p = IDFT(f_hat^i e^{+i pi rho a l.sigma_p / L})  (= f^i(v + a rho sigma_p))
//                        B_p = IDFT(f_hat^j e^{-i pi rho b m.sigma_p / L})  (= f^j(v - b rho sigma_p)),
//                      then the partial forward DFT of S_q over the chunk  -> P
//   3. radial_kernel   Q_hat+ = sum_terms sum_q w_q F(|k|, rho_q) / N^3 * DFT(S_q)
//                      L_hat  = sum_j G-_ij(|k|) f_hat^j          -> Gt, Lt (k_z <= N/2 half)
//   4. half_pass x2    inverse DFT of Gt and Lt along x and y, on the stored half
//   5. zpass_combine   inverse DFT along z (Hermitian rows, real result) fused with
//                      Q = IDFT(Gt) - f^i IDFT(Lt)
//
// The sigma-sum is taken before the forward transform of the gain because, for the
// VHS family, F(k, rho, sigma) does not depend on sigma; with an antipodal design the
// two orderings of an unlike pair share S_q and a like pair needs half the directions
// (see the host set-up).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gain.hpp"

namespace dgfs {

// ========================================================= FP64 conservation
// One workgroup per node: the s+4 invariants A Q in FP64, lambda = (A A^T)^{-1} A Q,
// then Q_out = Q - A^T lambda.  Rows of A: h_i^3 on species i (s rows), m_i h_i^3 v_d
// (3 rows), m_i h_i^3 |v|^2 (1 row), on species i's own grid (half-width Ls[i]).
// With UPDATE, the projected value is not stored but added to the state:
// f <- f + dt * Q_projected (forward-Euler step of a homogeneous relaxation).
// The grid size is a template argument for the compiled N (NC > 0), so the index
// arithmetic of the velocity coordinates uses constant divisors; NC = 0 reads it from Nrt.
template <typename TIN, bool UPDATE, int NC>
__global__ __launch_bounds__(1024) void conserve_kernel(const TIN* Q, double* out, TIN* fstate, double dt,
                                                        const double* __restrict__ Minv,
                                                        const double* __restrict__ mass,
                                                        const double* __restrict__ Ls, int s, int Nrt) {
    constexpr int R = 12;  // s + 4 <= 12
    __shared__ double red[16][R];
    __shared__ double lam[R];
    const int N = NC > 0 ? NC : Nrt;
    const int b = blockIdx.x;
    const int n3 = N * N * N;
    const int64_t tot = int64_t(s) * n3;
    const TIN* q = Q + int64_t(b) * tot;
    double* o = UPDATE ? nullptr : out + int64_t(b) * tot;
    TIN* fs = UPDATE ? fstate + int64_t(b) * tot : nullptr;
    const int nr = s + 4;
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    for (int i = 0; i < s; ++i) {
        const double L = Ls[i], h = 2.0 * L / N;
        const TIN* qi = q + int64_t(i) * n3;
        double a0 = 0.0, ax = 0.0, ay = 0.0, az = 0.0, ae = 0.0;
        for (int n = threadIdx.x; n < n3; n += 1024) {
            const double vx = -L + (n / (N * N)) * h, vy = -L + ((n / N) % N) * h, vz = -L + (n % N) * h;
            const double val = double(qi[n]);
            a0 += val;
            ax = fma(val, vx, ax);
            ay = fma(val, vy, ay);
            az = fma(val, vz, az);
            ae = fma(val, vx * vx + vy * vy + vz * vz, ae);
        }
        const double h3 = h * h * h, mh = mass[i] * h3;
#pragma unroll
        for (int r = 0; r < R - 4; ++r)
            if (r == i) acc[r] = h3 * a0;
        acc[R - 4] = fma(mh, ax, acc[R - 4]);
        acc[R - 3] = fma(mh, ay, acc[R - 3]);
        acc[R - 2] = fma(mh, az, acc[R - 2]);
        acc[R - 1] = fma(mh, ae, acc[R - 1]);
    }
    // block reduction
#pragma unroll
    for (int r = 0; r < R; ++r) {
        double v = acc[r];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[r] = v;
    }
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0)
        for (int r = 0; r < R; ++r) red[wave][r] = acc[r];
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot_r[R];
        for (int r = 0; r < R; ++r) {
            double v = 0.0;
            for (int w = 0; w < int(blockDim.x / 64); ++w) v += red[w][r];
            tot_r[r] = v;
        }
        // invariant vector in the order (species 0..s-1, px, py, pz, energy)
        double aq[R];
        for (int i = 0; i < s; ++i) aq[i] = tot_r[i];
        for (int d = 0; d < 4; ++d) aq[s + d] = tot_r[R - 4 + d];
        for (int r = 0; r < nr; ++r) {
            double v = 0.0;
            for (int c = 0; c < nr; ++c) v += Minv[r * nr + c] * aq[c];
            lam[r] = v;
        }
    }
    __syncthreads();
    for (int i = 0; i < s; ++i) {
        const double L = Ls[i], h = 2.0 * L / N, h3 = h * h * h, mh = mass[i] * h3;
        const double c0 = lam[i] * h3, cx_ = mh * lam[s], cy = mh * lam[s + 1], cz = mh * lam[s + 2],
                     ce = mh * lam[s + 3];
        const int64_t off = int64_t(i) * n3;
        for (int n = threadIdx.x; n < n3; n += 1024) {
            const double vx = -L + (n / (N * N)) * h, vy = -L + ((n / N) % N) * h, vz = -L + (n % N) * h;
            const double corr = c0 + cx_ * vx + cy * vy + cz * vz + ce * (vx * vx + vy * vy + vz * vz);
            const double v = double(q[off + n]) - corr;
            if constexpr (UPDATE)
                fs[off + n] = TIN(double(fs[off + n]) + dt * v);
            else
                o[off + n] = v;
        }
    }
}

// ======================================================= elementwise (stepping)
// out = a x + b y over n values (x, y, out may coincide elementwise).
template <typename T>
__global__ __launch_bounds__(256) void axpby_kernel(const T* x, const T* y, T* out, T a, T b, int64_t n) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t < n) out[t] = a * x[t] + b * y[t];
}

// ================================================================== launches
namespace {

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Compiled gain-kernel geometries (CH, CZ) per N and precision; the first is the default
// (the fastest measured on MI355X for that N; autotune.py re-measures on the device).
// (32, 2, 0): the matrix-core gain (FP32 VHS plans of the circular form; the others get
// the first geometry with CZ > 0).
// N = 36 and 72 are the padded grids of the dealiased form at N = 24 and 48 only.
constexpr int kTilesF32[][3] = {{16, 1, 1}, {16, 2, 1}, {16, 1, 2}, {24, 3, 1}, {24, 3, 2}, {24, 3, 4}, {24, 3, 3},
                                {24, 1, 1}, {32, 2, 0}, {32, 2, 1}, {32, 4, 1}, {32, 4, 2}, {48, 6, 2}, {48, 12, 4},
                                {48, 12, 2}, {48, 12, 1}, {48, 12, 3}, {64, 16, 4}, {36, 3, 2}, {72, 24, 4}};
constexpr int kTilesF64[][3] = {{16, 1, 1}, {24, 3, 2}, {32, 4, 2}, {48, 12, 4}, {64, 32, 8}, {36, 6, 4},
                                {72, 72, 8}};

}  // namespace

int tile_candidates(int N, int precision, GainGeometry* out, int max) {
    int n = 0;
    auto scan = [&](const auto& tab) {
        for (const auto& t : tab)
            if (t[0] == N && n < max) out[n++] = GainGeometry{t[1], t[2]};
    };
    if (precision == DGFS_FP64) scan(kTilesF64);
    else scan(kTilesF32);
    return n;
}

bool gain_geometry(int N, int precision, GainGeometry* g, bool matrix_ok) {
    GainGeometry cand[16];
    const int n = tile_candidates(N, precision, cand, 16);
    for (int k = 0; k < n; ++k)
        if (cand[k].CZ != 0 || matrix_ok) {
            *g = cand[k];
            return true;
        }
    return false;
}

hipError_t launch_collide(const dgfs_plan& p, const void* f, void* Q, int64_t nb, void* ws, bool pairs,
                          hipStream_t st, hipEvent_t* ev) {
    if (p.inner) {
        switch (p.N) {
            case 16: return run_dealias_16(p, *p.inner, f, Q, int(nb), ws, pairs, st, ev);
            case 24: return run_dealias_24(p, *p.inner, f, Q, int(nb), ws, pairs, st, ev);
            case 32: return run_dealias_32(p, *p.inner, f, Q, int(nb), ws, pairs, st, ev);
            case 48: return run_dealias_48(p, *p.inner, f, Q, int(nb), ws, pairs, st, ev);
            default: return hipErrorInvalidValue;
        }
    }
    if (p.vss) {
        switch (p.N) {
            case 16: return run_vss_16(p, f, Q, int(nb), ws, pairs, st, ev);
            case 24: return run_vss_24(p, f, Q, int(nb), ws, pairs, st, ev);
            case 32: return run_vss_32(p, f, Q, int(nb), ws, pairs, st, ev);
            case 48: return run_vss_48(p, f, Q, int(nb), ws, pairs, st, ev);
            default: return hipErrorInvalidValue;
        }
    }
    switch (p.N) {
        case 16: return run_tiles_16(p, f, Q, int(nb), ws, pairs, st, ev);
        case 24: return run_tiles_24(p, f, Q, int(nb), ws, pairs, st, ev);
        case 32: return run_tiles_32(p, f, Q, int(nb), ws, pairs, st, ev);
        case 48: return run_tiles_48(p, f, Q, int(nb), ws, pairs, st, ev);
        case 64: return run_tiles_64(p, f, Q, int(nb), ws, pairs, st, ev);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_conserve(const dgfs_plan& p, const void* Q, double* out, void* fstate, double dt, int64_t nb,
                           hipStream_t st) {
    const char* dev = static_cast<const char*>(p.dev);
    const double* minv = reinterpret_cast<const double*>(dev + p.off_minv);
    const double* mass = minv + (p.s + 4) * (p.s + 4);
    const double* Ls = mass + p.s;
    const dim3 grid(static_cast<unsigned>(nb)), block(1024);
    auto run = [&](auto tin, auto nc) {
        using TIN = decltype(tin);
        constexpr int NC = decltype(nc)::value;
        if (fstate)
            conserve_kernel<TIN, true, NC><<<grid, block, 0, st>>>(static_cast<const TIN*>(Q), nullptr,
                                                                   static_cast<TIN*>(fstate), dt, minv, mass, Ls,
                                                                   p.s, p.N);
        else
            conserve_kernel<TIN, false, NC><<<grid, block, 0, st>>>(static_cast<const TIN*>(Q), out, nullptr, 0.0,
                                                                    minv, mass, Ls, p.s, p.N);
    };
    auto by_n = [&](auto tin) {
        switch (p.N) {
            case 16: run(tin, std::integral_constant<int, 16>{}); break;
            case 24: run(tin, std::integral_constant<int, 24>{}); break;
            case 32: run(tin, std::integral_constant<int, 32>{}); break;
            case 48: run(tin, std::integral_constant<int, 48>{}); break;
            case 64: run(tin, std::integral_constant<int, 64>{}); break;
            default: run(tin, std::integral_constant<int, 0>{}); break;
        }
    };
    if (p.precision == DGFS_FP64) by_n(double{});
    else by_n(float{});
    return hipGetLastError();
}

hipError_t launch_axpby(const dgfs_plan& p, const void* x, const void* y, void* out, double a, double b, int64_t n,
                        hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const dim3 grid(static_cast<unsigned>((n + 255) / 256)), block(256);
    if (p.precision == DGFS_FP64)
        axpby_kernel<double><<<grid, block, 0, st>>>(static_cast<const double*>(x), static_cast<const double*>(y),
                                                      static_cast<double*>(out), a, b, n);
    else
        axpby_kernel<float><<<grid, block, 0, st>>>(static_cast<const float*>(x), static_cast<const float*>(y),
                                                     static_cast<float*>(out), float(a), float(b), n);
    return hipGetLastError();
}

}  // namespace dgfs
