// The dealiased (linear-convolution) form of eq. (sum): l + m = k with l, m, k all in
// [-N/2, N/2-1]^3, no wrap-around.  The spectra are zero-padded to NI = 3N/2 (l + m then
// never wraps onto a kept mode), the gain runs on the NI grid with the whole complex
// product kept (the padded spectrum is not Hermitian, so its shifted fields come from
// unpaired transforms), the loss product f nu is taken on the NI grid, and the kept modes
// are synthesised on the N grid, whose real part is the result.  Included by the vss_<NI>
// tile files, whose gain kernels keep the complex product.
#pragma once

#include "gain.hpp"

namespace dgfs {

template <int N>
__device__ __forceinline__ int mode_of(int idx) { return idx < N / 2 ? idx : idx - N; }

// fI[b][i] on the NI grid: the N-grid coefficients at their modes, zero elsewhere.
template <typename T, int N, int NI>
__global__ __launch_bounds__(256) void pad_kernel(const cx<T>* __restrict__ fN, cx<T>* __restrict__ fI,
                                                  int64_t nfields) {
    constexpr int64_t NI3 = int64_t(NI) * NI * NI, N3 = int64_t(N) * N * N;
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= nfields * NI3) return;
    const int64_t fld = t / NI3;
    const int e = int(t % NI3);
    const int mx = mode_of<NI>(e / (NI * NI)), my = mode_of<NI>((e / NI) % NI), mz = mode_of<NI>(e % NI);
    cx<T> v{T(0), T(0)};
    if (mx >= -N / 2 && mx < N / 2 && my >= -N / 2 && my < N / 2 && mz >= -N / 2 && mz < N / 2) {
        const int ix = (mx + N) % N, iy = (my + N) % N, iz = (mz + N) % N;
        v = fN[fld * N3 + (int64_t(ix) * N + iy) * N + iz];
    }
    fI[t] = v;
}

struct DealiasArgs {
    const void* P;       // [nb][ncls][nrho][CH][NI/CH][NI][NI] complex partials
    const void* fhatI;   // [nb][s][NI^3]
    void* G;             // [nb][nslots][N^3]  kept gain modes (N-grid index)
    void* nu;            // [nb][nslots][NI^3] loss spectrum G- f_hat^j summed over j
    const void* F;       // inner plan: [nftab][nrho][K2]
    const void* Gm;      // inner plan: [ngtab][K2]
    const void* tw;      // inner plan: [NI][CH]
    const int* slots;
    const int* gterms;
    const int* lterms;
    int s, ncls, nrho, nb, nslots, K2;
};

// Kept gain modes: one thread per (node, slot, N-grid mode k): the chunk partials at the
// NI index of k are combined and weighted with w_q F(|k|, rho_q) / NI^3, summed over
// radial points and classes in FP64.
template <typename T, int N, int NI, int CH>
__global__ __launch_bounds__(256) void dealias_gain_kernel(DealiasArgs a) {
    constexpr int NP = NI / CH;
    constexpr int64_t N3 = int64_t(N) * N * N, NI2 = int64_t(NI) * NI, PCHF = int64_t(NP) * NI2;
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= int64_t(a.nb) * a.nslots * N3) return;
    const int e = int(t % N3);
    const int64_t bs = t / N3;
    const int slot = int(bs % a.nslots);
    const int b = int(bs / a.nslots);
    const int mx = mode_of<N>(e / (N * N)), my = mode_of<N>((e / N) % N), mz = mode_of<N>(e % N);
    const int kx = (mx + NI) % NI, ky = (my + NI) % NI, kz = (mz + NI) % NI;
    const int kxp = kx % NP;
    const int k2 = mx * mx + my * my + mz * mz;
    const cx<T>* P = static_cast<const cx<T>*>(a.P);
    const T* F = static_cast<const T*>(a.F);
    const cx<T>* tw = static_cast<const cx<T>*>(a.tw);
    const int64_t eP = (int64_t(kxp) * NI + ky) * NI + kz;
    const int* sd = a.slots + 5 * slot;
    const int g0 = sd[1], ng = sd[2];
    double ax = 0.0, ay = 0.0;
    for (int gi = 0; gi < ng; ++gi) {
        const int cl = a.gterms[2 * (g0 + gi)], ft = a.gterms[2 * (g0 + gi) + 1];
        const T* Ft = F + int64_t(ft) * a.nrho * a.K2 + k2;
        for (int q = 0; q < a.nrho; ++q) {
            const cx<T>* Pb = P + ((int64_t(b) * a.ncls + cl) * a.nrho + q) * (CH * PCHF) + eP;
            cx<T> Z = Pb[0];
#pragma unroll
            for (int c = 1; c < CH; ++c) cmac(Z, tw[kx * CH + c], Pb[c * PCHF]);
            const double fq = double(Ft[int64_t(q) * a.K2]);
            ax = fma(fq, double(Z.x), ax);
            ay = fma(fq, double(Z.y), ay);
        }
    }
    static_cast<cx<T>*>(a.G)[t] = cx<T>{T(ax), T(ay)};
}

// Loss spectrum on the NI grid: nu[b][slot](k) = sum_j G-(|k|) f_hat^j(k).
template <typename T, int NI>
__global__ __launch_bounds__(256) void dealias_nu_kernel(DealiasArgs a) {
    constexpr int64_t NI3 = int64_t(NI) * NI * NI;
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= int64_t(a.nb) * a.nslots * NI3) return;
    const int e = int(t % NI3);
    const int64_t bs = t / NI3;
    const int slot = int(bs % a.nslots);
    const int b = int(bs / a.nslots);
    const int mx = mode_of<NI>(e / (NI * NI)), my = mode_of<NI>((e / NI) % NI), mz = mode_of<NI>(e % NI);
    const int k2 = mx * mx + my * my + mz * mz;
    const int* sd = a.slots + 5 * slot;
    const int l0 = sd[3], nl = sd[4];
    const cx<T>* fh = static_cast<const cx<T>*>(a.fhatI);
    const T* Gm = static_cast<const T*>(a.Gm);
    cx<T> acc{T(0), T(0)};
    for (int li = 0; li < nl; ++li) {
        const int sj = a.lterms[2 * (l0 + li)], gt = a.lterms[2 * (l0 + li) + 1];
        const T g = Gm[int64_t(gt) * a.K2 + k2];
        const cx<T> v = fh[(int64_t(b) * a.s + sj) * NI3 + e];
        acc.x = fma(g, v.x, acc.x);
        acc.y = fma(g, v.y, acc.y);
    }
    static_cast<cx<T>*>(a.nu)[t] = acc;
}

// nu[b][slot](x) *= f_I[b][species of slot](x) on the NI grid (both complex).
template <typename T, int NI>
__global__ __launch_bounds__(256) void dealias_product_kernel(cx<T>* __restrict__ nu, const cx<T>* __restrict__ fI,
                                                              const int* __restrict__ slots, int s, int nslots,
                                                              int nb) {
    constexpr int64_t NI3 = int64_t(NI) * NI * NI;
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= int64_t(nb) * nslots * NI3) return;
    const int64_t e = t % NI3;
    const int64_t bs = t / NI3;
    const int slot = int(bs % nslots);
    const int64_t b = bs / nslots;
    const cx<T> f = fI[(b * s + slots[5 * slot]) * NI3 + e];
    const cx<T> v = nu[t];
    nu[t] = cx<T>{f.x * v.x - f.y * v.y, f.x * v.y + f.y * v.x};
}

// G[b][slot](k) -= L(k) for the kept modes, L the loss coefficients on the NI grid.
template <typename T, int N, int NI>
__global__ __launch_bounds__(256) void dealias_subtract_kernel(cx<T>* __restrict__ G, const cx<T>* __restrict__ Lc,
                                                               int64_t nfields) {
    constexpr int64_t N3 = int64_t(N) * N * N, NI3 = int64_t(NI) * NI * NI;
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= nfields * N3) return;
    const int64_t fld = t / N3;
    const int e = int(t % N3);
    const int kx = (mode_of<N>(e / (N * N)) + NI) % NI, ky = (mode_of<N>((e / N) % N) + NI) % NI,
              kz = (mode_of<N>(e % N) + NI) % NI;
    const cx<T> l = Lc[fld * NI3 + (int64_t(kx) * NI + ky) * NI + kz];
    G[t] = cx<T>{G[t].x - l.x, G[t].y - l.y};
}

template <typename T>
__global__ __launch_bounds__(256) void real_part_kernel(const cx<T>* __restrict__ G, T* __restrict__ Q, int64_t n) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t < n) Q[t] = G[t].x;
}

namespace detail {

inline unsigned blocks_for(int64_t n) { return unsigned((n + 255) / 256); }

// outer: the N-grid plan (conservation tables, slots); inner: its NI = 3N/2 companion
// (phases, kernel-mode and loss tables, classes, slots of the NI grid).
template <typename T, int N, int CH, int CZ, bool PIPE>
hipError_t run_dealiased(const dgfs_plan& outer, const dgfs_plan& inner, const T* f, T* Q, int nb, void* ws,
                         bool pairs, hipStream_t st, hipEvent_t* ev) {
    constexpr int NI = 3 * N / 2;
    constexpr int64_t N3 = int64_t(N) * N * N, NI3 = int64_t(NI) * NI * NI;
    auto mark = [&](int k) {
        if (ev) hipEventRecord(ev[k], st);
    };
    const SlotSet& ss = pairs ? inner.pair_slots : inner.sum_slots;
    const int s = outer.s, ncls = int(inner.classes.size());
    char* w = static_cast<char*>(ws);
    auto carve = [&](int64_t count) {
        cx<T>* p = reinterpret_cast<cx<T>*>(w);
        w += align256(sizeof(cx<T>) * count);
        return p;
    };
    cx<T>* fN = carve(int64_t(nb) * s * N3);
    cx<T>* fhI = carve(int64_t(nb) * s * NI3);
    cx<T>* fI = carve(int64_t(nb) * s * NI3);
    cx<T>* P = carve(int64_t(nb) * ncls * inner.nrho * NI3);
    cx<T>* nu = carve(int64_t(nb) * ss.nslots * NI3);
    cx<T>* G = carve(int64_t(nb) * ss.nslots * N3);
    const char* dev = static_cast<const char*>(inner.dev);
    hipError_t e;

    mark(0);
    if ((e = fft3d<T, N>(fN, f, int64_t(nb) * s, -1, T(1.0 / double(N3)), st)) != hipSuccess) return e;
    pad_kernel<T, N, NI><<<blocks_for(int64_t(nb) * s * NI3), 256, 0, st>>>(fN, fhI, int64_t(nb) * s);
    if ((e = hipMemcpyAsync(fI, fhI, sizeof(cx<T>) * nb * s * NI3, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return e;
    if ((e = fft3d<T, NI>(fI, nullptr, int64_t(nb) * s, +1, T(1), st)) != hipSuccess) return e;
    mark(1);

    // the gain over the padded spectra with the NI-grid plan's classes
    GainArgs<T> ga;
    ga.fhat = fhI;
    ga.P = P;
    ga.PL = nullptr;
    ga.kx = reinterpret_cast<const cx<T>*>(dev + inner.off_kx);
    ga.yz = reinterpret_cast<const cx<T>*>(dev + inner.off_yz);
    ga.nyq = reinterpret_cast<const T*>(dev + inner.off_nyq);
    ga.cls = reinterpret_cast<const int*>(dev + inner.off_cls);
    ga.wdir = reinterpret_cast<const T*>(dev + inner.off_wdir);
    ga.s = s;
    ga.ncls = ncls;
    ga.nrho = inner.nrho;
    ga.nb = nb;
    const int64_t groups = ((nb + 7) / 8) * 8 * int64_t(ncls) * inner.nrho * CH;
    gain_kernel<T, NI, CH, CZ, PIPE, false, GAIN_COMPLEX>
        <<<dim3(unsigned(groups)), dim3(GainK<T, NI, CH, CZ>::NT), 0, st>>>(ga);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    mark(2);

    DealiasArgs da;
    da.P = P;
    da.fhatI = fhI;
    da.G = G;
    da.nu = nu;
    da.F = dev + inner.off_F;
    da.Gm = dev + inner.off_G;
    da.tw = dev + inner.off_tw;
    da.slots = reinterpret_cast<const int*>(dev + ss.off_slots);
    da.gterms = reinterpret_cast<const int*>(dev + ss.off_gterms);
    da.lterms = reinterpret_cast<const int*>(dev + ss.off_lterms);
    da.s = s;
    da.ncls = ncls;
    da.nrho = inner.nrho;
    da.nb = nb;
    da.nslots = ss.nslots;
    da.K2 = inner.K2;
    dealias_gain_kernel<T, N, NI, CH><<<blocks_for(int64_t(nb) * ss.nslots * N3), 256, 0, st>>>(da);
    dealias_nu_kernel<T, NI><<<blocks_for(int64_t(nb) * ss.nslots * NI3), 256, 0, st>>>(da);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    mark(3);

    // loss: nu on the NI grid, times the interpolant f_I, back to coefficients, kept modes
    if ((e = fft3d<T, NI>(nu, nullptr, int64_t(nb) * ss.nslots, +1, T(1), st)) != hipSuccess) return e;
    dealias_product_kernel<T, NI><<<blocks_for(int64_t(nb) * ss.nslots * NI3), 256, 0, st>>>(nu, fI, da.slots, s,
                                                                                           ss.nslots, nb);
    if ((e = fft3d<T, NI>(nu, nullptr, int64_t(nb) * ss.nslots, -1, T(1.0 / double(NI3)), st)) != hipSuccess) return e;
    dealias_subtract_kernel<T, N, NI><<<blocks_for(int64_t(nb) * ss.nslots * N3), 256, 0, st>>>(
        G, nu, int64_t(nb) * ss.nslots);
    if ((e = fft3d<T, N>(G, nullptr, int64_t(nb) * ss.nslots, +1, T(1), st)) != hipSuccess) return e;
    mark(4);
    real_part_kernel<T><<<blocks_for(int64_t(nb) * ss.nslots * N3), 256, 0, st>>>(G, Q, int64_t(nb) * ss.nslots * N3);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    mark(5);
    return hipSuccess;
}

}  // namespace detail
}  // namespace dgfs
