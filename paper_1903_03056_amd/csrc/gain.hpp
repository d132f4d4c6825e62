// The fused gain kernel, the radial-sum/loss kernel, the combination kernel and the
// launch sequence of one batch slice, as templates over (precision, N, tile).  Each
// tiles_<N>.hip instantiates them for one N.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fft.hpp"
#include "passes.hpp"
#include "plan.hpp"

namespace dgfs {

// ================================================================ gain kernel
// Geometry of one work item: the x-chunk c (x-indices = c mod CH, NP = N/CH of them)
// of one S_q field.  Each y/z pencil of the chunk is shared by CZ thread groups: group
// cz keeps the outputs with index = cz mod CZ (decimation in frequency), so a thread
// holds NS = N/CZ values per field.  The group index is uniform per wavefront
// (NTC = NP*N is a multiple of 64), so every twiddle is a compile-time constant.
template <typename T, int N, int CH, int CZ>
struct GainK {
    static constexpr int NP = N / CH;
    static constexpr int NS = N / CZ;
    static constexpr int NTC = NP * N;
    static constexpr int NT = NTC * CZ;
    static constexpr int KZH = N / 2 + 1;               // stored k_z of a partial (Hermitian half)
    static constexpr int NPEN = N * KZH;                // stored (k_y, k_z) pencils of a partial
    static constexpr int PX = (NPEN + NT - 1) / NT;     // stored pencils per thread (guarded)
    static constexpr int ROW = N + 1;                  // padded LDS row (bank spread)
    static constexpr int LDS = NP * N * ROW;
    static_assert(NP * CH == N && NS * CZ == N, "CH and CZ must divide N");
    static_assert(NTC % 64 == 0, "a CZ group must be whole wavefronts");
};

template <typename T>
struct GainArgs {
    const cx<T>* fhat;  // [nb][s][N^3], DFT / N^3
    cx<T>* P;           // [nb][ncls][nrho][CH][N/CH][N][N/2+1]  (k_z <= N/2 of each partial)
    const cx<T>* kx;    // [dirs][nrho][2][CH][N]  x-phase merged with the chunk split
    const cx<T>* yz;    // [dirs][nrho][2][2][N]   y- and z-phases
    const T* nyq;       // [dirs][nrho][2]         2 sin(theta_x N / 2) of the x-phase
    const int* cls;     // [ncls][4] = i, j, ndir, dir_offset
    const T* wdir;      // [ncls]
    int s, ncls, nrho, nb;
};

// out[j] = X[CZ j + CZI] of the length-N DFT (sign SIGN) of the sequence
// x[n] = src[n * stride]: the CZ strided input sub-sequences are combined with the
// split factors e^{SIGN 2 pi i t CZI / CZ}, twiddled by e^{SIGN 2 pi i l CZI / N},
// then transformed with an N/CZ-point FFT.
template <int N, int CZ, int CZI, int SIGN, int STRIDE, typename T>
__device__ __forceinline__ void split_fft(const cx<T>* src, cx<T>* out) {
    constexpr int NS = N / CZ;
    static_for<0, NS>([&](auto l) {
        cx<T> acc = src[l * STRIDE];
        static_for<1, CZ>([&](auto t) {
            constexpr long k = long(decltype(t)::value) * CZI;
            acc = acc + rot<SIGN, k, CZ>(src[(l + t * NS) * STRIDE]);
        });
        out[l] = rot<SIGN, long(decltype(l)::value) * CZI, long(N)>(acc);
        // keep at most a few loads in flight: the pencil's inputs are combined as they
        // arrive instead of all being held in registers at once
        if constexpr (decltype(l)::value % 4 == 3) __builtin_amdgcn_sched_barrier(0);
    });
    fft<NS, SIGN>(out);
}

// Call f(integral_constant<int, cz>) for the runtime (wave-uniform) group index cz.
template <int CZ, typename F>
__device__ __forceinline__ void with_group(int cz, F&& f) {
    if constexpr (CZ == 1) {
        f(std::integral_constant<int, 0>{});
    } else {
        static_for<0, CZ>([&](auto g) {
            if (cz == decltype(g)::value) f(g);
        });
    }
}

// y-pass (through LDS, in place on columns) and z-pass (rows, result kept) of one
// field whose x-pass output is in buf; out[j] = value at z-index CZ j + cz of the
// thread's pencil (m, r).
template <typename T, int N, int CH, int CZ, int SIGN>
__device__ __forceinline__ void yz_passes(cx<T>* buf, int cz, int m, int r, cx<T>* out) {
    using K = GainK<T, N, CH, CZ>;
    cx<T> v[K::NS];
    with_group<CZ>(cz, [&](auto g) {
        split_fft<N, CZ, decltype(g)::value, SIGN, K::ROW>(buf + (m * N) * K::ROW + r, v);
    });
    __syncthreads();
#pragma unroll
    for (int j = 0; j < K::NS; ++j) buf[(m * N + CZ * j + cz) * K::ROW + r] = v[j];
    __syncthreads();
    with_group<CZ>(cz, [&](auto g) {
        split_fft<N, CZ, decltype(g)::value, SIGN, 1>(buf + (m * N + r) * K::ROW, out);
    });
}

// Buffer loads: a wave-uniform base in the resource descriptor, the lane's byte offset
// in a VGPR and a uniform byte offset in an SGPR, so the strided x-pass loads need no
// per-lane 64-bit address arithmetic.  Offsets beyond the descriptor's range read 0.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t field_rsrc(const cx<T>* base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<cx<T>*>(base), 0, bytes, 0x00020000);
}

template <typename T>
__device__ __forceinline__ cx<T> bload(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    } else {
        return __builtin_bit_cast(cx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    }
}

// Work slots of the x-pass.  The Hermitian pairs P = (l_y, l_z) <-> -P (mod N) by a
// representative: rows 1..N/2-1 with all l_z, then rows 0 and N/2 with l_z in
// 1..N/2-1.  The four self-paired pencils (P = -P) follow: with SELF, as two slots that
// each take (l_y, 0) and (l_y, N/2) for l_y = 0 and l_y = N/2 (N^2/2 slots in all);
// otherwise one slot each (N^2/2 + 2 slots).  Returns false for a self-paired slot.
template <int N, bool SELF>
__device__ __forceinline__ bool pencil_slot(int slot, int& ly, int& lz) {
    constexpr int H = N / 2;
    constexpr int RA = (H - 1) * N;
    if (slot < RA) {
        ly = 1 + slot / N;
        lz = slot % N;
        return true;
    }
    const int t = slot - RA;
    if (t < 2 * (H - 1)) {
        ly = t < H - 1 ? 0 : H;
        lz = 1 + t % (H - 1);
        return true;
    }
    const int u = t - 2 * (H - 1);
    if constexpr (SELF) {
        ly = u * H;
        lz = 0;
    } else {
        ly = (u >> 1) * H;
        lz = (u & 1) * H;
    }
    return false;
}

// Chunk c of IDFT(f_hat * phase) for one shifted field: out[j] at (x = CH m + c,
// y = r, z = CZ j + cz).  The x-pass reads the spectrum from global memory (coalesced
// over (l_y, l_z)) and keeps only the chunk's x-outputs: the CH strided input
// sub-sequences are combined with kxt, which carries the x-phase, the split factor
// e^{2 pi i t c / CH} and the twiddle e^{2 pi i l c / N}.  The y- and z-phases are
// constant along an x-pencil and multiply its outputs.  With PIPE the loads of the
// next sub-sequence are issued before the current one is combined.
//
// f is real, so f_hat(l_x, -P) = conj(f_hat(-l_x, P)); with the linear x-phase this
// gives, for every output x-index n, G(-P)[n] = conj(G(P)[n] + delta_P (-1)^n) where
// delta_P = f_hat(N/2, P) (e^{i theta N/2} - e^{-i theta N/2}) accounts for the DFT
// index N/2 standing for the mode -N/2 on both sides.  So only one pencil of each pair
// is transformed; its partner costs a conjugate, one correction and its own y/z phase.
//
// A self-paired pencil obeys the same relation with itself: its x-output is
// a - i d (-1)^n / 2 with a real and d = f_hat(N/2, P) 2 sin(theta N/2) (f_hat(N/2, P) is
// real there).  With SELF two of them, P1 and P2, go through one transform of
// f_hat(., P1) + i f_hat(., P2), whose output (a1 - b2) + i (b1 + a2) (b = -d (-1)^n / 2)
// gives both.  That removes a round of the pass when N^2/2 + 2 slots would need one
// more than N^2/2; only the wavefront holding those two slots loads two pencils.
template <typename T, int N, int CH, int CZ, bool PIPE>
__device__ __forceinline__ void field_ifft(const cx<T>* __restrict__ fh, const cx<T>* __restrict__ kxt,
                                           const cx<T>* __restrict__ yzt, T nyq, int c, cx<T>* buf, int cz,
                                           int m, int r, cx<T>* out) {
    using K = GainK<T, N, CH, CZ>;
    constexpr int ROUNDS_ALL = (N * N / 2 + 2 + K::NT - 1) / K::NT;
    constexpr int ROUNDS_SELF = (N * N / 2 + K::NT - 1) / K::NT;
    constexpr bool SELF = ROUNDS_SELF < ROUNDS_ALL;
    constexpr int SLOTS = SELF ? N * N / 2 : N * N / 2 + 2;
    constexpr int ROUNDS = SELF ? ROUNDS_SELF : ROUNDS_ALL;
    constexpr int ES = int(sizeof(cx<T>));
    constexpr int RS = N * N * ES;  // bytes between x-planes of the spectrum
    const __amdgpu_buffer_rsrc_t rs = field_rsrc<T>(fh, N * RS);
    const int tid = threadIdx.x;
    // runtime loops keep the x-pass loads from being hoisted en masse
#pragma unroll 1
    for (int k = 0; k < ROUNDS; ++k) {
        const int slot = tid + k * K::NT;
        if (ROUNDS * K::NT != SLOTS && slot >= SLOTS) break;
        int ly, lz;
        const bool paired = pencil_slot<N, SELF>(slot, ly, lz);
        const int P = ly * N + lz;
        const int vo = P * ES;
        cx<T> y[K::NP];
#pragma unroll
        for (int l = 0; l < K::NP; ++l) y[l] = cx<T>{T(0), T(0)};
        if (SELF && __ballot(!paired) != 0) {
            // f(., P1) + i mk f(., P2) with both loads of an index issued together
            const int vo2 = paired ? vo : vo + (N / 2) * ES;
            const T mk = paired ? T(0) : T(1);
#pragma unroll 1
            for (int t = 0; t < CH; ++t) {
                cx<T> a[K::NP], b[K::NP];
#pragma unroll
                for (int l = 0; l < K::NP; ++l) {
                    a[l] = bload<T>(rs, vo, (l + t * K::NP) * RS);
                    b[l] = bload<T>(rs, vo2, (l + t * K::NP) * RS);
                }
#pragma unroll
                for (int l = 0; l < K::NP; ++l)
                    cmac(y[l], cx<T>{a[l].x - mk * b[l].y, a[l].y + mk * b[l].x}, kxt[l + t * K::NP]);
            }
        } else if constexpr (PIPE) {
            cx<T> nxt[K::NP];
#pragma unroll
            for (int l = 0; l < K::NP; ++l) nxt[l] = bload<T>(rs, vo, l * RS);
#pragma unroll 1
            for (int t = 0; t < CH; ++t) {
                cx<T> cur[K::NP];
#pragma unroll
                for (int l = 0; l < K::NP; ++l) cur[l] = nxt[l];
                if (t + 1 < CH) {
#pragma unroll
                    for (int l = 0; l < K::NP; ++l) nxt[l] = bload<T>(rs, vo, (l + (t + 1) * K::NP) * RS);
                }
#pragma unroll
                for (int l = 0; l < K::NP; ++l) cmac(y[l], cur[l], kxt[l + t * K::NP]);
            }
        } else {
#pragma unroll 1
            for (int t = 0; t < CH; ++t) {
#pragma unroll
                for (int l = 0; l < K::NP; ++l) {
                    const int jx = l + t * K::NP;
                    cmac(y[l], bload<T>(rs, vo, jx * RS), kxt[jx]);
                }
            }
        }
        fft<K::NP, +1>(y);
        const cx<T> fn = bload<T>(rs, vo, (N / 2) * RS);
        if (SELF && !paired) {
            const T h1 = T(0.5) * nyq * fn.x;
            const T h2 = T(0.5) * nyq * bload<T>(rs, vo + (N / 2) * ES, (N / 2) * RS).x;
            const cx<T> c1 = yzt[ly] * yzt[N], c2 = yzt[ly] * yzt[N + N / 2];
#pragma unroll
            for (int mm = 0; mm < K::NP; ++mm) {
                const bool odd = ((CH * mm + c) & 1) != 0;
                const T e1 = odd ? -h1 : h1, e2 = odd ? -h2 : h2;  // d (-1)^n / 2
                buf[(mm * N + ly) * K::ROW] = cx<T>{y[mm].x - e2, -e1} * c1;
                buf[(mm * N + ly) * K::ROW + N / 2] = cx<T>{y[mm].y + e1, -e2} * c2;
            }
            continue;
        }
        const cx<T> cyz = yzt[ly] * yzt[N + lz];
#pragma unroll
        for (int mm = 0; mm < K::NP; ++mm) buf[(mm * N + ly) * K::ROW + lz] = y[mm] * cyz;
        if (paired) {
            const int ly2 = (N - ly) % N, lz2 = (N - lz) % N;
            const cx<T> delta = cx<T>{-nyq * fn.y, nyq * fn.x};
            const cx<T> cyz2 = yzt[ly2] * yzt[N + lz2];
#pragma unroll
            for (int mm = 0; mm < K::NP; ++mm) {
                const bool odd = ((CH * mm + c) & 1) != 0;
                const cx<T> g = odd ? y[mm] - delta : y[mm] + delta;
                buf[(mm * N + ly2) * K::ROW + lz2] = cx<T>{g.x, -g.y} * cyz2;
            }
        }
    }
    __syncthreads();
    yz_passes<T, N, CH, CZ, +1>(buf, cz, m, r, out);
    __syncthreads();
}

template <typename T, int N, int CH, int CZ, bool PIPE>
__global__ __launch_bounds__((GainK<T, N, CH, CZ>::NT)) void gain_kernel(GainArgs<T> a) {
    using K = GainK<T, N, CH, CZ>;
    __shared__ cx<T> buf[K::LDS];
    // Work items of one node are placed on one XCD (workgroups are dealt to the 8
    // XCDs round-robin), so that node's spectra stay in that XCD's L2.
    const int ipn = a.ncls * a.nrho * CH;
    const int g = blockIdx.x;
    const int xcd = g & 7, local = g >> 3;
    const int b = (local / ipn) * 8 + xcd;
    if (b >= a.nb) return;
    int item = local % ipn;
    const int c = item % CH;
    item /= CH;
    const int q = item % a.nrho;
    const int cl = item / a.nrho;
    const int ci = a.cls[4 * cl], cj = a.cls[4 * cl + 1];
    const int ndir = a.cls[4 * cl + 2], doff = a.cls[4 * cl + 3];
    const T w = a.wdir[cl];
    constexpr int64_t N3 = int64_t(N) * N * N;
    const cx<T>* fhi = a.fhat + (int64_t(b) * a.s + ci) * N3;
    const cx<T>* fhj = a.fhat + (int64_t(b) * a.s + cj) * N3;
    const int tid = threadIdx.x;
    const int cz = tid / K::NTC, u = tid % K::NTC;
    const int m = u / N, r = u % N;

    // Only Re(S_q) reaches the result: the radial operator multiplies DFT(S_q) by a
    // real F that is even in k, so Re IDFT(F DFT(S)) = IDFT(F DFT(Re S)).
    T S[K::NS];
#pragma unroll
    for (int n = 0; n < K::NS; ++n) S[n] = T(0);

    for (int d = 0; d < ndir; ++d) {
        const int64_t base = (int64_t(doff + d) * a.nrho + q) * 2;
        cx<T> A[K::NS], B[K::NS];
        field_ifft<T, N, CH, CZ, PIPE>(fhi, a.kx + ((base + 0) * CH + c) * N, a.yz + (base + 0) * 2 * N, a.nyq[base],
                                 c, buf, cz, m, r, A);
        field_ifft<T, N, CH, CZ, PIPE>(fhj, a.kx + ((base + 1) * CH + c) * N, a.yz + (base + 1) * 2 * N,
                                 a.nyq[base + 1], c, buf, cz, m, r, B);
#pragma unroll
        for (int n = 0; n < K::NS; ++n) S[n] = fma(w, fma(A[n].x, B[n].x, -A[n].y * B[n].y), S[n]);
    }

    // forward DFT of Re S_q: z and y through LDS, then the chunk's part of x
#pragma unroll
    for (int j = 0; j < K::NS; ++j) buf[(m * N + r) * K::ROW + CZ * j + cz] = cx<T>{S[j], T(0)};
    __syncthreads();
    {
        cx<T> v[K::NS];
        with_group<CZ>(cz, [&](auto gg) {
            split_fft<N, CZ, decltype(gg)::value, -1, 1>(buf + (m * N + r) * K::ROW, v);
        });
        __syncthreads();
#pragma unroll
        for (int j = 0; j < K::NS; ++j) buf[(m * N + r) * K::ROW + CZ * j + cz] = v[j];
        __syncthreads();
        with_group<CZ>(cz, [&](auto gg) {
            split_fft<N, CZ, decltype(gg)::value, -1, K::ROW>(buf + (m * N) * K::ROW + r, v);
        });
        __syncthreads();
#pragma unroll
        for (int j = 0; j < K::NS; ++j) buf[(m * N + CZ * j + cz) * K::ROW + r] = v[j];
        __syncthreads();
    }
    // The chunk's partial is the DFT of a real array over (x-planes of the chunk, y, z),
    // so it is Hermitian in (k_xp, k_y, k_z): only k_z <= N/2 is stored, the radial kernel
    // reads the rest as conjugates of the mirrored entries.
    constexpr int64_t PCH = int64_t(K::NP) * K::NPEN;  // stored values of one chunk partial
    cx<T>* Pout = a.P + ((int64_t(b) * a.ncls + cl) * a.nrho + q) * (CH * PCH) + int64_t(c) * PCH;
#pragma unroll 1
    for (int k = 0; k < K::PX; ++k) {
        const int P = tid + k * K::NT;
        if (K::PX * K::NT != K::NPEN && P >= K::NPEN) break;
        const int ky = P / K::KZH, kz = P % K::KZH;
        cx<T> v[K::NP];
#pragma unroll
        for (int mm = 0; mm < K::NP; ++mm) v[mm] = buf[(mm * N + ky) * K::ROW + kz];
        fft<K::NP, -1>(v);
#pragma unroll
        for (int kk = 0; kk < K::NP; ++kk) Pout[kk * K::NPEN + P] = v[kk];
    }
}

// =============================================================== radial kernel
template <typename T>
struct RadialArgs {
    const cx<T>* P;
    const cx<T>* fhat;
    cx<T>* Gt;          // [nb][nslots][N^3]
    cx<T>* Lt;          // [nb][nslots][N^3]
    const T* F;         // [nftab][nrho][K2]  w_q F(|k|, rho_q) / N^3
    const T* G;         // [ngtab][K2]        G-(|k|)
    const cx<T>* tw;    // [N][CH]  e^{-2 pi i kx c / N}
    const int* slots;   // [nslots][5]
    const int* gterms;  // [..][2]
    const int* lterms;  // [..][2]
    int s, ncls, nrho, nb, nslots, K2;
};

// One thread per Hermitian pair {k, -k} of the output spectrum: it takes the
// representative with k_z <= N/2 (the stored half of the partials), forms
// Q_hat+(k) = sum_terms sum_q w_q F(|k|, rho_q)/N^3 DFT(S_q)(k) and the loss spectrum
// L(k) = sum_j G-(|k|) f_hat^j(k) for the CH x-modes k_x = k_xp + j N/CH, and writes
// both at k and their conjugates at -k (S_q and f are real, F and G- are real and even
// in k).  Pairs with k_z = 0 or N/2 lie wholly in the stored half and are written once.
template <typename T, int N, int CH>
__global__ __launch_bounds__(256) void radial_kernel(RadialArgs<T> a) {
    constexpr int NP = N / CH;
    constexpr int KZH = N / 2 + 1;
    constexpr int64_t N2 = int64_t(N) * N, N3 = N2 * N, PCH = int64_t(NP) * N * KZH;
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= int64_t(a.nb) * a.nslots * PCH) return;
    const int e = int(t % PCH);
    const int64_t bs = t / PCH;
    const int slot = int(bs % a.nslots);
    const int b = int(bs / a.nslots);
    const int kz = e % KZH, ky = (e / KZH) % N, kxp = e / (N * KZH);
    auto sq = [](int k) {
        const int mk = k < N / 2 ? k : k - N;
        return mk * mk;
    };
    const int kyz2 = sq(ky) + sq(kz);
    int k2[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) k2[j] = sq(kxp + j * NP) + kyz2;
    const int* sd = a.slots + 5 * slot;
    const int g0 = sd[1], ng = sd[2], l0 = sd[3], nl = sd[4];

    cx<T> acc[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) acc[j] = cx<T>{T(0), T(0)};
    for (int gi = 0; gi < ng; ++gi) {
        const int cl = a.gterms[2 * (g0 + gi)], ft = a.gterms[2 * (g0 + gi) + 1];
        const cx<T>* Pb = a.P + (int64_t(b) * a.ncls + cl) * a.nrho * (CH * PCH) + e;
        const T* Ft = a.F + int64_t(ft) * a.nrho * a.K2;
        for (int q = 0; q < a.nrho; ++q) {
            cx<T> pc[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) pc[c] = Pb[int64_t(q) * (CH * PCH) + c * PCH];
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int kx = kxp + j * NP;
                cx<T> Sk = pc[0];
#pragma unroll
                for (int c = 1; c < CH; ++c) cmac(Sk, a.tw[kx * CH + c], pc[c]);
                const T fq = Ft[q * a.K2 + k2[j]];
                acc[j].x = fma(fq, Sk.x, acc[j].x);
                acc[j].y = fma(fq, Sk.y, acc[j].y);
            }
        }
    }
    cx<T> lac[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) lac[j] = cx<T>{T(0), T(0)};
    for (int li = 0; li < nl; ++li) {
        const int sj = a.lterms[2 * (l0 + li)], gt = a.lterms[2 * (l0 + li) + 1];
        const cx<T>* fj = a.fhat + (int64_t(b) * a.s + sj) * N3 + ky * N + kz;
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int kx = kxp + j * NP;
            const T gm = a.G[int64_t(gt) * a.K2 + k2[j]];
            const cx<T> v = fj[kx * N2];
            lac[j].x = fma(gm, v.x, lac[j].x);
            lac[j].y = fma(gm, v.y, lac[j].y);
        }
    }
    const int64_t ob = (int64_t(b) * a.nslots + slot) * N3;
    const bool mirror = kz != 0 && kz != N / 2;
    const int ky2 = (N - ky) % N, kz2 = (N - kz) % N;
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        const int kx = kxp + j * NP;
        const int64_t o = ob + kx * N2 + ky * N + kz;
        a.Gt[o] = acc[j];
        a.Lt[o] = lac[j];
        if (mirror) {
            const int64_t o2 = ob + ((N - kx) % N) * N2 + ky2 * N + kz2;
            a.Gt[o2] = cx<T>{acc[j].x, -acc[j].y};
            a.Lt[o2] = cx<T>{lac[j].x, -lac[j].y};
        }
    }
}

// ============================================================ combine kernel
template <typename T>
__global__ __launch_bounds__(256) void combine_kernel(const cx<T>* __restrict__ Gt, const cx<T>* __restrict__ Lt,
                                                      const T* __restrict__ f, T* __restrict__ Q,
                                                      const int* __restrict__ slots, int nslots, int s,
                                                      int64_t n3, int64_t total) {
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= total) return;
    const int64_t n = t % n3;
    const int64_t bs = t / n3;
    const int slot = int(bs % nslots);
    const int64_t b = bs / nslots;
    const int sp = slots[5 * slot];
    Q[t] = Gt[t].x - f[(b * s + sp) * n3 + n] * Lt[t].x;
}

namespace detail {

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ev (optional): 6 events recorded at the stage boundaries (start, after forward FFT,
// after gain, after radial, after inverse FFTs, after combine).
template <typename T, int N, int CH, int CZ, bool PIPE>
hipError_t run_slice(const dgfs_plan& p, const T* f, T* Q, int nb, void* ws, bool pairs, hipStream_t st,
                     hipEvent_t* ev) {
    auto mark = [&](int k) {
        if (ev) hipEventRecord(ev[k], st);
    };
    const SlotSet& ss = pairs ? p.pair_slots : p.sum_slots;
    constexpr int64_t N3 = int64_t(N) * N * N;
    const int ncls = int(p.classes.size());
    char* w = static_cast<char*>(ws);
    cx<T>* fhat = reinterpret_cast<cx<T>*>(w);
    w += align256(sizeof(cx<T>) * nb * p.s * N3);
    cx<T>* P = reinterpret_cast<cx<T>*>(w);
    w += align256(sizeof(cx<T>) * int64_t(nb) * ncls * p.nrho * (N3 / N) * (N / 2 + 1));
    cx<T>* Gt = reinterpret_cast<cx<T>*>(w);
    cx<T>* Lt = Gt + int64_t(nb) * ss.nslots * N3;  // contiguous with Gt

    const char* dev = static_cast<const char*>(p.dev);
    mark(0);
    hipError_t e = fft3d<T, N>(fhat, f, int64_t(nb) * p.s, -1, T(1.0 / double(N3)), st);
    if (e != hipSuccess) return e;
    mark(1);

    GainArgs<T> ga;
    ga.fhat = fhat;
    ga.P = P;
    ga.kx = reinterpret_cast<const cx<T>*>(dev + p.off_kx);
    ga.yz = reinterpret_cast<const cx<T>*>(dev + p.off_yz);
    ga.nyq = reinterpret_cast<const T*>(dev + p.off_nyq);
    ga.cls = reinterpret_cast<const int*>(dev + p.off_cls);
    ga.wdir = reinterpret_cast<const T*>(dev + p.off_wdir);
    ga.s = p.s;
    ga.ncls = ncls;
    ga.nrho = p.nrho;
    ga.nb = nb;
    const int64_t ipn = int64_t(ncls) * p.nrho * CH;
    const int64_t groups = ((nb + 7) / 8) * 8 * ipn;
    gain_kernel<T, N, CH, CZ, PIPE><<<dim3(unsigned(groups)), dim3(GainK<T, N, CH, CZ>::NT), 0, st>>>(ga);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    mark(2);

    RadialArgs<T> ra;
    ra.P = P;
    ra.fhat = fhat;
    ra.Gt = Gt;
    ra.Lt = Lt;
    ra.F = reinterpret_cast<const T*>(dev + p.off_F);
    ra.G = reinterpret_cast<const T*>(dev + p.off_G);
    ra.tw = reinterpret_cast<const cx<T>*>(dev + p.off_tw);
    ra.slots = reinterpret_cast<const int*>(dev + ss.off_slots);
    ra.gterms = reinterpret_cast<const int*>(dev + ss.off_gterms);
    ra.lterms = reinterpret_cast<const int*>(dev + ss.off_lterms);
    ra.s = p.s;
    ra.ncls = ncls;
    ra.nrho = p.nrho;
    ra.nb = nb;
    ra.nslots = ss.nslots;
    ra.K2 = p.K2;
    const int64_t rthreads = int64_t(nb) * ss.nslots * (N / CH) * N * (N / 2 + 1);
    radial_kernel<T, N, CH><<<dim3(unsigned((rthreads + 255) / 256)), dim3(256), 0, st>>>(ra);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    mark(3);

    e = fft3d<T, N>(Gt, nullptr, 2 * int64_t(nb) * ss.nslots, +1, T(1), st);
    if (e != hipSuccess) return e;
    mark(4);

    const int64_t total = int64_t(nb) * ss.nslots * N3;
    combine_kernel<T><<<dim3(unsigned((total + 255) / 256)), dim3(256), 0, st>>>(
        Gt, Lt, f, Q, ra.slots, ss.nslots, p.s, N3, total);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    mark(5);
    return hipSuccess;
}

}  // namespace detail

// Per-N entry points (tiles_<N>.hip): run one slice with the plan's tile geometry.
hipError_t run_tiles_16(const dgfs_plan& p, const void* f, void* Q, int nb, void* ws, bool pairs, hipStream_t st,
                        hipEvent_t* ev);
hipError_t run_tiles_24(const dgfs_plan& p, const void* f, void* Q, int nb, void* ws, bool pairs, hipStream_t st,
                        hipEvent_t* ev);
hipError_t run_tiles_32(const dgfs_plan& p, const void* f, void* Q, int nb, void* ws, bool pairs, hipStream_t st,
                        hipEvent_t* ev);
hipError_t run_tiles_48(const dgfs_plan& p, const void* f, void* Q, int nb, void* ws, bool pairs, hipStream_t st,
                        hipEvent_t* ev);

}  // namespace dgfs
