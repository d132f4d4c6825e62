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
// What a gain work item accumulates and stores:
// GAIN_REAL     Re S summed over the class's directions (VHS: F real and even in k);
//               the Hermitian half of the partial is stored.
// GAIN_COMPLEX  the complex S summed over the class's directions, whole spectrum stored
//               (the dealiased form, whose inputs are not spectra of real fields: the
//               shifted fields come from unpaired transforms).
// GAIN_VSS      VSS (F depends on sigma): a class holds at most two directions; their
//               real parts are transformed together as Re S_0 + i Re S_1 (whole spectrum
//               stored), and their imaginary parts, which reach the result only on the
//               planes k_x, k_y or k_z = N/2 (the literal Nyquist reading), are reduced
//               to those planes (sums with (-1)^x, (-1)^y, (-1)^z) and stored.
enum { GAIN_REAL = 0, GAIN_COMPLEX = 1, GAIN_VSS = 2 };

// Geometry of one work item: the x-chunk c (x-indices = c mod CH, NP = N/CH of them)
// of one S_q field.  Each y/z pencil of the chunk is shared by CZ thread groups: group
// cz keeps the outputs with index = cz mod CZ (decimation in frequency), so a thread
// holds NS = N/CZ values per field.  The group index is uniform per wavefront when
// NTC = NP*N is a multiple of 64, so every twiddle is a compile-time constant; the padded
// grids of the dealiased form (36, 72) have no such split, and there the one wavefront
// that straddles two groups runs both groups' code under its lane masks.
template <typename T, int N, int CH, int CZ>
struct GainK {
    static constexpr int NP = N / CH;
    static constexpr int NS = N / CZ;
    static constexpr int NTC = NP * N;
    static constexpr int NT = NTC * CZ;
    static constexpr int KZH = N / 2 + 1;               // stored k_z of a partial (Hermitian half)
    static constexpr int NPEN = N * KZH;                // stored (k_y, k_z) pencils of a partial
    static constexpr int PX = (NPEN + NT - 1) / NT;     // stored pencils per thread (guarded)
    static constexpr int NPENF = N * N;                 // every (k_y, k_z) pencil (VSS: complex field)
    static constexpr int PXF = (NPENF + NT - 1) / NT;
    static constexpr int ROW = N + 1;                  // padded LDS row (bank spread)
    static constexpr int LDS = NP * N * ROW;
    // packed form: line-data regions [2][NP][N+1], the correction array [N][ROWC] (in
    // the main buffer) and the thread groups GC of its transforms (one wavefront each)
    static constexpr int LINES = 2 * NP * (N + 1);
    static constexpr int ROWC = N + 2 * NP + 1;
    static constexpr int GC = (N % 4 == 0 && 256 <= NT) ? 4 : (N % 3 == 0 && 192 <= NT) ? 3 : (128 <= NT) ? 2 : 1;
    static_assert(NP * CH == N && NS * CZ == N, "CH and CZ must divide N");
    static_assert(NTC % 64 == 0 || N % 9 == 0, "a CZ group must be whole wavefronts (except the 36, 72 grids)");
};

template <typename T>
struct GainArgs {
    const cx<T>* fhat;  // [nb][s][N^3], DFT / N^3
    cx<T>* P;           // [nb][ncls][nrho][CH][N/CH][N][N/2+1]  (k_z <= N/2 of each partial);
                        // GAIN_COMPLEX, GAIN_VSS: [nb][ncls][nrho][CH][N/CH][N][N]  (whole spectrum)
    T* PL;              // GAIN_VSS: [nb][ncls][nrho][2][(2 + CH) N^2]  Nyquist-plane sums of Im S_d:
                        //   [x][y] over z, [x][z] over y, then per chunk [y][z] over its x
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

// sum_t of the chunk terms in[l + t NP] * kx[l + t NP] for one pencil, with two load
// buffers in turn: the next batch of NP loads is in flight while the other is consumed,
// and no register copies between batches.  U tables (one per output) share the loads.
// (The packed N = 48 form's x-pass; at N = 32 the one-field x-pass keeps its rotating
// buffer, which compiles without spills there.)
template <typename T, int NP, int CH, int U>
__device__ __forceinline__ void x_sum_pipe(__amdgpu_buffer_rsrc_t rs, int vo, int rs_stride,
                                           const cx<T>* const (&kx)[U], cx<T>* const (&y)[U]) {
    cx<T> b0[NP], b1[NP];
    auto load = [&](cx<T>* b, int t) {
#pragma unroll
        for (int l = 0; l < NP; ++l) b[l] = bload<T>(rs, vo, (l + t * NP) * rs_stride);
    };
    auto use = [&](const cx<T>* b, int t) {
#pragma unroll
        for (int l = 0; l < NP; ++l)
#pragma unroll
            for (int u = 0; u < U; ++u) cmac(y[u][l], b[l], kx[u][l + t * NP]);
    };
    load(b0, 0);
    int t = 0;
#pragma unroll 1
    for (; t + 2 < CH; t += 2) {
        load(b1, t + 1);
        use(b0, t);
        load(b0, t + 2);
        use(b1, t + 1);
    }
    if constexpr (CH % 2 == 0) {
        load(b1, CH - 1);
        use(b0, CH - 2);
        use(b1, CH - 1);
    } else {
        use(b0, CH - 1);
    }
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
//
// With HERM = false the spectrum is that of a complex field (no pairing): every one of the
// N^2 x-pencils is transformed and stored with its own y/z phase.
template <typename T, int N, int CH, int CZ, bool PIPE, bool HERM = true>
__device__ __forceinline__ void field_ifft(const cx<T>* __restrict__ fh, const cx<T>* __restrict__ kxt,
                                           const cx<T>* __restrict__ yzt, T nyq, int c, cx<T>* buf, int cz,
                                           int m, int r, cx<T>* out) {
    using K = GainK<T, N, CH, CZ>;
    if constexpr (!HERM) {
        constexpr int ES = int(sizeof(cx<T>));
        constexpr int RS = N * N * ES;
        const __amdgpu_buffer_rsrc_t rs = field_rsrc<T>(fh, N * RS);
#pragma unroll 1
        for (int k = 0; k < (N * N + K::NT - 1) / K::NT; ++k) {
            const int P = int(threadIdx.x) + k * K::NT;
            if ((N * N) % K::NT != 0 && P >= N * N) break;
            const int ly = P / N, lz = P % N;
            cx<T> y[K::NP];
#pragma unroll
            for (int l = 0; l < K::NP; ++l) y[l] = cx<T>{T(0), T(0)};
#pragma unroll 1
            for (int t = 0; t < CH; ++t) {
#pragma unroll
                for (int l = 0; l < K::NP; ++l) cmac(y[l], bload<T>(rs, P * ES, (l + t * K::NP) * RS), kxt[l + t * K::NP]);
            }
            fft<K::NP, +1>(y);
            const cx<T> cyz = yzt[ly] * yzt[N + lz];
#pragma unroll
            for (int mm = 0; mm < K::NP; ++mm) buf[(mm * N + ly) * K::ROW + lz] = y[mm] * cyz;
        }
        __syncthreads();
        yz_passes<T, N, CH, CZ, +1>(buf, cz, m, r, out);
        __syncthreads();
        return;
    }
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

// ====================================================== packed pair of fields
// Geometries the packed form supports: at most two x-pass rounds (their plane values
// stay in registers) and one lane per correction column.
template <typename T, int N, int CH, int CZ>
constexpr bool pack_ok() {
    using K = GainK<T, N, CH, CZ>;
    constexpr int ra = (N * N / 2 + 2 + K::NT - 1) / K::NT, rs = (N * N / 2 + K::NT - 1) / K::NT;
    return (rs < ra ? rs : ra) <= 2 && N + 2 * K::NP <= 64 && N * K::ROWC <= K::LDS;
}

// The chunk x-transform of one pencil P of one field (with SELF in a wavefront holding
// self-paired slots: of f(., P) + i mk f(., P + N/2), both loads of an index together).
template <typename T, int N, int CH, bool PIPE>
__device__ __forceinline__ void x_pencil(__amdgpu_buffer_rsrc_t rs, int vo, int vo2, T mk, bool two,
                                         const cx<T>* __restrict__ kxt, cx<T>* y) {
    constexpr int NP = N / CH;
    constexpr int RS = N * N * int(sizeof(cx<T>));
#pragma unroll
    for (int l = 0; l < NP; ++l) y[l] = cx<T>{T(0), T(0)};
    if (two) {
#pragma unroll 1
        for (int t = 0; t < CH; ++t) {
            cx<T> a[NP], b[NP];
#pragma unroll
            for (int l = 0; l < NP; ++l) {
                a[l] = bload<T>(rs, vo, (l + t * NP) * RS);
                b[l] = bload<T>(rs, vo2, (l + t * NP) * RS);
            }
#pragma unroll
            for (int l = 0; l < NP; ++l)
                cmac(y[l], cx<T>{a[l].x - mk * b[l].y, a[l].y + mk * b[l].x}, kxt[l + t * NP]);
        }
    } else if constexpr (PIPE) {
        const cx<T>* const kx1[1] = {kxt};
        cx<T>* const y1[1] = {y};
        x_sum_pipe<T, NP, CH, 1>(rs, vo, RS, kx1, y1);
    } else {
#pragma unroll 1
        for (int t = 0; t < CH; ++t) {
#pragma unroll
            for (int l = 0; l < NP; ++l) cmac(y[l], bload<T>(rs, vo, (l + t * NP) * RS), kxt[l + t * NP]);
        }
    }
    fft<NP, +1>(y);
}

// x_pencil for two fields with the same spectrum (a like class: A and B both shift f^i)
// on a paired slot: every input is loaded once and enters both sums, each with its own
// phase table; each output takes the same operations in the same order as x_pencil's.
template <typename T, int N, int CH, bool PIPE>
__device__ __forceinline__ void x_pencil2(__amdgpu_buffer_rsrc_t rs, int vo, const cx<T>* __restrict__ kxa,
                                          const cx<T>* __restrict__ kxb, cx<T>* ya, cx<T>* yb) {
    constexpr int NP = N / CH;
    constexpr int RS = N * N * int(sizeof(cx<T>));
#pragma unroll
    for (int l = 0; l < NP; ++l) ya[l] = yb[l] = cx<T>{T(0), T(0)};
    if constexpr (PIPE) {
        const cx<T>* const kx2[2] = {kxa, kxb};
        cx<T>* const y2[2] = {ya, yb};
        x_sum_pipe<T, NP, CH, 2>(rs, vo, RS, kx2, y2);
    } else {
#pragma unroll 1
        for (int t = 0; t < CH; ++t) {
#pragma unroll
            for (int l = 0; l < NP; ++l) {
                const cx<T> v = bload<T>(rs, vo, (l + t * NP) * RS);
                cmac(ya[l], v, kxa[l + t * NP]);
                cmac(yb[l], v, kxb[l + t * NP]);
            }
        }
    }
    fft<NP, +1>(ya);
    fft<NP, +1>(yb);
}

// The x-passes of two fields with different spectra (an unlike class) interleaved: both
// fields' loads of a batch are in flight together, each field in two buffers in turn.
template <typename T, int N, int CH>
__device__ __forceinline__ void x_pencil_ab(__amdgpu_buffer_rsrc_t rsa, __amdgpu_buffer_rsrc_t rsb, int vo,
                                            const cx<T>* __restrict__ kxa, const cx<T>* __restrict__ kxb,
                                            cx<T>* ya, cx<T>* yb) {
    constexpr int NP = N / CH;
    constexpr int RS = N * N * int(sizeof(cx<T>));
#pragma unroll
    for (int l = 0; l < NP; ++l) ya[l] = yb[l] = cx<T>{T(0), T(0)};
    cx<T> a0[NP], a1[NP], b0[NP], b1[NP];
    auto load = [&](cx<T>* a, cx<T>* b, int t) {
#pragma unroll
        for (int l = 0; l < NP; ++l) {
            a[l] = bload<T>(rsa, vo, (l + t * NP) * RS);
            b[l] = bload<T>(rsb, vo, (l + t * NP) * RS);
        }
    };
    auto use = [&](const cx<T>* a, const cx<T>* b, int t) {
#pragma unroll
        for (int l = 0; l < NP; ++l) {
            cmac(ya[l], a[l], kxa[l + t * NP]);
            cmac(yb[l], b[l], kxb[l + t * NP]);
        }
    };
    load(a0, b0, 0);
    int t = 0;
#pragma unroll 1
    for (; t + 2 < CH; t += 2) {
        load(a1, b1, t + 1);
        use(a0, b0, t);
        load(a0, b0, t + 2);
        use(a1, b1, t + 1);
    }
    if constexpr (CH % 2 == 0) {
        load(a1, b1, CH - 1);
        use(a0, b0, CH - 2);
        use(a1, b1, CH - 1);
    } else {
        use(a0, b0, CH - 1);
    }
    fft<NP, +1>(ya);
    fft<NP, +1>(yb);
}

template <typename T>
__device__ __forceinline__ cx<T> pack_ab(cx<T> a, cx<T> b) { return cx<T>{a.x - b.y, a.y + b.x}; }          // a + i b
template <typename T>
__device__ __forceinline__ cx<T> pack_conj(cx<T> a, cx<T> b) { return cx<T>{a.x + b.y, b.x - a.y}; }        // conj(a) + i conj(b)
template <typename T>
__device__ __forceinline__ cx<T> pack_nconj(cx<T> a, cx<T> b) { return cx<T>{-a.x - b.y, a.y - b.x}; }      // -(conj(a) + i conj(b))

// One direction of a gain class with both shifted fields A = f^i(v + a rho sigma) and
// B = f^j(v - b rho sigma) carried by one complex transform.
//
// After the x-pass of a field, split its mixed-domain data G(x, P) (P = (l_y, l_z)) into
// the part that is Hermitian in P, whose y/z transform is real, and the anti-Hermitian
// rest.  For a pencil P with partner -P (see field_ifft for y, delta_P and the sign s_n),
// with c = cyz(P), c^ = conj(cyz(-P)), c~ = (c + c^)/2:
//   Herm(P)[n] = y[n] c~ + s_n delta c^ / 2,          Herm(-P) = conj(Herm(P)),
//   AH(P)[n]   = (c - c^)/2 (y[n] + s_n delta / 2) - s_n delta c~ / 2.
// The y/z transform of Herm_A + i Herm_B gives a + i b with a = Re A, b = Re B.  The
// anti-Hermitian part has two pieces, each anti-Hermitian by itself: a plane piece
// -delta c~ / 2 times s_n (its transform is (-1)^x times one 2-D transform), and a line
// piece, nonzero only where c != c^, i.e. on the Nyquist lines l_y = N/2 or l_z = N/2
// (1-D transforms along the other index).  Their transforms are purely imaginary, i alpha,
// so the pieces of A and B are packed the same way: E = i alpha_A - alpha_B.  Then
// Re(A B) = a b - alpha_A alpha_B = Re Z Im Z + Re E Im E.
template <typename T, int N, int CH, int CZ, bool PIPE>
__device__ __forceinline__ void packed_direction(const cx<T>* __restrict__ fa, const cx<T>* __restrict__ fb,
                                                 const cx<T>* __restrict__ kxa, const cx<T>* __restrict__ yza,
                                                 T nyqa, const cx<T>* __restrict__ kxb,
                                                 const cx<T>* __restrict__ yzb, T nyqb, int c, cx<T>* buf, int cz,
                                                 int m, int r, T w, T* S) {
    using K = GainK<T, N, CH, CZ>;
    constexpr int NP = K::NP, H = N / 2;
    constexpr int ROUNDS_ALL = (N * N / 2 + 2 + K::NT - 1) / K::NT;
    constexpr int ROUNDS_SELF = (N * N / 2 + K::NT - 1) / K::NT;
    constexpr bool SELF = ROUNDS_SELF < ROUNDS_ALL;
    constexpr int SLOTS = SELF ? N * N / 2 : N * N / 2 + 2;
    constexpr int ROUNDS = SELF ? ROUNDS_SELF : ROUNDS_ALL;
    static_assert(ROUNDS <= 2, "the plane values of at most two rounds are kept in registers");
    static_assert(N + 2 * NP <= 64, "one lane per correction column");
    static_assert(N * K::ROWC <= K::LDS, "the correction array must fit the main buffer");
    constexpr int ES = int(sizeof(cx<T>));
    constexpr int RS = N * N * ES;
    cx<T>* LY = buf + K::LDS;           // [NP][N+1]: line l_y = N/2, indexed [x][l_z]
    cx<T>* LZ = LY + NP * (N + 1);      // [NP][N+1]: line l_z = N/2, indexed [x][l_y]
    const __amdgpu_buffer_rsrc_t rsa = field_rsrc<T>(fa, N * RS), rsb = field_rsrc<T>(fb, N * RS);
    const bool same = fa == fb;   // a like class: both fields shift one spectrum
    const int tid = threadIdx.x;
    cx<T> pl[2][2];  // plane values of the slot's two pencils, per round

#pragma unroll 1
    for (int k = 0; k < ROUNDS; ++k) {
        const int slot = tid + k * K::NT;
        if (ROUNDS * K::NT != SLOTS && slot >= SLOTS) break;
        int ly, lz;
        const bool paired = pencil_slot<N, SELF>(slot, ly, lz);
        const int vo = (ly * N + lz) * ES;
        const bool two = SELF && __ballot(!paired) != 0;
        const int vo2 = (SELF && !paired) ? vo + H * ES : vo;
        const T mk = (SELF && !paired) ? T(1) : T(0);
        cx<T> ya[NP], yb[NP];
        if (same && !two) {
            x_pencil2<T, N, CH, PIPE>(rsa, vo, kxa, kxb, ya, yb);
        } else if (PIPE && !two) {
            x_pencil_ab<T, N, CH>(rsa, rsb, vo, kxa, kxb, ya, yb);
        } else {
            x_pencil<T, N, CH, PIPE>(rsa, vo, vo2, mk, two, kxa, ya);
            x_pencil<T, N, CH, PIPE>(rsb, vo, vo2, mk, two, kxb, yb);
        }
        const cx<T> fna = bload<T>(rsa, vo, H * RS), fnb = bload<T>(rsb, vo, H * RS);
        cx<T> p0, p1;
        if (paired) {
            const int ly2 = (N - ly) % N, lz2 = (N - lz) % N;
            const cx<T> da = cx<T>{-nyqa * fna.y, nyqa * fna.x}, db = cx<T>{-nyqb * fnb.y, nyqb * fnb.x};
            const cx<T> ca = yza[ly] * yza[N + lz], cb = yzb[ly] * yzb[N + lz];
            const cx<T> c2a = yza[ly2] * yza[N + lz2], c2b = yzb[ly2] * yzb[N + lz2];
            const cx<T> cha = cx<T>{c2a.x, -c2a.y}, chb = cx<T>{c2b.x, -c2b.y};
            const cx<T> cta = T(0.5) * (ca + cha), ctb = T(0.5) * (cb + chb);
            const cx<T> dha = T(0.5) * (da * cha), dhb = T(0.5) * (db * chb);
#pragma unroll
            for (int mm = 0; mm < NP; ++mm) {
                const bool odd = ((CH * mm + c) & 1) != 0;
                const cx<T> ha = odd ? ya[mm] * cta - dha : ya[mm] * cta + dha;
                const cx<T> hb = odd ? yb[mm] * ctb - dhb : yb[mm] * ctb + dhb;
                buf[(mm * N + ly) * K::ROW + lz] = pack_ab(ha, hb);
                buf[(mm * N + ly2) * K::ROW + lz2] = pack_conj(ha, hb);
            }
            if (ly == H || lz == H) {  // line piece (c != c^ only here)
                const cx<T> ga = T(0.5) * (ca - cha), gb = T(0.5) * (cb - chb);
                const cx<T> hda = T(0.5) * da, hdb = T(0.5) * db;
#pragma unroll
                for (int mm = 0; mm < NP; ++mm) {
                    const bool odd = ((CH * mm + c) & 1) != 0;
                    const cx<T> la = ga * (odd ? ya[mm] - hda : ya[mm] + hda);
                    const cx<T> lb = gb * (odd ? yb[mm] - hdb : yb[mm] + hdb);
                    if (ly == H) {
                        LY[mm * (N + 1) + lz] = pack_ab(la, lb);
                        LY[mm * (N + 1) + lz2] = pack_nconj(la, lb);
                    } else {
                        LZ[mm * (N + 1) + ly] = pack_ab(la, lb);
                        LZ[mm * (N + 1) + ly2] = pack_nconj(la, lb);
                    }
                }
            }
            const cx<T> pia = T(-0.5) * (da * cta), pib = T(-0.5) * (db * ctb);
            p0 = pack_ab(pia, pib);
            p1 = pack_nconj(pia, pib);
        } else {
            // self-paired pencils: (ly, lz) alone, or with SELF the pair (ly, 0), (ly, N/2)
            // from one transform of f(., P1) + i f(., P2) per field
            const T f2a = SELF ? bload<T>(rsa, vo + H * ES, H * RS).x : T(0);
            const T f2b = SELF ? bload<T>(rsb, vo + H * ES, H * RS).x : T(0);
            const T d1a = nyqa * fna.x, d1b = nyqb * fnb.x, d2a = nyqa * f2a, d2b = nyqb * f2b;
            const int lzs[2] = {SELF ? 0 : lz, H};
            const T dsa[2] = {d1a, d2a}, dsb[2] = {d1b, d2b};
#pragma unroll
            for (int e = 0; e < (SELF ? 2 : 1); ++e) {
                const int lze = lzs[e];
                const cx<T> ca = yza[ly] * yza[N + lze], cb = yzb[ly] * yzb[N + lze];
                const bool line = ly == H || lze == H;
#pragma unroll
                for (int mm = 0; mm < NP; ++mm) {
                    const bool odd = ((CH * mm + c) & 1) != 0;
                    cx<T> ua = ya[mm], ub = yb[mm];
                    if (SELF) {  // unscramble: y_k = a_k - i d_k (-1)^n / 2
                        const T e1a = T(0.5) * (odd ? -d1a : d1a), e2a = T(0.5) * (odd ? -d2a : d2a);
                        const T e1b = T(0.5) * (odd ? -d1b : d1b), e2b = T(0.5) * (odd ? -d2b : d2b);
                        ua = e == 0 ? cx<T>{ya[mm].x - e2a, -e1a} : cx<T>{ya[mm].y + e1a, -e2a};
                        ub = e == 0 ? cx<T>{yb[mm].x - e2b, -e1b} : cx<T>{yb[mm].y + e1b, -e2b};
                    }
                    const cx<T> va = ua * ca, vb = ub * cb;
                    buf[(mm * N + ly) * K::ROW + lze] = cx<T>{va.x, vb.x};
                    if (line) {
                        // (c - conj c)/2 (y + s delta / 2) with delta = i d
                        const T sa = T(0.5) * (odd ? -dsa[e] : dsa[e]), sb = T(0.5) * (odd ? -dsb[e] : dsb[e]);
                        const cx<T> la = cx<T>{T(0), ca.y} * cx<T>{ua.x, ua.y + sa};
                        const cx<T> lb = cx<T>{T(0), cb.y} * cx<T>{ub.x, ub.y + sb};
                        if (ly == H) LY[mm * (N + 1) + lze] = pack_ab(la, lb);
                        else LZ[mm * (N + 1) + ly] = pack_ab(la, lb);
                    }
                }
                const cx<T> pia = cx<T>{T(0), T(-0.5) * dsa[e] * ca.x}, pib = cx<T>{T(0), T(-0.5) * dsb[e] * cb.x};
                if (e == 0) p0 = pack_ab(pia, pib);
                else p1 = pack_ab(pia, pib);
            }
        }
        if (k == 0) {
            pl[0][0] = p0;
            pl[0][1] = p1;
        } else {
            pl[1][0] = p0;
            pl[1][1] = p1;
        }
    }
    __syncthreads();
    cx<T> Z[K::NS];
    yz_passes<T, N, CH, CZ, +1>(buf, cz, m, r, Z);
    __syncthreads();

    // the correction array CB[N][ROWC] in the main buffer: the plane at columns 0..N-1
    // ([l_y][l_z]), then line l_y = N/2 transposed ([l_z][N + x]), then line l_z = N/2
    // transposed ([l_y][N + NP + x], zero at l_y = N/2)
    cx<T>* CB = buf;
#pragma unroll 1
    for (int k = 0; k < ROUNDS; ++k) {
        const int slot = tid + k * K::NT;
        if (ROUNDS * K::NT != SLOTS && slot >= SLOTS) break;
        int ly, lz;
        const bool paired = pencil_slot<N, SELF>(slot, ly, lz);
        const cx<T> v0 = k == 0 ? pl[0][0] : pl[1][0], v1 = k == 0 ? pl[0][1] : pl[1][1];
        if (paired) {
            CB[ly * K::ROWC + lz] = v0;
            CB[((N - ly) % N) * K::ROWC + (N - lz) % N] = v1;
        } else {
            CB[ly * K::ROWC + (SELF ? 0 : lz)] = v0;
            if (SELF) CB[ly * K::ROWC + H] = v1;
        }
    }
    for (int t = tid; t < NP * N; t += K::NT) {
        const int mm = t / N, l = t % N;
        CB[l * K::ROWC + N + mm] = LY[mm * (N + 1) + l];
        CB[l * K::ROWC + N + NP + mm] = l == H ? cx<T>{T(0), T(0)} : LZ[mm * (N + 1) + l];
    }
    __syncthreads();
    const int g = tid / 64, p = tid % 64;
    {
        constexpr int NJ = N / K::GC;
        cx<T> v[NJ];
        const bool act = g < K::GC && p < N + 2 * NP;
        if (act) {
            with_group<K::GC>(g, [&](auto gg) { split_fft<N, K::GC, decltype(gg)::value, +1, K::ROWC>(CB + p, v); });
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) CB[(K::GC * j + g) * K::ROWC + p] = v[j];
        }
        __syncthreads();
        const bool act2 = g < K::GC && p < N;
        if (act2) {
            with_group<K::GC>(g, [&](auto gg) { split_fft<N, K::GC, decltype(gg)::value, +1, 1>(CB + p * K::ROWC, v); });
        }
        __syncthreads();
        if (act2) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) CB[p * K::ROWC + K::GC * j + g] = v[j];
        }
        __syncthreads();
    }
    // E at the thread's points (x = CH m + c, y = r, z = CZ j + cz)
    const T sx = ((CH * m + c) & 1) ? T(-1) : T(1), sy = (r & 1) ? T(-1) : T(1);
    const cx<T> t3 = CB[r * K::ROWC + N + NP + m];
#pragma unroll
    for (int j = 0; j < K::NS; ++j) {
        const int nz = CZ * j + cz;
        const cx<T> t1 = CB[r * K::ROWC + nz], t2 = CB[nz * K::ROWC + N + m];
        const T sz = (nz & 1) ? T(-1) : T(1);
        const T ex = sx * t1.x + sy * t2.x + sz * t3.x, ey = sx * t1.y + sy * t2.y + sz * t3.y;
        S[j] = fma(w, fma(Z[j].x, Z[j].y, ex * ey), S[j]);
    }
    __syncthreads();
}

// Forward transform of one work item's field, held in buf (LDS) as rows (plane m of the
// chunk, y) of z values with row stride N + 1: z and y passes through LDS, then the chunk's
// part of the x-transform; stores the chunk partial (Pq: the partials of this (node, class,
// rho_q), chunk c at offset c * N/CH * pencils).  CPLX: the field is complex and every (k_y,
// k_z) pencil is stored; otherwise the field is real, its partial Hermitian, and only
// k_z <= N/2 is stored.  Needs every thread of the work item (GainK<T, N, CH, CZ>::NT).
template <typename T, int N, int CH, int CZ, bool CPLX>
__device__ __forceinline__ void store_partial(cx<T>* buf, cx<T>* Pq, int c) {
    using K = GainK<T, N, CH, CZ>;
    const int tid = threadIdx.x;
    const int cz = tid / K::NTC, u = tid % K::NTC;
    const int m = u / N, r = u % N;
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
    if constexpr (CPLX) {
        // the transform of a complex field: every (k_y, k_z) pencil is stored
        constexpr int64_t PCHF = int64_t(K::NP) * K::NPENF;
        cx<T>* Pout = Pq + int64_t(c) * PCHF;
#pragma unroll 1
        for (int k = 0; k < K::PXF; ++k) {
            const int P = tid + k * K::NT;
            if (K::PXF * K::NT != K::NPENF && P >= K::NPENF) break;
            const int ky = P / N, kz = P % N;
            cx<T> v[K::NP];
#pragma unroll
            for (int mm = 0; mm < K::NP; ++mm) v[mm] = buf[(mm * N + ky) * K::ROW + kz];
            fft<K::NP, -1>(v);
#pragma unroll
            for (int kk = 0; kk < K::NP; ++kk) Pout[kk * K::NPENF + P] = v[kk];
        }
        return;
    }
    // The chunk's partial is the DFT of a real array over (x-planes of the chunk, y, z),
    // so it is Hermitian in (k_xp, k_y, k_z): only k_z <= N/2 is stored, the radial kernel
    // reads the rest as conjugates of the mirrored entries.
    constexpr int64_t PCH = int64_t(K::NP) * K::NPEN;  // stored values of one chunk partial
    cx<T>* Pout = Pq + int64_t(c) * PCH;
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

template <typename T, int N, int CH, int CZ, bool PIPE, bool PACK, int MODE>
__global__ __launch_bounds__((GainK<T, N, CH, CZ>::NT)) void gain_kernel(GainArgs<T> a) {
    using K = GainK<T, N, CH, CZ>;
    constexpr bool CPLX = MODE != GAIN_REAL;  // the whole spectrum of a complex field is stored
    static_assert(!(PACK && CPLX), "the packed two-field form keeps only Re(A B)");
    __shared__ cx<T> buf[K::LDS + ((PACK && pack_ok<T, N, CH, CZ>()) ? K::LINES : 0)];
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

    // VHS: only Re(S_q) reaches the result, since the radial operator multiplies
    // DFT(S_q) by a real F that is even in k: Re IDFT(F DFT(S)) = IDFT(F DFT(Re S)).
    // VSS: F depends on the direction and, at indices with a Nyquist component, F at the
    // mode of k is not the conjugate of F at the mode of the mirror index, so there the
    // imaginary part of S (from the Nyquist modes of the shifted fields) contributes.
    T S[K::NS], S1[CPLX ? K::NS : 1];
#pragma unroll
    for (int n = 0; n < K::NS; ++n) S[n] = T(0);
#pragma unroll
    for (int n = 0; n < (CPLX ? K::NS : 1); ++n) S1[n] = T(0);

    // GAIN_VSS: reduce Im S of direction d (in im[]) to the three Nyquist planes
    auto nyquist_planes = [&](int d, const T* im) {
        constexpr int N2 = N * N;
        T* PL = a.PL + (((int64_t(b) * a.ncls + cl) * a.nrho + q) * 2 + d) * int64_t((2 + CH) * N2);
#pragma unroll
        for (int j = 0; j < K::NS; ++j) buf[(m * N + r) * K::ROW + CZ * j + cz] = cx<T>{im[j], T(0)};
        __syncthreads();
        if (cz == 0) {  // over z: [x][y]
            T acc = T(0);
            for (int z = 0; z < N; ++z) acc += (z & 1) ? -buf[(m * N + r) * K::ROW + z].x : buf[(m * N + r) * K::ROW + z].x;
            PL[(c + CH * m) * N + r] = acc;
        }
        for (int e = tid; e < K::NP * N; e += K::NT) {  // over y: [x][z]
            const int mm = e / N, z = e % N;
            T acc = T(0);
            for (int y = 0; y < N; ++y) acc += (y & 1) ? -buf[(mm * N + y) * K::ROW + z].x : buf[(mm * N + y) * K::ROW + z].x;
            PL[N2 + (c + CH * mm) * N + z] = acc;
        }
        for (int e = tid; e < N2; e += K::NT) {  // over this chunk's x: [y][z]
            const int y = e / N, z = e % N;
            T acc = T(0);
            for (int mm = 0; mm < K::NP; ++mm) {
                const T v = buf[(mm * N + y) * K::ROW + z].x;
                acc += ((c + CH * mm) & 1) ? -v : v;
            }
            PL[2 * N2 + c * N2 + e] = acc;
        }
        __syncthreads();
    };

    auto direction = [&](int d, T* Sd) {
        const int64_t base = (int64_t(doff + d) * a.nrho + q) * 2;
        if constexpr (PACK && pack_ok<T, N, CH, CZ>()) {
            packed_direction<T, N, CH, CZ, PIPE>(fhi, fhj, a.kx + ((base + 0) * CH + c) * N, a.yz + (base + 0) * 2 * N,
                                                 a.nyq[base], a.kx + ((base + 1) * CH + c) * N,
                                                 a.yz + (base + 1) * 2 * N, a.nyq[base + 1], c, buf, cz, m, r, w, Sd);
        } else {
            cx<T> A[K::NS], B[K::NS];
            constexpr bool HERM = MODE != GAIN_COMPLEX;
            field_ifft<T, N, CH, CZ, PIPE, HERM>(fhi, a.kx + ((base + 0) * CH + c) * N, a.yz + (base + 0) * 2 * N,
                                                 a.nyq[base], c, buf, cz, m, r, A);
            field_ifft<T, N, CH, CZ, PIPE, HERM>(fhj, a.kx + ((base + 1) * CH + c) * N, a.yz + (base + 1) * 2 * N,
                                                 a.nyq[base + 1], c, buf, cz, m, r, B);
#pragma unroll
            for (int n = 0; n < K::NS; ++n) Sd[n] = fma(w, fma(A[n].x, B[n].x, -A[n].y * B[n].y), Sd[n]);
            if constexpr (MODE == GAIN_COMPLEX) {
#pragma unroll
                for (int n = 0; n < K::NS; ++n) S1[n] = fma(w, fma(A[n].x, B[n].y, A[n].y * B[n].x), S1[n]);
            }
            if constexpr (MODE == GAIN_VSS) {
                T im[K::NS];
#pragma unroll
                for (int n = 0; n < K::NS; ++n) im[n] = w * fma(A[n].x, B[n].y, A[n].y * B[n].x);
                nyquist_planes(d, im);
            }
        }
    };
    if constexpr (MODE == GAIN_VSS) {
        direction(0, S);
        if (ndir > 1) {
            direction(1, S1);
        } else {  // a one-direction class: its second plane sums are zero
            T zero[K::NS];
#pragma unroll
            for (int n = 0; n < K::NS; ++n) zero[n] = T(0);
            nyquist_planes(1, zero);
        }
    } else {
        for (int d = 0; d < ndir; ++d) direction(d, S);
    }

    // forward DFT of Re S_q (complex modes: of S + i S1): the field goes to LDS as rows
    // (plane, y) of z values
#pragma unroll
    for (int j = 0; j < K::NS; ++j) {
        if constexpr (CPLX) buf[(m * N + r) * K::ROW + CZ * j + cz] = cx<T>{S[j], S1[j]};
        else buf[(m * N + r) * K::ROW + CZ * j + cz] = cx<T>{S[j], T(0)};
    }
    __syncthreads();
    cx<T>* Pq = a.P + ((int64_t(b) * a.ncls + cl) * a.nrho + q) * int64_t(CH) * K::NP * (CPLX ? K::NPENF : K::NPEN);
    store_partial<T, N, CH, CZ, CPLX>(buf, Pq, c);
}

// =============================================================== radial kernel
// VSS: the Hermitian part of sum_d F_d DFT(S_d), with S_d = Re S_d + i Im S_d, Z the
// spectrum of Re S_0 + i Re S_1 and V_d = DFT(Im S_d):
//   sum_d F_H,d U_d + i F_A,d V_d,  U_0 = (Z(k) + conj Z(-k))/2, U_1 = (Z(k) - conj Z(-k))/(2i),
// F_H, F_A the Hermitian and anti-Hermitian parts of F (F_A vanishes off the Nyquist
// planes, where V_d is needed).
template <typename T, typename A = double>
__device__ __forceinline__ void vss_accumulate(cx<A>& acc, const cx<T> h[2], const cx<T> fa[2], A u0x,
                                               A u0y, A u1x, A u1y, bool nyq, const cx<T> v[2]) {
    acc.x += A(h[0].x) * u0x - A(h[0].y) * u0y + A(h[1].x) * u1x - A(h[1].y) * u1y;
    acc.y += A(h[0].x) * u0y + A(h[0].y) * u0x + A(h[1].x) * u1y + A(h[1].y) * u1x;
    if (nyq) {
#pragma unroll
        for (int d = 0; d < 2; ++d) {  // i F_A V
            acc.x -= A(fa[d].x) * A(v[d].y) + A(fa[d].y) * A(v[d].x);
            acc.y += A(fa[d].x) * A(v[d].x) - A(fa[d].y) * A(v[d].y);
        }
    }
}

// Slot of entry (r, c) of a Nyquist plane in the mirror-paired layout: each entry and
// its plane mirror ((N - r) % N, (N - c) % N) fill one aligned pair of slots (rows r and
// N - r interleaved; in the self-mirror rows 0 and N/2, columns c and N - c), and the four
// entries that are their own mirror take the last two slots of those two rows.
template <int N>
__device__ __forceinline__ int vpair_slot(int r, int c) {
    constexpr int H = N / 2;
    if (r != 0 && r != H) {
        const int lo = r < H ? r : N - r;
        return 2 * N * lo + 2 * (r < H ? c : (N - c) % N) + (r < H ? 0 : 1);
    }
    const int base = r == 0 ? 0 : N;
    if (c != 0 && c != H) return base + 2 * ((c < H ? c : N - c) - 1) + (c < H ? 0 : 1);
    return base + N - 2 + (c == 0 ? 0 : 1);
}
// Slot of mode k (with a component at the Nyquist index) in the three mirror-paired
// planes: [k_x][k_y] where k_z = N/2, else [k_x][k_z] where k_y = N/2, else [k_y][k_z].
template <int N>
__device__ __forceinline__ int vplane_slot(int kx, int ky, int kz) {
    if (kz == N / 2) return vpair_slot<N>(kx, ky);
    if (ky == N / 2) return N * N + vpair_slot<N>(kx, kz);
    return 2 * N * N + vpair_slot<N>(ky, kz);
}
// W at k and at its plane mirror from the aligned pair holding them.
template <typename T, int N>
__device__ __forceinline__ void w_pair(const cx<T>* Vb, int kx, int ky, int kz, cx<T>& w, cx<T>& wm) {
    const int sl = vplane_slot<N>(kx, ky, kz);
    const cx<T> p0 = Vb[sl & ~1], p1 = Vb[sl | 1];
    const bool self = (kx == 0 || kx == N / 2) + (ky == 0 || ky == N / 2) + (kz == 0 || kz == N / 2) == 3;
    w = (sl & 1) ? p1 : p0;
    wm = self ? w : ((sl & 1) ? p0 : p1);
}

// W = DFT(Im S_0 + i Im S_1) on the three Nyquist planes from the plane sums: one block
// per (node, class, rho), one thread group of N per plane; the first pass transforms
// along the plane's first axis (coalesced column reads), the second along its second
// axis, the result leaves through LDS with coalesced stores.  Each V_d = DFT(Im S_d) is
// Hermitian on its plane, so the radial kernel separates them from W at k and at the
// plane mirror of k.
template <typename T, int N, int CH>
__global__ __launch_bounds__(3 * N) void nyquist_dft_kernel(const T* __restrict__ PL, cx<T>* __restrict__ V) {
    constexpr int N2 = N * N;
    const int64_t it = blockIdx.x;  // (node, class, rho)
    const int plane = threadIdx.x / N, t = threadIdx.x % N;
    __shared__ cx<T> Ls[3][N][N + 1];
    const T* p0 = PL + (it * 2 + 0) * int64_t((2 + CH) * N2);
    const T* p1 = PL + (it * 2 + 1) * int64_t((2 + CH) * N2);
    auto at = [&](const T* pl, int r) {
        if (plane < 2) return pl[plane * N2 + r * N + t];
        T v = T(0);
#pragma unroll
        for (int c = 0; c < CH; ++c) v += pl[2 * N2 + c * N2 + r * N + t];
        return v;
    };
    {
        cx<T> x[N];  // column t of the plane, transformed along its first axis
#pragma unroll
        for (int r = 0; r < N; ++r) x[r] = cx<T>{at(p0, r), at(p1, r)};
        fft<N, -1>(x);
#pragma unroll
        for (int k = 0; k < N; ++k) Ls[plane][k][t] = x[k];
    }
    __syncthreads();
    {
        cx<T> x[N];  // row t (first-axis mode t), transformed along the second axis
#pragma unroll
        for (int c2 = 0; c2 < N; ++c2) x[c2] = Ls[plane][t][c2];
        fft<N, -1>(x);
#pragma unroll
        for (int k = 0; k < N; ++k) Ls[plane][t][k] = x[k];
    }
    __syncthreads();
    cx<T>* out = V + it * int64_t(3 * N2) + plane * N2;   // mirror-paired slots (vpair_slot)
    for (int row = 0; row < N; ++row) out[vpair_slot<N>(row, t)] = Ls[plane][row][t];
}


// V_0 and V_1 at k from W at k and at its plane mirror.
template <typename T>
__device__ __forceinline__ void split_w(const cx<T>& W, const cx<T>& Wm, cx<T> v[2]) {
    v[0] = cx<T>{T(0.5) * (W.x + Wm.x), T(0.5) * (W.y - Wm.y)};
    v[1] = cx<T>{T(0.5) * (W.y + Wm.y), T(0.5) * (Wm.x - W.x)};
}

template <typename T>
struct RadialArgs {
    const cx<T>* P;
    const cx<T>* fhat;
    cx<T>* Gt;          // [nb][nslots][N][N][N/2+1]  gain spectrum, the k_z <= N/2 half
    cx<T>* Lt;          // [nb][nslots][N][N][N/2+1]  loss spectrum, the same half
    const T* F;         // [nftab][nrho][K2]  w_q F(|k|, rho_q) / N^3
    const cx<T>* Fv;    // VSS: [nftab][nrho][2 directions][2][N][N][N/2+1]  F_H, F_A: the Hermitian and
                        //      anti-Hermitian parts (in the index sense) of w_q w_sigma F / N^3
    const cx<T>* V;     // VSS: [nb][ncls][nrho][3][N^2]  DFT(Im S_0 + i Im S_1) on the planes k_z, k_y, k_x = N/2,
                        //      each plane in the mirror-paired slots of vpair_slot
    const T* G;         // [ngtab][K2]        G-(|k|)
    const cx<T>* tw;    // [N][CH]  e^{-2 pi i kx c / N}
    const int* slots;   // [nslots][5]
    const int* gterms;  // [..][2]
    const int* lterms;  // [..][2]
    const int* cuses;   // [ncls][4]  (slot, F table) x 2 per class, -1 if unused
    int s, ncls, nrho, nb, nslots, K2;
};

// One thread per Hermitian pair {k, -k} of the output spectrum: it takes the
// representative with k_z <= N/2 (the stored half of the partials), forms
// Q_hat+(k) = sum_terms sum_q w_q F(|k|, rho_q)/N^3 DFT(S_q)(k) and the loss spectrum
// L(k) = sum_j G-(|k|) f_hat^j(k) for the CH x-modes k_x = k_xp + j N/CH, and writes
// both to the k_z <= N/2 half of the output spectra: the spectra are Hermitian (S_q and
// f are real, F and G- are real and even in k), and the inverse transform takes them as
// such.
// VSS: each class (up to two directions) partial is the whole spectrum Z of
// Re S_0 + i Re S_1; the thread reads Z at k and -k and adds the Nyquist-plane terms
// (vss_accumulate).
template <typename T, int N, int CH, bool VSS>
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

    // the sum over radial points and classes is kept in FP64 (free here: the kernel is
    // bound by its reads of the partials)
    cx<double> acc[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) acc[j] = cx<double>{0.0, 0.0};
    if constexpr (VSS) {
        constexpr int64_t PCHF = int64_t(NP) * N2, NREP = N2 * KZH;
        const int kxpm = (NP - kxp) % NP, kym = (N - ky) % N, kzm = (N - kz) % N;
        const int64_t eP = (int64_t(kxp) * N + ky) * N + kz, ePm = (int64_t(kxpm) * N + kym) * N + kzm;
        for (int gi = 0; gi < ng; ++gi) {
            const int cl = a.gterms[2 * (g0 + gi)], ft = a.gterms[2 * (g0 + gi) + 1];
            const cx<T>* Pb = a.P + (int64_t(b) * a.ncls + cl) * a.nrho * (CH * PCHF);
            const cx<T>* Fb = a.Fv + int64_t(ft) * a.nrho * 4 * NREP + (int64_t(kxp) * N + ky) * KZH + kz;
            const cx<T>* Vb = a.V + (int64_t(b) * a.ncls + cl) * a.nrho * (3 * N2);
            for (int q = 0; q < a.nrho; ++q) {
                cx<T> pc[CH], pm[CH];
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    pc[c] = Pb[int64_t(q) * (CH * PCHF) + c * PCHF + eP];
                    pm[c] = Pb[int64_t(q) * (CH * PCHF) + c * PCHF + ePm];
                }
#pragma unroll
                for (int j = 0; j < CH; ++j) {
                    const int kx = kxp + j * NP, kxm = (N - kx) % N;
                    cx<T> Z = pc[0], Zm = pm[0];
#pragma unroll
                    for (int c = 1; c < CH; ++c) {
                        cmac(Z, a.tw[kx * CH + c], pc[c]);
                        cmac(Zm, a.tw[kxm * CH + c], pm[c]);
                    }
                    cx<T> h[2], fa[2], v[2];
#pragma unroll
                    for (int d = 0; d < 2; ++d) {
                        h[d] = Fb[((int64_t(q) * 2 + d) * 2 + 0) * NREP + int64_t(j) * NP * N * KZH];
                        fa[d] = Fb[((int64_t(q) * 2 + d) * 2 + 1) * NREP + int64_t(j) * NP * N * KZH];
                    }
                    const bool nyq = kx == N / 2 || ky == N / 2 || kz == N / 2;
                    if (nyq)
                    {
                        cx<T> w, wm;
                        w_pair<T, N>(Vb + int64_t(q) * (3 * N2), kx, ky, kz, w, wm);
                        split_w<T>(w, wm, v);
                    }
                    vss_accumulate<T>(acc[j], h, fa, 0.5 * (double(Z.x) + double(Zm.x)),
                                      0.5 * (double(Z.y) - double(Zm.y)), 0.5 * (double(Z.y) + double(Zm.y)),
                                      0.5 * (double(Zm.x) - double(Z.x)), nyq, v);
                }
            }
        }
    }
    // the chunk twiddles e^{-2 pi i kxp c / N} of this thread's k_xp, loaded once
    cx<T> twc[CH];
#pragma unroll
    for (int c = 1; c < CH; ++c) twc[c] = a.tw[kxp * CH + c];
    for (int gi = 0; gi < (VSS ? 0 : ng); ++gi) {
        const int cl = a.gterms[2 * (g0 + gi)], ft = a.gterms[2 * (g0 + gi) + 1];
        const cx<T>* Pb = a.P + (int64_t(b) * a.ncls + cl) * a.nrho * (CH * PCH) + e;
        const T* Ft = a.F + int64_t(ft) * a.nrho * a.K2;
        for (int q = 0; q < a.nrho; ++q) {
            // the last radix-CH step of the x-transform (decimation in time): with
            // k_x = k_xp + j N/CH, DFT(S)(k_x) = sum_c (e^{-2 pi i kxp c / N} P_c) e^{-2 pi i j c / CH}
            cx<T> y[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const cx<T> pc = Pb[int64_t(q) * (CH * PCH) + c * PCH];
                y[c] = c == 0 ? pc : pc * twc[c];
            }
            fft<CH, -1>(y);
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const double fq = double(Ft[q * a.K2 + k2[j]]);
                acc[j].x = fma(fq, double(y[j].x), acc[j].x);
                acc[j].y = fma(fq, double(y[j].y), acc[j].y);
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
    const int64_t ob = (int64_t(b) * a.nslots + slot) * (N2 * KZH);
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        const int64_t o = ob + (int64_t(kxp + j * NP) * N + ky) * KZH + kz;
        a.Gt[o] = cx<T>{T(acc[j].x), T(acc[j].y)};
        a.Lt[o] = lac[j];
    }
}

// Row r (0 <= r < NP N) of the radial thread order, as the (k_xp, k_y) row of a chunk
// partial, enumerated in mirror pairs: the groups k_xp = 0 and k_xp = NP/2 (each its own
// mirror in k_xp; rows k_y and -k_y adjacent, 0 and N/2 first), then the rows of k_xp
// and NP - k_xp for k_xp = 1 .. NP/2 - 1, each beside its mirror.  A thread reads the
// partials at k and -k, so with this order a workgroup's reads of a row and of its
// mirror row fall in the same cache lines at the same time.
template <int N, int NP>
__device__ __forceinline__ void mirror_paired_row(int r, int& kxp, int& ky) {
    static_assert(NP % 2 == 0, "row pairing needs an even number of x-planes per chunk");
    if (r < 2 * N) {
        kxp = r < N ? 0 : NP / 2;
        const int rr = r < N ? r : r - N, i = rr >> 1;
        ky = (rr & 1) ? (i == 0 ? N / 2 : N - i) : i;
        return;
    }
    const int g = (r - 2 * N) / (2 * N), rr = (r - 2 * N) % (2 * N), i = rr >> 1;
    kxp = (rr & 1) ? NP - 1 - g : 1 + g;
    ky = (rr & 1) ? (N - i) % N : i;
}

// VSS radial sum with every slot of NB nodes in one thread: per class (up to two
// directions), use and radial point the table values are loaded once and applied to the
// NB nodes' partials (read at k and -k; the second use of an unlike class finds them in
// L2).  The per-slot
// accumulators are indexed with compile-time slots (SMAX >= nslots) under uniform
// compares, so they stay in registers.  They are of the plan precision (FP32 plans sum in
// FP32): that halves their registers and lets three waves share a SIMD, which is what
// this latency-bound kernel needs.  Loss terms and outputs as in radial_kernel.
template <typename T, int N, int CH, int NB, int SMAX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void radial_vss_kernel(RadialArgs<T> a) {
    constexpr int NP = N / CH;
    constexpr int KZH = N / 2 + 1;
    constexpr int64_t N2 = int64_t(N) * N, N3 = N2 * N, PCH = int64_t(NP) * N * KZH;
    constexpr int64_t PCHF = int64_t(NP) * N2, NREP = N2 * KZH;
    // Blocks with consecutive indices take the same 256 stored entries for consecutive
    // node groups, so a block's slice of the kernel-mode tables is read from its XCD's L2
    // by the node groups that follow, not from memory per group.
    const int64_t ngroups = (a.nb + NB - 1) / NB;
    const int64_t ng = int64_t(blockIdx.x) % ngroups;
    const int64_t eblk = int64_t(blockIdx.x) / ngroups;
    if (eblk * 256 + threadIdx.x >= PCH) return;
    const int e = int(eblk * 256 + threadIdx.x);
    const int b0 = int(ng) * NB;
    const int kz = e % KZH;
    int kxp, ky;
    mirror_paired_row<N, NP>(e / KZH, kxp, ky);
    const int kxpm = (NP - kxp) % NP, kym = (N - ky) % N, kzm = (N - kz) % N;
    const int64_t eP = (int64_t(kxp) * N + ky) * N + kz, ePm = (int64_t(kxpm) * N + kym) * N + kzm;
    const int64_t fo = (int64_t(kxp) * N + ky) * KZH + kz;

    cx<T> acc[NB][SMAX][CH];
#pragma unroll
    for (int u = 0; u < NB; ++u)
#pragma unroll
        for (int sl = 0; sl < SMAX; ++sl)
#pragma unroll
            for (int j = 0; j < CH; ++j) acc[u][sl][j] = cx<T>{T(0), T(0)};

    constexpr int N2I = N * N;
    bool nyq[CH];
    int wi[CH];   // the aligned pair holding W at k and at its plane mirror (pair 0 off the planes)
    bool wodd[CH], wself[CH];
    bool nyq_any = false;
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        const int kx = kxp + j * NP;
        nyq[j] = kx == N / 2 || ky == N / 2 || kz == N / 2;
        const int sl = nyq[j] ? vplane_slot<N>(kx, ky, kz) : 0;
        wi[j] = sl & ~1;
        wodd[j] = (sl & 1) != 0;
        wself[j] = (kx == 0 || kx == N / 2) + (ky == 0 || ky == N / 2) + (kz == 0 || kz == N / 2) == 3;
        nyq_any = nyq_any || nyq[j];
    }
    for (int cl = 0; cl < a.ncls; ++cl) {
        const int s0 = a.cuses[4 * cl], s1 = a.cuses[4 * cl + 2];
        if (s0 < 0) continue;
        const cx<T>* F0 = a.Fv + int64_t(a.cuses[4 * cl + 1]) * a.nrho * 4 * NREP + fo;
        const cx<T>* F1 = a.Fv + int64_t(s1 >= 0 ? a.cuses[4 * cl + 3] : a.cuses[4 * cl + 1]) * a.nrho * 4 * NREP + fo;
        for (int q = 0; q < a.nrho; ++q) {
            // F_H of both uses and both directions; F_A only where some lane has a Nyquist mode
            cx<T> h0[CH][2], h1[CH][2], a0[CH][2], a1[CH][2];
#pragma unroll
            for (int j = 0; j < CH; ++j)
#pragma unroll
                for (int d = 0; d < 2; ++d) {
                    const int64_t o = ((int64_t(q) * 2 + d) * 2) * NREP + int64_t(j) * NP * N * KZH;
                    h0[j][d] = F0[o];
                    h1[j][d] = F1[o];
                    a0[j][d] = cx<T>{T(0), T(0)};
                    a1[j][d] = cx<T>{T(0), T(0)};
                }
            if (nyq_any) {
#pragma unroll
                for (int j = 0; j < CH; ++j) {
#pragma unroll
                    for (int d = 0; d < 2; ++d) {
                        const int64_t o = ((int64_t(q) * 2 + d) * 2 + 1) * NREP + int64_t(j) * NP * N * KZH;
                        a0[j][d] = F0[o];
                        a1[j][d] = F1[o];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int b = b0 + u;
                if (b >= a.nb) break;
                const cx<T>* Pb = a.P + ((int64_t(b) * a.ncls + cl) * a.nrho + q) * (CH * PCHF);
                const cx<T>* Vb = a.V + ((int64_t(b) * a.ncls + cl) * a.nrho + q) * (3 * N2I);
                cx<T> pc[CH], pm[CH], w0[CH], w1[CH];
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    pc[c] = Pb[c * PCHF + eP];
                    pm[c] = Pb[c * PCHF + ePm];
                }
                // the Nyquist-plane values, read with the partials (every lane, the
                // lanes off the planes all at one address) rather than after them
#pragma unroll
                for (int j = 0; j < CH; ++j) {
                    w0[j] = Vb[wi[j]];
                    w1[j] = Vb[wi[j] + 1];
                }
#pragma unroll
                for (int j = 0; j < CH; ++j) {
                    const int kx = kxp + j * NP, kxm = (N - kx) % N;
                    cx<T> Z = pc[0], Zm = pm[0];
#pragma unroll
                    for (int c = 1; c < CH; ++c) {
                        cmac(Z, a.tw[kx * CH + c], pc[c]);
                        cmac(Zm, a.tw[kxm * CH + c], pm[c]);
                    }
                    cx<T> v[2];
                    if (nyq[j]) {
                        const cx<T> w = wodd[j] ? w1[j] : w0[j];
                        split_w<T>(w, wself[j] ? w : (wodd[j] ? w0[j] : w1[j]), v);
                    }
                    const T u0x = T(0.5) * (Z.x + Zm.x), u0y = T(0.5) * (Z.y - Zm.y);
                    const T u1x = T(0.5) * (Z.y + Zm.y), u1y = T(0.5) * (Zm.x - Z.x);
#pragma unroll
                    for (int sl = 0; sl < SMAX; ++sl) {
                        if (sl == s0) vss_accumulate<T, T>(acc[u][sl][j], h0[j], a0[j], u0x, u0y, u1x, u1y, nyq[j], v);
                        if (sl == s1) vss_accumulate<T, T>(acc[u][sl][j], h1[j], a1[j], u0x, u0y, u1x, u1y, nyq[j], v);
                    }
                }
            }
        }
    }

    int k2[CH];
    auto sq = [](int k) {
        const int mk = k < N / 2 ? k : k - N;
        return mk * mk;
    };
#pragma unroll
    for (int j = 0; j < CH; ++j) k2[j] = sq(kxp + j * NP) + sq(ky) + sq(kz);
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int b = b0 + u;
        if (b >= a.nb) break;
#pragma unroll
        for (int sl = 0; sl < SMAX; ++sl) {
            if (sl >= a.nslots) break;
            const int* sd = a.slots + 5 * sl;
            const int l0 = sd[3], nl = sd[4];
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
            const int64_t ob = (int64_t(b) * a.nslots + sl) * (N2 * KZH);
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int64_t o = ob + (int64_t(kxp + j * NP) * N + ky) * KZH + kz;
                a.Gt[o] = cx<T>{T(acc[u][sl][j].x), T(acc[u][sl][j].y)};
                a.Lt[o] = lac[j];
            }
        }
    }
}

// ====================================================== inverse transform + combine
// The inverse transform of the gain and loss spectra (Hermitian, the k_z <= N/2 half
// stored): the x- and y-passes run on the half in place (half_pass_kernel); the z-pass
// restores each row's conjugate half, transforms it and keeps the real part, fused with
// the combination Q = g - f_i l of the slot's species i (zpass_combine_kernel).
template <typename T, int N, int AXIS>
__global__ __launch_bounds__(256) void half_pass_kernel(cx<T>* data, int64_t npencils) {
    constexpr int KZH = N / 2 + 1;
    constexpr int64_t NH = int64_t(N) * N * KZH;
    const int64_t pid = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (pid >= npencils) return;
    const int64_t field = pid / (N * KZH);
    const int r = int(pid - field * (N * KZH));
    int64_t base, stride;
    if constexpr (AXIS == 0) {  // r = (k_y, k_z)
        base = field * NH + r;
        stride = int64_t(N) * KZH;
    } else {                    // r = (x, k_z)
        base = field * NH + int64_t(r / KZH) * (N * KZH) + (r % KZH);
        stride = KZH;
    }
    cx<T> v[N];
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = data[base + k * stride];
    fft<N, +1>(v);
#pragma unroll
    for (int k = 0; k < N; ++k) data[base + k * stride] = v[k];
}

template <typename T, int N>
__global__ __launch_bounds__(256) void zpass_combine_kernel(const cx<T>* __restrict__ Gh,
                                                            const cx<T>* __restrict__ Lh, const T* __restrict__ f,
                                                            T* __restrict__ Q, const int* __restrict__ slots,
                                                            int nslots, int s, int64_t nrows) {
    constexpr int KZH = N / 2 + 1;
    constexpr int64_t N2 = int64_t(N) * N, N3 = N2 * N;
    const int64_t row = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (row >= nrows) return;
    const int64_t bs = row / N2;         // (node, slot)
    const int64_t xy = row - bs * N2;
    const int slot = int(bs % nslots);
    const int64_t b = bs / nslots;
    const int sp = slots[5 * slot];
    const cx<T>* g = Gh + row * KZH;
    const cx<T>* l = Lh + row * KZH;
    cx<T> vg[N], vl[N];
#pragma unroll
    for (int k = 0; k < KZH; ++k) {
        vg[k] = g[k];
        vl[k] = l[k];
    }
#pragma unroll
    for (int k = KZH; k < N; ++k) {
        vg[k] = cx<T>{vg[N - k].x, -vg[N - k].y};
        vl[k] = cx<T>{vl[N - k].x, -vl[N - k].y};
    }
    fft<N, +1>(vg);
    fft<N, +1>(vl);
    const T* fr = f + (b * s + sp) * N3 + xy * N;
    T* q = Q + bs * N3 + xy * N;
#pragma unroll
    for (int z = 0; z < N; ++z) q[z] = vg[z].x - fr[z] * vl[z].x;
}

// The gain stage of FP32 VHS plans at N = 32 on the matrix cores (gain_mfma.hip, geometry
// (2, 0)): prepares each (node, species) input in `prep` (mfma_prep_bytes per pair) and
// writes the chunk partials P exactly as gain_kernel<float, 32, 2, 1> lays them out.
hipError_t launch_gain_mfma32(const dgfs_plan& p, const float* f, cx<float>* P, void* prep, int nb, hipStream_t st);

namespace detail {

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ev (optional): 6 events recorded at the stage boundaries (start, after forward FFT,
// after gain, after radial, after the inverse x/y passes, after the z-pass + combine).
// MF: the gain stage runs on the matrix cores (FP32, N = 32, VHS only).
template <typename T, int N, int CH, int CZ, bool PIPE, bool PACK, bool VSS, bool MF = false>
hipError_t run_slice(const dgfs_plan& p, const T* f, T* Q, int nb, void* ws, bool pairs, hipStream_t st,
                     hipEvent_t* ev) {
    static_assert(!MF || (std::is_same_v<T, float> && N == 32 && CH == 2 && !VSS), "matrix-core gain: FP32 VHS N = 32");
    constexpr int MODE = VSS ? GAIN_VSS : GAIN_REAL;
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
    w += align256(sizeof(cx<T>) * int64_t(nb) * ncls * p.nrho * (VSS ? N3 : (N3 / N) * (N / 2 + 1)));
    T* PL = nullptr;
    cx<T>* Vn = nullptr;
    if constexpr (VSS) {
        PL = reinterpret_cast<T*>(w);
        w += align256(sizeof(T) * int64_t(nb) * ncls * p.nrho * 2 * (2 + CH) * N * N);
        Vn = reinterpret_cast<cx<T>*>(w);
        w += align256(sizeof(cx<T>) * int64_t(nb) * ncls * p.nrho * 3 * N * N);
    }
    constexpr int64_t NH = int64_t(N) * N * (N / 2 + 1);  // stored half of a spectrum
    cx<T>* Gt = reinterpret_cast<cx<T>*>(w);
    cx<T>* Lt = Gt + int64_t(nb) * ss.nslots * NH;  // contiguous with Gt

    const char* dev = static_cast<const char*>(p.dev);
    mark(0);
    hipError_t e = fft3d<T, N>(fhat, f, int64_t(nb) * p.s, -1, T(1.0 / double(N3)), st);
    if (e != hipSuccess) return e;
    mark(1);

    GainArgs<T> ga;
    ga.fhat = fhat;
    ga.P = P;
    ga.PL = PL;
    ga.kx = reinterpret_cast<const cx<T>*>(dev + p.off_kx);
    ga.yz = reinterpret_cast<const cx<T>*>(dev + p.off_yz);
    ga.nyq = reinterpret_cast<const T*>(dev + p.off_nyq);
    ga.cls = reinterpret_cast<const int*>(dev + p.off_cls);
    ga.wdir = reinterpret_cast<const T*>(dev + p.off_wdir);
    ga.s = p.s;
    ga.ncls = ncls;
    ga.nrho = p.nrho;
    ga.nb = nb;
    if constexpr (MF) {
        // the prepared inputs follow the loss spectra
        char* prep = reinterpret_cast<char*>(Lt + int64_t(nb) * ss.nslots * NH);
        prep += (256 - reinterpret_cast<uintptr_t>(prep) % 256) % 256;
        if ((e = launch_gain_mfma32(p, f, P, prep, nb, st)) != hipSuccess) return e;
    } else {
        const int64_t ipn = int64_t(ncls) * p.nrho * CH;
        const int64_t groups = ((nb + 7) / 8) * 8 * ipn;
        gain_kernel<T, N, CH, CZ, PIPE, PACK, MODE><<<dim3(unsigned(groups)), dim3(GainK<T, N, CH, CZ>::NT), 0, st>>>(ga);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if constexpr (VSS) {
        nyquist_dft_kernel<T, N, CH><<<dim3(unsigned(int64_t(nb) * ncls * p.nrho)), dim3(3 * N), 0, st>>>(PL, Vn);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    mark(2);

    RadialArgs<T> ra;
    ra.P = P;
    ra.fhat = fhat;
    ra.Gt = Gt;
    ra.Lt = Lt;
    ra.F = reinterpret_cast<const T*>(dev + p.off_F);
    ra.Fv = reinterpret_cast<const cx<T>*>(dev + p.off_F);
    ra.V = Vn;
    ra.G = reinterpret_cast<const T*>(dev + p.off_G);
    ra.tw = reinterpret_cast<const cx<T>*>(dev + p.off_tw);
    ra.slots = reinterpret_cast<const int*>(dev + ss.off_slots);
    ra.gterms = reinterpret_cast<const int*>(dev + ss.off_gterms);
    ra.lterms = reinterpret_cast<const int*>(dev + ss.off_lterms);
    ra.cuses = reinterpret_cast<const int*>(dev + ss.off_cuses);
    ra.s = p.s;
    ra.ncls = ncls;
    ra.nrho = p.nrho;
    ra.nb = nb;
    ra.nslots = ss.nslots;
    ra.K2 = p.K2;
    const int64_t pch = int64_t(N / CH) * N * (N / 2 + 1);
    // VSS with few slots: the fused kernel (NB nodes x every slot per thread, accumulators
    // of NB x SMAX x CH complex doubles kept to at most 16 of them)
    constexpr int NB2 = (2 * CH <= 4) ? 4 : (2 * CH <= 8 ? 2 : 1);
    constexpr int NB4 = (4 * CH <= 4) ? 4 : (4 * CH <= 8 ? 2 : 1);
    const int64_t rthreads = int64_t(nb) * ss.nslots * pch;
    if constexpr (VSS) {
        if (ss.nslots <= 2) {
            const int64_t blocks = int64_t((nb + NB2 - 1) / NB2) * ((pch + 255) / 256);
            radial_vss_kernel<T, N, CH, NB2, 2><<<dim3(unsigned(blocks)), dim3(256), 0, st>>>(ra);
        } else if (ss.nslots <= 4) {
            const int64_t blocks = int64_t((nb + NB4 - 1) / NB4) * ((pch + 255) / 256);
            radial_vss_kernel<T, N, CH, NB4, 4><<<dim3(unsigned(blocks)), dim3(256), 0, st>>>(ra);
        } else {
            radial_kernel<T, N, CH, true><<<dim3(unsigned((rthreads + 255) / 256)), dim3(256), 0, st>>>(ra);
        }
    } else {
        radial_kernel<T, N, CH, false><<<dim3(unsigned((rthreads + 255) / 256)), dim3(256), 0, st>>>(ra);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    mark(3);

    {
        const int64_t np = 2 * int64_t(nb) * ss.nslots * N * (N / 2 + 1);
        half_pass_kernel<T, N, 0><<<dim3(unsigned((np + 255) / 256)), dim3(256), 0, st>>>(Gt, np);
        half_pass_kernel<T, N, 1><<<dim3(unsigned((np + 255) / 256)), dim3(256), 0, st>>>(Gt, np);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    mark(4);

    const int64_t rows = int64_t(nb) * ss.nslots * N * N;
    zpass_combine_kernel<T, N><<<dim3(unsigned((rows + 255) / 256)), dim3(256), 0, st>>>(
        Gt, Lt, f, Q, ra.slots, ss.nslots, p.s, rows);
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
hipError_t run_tiles_64(const dgfs_plan& p, const void* f, void* Q, int nb, void* ws, bool pairs, hipStream_t st,
                        hipEvent_t* ev);
// The same for plans with a VSS kernel (vss_<N>.hip).
hipError_t run_vss_16(const dgfs_plan& p, const void* f, void* Q, int nb, void* ws, bool pairs, hipStream_t st,
                      hipEvent_t* ev);
hipError_t run_vss_24(const dgfs_plan& p, const void* f, void* Q, int nb, void* ws, bool pairs, hipStream_t st,
                      hipEvent_t* ev);
hipError_t run_vss_32(const dgfs_plan& p, const void* f, void* Q, int nb, void* ws, bool pairs, hipStream_t st,
                      hipEvent_t* ev);
hipError_t run_vss_48(const dgfs_plan& p, const void* f, void* Q, int nb, void* ws, bool pairs, hipStream_t st,
                      hipEvent_t* ev);

}  // namespace dgfs
