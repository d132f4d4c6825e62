// The gain stage of Sec. 4 on the matrix cores, for FP32 plans with VHS kernels at N = 32
// (gain geometry (2, 0)).  It produces the same chunk partials as gain_kernel<float, 32, 2,
// 1>: for each (node, gain class, rho_q, x-chunk c) the partial forward DFT of
// S_q = sum_p w_p Re(A_p B_p) over the x-planes x = 2m + c.
//
// The shifted field A = f(v + a rho sigma) is formed in physical space as a separable
// operator, A = (R_x (x) R_y (x) R_z) f, with the N x N trigonometric-shift matrices
//   R(n, m) = (1/N) sum_{l=-N/2}^{N/2-1} e^{i l (2 pi (n-m)/N + theta)},
// theta = +-pi rho c sigma_d / L per axis (the same phases as the spectral form; the DFT
// index N/2 is the mode -N/2).  R = C + i s u u^T with C = Re R (circulant), s =
// -sin(N theta / 2) / N and u = ((-1)^n): the imaginary part is rank one.  Expanding the
// product over the three axes:
//   Re A = T - s_x s_y u_x u_y L_xy(z) - s_x s_z u_x u_z L_xz(y) - s_y s_z u_y u_z L_yz(x)
//   Im A = s_x u_x P_x(y,z) + s_y u_y P_y(x,z) + s_z u_z P_z(x,y) - s_x s_y s_z u_x u_y u_z a_xyz
// with T = C_x C_y C_z f, P_x = C_y C_z a_x, P_y = C_x C_z a_y, P_z = C_x C_y a_z,
// L_xy = C_z a_xy, L_xz = C_y a_xz, L_yz = C_x a_yz, where a_E is f summed with the signs
// (-1)^n over the axes in E.  T is three dense contractions (the MFMAs); the other terms
// are planes, lines and a scalar.  On one x-plane every term but T and s_x u_x P_x is a
// line in y times u_z or u_y times a line in z, so each of Re A and Im A gets its
// corrections from one more 32x32x16 product over four k-slots (corr_a, corr_b).
//
// Arithmetic: every MFMA operand is split as hi + lo in FP16 (hi = f16(v), lo = f16(v -
// hi)) and a product is hi*hi + hi*lo + lo*hi, accumulated in FP32 (about 2^-22 of each
// operand).  The input of each (node, species) is scaled by a power of two so that its
// largest value lies in [2^7, 2^8), which keeps every split operand in FP16's normal range
// (planes of alternating sums reach 2^13 times the shift matrices' row sums); the scale is
// undone in the class weight.
//
// Work item layout (512 threads = 8 wavefronts): wavefront w owns the x-planes m = 2w,
// 2w + 1 of the chunk; after the last contraction lane l of a wavefront holds, per plane,
// the rows y = 8(r/4) + 4(l/32) + r%4 (r < 16) at z = l%32 (the MFMA 32x32 output layout).
#include "gain.hpp"

namespace dgfs {
namespace mfma {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef float f8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

constexpr int N = 32;
constexpr int NT = 512;
constexpr int PST = 1032;                  // LDS plane stride of the x-contracted field (halves)
constexpr int VS = 36;                     // LDS row stride of the per-plane vectors (floats)
constexpr int TABW = 3 * 32;               // words per field table: [x, y, z][32] (hi | lo << 16)
constexpr int PREPH = 2 * 32768 + 2048;    // halves per (node, species): f hi, f lo, a_x hi, a_x lo
constexpr int AUX = 64;                    // floats per (node, species) after the halves
static_assert(size_t(PREPH) * 2 + AUX * 4 == mfma_prep_bytes, "prepared-input layout");

struct Args {
    const float* f;        // [nb][s][N^3] input (x-major, z fastest)
    _Float16* prep;        // [nb][s]: PREPH halves then AUX floats (mfma_prep_bytes each)
    const unsigned* tab;   // [dirs][nrho][2 fields][TABW]: r(j) = c(-j mod N) of each axis's
                           // shift-matrix real part C(n, m) = c((n - m) mod N), FP16 hi | lo << 16
    const float* sc;       // [dirs][nrho][2 fields][4]: s_x, s_y, s_z
    const int* cls;        // [ncls][4] = i, j, ndir, dir_offset
    const float* wdir;     // [ncls]
    cx<float>* P;          // chunk partials, as gain_kernel<float, 32, 2, 1>
    int s, ncls, nrho, nb;
};

__device__ __forceinline__ const _Float16* prep_h(const Args& a, int fs) {
    return reinterpret_cast<const _Float16*>(reinterpret_cast<const char*>(a.prep) + size_t(fs) * mfma_prep_bytes);
}
__device__ __forceinline__ const float* prep_aux(const Args& a, int fs) {
    return reinterpret_cast<const float*>(reinterpret_cast<const char*>(a.prep) + size_t(fs) * mfma_prep_bytes +
                                          size_t(PREPH) * 2);
}

// v = hi + lo with hi = f16(v) and lo = f16(v - hi); v - hi is exact in FP32, so lo takes
// one rounding.
__device__ __forceinline__ void split8(f8v v, h8& hi, h8& lo) {
    hi = __builtin_convertvector(v, h8);
    lo = __builtin_convertvector(v - __builtin_convertvector(hi, f8v), h8);
}
__device__ __forceinline__ void split4(f4v v, h4& hi, h4& lo) {
    hi = __builtin_convertvector(v, h4);
    lo = __builtin_convertvector(v - __builtin_convertvector(hi, f4v), h4);
}
__device__ __forceinline__ h8 ld8(const _Float16* p) { return *reinterpret_cast<const h8*>(p); }
// v plus v of lane l ^ 32 (l ^ 16): one v_permlane32_swap (v_permlane16_swap) exchanges the
// halves (rows), so the butterfly sums need no LDS crossbar round trip
__device__ __forceinline__ float sum_xor32(float v) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float sum_xor16(float v) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// 16-byte buffer load: wave-uniform descriptor, lane offset in a VGPR, uniform offset in
// an SGPR (no per-lane 64-bit addresses)
__device__ __forceinline__ h8 bld8(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(h8, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

// hi | lo << 16 of v in FP16 (hi = f16(v), lo = f16(v - hi)).
__device__ __forceinline__ unsigned split_pk(float v) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const _Float16 hi = _Float16(v);
    const _Float16 lo = _Float16(v - float(hi));
    return __builtin_bit_cast(unsigned, h2{hi, lo});
}
// Operands of a rank-two term u_y b(z) + a(y) u_z of a 32 x 32 tile (u = (-1)^n), one
// 32x32x16 product over k-slots 0..3: A[y][k] = (u_y, u_y, a_hi(y), a_lo(y)) and B[k][z] =
// (b_hi(z), b_lo(z), u_z, u_z).  Lane l < 32 supplies y = z = l; uu = (u_l, u_l) in FP16 on
// those lanes and 0 elsewhere, which zeroes the other lanes' (finite) k-slots.
__device__ __forceinline__ h8 corr_a(unsigned uu, float av) {
    return __builtin_bit_cast(h8, u4v{uu, split_pk(av), 0u, 0u});
}
__device__ __forceinline__ h8 corr_b(unsigned uu, float bv) {
    return __builtin_bit_cast(h8, u4v{split_pk(bv), uu, 0u, 0u});
}

#define MF32(a, b, c) __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0)
#define MF16(a, b, c) __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0)

// ------------------------------------------------------------------ input preparation
// One workgroup of 1024 threads per (node, species): the scale 2^k, f hi/lo transposed to [col = (y, z)][x]
// (the A operand of the x-contraction), a_x = sum_x (-1)^x f as hi/lo [y][z], then
// a_xz(y) = sum_z (-1)^z a_x(y, z) with its own scale, a_xyz, and 2^-k.
// aux: [0, 32) a_xz(y) * 2^-j, [32] a_xyz, [33] 2^-k, [34] 2^j.
constexpr int PT = 1024;   // threads of the preparation kernel: one per (y, z) column
__global__ __launch_bounds__(PT) void prep_kernel(Args a) {
    const int fs = blockIdx.x, tid = threadIdx.x;
    const float* f = a.f + size_t(fs) * (N * N * N);
    _Float16* out = reinterpret_cast<_Float16*>(reinterpret_cast<char*>(a.prep) + size_t(fs) * mfma_prep_bytes);
    float* aux = reinterpret_cast<float*>(out + PREPH);
    __shared__ float red[PT];
    __shared__ float ax[N * N];
    __shared__ float axz[N];
    float mx = 0.f;
    for (int i = tid; i < N * N * N; i += PT) mx = fmaxf(mx, fabsf(f[i]));
    red[tid] = mx;
    __syncthreads();
    for (int k = PT / 2; k > 0; k >>= 1) {
        if (tid < k) red[tid] = fmaxf(red[tid], red[tid + k]);
        __syncthreads();
    }
    const float M = red[0];
    int e = 0;
    if (M > 0.f && M <= 3.0e38f) (void)frexpf(M, &e);   // M = m 2^e, m in [0.5, 1)
    const int k = (M > 0.f && M <= 3.0e38f) ? max(-120, min(120, 8 - e)) : 0;
    const float scale = ldexpf(1.f, k);
    for (int col = tid; col < N * N; col += PT) {
        const int y = col >> 5, z = col & 31;
        float acc = 0.f;
#pragma unroll
        for (int xb = 0; xb < 4; ++xb) {
            f8v v;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int x = 8 * xb + j;
                v[j] = f[(x * N + y) * N + z] * scale;
                acc += (x & 1) ? -v[j] : v[j];
            }
            h8 hi, lo;
            split8(v, hi, lo);
            *reinterpret_cast<h8*>(out + col * 32 + 8 * xb) = hi;
            *reinterpret_cast<h8*>(out + 32768 + col * 32 + 8 * xb) = lo;
        }
        ax[col] = acc;
        const _Float16 h = _Float16(acc);
        out[65536 + col] = h;
        out[65536 + 1024 + col] = _Float16(acc - float(h));
    }
    __syncthreads();
    if (tid < N) {
        float acc = 0.f;
        for (int z = 0; z < N; ++z) acc += (z & 1) ? -ax[tid * N + z] : ax[tid * N + z];
        axz[tid] = acc;
    }
    __syncthreads();
    __shared__ float colscale;
    if (tid == 0) {
        float axyz = 0.f, am = 0.f;
        for (int y = 0; y < N; ++y) {
            axyz += (y & 1) ? -axz[y] : axz[y];
            am = fmaxf(am, fabsf(axz[y]));
        }
        int ej = 0;
        if (am > 0.f && am <= 3.0e38f) (void)frexpf(am, &ej);
        colscale = ldexpf(1.f, (am > 0.f && am <= 3.0e38f) ? max(-120, min(120, 8 - ej)) : 0);
        aux[32] = axyz;
        aux[33] = ldexpf(1.f, -k);
        aux[34] = colscale;
    }
    __syncthreads();
    if (tid < N) aux[tid] = axz[tid] * colscale;
}

// ------------------------------------------------------------------ gain kernel
struct Lds {
    // The small arrays first: their addresses stay below 64 KB, within the reach of the
    // LDS instructions' immediate offsets.
    unsigned Cv[3][3][2][64];      // shift vectors r of three fields in flight, [axis][hi, lo]: word o
                                   // holds r(o mod 32) and r((o + 1) mod 32) in FP16
    float Lxy[3][32];
    float Px[3][4 * 64 * 4];       // s_x u_x P_x in the output layout, three fields in flight
    float W[8][2][3 * VS];         // per wavefront and field: C_y v_2w, C_y v_2w+1, C_y a_xz
    float V[2][17 * VS];           // [buffer]: v_m(y) = sum_z (-1)^z (C_x f)(x_m, y, z), then a_xz(y)
    _Float16 G1[2][2][16 * PST];   // x-contracted field [buffer][hi, lo][plane]: rows y, 16-byte
                                   // blocks of z rotated by y/4 (conflict-free row reads)
};
static_assert(sizeof(Lds) <= 160 * 1024, "LDS");

__device__ __forceinline__ int g1off(int m, int y, int blk) { return m * PST + y * 32 + ((blk + (y >> 2)) & 3) * 8; }

// Thread t < 96 of a table (axis t / 32, j = t % 32) holds v = r(j) and vn = r(j + 1) as
// hi | lo << 16 and writes the words j and j + 32 of its axis in buffer cb.
__device__ __forceinline__ void put_vectors(Lds& L, int cb, int t, unsigned v, unsigned vn) {
    const int ax = t >> 5, j = t & 31;
    const unsigned wh = __builtin_amdgcn_perm(vn, v, 0x05040100u);   // hi(r(j)) | hi(r(j + 1)) << 16
    const unsigned wl = __builtin_amdgcn_perm(vn, v, 0x07060302u);
    L.Cv[cb][ax][0][j] = wh;
    L.Cv[cb][ax][0][j + 32] = wh;
    L.Cv[cb][ax][1][j] = wl;
    L.Cv[cb][ax][1][j + 32] = wl;
}
__device__ __forceinline__ int next_entry(int t) { return (t & ~31) | ((t + 1) & 31); }
// Write the shift vectors of table tb into LDS buffer cb (threads 0..95).
__device__ __forceinline__ void stage_vectors(const Args& a, int tb, Lds& L, int cb) {
    const int t = threadIdx.x;
    if (t < TABW) put_vectors(L, cb, t, a.tab[size_t(tb) * TABW + t], a.tab[size_t(tb) * TABW + next_entry(t)]);
}
// An operand of 8 matrix entries of one axis in FP16 hi and lo: two runs of four,
// r(o1..o1+3) and r(o2..o2+3) (0 <= o1, o2 < 32), two words each.
__device__ __forceinline__ void vec_operand(const unsigned (*v)[64], int o1, int o2, h8& hi, h8& lo) {
    const unsigned* p1 = &v[0][o1];
    const unsigned* p2 = &v[0][o2];
    hi = __builtin_bit_cast(h8, u4v{p1[0], p1[2], p2[0], p2[2]});
    lo = __builtin_bit_cast(h8, u4v{p1[64], p1[66], p2[64], p2[66]});
}
// B operand of the x-contraction (16x16x32, k = x' = 8g + e, n = m): C_x[2m + c][x'] =
// r_x((x' - 2m - c) mod N).
__device__ __forceinline__ void op_x(const Lds& L, int cb, int c, h8& hi, h8& lo) {
    const int l = threadIdx.x & 63, g = l >> 4, m = l & 15;
    const int o = (8 * g - 2 * m - c) & 31;
    vec_operand(L.Cv[cb][0], o, o + 4, hi, lo);
}
// B operand of the z-contraction (32x32x16, k = z = 16s + 8h + e, n = z_out = l%32):
// C_z[z_out][z] = r_z((z - z_out) mod N).
__device__ __forceinline__ void op_z(const Lds& L, int cb, int s, h8& hi, h8& lo) {
    const int l = threadIdx.x & 63, h = l >> 5, l32 = l & 31;
    const int o = (16 * s + 8 * h - l32) & 31;
    vec_operand(L.Cv[cb][2], o, o + 4, hi, lo);
}
// A operand of the y-contraction (32x32x16, row y_out = l%32, k-slot (s, h, e) = the row
// 8(r/4) + 4h + r%4, r = 8s + e, of the previous output): C_y[y_out][y] = r_y((y - y_out) mod N).
__device__ __forceinline__ void op_y(const Lds& L, int cb, int s, h8& hi, h8& lo) {
    const int l = threadIdx.x & 63, h = l >> 5, l32 = l & 31;
    vec_operand(L.Cv[cb][1], (16 * s + 4 * h - l32) & 31, (16 * s + 8 + 4 * h - l32) & 31, hi, lo);
}

// s_x u_x P_x = s_x u_x C_y C_z a_x in the output layout (kx = s_x u_x of the field) and
// L_xy = C_z a_xy of one field (one wavefront).
// The a_x plane's A operands of one field (rows y = l%32, z = 16s + 8(l/32) + e).
__device__ __forceinline__ void load_alpha(const Args& a, int fs, h8* ah, h8* al) {
    const int l = threadIdx.x & 63, h = l >> 5, l32 = l & 31;
    const _Float16* aH = prep_h(a, fs) + 65536;
    const _Float16* aL = aH + 1024;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        ah[s] = ld8(aH + l32 * 32 + 16 * s + 8 * h);
        al[s] = ld8(aL + l32 * 32 + 16 * s + 8 * h);
    }
}
__device__ __forceinline__ void alpha_plane(const h8* ah, const h8* al, int cb, Lds& L, int pb, float kx) {
    const int l = threadIdx.x & 63, h = l >> 5, l32 = l & 31;
    f16v dA = {};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        h8 bzh, bzl;
        op_z(L, cb, s, bzh, bzl);
        dA = MF32(ah[s], bzh, dA);
        dA = MF32(ah[s], bzl, dA);
        dA = MF32(al[s], bzh, dA);
    }
    float a1 = 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) a1 += (r & 1) ? -dA[r] : dA[r];
    a1 = sum_xor32(a1);
    if (h == 0) L.Lxy[pb][l32] = a1;
    f16v px = {};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        h8 tyh, tyl;
        op_y(L, cb, s, tyh, tyl);
        f8v va;
#pragma unroll
        for (int e = 0; e < 8; ++e) va[e] = dA[8 * s + e];
        h8 ph, pl;
        split8(va, ph, pl);
        px = MF32(tyh, ph, px);
        px = MF32(tyh, pl, px);
        px = MF32(tyl, ph, px);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
        *reinterpret_cast<f4v*>(&L.Px[pb][(j * 64 + l) * 4]) =
            f4v{kx * px[4 * j], kx * px[4 * j + 1], kx * px[4 * j + 2], kx * px[4 * j + 3]};
}

// What the first field of a direction leaves for the second: Re A and the pieces of its
// Im A (P_z stays in the wavefront's LDS area, s_x u_x P_x in its buffer).
struct FieldState {
    f16v T[2];       // Re A of the two planes
    float py[2];     // P_y(x_m, z)
    float sy, sz, pnt;
};

// The x-contraction of one field (between two barriers).  fs: (node, species) index of
// the input, c: chunk, bf: G1/V buffer, pb: the field's shift-vector buffer (the P_x
// buffer index: both are per field in flight); nxt_tb >= 0: the table of the field after
// it, whose shift vectors go to (pb + 1) % 3 (last read by the field before the previous
// one, which every wavefront finished before the previous barrier).
// Also gathers what the rest of the field needs (zy: the z and y operands, the Nyquist
// coefficients, a_xyz and the a_xz column's scale) before the barrier, so that those reads
// overlap the wait.
struct ZYOps {
    h8 bzh[2], bzl[2], tyh[2], tyl[2];
    float sx, sy, sz, axyz, colscale;
};
__device__ __forceinline__ void x_stage(const Args& a, int fs, int tb, int c, Lds& L, int bf, int pb, int nxt_tb,
                                        ZYOps& zy) {
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, mm = l & 15;
    const _Float16* fH = prep_h(a, fs);
    // Global reads first, consumed late: the operands of the contraction (all sixteen
    // loads before the first product), the next field's shift vectors, the field's scalars.
    const __amdgpu_buffer_rsrc_t rf = __builtin_amdgcn_make_buffer_rsrc(const_cast<_Float16*>(fH), 0, 2 * 65536, 0x00020000);
    const int vx = ((4 * w * 32 + mm) * 32 + 8 * g) * 2;   // this lane's bytes within a tile
    h8 xh[8], xl[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int so = ((t >> 1) * 32 + 16 * (t & 1)) * 64;  // the tile's (y, z) columns, 64 bytes each
        xh[t] = bld8(rf, vx, so);
        xl[t] = bld8(rf, vx, so + 65536);
    }
    const bool stage = nxt_tb >= 0 && tid < TABW;
    const unsigned vnext = stage ? a.tab[size_t(nxt_tb) * TABW + tid] : 0u;
    const unsigned vnext1 = stage ? a.tab[size_t(nxt_tb) * TABW + next_entry(tid)] : 0u;
    const float* aux = prep_aux(a, fs);
    const float vaux = (w == 1 && l < 32) ? aux[l] : 0.f;
    zy.sx = a.sc[4 * tb];
    zy.sy = a.sc[4 * tb + 1];
    zy.sz = a.sc[4 * tb + 2];
    zy.axyz = aux[32];
    zy.colscale = aux[34];
    // G1[m][y][z] = sum_x' C_x[2m + c][x'] f[x'][y][z]; 16x16x32 tiles of 16 (y, z)
    // columns, lane (m = l%16, g = l/16) keeping z = 16 tt + 4 g + r.  The G1 buffer bf was
    // last read by the field before the previous one.
    h8 bxh, bxl;
    op_x(L, pb, c, bxh, bxl);
    f4v X[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) X[t] = MF16(xh[t], bxh, (f4v{}));
#pragma unroll
    for (int t = 0; t < 8; ++t) X[t] = MF16(xh[t], bxl, X[t]);
#pragma unroll
    for (int t = 0; t < 8; ++t) X[t] = MF16(xl[t], bxh, X[t]);
    _Float16* GH = L.G1[bf][0];
    _Float16* GL = L.G1[bf][1];
#pragma unroll
    for (int yi = 0; yi < 4; ++yi) {
        const int y = 4 * w + yi;
        float vpart = 0.f;
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const f4v acc = X[2 * yi + tt];
            vpart += acc[0] - acc[1] + acc[2] - acc[3];
            h4 hi, lo;
            split4(acc, hi, lo);
            const int o = g1off(mm, y, 2 * tt + (g >> 1)) + 4 * (g & 1);
            *reinterpret_cast<h4*>(&GH[o]) = hi;
            *reinterpret_cast<h4*>(&GL[o]) = lo;
        }
        vpart = sum_xor32(sum_xor16(vpart));
        if (g == 0) L.V[bf][mm * VS + y] = vpart;
    }
    if (w == 1 && l < 32) L.V[bf][16 * VS + l] = vaux;
    if (stage) put_vectors(L, (pb + 1) % 3, tid, vnext, vnext1);   // the next field's shift vectors
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        op_z(L, pb, s, zy.bzh[s], zy.bzl[s]);
        op_y(L, pb, s, zy.tyh[s], zy.tyl[s]);
    }
}

// The rest of one field, after the barrier that publishes its G1 and V: the wavefront
// nxt_wave prepares the next field's P_x (input nxt_fs, table nxt_tb), then each
// wavefront's plane vectors go through C_y, its two planes through the z- and
// y-contractions and the corrections.  tb: the
// field's table, bf: its G1/V buffer (0: first field of the direction, 1: second), pb/pbA:
// the P_x (and shift-vector) buffers of this field and of the direction's first field.
// ACC = false keeps the field in st; ACC = true accumulates S += Re A Re B - Im A Im B
// with A from st and B this field.
template <bool ACC>
__device__ __forceinline__ void yz_stage(const Args& a, int fs, int tb, int c, Lds& L, int bf, int pb, int pbA,
                                         const ZYOps& zy, FieldState& st, int nxt_wave, int nxt_fs, int nxt_tb,
                                         float (*S)[16]) {
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, h = l >> 5, l32 = l & 31;
    const float sx = zy.sx, sy = zy.sy, sz = zy.sz;
    _Float16* GH = L.G1[bf][0];
    _Float16* GL = L.G1[bf][1];
    const h8* bzh = zy.bzh;
    const h8* bzl = zy.bzl;
    const h8* tyh = zy.tyh;
    const h8* tyl = zy.tyl;
    // the next field's P_x (its buffer was last read before the previous barrier)
    if (w == nxt_wave) {
        h8 ah[2], al[2];
        load_alpha(a, nxt_fs, ah, al);
        alpha_plane(ah, al, (pb + 1) % 3, L, (pb + 1) % 3, a.sc[4 * nxt_tb] * ((c & 1) ? -1.f : 1.f));
    }
    // ---- C_y [v_2w | v_2w+1 | a_xz]: this wavefront's P_z(x_m, y) and L_xz(y); L_yz(x_m)
    float lyz0, lyz1;
    {
        const int n = l32;
        const int row = n == 0 ? 2 * w : n == 1 ? 2 * w + 1 : 16;
        f16v d = {};
        float ly = 0.f;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            f8v v = {};
            if (n < 3) {
                const float* src = &L.V[bf][row * VS + 16 * s + 4 * h];
                const f4v v0 = *reinterpret_cast<const f4v*>(src), v1 = *reinterpret_cast<const f4v*>(src + 8);
                v = f8v{v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3]};
                ly += v0[0] - v0[1] + v0[2] - v0[3] + v1[0] - v1[1] + v1[2] - v1[3];
            }
            h8 bh, bl;
            split8(v, bh, bl);
            d = MF32(tyh[s], bh, d);
            d = MF32(tyh[s], bl, d);
            d = MF32(tyl[s], bh, d);
        }
        ly = sum_xor32(ly);
        lyz0 = __builtin_amdgcn_readlane(ly, 0);
        lyz1 = __builtin_amdgcn_readlane(ly, 1);
        if (n < 3) {
            const float un = n == 2 ? zy.colscale : 1.f;   // the a_xz column was stored times 2^j
            const float inv = 1.f / un;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                *reinterpret_cast<f4v*>(&L.W[w][bf][n * VS + 8 * j + 4 * h]) =
                    f4v{d[4 * j] * inv, d[4 * j + 1] * inv, d[4 * j + 2] * inv, d[4 * j + 3] * inv};
        }
    }
    // ---- z- then y-contraction of this wavefront's two planes, with the corrections (signs:
    // u_x = (-1)^c for every plane of the chunk, u_y by the row's parity r%2, u_z by the
    // lane's parity) as rank-two products on the matrix cores:
    //   Re A = T + u_y b_re(z) + a_re(y) u_z,   b_re = -(s_x s_y u_x L_xy + s_y s_z u_z L_yz(x_m)),
    //                                           a_re = -s_x s_z u_x L_xz,
    //   Im A = s_x u_x P_x + u_y b_im(z) + a_im(y) u_z,   b_im = s_y P_y(x_m) - s_x s_y s_z u_x u_z a_xyz,
    //                                                     a_im = s_z P_z(x_m).
    // Re A is formed in each field's own stage (its term starts the y-contraction's
    // accumulation); the first field keeps it with P_y, s_y and its a_xyz term, and the
    // second forms both fields' Im A and accumulates S += Re A Re B - Im A Im B (the class
    // weight is applied once at the end).
    const float ux = (c & 1) ? -1.f : 1.f, uz = (l & 1) ? -1.f : 1.f;
    const float pnt = sx * sy * sz * ux * uz * zy.axyz;
    const unsigned uu = l < 32 ? ((l & 1) ? 0xBC00BC00u : 0x3C003C00u) : 0u;
    const h8 aRe = corr_a(uu, -sx * sz * ux * L.W[w][bf][2 * VS + l32]);
    const float lxy = L.Lxy[pb][l32];
    // z-contraction of the two planes, their chains interleaved
    f16v d1[2] = {f16v{}, f16v{}};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        h8 ah[2], al[2];
#pragma unroll
        for (int pi = 0; pi < 2; ++pi) {
            const int o = g1off(2 * w + pi, l32, 2 * s + h);
            ah[pi] = ld8(GH + o);
            al[pi] = ld8(GL + o);
        }
#pragma unroll
        for (int pi = 0; pi < 2; ++pi) d1[pi] = MF32(ah[pi], bzh[s], d1[pi]);
#pragma unroll
        for (int pi = 0; pi < 2; ++pi) d1[pi] = MF32(ah[pi], bzl[s], d1[pi]);
#pragma unroll
        for (int pi = 0; pi < 2; ++pi) d1[pi] = MF32(al[pi], bzh[s], d1[pi]);
    }
    float py[2];
#pragma unroll
    for (int pi = 0; pi < 2; ++pi) {
        float a1 = 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r) a1 += (r & 1) ? -d1[pi][r] : d1[pi][r];
        py[pi] = sum_xor32(a1);   // P_y(x_m, z) = sum_y (-1)^y (C_x C_z f)
    }
    // y-contraction, interleaved likewise (Re A's rank-two term starts each chain)
    f16v d2[2];
#pragma unroll
    for (int pi = 0; pi < 2; ++pi)
        d2[pi] = MF32(aRe, corr_b(uu, -(sx * sy * ux * lxy + sy * sz * uz * (pi == 0 ? lyz0 : lyz1))), (f16v{}));
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        h8 bh[2], bl[2];
#pragma unroll
        for (int pi = 0; pi < 2; ++pi) {
            f8v v;
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = d1[pi][8 * s + e];
            split8(v, bh[pi], bl[pi]);
        }
#pragma unroll
        for (int pi = 0; pi < 2; ++pi) d2[pi] = MF32(tyh[s], bh[pi], d2[pi]);
#pragma unroll
        for (int pi = 0; pi < 2; ++pi) d2[pi] = MF32(tyh[s], bl[pi], d2[pi]);
#pragma unroll
        for (int pi = 0; pi < 2; ++pi) d2[pi] = MF32(tyl[s], bh[pi], d2[pi]);
    }
#pragma unroll
    for (int pi = 0; pi < 2; ++pi) {
        if constexpr (!ACC) {
            st.T[pi] = d2[pi];
            st.py[pi] = py[pi];
        } else {
            f16v pxB, pxA;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const f4v vb = *reinterpret_cast<const f4v*>(&L.Px[pb][(j * 64 + l) * 4]);
                const f4v va = *reinterpret_cast<const f4v*>(&L.Px[pbA][(j * 64 + l) * 4]);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    pxB[4 * j + i] = vb[i];
                    pxA[4 * j + i] = va[i];
                }
            }
            const f16v imB = MF32(corr_a(uu, sz * L.W[w][bf][pi * VS + l32]), corr_b(uu, sy * py[pi] - pnt), pxB);
            const f16v imA =
                MF32(corr_a(uu, st.sz * L.W[w][bf ^ 1][pi * VS + l32]), corr_b(uu, st.sy * st.py[pi] - st.pnt), pxA);
#pragma unroll
            for (int r = 0; r < 16; ++r) S[pi][r] = fmaf(-imA[r], imB[r], fmaf(st.T[pi][r], d2[pi][r], S[pi][r]));
        }
    }
    if constexpr (!ACC) {
        st.sy = sy;
        st.sz = sz;
        st.pnt = pnt;
    }
}

union alignas(16) Smem {
    Lds m;
    cx<float> buf[GainK<float, N, 2, 1>::LDS];
};

// Work items are dealt to the 8 XCDs round-robin; on one XCD, the items of NG nodes
// (b, b + 8, ...) run interleaved, same item next to each other, so that the nodes'
// prepared inputs and the item's shift tables are read from that XCD's L2.
constexpr int NG = 4;

__global__ __launch_bounds__(NT) void gain_kernel(Args a) {
    __shared__ Smem sm;
    Lds& L = sm.m;
    const int ipn = a.ncls * a.nrho * 2;
    const int gi = blockIdx.x;
    const int xcd = gi & 7, local = gi >> 3;
    const int grp = local / (ipn * NG), rem = local % (ipn * NG);
    const int b = (grp * NG + rem % NG) * 8 + xcd;
    if (b >= a.nb) return;
    int item = rem / NG;
    const int c = item % 2;
    item /= 2;
    const int q = item % a.nrho;
    const int cl = item / a.nrho;
    const int ci = a.cls[4 * cl], cj = a.cls[4 * cl + 1], ndir = a.cls[4 * cl + 2], doff = a.cls[4 * cl + 3];
    const int fA = b * a.s + ci, fB = b * a.s + cj;
    const int w = threadIdx.x >> 6;
    auto tab = [&](int d, int fld) { return ((doff + d) * a.nrho + q) * 2 + fld; };
    float S[2][16];
#pragma unroll
    for (int pi = 0; pi < 2; ++pi)
#pragma unroll
        for (int r = 0; r < 16; ++r) S[pi][r] = 0.f;
    // Field k of the work item: direction k / 2, first (A, species i) or second (B,
    // species j) field: its x-contraction, the barrier that publishes it, the rest.
    // (Running the stages of fields k and k + 1 in the other order on half of the
    // wavefronts, to pair one wavefront's matrix-core phases with the other's VALU phases
    // on each SIMD, measured 2 % slower.)
    stage_vectors(a, tab(0, 0), L, 0);
    __syncthreads();
    if (w == 0) {
        h8 ah[2], al[2];
        load_alpha(a, fA, ah, al);
        alpha_plane(ah, al, 0, L, 0, a.sc[4 * tab(0, 0)] * ((c & 1) ? -1.f : 1.f));
    }
    const int nf = 2 * ndir;
#pragma unroll 1
    for (int k = 0; k < nf; k += 2) {
        const int d = k / 2;
        FieldState st;
        ZYOps zy;
        x_stage(a, fA, tab(d, 0), c, L, 0, k % 3, tab(d, 1), zy);
        __syncthreads();
        yz_stage<false>(a, fA, tab(d, 0), c, L, 0, k % 3, 0, zy, st, (k + 1) % 8, fB, tab(d, 1), S);
        const bool more = k + 2 < nf;
        x_stage(a, fB, tab(d, 1), c, L, 1, (k + 1) % 3, more ? tab(d + 1, 0) : -1, zy);
        __syncthreads();
        yz_stage<true>(a, fB, tab(d, 1), c, L, 1, (k + 1) % 3, k % 3, zy, st, more ? (k + 2) % 8 : -1, fA,
                       more ? tab(d + 1, 0) : 0, S);
    }
    // the class weight and the undoing of both inputs' scales
    const float wgt = a.wdir[cl] * prep_aux(a, fA)[33] * prep_aux(a, fB)[33];
    __syncthreads();  // every wavefront is done with the contraction buffers
    // S_q to LDS as rows (plane m, y) of z values, then the forward transform of gain_kernel
    using K = GainK<float, N, 2, 1>;
    {
        const int l = threadIdx.x & 63, h = l >> 5;
#pragma unroll
        for (int pi = 0; pi < 2; ++pi)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int y = 8 * (r / 4) + 4 * h + r % 4;
                sm.buf[((2 * w + pi) * N + y) * K::ROW + (l & 31)] = cx<float>{wgt * S[pi][r], 0.f};
            }
    }
    __syncthreads();
    cx<float>* Pq = a.P + ((int64_t(b) * a.ncls + cl) * a.nrho + q) * int64_t(2) * K::NP * K::NPEN;
    store_partial<float, N, 2, 1, false>(sm.buf, Pq, c);
}

}  // namespace mfma

hipError_t launch_gain_mfma32(const dgfs_plan& p, const float* f, cx<float>* P, void* prep, int nb, hipStream_t st) {
    const char* dev = static_cast<const char*>(p.dev);
    mfma::Args a;
    a.f = f;
    a.prep = static_cast<_Float16*>(prep);
    a.tab = reinterpret_cast<const unsigned*>(dev + p.off_mtab);
    a.sc = reinterpret_cast<const float*>(dev + p.off_msc);
    a.cls = reinterpret_cast<const int*>(dev + p.off_cls);
    a.wdir = reinterpret_cast<const float*>(dev + p.off_wdir);
    a.P = P;
    a.s = p.s;
    a.ncls = int(p.classes.size());
    a.nrho = p.nrho;
    a.nb = nb;
    mfma::prep_kernel<<<dim3(unsigned(int64_t(nb) * p.s)), dim3(mfma::PT), 0, st>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t ipn = int64_t(a.ncls) * p.nrho * 2;
    const int64_t groups = ((nb + 8 * mfma::NG - 1) / (8 * mfma::NG)) * 8 * mfma::NG * ipn;
    mfma::gain_kernel<<<dim3(unsigned(groups)), dim3(mfma::NT), 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace dgfs
