// C ABI of the collision library: validation, host-side precomputation (FP64),
// upload of the plan tables, workspace slicing and launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "dgfs.h"
#include "plan.hpp"
#include "precompute.hpp"

namespace {

thread_local std::string g_err;

dgfs_status fail(dgfs_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

constexpr double kPi = 3.14159265358979323846264338327950288;

int signed_mode(int j, int N) { return j < N / 2 ? j : j - N; }

bool n_supported(int N) { return N == 16 || N == 24 || N == 32 || N == 48 || N == 64; }

dgfs_status check(const dgfs_problem* p) {
    if (!p) return fail(DGFS_EINVAL, "problem is NULL");
    if (p->s < 1 || p->s > 8) return fail(DGFS_EINVAL, "s must be in [1, 8]");
    if (!p->mass || !p->kernel) return fail(DGFS_EINVAL, "mass and kernel arrays are required");
    for (int i = 0; i < p->s; ++i)
        if (!(p->mass[i] > 0.0) || !std::isfinite(p->mass[i])) return fail(DGFS_EINVAL, "masses must be positive");
    if (p->L_species) {
        for (int i = 0; i < p->s; ++i)
            if (!(p->L_species[i] > 0.0) || !std::isfinite(p->L_species[i]))
                return fail(DGFS_EINVAL, "L_species must be positive");
    } else if (!(p->L > 0.0) || !std::isfinite(p->L)) {
        return fail(DGFS_EINVAL, "L must be positive");
    }
    if (p->N < 4 || p->N % 2 != 0) return fail(DGFS_EINVAL, "N must be even and >= 4");
    if (p->M != 6 && p->M != 12 && p->M != 24) return fail(DGFS_EINVAL, "no spherical design for this M (6, 12, 24)");
    if (p->n_rho < 1 || p->n_rho > 128) return fail(DGFS_EINVAL, "n_rho must be in [1, 128]");
    if (p->precision != DGFS_FP32 && p->precision != DGFS_FP64) return fail(DGFS_EINVAL, "unknown precision");
    for (int i = 0; i < p->s; ++i)
        for (int j = 0; j < p->s; ++j) {
            const dgfs_pair_kernel& k = p->kernel[i * p->s + j];
            const dgfs_pair_kernel& t = p->kernel[j * p->s + i];
            if (!(k.omega >= 0.5 && k.omega <= 1.0)) return fail(DGFS_EINVAL, "omega must be in [0.5, 1]");
            if (!(k.alpha >= 1.0 && k.alpha <= 2.0)) return fail(DGFS_EINVAL, "alpha must be in [1, 2]");
            if (!(k.prefactor > 0.0) || !std::isfinite(k.prefactor))
                return fail(DGFS_EINVAL, "prefactor must be positive");
            if (k.omega != t.omega || k.alpha != t.alpha || k.prefactor != t.prefactor)
                return fail(DGFS_EINVAL, "kernel must be symmetric in (i, j)");
        }
    if (!n_supported(p->N)) return fail(DGFS_EUNSUPPORTED, "N must be 16, 24, 32, 48 or 64");
    if (p->N == 64)
        for (int i = 0; i < p->s * p->s; ++i)
            if (p->kernel[i].alpha != 1.0) return fail(DGFS_EUNSUPPORTED, "VSS kernels need N <= 48");
    if (p->dealias != 0 && p->dealias != 1) return fail(DGFS_EINVAL, "dealias must be 0 or 1");
    if (p->dealias) {
        if (p->N != 16 && p->N != 24 && p->N != 32 && p->N != 48)
            return fail(DGFS_EUNSUPPORTED, "the dealiased form needs N = 16, 24, 32 or 48");
        for (int i = 0; i < p->s * p->s; ++i)
            if (p->kernel[i].alpha != 1.0) return fail(DGFS_EUNSUPPORTED, "the dealiased form needs alpha = 1");
        if (p->L_species)
            for (int i = 1; i < p->s; ++i)
                if (p->L_species[i] != p->L_species[0])
                    return fail(DGFS_EUNSUPPORTED, "the dealiased form needs one common grid");
        if (p->tile_ch != 0 || p->tile_cz != 0) return fail(DGFS_EUNSUPPORTED, "the dealiased form uses the default tile");
    }
    dgfs::GainGeometry g;
    if (!dgfs::gain_geometry(p->N, p->precision, &g))
        return fail(DGFS_EUNSUPPORTED, "no kernel for this N at this precision");
    if (p->tile_ch != 0 && p->tile_cz == 0)
        for (int i = 0; i < p->s * p->s; ++i)
            if (p->kernel[i].alpha != 1.0)
                return fail(DGFS_EUNSUPPORTED, "the matrix-core geometry (cz = 0) needs alpha = 1");
    if (p->tile_ch != 0 || p->tile_cz != 0) {
        dgfs::GainGeometry cand[16];
        const int n = dgfs::tile_candidates(p->N, p->precision, cand, 16);
        bool ok = false;
        for (int k = 0; k < n; ++k) ok = ok || (cand[k].CH == p->tile_ch && cand[k].CZ == p->tile_cz);
        if (!ok) return fail(DGFS_EUNSUPPORTED, "tile geometry not compiled for this N and precision");
    }
    return DGFS_OK;
}

// Whether the default geometry may be the matrix-core one: VHS kernels (alpha = 1) and
// the circular form.
bool matrix_default(const dgfs_problem* p) {
    if (p->dealias) return false;
    for (int i = 0; i < p->s * p->s; ++i)
        if (p->kernel[i].alpha != 1.0) return false;
    return true;
}

// Half-width of the box the ordered pair (i, j) is evaluated on: the common L, or with
// species-specific grids the wider of the two species' boxes.
double pair_box(const dgfs_problem* p, int i, int j) {
    return p->L_species ? std::max(p->L_species[i], p->L_species[j]) : p->L;
}

dgfs::PairParams pair_params(const dgfs_problem* p, int i, int j) {
    dgfs::PairParams pp;
    const double mi = p->mass[i], mj = p->mass[j];
    pp.a = mj / (mi + mj);
    pp.b = mi / (mi + mj);
    pp.gamma = 2.0 * (1.0 - p->kernel[i * p->s + j].omega);
    pp.C = p->kernel[i * p->s + j].prefactor;
    pp.alpha = p->kernel[i * p->s + j].alpha;
    pp.R = dgfs::pre::truncation_radius(pair_box(p, i, j), mi, mj);
    dgfs::pre::gauss_legendre(p->n_rho, pp.R, pp.rho, pp.wrho);
    return pp;
}

// Symmetric positive definite solve by Gauss-Jordan with partial pivoting: inverse of A (n x n).
bool invert(std::vector<double> A, int n, std::vector<double>& inv) {
    inv.assign(n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0.0) return false;
        for (int k = 0; k < n; ++k) {
            std::swap(A[c * n + k], A[piv * n + k]);
            std::swap(inv[c * n + k], inv[piv * n + k]);
        }
        const double d = A[c * n + c];
        for (int k = 0; k < n; ++k) {
            A[c * n + k] /= d;
            inv[c * n + k] /= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double fct = A[r * n + c];
            if (fct == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                A[r * n + k] -= fct * A[c * n + k];
                inv[r * n + k] -= fct * inv[c * n + k];
            }
        }
    }
    return true;
}

inline size_t detail_align(size_t x) { return (x + 255) & ~size_t(255); }

template <typename T>
void push_real(std::vector<char>& blob, size_t& off, const std::vector<double>& v) {
    off = (blob.size() + 255) & ~size_t(255);
    blob.resize(off + v.size() * sizeof(T));
    T* dst = reinterpret_cast<T*>(blob.data() + off);
    for (size_t k = 0; k < v.size(); ++k) dst[k] = T(v[k]);
}

template <typename T>
void push_cplx(std::vector<char>& blob, size_t& off, const std::vector<std::complex<double>>& v) {
    off = (blob.size() + 255) & ~size_t(255);
    blob.resize(off + v.size() * 2 * sizeof(T));
    T* dst = reinterpret_cast<T*>(blob.data() + off);
    for (size_t k = 0; k < v.size(); ++k) {
        dst[2 * k] = T(v[k].real());
        dst[2 * k + 1] = T(v[k].imag());
    }
}

void push_int(std::vector<char>& blob, size_t& off, const std::vector<int>& v) {
    off = (blob.size() + 255) & ~size_t(255);
    blob.resize(off + v.size() * sizeof(int));
    std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(int));
}

void push_double(std::vector<char>& blob, size_t& off, const std::vector<double>& v) { push_real<double>(blob, off, v); }

// FP64 conservation data: the inverse Gram matrix (A A^T)^{-1} of the s+4 invariant
// rows, then the masses and the grid half-widths.  Rows of A: h_i^3 on species i (s
// rows), m_i h_i^3 v_d (3 rows), m_i h_i^3 |v|^2 (1 row), with h_i = 2 L_i / N and
// v = -L_i + n h_i on species i's grid; A A^T in closed form from the power sums of the
// one-dimensional grid of each species.
std::vector<double> conserve_pack(const std::vector<double>& mass, const std::vector<double>& Ls, int N) {
    const int s = int(mass.size()), nr = s + 4;
    const double Nd = N;
    std::vector<double> Gm(nr * nr, 0.0);
    for (int i = 0; i < s; ++i) {
        const double L = Ls[i], h = 2.0 * L / N, h6 = std::pow(h, 6), m = mass[i];
        double S1 = 0, S2 = 0, S3 = 0, S4 = 0;
        for (int n = 0; n < N; ++n) {
            const double v = -L + n * h;
            S1 += v;
            S2 += v * v;
            S3 += v * v * v;
            S4 += v * v * v * v;
        }
        Gm[i * nr + i] = h6 * Nd * Nd * Nd;
        for (int d = 0; d < 3; ++d) Gm[i * nr + s + d] = Gm[(s + d) * nr + i] = m * h6 * Nd * Nd * S1;
        Gm[i * nr + s + 3] = Gm[(s + 3) * nr + i] = m * h6 * 3.0 * Nd * Nd * S2;
        const double m2h6 = m * m * h6;
        for (int d = 0; d < 3; ++d)
            for (int e = 0; e < 3; ++e) Gm[(s + d) * nr + s + e] += m2h6 * (d == e ? Nd * Nd * S2 : Nd * S1 * S1);
        for (int d = 0; d < 3; ++d) {
            const double x = m2h6 * (Nd * Nd * S3 + 2.0 * Nd * S1 * S2);
            Gm[(s + d) * nr + s + 3] += x;
            Gm[(s + 3) * nr + s + d] += x;
        }
        Gm[(s + 3) * nr + s + 3] += m2h6 * (3.0 * Nd * Nd * S4 + 6.0 * Nd * S2 * S2);
    }
    std::vector<double> inv;
    invert(Gm, nr, inv);
    inv.insert(inv.end(), mass.begin(), mass.end());
    inv.insert(inv.end(), Ls.begin(), Ls.end());
    return inv;
}

// Build every host table and lay it out in one byte blob for the device.
// Kernel-mode tables of one VSS class (up to two directions) for one target species,
// [nrho][2 directions][2][N][N][N/2+1] complex over the stored half k_z <= N/2: with
//   T1(q, k) = w_rho_q w_sigma F(mode of k, rho_q, sigma_eff) / N^3 and
//   T2(q, k) = conj of the same at the mode of the mirror index (-k) mod N,
// the entries are F_H = (T1 + T2)/2 and F_A = (T1 - T2)/2 (F_A vanishes unless k has a
// component at the Nyquist index, whose mirror is not the mode -k).  sigma_eff = sigma
// for the class's own ordering (i, j) and -sigma for the target j of an unlike class (its
// products are those of (j, i) at -sigma).  A like class that keeps one of each antipodal
// pair adds F(k, -sigma) = conj F(k, sigma): 2 Re F.  A missing second direction is zero.
void vss_table(const dgfs_plan& P, const dgfs::GainClass& c, bool own, const dgfs::PairParams& pp,
               std::vector<std::complex<double>>& out) {
    const int N = P.N, KZH = N / 2 + 1, nrho = P.nrho;
    const double n3 = double(N) * N * N, L = P.L;
    const bool like_half = c.i == c.j && P.antipodal;
    const double wsig = 4.0 * kPi / P.M;
    const size_t nrep = size_t(N) * N * KZH;
    const size_t base = out.size();
    out.resize(base + size_t(nrho) * 4 * nrep, std::complex<double>(0.0, 0.0));
    auto mode = [N](int idx) { return double(idx < N / 2 ? idx : idx - N); };
    const int K2 = P.K2;
    for (int q = 0; q < nrho; ++q) {
        // j_l(z) per |k|^2, shared by every direction and mode of this radial point
        const double rho = pp.rho[q];
        const double zmax = kPi * pp.a * rho * std::sqrt(double(K2 - 1)) / L;
        const int lmax = dgfs::pre::vss_terms(zmax);
        dgfs::pre::VssSeries S(pp.alpha, lmax);
        std::vector<std::vector<double>> jtab(K2);
        std::vector<int> nterm(K2);
        for (int k2 = 0; k2 < K2; ++k2) {
            const double z = kPi * pp.a * rho * std::sqrt(double(k2)) / L;
            nterm[k2] = std::min(lmax, dgfs::pre::vss_terms(z)) + 1;
            dgfs::pre::sph_bessel(nterm[k2] - 1, z, jtab[k2]);
        }
        const double pref = pp.C * std::pow(rho, pp.gamma + 2.0) * pp.wrho[q] * wsig / n3;
        for (int d = 0; d < c.ndir; ++d) {
            const double* s0 = &P.sigma[3 * c.dirs[d]];
            const double sg[3] = {own ? s0[0] : -s0[0], own ? s0[1] : -s0[1], own ? s0[2] : -s0[2]};
            auto Feff = [&](const double k[3]) {
                const int k2 = int(std::lround(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]));
                const double mu =
                    k2 > 0 ? (k[0] * sg[0] + k[1] * sg[1] + k[2] * sg[2]) / std::sqrt(double(k2)) : 0.0;
                double re, im;
                dgfs::pre::vss_sum(S, jtab[k2].data(), nterm[k2], mu, re, im);
                return like_half ? std::complex<double>(2.0 * re, 0.0) : std::complex<double>(re, im);
            };
            std::complex<double>* th = &out[base + ((size_t(q) * 2 + d) * 2 + 0) * nrep];
            std::complex<double>* ta = &out[base + ((size_t(q) * 2 + d) * 2 + 1) * nrep];
            for (int kx = 0; kx < N; ++kx)
                for (int ky = 0; ky < N; ++ky)
                    for (int kz = 0; kz < KZH; ++kz) {
                        const size_t o = (size_t(kx) * N + ky) * KZH + kz;
                        const double k[3] = {mode(kx), mode(ky), mode(kz)};
                        const std::complex<double> t1 = pref * Feff(k);
                        if (kx == N / 2 || ky == N / 2 || kz == N / 2) {
                            const double km[3] = {mode((N - kx) % N), mode((N - ky) % N), mode((N - kz) % N)};
                            const std::complex<double> t2 = pref * std::conj(Feff(km));
                            th[o] = 0.5 * (t1 + t2);
                            ta[o] = 0.5 * (t1 - t2);
                        } else {
                            th[o] = t1;  // F(-k) = conj F(k): no anti-Hermitian part
                        }
                    }
        }
    }
}

// Push a slot set's descriptors, with the per-class view of its gain terms (each class
// feeds at most two slots: its own ordering and, for an unlike pair, the mirrored one).
void push_uses(dgfs::SlotSet& S, int ncls, std::vector<char>& blob) {
    S.cuses.assign(size_t(ncls) * 4, -1);
    for (int sl = 0; sl < S.nslots; ++sl) {
        const int g0 = S.slots[5 * sl + 1], ng = S.slots[5 * sl + 2];
        for (int gi = g0; gi < g0 + ng; ++gi) {
            const int cl = S.gterms[2 * gi], ft = S.gterms[2 * gi + 1];
            int* u = &S.cuses[4 * size_t(cl)];
            if (u[0] < 0) {
                u[0] = sl;
                u[1] = ft;
            } else {
                u[2] = sl;
                u[3] = ft;
            }
        }
    }
    push_int(blob, S.off_slots, S.slots);
    push_int(blob, S.off_gterms, S.gterms);
    push_int(blob, S.off_lterms, S.lterms);
    push_int(blob, S.off_cuses, S.cuses);
}

// Matrix-core gain tables (geometry CZ = 0: FP32 VHS plans at N = 32).  The real part of
// each axis's shift matrix is circulant, C(n, m) = c((n - m) mod N) with
// c(d) = (1/N) sum_{l=-N/2}^{N/2-1} cos(l (2 pi d / N + theta)), theta as for the phases.
// Per (direction, rho, field) and axis x, y, z: r(j) = c(-j mod N) for j < N, each as one
// word FP16 hi | FP16 lo << 16 (hi = f16(v), lo = f16(v - hi), v = float(r(j))); then the
// Nyquist coefficients s = -sin(N theta / 2) / N of the three axes.
void build_mfma_tables(dgfs_plan& P, std::vector<char>& blob) {
    const int N = P.N, nrho = P.nrho;
    std::vector<uint32_t> tab(size_t(P.total_dirs) * nrho * 2 * 3 * N);
    std::vector<double> sc(size_t(P.total_dirs) * nrho * 2 * 4, 0.0);
    for (const auto& c : P.classes) {
        const dgfs::PairParams& pp = P.pair[c.i * P.s + c.j];
        for (int d = 0; d < c.ndir; ++d) {
            const double* sg = &P.sigma[3 * c.dirs[d]];
            for (int q = 0; q < nrho; ++q)
                for (int fld = 0; fld < 2; ++fld) {
                    const double sgn = fld == 0 ? 1.0 : -1.0, coef = fld == 0 ? c.a : c.b;
                    const size_t t = (size_t(c.dir_offset + d) * nrho + q) * 2 + fld;
                    for (int ax = 0; ax < 3; ++ax) {
                        const double th = sgn * kPi * pp.rho[q] * coef * sg[ax] / P.L;
                        for (int j = 0; j < N; ++j) {
                            const int dd = (N - j) % N;
                            double acc = 0.0;
                            for (int l = -N / 2; l < N / 2; ++l) acc += std::cos(l * (2.0 * kPi * dd / N + th));
                            const float v = float(acc / N);
                            const _Float16 hi = _Float16(v), lo = _Float16(v - float(hi));
                            uint16_t hb, lb;
                            std::memcpy(&hb, &hi, 2);
                            std::memcpy(&lb, &lo, 2);
                            tab[(t * 3 + ax) * N + j] = uint32_t(hb) | (uint32_t(lb) << 16);
                        }
                        sc[t * 4 + ax] = -std::sin(N * th / 2.0) / N;
                    }
                }
        }
    }
    P.off_mtab = (blob.size() + 255) & ~size_t(255);
    blob.resize(P.off_mtab + tab.size() * sizeof(uint32_t));
    std::memcpy(blob.data() + P.off_mtab, tab.data(), tab.size() * sizeof(uint32_t));
    push_real<float>(blob, P.off_msc, sc);
}

template <typename T>
void build_tables(dgfs_plan& P, std::vector<char>& blob) {
    const int N = P.N, s = P.s, nrho = P.nrho, CH = P.geo.CH, NP = N / CH;
    const double L = P.L;
    // ---------------- phase tables [dirs][nrho][2][CH][N] and [dirs][nrho][2][2][N]
    std::vector<std::complex<double>> kx(size_t(P.total_dirs) * nrho * 2 * CH * N);
    std::vector<std::complex<double>> yz(size_t(P.total_dirs) * nrho * 2 * 2 * N);
    std::vector<double> nyq(size_t(P.total_dirs) * nrho * 2);
    std::vector<int> cls;
    std::vector<double> wdir;
    std::vector<int> design_index;  // global direction -> design point
    for (const auto& c : P.classes) {
        cls.insert(cls.end(), {c.i, c.j, c.ndir, c.dir_offset});
        wdir.push_back(c.weight);
    }
    for (size_t k = 0; k < P.classes.size(); ++k) {
        const auto& c = P.classes[k];
        const dgfs::PairParams& pp = P.pair[c.i * s + c.j];
        const std::vector<int>& dirs = c.dirs;
        for (int d = 0; d < c.ndir; ++d) {
            const int gd = c.dir_offset + d;
            const double* sg = &P.sigma[3 * dirs[d]];
            for (int q = 0; q < nrho; ++q) {
                for (int fld = 0; fld < 2; ++fld) {
                    const double sgn = fld == 0 ? 1.0 : -1.0;
                    const double coef = fld == 0 ? c.a : c.b;
                    const double th[3] = {sgn * kPi * pp.rho[q] * coef * sg[0] / L,
                                          sgn * kPi * pp.rho[q] * coef * sg[1] / L,
                                          sgn * kPi * pp.rho[q] * coef * sg[2] / L};
                    const size_t base = (size_t(gd) * nrho + q) * 2 + fld;
                    for (int cc = 0; cc < CH; ++cc)
                        for (int t = 0; t < CH; ++t)
                            for (int l = 0; l < NP; ++l) {
                                const int jx = l + t * NP;
                                const double ang = th[0] * signed_mode(jx, N) +
                                                   2.0 * kPi * (double(t * cc) / CH + double(l * cc) / N);
                                kx[(base * CH + cc) * N + jx] = std::polar(1.0, ang);
                            }
                    nyq[base] = 2.0 * std::sin(th[0] * (N / 2));
                    for (int jj = 0; jj < N; ++jj) {
                        yz[(base * 2 + 0) * N + jj] = std::polar(1.0, th[1] * signed_mode(jj, N));
                        yz[(base * 2 + 1) * N + jj] = std::polar(1.0, th[2] * signed_mode(jj, N));
                    }
                }
            }
        }
    }
    push_cplx<T>(blob, P.off_kx, kx);
    push_cplx<T>(blob, P.off_yz, yz);
    if (P.geo.CZ == 0) build_mfma_tables(P, blob);
    push_real<T>(blob, P.off_nyq, nyq);
    push_int(blob, P.off_cls, cls);
    push_real<T>(blob, P.off_wdir, wdir);

    // ---------------- F tables per (class, target) and G tables per ordered pair
    const int K2 = P.K2;
    const double n3 = double(N) * N * N;
    std::vector<double> F;
    std::vector<std::complex<double>> Fv;
    std::vector<std::vector<int>> ftab(P.classes.size(), std::vector<int>(s, -1));
    int nft = 0;
    for (size_t k = 0; k < P.classes.size(); ++k) {
        const auto& c = P.classes[k];
        std::vector<int> targets = {c.i};
        if (c.i != c.j && P.antipodal) targets.push_back(c.j);
        for (int tg : targets) {
            const int other = tg == c.i ? c.j : c.i;
            if (!P.mask[tg * s + other]) continue;
            const dgfs::PairParams& pp = P.pair[tg * s + other];
            if (P.vss) {
                vss_table(P, c, tg == c.i, pp, Fv);
            } else {
                for (int q = 0; q < nrho; ++q)
                    for (int k2 = 0; k2 < K2; ++k2)
                        F.push_back(pp.wrho[q] *
                                    dgfs::pre::kernel_mode(std::sqrt(double(k2)), pp.rho[q], pp.a, pp.gamma, pp.C, L) /
                                    n3);
            }
            ftab[k][tg] = nft++;
        }
    }
    P.nftab = nft;
    std::vector<double> G(size_t(s) * s * K2);
    for (int i = 0; i < s; ++i)
        for (int j = 0; j < s; ++j) {
            const dgfs::PairParams& pp = P.pair[i * s + j];
            if (j < i) {  // G- depends on (C, gamma, R), all symmetric in (i, j)
                std::copy_n(&G[size_t(j * s + i) * K2], K2, &G[size_t(i * s + j) * K2]);
                continue;
            }
            for (int k2 = 0; k2 < K2; ++k2)
                G[size_t(i * s + j) * K2 + k2] = dgfs::pre::loss_weight(std::sqrt(double(k2)), pp.R, pp.gamma, pp.C, L) *
                                                 dgfs::pre::vss_loss_factor(pp.alpha);
        }
    P.ngtab = s * s;
    if (P.vss) push_cplx<T>(blob, P.off_F, Fv);
    else push_real<T>(blob, P.off_F, F);
    push_real<T>(blob, P.off_G, G);

    // ---------------- chunk-combine twiddles e^{-2 pi i kx c / N}, [N][CH]
    std::vector<std::complex<double>> tw(size_t(N) * CH);
    for (int kxi = 0; kxi < N; ++kxi)
        for (int cc = 0; cc < CH; ++cc) tw[kxi * CH + cc] = std::polar(1.0, -2.0 * kPi * double(kxi * cc % N) / N);
    push_cplx<T>(blob, P.off_tw, tw);

    // ---------------- slots: summed (one per species) and per ordered pair
    {
        dgfs::SlotSet& S = P.sum_slots;
        S = dgfs::SlotSet();
        S.nslots = s;
        for (int i = 0; i < s; ++i) {
            const int g0 = int(S.gterms.size() / 2), l0 = int(S.lterms.size() / 2);
            for (size_t k = 0; k < P.classes.size(); ++k)
                if (ftab[k][i] >= 0) S.gterms.insert(S.gterms.end(), {int(k), ftab[k][i]});
            for (int j = 0; j < s; ++j)
                if (P.mask[i * s + j]) S.lterms.insert(S.lterms.end(), {j, i * s + j});
            S.slots.insert(S.slots.end(), {i, g0, int(S.gterms.size() / 2) - g0, l0, int(S.lterms.size() / 2) - l0});
        }
        push_uses(S, int(P.classes.size()), blob);
    }
    {
        dgfs::SlotSet& S = P.pair_slots;
        S = dgfs::SlotSet();
        S.nslots = s * s;
        for (int i = 0; i < s; ++i)
            for (int j = 0; j < s; ++j) {
                const int g0 = int(S.gterms.size() / 2), l0 = int(S.lterms.size() / 2);
                if (!P.mask[i * s + j]) {  // evaluated elsewhere: an empty slot (zero output)
                    S.slots.insert(S.slots.end(), {i, g0, 0, l0, 0});
                    continue;
                }
                // every class of the pair (one, or with a VSS kernel one per direction)
                for (size_t k = 0; k < P.classes.size(); ++k) {
                    const auto& c = P.classes[k];
                    const bool of_pair = (c.i == i && c.j == j) || (P.antipodal && c.i == j && c.j == i);
                    if (of_pair && ftab[k][i] >= 0) S.gterms.insert(S.gterms.end(), {int(k), ftab[k][i]});
                }
                S.lterms.insert(S.lterms.end(), {j, i * s + j});
                S.slots.insert(S.slots.end(), {i, g0, int(S.gterms.size() / 2) - g0, l0, 1});
            }
        push_uses(S, int(P.classes.size()), blob);
    }

    // ---------------- plain per-point FP64 path: per ordered pair, all M directions
    if (P.precision == DGFS_FP64) {
        std::vector<std::complex<double>> ph(size_t(s) * s * nrho * P.M * 2 * 3 * N);
        std::vector<double> pF(size_t(s) * s * nrho * K2);
        for (int i = 0; i < s; ++i)
            for (int j = 0; j < s; ++j) {
                const int pr = i * s + j;
                const dgfs::PairParams& pp = P.pair[pr];
                for (int q = 0; q < nrho; ++q) {
                    for (int d = 0; d < P.M; ++d)
                        for (int fld = 0; fld < 2; ++fld) {
                            const double sgn = fld == 0 ? 1.0 : -1.0;
                            const double coef = fld == 0 ? pp.a : pp.b;
                            for (int dim = 0; dim < 3; ++dim) {
                                const double th = sgn * kPi * pp.rho[q] * coef * P.sigma[3 * d + dim] / L;
                                for (int jj = 0; jj < N; ++jj)
                                    ph[((((size_t(pr) * nrho + q) * P.M + d) * 2 + fld) * 3 + dim) * N + jj] =
                                        std::polar(1.0, th * signed_mode(jj, N));
                            }
                        }
                    for (int k2 = 0; k2 < K2; ++k2)
                        pF[(size_t(pr) * nrho + q) * K2 + k2] =
                            pp.wrho[q] * dgfs::pre::kernel_mode(std::sqrt(double(k2)), pp.rho[q], pp.a, pp.gamma,
                                                                pp.C, L) / n3;
                }
            }
        push_cplx<double>(blob, P.off_plain_ph, ph);
        push_double(blob, P.off_plain_F, pF);
    }

    push_double(blob, P.off_minv, conserve_pack(P.mass, P.Ls, N));
}

}  // namespace

namespace {

dgfs_status upload(dgfs_plan* P, const std::vector<char>& blob) {
    if (hipGetDevice(&P->device) != hipSuccess) return fail(DGFS_EDEVICE, "no HIP device");
    P->dev_bytes = blob.size();
    if (hipMalloc(&P->dev, P->dev_bytes) != hipSuccess) {
        P->dev = nullptr;
        return fail(DGFS_ENOMEM, "device allocation of the plan tables failed");
    }
    if (hipMemcpy(P->dev, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess)
        return fail(DGFS_EDEVICE, "upload of the plan tables failed");
    return DGFS_OK;
}

// A plan on one common grid (problem->L) that evaluates the ordered pairs set in mask.
dgfs_status create_single(const dgfs_problem* problem, const std::vector<unsigned char>& mask, dgfs_plan** out) {
    auto* P = new dgfs_plan();
    P->s = problem->s;
    P->N = problem->N;
    P->M = problem->M;
    P->nrho = problem->n_rho;
    P->precision = problem->precision;
    P->L = problem->L;
    P->mass.assign(problem->mass, problem->mass + problem->s);
    P->Ls.assign(problem->s, problem->L);
    P->mask = mask;
    dgfs::gain_geometry(P->N, P->precision, &P->geo, matrix_default(problem));
    if (problem->tile_ch != 0 || problem->tile_cz != 0) P->geo = dgfs::GainGeometry{problem->tile_ch, problem->tile_cz};
    dgfs::pre::design(P->M, P->sigma);
    P->antipodal = dgfs::pre::antipodal(P->sigma);
    P->K2 = 3 * (P->N / 2) * (P->N / 2) + 1;
    for (int i = 0; i < P->s; ++i)
        for (int j = 0; j < P->s; ++j) P->pair.push_back(pair_params(problem, i, j));
    for (const auto& pp : P->pair) P->vss = P->vss || pp.alpha != 1.0;
    // gain classes of the pairs this plan evaluates (the mask is symmetric)
    int off = 0;
    const double w = 4.0 * kPi / P->M;
    for (int i = 0; i < P->s; ++i)
        for (int j = 0; j < P->s; ++j) {
            if (P->antipodal && j < i) continue;
            if (!P->mask[i * P->s + j]) continue;
            dgfs::GainClass c;
            c.i = i;
            c.j = j;
            c.a = P->pair[i * P->s + j].a;
            c.b = P->pair[i * P->s + j].b;
            const bool half = P->antipodal && i == j;
            std::vector<int> dirs;
            for (int p = 0; p < P->M; ++p) {
                if (half) {  // keep the first of each antipodal pair
                    int anti = -1;
                    for (int q = 0; q < P->M; ++q) {
                        double d = 0;
                        for (int e = 0; e < 3; ++e) d += std::fabs(P->sigma[3 * p + e] + P->sigma[3 * q + e]);
                        if (d < 1e-12) anti = q;
                    }
                    if (anti < p) continue;
                }
                dirs.push_back(p);
            }
            if (!P->vss) {
                c.dirs = dirs;
                c.ndir = int(dirs.size());
                c.weight = half ? 2.0 * w : w;
                c.dir_offset = off;
                off += c.ndir;
                P->classes.push_back(c);
                continue;
            }
            for (size_t d0 = 0; d0 < dirs.size(); d0 += 2) {  // two directions per class
                c.dirs.assign(dirs.begin() + d0, dirs.begin() + std::min(dirs.size(), d0 + 2));
                c.ndir = int(c.dirs.size());
                c.weight = 1.0;
                c.dir_offset = off;
                off += c.ndir;
                P->classes.push_back(c);
            }
        }
    P->total_dirs = off;

    std::vector<char> blob;
    if (P->precision == DGFS_FP64) build_tables<double>(*P, blob);
    else build_tables<float>(*P, blob);
    const dgfs_status st = upload(P, blob);
    if (st != DGFS_OK) {
        dgfs_plan_destroy(P);
        return st;
    }
    *out = P;
    return DGFS_OK;
}

// Species-specific grids: one single-grid part per distinct pair box, with the maps that
// carry each species onto the box and the results back (the reading of the remark after
// eq. (domain) in Sec. 4 on independent grids per species).
dgfs_status create_species_grids(const dgfs_problem* problem, dgfs_plan** out) {
    const int s = problem->s;
    auto* P = new dgfs_plan();
    P->s = s;
    P->N = problem->N;
    P->M = problem->M;
    P->nrho = problem->n_rho;
    P->precision = problem->precision;
    P->mass.assign(problem->mass, problem->mass + s);
    P->Ls.assign(problem->L_species, problem->L_species + s);
    P->L = *std::max_element(P->Ls.begin(), P->Ls.end());
    P->mask.assign(size_t(s) * s, 1);
    dgfs::gain_geometry(P->N, P->precision, &P->geo, matrix_default(problem));
    if (problem->tile_ch != 0 || problem->tile_cz != 0) P->geo = dgfs::GainGeometry{problem->tile_ch, problem->tile_cz};
    std::vector<double> boxes;
    for (int i = 0; i < s; ++i)
        for (int j = 0; j < s; ++j) boxes.push_back(pair_box(problem, i, j));
    std::sort(boxes.begin(), boxes.end());
    boxes.erase(std::unique(boxes.begin(), boxes.end()), boxes.end());

    std::vector<char> blob;
    push_double(blob, P->off_minv, conserve_pack(P->mass, P->Ls, P->N));
    auto push_map = [&](double from, double to) {
        std::vector<double> T;
        dgfs::pre::interpolation_matrix(P->N, from, to, T);
        size_t off = 0;
        if (P->precision == DGFS_FP64) push_real<double>(blob, off, T);
        else push_real<float>(blob, off, T);
        return static_cast<long long>(off);
    };
    for (double box : boxes) {
        dgfs_plan::GridPart part;
        part.L = box;
        for (int i = 0; i < s; ++i) {
            bool used = false;
            for (int j = 0; j < s; ++j) used = used || pair_box(problem, i, j) == box;
            if (used) part.species.push_back(i);
        }
        const int sg = int(part.species.size());
        std::vector<double> m;
        std::vector<dgfs_pair_kernel> kern;
        std::vector<unsigned char> mask;
        for (int k = 0; k < sg; ++k) {
            const int i = part.species[k];
            m.push_back(problem->mass[i]);
            for (int l = 0; l < sg; ++l) {
                const int j = part.species[l];
                kern.push_back(problem->kernel[i * s + j]);
                mask.push_back(pair_box(problem, i, j) == box ? 1 : 0);
            }
            part.t_in.push_back(P->Ls[i] == box ? -1 : push_map(P->Ls[i], box));
            part.t_out.push_back(P->Ls[i] == box ? -1 : push_map(box, P->Ls[i]));
        }
        dgfs_problem sub = *problem;
        sub.s = sg;
        sub.mass = m.data();
        sub.L = box;
        sub.L_species = nullptr;
        sub.kernel = kern.data();
        const dgfs_status st = create_single(&sub, mask, &part.plan);
        if (st != DGFS_OK) {
            dgfs_plan_destroy(P);
            return st;
        }
        P->parts.push_back(std::move(part));
    }
    const dgfs_status st = upload(P, blob);
    if (st != DGFS_OK) {
        dgfs_plan_destroy(P);
        return st;
    }
    *out = P;
    return DGFS_OK;
}

// Byte layout of one part's share of the workspace for nb nodes.
struct PartLayout {
    size_t sub, X, Y, tmp, total;
};

PartLayout part_layout(const dgfs_plan& P, const dgfs_plan::GridPart& part, int64_t nb, bool pairs) {
    const size_t E = P.elem() * P.n3() * size_t(nb);
    const size_t sg = part.species.size();
    PartLayout l;
    l.sub = 0;
    l.X = detail_align(part.plan->ws_per_node(pairs) * size_t(nb) + part.plan->ws_slack());
    l.Y = l.X + detail_align(E * sg);
    l.tmp = l.Y + detail_align(E * (pairs ? sg * sg : sg));
    l.total = l.tmp + detail_align(2 * E);
    return l;
}

// One slice of nb nodes through every part.  stage_ms (optional, synchronous): adds the
// part's stage times, with the moves between grids counted in the first and last stage.
dgfs_status run_parts(const dgfs_plan& P, const void* f, void* Q, int64_t nb, void* ws, bool pairs, hipStream_t st,
                      hipEvent_t* ev, float* stage_ms) {
    const size_t E = P.elem();
    const int64_t n3 = int64_t(P.n3());
    const int s = P.s;
    const char* dev = static_cast<const char*>(P.dev);
    std::vector<unsigned char> written(s, 0);
    for (const auto& part : P.parts) {
        const int sg = int(part.species.size());
        const PartLayout lay = part_layout(P, part, nb, pairs);
        char* w = static_cast<char*>(ws);
        char* X = w + lay.X;
        char* Y = w + lay.Y;
        char* tmp = w + lay.tmp;
        auto map = [&](long long off) { return off < 0 ? nullptr : static_cast<const void*>(dev + off); };
        auto ok = [](hipError_t e) { return e == hipSuccess; };
        if (ev) hipEventRecord(ev[6], st);
        for (int k = 0; k < sg; ++k) {
            const int i = part.species[k];
            if (!ok(dgfs::launch_move(P, static_cast<const char*>(f) + size_t(i) * n3 * E, int64_t(s) * n3,
                                      X + size_t(k) * n3 * E, int64_t(sg) * n3, map(part.t_in[k]), nb, false, tmp, st)))
                return fail(DGFS_EDEVICE, "kernel launch failed (grid move)");
        }
        hipError_t e = dgfs::launch_collide(*part.plan, X, Y, nb, w + lay.sub, pairs, st, ev);
        if (e != hipSuccess) return fail(DGFS_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
        for (int k = 0; k < sg; ++k) {
            const int i = part.species[k];
            if (!pairs) {
                if (!ok(dgfs::launch_move(P, Y + size_t(k) * n3 * E, int64_t(sg) * n3,
                                          static_cast<char*>(Q) + size_t(i) * n3 * E, int64_t(s) * n3,
                                          map(part.t_out[k]), nb, written[i] != 0, tmp, st)))
                    return fail(DGFS_EDEVICE, "kernel launch failed (grid move)");
                written[i] = 1;
                continue;
            }
            for (int l = 0; l < sg; ++l) {
                const int j = part.species[l];
                if (!part.plan->mask[k * sg + l]) continue;
                if (!ok(dgfs::launch_move(P, Y + size_t(k * sg + l) * n3 * E, int64_t(sg) * sg * n3,
                                          static_cast<char*>(Q) + size_t(i * s + j) * n3 * E, int64_t(s) * s * n3,
                                          map(part.t_out[k]), nb, false, tmp, st)))
                    return fail(DGFS_EDEVICE, "kernel launch failed (grid move)");
            }
        }
        if (ev) {
            hipEventRecord(ev[7], st);
            if (hipEventSynchronize(ev[7]) != hipSuccess) return fail(DGFS_EDEVICE, "hipEventSynchronize failed");
            float ms = 0.0f;
            hipEventElapsedTime(&ms, ev[6], ev[1]);
            stage_ms[0] += ms;
            for (int k = 1; k < 4; ++k) {
                hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
                stage_ms[k] += ms;
            }
            hipEventElapsedTime(&ms, ev[4], ev[7]);
            stage_ms[4] += ms;
        }
    }
    return DGFS_OK;
}

}  // namespace

namespace dgfs {
dgfs_status set_error(dgfs_status st, const std::string& msg) { return fail(st, msg); }
}  // namespace dgfs

static dgfs_status collide_impl(const dgfs_plan* plan, const void* f, void* Q, int64_t batch, void* ws,
                                size_t ws_bytes, void* stream, bool pairs, float* stage_ms);

namespace dgfs {
dgfs_status collide_with_workspace(const dgfs_plan* plan, const void* f, void* Q, int64_t batch, void* ws,
                                   size_t ws_bytes, void* stream) {
    return collide_impl(plan, f, Q, batch, ws, ws_bytes, stream, false, nullptr);
}
}  // namespace dgfs

size_t dgfs_plan::ws_per_node(bool pairs) const {
    if (!parts.empty()) {
        // per node, the largest part (its layout for one node, less its one-off slack)
        size_t best = 0;
        for (const auto& part : parts) {
            const size_t sg = part.species.size(), E = elem() * n3();
            best = std::max(best, part.plan->ws_per_node(pairs) + E * (sg + (pairs ? sg * sg : sg) + 2));
        }
        return best;
    }
    const size_t c = 2 * elem() * n3();
    // a partial: the Hermitian half of a real field's spectrum, or (VSS) the whole
    // spectrum of Re S_0 + i Re S_1 plus the Nyquist-plane sums of Im S_d and their DFTs
    const size_t N2 = size_t(N) * N;
    const size_t part = vss ? 2 * elem() * n3() + elem() * 2 * (2 + size_t(geo.CH)) * N2 + 2 * elem() * 3 * N2
                            : 2 * elem() * size_t(N) * N * (N / 2 + 1);
    const int nslots = pairs ? s * s : s;
    if (inner)
        return dgfs::dealias_ws_per_node(elem(), N, s, int(inner->classes.size()), inner->nrho, nslots);
    // f_hat, the partials, and the gain and loss spectra of every slot (their k_z <= N/2
    // halves: the spectra are Hermitian)
    const size_t half = 2 * elem() * size_t(N) * N * (N / 2 + 1);
    // the matrix-core gain's prepared inputs (one alignment more: ws_slack)
    const size_t prep = geo.CZ == 0 ? size_t(s) * dgfs::mfma_prep_bytes : 0;
    return c * size_t(s) + 2 * half * size_t(nslots) + part * classes.size() * size_t(nrho) + prep;
}

extern "C" {

dgfs_status dgfs_check_problem(const dgfs_problem* problem) { return check(problem); }

dgfs_status dgfs_pair_prefactor(double m_i, double m_j, double omega, double alpha, double kn0, double* C) {
    if (!C) return fail(DGFS_EINVAL, "C is required");
    if (!(m_i > 0.0) || !(m_j > 0.0) || !std::isfinite(m_i) || !std::isfinite(m_j))
        return fail(DGFS_EINVAL, "masses must be positive");
    if (!(kn0 > 0.0) || !std::isfinite(kn0)) return fail(DGFS_EINVAL, "kn0 must be positive");
    if (!(omega >= 0.5 && omega <= 1.0)) return fail(DGFS_EINVAL, "omega must be in [0.5, 1]");
    if (!(alpha >= 1.0 && alpha <= 2.0)) return fail(DGFS_EINVAL, "alpha must be in [1, 2]");
    *C = dgfs::pre::pair_prefactor(m_i, m_j, omega, alpha, kn0);
    return DGFS_OK;
}

dgfs_status dgfs_design(int32_t M, double* sigma) {
    std::vector<double> pts;
    if (!dgfs::pre::design(M, pts)) return fail(DGFS_EINVAL, "no spherical design for this M (6, 12, 24)");
    if (sigma) std::copy(pts.begin(), pts.end(), sigma);
    return DGFS_OK;
}

dgfs_status dgfs_pair_tables(const dgfs_problem* problem, int32_t i, int32_t j, double* info, double* rho,
                             double* w_rho, double* loss) {
    dgfs_status st = check(problem);
    if (st == DGFS_EINVAL) return st;
    if (i < 0 || j < 0 || i >= problem->s || j >= problem->s) return fail(DGFS_EINVAL, "pair index out of range");
    dgfs::PairParams pp = pair_params(problem, i, j);
    std::vector<double> pts;
    dgfs::pre::design(problem->M, pts);
    const bool anti = dgfs::pre::antipodal(pts);
    if (info) {
        info[0] = pp.a;
        info[1] = pp.b;
        info[2] = pp.gamma;
        info[3] = pp.C;
        info[4] = pp.R;
        info[5] = (i == j && anti) ? problem->M / 2 : problem->M;
    }
    if (rho) std::copy(pp.rho.begin(), pp.rho.end(), rho);
    if (w_rho) std::copy(pp.wrho.begin(), pp.wrho.end(), w_rho);
    if (loss) {
        const int K2 = 3 * (problem->N / 2) * (problem->N / 2) + 1;
        for (int k2 = 0; k2 < K2; ++k2)
            loss[k2] = dgfs::pre::loss_weight(std::sqrt(double(k2)), pp.R, pp.gamma, pp.C, pair_box(problem, i, j)) *
                       dgfs::pre::vss_loss_factor(pp.alpha);
    }
    return DGFS_OK;
}

dgfs_status dgfs_plan_create(const dgfs_problem* problem, dgfs_plan** out) {
    if (!out) return fail(DGFS_EINVAL, "out is NULL");
    dgfs_status st = check(problem);
    if (st != DGFS_OK) return st;
    bool one_box = true;
    if (problem->L_species)
        for (int i = 1; i < problem->s; ++i) one_box = one_box && problem->L_species[i] == problem->L_species[0];
    if (!one_box) return create_species_grids(problem, out);
    dgfs_problem single = *problem;
    if (problem->L_species) {
        single.L = problem->L_species[0];
        single.L_species = nullptr;
    }
    const std::vector<unsigned char> all(size_t(problem->s) * problem->s, 1);
    if (!problem->dealias) return create_single(&single, all, out);
    // dealiased: this plan keeps the N-grid conservation tables; its companion on the
    // 3N/2 grid holds the tables of the padded gain and loss
    single.dealias = 0;
    dgfs_plan* outer = nullptr;
    if ((st = create_single(&single, all, &outer)) != DGFS_OK) return st;
    dgfs_problem wide = single;
    wide.N = 3 * problem->N / 2;
    if ((st = create_single(&wide, all, &outer->inner)) != DGFS_OK) {
        dgfs_plan_destroy(outer);
        return st;
    }
    *out = outer;
    return DGFS_OK;
}

void dgfs_plan_destroy(dgfs_plan* plan) {
    if (!plan) return;
    for (auto& part : plan->parts) dgfs_plan_destroy(part.plan);
    if (plan->inner) dgfs_plan_destroy(plan->inner);
    if (plan->dev) hipFree(plan->dev);
    delete plan;
}

dgfs_status dgfs_workspace_size(const dgfs_plan* plan, int64_t batch, size_t* bytes) {
    if (!plan || !bytes) return fail(DGFS_EINVAL, "plan and bytes are required");
    if (batch < 1) return fail(DGFS_EINVAL, "batch must be >= 1");
    // the pair-resolved mode needs the larger slot set; size for it (and at least what
    // the plain FP64 path needs for one node)
    *bytes = std::max(plan->ws_per_node(true) * size_t(batch) + plan->ws_slack(), dgfs::plain_ws_bytes(*plan) + 256);
    return DGFS_OK;
}

static dgfs_status collide_impl(const dgfs_plan* plan, const void* f, void* Q, int64_t batch, void* ws,
                                size_t ws_bytes, void* stream, bool pairs, float* stage_ms) {
    if (!plan) return fail(DGFS_EINVAL, "plan is NULL");
    if (batch < 0) return fail(DGFS_EINVAL, "batch must be >= 0");
    if (batch == 0) return DGFS_OK;
    if (!f || !Q || !ws) return fail(DGFS_EINVAL, "f, Q and workspace are required");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(DGFS_EINVAL, "workspace must be 256-byte aligned");
    const size_t per = plan->ws_per_node(pairs);
    if (ws_bytes < per + plan->ws_slack()) return fail(DGFS_ENOMEM, "workspace smaller than one node");
    const int64_t slice = std::min<int64_t>(batch, int64_t((ws_bytes - plan->ws_slack()) / per));
    const int nslots = pairs ? plan->s * plan->s : plan->s;
    const size_t in_stride = size_t(plan->s) * plan->n3() * plan->elem();
    const size_t out_stride = size_t(nslots) * plan->n3() * plan->elem();
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t ev[8] = {};
    if (stage_ms) {
        for (int k = 0; k < 5; ++k) stage_ms[k] = 0.0f;
        for (auto& e : ev)
            if (hipEventCreate(&e) != hipSuccess) return fail(DGFS_EDEVICE, "hipEventCreate failed");
    }
    dgfs_status result = DGFS_OK;
    for (int64_t b0 = 0; b0 < batch; b0 += slice) {
        const int64_t nb = std::min(slice, batch - b0);
        if (!plan->parts.empty()) {
            result = run_parts(*plan, static_cast<const char*>(f) + b0 * in_stride,
                               static_cast<char*>(Q) + b0 * out_stride, nb, ws, pairs, st, stage_ms ? ev : nullptr,
                               stage_ms);
            if (result != DGFS_OK) break;
            continue;
        }
        hipError_t e = dgfs::launch_collide(*plan, static_cast<const char*>(f) + b0 * in_stride,
                                            static_cast<char*>(Q) + b0 * out_stride, nb, ws, pairs, st,
                                            stage_ms ? ev : nullptr);
        if (e != hipSuccess) {
            result = fail(DGFS_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
            break;
        }
        if (stage_ms) {
            if (hipEventSynchronize(ev[5]) != hipSuccess) {
                result = fail(DGFS_EDEVICE, "hipEventSynchronize failed");
                break;
            }
            for (int k = 0; k < 5; ++k) {
                float ms = 0.0f;
                hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
                stage_ms[k] += ms;
            }
        }
    }
    if (stage_ms)
        for (auto& e : ev) hipEventDestroy(e);
    return result;
}

dgfs_status dgfs_collide(const dgfs_plan* plan, const void* f, void* Q, int64_t batch, void* workspace,
                         size_t ws_bytes, void* stream) {
    return collide_impl(plan, f, Q, batch, workspace, ws_bytes, stream, false, nullptr);
}

dgfs_status dgfs_collide_timed(const dgfs_plan* plan, const void* f, void* Q, int64_t batch, void* workspace,
                               size_t ws_bytes, void* stream, float* stage_ms) {
    if (!stage_ms) return fail(DGFS_EINVAL, "stage_ms is required");
    return collide_impl(plan, f, Q, batch, workspace, ws_bytes, stream, false, stage_ms);
}

dgfs_status dgfs_collide_pairs(const dgfs_plan* plan, const void* f, void* Q, int64_t batch, void* workspace,
                               size_t ws_bytes, void* stream) {
    return collide_impl(plan, f, Q, batch, workspace, ws_bytes, stream, true, nullptr);
}

dgfs_status dgfs_collide_plain(const dgfs_plan* plan, const double* f, double* Q, int64_t batch, void* workspace,
                               size_t ws_bytes, void* stream) {
    if (!plan) return fail(DGFS_EINVAL, "plan is NULL");
    if (plan->precision != DGFS_FP64) return fail(DGFS_EUNSUPPORTED, "the plain path needs an FP64 plan");
    if (!plan->parts.empty()) return fail(DGFS_EUNSUPPORTED, "the plain path has one common grid");
    if (plan->vss) return fail(DGFS_EUNSUPPORTED, "the plain path covers the VHS family (alpha = 1)");
    if (plan->inner) return fail(DGFS_EUNSUPPORTED, "the plain path evaluates the circular form");
    if (plan->N > 48) return fail(DGFS_EUNSUPPORTED, "the plain path is compiled for N <= 48");
    if (batch < 0) return fail(DGFS_EINVAL, "batch must be >= 0");
    if (batch == 0) return DGFS_OK;
    if (!f || !Q || !workspace) return fail(DGFS_EINVAL, "f, Q and workspace are required");
    if (static_cast<const void*>(f) == static_cast<void*>(Q)) return fail(DGFS_EINVAL, "f and Q must not overlap");
    if (ws_bytes < dgfs::plain_ws_bytes(*plan)) return fail(DGFS_ENOMEM, "workspace smaller than one node");
    hipError_t e = dgfs::launch_collide_plain(*plan, f, Q, batch, workspace, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(DGFS_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return DGFS_OK;
}

dgfs_status dgfs_conserve(const dgfs_plan* plan, const void* Q_raw, double* Q_out, int64_t batch, void* stream) {
    if (!plan) return fail(DGFS_EINVAL, "plan is NULL");
    if (batch < 0) return fail(DGFS_EINVAL, "batch must be >= 0");
    if (batch == 0) return DGFS_OK;
    if (!Q_raw || !Q_out) return fail(DGFS_EINVAL, "Q_raw and Q_out are required");
    if (plan->precision != DGFS_FP64 && static_cast<const void*>(Q_out) == Q_raw)
        return fail(DGFS_EINVAL, "Q_out may alias Q_raw only for FP64 plans");
    hipError_t e = dgfs::launch_conserve(*plan, Q_raw, Q_out, nullptr, 0.0, batch, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(DGFS_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return DGFS_OK;
}

dgfs_status dgfs_conserve_update(const dgfs_plan* plan, const void* Q_raw, void* f, double dt, int64_t batch,
                                 void* stream) {
    if (!plan) return fail(DGFS_EINVAL, "plan is NULL");
    if (batch < 0) return fail(DGFS_EINVAL, "batch must be >= 0");
    if (batch == 0) return DGFS_OK;
    if (!Q_raw || !f) return fail(DGFS_EINVAL, "Q_raw and f are required");
    if (Q_raw == static_cast<const void*>(f)) return fail(DGFS_EINVAL, "Q_raw and f must not overlap");
    if (!std::isfinite(dt)) return fail(DGFS_EINVAL, "dt must be finite");
    hipError_t e = dgfs::launch_conserve(*plan, Q_raw, nullptr, f, dt, batch, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(DGFS_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return DGFS_OK;
}

// ------------------------------------------------------------------ stepping
static size_t state_bytes(const dgfs_plan* plan, int64_t batch) {
    return (size_t(batch) * plan->s * plan->n3() * plan->elem() + 255) & ~size_t(255);
}

dgfs_status dgfs_relax_workspace_size(const dgfs_plan* plan, int64_t batch, int32_t scheme, size_t* bytes) {
    if (!plan || !bytes) return fail(DGFS_EINVAL, "plan and bytes are required");
    if (batch < 1) return fail(DGFS_EINVAL, "batch must be >= 1");
    if (scheme != DGFS_EULER && scheme != DGFS_SSPRK2) return fail(DGFS_EINVAL, "unknown scheme");
    *bytes = state_bytes(plan, batch) * (scheme == DGFS_SSPRK2 ? 2 : 1) + plan->ws_per_node(false) * size_t(batch) +
             plan->ws_slack();
    return DGFS_OK;
}

dgfs_status dgfs_relax(const dgfs_plan* plan, void* f, int64_t batch, double dt, int32_t steps, int32_t scheme,
                       void* workspace, size_t ws_bytes, void* stream) {
    if (!plan) return fail(DGFS_EINVAL, "plan is NULL");
    if (batch < 0 || steps < 0) return fail(DGFS_EINVAL, "batch and steps must be >= 0");
    if (scheme != DGFS_EULER && scheme != DGFS_SSPRK2) return fail(DGFS_EINVAL, "unknown scheme");
    if (!std::isfinite(dt)) return fail(DGFS_EINVAL, "dt must be finite");
    if (batch == 0 || steps == 0) return DGFS_OK;
    if (!f || !workspace) return fail(DGFS_EINVAL, "f and workspace are required");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(DGFS_EINVAL, "workspace must be 256-byte aligned");
    const size_t sb = state_bytes(plan, batch);
    const size_t fixed = sb * (scheme == DGFS_SSPRK2 ? 2 : 1);
    if (ws_bytes < fixed + plan->ws_per_node(false) + plan->ws_slack())
        return fail(DGFS_ENOMEM, "workspace smaller than the stage states plus one node");
    char* w = static_cast<char*>(workspace);
    void* Q = w;
    void* f1 = scheme == DGFS_SSPRK2 ? w + sb : nullptr;
    void* cw = w + fixed;
    const size_t cwb = ws_bytes - fixed;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = batch * plan->s * int64_t(plan->n3());
    auto dev = [&](hipError_t e) {
        return e == hipSuccess ? DGFS_OK : fail(DGFS_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    };
    dgfs_status rc = DGFS_OK;
    for (int32_t k = 0; k < steps && rc == DGFS_OK; ++k) {
        if (scheme == DGFS_EULER) {
            if ((rc = collide_impl(plan, f, Q, batch, cw, cwb, stream, false, nullptr)) != DGFS_OK) break;
            rc = dev(dgfs::launch_conserve(*plan, Q, nullptr, f, dt, batch, st));
            continue;
        }
        // f1 = f + dt L(f);  f1 <- f1 + dt L(f1);  f <- (f + f1) / 2
        if ((rc = dev(hipMemcpyAsync(f1, f, size_t(n) * plan->elem(), hipMemcpyDeviceToDevice, st))) != DGFS_OK) break;
        if ((rc = collide_impl(plan, f, Q, batch, cw, cwb, stream, false, nullptr)) != DGFS_OK) break;
        if ((rc = dev(dgfs::launch_conserve(*plan, Q, nullptr, f1, dt, batch, st))) != DGFS_OK) break;
        if ((rc = collide_impl(plan, f1, Q, batch, cw, cwb, stream, false, nullptr)) != DGFS_OK) break;
        if ((rc = dev(dgfs::launch_conserve(*plan, Q, nullptr, f1, dt, batch, st))) != DGFS_OK) break;
        rc = dev(dgfs::launch_axpby(*plan, f, f1, f, 0.5, 0.5, n, st));
    }
    return rc;
}

dgfs_status dgfs_kernel_mode(double alpha, double gamma, double C, double a, double L, double rho, const double* k,
                             const double* sigma, double* F) {
    if (!k || !sigma || !F) return fail(DGFS_EINVAL, "k, sigma and F are required");
    if (!(alpha >= 1.0 && alpha <= 2.0)) return fail(DGFS_EINVAL, "alpha must be in [1, 2]");
    if (!(L > 0.0) || !(rho >= 0.0)) return fail(DGFS_EINVAL, "L must be positive and rho non-negative");
    dgfs::pre::kernel_mode_vss(k, rho, sigma, a, gamma, alpha, C, L, F[0], F[1]);
    return DGFS_OK;
}

dgfs_status dgfs_tile_candidates(int32_t N, int32_t precision, int32_t* pairs, int32_t max_pairs, int32_t* count) {
    if (!count) return fail(DGFS_EINVAL, "count is required");
    dgfs::GainGeometry cand[16];
    const int n = dgfs::tile_candidates(N, precision, cand, 16);
    *count = 0;
    for (int k = 0; k < n && k < max_pairs; ++k) {
        if (pairs) {
            pairs[2 * k] = cand[k].CH;
            pairs[2 * k + 1] = cand[k].CZ;
        }
        *count = k + 1;
    }
    return DGFS_OK;
}

// ------------------------------------------------------------------- groups
struct dgfs_group {
    std::vector<const dgfs_plan*> plans;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;
    int device = 0;
};

static size_t group_offset(const dgfs_group* g, const int64_t* batch, size_t k) {
    size_t off = 0;
    for (size_t i = 0; i < k; ++i) {
        size_t b = 0;
        dgfs_workspace_size(g->plans[i], std::max<int64_t>(batch[i], 1), &b);
        off += (b + 255) & ~size_t(255);
    }
    return off;
}

dgfs_status dgfs_group_create(const dgfs_plan* const* plans, int32_t nplans, dgfs_group** out) {
    if (!plans || !out || nplans < 1 || nplans > 64) return fail(DGFS_EINVAL, "need 1..64 plans and out");
    auto* g = new dgfs_group();
    hipGetDevice(&g->device);
    for (int k = 0; k < nplans; ++k) {
        if (!plans[k]) {
            dgfs_group_destroy(g);
            return fail(DGFS_EINVAL, "NULL plan in group");
        }
        g->plans.push_back(plans[k]);
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            if (st) hipStreamDestroy(st);
            dgfs_group_destroy(g);
            return fail(DGFS_EDEVICE, "stream/event creation failed");
        }
        g->streams.push_back(st);
        g->join.push_back(ev);
    }
    if (hipEventCreateWithFlags(&g->fork, hipEventDisableTiming) != hipSuccess) {
        dgfs_group_destroy(g);
        return fail(DGFS_EDEVICE, "event creation failed");
    }
    *out = g;
    return DGFS_OK;
}

void dgfs_group_destroy(dgfs_group* g) {
    if (!g) return;
    for (auto st : g->streams)
        if (st) hipStreamDestroy(st);
    for (auto ev : g->join)
        if (ev) hipEventDestroy(ev);
    if (g->fork) hipEventDestroy(g->fork);
    delete g;
}

dgfs_status dgfs_group_workspace_size(const dgfs_group* g, const int64_t* batch, size_t* bytes) {
    if (!g || !batch || !bytes) return fail(DGFS_EINVAL, "group, batch and bytes are required");
    for (size_t k = 0; k < g->plans.size(); ++k)
        if (batch[k] < 0) return fail(DGFS_EINVAL, "batch must be >= 0");
    *bytes = group_offset(g, batch, g->plans.size());
    return DGFS_OK;
}

dgfs_status dgfs_group_collide(dgfs_group* g, const void* const* f, void* const* Q, const int64_t* batch,
                               void* ws, size_t ws_bytes, void* stream) {
    if (!g || !f || !Q || !batch || !ws) return fail(DGFS_EINVAL, "group, f, Q, batch and workspace are required");
    size_t need = 0;
    dgfs_status st = dgfs_group_workspace_size(g, batch, &need);
    if (st != DGFS_OK) return st;
    if (ws_bytes < need) return fail(DGFS_ENOMEM, "group workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(DGFS_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t main = static_cast<hipStream_t>(stream);
    if (hipEventRecord(g->fork, main) != hipSuccess) return fail(DGFS_EDEVICE, "hipEventRecord failed");
    for (size_t k = 0; k < g->plans.size(); ++k) {
        if (batch[k] == 0) continue;
        if (hipStreamWaitEvent(g->streams[k], g->fork, 0) != hipSuccess)
            return fail(DGFS_EDEVICE, "hipStreamWaitEvent failed");
        const size_t off = group_offset(g, batch, k);
        size_t b = 0;
        dgfs_workspace_size(g->plans[k], batch[k], &b);
        st = collide_impl(g->plans[k], f[k], Q[k], batch[k], static_cast<char*>(ws) + off, b, g->streams[k], false,
                          nullptr);
        if (st != DGFS_OK) return st;
        if (hipEventRecord(g->join[k], g->streams[k]) != hipSuccess ||
            hipStreamWaitEvent(main, g->join[k], 0) != hipSuccess)
            return fail(DGFS_EDEVICE, "join failed");
    }
    return DGFS_OK;
}

dgfs_status dgfs_group_capture(dgfs_group* g, const void* const* f, void* const* Q, const int64_t* batch, void* ws,
                               size_t ws_bytes, void* stream, void** graph) {
    if (!graph) return fail(DGFS_EINVAL, "graph is required");
    if (!stream) return fail(DGFS_EINVAL, "capture needs a non-default stream");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(DGFS_EDEVICE, "hipStreamBeginCapture failed");
    dgfs_status rc = dgfs_group_collide(g, f, Q, batch, ws, ws_bytes, stream);
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(st, &gr);
    if (rc != DGFS_OK) {
        if (gr) hipGraphDestroy(gr);
        return rc;
    }
    if (e != hipSuccess || !gr) return fail(DGFS_EDEVICE, "hipStreamEndCapture failed");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
    hipGraphDestroy(gr);
    if (e != hipSuccess) return fail(DGFS_EDEVICE, "hipGraphInstantiate failed");
    *graph = exec;
    return DGFS_OK;
}

dgfs_status dgfs_graph_launch(void* graph, void* stream) {
    if (!graph) return fail(DGFS_EINVAL, "graph is NULL");
    if (hipGraphLaunch(static_cast<hipGraphExec_t>(graph), static_cast<hipStream_t>(stream)) != hipSuccess)
        return fail(DGFS_EDEVICE, "hipGraphLaunch failed");
    return DGFS_OK;
}

void dgfs_graph_destroy(void* graph) {
    if (graph) hipGraphExecDestroy(static_cast<hipGraphExec_t>(graph));
}

dgfs_status dgfs_interpolation_matrix(int32_t N, double L_from, double L_to, double* T) {
    if (!T) return fail(DGFS_EINVAL, "T is required");
    if (N < 2 || N % 2 != 0 || N > 1024) return fail(DGFS_EINVAL, "N must be even and in [2, 1024]");
    if (!(L_from > 0.0) || !(L_to > 0.0) || !std::isfinite(L_from) || !std::isfinite(L_to))
        return fail(DGFS_EINVAL, "half-widths must be positive");
    std::vector<double> m;
    dgfs::pre::interpolation_matrix(N, L_from, L_to, m);
    std::copy(m.begin(), m.end(), T);
    return DGFS_OK;
}

const char* dgfs_status_string(dgfs_status status) {
    switch (status) {
        case DGFS_OK: return "ok";
        case DGFS_EINVAL: return "invalid argument";
        case DGFS_EUNSUPPORTED: return "unsupported";
        case DGFS_ENOMEM: return "out of memory";
        case DGFS_EDEVICE: return "device error";
    }
    return "unknown status";
}

const char* dgfs_last_error(void) { return g_err.c_str(); }

}  // extern "C"
