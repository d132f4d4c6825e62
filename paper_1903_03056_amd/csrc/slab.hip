// The 1-D slab of Sec. 5: nodal DG transport (GLL points, upwind flux, diagonal mass)
// with inflow and diffuse-wall boundaries (Sec. 2), stepped by forward Euler or SSP-RK2
// around the batched collision operator and its FP64 conservation projection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "dgfs.h"
#include "plan.hpp"

struct dgfs_slab {
    const dgfs_plan* plan = nullptr;
    dgfs_slab_desc desc{};
    int Ne = 0, K = 0, s = 0, N = 0;
    double h = 0;
    int64_t nodes = 0;
    void* dev = nullptr;  // one block: coef, vx, boundary tables, wall denominators
    size_t off_coef = 0, off_vx = 0, off_bt = 0, off_den = 0;
};

namespace {

constexpr int kMaxK = 8;
constexpr double kPi = 3.14159265358979323846264338327950288;

// Legendre P_n and its derivative at x by the three-term recurrence.
void legendre(int n, double x, double& p, double& dp) {
    double p0 = 1.0, p1 = x;
    if (n == 0) {
        p = 1.0;
        dp = 0.0;
        return;
    }
    for (int k = 1; k < n; ++k) {
        const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    p = p1;
    dp = n * (x * p1 - p0) / (x * x - 1.0);  // valid off the ends, where it is used
}

// GLL points: the ends and the roots of P'_{K-1}, found by sign changes of P'_{K-1} on
// a fine grid and bisection to full precision; weights 2 / (K (K-1) P_{K-1}(x)^2).
void gll_rule(int K, std::vector<double>& x, std::vector<double>& w) {
    x.assign(1, -1.0);
    const int n = K - 1, samples = 4000;
    auto dP = [n](double t) {
        double p, dp;
        legendre(n, t, p, dp);
        return dp;
    };
    double a = -1.0 + 1e-9, fa = dP(a);
    for (int k = 1; k <= samples; ++k) {
        const double b = -1.0 + 1e-9 + (2.0 - 2e-9) * k / samples, fb = dP(b);
        if ((fa < 0) != (fb < 0)) {
            double lo = a, hi = b, flo = fa;
            for (int it = 0; it < 200 && hi - lo > 1e-17; ++it) {
                const double mid = 0.5 * (lo + hi), fm = dP(mid);
                if ((fm < 0) == (flo < 0)) {
                    lo = mid;
                    flo = fm;
                } else {
                    hi = mid;
                }
            }
            x.push_back(0.5 * (lo + hi));
        }
        a = b;
        fa = fb;
    }
    x.push_back(1.0);
    w.resize(x.size());
    for (size_t k = 0; k < x.size(); ++k) {
        double p, dp;
        legendre(n, x[k], p, dp);
        w[k] = 2.0 / (double(K) * (K - 1) * p * p);
    }
}

// D[q][m] = derivative of the m-th Lagrange polynomial through x at x_q (barycentric).
std::vector<double> lagrange_diff(const std::vector<double>& x) {
    const int K = int(x.size());
    std::vector<double> lam(K, 1.0), D(size_t(K) * K, 0.0);
    for (int m = 0; m < K; ++m)
        for (int n = 0; n < K; ++n)
            if (n != m) lam[m] /= (x[m] - x[n]);
    for (int q = 0; q < K; ++q) {
        double diag = 0.0;
        for (int m = 0; m < K; ++m)
            if (m != q) {
                D[q * K + m] = lam[m] / lam[q] / (x[q] - x[m]);
                diag -= D[q * K + m];
            }
        D[q * K + q] = diag;
    }
    return D;
}

double maxwellian_1d(double v, double m, double u, double T) { return std::exp(-m * (v - u) * (v - u) / T); }

// ------------------------------------------------------------------- kernels
constexpr int kWallBlocks = 64;  // blocks per (wall, species) of the wall reduction

// Per side and species, partial sums over a slice of the velocity grid of
// -sum_{vx n >= 0} (vx n) f_trace; the transport kernel adds the kWallBlocks partials and
// divides by den (the matching sum over the incoming half for the unit wall Maxwellian,
// precomputed) to get n_w.
template <typename T, int N>
__global__ __launch_bounds__(256) void wall_density_kernel(const T* __restrict__ f, const T* __restrict__ vx,
                                                           double* __restrict__ part, int s, int64_t left_node,
                                                           int64_t right_node, int left_wall, int right_wall) {
    constexpr int N3 = N * N * N, SLICE = N3 / kWallBlocks;
    const int blk = blockIdx.x % kWallBlocks, si = blockIdx.x / kWallBlocks;
    const int side = si / s, i = si % s;
    if ((side == 0 && !left_wall) || (side == 1 && !right_wall)) return;
    const T* tr = f + ((side == 0 ? left_node : right_node) * s + i) * int64_t(N3);
    const double normal = side == 0 ? -1.0 : 1.0;
    double acc = 0.0;
    for (int v = blk * SLICE + threadIdx.x; v < (blk + 1) * SLICE; v += 256) {
        const double vn = double(vx[i * N + v / (N * N)]) * normal;
        if (vn >= 0.0) acc += vn * double(tr[v]);
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(side * s + i) * kWallBlocks + blk] = -red[0];
}

struct TransportArgs {
    const double* coef;  // [K][K] c_lm = w_l D_lm, then [K] 2/(h w_m)
    const void* vx;      // [s][N]
    const void* bt;      // [2][s][N^3]  inflow state, or unit wall Maxwellian
    const double* den;   // [2][s]       wall denominators
    const double* part;  // [2][s][kWallBlocks] wall numerator partials
    int Ne, K, s, left_wall, right_wall;
    double dt;
};

// out = in + dt T(in) for every node: one thread per (element, species, velocity) holds
// the element's K values and its two neighbour traces.
template <typename T, int N>
__global__ __launch_bounds__(256) void transport_kernel(const T* __restrict__ in, T* __restrict__ out, TransportArgs a) {
    constexpr int N3 = N * N * N;
    const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t >= int64_t(a.Ne) * a.s * N3) return;
    const int v = int(t % N3);
    const int es = int(t / N3);
    const int i = es % a.s, e = es / a.s;
    const int K = a.K;
    const T* vxt = static_cast<const T*>(a.vx);
    const T* bt = static_cast<const T*>(a.bt);
    const T vx = vxt[i * N + v / (N * N)];
    auto at = [&](int ee, int m) { return in[((int64_t(ee) * K + m) * a.s + i) * N3 + v]; };
    auto wall_density = [&](int side) {
        double num = 0.0;
        const double* pp = a.part + (side * a.s + i) * kWallBlocks;
        for (int k = 0; k < kWallBlocks; ++k) num += pp[k];
        return T(num / a.den[side * a.s + i]);
    };
    T F[kMaxK];
    for (int m = 0; m < K; ++m) F[m] = at(e, m);
    // outside values at the two faces (only used for incoming velocities)
    T outl, outr;
    if (e > 0) outl = at(e - 1, K - 1);
    else outl = bt[(0 * a.s + i) * int64_t(N3) + v] * (a.left_wall ? wall_density(0) : T(1));
    if (e < a.Ne - 1) outr = at(e + 1, 0);
    else outr = bt[(1 * a.s + i) * int64_t(N3) + v] * (a.right_wall ? wall_density(1) : T(1));
    const T fl = vx <= T(0) ? F[0] : outl;        // left face, normal -1
    const T fr = vx >= T(0) ? F[K - 1] : outr;    // right face, normal +1
    for (int m = 0; m < K; ++m) {
        T vol = T(0);
        for (int l = 0; l < K; ++l) vol += T(a.coef[l * K + m]) * F[l];
        T r = vx * vol;
        if (m == K - 1) r -= vx * fr;
        if (m == 0) r += vx * fl;
        out[((int64_t(e) * K + m) * a.s + i) * N3 + v] = F[m] + T(a.dt) * T(a.coef[K * K + m]) * r;
    }
}

template <typename T, int N>
hipError_t run_transport(const dgfs_slab& S, const void* in, void* out, double dt, double* part, hipStream_t st) {
    const char* dev = static_cast<const char*>(S.dev);
    const int lw = S.desc.left.kind == DGFS_BC_WALL, rw = S.desc.right.kind == DGFS_BC_WALL;
    if (lw || rw) {
        wall_density_kernel<T, N><<<dim3(unsigned(2 * S.s * kWallBlocks)), dim3(256), 0, st>>>(
            static_cast<const T*>(in), reinterpret_cast<const T*>(dev + S.off_vx), part, S.s, 0, S.nodes - 1, lw, rw);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    TransportArgs a;
    a.coef = reinterpret_cast<const double*>(dev + S.off_coef);
    a.vx = dev + S.off_vx;
    a.bt = dev + S.off_bt;
    a.den = reinterpret_cast<const double*>(dev + S.off_den);
    a.part = part;
    a.Ne = S.Ne;
    a.K = S.K;
    a.s = S.s;
    a.left_wall = lw;
    a.right_wall = rw;
    a.dt = dt;
    const int64_t n = int64_t(S.Ne) * S.s * N * N * N;
    transport_kernel<T, N><<<dim3(unsigned((n + 255) / 256)), dim3(256), 0, st>>>(static_cast<const T*>(in),
                                                                                 static_cast<T*>(out), a);
    return hipGetLastError();
}

template <typename T>
hipError_t transport_n(const dgfs_slab& S, const void* in, void* out, double dt, double* part, hipStream_t st) {
    switch (S.N) {
        case 16: return run_transport<T, 16>(S, in, out, dt, part, st);
        case 24: return run_transport<T, 24>(S, in, out, dt, part, st);
        case 32: return run_transport<T, 32>(S, in, out, dt, part, st);
        case 48: return run_transport<T, 48>(S, in, out, dt, part, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t transport(const dgfs_slab& S, const void* in, void* out, double dt, double* part, hipStream_t st) {
    return S.plan->precision == DGFS_FP64 ? transport_n<double>(S, in, out, dt, part, st)
                                          : transport_n<float>(S, in, out, dt, part, st);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <typename T>
void push(std::vector<char>& blob, size_t& off, const std::vector<double>& v) {
    off = align256(blob.size());
    blob.resize(off + v.size() * sizeof(T));
    T* d = reinterpret_cast<T*>(blob.data() + off);
    for (size_t k = 0; k < v.size(); ++k) d[k] = T(v[k]);
}

dgfs_status check_boundary(const dgfs_boundary& b, int s) {
    if (b.kind != DGFS_BC_INFLOW && b.kind != DGFS_BC_WALL) return dgfs::set_error(DGFS_EINVAL, "unknown boundary kind");
    if (!(b.T > 0.0) || !std::isfinite(b.T)) return dgfs::set_error(DGFS_EINVAL, "boundary temperature must be positive");
    if (b.kind == DGFS_BC_WALL && b.u[0] != 0.0)
        return dgfs::set_error(DGFS_EINVAL, "a wall moves only along the wall (u[0] must be 0)");
    if (b.kind == DGFS_BC_INFLOW)
        for (int i = 0; i < s; ++i)
            if (!(b.n[i] >= 0.0) || !std::isfinite(b.n[i]))
                return dgfs::set_error(DGFS_EINVAL, "inflow densities must be non-negative");
    return DGFS_OK;
}

size_t state_bytes(const dgfs_slab& S) { return align256(size_t(S.nodes) * S.s * S.plan->n3() * S.plan->elem()); }

// wall-density partials: [2 sides][8 species][kWallBlocks] doubles
constexpr size_t kPartBytes = 2 * 8 * kWallBlocks * sizeof(double);

}  // namespace

extern "C" {

dgfs_status dgfs_slab_gll(int32_t K, double* xi, double* w) {
    if (K < 2 || K > kMaxK) return dgfs::set_error(DGFS_EINVAL, "K must be in [2, 8]");
    if (!xi || !w) return dgfs::set_error(DGFS_EINVAL, "xi and w are required");
    std::vector<double> x, ww;
    gll_rule(K, x, ww);
    if (int(x.size()) != K) return dgfs::set_error(DGFS_EDEVICE, "GLL root search failed");
    std::copy(x.begin(), x.end(), xi);
    std::copy(ww.begin(), ww.end(), w);
    return DGFS_OK;
}

dgfs_status dgfs_slab_create(const dgfs_plan* plan, const dgfs_slab_desc* desc, dgfs_slab** out) {
    if (!plan || !desc || !out) return dgfs::set_error(DGFS_EINVAL, "plan, desc and out are required");
    if (desc->Ne < 1) return dgfs::set_error(DGFS_EINVAL, "Ne must be >= 1");
    if (desc->K < 2 || desc->K > kMaxK) return dgfs::set_error(DGFS_EINVAL, "K must be in [2, 8]");
    if (!(desc->x1 > desc->x0) || !std::isfinite(desc->x0) || !std::isfinite(desc->x1))
        return dgfs::set_error(DGFS_EINVAL, "need x1 > x0");
    if (desc->collide != 0 && desc->collide != 1) return dgfs::set_error(DGFS_EINVAL, "collide must be 0 or 1");
    if (plan->N > 48) return dgfs::set_error(DGFS_EUNSUPPORTED, "the slab transport is compiled for N <= 48");
    dgfs_status st = check_boundary(desc->left, plan->s);
    if (st != DGFS_OK) return st;
    if ((st = check_boundary(desc->right, plan->s)) != DGFS_OK) return st;
    auto* S = new dgfs_slab();
    S->plan = plan;
    S->desc = *desc;
    S->Ne = desc->Ne;
    S->K = desc->K;
    S->s = plan->s;
    S->N = plan->N;
    S->h = (desc->x1 - desc->x0) / desc->Ne;
    S->nodes = int64_t(desc->Ne) * desc->K;
    std::vector<double> xi, w;
    gll_rule(S->K, xi, w);
    if (int(xi.size()) != S->K) {
        delete S;
        return dgfs::set_error(DGFS_EDEVICE, "GLL root search failed");
    }
    const std::vector<double> D = lagrange_diff(xi);
    const int K = S->K, N = S->N, s = S->s;
    std::vector<double> coef(size_t(K) * K + K);
    for (int l = 0; l < K; ++l)
        for (int m = 0; m < K; ++m) coef[l * K + m] = w[l] * D[l * K + m];
    for (int m = 0; m < K; ++m) coef[K * K + m] = 2.0 / (S->h * w[m]);
    const size_t n3 = size_t(N) * N * N;
    std::vector<double> vx(size_t(s) * N), bt(2 * size_t(s) * n3), den(2 * size_t(s), 1.0);
    for (int i = 0; i < s; ++i)
        for (int n = 0; n < N; ++n) vx[i * N + n] = -plan->Ls[i] + n * (2.0 * plan->Ls[i] / N);
    for (int side = 0; side < 2; ++side) {
        const dgfs_boundary& b = side == 0 ? desc->left : desc->right;
        const double normal = side == 0 ? -1.0 : 1.0;
        for (int i = 0; i < s; ++i) {
            const double m = plan->mass[i], L = plan->Ls[i], hv = 2.0 * L / N;
            const double n = b.kind == DGFS_BC_INFLOW ? b.n[i] : 1.0;
            const double pre = n * std::pow(m / (kPi * b.T), 1.5);
            std::vector<double> g[3];
            for (int a = 0; a < 3; ++a) {
                g[a].resize(N);
                for (int k = 0; k < N; ++k) g[a][k] = maxwellian_1d(-L + k * hv, m, b.u[a], b.T);
            }
            double dsum = 0.0;
            for (int ix = 0; ix < N; ++ix)
                for (int iy = 0; iy < N; ++iy)
                    for (int iz = 0; iz < N; ++iz) {
                        const double val = pre * g[0][ix] * g[1][iy] * g[2][iz];
                        bt[(size_t(side) * s + i) * n3 + (size_t(ix) * N + iy) * N + iz] = val;
                        const double vn = vx[i * N + ix] * normal;
                        if (vn < 0.0) dsum += vn * val;
                    }
            if (b.kind == DGFS_BC_WALL) den[side * s + i] = dsum;
        }
    }
    std::vector<char> blob;
    push<double>(blob, S->off_coef, coef);
    if (plan->precision == DGFS_FP64) {
        push<double>(blob, S->off_vx, vx);
        push<double>(blob, S->off_bt, bt);
    } else {
        push<float>(blob, S->off_vx, vx);
        push<float>(blob, S->off_bt, bt);
    }
    push<double>(blob, S->off_den, den);
    if (hipMalloc(&S->dev, blob.size()) != hipSuccess) {
        delete S;
        return dgfs::set_error(DGFS_ENOMEM, "hipMalloc of the slab tables failed");
    }
    if (hipMemcpy(S->dev, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(S->dev);
        delete S;
        return dgfs::set_error(DGFS_EDEVICE, "upload of the slab tables failed");
    }
    *out = S;
    return DGFS_OK;
}

void dgfs_slab_destroy(dgfs_slab* slab) {
    if (!slab) return;
    if (slab->dev) hipFree(slab->dev);
    delete slab;
}

dgfs_status dgfs_slab_workspace_size(const dgfs_slab* slab, int32_t scheme, size_t* bytes) {
    if (!slab || !bytes) return dgfs::set_error(DGFS_EINVAL, "slab and bytes are required");
    if (scheme != DGFS_EULER && scheme != DGFS_SSPRK2) return dgfs::set_error(DGFS_EINVAL, "unknown scheme");
    size_t cw = 0;
    if (slab->desc.collide) {
        dgfs_status st = dgfs_workspace_size(slab->plan, slab->nodes, &cw);
        if (st != DGFS_OK) return st;
    }
    // f1, f2 (SSP-RK2) or f1 (Euler), Q, the wall-density partials, the collide workspace
    const size_t sb = state_bytes(*slab);
    *bytes = sb * (scheme == DGFS_SSPRK2 ? 3 : 2) + kPartBytes + cw;
    return DGFS_OK;
}

dgfs_status dgfs_slab_step(const dgfs_slab* slab, void* f, double dt, int32_t steps, int32_t scheme, void* workspace,
                           size_t ws_bytes, void* stream) {
    if (!slab) return dgfs::set_error(DGFS_EINVAL, "slab is NULL");
    if (steps < 0) return dgfs::set_error(DGFS_EINVAL, "steps must be >= 0");
    if (scheme != DGFS_EULER && scheme != DGFS_SSPRK2) return dgfs::set_error(DGFS_EINVAL, "unknown scheme");
    if (!std::isfinite(dt)) return dgfs::set_error(DGFS_EINVAL, "dt must be finite");
    if (steps == 0) return DGFS_OK;
    if (!f || !workspace) return dgfs::set_error(DGFS_EINVAL, "f and workspace are required");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return dgfs::set_error(DGFS_EINVAL, "workspace must be 256-byte aligned");
    size_t need = 0;
    dgfs_status rc = dgfs_slab_workspace_size(slab, scheme, &need);
    if (rc != DGFS_OK) return rc;
    if (ws_bytes < need) return dgfs::set_error(DGFS_ENOMEM, "workspace smaller than dgfs_slab_workspace_size");
    const dgfs_slab& S = *slab;
    const size_t sb = state_bytes(S);
    char* w = static_cast<char*>(workspace);
    void* f1 = w;
    void* f2 = scheme == DGFS_SSPRK2 ? w + sb : nullptr;
    void* Q = w + sb * (scheme == DGFS_SSPRK2 ? 2 : 1);
    double* nw = reinterpret_cast<double*>(w + sb * (scheme == DGFS_SSPRK2 ? 3 : 2));
    void* cw = w + sb * (scheme == DGFS_SSPRK2 ? 3 : 2) + kPartBytes;
    const size_t cwb = ws_bytes - (sb * (scheme == DGFS_SSPRK2 ? 3 : 2) + kPartBytes);
    hipStream_t st = static_cast<hipStream_t>(stream);
    auto dev = [&](hipError_t e) {
        return e == hipSuccess ? DGFS_OK
                               : dgfs::set_error(DGFS_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    };
    // out = in + dt L(in): transport into out, then the projected collision update
    auto stage = [&](const void* in, void* outp) -> dgfs_status {
        dgfs_status r = DGFS_OK;
        if (S.desc.collide && (r = dgfs_collide(S.plan, in, Q, S.nodes, cw, cwb, stream)) != DGFS_OK) return r;
        if ((r = dev(transport(S, in, outp, dt, nw, st))) != DGFS_OK) return r;
        if (S.desc.collide) r = dev(dgfs::launch_conserve(*S.plan, Q, nullptr, outp, dt, S.nodes, st));
        return r;
    };
    const int64_t n = S.nodes * S.s * int64_t(S.plan->n3());
    for (int32_t k = 0; k < steps && rc == DGFS_OK; ++k) {
        if (scheme == DGFS_EULER) {
            if ((rc = stage(f, f1)) != DGFS_OK) break;
            rc = dev(hipMemcpyAsync(f, f1, size_t(n) * S.plan->elem(), hipMemcpyDeviceToDevice, st));
            continue;
        }
        if ((rc = stage(f, f1)) != DGFS_OK) break;
        if ((rc = stage(f1, f2)) != DGFS_OK) break;
        rc = dev(dgfs::launch_axpby(*S.plan, f, f2, f, 0.5, 0.5, n, st));
    }
    return rc;
}

}  // extern "C"
