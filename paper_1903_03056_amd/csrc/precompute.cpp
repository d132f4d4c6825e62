#include "precompute.hpp"

#include <algorithm>
#include <array>
#include <cmath>

namespace dgfs {
namespace pre {

namespace {
constexpr double kPi = 3.14159265358979323846264338327950288;

// Legendre P_n(x) and P_n'(x) by the three-term recurrence.
void legendre(int n, double x, double& p, double& dp) {
    double p0 = 1.0, p1 = x;
    if (n == 0) {
        p = 1.0;
        dp = 0.0;
        return;
    }
    for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
    }
    p = p1;
    dp = n * (x * p1 - p0) / (x * x - 1.0);
}
}  // namespace

void gauss_legendre(int n, double R, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double t = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double p = 0, dp = 0;
        for (int it = 0; it < 100; ++it) {
            legendre(n, t, p, dp);
            double dt = p / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-17) break;
        }
        legendre(n, t, p, dp);
        // node t in (-1, 1), descending in i; map to [0, R] ascending
        x[n - 1 - i] = 0.5 * R * (t + 1.0);
        w[n - 1 - i] = 0.5 * R * 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

namespace {
void lexsort(std::vector<double>& pts) {
    const int M = int(pts.size() / 3);
    std::vector<std::array<double, 3>> v(M);
    for (int i = 0; i < M; ++i) v[i] = {pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]};
    std::sort(v.begin(), v.end());
    for (int i = 0; i < M; ++i)
        for (int d = 0; d < 3; ++d) pts[3 * i + d] = v[i][d];
}

// Roots of 105 t^3 - 105 t^2 + 21 t - 1 in (0, 1), ascending, by bracketing + bisection.
std::array<double, 3> cubic_roots() {
    auto p = [](double t) { return ((105.0 * t - 105.0) * t + 21.0) * t - 1.0; };
    std::array<double, 3> r{};
    int found = 0;
    const int steps = 1000;
    for (int k = 0; k < steps && found < 3; ++k) {
        double a = double(k) / steps, b = double(k + 1) / steps;
        if ((p(a) < 0) != (p(b) < 0)) {
            for (int it = 0; it < 200; ++it) {
                double m = 0.5 * (a + b);
                if ((p(a) < 0) != (p(m) < 0)) b = m; else a = m;
            }
            r[found++] = 0.5 * (a + b);
        }
    }
    return r;
}
}  // namespace

bool design(int M, std::vector<double>& pts) {
    pts.clear();
    if (M == 6) {
        for (int s : {1, -1})
            for (int d = 0; d < 3; ++d) {
                double p[3] = {0, 0, 0};
                p[d] = s;
                pts.insert(pts.end(), p, p + 3);
            }
    } else if (M == 12) {
        const double phi = 0.5 * (1.0 + std::sqrt(5.0));
        const double nrm = std::sqrt(1.0 + phi * phi);
        for (int s1 : {1, -1})
            for (int s2 : {1, -1}) {
                double x = 0.0, y = s1, z = s2 * phi;
                double cyc[3][3] = {{x, y, z}, {z, x, y}, {y, z, x}};
                for (auto& c : cyc)
                    for (double v : c) pts.push_back(v / nrm);
            }
    } else if (M == 24) {
        // Orbit of g under the 24 cube rotations (signed permutations, det +1); a
        // 7-design because the invariant harmonics of degree 4 and 6 vanish at g.
        std::array<double, 3> t = cubic_roots();
        double g[3] = {std::sqrt(t[0]), std::sqrt(t[1]), std::sqrt(t[2])};
        int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
        int parity[6] = {1, -1, -1, 1, 1, -1};
        for (int pi = 0; pi < 6; ++pi)
            for (int sgn = 0; sgn < 8; ++sgn) {
                int s[3] = {(sgn & 1) ? -1 : 1, (sgn & 2) ? -1 : 1, (sgn & 4) ? -1 : 1};
                if (parity[pi] * s[0] * s[1] * s[2] != 1) continue;
                for (int r = 0; r < 3; ++r) pts.push_back(s[r] * g[perm[pi][r]]);
            }
    } else {
        return false;
    }
    lexsort(pts);
    return true;
}

bool antipodal(const std::vector<double>& pts) {
    const int M = int(pts.size() / 3);
    for (int i = 0; i < M; ++i) {
        bool hit = false;
        for (int j = 0; j < M && !hit; ++j) {
            double d = 0;
            for (int k = 0; k < 3; ++k) d += std::fabs(pts[3 * i + k] + pts[3 * j + k]);
            hit = d < 1e-12;
        }
        if (!hit) return false;
    }
    return true;
}

double support_radius(double L, double mi, double mj) {
    return 2.0 * L / (std::max(4.0 * mj / (mi + mj), 2.0) + std::sqrt(1.0 + mj / mi) + 1.0);
}

double truncation_radius(double L, double mi, double mj) {
    return 2.0 * std::min(support_radius(L, mi, mj), support_radius(L, mj, mi));
}

double pair_prefactor(double mi, double mj, double omega, double alpha, double kn0) {
    const double mu = mi * mj / (mi + mj);
    return alpha / (kn0 * std::pow(2.0, 1.0 + alpha) * std::tgamma(2.5 - omega) * kPi * std::pow(mu, omega - 0.5));
}

double sinc(double x) {
    if (std::fabs(x) < 1e-4) {
        double x2 = x * x;
        return 1.0 - x2 / 6.0 + x2 * x2 / 120.0;
    }
    return std::sin(x) / x;
}

double kernel_mode(double kabs, double rho, double a, double gamma, double C, double L) {
    return 4.0 * kPi * C * std::pow(rho, gamma + 2.0) * sinc(kPi * a * rho * kabs / L);
}

VssSeries::VssSeries(double alpha_, int lmax) : alpha(alpha_), lam(size_t(lmax) + 1) {
    const double beta = alpha - 1.0;
    double l0 = 2.0 * kPi * std::pow(2.0, alpha) / alpha;
    for (int l = 0; l <= lmax; ++l) {
        lam[l] = (2.0 * l + 1.0) * l0;
        l0 *= (beta - l) / (beta + l + 2.0);
    }
}

int vss_terms(double z) {
    // j_l(z) < 1e-17 |j|_max well before l = z + 9 z^{1/3} + 30
    return int(z + 9.0 * std::cbrt(z) + 30.0);
}

void sph_bessel(int lmax, double z, std::vector<double>& j) {
    j.assign(size_t(lmax) + 1, 0.0);
    if (z == 0.0) {
        j[0] = 1.0;
        return;
    }
    // Miller: recur j_{l-1} = (2l+1)/z j_l - j_{l+1} downwards from far above
    // max(lmax, z), where the minimal solution dominates, then normalise by j_0 or j_1
    // (they never vanish together).
    const int top = std::max(lmax, int(z)) + int(std::sqrt(160.0 * (std::max(lmax, int(z)) + 1))) + 20;
    double jp = 0.0, jc = 1e-300;
    for (int l = top; l >= 1; --l) {
        const double jm = (2.0 * l + 1.0) / z * jc - jp;
        jp = jc;
        jc = jm;
        if (l - 1 <= lmax) j[l - 1] = jc;
        if (std::fabs(jc) > 1e250) {  // rescale what is stored and the recurrence state
            jc *= 1e-250;
            jp *= 1e-250;
            for (int m = l - 1; m <= lmax; ++m) j[m] *= 1e-250;
        }
    }
    const double s = std::sin(z), c = std::cos(z);
    const double j0 = s / z, j1 = s / (z * z) - c / z;
    double scale;
    if (std::fabs(j0) >= std::fabs(j1) || lmax < 1) scale = j0 / j[0];
    else scale = j1 / j[1];
    for (double& v : j) v *= scale;
}

void vss_sum(const VssSeries& S, const double* j, int nterms, double mu, double& re, double& im) {
    // (-i)^l cycles 1, -i, -1, i; P_l(mu) by the three-term recurrence
    double p0 = 1.0, p1 = mu;
    double r = 0.0, i = 0.0;
    for (int l = 0; l < nterms; ++l) {
        const double pl = l == 0 ? p0 : p1;
        const double t = S.lam[l] * j[l] * pl;
        switch (l & 3) {
            case 0: r += t; break;
            case 1: i -= t; break;
            case 2: r -= t; break;
            default: i += t; break;
        }
        if (l >= 1) {
            const double pn = ((2.0 * l + 1.0) * mu * p1 - l * p0) / (l + 1.0);
            p0 = p1;
            p1 = pn;
        }
    }
    re = r;
    im = i;
}

void kernel_mode_vss(const double k[3], double rho, const double sigma[3], double a, double gamma, double alpha,
                     double C, double L, double& re, double& im) {
    const double kabs = std::sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    const double mu = kabs > 0.0 ? (k[0] * sigma[0] + k[1] * sigma[1] + k[2] * sigma[2]) / kabs : 0.0;
    const double z = kPi * a * rho * kabs / L;
    const int n = vss_terms(z);
    VssSeries S(alpha, n);
    std::vector<double> j;
    sph_bessel(n, z, j);
    vss_sum(S, j.data(), n + 1, mu, re, im);
    const double f = C * std::pow(rho, gamma + 2.0);
    re *= f;
    im *= f;
}

double vss_loss_factor(double alpha) { return std::pow(2.0, alpha - 1.0) / alpha; }

namespace {
// 20-point Gauss-Legendre on [-1, 1], built once.
struct GL20 {
    std::vector<double> x, w;
    GL20() {
        gauss_legendre(20, 2.0, x, w);
        for (auto& v : x) v -= 1.0;
    }
};
const GL20& gl20() {
    static GL20 g;
    return g;
}

double composite(double R, double gamma, double kappa, int refine) {
    const GL20& g = gl20();
    auto f = [&](double r) { return std::pow(r, gamma + 2.0) * sinc(kappa * r); };
    // graded breakpoints R 2^-k, k = 0..40, each dyadic interval [u, 2u] split into
    // pieces no wider than ~ (1/refine) of the local oscillation length.
    double total = 0.0;
    double hi = R;
    for (int k = 0; k < 40; ++k) {
        double lo = hi * 0.5;
        double width = hi - lo;
        double osc = 6.0 / (1.0 + kappa);  // about one period of sinc per piece
        int pieces = std::max(1, int(std::ceil(width / osc))) * refine;
        double h = width / pieces;
        for (int p = 0; p < pieces; ++p) {
            double a = lo + p * h, c = 0.5 * h, mid = a + c;
            double s = 0.0;
            for (size_t q = 0; q < g.x.size(); ++q) s += g.w[q] * f(mid + c * g.x[q]);
            total += c * s;
        }
        hi = lo;
    }
    return total;  // the remaining [0, R 2^-40] contributes < R^{gamma+3} 2^-120
}
}  // namespace

double loss_weight(double mabs, double R, double gamma, double C, double L) {
    const double kappa = kPi * mabs / L;
    const double scale = std::pow(R, gamma + 3.0) / (gamma + 3.0);
    double prev = composite(R, gamma, kappa, 1);
    double cur = prev;
    for (int refine = 2; refine <= 64; refine *= 2) {
        cur = composite(R, gamma, kappa, refine);
        if (std::fabs(cur - prev) <= 1e-15 * scale) break;
        prev = cur;
    }
    return 16.0 * kPi * kPi * C * cur;
}

void interpolation_matrix(int N, double L_from, double L_to, std::vector<double>& T) {
    T.assign(size_t(N) * N, 0.0);
    const double h_from = 2.0 * L_from / N, h_to = 2.0 * L_to / N;
    for (int r = 0; r < N; ++r) {
        const double v = -L_to + r * h_to;
        if (!(v >= -L_from && v < L_from)) continue;
        for (int n = 0; n < N; ++n) {
            const double vn = -L_from + n * h_from;
            double acc = 0.0;
            for (int j = 0; j < N; ++j) {
                const int k = j < N / 2 ? j : j - N;
                // c_k(v) e^{-i pi k v_n / L}; the Nyquist mode uses cos(pi N v / 2L)
                const double an = -kPi * k * vn / L_from;
                if (k == -N / 2)
                    acc += std::cos(kPi * (N / 2) * v / L_from) * std::cos(an);
                else
                    acc += std::cos(kPi * k * v / L_from + an);
            }
            T[size_t(r) * N + n] = acc / N;
        }
    }
}

}  // namespace pre
}  // namespace dgfs
