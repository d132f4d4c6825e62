// Host-side FP64 precomputation for the fast spectral collision operator (Sec. 4):
// Gauss-Legendre radial rule, spherical designs, truncation radius, the kernel mode
// F(|k|, rho) and the loss weight G-(|m|) of the VHS family, and the sigma-dependent
// kernel mode of the VSS family.
#pragma once

#include <vector>
#include <complex>

namespace dgfs {
namespace pre {

// Gauss-Legendre nodes/weights on [0, R], ascending (Newton on P_n).
void gauss_legendre(int n, double R, std::vector<double>& x, std::vector<double>& w);

// Spherical design of M points (6, 12, 24) as [M][3], lexicographically sorted by
// (x, y, z).  Returns false for an unsupported M.
bool design(int M, std::vector<double>& pts);

// True when the point set is closed under p -> -p.
bool antipodal(const std::vector<double>& pts);

// Largest support radius S allowed by the anti-aliasing condition (Sec. 4,
// eq. domain) for the ordered pair (i, j), and R_ij = 2 min(S_ij, S_ji).
double support_radius(double L, double mi, double mj);
double truncation_radius(double L, double mi, double mj);

// C_ij = Kn_ij^{-1} times the constant of the dimensionless VSS kernel (Sec. 3, eqs. Kn
// and NVSS).  Kn_ij^{-1} carries sqrt(1 + m_i/m_j) and the kernel constant divides by it,
// leaving alpha / (Kn0 2^{1+alpha} Gamma(5/2 - omega) pi mu_ij^{omega - 1/2}) with the
// reduced mass mu_ij = m_i m_j / (m_i + m_j); symmetric in (i, j).
double pair_prefactor(double mi, double mj, double omega, double alpha, double kn0);

// sin(x)/x with the removable point.
double sinc(double x);

// F(|k|, rho) = 4 pi C rho^{gamma+2} sinc(pi a rho |k| / L)          (alpha = 1)
double kernel_mode(double kabs, double rho, double a, double gamma, double C, double L);

// Variable soft spheres (Sec. 2 eq. VSS, 1 < alpha <= 2): B = C rho^gamma (1 + sigma.g_hat)^{alpha-1}.
// The kernel mode of Sec. 4 (below eq. GG) then depends on mu = sigma.k_hat.  With the
// plane-wave expansion of e^{-i z k_hat.g_hat} and the Funk-Hecke formula,
//   F(k, rho, sigma) = C rho^{gamma+2} sum_l (2l+1) (-i)^l lambda_l j_l(z) P_l(mu),
//   z = pi a rho |k| / L,  lambda_l = 2 pi int_{-1}^{1} (1+t)^{alpha-1} P_l(t) dt,
// where lambda_0 = 2 pi 2^alpha / alpha and lambda_{l+1} = lambda_l (beta - l)/(beta + l + 2),
// beta = alpha - 1 (from the closed form of int (1+t)^beta P_l).  The series is cut where
// j_l(z) has fallen below double precision.
struct VssSeries {
    double alpha = 1.0;
    std::vector<double> lam;  // (2l+1) (-i)^l lambda_l up to the real/imaginary split: (2l+1) lambda_l
    explicit VssSeries(double alpha_, int lmax);
};
// Number of terms of the series at argument z.
int vss_terms(double z);
// j_0(z) .. j_lmax(z) (spherical Bessel functions of the first kind).
void sph_bessel(int lmax, double z, std::vector<double>& j);
// sum_l (2l+1) (-i)^l lambda_l j_l P_l(mu) for precomputed j = j_l(z), l < nterms; real and
// imaginary parts in re, im.
void vss_sum(const VssSeries& S, const double* j, int nterms, double mu, double& re, double& im);
// F(k, rho, sigma) for the signed mode vector k (complex result in re, im).
void kernel_mode_vss(const double k[3], double rho, const double sigma[3], double a, double gamma, double alpha,
                     double C, double L, double& re, double& im);
// int_{S^2} (1 + sigma.g_hat)^{alpha-1} dsigma / (4 pi) = 2^{alpha-1} / alpha: the factor the
// loss weight G- of the VHS family gains for a VSS kernel.
double vss_loss_factor(double alpha);

// G-(|m|) = 16 pi^2 C int_0^R rho^{gamma+2} sinc(pi rho |m| / L) d rho, by composite
// Gauss-Legendre on panels graded geometrically towards rho = 0 (where rho^{gamma+2}
// is not smooth for fractional gamma) and no wider than the oscillation allows;
// the panel count is doubled until two values agree to 1e-15 of the integrand scale.
double loss_weight(double mabs, double R, double gamma, double C, double L);

// One-dimensional map between two grids of N points, v_n = -L + n 2L/N: row n' holds the
// weights that evaluate, at point n' of the grid L_to, the real trigonometric interpolant
// of samples on the grid L_from (modes -N/2..N/2-1, the Nyquist mode split evenly between
// +N/2 and -N/2).  Rows of points outside [-L_from, L_from) are zero.  T is [N][N].
void interpolation_matrix(int N, double L_from, double L_to, std::vector<double>& T);

}  // namespace pre
}  // namespace dgfs
