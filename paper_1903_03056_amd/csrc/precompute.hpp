// Host-side FP64 precomputation for the fast spectral collision operator (Sec. 4):
// Gauss-Legendre radial rule, spherical designs, truncation radius, the kernel mode
// F(|k|, rho) and the loss weight G-(|m|) of the VHS family.
#pragma once

#include <vector>

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

// sin(x)/x with the removable point.
double sinc(double x);

// F(|k|, rho) = 4 pi C rho^{gamma+2} sinc(pi a rho |k| / L)          (alpha = 1)
double kernel_mode(double kabs, double rho, double a, double gamma, double C, double L);

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
