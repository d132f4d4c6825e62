"""The nodal discontinuous Galerkin discretisation of the 1-D slab (Sec. 5), in FP64
(oracle; test infrastructure).

Physical space [x0, x1] is cut into Ne equal elements; on each, every species' f is
the Lagrange interpolant through the K Gauss-Lobatto-Legendre (GLL) points (eq. of the
nodal basis in Sec. 5.1).  With the GLL points also used as quadrature points:

* the mass matrix is diagonal, M_mm = (h/2) w_m;
* the stiffness matrix S_ml = int phi_l d(phi_m)/dx dx is w_l D_lm, with D_lm the
  derivative of the m-th Lagrange polynomial at point l (the GLL rule with K points is
  exact for the degree 2K - 3 integrand);
* the collision tensor H is diagonal, H_mll = (h/2) w_m (the Sec. 5.1 example: K = 3
  gives 1/3, 4/3, 1/3 on the standard element), so the collision term at node m is
  Q(F_m) (with the pair prefactors already holding 1/Kn_ij).

Weak form (eq. weakForm) per element, node m, species i and velocity v (1-D: v . grad
uses v_x only):

    (h/2) w_m dF_m/dt = v_x sum_l w_l D_lm F_l - [phi_m F* . n] on the faces + (h/2) w_m Q_m,

with the upwind flux (eq. flux): at the right face (n = +1) F* = v_x f(inside) when
v_x >= 0 and v_x f(outside) otherwise; at the left face (n = -1) the flux normal
component is -v_x f*, f* = f(inside) when v_x <= 0.  Outside the domain the state is
given by the boundary conditions of Sec. 2:

* inflow equilibrium (eq. bc_inlet): a Maxwellian with prescribed density, velocity
  and temperature, for the incoming velocities;
* purely diffuse wall (eq. bc_wall with accommodation 1): n_w times the wall Maxwellian,
  with n_w from eq. bc_nwall (zero net mass flux through the wall), its velocity
  integrals taken as sums over the velocity grid.

The Maxwellian is the nondimensional one of Sec. 3,
n (m/(pi T))^{3/2} exp(-m |v - u|^2 / T).

Time stepping: ``stepping.ssprk2`` with L(f) = transport(f) + P(Q(f)) at every node.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from numpy.polynomial import legendre as Lg

from . import grids as G
from . import moments as Mo
from . import spectral as S


def gll(K: int):
    """GLL points (ascending, the ends -1 and 1 included) and weights on [-1, 1]: the
    interior points are the roots of P'_{K-1}, the weights 2 / (K (K-1) P_{K-1}(x)^2)."""
    if K < 2:
        raise ValueError("K >= 2")
    c = np.zeros(K)
    c[-1] = 1.0
    inner = np.sort(Lg.legroots(Lg.legder(c))) if K > 2 else np.array([])
    x = np.concatenate([[-1.0], inner, [1.0]])
    w = 2.0 / (K * (K - 1) * Lg.legval(x, c) ** 2)
    return x, w


def lagrange_derivative(x: np.ndarray) -> np.ndarray:
    """D[q, m] = d phi_m / d xi at x_q for the Lagrange basis through the points x
    (barycentric form)."""
    K = len(x)
    lam = np.array([1.0 / np.prod([x[m] - x[n] for n in range(K) if n != m]) for m in range(K)])
    D = np.zeros((K, K))
    for q in range(K):
        for m in range(K):
            if q != m:
                D[q, m] = lam[m] / lam[q] / (x[q] - x[m])
        D[q, q] = -D[q].sum()
    return D


def maxwellian(N: int, L: float, m: float, n: float, u, T: float) -> np.ndarray:
    v = Mo.grid(N, L)
    u = np.asarray(u, dtype=np.float64)
    e = [np.exp(-m * (v - u[a]) ** 2 / T) for a in range(3)]
    return n * (m / (np.pi * T)) ** 1.5 * e[0][:, None, None] * e[1][None, :, None] * e[2][None, None, :]


@dataclass
class Boundary:
    """kind 'inflow' (n per species, u, T) or 'wall' (u, T; purely diffuse)."""
    kind: str
    u: tuple = (0.0, 0.0, 0.0)
    T: float = 1.0
    n: tuple = ()


@dataclass
class Slab:
    x0: float
    x1: float
    Ne: int
    K: int
    masses: tuple
    N: int
    Ls: tuple                # velocity half-width per species
    left: Boundary
    right: Boundary
    xi: np.ndarray = field(init=False)
    w: np.ndarray = field(init=False)
    D: np.ndarray = field(init=False)

    def __post_init__(self):
        self.xi, self.w = gll(self.K)
        self.D = lagrange_derivative(self.xi)

    @property
    def h(self) -> float:
        return (self.x1 - self.x0) / self.Ne

    @property
    def s(self) -> int:
        return len(self.masses)

    def node_positions(self) -> np.ndarray:
        """[Ne][K] physical coordinates of the nodes (affine map of Sec. 5.1)."""
        xl = self.x0 + self.h * np.arange(self.Ne)
        return xl[:, None] * (1 - self.xi[None, :]) / 2 + (xl[:, None] + self.h) * (1 + self.xi[None, :]) / 2

    def vx(self, i: int) -> np.ndarray:
        return Mo.grid(self.N, self.Ls[i])[:, None, None]

    def exterior(self, bc: Boundary, trace: np.ndarray, normal: float) -> np.ndarray:
        """Outside state [s][N][N][N] at a boundary with outward normal +-1 (x direction),
        given the inside trace there."""
        out = np.zeros_like(trace)
        for i in range(self.s):
            m, L = self.masses[i], self.Ls[i]
            if bc.kind == "inflow":
                out[i] = maxwellian(self.N, L, m, bc.n[i], bc.u, bc.T)
                continue
            Mw = maxwellian(self.N, L, m, 1.0, bc.u, bc.T)
            vn = np.broadcast_to((self.vx(i) - bc.u[0]) * normal, trace[i].shape)
            num = -np.sum(np.where(vn >= 0, vn * trace[i], 0.0))
            den = np.sum(np.where(vn < 0, vn * Mw, 0.0))
            out[i] = (num / den) * Mw
        return out

    def transport(self, F: np.ndarray) -> np.ndarray:
        """dF/dt of the transport part: F [Ne][K][s][N][N][N]."""
        Ne, K, h = self.Ne, self.K, self.h
        out = np.zeros_like(F)
        ext_left = self.exterior(self.left, F[0, 0], -1.0)
        ext_right = self.exterior(self.right, F[Ne - 1, K - 1], +1.0)
        for e in range(Ne):
            outside_l = F[e - 1, K - 1] if e > 0 else ext_left
            outside_r = F[e + 1, 0] if e < Ne - 1 else ext_right
            for i in range(self.s):
                vx = self.vx(i)
                for m in range(K):
                    vol = vx * sum(self.w[l] * self.D[l, m] * F[e, l, i] for l in range(K))
                    face = np.zeros_like(vol)
                    if m == K - 1:      # right face, n = +1: subtract v_x f*
                        fstar = np.where(vx >= 0, F[e, K - 1, i], outside_r[i])
                        face -= vx * fstar
                    if m == 0:          # left face, n = -1: subtract (-v_x) f*
                        fstar = np.where(vx <= 0, F[e, 0, i], outside_l[i])
                        face += vx * fstar
                    out[e, m, i] = 2.0 / (h * self.w[m]) * (vol + face)
        return out

    def boundary_mass_flux(self, F: np.ndarray) -> np.ndarray:
        """Per species: the net inflow of mass through both ends of the slab under the
        upwind fluxes, sum over v of (v_x f* at x0) - (v_x f* at x1), times h_v^3."""
        Ne, K = self.Ne, self.K
        ext_left = self.exterior(self.left, F[0, 0], -1.0)
        ext_right = self.exterior(self.right, F[Ne - 1, K - 1], +1.0)
        out = np.zeros(self.s)
        for i in range(self.s):
            vx = self.vx(i)
            fl = np.where(vx <= 0, F[0, 0, i], ext_left[i])
            fr = np.where(vx >= 0, F[Ne - 1, K - 1, i], ext_right[i])
            out[i] = np.sum(vx * fl - vx * fr) * (2 * self.Ls[i] / self.N) ** 3
        return out

    def mass(self, F: np.ndarray) -> np.ndarray:
        """Per species: the total mass sum_e sum_m (h/2) w_m n(F_em) (GLL quadrature)."""
        out = np.zeros(self.s)
        for i in range(self.s):
            hv3 = (2 * self.Ls[i] / self.N) ** 3
            out[i] = sum(self.h / 2 * self.w[m] * F[e, m, i].sum() * hv3 for e in range(self.Ne) for m in range(self.K))
        return out


def slab_rhs(slab: Slab, prob, collide: bool = True, project: bool = True):
    """L(F) = transport(F) + P(Q(F_node)) at every node (Q from the oracle operator)."""
    Ls = tuple(slab.Ls)

    def rhs(F):
        out = slab.transport(F)
        if collide:
            for e in range(slab.Ne):
                for m in range(slab.K):
                    f = F[e, m]
                    Q = S.collide(f, prob) if len(set(Ls)) == 1 else G.collide(f, prob, Ls)
                    out[e, m] += Mo.conserve(Q, prob.masses, Ls) if project else Q
        return out
    return rhs
