"""Dense FP64 boundary-element solver of the linearised Poisson-Boltzmann
model (TEST INFRASTRUCTURE ONLY; see the package docstring).

Section 2.1 names the screened solvent, lap phi = kappa^2 phi outside the
molecule, as the model the method is being extended to, without giving its
integral equation.  The reading used here is the standard second-kind pair
for the surface potential u = phi and its interior normal derivative
v = d phi / dn (n outward), written out below.  With
G0 = 1/(4 pi r), Gk = exp(-kappa r)/(4 pi r), h = G0 - Gk, eps = eps_out/eps_in,
single layer V[s](x) = int G s, double layer K[m](x) = int dG/dn' m,
adjoint double layer K'[s](x) = int dG/dn_x s and D[m](x) = d/dn_x int dG/dn' m:

* interior Green identity at the boundary (Laplace, charges q_k / eps_in):
      u/2 + K0 u - V0 v = S,     S(x) = sum_k q_k G0(x, r_k) / eps_in;
* exterior identity (screened), with the exterior flux (1/eps) v:
      u/2 - Kk u + Vk v / eps = 0;
* their normal derivatives (interior limit of dV/dn is K' + 1/2, exterior
  K' - 1/2; dK/dn = D has no jump):
      v/2 - K0' v + D0 u = dS/dn,    v/(2 eps) + Kk' v / eps - Dk u = 0.

The first plus eps times the second, and the sum of the last two, give

      (1+eps)/2 u + (K0 - eps Kk) u - (V0 - Vk) v = S
      (1+1/eps)/2 v - (K0' - Kk'/eps) v + (D0 - Dk) u = dS/dn,

in which V0 - Vk has a bounded kernel and D0 - Dk one of order 1/r: both
integrable.  Collocation at the panel centroids with one point per panel
(Section 2.1) gives the 2N x 2N system.  Off-diagonal entries are a_j times the
kernel at (c_i, c_j).  Of the self entries, those of K0, Kk, K0' and Kk'
vanish for a flat panel (the kernels carry (x - x').n, zero in its plane).
The two others are integrals over panel i of radial functions of |x - c_i|,
taken exactly by polar integration about the centroid:
int_T f(R) dA = sum over edges of int F(rho(t)) dt, F(rho) = int_0^rho f(s) s ds,
rho(t) = P / cos t over the edge's angular range (P: centroid-edge distance),
with 48-point Gauss-Legendre in t per edge:
      V self: f = h,              F = (rho + expm1(-kappa rho)/kappa) / (4 pi)
      D self: f = -h'(R)/R,       F = kappa/(4 pi) + expm1(-kappa rho)/(4 pi rho).
The energy is dG = 2 pi K sum_k q_k phi_reac(r_k) (the factor 4 pi turns the
1/(4 pi r) units of G into those of K), with
phi_reac(r) = sum_j a_j (G0(r, c_j) v_j - dG0/dn_j(r, c_j) u_j), the interior
representation less the charges' own Coulomb potential.

At kappa = 0 the V and D terms cancel and the two equations decouple:
(1+eps)/2 u + (1-eps) K0 u = S and (1+1/eps)/2 v - (1-1/eps) K0' v = dS/dn,
the Poisson model in this formulation.  Pins (tests/test_oracle_lpb.py): the
screened Born ion and Kirkwood's screened sphere series (closed_forms),
converging under refinement; the small-kappa limits of the two self
integrals (V_ii / kappa -> a_i / 4 pi, D_ii / kappa^2 -> int_T 1/R dA / 8 pi,
the latter from the pinned flat-triangle formula); an adaptive quadrature of
the self integrals.
"""
from __future__ import annotations

import numpy as np

K_COULOMB = 332.06
_GL_T, _GL_W = np.polynomial.legendre.leggauss(48)


def _radial_terms(r, kappa):
    """G0, G0', G0'', Gk, Gk', Gk'' at distances r (arrays)."""
    q = 1.0 / (4.0 * np.pi)
    G0 = q / r
    G0p = -q / r ** 2
    G0pp = 2.0 * q / r ** 3
    e = np.exp(-kappa * r)
    kr = kappa * r
    Gk = q * e / r
    Gkp = -q * e * (1.0 + kr) / r ** 2
    Gkpp = q * e * (2.0 + 2.0 * kr + kr * kr) / r ** 3
    return G0, G0p, G0pp, Gk, Gkp, Gkpp


def _polar_self(verts, tris, c, F):
    """int over each panel of f(|x - c_i|) dA, from F(rho) = int_0^rho f(s) s ds."""
    V = np.asarray(verts, dtype=np.float64)[np.asarray(tris)]
    out = np.zeros(len(V))
    for e in range(3):
        a, b = V[:, e], V[:, (e + 1) % 3]
        t = b - a
        L = np.linalg.norm(t, axis=1)
        t = t / L[:, None]
        foot = a + np.einsum("ij,ij->i", c - a, t)[:, None] * t
        P = np.linalg.norm(c - foot, axis=1)
        ta = np.arctan2(np.einsum("ij,ij->i", a - foot, t), P)
        tb = np.arctan2(np.einsum("ij,ij->i", b - foot, t), P)
        mid, half = 0.5 * (ta + tb), 0.5 * (tb - ta)
        th = mid[:, None] + half[:, None] * _GL_T[None, :]
        rho = P[:, None] / np.cos(th)
        out += half * np.sum(_GL_W[None, :] * F(rho), axis=1)
    return out


def self_integrals(verts, tris, c, kappa):
    """(V_ii, D_ii): int over panel i of h(R) and of -h'(R)/R, R = |x - c_i|."""
    if kappa == 0.0:
        z = np.zeros(len(tris))
        return z, z
    q = 1.0 / (4.0 * np.pi)
    FV = lambda rho: q * (rho + np.expm1(-kappa * rho) / kappa)
    FD = lambda rho: q * (kappa + np.expm1(-kappa * rho) / rho)
    return _polar_self(verts, tris, c, FV), _polar_self(verts, tris, c, FD)


class LPB:
    """The discrete system of one mesh at (eps_in, eps_out, kappa)."""

    def __init__(self, g, verts, tris, eps_in, eps_out, kappa):
        self.g, self.eps_in, self.eps_out, self.kappa = g, float(eps_in), float(eps_out), float(kappa)
        self.eps = self.eps_out / self.eps_in
        self.Vself, self.Dself = self_integrals(verts, tris, g.c, self.kappa)

    @property
    def N(self):
        return self.g.N

    def rows(self, i0, i1):
        """Rows i0..i1-1 of the four blocks (Muu, Muv, Mvu, Mvv), each
        (i1 - i0) x N, diagonal entries included."""
        g, k, eps = self.g, self.kappa, self.eps
        ci, ni = g.c[i0:i1], g.n[i0:i1]
        d = ci[:, None, :] - g.c[None, :, :]
        r = np.linalg.norm(d, axis=2)
        own = np.zeros_like(r, dtype=bool)
        own[np.arange(i1 - i0), np.arange(i0, i1)] = True
        r = np.where(own, 1.0, r)
        G0, G0p, G0pp, Gk, Gkp, Gkpp = _radial_terms(r, k)
        nid = np.einsum("ik,ijk->ij", ni, d) / r            # n_i . d / r
        njd = np.einsum("jk,ijk->ij", g.n, d) / r           # n_j . d / r
        ninj = ni @ g.n.T
        a = g.a[None, :]
        dn_src = lambda Gp: -Gp * njd                        # dG/dn_j
        dn_tgt = lambda Gp: Gp * nid                         # dG/dn_i
        hp, hpp = G0p - Gkp, G0pp - Gkpp
        d2 = -((hpp - hp / r) * nid * njd + (hp / r) * ninj)  # d2 h / dn_i dn_j
        Muu = a * (dn_src(G0p) - eps * dn_src(Gkp))
        Muv = -a * (G0 - Gk)
        Mvu = a * d2
        Mvv = -a * (dn_tgt(G0p) - dn_tgt(Gkp) / eps)
        for M in (Muu, Muv, Mvu, Mvv):
            M[own] = 0.0
        ii = np.arange(i1 - i0)
        Muu[ii, np.arange(i0, i1)] = 0.5 * (1.0 + eps)
        Mvv[ii, np.arange(i0, i1)] = 0.5 * (1.0 + 1.0 / eps)
        Muv[ii, np.arange(i0, i1)] = -self.Vself[i0:i1]
        Mvu[ii, np.arange(i0, i1)] = self.Dself[i0:i1]
        return Muu, Muv, Mvu, Mvv

    def assemble(self):
        N = self.N
        M = np.zeros((2 * N, 2 * N))
        for i0 in range(0, N, 512):
            i1 = min(N, i0 + 512)
            Muu, Muv, Mvu, Mvv = self.rows(i0, i1)
            M[i0:i1, :N], M[i0:i1, N:] = Muu, Muv
            M[N + i0:N + i1, :N], M[N + i0:N + i1, N:] = Mvu, Mvv
        return M

    def apply(self, uv):
        """M [u; v] without assembling (row blocks)."""
        N = self.N
        uv = np.asarray(uv, dtype=np.float64)
        u, v = uv[:N], uv[N:]
        out = np.zeros(2 * N)
        for i0 in range(0, N, 512):
            i1 = min(N, i0 + 512)
            Muu, Muv, Mvu, Mvv = self.rows(i0, i1)
            out[i0:i1] = Muu @ u + Muv @ v
            out[N + i0:N + i1] = Mvu @ u + Mvv @ v
        return out

    def rhs(self, rq, q):
        """[S; dS/dn] at the centroids."""
        g = self.g
        d = g.c[:, None, :] - np.asarray(rq, dtype=np.float64)[None, :, :]
        r = np.linalg.norm(d, axis=2)
        q = np.asarray(q, dtype=np.float64)
        S = (1.0 / (4.0 * np.pi * r)) @ q / self.eps_in
        dS = (-(np.einsum("ik,ijk->ij", g.n, d) / r) / (4.0 * np.pi * r * r)) @ q / self.eps_in
        return np.concatenate([S, dS])

    def solve(self, rq, q):
        """[u; v] by a LAPACK solve of the assembled system."""
        return np.linalg.solve(self.assemble(), self.rhs(rq, q))

    def reaction_potential(self, rq, uv):
        g = self.g
        N = self.N
        u, v = uv[:N], uv[N:]
        d = np.asarray(rq, dtype=np.float64)[:, None, :] - g.c[None, :, :]
        r = np.linalg.norm(d, axis=2)
        G0 = 1.0 / (4.0 * np.pi * r)
        dG0dnj = np.einsum("jk,ijk->ij", g.n, d) / (4.0 * np.pi * r ** 3)   # n_j . (r - c_j) / (4 pi r^3)
        return (G0 * g.a[None, :]) @ v - (dG0dnj * g.a[None, :]) @ u

    def energy(self, rq, q, uv):
        """dG = 2 pi K sum_k q_k phi_reac(r_k) (kcal/mol)."""
        phi = self.reaction_potential(rq, uv)
        return 2.0 * np.pi * K_COULOMB * float(np.dot(np.asarray(q, dtype=np.float64), phi))
