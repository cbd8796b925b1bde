"""Closed-form solvation energies of a dielectric sphere (pins of the oracle).

TEST INFRASTRUCTURE ONLY.

All energies in kcal/mol with K = 332.06 kcal A/(mol e^2), charges in e,
lengths in A.  A sphere of radius ``a`` (permittivity eps_in) in a medium of
permittivity eps_out, point charges q_i at r_i with |r_i| < a.

* Born ion (one charge at the centre):
      dG = -(K q^2 / 2a) (1/eps_in - 1/eps_out).
* Kirkwood reaction-field series (textbook solution of the Section 2.1
  model for a sphere):
      dG = (K/2) sum_ij q_i q_j sum_n c_n (|r_i||r_j|)^n / a^(2n+1) P_n(cos g_ij),
      c_n = (n+1)(eps_in - eps_out) / (eps_in (n eps_in + (n+1) eps_out)).
* BIBEE sphere series (eq. CFA and the scale-factor 0 and +1/2 variants of
  Section 2.2, applied to the sphere analytically): the surface charge is
  s times the normal field, with s = f (CFA: the principal-value operator
  replaced by -1/2), s = f/(1 - f/2) (P: replaced by 0) or s = f/(1 - f)
  (replaced by +1/2).  On a sphere of radius a the normal field of a charge
  at r' expands in Legendre terms n with weight (n+1) r'^n / a^(n+2), and the
  single-layer potential of the n-th surface harmonic inside the sphere is
  r^n / ((2n+1) a^(n-1)) times it, which gives the reaction-field series
  below with
      c_n = -s (n+1) / (eps_in (2n+1)).
  For n = 0, c_0 = c_0^CFA: the CFA is exact for a centred charge, whose
  normal field is uniform on the sphere.
* Linearised Poisson-Boltzmann solvent (Section 2.1: the screened equation
  lap phi = kappa^2 phi outside, no ion-exclusion layer): the same series
  with the exterior solution k_n(kappa r) P_n instead of r^(-n-1) P_n.
  Matching potential and displacement at r = a for each Legendre term gives
      c_n = ((n+1) eps_in + eps_out l_n) / (eps_in (n eps_in - eps_out l_n)),
      l_n = x k_n'(x) / k_n(x),  x = kappa a,
  with k_n the modified spherical Bessel function of the second kind
  (l_n from the ratio recurrence in _lpb_lambda; the tests check it against
  scipy.special.spherical_kn).  kappa = 0 gives l_n = -(n+1), the Kirkwood
  coefficients above; n = 0 gives the screened Born ion,
      dG = (K q^2 / 2a) (1 / (eps_out (1 + kappa a)) - 1/eps_in).
"""
from __future__ import annotations

import numpy as np

K_COULOMB = 332.06


def born(q: float, R: float, eps_in: float, eps_out: float) -> float:
    return -(K_COULOMB * q * q / (2.0 * R)) * (1.0 / eps_in - 1.0 / eps_out)


def _legendre_all(nmax: int, x: np.ndarray) -> np.ndarray:
    """P_0..P_nmax at x (Bonnet recurrence)."""
    P = np.zeros((nmax + 1,) + x.shape)
    P[0] = 1.0
    if nmax >= 1:
        P[1] = x
    for n in range(2, nmax + 1):
        P[n] = ((2 * n - 1) * x * P[n - 1] - (n - 1) * P[n - 2]) / n
    return P


def _coeffs(kind: str, nmax: int, eps_in: float, eps_out: float) -> np.ndarray:
    n = np.arange(nmax + 1, dtype=np.float64)
    f = 1.0 - eps_in / eps_out
    if kind == "exact":
        return (n + 1) * (eps_in - eps_out) / (eps_in * (n * eps_in + (n + 1) * eps_out))
    if kind == "cfa":
        return -f * (n + 1) / (eps_in * (2 * n + 1))
    if kind == "p":
        return -(f / (1.0 - 0.5 * f)) * (n + 1) / (eps_in * (2 * n + 1))
    if kind == "plus_half":
        return -(f / (1.0 - f)) * (n + 1) / (eps_in * (2 * n + 1))
    raise ValueError(kind)


def _series_matrix(pos, a, nmax, c):
    pos = np.asarray(pos, dtype=np.float64)
    r = np.linalg.norm(pos, axis=1)
    rr = np.outer(r, r)
    with np.errstate(invalid="ignore", divide="ignore"):
        cosg = (pos @ pos.T) / rr
    cosg = np.where(rr > 0, cosg, 1.0)
    cosg = np.clip(cosg, -1.0, 1.0)
    P = _legendre_all(nmax, cosg)
    t = rr / (a * a)
    M = np.zeros_like(rr)
    tn = np.ones_like(rr)
    for n in range(nmax + 1):
        M += c[n] * tn * P[n]
        tn = tn * t
    return M / a  # (K/2) q^T M q is the energy


def sphere_energy(pos, q, a, eps_in, eps_out, kind="exact", nmax=60) -> float:
    """Solvation energy of charges inside a sphere: kind in {exact, cfa, p, plus_half}."""
    q = np.asarray(q, dtype=np.float64)
    M = _series_matrix(pos, a, nmax, _coeffs(kind, nmax, eps_in, eps_out))
    return 0.5 * K_COULOMB * float(q @ M @ q)


def sphere_energy_grad_q(pos, q, a, eps_in, eps_out, kind="exact", nmax=60) -> np.ndarray:
    """d dG / d q_i = K sum_j M_ij q_j (M symmetric)."""
    q = np.asarray(q, dtype=np.float64)
    M = _series_matrix(pos, a, nmax, _coeffs(kind, nmax, eps_in, eps_out))
    return K_COULOMB * (M @ q)


def born_screened(q: float, R: float, eps_in: float, eps_out: float, kappa: float) -> float:
    return (K_COULOMB * q * q / (2.0 * R)) * (1.0 / (eps_out * (1.0 + kappa * R)) - 1.0 / eps_in)


def _lpb_lambda(nmax: int, x: float) -> np.ndarray:
    """l_n = x k_n'(x) / k_n(x) = n - x k_{n+1}(x)/k_n(x), with the ratio
    r_n = k_{n+1}/k_n from r_0 = 1 + 1/x and the three-term recurrence
    k_{n+1} = k_{n-1} + (2n+1)/x k_n, i.e. r_n = 1/r_{n-1} + (2n+1)/x (no
    overflow at small x, where k_n itself does)."""
    n = np.arange(nmax + 1, dtype=np.float64)
    if x == 0.0:
        return -(n + 1)
    r = np.zeros(nmax + 1)
    r[0] = 1.0 + 1.0 / x
    for k in range(1, nmax + 1):
        r[k] = 1.0 / r[k - 1] + (2 * k + 1) / x
    return n - x * r


def _coeffs_lpb(nmax: int, eps_in: float, eps_out: float, kappa: float, a: float) -> np.ndarray:
    n = np.arange(nmax + 1, dtype=np.float64)
    lam = _lpb_lambda(nmax, kappa * a)
    return ((n + 1) * eps_in + eps_out * lam) / (eps_in * (n * eps_in - eps_out * lam))


def sphere_energy_lpb(pos, q, a, eps_in, eps_out, kappa, nmax=60) -> float:
    """Solvation energy of charges inside a sphere in a screened (linearised
    Poisson-Boltzmann) solvent with inverse Debye length kappa (1/A)."""
    q = np.asarray(q, dtype=np.float64)
    M = _series_matrix(pos, a, nmax, _coeffs_lpb(nmax, eps_in, eps_out, kappa, a))
    return 0.5 * K_COULOMB * float(q @ M @ q)
