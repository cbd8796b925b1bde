"""Solid harmonics and multipole / local expansions by their definitions.

TEST INFRASTRUCTURE ONLY.

Section 2.3 represents far clusters by a multipole expansion (ME) truncated
after p terms and evaluates far fields through a local expansion (LE).
p = 10 means degrees n = 0..9 (55 complex coefficients with m >= 0).  This
module defines the harmonics and the two expansions directly from the
associated Legendre functions (scipy.special.lpmv, Condon-Shortley phase),
for the 1/|x - y| kernel (the 1/(4 pi) of G is applied outside):

    R_n^m(r) = r^n     P_n^m(cos t) e^{i m phi} / (n+m)!      (regular)
    I_n^m(r) = (n-m)!  P_n^m(cos t) e^{i m phi} / r^{n+1}     (irregular)

for m >= 0, and R_n^{-m} = (-1)^m conj(R_n^m), I_n^{-m} = (-1)^m conj(I_n^m).
With these, 1/|x - y| = sum_{n,m} conj(R_n^m(y)) I_n^m(x) for |y| < |x|
(the Legendre addition theorem), so

    ME about X:  M_n^m = sum_j w_j conj(R_n^m(y_j - X)),  phi(x) = sum M_n^m I_n^m(x - X)
    LE about X:  L_n^m = sum_j w_j conj(I_n^m(y_j - X)),  phi(x) = sum L_n^m R_n^m(x - X)

Scaled, packed storage (the layout the GPU library exposes for its cells):
a cell of side s stores Mt_n^m = M_n^m / s^n and Lt_n^m = s^(n+1) L_n^m, as
p^2 reals ordered by degree n, then [Re m=0, Re m=1, Im m=1, ..., Re m=n,
Im m=n]; index(n, 0) = n^2, index of Re(n, m) = n^2 + 2m - 1, of Im(n, m) =
n^2 + 2m.  Coefficients with m < 0 follow from the symmetry above because
the weights are real.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import lpmv


def _sph(r):
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    rho = np.linalg.norm(r, axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        ct = np.where(rho > 0, r[:, 2] / rho, 1.0)
    ct = np.clip(ct, -1.0, 1.0)
    phi = np.arctan2(r[:, 1], r[:, 0])
    return rho, ct, phi


def R(n: int, m: int, r) -> np.ndarray:
    """Regular solid harmonic R_n^m at points r (k,3); complex (k,)."""
    if abs(m) > n:
        return np.zeros(np.atleast_2d(r).shape[0], dtype=np.complex128)
    if m < 0:
        return (-1) ** (-m) * np.conj(R(n, -m, r))
    rho, ct, phi = _sph(r)
    return rho ** n * lpmv(m, n, ct) * np.exp(1j * m * phi) / math.factorial(n + m)


def I(n: int, m: int, r) -> np.ndarray:
    """Irregular solid harmonic I_n^m at points r (k,3); complex (k,)."""
    if abs(m) > n:
        return np.zeros(np.atleast_2d(r).shape[0], dtype=np.complex128)
    if m < 0:
        return (-1) ** (-m) * np.conj(I(n, -m, r))
    rho, ct, phi = _sph(r)
    return math.factorial(n - m) * lpmv(m, n, ct) * np.exp(1j * m * phi) / rho ** (n + 1)


def n_coeff(p: int) -> int:
    return p * p


def index(n: int, m: int, part: str = "re") -> int:
    if m == 0:
        return n * n
    return n * n + 2 * m - (1 if part == "re" else 0)


def pack(coeffs: dict, p: int) -> np.ndarray:
    """{(n, m): complex, m >= 0} -> packed reals."""
    out = np.zeros(p * p)
    for n in range(p):
        out[index(n, 0)] = coeffs[(n, 0)].real
        for m in range(1, n + 1):
            out[index(n, m, "re")] = coeffs[(n, m)].real
            out[index(n, m, "im")] = coeffs[(n, m)].imag
    return out


def unpack(v: np.ndarray, p: int) -> dict:
    """packed reals -> {(n, m): complex} for m = -n..n."""
    c = {}
    for n in range(p):
        c[(n, 0)] = complex(v[index(n, 0)], 0.0)
        for m in range(1, n + 1):
            z = complex(v[index(n, m, "re")], v[index(n, m, "im")])
            c[(n, m)] = z
            c[(n, -m)] = (-1) ** m * np.conj(z)
    return c


def p2m(y, w, X, s, p) -> np.ndarray:
    """Packed scaled ME of monopoles w at y about X for a cell of side s."""
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    w = np.asarray(w, dtype=np.float64)
    rel = (y - np.asarray(X)[None, :])
    c = {}
    for n in range(p):
        for m in range(0, n + 1):
            c[(n, m)] = complex(np.sum(w * np.conj(R(n, m, rel)))) / s ** n
    return pack(c, p)


def p2l(y, w, X, s, p) -> np.ndarray:
    """Packed scaled LE about X (cell side s) of monopoles w at y, taken
    directly from the sources (no truncation of any ME)."""
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    w = np.asarray(w, dtype=np.float64)
    rel = (y - np.asarray(X)[None, :])
    c = {}
    for n in range(p):
        for m in range(0, n + 1):
            c[(n, m)] = complex(np.sum(w * np.conj(I(n, m, rel)))) * s ** (n + 1)
    return pack(c, p)


def eval_me(v, X, s, p, x) -> np.ndarray:
    """phi(x) = sum M_n^m I_n^m(x - X) from a packed scaled ME."""
    c = unpack(v, p)
    rel = np.atleast_2d(np.asarray(x, dtype=np.float64)) - np.asarray(X)[None, :]
    out = np.zeros(rel.shape[0], dtype=np.complex128)
    for n in range(p):
        for m in range(-n, n + 1):
            out += c[(n, m)] * s ** n * I(n, m, rel)
    return out.real


def eval_le(v, X, s, p, x) -> np.ndarray:
    """phi(x) = sum L_n^m R_n^m(x - X) from a packed scaled LE."""
    c = unpack(v, p)
    rel = np.atleast_2d(np.asarray(x, dtype=np.float64)) - np.asarray(X)[None, :]
    out = np.zeros(rel.shape[0], dtype=np.complex128)
    for n in range(p):
        for m in range(-n, n + 1):
            out += c[(n, m)] / s ** (n + 1) * R(n, m, rel)
    return out.real
