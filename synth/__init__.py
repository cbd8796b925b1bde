"""Seeded synthetic surfaces and point charges.

This module only makes inputs: triangle meshes (vertices and triangles) and
point charges (positions and values).  It holds none of the method's
arithmetic (no panel geometry, no kernels, no expansions), so both the FP64
oracle and the GPU library can consume its output without sharing code.

The surfaces stand in for the paper's molecular surfaces (Section 4 and the
Appendix use PDB structures meshed with MSMS, which are not available): a
protein-scale closed surface of 1e4..1e6 flat triangles, with charges inside
it, and many randomly rotated copies on a Cartesian lattice for the crowded
protein-solution workload of Section 4.5.

Conventions
-----------
* ``icosphere(level)``: icosahedron subdivided ``level`` times (each triangle
  into four), midpoints projected onto the unit sphere after every
  subdivision; triangles are counter-clockwise seen from outside, so the
  right-hand normal points outward.  20 * 4**level triangles.
* Real orthonormal spherical harmonics Y_lm (m = -l..l, Condon-Shortley phase)
  for the blobby radius perturbation.
* Every random draw comes from ``numpy.random.default_rng(seed)`` in the order
  documented in each function.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Problem", "icosphere", "real_sph_harm", "blobby_radius", "blobby_surface",
    "born", "kirkwood", "blobby", "crowded", "differentiation", "config",
    "random_rotations", "CONFIGS",
]


@dataclass
class Problem:
    """A surface mesh plus point charges (all float64 / int32, C order)."""
    name: str
    verts: np.ndarray      # (V, 3) float64
    tris: np.ndarray       # (N, 3) int32, CCW seen from outside
    charge_pos: np.ndarray  # (Q, 3) float64
    q: np.ndarray          # (Q,) float64, units of e
    eps_in: float = 4.0
    eps_out: float = 80.0

    @property
    def n_panels(self) -> int:
        return int(self.tris.shape[0])

    @property
    def n_charges(self) -> int:
        return int(self.q.shape[0])


def _icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ], dtype=np.float64)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, f


def icosphere(level: int):
    """Unit icosphere: returns (verts (V,3) float64, tris (N,3) int32)."""
    if level < 0:
        raise ValueError("level must be >= 0")
    v, f = _icosahedron()
    for _ in range(level):
        nv = v.shape[0]
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=0)
        e.sort(axis=1)
        key = e[:, 0] * (nv + 1) + e[:, 1]
        uniq, inv = np.unique(key, return_inverse=True)
        a = uniq // (nv + 1)
        b = uniq % (nv + 1)
        mid = v[a] + v[b]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        nf = f.shape[0]
        mid_idx = inv.reshape(3, nf).T + nv  # columns: edge01, edge12, edge20
        ab, bc, ca = mid_idx[:, 0], mid_idx[:, 1], mid_idx[:, 2]
        a0, b0, c0 = f[:, 0], f[:, 1], f[:, 2]
        f = np.concatenate([
            np.stack([a0, ab, ca], axis=1),
            np.stack([b0, bc, ab], axis=1),
            np.stack([c0, ca, bc], axis=1),
            np.stack([ab, bc, ca], axis=1),
        ], axis=0)
        v = np.concatenate([v, mid], axis=0)
    return np.ascontiguousarray(v), np.ascontiguousarray(f.astype(np.int32))


def _assoc_legendre_table(lmax: int, x: np.ndarray) -> dict:
    """P_l^m(x) for 0 <= m <= l <= lmax with the Condon-Shortley phase."""
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    P = {}
    pmm = np.ones_like(x)
    for m in range(lmax + 1):
        if m > 0:
            pmm = -(2 * m - 1) * s * pmm
        P[(m, m)] = pmm
        if m + 1 <= lmax:
            P[(m + 1, m)] = (2 * m + 1) * x * pmm
        for l in range(m + 2, lmax + 1):
            P[(l, m)] = ((2 * l - 1) * x * P[(l - 1, m)] - (l + m - 1) * P[(l - 2, m)]) / (l - m)
    return P


def real_sph_harm(lmax: int, theta: np.ndarray, phi: np.ndarray) -> dict:
    """Real orthonormal Y_lm(theta, phi) for l <= lmax, m = -l..l."""
    x = np.cos(theta)
    P = _assoc_legendre_table(lmax, x)
    Y = {}
    for l in range(lmax + 1):
        for m in range(0, l + 1):
            norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
            if m == 0:
                Y[(l, 0)] = norm * P[(l, 0)]
            else:
                Y[(l, m)] = math.sqrt(2.0) * norm * P[(l, m)] * np.cos(m * phi)
                Y[(l, -m)] = math.sqrt(2.0) * norm * P[(l, m)] * np.sin(m * phi)
    return Y


def blobby_coeffs(seed: int) -> dict:
    """a_lm ~ N(0, (0.05/l)^2) for l = 2..6, m = -l..l, drawn in that order."""
    rng = np.random.default_rng(seed)
    a = {}
    for l in range(2, 7):
        for m in range(-l, l + 1):
            a[(l, m)] = float(rng.normal(0.0, 0.05 / l))
    return a


def blobby_radius(R: float, coeffs: dict, theta, phi):
    """r(theta, phi) = R * (1 + sum a_lm Y_lm(theta, phi))."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    Y = real_sph_harm(6, theta, phi)
    s = np.zeros_like(theta)
    for (l, m), c in coeffs.items():
        s = s + c * Y[(l, m)]
    return R * (1.0 + s)


def _angles(p):
    r = np.linalg.norm(p, axis=1)
    theta = np.arccos(np.clip(p[:, 2] / r, -1.0, 1.0))
    phi = np.arctan2(p[:, 1], p[:, 0])
    return r, theta, phi


def blobby_surface(level: int, R: float, coeffs: dict):
    """Icosphere vertices pushed radially to r(theta, phi)."""
    v, f = icosphere(level)
    _, th, ph = _angles(v)
    r = blobby_radius(R, coeffs, th, ph)
    return np.ascontiguousarray(v * r[:, None]), f


def sample_interior(n: int, R: float, coeffs: dict, shrink: float, seed: int, rmax: float):
    """n points uniform in {r < shrink * r(theta, phi)} by rejection from the
    cube [-rmax, rmax]^3 (candidates drawn in batches of 4096 triples)."""
    rng = np.random.default_rng(seed)
    out = []
    have = 0
    while have < n:
        c = rng.uniform(-rmax, rmax, size=(4096, 3))
        r, th, ph = _angles(c)
        ok = r < shrink * blobby_radius(R, coeffs, th, ph)
        c = c[ok]
        out.append(c)
        have += c.shape[0]
    return np.ascontiguousarray(np.concatenate(out, axis=0)[:n])


def random_rotations(n: int, seed: int) -> np.ndarray:
    """n uniform random rotation matrices from normalised Gaussian quaternions."""
    rng = np.random.default_rng(seed)
    qv = rng.normal(size=(n, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    Rm = np.empty((n, 3, 3))
    Rm[:, 0, 0] = 1 - 2 * (y * y + z * z)
    Rm[:, 0, 1] = 2 * (x * y - z * w)
    Rm[:, 0, 2] = 2 * (x * z + y * w)
    Rm[:, 1, 0] = 2 * (x * y + z * w)
    Rm[:, 1, 1] = 1 - 2 * (x * x + z * z)
    Rm[:, 1, 2] = 2 * (y * z - x * w)
    Rm[:, 2, 0] = 2 * (x * z - y * w)
    Rm[:, 2, 1] = 2 * (y * z + x * w)
    Rm[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return Rm


# ---------------------------------------------------------------- workloads

def born(level: int = 3, R: float = 2.0, q: float = 1.0) -> Problem:
    """Sphere of radius R (icosphere), one charge q at the centre."""
    v, f = icosphere(level)
    return Problem(f"born-L{level}", v * R, f, np.zeros((1, 3)), np.array([float(q)]))


def kirkwood(level: int = 6, R: float = 20.0, n_charges: int = 100, r_max: float = 18.0,
             seed: int = 2) -> Problem:
    """Sphere of radius R with n_charges charges uniform in the ball r < r_max.

    Draw order from default_rng(seed): n Gaussian triples (directions), n
    uniforms (radius r_max * U**(1/3)), then a permutation of n/2 x (+1) and
    n/2 x (-1)."""
    v, f = icosphere(level)
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n_charges, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = r_max * rng.uniform(size=n_charges) ** (1.0 / 3.0)
    pos = d * r[:, None]
    signs = np.concatenate([np.ones(n_charges // 2), -np.ones(n_charges - n_charges // 2)])
    q = rng.permutation(signs)
    return Problem(f"kirkwood-L{level}", v * R, f, np.ascontiguousarray(pos), q)


def _blobby_charges(n, R, coeffs, seed, qmax, verts):
    rmax = 1.05 * 0.8 * float(np.linalg.norm(verts, axis=1).max())
    pos = sample_interior(n, R, coeffs, 0.8, seed, rmax)
    rng = np.random.default_rng(seed + 1)
    q = rng.uniform(-qmax, qmax, size=n)
    q = q - q.mean()
    return pos, q


def blobby(level: int = 8, R: float = 25.0, n_charges: int = 2000, shape_seed: int = 3,
           charge_seed: int = 30) -> Problem:
    """Protein-like closed surface: icosphere pushed to R(1 + sum a_lm Y_lm),
    a_lm ~ N(0, (0.05/l)^2), l = 2..6; charges uniform in r < 0.8 r(theta, phi)
    (rejection, default_rng(charge_seed)), values U[-0.8, 0.8]
    (default_rng(charge_seed + 1)) shifted to net zero.  The charges depend on
    the analytic radius only, so every mesh level shares them."""
    coeffs = blobby_coeffs(shape_seed)
    v, f = blobby_surface(level, R, coeffs)
    # the rejection box comes from the level-5 vertex radii whatever the mesh
    # level, so that every level draws the same charges
    vb, _ = blobby_surface(5, R, coeffs)
    pos, q = _blobby_charges(n_charges, R, coeffs, charge_seed, 0.8, vb * 1.02)
    return Problem(f"blobby-L{level}", v, f, pos, q)


def crowded(n_side: int = 8, spacing: float = 40.0, level: int = 5, R: float = 15.0,
            n_charges: int = 1000, shape_seed: int = 4, charge_seed: int = 400,
            rot_seed: int = 40) -> Problem:
    """n_side**3 randomly rotated copies of one blobby molecule on a cubic
    lattice of the given spacing (copy (i,j,k) centred at spacing*(i,j,k),
    i fastest)."""
    coeffs = blobby_coeffs(shape_seed)
    v, f = blobby_surface(level, R, coeffs)
    vb, _ = blobby_surface(5, R, coeffs)
    pos, q = _blobby_charges(n_charges, R, coeffs, charge_seed, 0.8, vb * 1.02)
    n = n_side ** 3
    rots = random_rotations(n, rot_seed)
    idx = np.arange(n)
    centres = spacing * np.stack([idx % n_side, (idx // n_side) % n_side, idx // (n_side * n_side)], axis=1)
    V = np.einsum("kij,vj->kvi", rots, v) + centres[:, None, :]
    P = np.einsum("kij,vj->kvi", rots, pos) + centres[:, None, :]
    T = f[None, :, :].astype(np.int64) + (np.arange(n) * v.shape[0])[:, None, None]
    return Problem(f"crowded-{n}x-L{level}",
                   np.ascontiguousarray(V.reshape(-1, 3)),
                   np.ascontiguousarray(T.reshape(-1, 3).astype(np.int32)),
                   np.ascontiguousarray(P.reshape(-1, 3)),
                   np.ascontiguousarray(np.tile(q, n)))


def differentiation(level: int = 7) -> Problem:
    """The blobby surface and charges at another mesh level (7 for the GPU,
    4 for the dense adjoint)."""
    p = blobby(level=level)
    p.name = f"diff-L{level}"
    return p


CONFIGS = {
    "born": lambda: born(3),
    "kirkwood": lambda: kirkwood(6),
    "blobby": lambda: blobby(8),
    "crowded": lambda: crowded(),
    "diff": lambda: differentiation(7),
}


def config(name: str) -> Problem:
    return CONFIGS[name]()
