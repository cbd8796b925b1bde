"""ctypes front end of the FP64 dense oracle (bem_dense.c).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Equations (Section 2.1 matrix statement, eq. ASC, eq. reac, the solvation
energy, and eq. CFA of Section 2.2), with the readings fixed where the text
is ambiguous:

* A = (1 - f/2) I - f K',  f = 1 - eps_in/eps_out, K'_ii = 0 (flat panels);
  the right-hand side is f E with E = B q the normal field of the charges.
  (Interior limit of the normal derivative of the single layer in eq. ASC.)
* dG = (2 pi K / eps_in) q^T C x: eq. ASC carries no 1/eps_in on the charge
  term, so the reaction potential of the energy formula is (1/eps_in) times
  4 pi K times the single-layer potential of x.
* BIBEE (Section 2.2, eq. CFA and the sentence after it): the
  principal-value operator K' is replaced by a scaled identity, -1/2 I for
  BIBEE/CFA (x = f E), 0 for BIBEE/P (x = f E / (1 - f/2)) and +1/2 I for
  the third variant (x = f E / (1 - f)); the interior jump +1/2 of the
  normal derivative stays in every case.
* Binding (Section 4.4, eq. binding-free-energy-estimate): the solvation
  energy of the complex minus those of the two unbound partners.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

K_COULOMB = 332.06  # kcal A / (mol e^2)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bem_dense.c")
_LIB_PATH = os.path.join(_HERE, "libbem_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile bem_dense.c with gcc (plain C, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
            "-fno-fast-math", "-o", tmp, _SRC, "-lm",
        ])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            P = ctypes.c_void_p
            I = ctypes.c_int64
            D = ctypes.c_double
            lib.or_geometry.argtypes = [P, I, P, I, P, P, P]
            lib.or_geometry.restype = ctypes.c_int
            lib.or_field_B.argtypes = [P, P, I, P, P, I, P]
            lib.or_apply_Kp_rows.argtypes = [P, P, P, I, P, P, I, P]
            lib.or_apply_A_rows.argtypes = [P, P, P, I, D, P, P, I, P]
            lib.or_apply_KpT_rows.argtypes = [P, P, P, I, P, P, I, P]
            lib.or_apply_AT_rows.argtypes = [P, P, P, I, D, P, P, I, P]
            lib.or_apply_C.argtypes = [P, P, I, P, I, P, P]
            lib.or_apply_CT.argtypes = [P, P, I, P, P, I, P]
            lib.or_apply_BT.argtypes = [P, P, I, P, I, P, P]
            lib.or_grad_at_points.argtypes = [P, P, I, P, P, P, I, P]
            lib.or_assemble_A.argtypes = [P, P, P, I, D, P]
            lib.or_gmres.argtypes = [P, P, P, I, D, ctypes.c_int, P, P, D, ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
            lib.or_gmres.restype = ctypes.c_int
            _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Geometry:
    c: np.ndarray  # (N,3) centroids
    n: np.ndarray  # (N,3) outward unit normals
    a: np.ndarray  # (N,) areas

    @property
    def N(self):
        return int(self.a.shape[0])


def geometry(verts, tris) -> Geometry:
    """Centroid, outward unit normal and area of every flat triangle
    (Section 2.1: planar triangles, one centroid quadrature point)."""
    lib = _load()
    verts = _f64(verts)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    N = tris.shape[0]
    c = np.zeros((N, 3)); n = np.zeros((N, 3)); a = np.zeros(N)
    rc = lib.or_geometry(_p(verts), verts.shape[0], _p(tris), N, _p(c), _p(n), _p(a))
    if rc != 0:
        raise ValueError(f"invalid mesh (code {rc})")
    return Geometry(c, n, a)


def f_factor(eps_in, eps_out):
    return 1.0 - eps_in / eps_out


def kappa(eps_in):
    """Energy prefactor 2 pi K / eps_in (kcal/mol per e * potential unit)."""
    return 2.0 * np.pi * K_COULOMB / eps_in


def field_B(g: Geometry, rq, q):
    """E = B q: normal field of the charges at the centroids."""
    lib = _load(); rq = _f64(rq); q = _f64(q)
    E = np.zeros(g.N)
    lib.or_field_B(_p(g.c), _p(g.n), g.N, _p(rq), _p(q), q.shape[0], _p(E))
    return E


def apply_A(g: Geometry, f, x, rows=None):
    lib = _load(); x = _f64(x)
    if rows is None:
        out = np.zeros(g.N)
        lib.or_apply_A_rows(_p(g.c), _p(g.n), _p(g.a), g.N, f, _p(x), None, 0, _p(out))
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.zeros(rows.shape[0])
        lib.or_apply_A_rows(_p(g.c), _p(g.n), _p(g.a), g.N, f, _p(x), _p(rows), rows.shape[0], _p(out))
    return out


def apply_AT(g: Geometry, f, y, rows=None):
    lib = _load(); y = _f64(y)
    if rows is None:
        out = np.zeros(g.N)
        lib.or_apply_AT_rows(_p(g.c), _p(g.n), _p(g.a), g.N, f, _p(y), None, 0, _p(out))
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.zeros(rows.shape[0])
        lib.or_apply_AT_rows(_p(g.c), _p(g.n), _p(g.a), g.N, f, _p(y), _p(rows), rows.shape[0], _p(out))
    return out


def apply_Kp(g: Geometry, x, rows=None):
    lib = _load(); x = _f64(x)
    rows_a = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    R = g.N if rows is None else rows_a.shape[0]
    out = np.zeros(R)
    lib.or_apply_Kp_rows(_p(g.c), _p(g.n), _p(g.a), g.N, _p(x), _p(rows_a), 0 if rows is None else R, _p(out))
    return out


def apply_C(g: Geometry, rq, x):
    lib = _load(); rq = _f64(rq); x = _f64(x)
    out = np.zeros(rq.shape[0])
    lib.or_apply_C(_p(g.c), _p(g.a), g.N, _p(rq), rq.shape[0], _p(x), _p(out))
    return out


def apply_CT(g: Geometry, rq, q):
    lib = _load(); rq = _f64(rq); q = _f64(q)
    out = np.zeros(g.N)
    lib.or_apply_CT(_p(g.c), _p(g.a), g.N, _p(rq), _p(q), q.shape[0], _p(out))
    return out


def apply_BT(g: Geometry, rq, y):
    lib = _load(); rq = _f64(rq); y = _f64(y)
    out = np.zeros(rq.shape[0])
    lib.or_apply_BT(_p(g.c), _p(g.n), g.N, _p(rq), rq.shape[0], _p(y), _p(out))
    return out


def grad_at_points(g: Geometry, rq, w=None, d=None):
    """grad of SL(w) + DL(d) (monopoles w_j, dipoles d_j n_j at c_j) at rq."""
    lib = _load(); rq = _f64(rq)
    w = None if w is None else _f64(w)
    d = None if d is None else _f64(d)
    out = np.zeros((rq.shape[0], 3))
    lib.or_grad_at_points(_p(g.c), _p(g.n), g.N, _p(w), _p(d), _p(rq), rq.shape[0], _p(out))
    return out


def assemble_A(g: Geometry, f):
    lib = _load()
    Am = np.zeros((g.N, g.N))
    lib.or_assemble_A(_p(g.c), _p(g.n), _p(g.a), g.N, f, _p(Am))
    return Am


@dataclass
class SolveInfo:
    iters: int
    rel_residual: float
    converged: bool


def gmres(g: Geometry, f, b, tol=1e-8, maxit=500, restart=0, transpose=False):
    """Restarted GMRES on A (or A^T) from x0 = 0 (see bem_dense.c)."""
    lib = _load(); b = _f64(b)
    x = np.zeros(g.N)
    it = ctypes.c_int(0); rr = ctypes.c_double(0.0)
    rc = lib.or_gmres(_p(g.c), _p(g.n), _p(g.a), g.N, f, 1 if transpose else 0, _p(b), _p(x), tol,
                      int(maxit), int(restart), ctypes.byref(it), ctypes.byref(rr))
    return x, SolveInfo(it.value, rr.value, rc == 0)


def solve(g: Geometry, rq, q, eps_in, eps_out, tol=1e-8, maxit=500, restart=0):
    """x solving A x = f E (the induced surface charge density)."""
    f = f_factor(eps_in, eps_out)
    b = f * field_B(g, rq, q)
    return gmres(g, f, b, tol, maxit, restart)


def solvation_energy(g: Geometry, rq, q, x, eps_in):
    """dG = kappa q^T C x in kcal/mol."""
    phi = apply_C(g, rq, x)
    return kappa(eps_in) * float(np.dot(_f64(q), phi))


def bibee_x(g: Geometry, rq, q, eps_in, eps_out, kind="cfa"):
    f = f_factor(eps_in, eps_out)
    E = field_B(g, rq, q)
    if kind == "cfa":
        return f * E
    if kind == "p":
        return f * E / (1.0 - 0.5 * f)
    if kind == "plus_half":
        return f * E / (1.0 - f)
    raise ValueError(kind)


def bibee_energy(g: Geometry, rq, q, eps_in, eps_out, kind="cfa"):
    return solvation_energy(g, rq, q, bibee_x(g, rq, q, eps_in, eps_out, kind), eps_in)


def molecule_energy(verts, tris, rq, q, eps_in, eps_out, method="bem", tol=1e-10, maxit=500, restart=0):
    """Solvation energy of one molecule (surface mesh plus charges) in
    kcal/mol: method "bem" solves the full system, "cfa", "p" or "plus_half"
    takes the BIBEE surface charge."""
    g = geometry(verts, tris)
    if method == "bem":
        x, _ = solve(g, rq, q, eps_in, eps_out, tol=tol, maxit=maxit, restart=restart)
    else:
        x = bibee_x(g, rq, q, eps_in, eps_out, method)
    return solvation_energy(g, rq, q, x, eps_in)


def binding_energy(complex_, protein, inhibitor, eps_in, eps_out, method="bem", tol=1e-10):
    """dG_bind = dG_complex - dG_protein - dG_inhibitor (Section 4.4, eq.
    binding-free-energy-estimate); each argument is (verts, tris, rq, q).
    Returns (bind, complex, protein, inhibitor)."""
    parts = [molecule_energy(*m, eps_in, eps_out, method=method, tol=tol) for m in (complex_, protein, inhibitor)]
    return (parts[0] - parts[1] - parts[2], parts[0], parts[1], parts[2])


def adjoint_grad(g: Geometry, rq, q, x, eps_in, eps_out, tol=1e-10, maxit=500, restart=0):
    """(d dG/dq [Q], d dG/d r_q [Q,3], y, info) for dG = kappa q^T C A^-1 f B q.

    A^T y = C^T q;  d dG/dq = kappa (C x + f B^T y);
    d dG/dr_q = kappa q_q [grad SL(a x) + f grad DL(y)](r_q)."""
    f = f_factor(eps_in, eps_out)
    kap = kappa(eps_in)
    ct = apply_CT(g, rq, q)
    y, info = gmres(g, f, ct, tol, maxit, restart, transpose=True)
    dq = kap * (apply_C(g, rq, x) + f * apply_BT(g, rq, y))
    gr = grad_at_points(g, rq, w=g.a * _f64(x), d=f * y)
    dpos = kap * _f64(q)[:, None] * gr
    return dq, dpos, y, info


__all__ = [
    "K_COULOMB", "build", "Geometry", "geometry", "f_factor", "kappa", "field_B", "apply_A",
    "apply_AT", "apply_Kp", "apply_C", "apply_CT", "apply_BT", "grad_at_points", "assemble_A",
    "SolveInfo", "gmres", "solve", "solvation_energy", "bibee_x", "bibee_energy", "adjoint_grad",
    "molecule_energy", "binding_energy",
]
