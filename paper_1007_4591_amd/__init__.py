"""MI355X-native fast-multipole boundary-element electrostatics.

Thin ctypes binding of ``libbemfmm.so`` (C-ABI declared in
``include/bemfmm.h``).  The names follow the C entry points; the functions
here only marshal arguments (torch CUDA tensors -> device pointers, the
current HIP stream) and turn status codes into exceptions.  Every step of
the computation runs in the library's HIP kernels; there is no fallback.

PyTorch is used for device memory and streams only.  It is imported before
the library is loaded so both share one HIP runtime.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import build as _build

# ------------------------------------------------------------ constants
FP64, FP32, FP32_REFINED = 0, 1, 2
OP_A, OP_AT, OP_B, OP_BT, OP_C, OP_CT = range(6)
BIBEE_CFA, BIBEE_P, BIBEE_PLUS_HALF = 0, 1, 2
ENERGY_BEM, ENERGY_BIBEE_CFA, ENERGY_BIBEE_P, ENERGY_BIBEE_PLUS_HALF = 0, 1, 2, 3
MAC_THETA, MAC_ADJACENT = 0, 1
_STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENOCONV", 5: "ESTATE"}


class BemfmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bemfmm {_STATUS.get(code, code)}: {msg}")
        self.code = code


class NotConverged(BemfmmError):
    pass


class _Params(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("ncrit", ctypes.c_int), ("theta", ctypes.c_double),
                ("mac", ctypes.c_int), ("eps_in", ctypes.c_double), ("eps_out", ctypes.c_double),
                ("near_quad", ctypes.c_double)]


class _SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int), ("converged", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double)]


class _TreeInfo(ctypes.Structure):
    _fields_ = [("n_panels", ctypes.c_int64), ("n_charges", ctypes.c_int64), ("leaf_level", ctypes.c_int),
                ("n_cells", ctypes.c_int64), ("n_leaves", ctypes.c_int64), ("n_near_pairs", ctypes.c_int64),
                ("n_far_pairs", ctypes.c_int64), ("n_m2l_panel_pairs", ctypes.c_int64),
                ("n_offsets", ctypes.c_int64),
                ("p2p_pairs_panels", ctypes.c_int64), ("lo", ctypes.c_double * 3), ("side", ctypes.c_double),
                ("n_nearquad_pairs", ctypes.c_int64)]


@dataclass
class Params:
    """Tree and FMM parameters (see bemfmm_params)."""
    p: int = 10
    ncrit: int = 64
    theta: float = 0.5
    mac: int = MAC_THETA
    eps_in: float = 4.0
    eps_out: float = 80.0
    near_quad: float = 0.0

    def _c(self):
        return _Params(int(self.p), int(self.ncrit), float(self.theta), int(self.mac), float(self.eps_in),
                       float(self.eps_out), float(self.near_quad))


@dataclass
class SolveInfo:
    iters: int
    outer_iters: int
    converged: bool
    rel_residual: float
    seconds: float


_lib = None


def library_path() -> str:
    return _build.LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        raise RuntimeError(
            f"{_build.LIB} is missing: build the HIP library first (python -m paper_1007_4591_amd.build "
            "or __graft_entry__.build())")
    lib = ctypes.CDLL(_build.LIB)
    P, I64, I, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.bemfmm_build_tree.argtypes = [P, I64, P, I64, P, I64, ctypes.POINTER(_Params), P, ctypes.POINTER(P)]
    lib.bemfmm_set_charges.argtypes = [P, P, P]
    lib.bemfmm_set_charges_noalloc.argtypes = [P, P, P]
    lib.bemfmm_tree_destroy.argtypes = [P]
    lib.bemfmm_tree_get_info.argtypes = [P, ctypes.POINTER(_TreeInfo)]
    lib.bemfmm_fmm_matvec.argtypes = [P, I, I, P, P, P]
    lib.bemfmm_solve_bem.argtypes = [P, P, P, D, I, I, I, ctypes.POINTER(_SolveInfo), P]
    lib.bemfmm_bibee_energy.argtypes = [P, P, I, I, ctypes.POINTER(D), P]
    lib.bemfmm_solvation_energy.argtypes = [P, P, P, I, ctypes.POINTER(D), P]
    lib.bemfmm_adjoint_grad.argtypes = [P, P, P, D, I, I, I, P, P, ctypes.POINTER(_SolveInfo), P]
    lib.bemfmm_last_error.restype = ctypes.c_char_p
    lib.bemfmm_tree_export.argtypes = [P] + [P] * 11
    lib.bemfmm_debug_expansions.argtypes = [P, I, I, P]
    lib.bemfmm_debug_fields.argtypes = [P, I, P, P]
    lib.bemfmm_profile.argtypes = [P, I, I]
    lib.bemfmm_profile_get.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(D), ctypes.POINTER(I64)]
    lib.bemfmm_release_cache.argtypes = []
    lib.bemfmm_profile_select.argtypes = [P, I, I]
    lib.bemfmm_debug_record.argtypes = [P, I]
    lib.bemfmm_binding_energy.argtypes = [P, P, P, P, P, P, I, I, D, I, I, ctypes.POINTER(D), P]
    lib.bemfmm_lpb_matvec.argtypes = [P, D, P, P, P]
    lib.bemfmm_lpb_solve.argtypes = [P, P, D, P, D, I, I, ctypes.POINTER(_SolveInfo), P]
    lib.bemfmm_lpb_energy.argtypes = [P, P, P, ctypes.POINTER(D), P]
    for name in ("bemfmm_build_tree", "bemfmm_set_charges", "bemfmm_set_charges_noalloc", "bemfmm_tree_destroy", "bemfmm_tree_get_info",
                 "bemfmm_fmm_matvec", "bemfmm_solve_bem", "bemfmm_bibee_energy", "bemfmm_solvation_energy",
                 "bemfmm_adjoint_grad", "bemfmm_tree_export", "bemfmm_debug_expansions", "bemfmm_debug_fields",
                 "bemfmm_profile", "bemfmm_profile_get", "bemfmm_release_cache", "bemfmm_profile_select",
                 "bemfmm_debug_record", "bemfmm_binding_energy", "bemfmm_lpb_matvec", "bemfmm_lpb_solve",
                 "bemfmm_lpb_energy"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc, lib=None):
    if rc != 0:
        lib = lib or _load()
        msg = lib.bemfmm_last_error().decode()
        if rc == 4:
            raise NotConverged(rc, msg)
        raise BemfmmError(rc, msg)


def _dev():
    if not torch.cuda.is_available():
        raise RuntimeError("bemfmm needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch.device("cuda", torch.cuda.current_device())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _to_dev(a, dtype):
    if isinstance(a, torch.Tensor):
        t = a.detach()
        if t.device.type != "cuda":
            t = t.to(_dev())
        return t.to(dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), device=_dev()).to(dtype).contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


class Tree:
    """A built octree (bemfmm_tree handle) plus its sizes."""

    def __init__(self, handle, params: Params):
        self._h = handle
        self.params = params
        self.info = self._info()

    def _info(self):
        inf = _TreeInfo()
        _check(_load().bemfmm_tree_get_info(self._h, ctypes.byref(inf)))
        return {f: (list(getattr(inf, f)) if f == "lo" else getattr(inf, f)) for f, _ in _TreeInfo._fields_}

    @property
    def handle(self):
        if self._h is None:
            raise BemfmmError(5, "tree destroyed")
        return self._h

    @property
    def n_panels(self):
        return int(self.info["n_panels"])

    @property
    def n_charges(self):
        return int(self.info["n_charges"])

    def __del__(self):
        try:
            if self._h is not None and _lib is not None:
                _lib.bemfmm_tree_destroy(self._h)
                self._h = None
        except Exception:
            pass


def build_tree(verts, tris, charge_pos, params: Params | None = None, stream=None) -> Tree:
    """bemfmm_build_tree: octree, Morton order and lists on the GPU."""
    lib = _load()
    params = params or Params()
    v = _to_dev(verts, torch.float64)
    t = _to_dev(tris, torch.int32)
    q = _to_dev(charge_pos, torch.float64) if charge_pos is not None else torch.zeros((0, 3), dtype=torch.float64,
                                                                                      device=_dev())
    h = ctypes.c_void_p()
    cp = params._c()
    rc = lib.bemfmm_build_tree(_ptr(v), v.shape[0], _ptr(t), t.shape[0], _ptr(q), q.shape[0], ctypes.byref(cp),
                               _stream(stream), ctypes.byref(h))
    _check(rc, lib)
    return Tree(h, params)


def set_charges(tree: Tree, charge_pos, stream=None):
    """bemfmm_set_charges: move charges inside their leaf cells."""
    q = _to_dev(charge_pos, torch.float64)
    _check(_load().bemfmm_set_charges(tree.handle, _ptr(q), _stream(stream)))


def set_charges_noalloc(tree: Tree, charge_pos, stream=None):
    """bemfmm_set_charges_noalloc: set_charges without device allocation
    (the staging lives in the library's fixed per-device array)."""
    q = _to_dev(charge_pos, torch.float64)
    _check(_load().bemfmm_set_charges_noalloc(tree.handle, _ptr(q), _stream(stream)))


def tree_destroy(tree: Tree):
    if tree._h is not None:
        _check(_load().bemfmm_tree_destroy(tree._h))
        tree._h = None


_IN_SIZE = {OP_A: "N", OP_AT: "N", OP_B: "Q", OP_BT: "N", OP_C: "N", OP_CT: "Q"}
_OUT_SIZE = {OP_A: "N", OP_AT: "N", OP_B: "N", OP_BT: "Q", OP_C: "Q", OP_CT: "N"}


def fmm_matvec(tree: Tree, op: int, precision: int, x, y=None, stream=None):
    """bemfmm_fmm_matvec: y = op(x) (FP64 device tensors, caller order)."""
    sizes = {"N": tree.n_panels, "Q": tree.n_charges}
    xd = _to_dev(x, torch.float64)
    if xd.numel() != sizes[_IN_SIZE[op]]:
        raise ValueError(f"x has {xd.numel()} entries, operator {op} needs {sizes[_IN_SIZE[op]]}")
    n_out = sizes[_OUT_SIZE[op]]
    if y is None:
        y = torch.empty(n_out, dtype=torch.float64, device=xd.device)
    elif y.numel() != n_out or y.dtype != torch.float64 or not y.is_contiguous():
        raise ValueError("y must be a contiguous float64 tensor of the output size")
    _check(_load().bemfmm_fmm_matvec(tree.handle, int(op), int(precision), _ptr(xd), _ptr(y), _stream(stream)))
    return y


def _info(si: _SolveInfo) -> SolveInfo:
    return SolveInfo(si.iters, si.outer_iters, bool(si.converged), si.rel_residual, si.seconds)


def solve_bem(tree: Tree, q, tol=1e-6, maxit=200, restart=30, precision=FP32_REFINED, x=None, stream=None,
              raise_on_noconv=True):
    """bemfmm_solve_bem: x solving A x = f B q; returns (x, SolveInfo)."""
    qd = _to_dev(q, torch.float64)
    if x is None:
        x = torch.empty(tree.n_panels, dtype=torch.float64, device=qd.device)
    si = _SolveInfo()
    rc = _load().bemfmm_solve_bem(tree.handle, _ptr(qd), _ptr(x), float(tol), int(maxit), int(restart),
                                  int(precision), ctypes.byref(si), _stream(stream))
    if rc == 4 and not raise_on_noconv:
        return x, _info(si)
    _check(rc)
    return x, _info(si)


def lpb_matvec(tree: Tree, kappa, uv, y=None, stream=None):
    """bemfmm_lpb_matvec: y = M uv, the linearised Poisson-Boltzmann operator
    on uv = (u, v) [2N]."""
    d = _to_dev(uv, torch.float64)
    if y is None:
        y = torch.empty(2 * tree.n_panels, dtype=torch.float64, device=d.device)
    _check(_load().bemfmm_lpb_matvec(tree.handle, float(kappa), _ptr(d), _ptr(y), _stream(stream)))
    return y


def lpb_solve(tree: Tree, q, kappa, tol=1e-8, maxit=300, restart=50, uv=None, stream=None):
    """bemfmm_lpb_solve: uv = (u, v) of the screened-solvent system; returns (uv, SolveInfo)."""
    qd = _to_dev(q, torch.float64)
    if uv is None:
        uv = torch.empty(2 * tree.n_panels, dtype=torch.float64, device=qd.device)
    si = _SolveInfo()
    _check(_load().bemfmm_lpb_solve(tree.handle, _ptr(qd), float(kappa), _ptr(uv), float(tol), int(maxit),
                                    int(restart), ctypes.byref(si), _stream(stream)))
    return uv, _info(si)


def lpb_energy(tree: Tree, q, uv, stream=None) -> float:
    """bemfmm_lpb_energy: solvation energy (kcal/mol) of a solution uv."""
    qd = _to_dev(q, torch.float64)
    d = _to_dev(uv, torch.float64)
    out = ctypes.c_double()
    _check(_load().bemfmm_lpb_energy(tree.handle, _ptr(qd), _ptr(d), ctypes.byref(out), _stream(stream)))
    return out.value


def bibee_energy(tree: Tree, q, kind=BIBEE_CFA, precision=FP32, stream=None) -> float:
    qd = _to_dev(q, torch.float64)
    out = ctypes.c_double()
    _check(_load().bemfmm_bibee_energy(tree.handle, _ptr(qd), int(kind), int(precision), ctypes.byref(out),
                                       _stream(stream)))
    return out.value


def binding_energy(complex_tree: Tree, q_complex, protein_tree: Tree, q_protein, inhibitor_tree: Tree, q_inhibitor,
                   method=ENERGY_BEM, precision=FP32_REFINED, tol=1e-6, maxit=300, restart=30, stream=None) -> dict:
    """bemfmm_binding_energy: dG_bind = dG_complex - dG_protein - dG_inhibitor
    (kcal/mol), with the three parts."""
    qs = [_to_dev(q, torch.float64) for q in (q_complex, q_protein, q_inhibitor)]
    out = (ctypes.c_double * 4)()
    _check(_load().bemfmm_binding_energy(complex_tree.handle, _ptr(qs[0]), protein_tree.handle, _ptr(qs[1]),
                                         inhibitor_tree.handle, _ptr(qs[2]), int(method), int(precision), float(tol),
                                         int(maxit), int(restart), out, _stream(stream)))
    return {"binding": out[0], "complex": out[1], "protein": out[2], "inhibitor": out[3]}


def solvation_energy(tree: Tree, q, x, precision=FP64, stream=None) -> float:
    qd = _to_dev(q, torch.float64)
    xd = _to_dev(x, torch.float64)
    out = ctypes.c_double()
    _check(_load().bemfmm_solvation_energy(tree.handle, _ptr(qd), _ptr(xd), int(precision), ctypes.byref(out),
                                           _stream(stream)))
    return out.value


def adjoint_grad(tree: Tree, q, x, tol=1e-8, maxit=200, restart=30, precision=FP64, want_dq=True,
                 want_dpos=True, stream=None):
    """bemfmm_adjoint_grad: (dG/dq [Q], dG/dpos [Q,3], SolveInfo)."""
    qd = _to_dev(q, torch.float64)
    xd = _to_dev(x, torch.float64)
    Q = tree.n_charges
    dq = torch.empty(Q, dtype=torch.float64, device=qd.device) if want_dq else None
    dp = torch.empty((Q, 3), dtype=torch.float64, device=qd.device) if want_dpos else None
    si = _SolveInfo()
    _check(_load().bemfmm_adjoint_grad(tree.handle, _ptr(qd), _ptr(xd), float(tol), int(maxit), int(restart),
                                       int(precision), _ptr(dq), _ptr(dp), ctypes.byref(si), _stream(stream)))
    return dq, dp, _info(si)


def tree_export(tree: Tree) -> dict:
    """bemfmm_tree_export as numpy arrays."""
    inf = tree._info()
    N, Q, C = inf["n_panels"], inf["n_charges"], inf["n_cells"]
    NL, NN, NF = inf["n_leaves"], inf["n_near_pairs"], inf["n_far_pairs"]
    out = {
        "panel_perm": np.zeros(N, np.int32), "charge_perm": np.zeros(Q, np.int32),
        "panel_key": np.zeros(N, np.uint32), "charge_key": np.zeros(Q, np.uint32),
        "cell_key": np.zeros(C, np.uint32), "cell_level": np.zeros(C, np.int32),
        "cell_range": np.zeros((C, 4), np.int32), "cell_parent": np.zeros(C, np.int32),
        "near_ptr": np.zeros(NL + 1, np.int32), "near_idx": np.zeros(max(NN, 0), np.int32),
        "far_pairs": np.zeros((NF, 3), np.int32),
    }
    args = [out[k].ctypes.data_as(ctypes.c_void_p) if out[k].size else None for k in
            ("panel_perm", "charge_perm", "panel_key", "charge_key", "cell_key", "cell_level", "cell_range",
             "cell_parent", "near_ptr", "near_idx", "far_pairs")]
    torch.cuda.synchronize()
    _check(_load().bemfmm_tree_export(tree.handle, *args))
    out["info"] = inf
    return out


def debug_expansions(tree: Tree, precision: int, which: int) -> np.ndarray:
    p = tree.params.p
    out = np.zeros((tree.info["n_cells"], p * p))
    _check(_load().bemfmm_debug_expansions(tree.handle, int(precision), int(which),
                                           out.ctypes.data_as(ctypes.c_void_p)))
    return out


def debug_record(tree: Tree, enable: bool = True):
    """bemfmm_debug_record: later products also keep their near and far parts."""
    _check(_load().bemfmm_debug_record(tree.handle, 1 if enable else 0))


def debug_fields(tree: Tree, precision: int, n_targets: int):
    near = np.zeros(n_targets)
    far = np.zeros(n_targets)
    _check(_load().bemfmm_debug_fields(tree.handle, int(precision), near.ctypes.data_as(ctypes.c_void_p),
                                       far.ctypes.data_as(ctypes.c_void_p)))
    return near, far


def profile(tree: Tree, enable: bool, reset: bool = True):
    _check(_load().bemfmm_profile(tree.handle, 1 if enable else 0, 1 if reset else 0))


def profile_select(tree: Tree, op: int = -1, precision: int = -1):
    """Record stage times only for products of `op` at `precision` (-1: any)."""
    _check(_load().bemfmm_profile_select(tree.handle, int(op), int(precision)))


def release_cache():
    """Return the device memory the library keeps cached for reuse."""
    _check(_load().bemfmm_release_cache())


def profile_get(tree: Tree, stage: str):
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(_load().bemfmm_profile_get(tree.handle, stage.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


__all__ = [
    "FP64", "FP32", "FP32_REFINED", "OP_A", "OP_AT", "OP_B", "OP_BT", "OP_C", "OP_CT", "BIBEE_CFA", "BIBEE_P",
    "BIBEE_PLUS_HALF", "ENERGY_BEM", "ENERGY_BIBEE_CFA", "ENERGY_BIBEE_P", "ENERGY_BIBEE_PLUS_HALF", "binding_energy",
    "debug_record",
    "MAC_THETA", "MAC_ADJACENT", "Params", "SolveInfo", "Tree", "BemfmmError", "NotConverged", "build_tree",
    "set_charges", "set_charges_noalloc", "tree_destroy", "fmm_matvec", "solve_bem", "bibee_energy", "solvation_energy", "adjoint_grad",
    "tree_export", "debug_expansions", "debug_fields", "profile", "profile_get", "library_path",
    "release_cache", "profile_select", "lpb_matvec", "lpb_solve", "lpb_energy",
]
