"""Parity at the benchmark's full sizes, in the launch configuration that
bench.py times (p = 10, theta = 0.5, ncrit = 64): sampled outputs that the
oracle computes one by one, energies where the dense oracle is affordable,
finite differences on the differentiation workload, and invariances."""
import numpy as np
import pytest

import oracle
import synth

from gpu_common import requires_gpu, lib, dev, host, rel_l2

pytestmark = [pytest.mark.gpu, requires_gpu]
EPS_IN, EPS_OUT = 4.0, 80.0
F = 1.0 - EPS_IN / EPS_OUT


def _sampled_rows(name, make, nrows, seed):
    B = lib()
    p = make()
    print(f"[full] {name} N={p.n_panels} Q={p.n_charges}", flush=True)
    g = oracle.geometry(p.verts, p.tris)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params())
    rng = np.random.default_rng(seed)
    x = rng.normal(size=p.n_panels)
    rows = np.sort(rng.choice(p.n_panels, size=nrows, replace=False))
    want = oracle.apply_A(g, F, x, rows=rows)
    wantT = oracle.apply_AT(g, F, x, rows=rows)
    out = {}
    for prec in (1, 0):
        got = host(B.fmm_matvec(t, 0, prec, dev(x)))[rows]
        gotT = host(B.fmm_matvec(t, 1, prec, dev(x)))[rows]
        out[prec] = (rel_l2(got, want), rel_l2(gotT, wantT))
        print(f"    prec={prec} A err={out[prec][0]:.2e} A^T err={out[prec][1]:.2e}", flush=True)
    return out, t


def test_blobby_full_sampled_rows():
    errs, t = _sampled_rows("blobby-L8", lambda: synth.blobby(8), 256, 3)
    for prec in (0, 1):
        assert errs[prec][0] <= 1e-5 and errs[prec][1] <= 1e-5


def test_crowded_full_sampled_rows():
    errs, t = _sampled_rows("crowded-512x-L5", lambda: synth.crowded(), 128, 4)
    for prec in (0, 1):
        assert errs[prec][0] <= 1e-5 and errs[prec][1] <= 1e-5


def test_blobby_full_bibee_and_solve():
    """BIBEE/CFA energy at 1.31M panels vs the dense oracle (B q and C x are
    N x Q sums); the FP32-refined solve reaches 1e-6 and agrees with the
    FP64 solve."""
    B = lib()
    p = synth.blobby(8)
    g = oracle.geometry(p.verts, p.tris)
    want = oracle.bibee_energy(g, p.charge_pos, p.q, EPS_IN, EPS_OUT, "cfa")
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params())
    got32 = B.bibee_energy(t, dev(p.q), 0, 1)
    got64 = B.bibee_energy(t, dev(p.q), 0, 0)
    print(f"[full-bibee] want={want:.8f} fp32={got32:.8f} fp64={got64:.8f}", flush=True)
    assert abs(got64 - want) <= 1e-5 * abs(want)
    assert abs(got32 - want) <= 1e-4 * abs(want)
    x64, i64 = B.solve_bem(t, dev(p.q), tol=1e-6, precision=0)
    x32, i32 = B.solve_bem(t, dev(p.q), tol=1e-6, precision=2)
    e64 = B.solvation_energy(t, dev(p.q), x64)
    e32 = B.solvation_energy(t, dev(p.q), x32)
    print(f"[full-solve] fp64 {e64:.8f} ({i64.iters} it) refined {e32:.8f} ({i32.iters} it, {i32.outer_iters} outer)",
          flush=True)
    assert i64.converged and i32.converged
    assert abs(e32 - e64) <= 1e-5 * abs(e64)
    # sampled rows of the final residual with the dense oracle operator
    rows = np.sort(np.random.default_rng(9).choice(p.n_panels, size=64, replace=False))
    rhs = F * oracle.field_B(g, p.charge_pos, p.q)
    r = oracle.apply_A(g, F, host(x32), rows=rows) - rhs[rows]
    assert np.linalg.norm(r) <= 1e-5 * np.linalg.norm(rhs[rows])


def test_differentiation_fd_20_components():
    """dG/dq and dG/dr at the level-7 differentiation workload vs central
    differences (h = 1e-4 e and 1e-4 A) on 20 seeded components, on a frozen
    tree with FP64 solves to 1e-11."""
    B = lib()
    p = synth.differentiation(7)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params())
    q = p.q.copy()
    pos = p.charge_pos.copy()

    def energy(qv, pv):
        B.set_charges(t, dev(pv))
        x, _ = B.solve_bem(t, dev(qv), tol=1e-11, maxit=400, precision=0)
        return B.solvation_energy(t, dev(qv), x)

    B.set_charges(t, dev(pos))
    x, _ = B.solve_bem(t, dev(q), tol=1e-11, maxit=400, precision=0)
    dq, dpos, _ = B.adjoint_grad(t, dev(q), x, tol=1e-11, maxit=400, precision=0)
    dq, dpos = host(dq), host(dpos)
    rng = np.random.default_rng(50)
    comps = rng.choice(p.n_charges * 4, size=20, replace=False)
    h = 1e-4
    worst_q = worst_r = 0.0
    for c in comps:
        k, d = divmod(int(c), 4)
        if d == 3:
            qp = q.copy(); qp[k] += h
            qm = q.copy(); qm[k] -= h
            fd = (energy(qp, pos) - energy(qm, pos)) / (2 * h)
            err = abs(dq[k] - fd) / max(abs(fd), 1e-3)
            worst_q = max(worst_q, err)
        else:
            pp = pos.copy(); pp[k, d] += h
            pm = pos.copy(); pm[k, d] -= h
            fd = (energy(q, pp) - energy(q, pm)) / (2 * h)
            err = abs(dpos[k, d] - fd) / max(abs(fd), 1e-2)
            worst_r = max(worst_r, err)
    B.set_charges(t, dev(pos))
    print(f"[fd] worst rel err dq={worst_q:.2e} dpos={worst_r:.2e}", flush=True)
    assert worst_q <= 1e-4 and worst_r <= 1e-2


def test_rotation_translation_invariance():
    """The discrete BEM energy does not depend on where the molecule sits or
    how it is turned; the FMM tree does, so the energies agree to about the
    FMM error."""
    B = lib()
    p = synth.blobby(5)
    rots = synth.random_rotations(3, 77)
    energies = []
    for k in range(4):
        if k == 0:
            V, P = p.verts, p.charge_pos
        else:
            shift = np.array([3.1, -7.7, 12.5]) * k
            V = p.verts @ rots[k - 1].T + shift
            P = p.charge_pos @ rots[k - 1].T + shift
        t = B.build_tree(V, p.tris, P, B.Params())
        x, _ = B.solve_bem(t, dev(p.q), tol=1e-9, precision=0)
        energies.append(B.solvation_energy(t, dev(p.q), x))
    e = np.array(energies)
    print(f"[invariance] {e}", flush=True)
    assert np.abs(e - e[0]).max() <= 1e-6 * abs(e[0])


def test_linearity():
    B = lib()
    p = synth.blobby(5)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params())
    rng = np.random.default_rng(4)
    x1, x2 = rng.normal(size=p.n_panels), rng.normal(size=p.n_panels)
    for prec, tol in ((0, 1e-13), (1, 1e-6)):
        y1 = host(B.fmm_matvec(t, 0, prec, dev(x1)))
        y2 = host(B.fmm_matvec(t, 0, prec, dev(x2)))
        y3 = host(B.fmm_matvec(t, 0, prec, dev(2.0 * x1 - 3.0 * x2)))
        assert rel_l2(y3, 2.0 * y1 - 3.0 * y2) <= tol
