"""Edge cases of the GPU path against the FP64 dense oracle: no charges, a
single panel, panel counts that fill no tile or chunk evenly, the extreme
expansion orders (p = 1 and the maximum p = 11) and the extreme MAC
parameters (theta = 0.3 and 1.0).  Operators of Section 2.1, fast summation
of Section 2.3."""
import numpy as np
import pytest

import oracle
import synth

from gpu_common import requires_gpu, lib, dev, host, rel_l2, leaf_boxes

pytestmark = [pytest.mark.gpu, requires_gpu]
EPS_IN, EPS_OUT = 4.0, 80.0
F = 1.0 - EPS_IN / EPS_OUT


def _ops_vs_dense(B, verts, tris, cpos, params, precs=(0, 1), seed=3):
    g = oracle.geometry(verts, tris)
    N, Q = tris.shape[0], cpos.shape[0]
    rng = np.random.default_rng(seed)
    x, y, qv = rng.normal(size=N), rng.normal(size=N), rng.normal(size=Q)
    want = {0: oracle.apply_A(g, F, x), 1: oracle.apply_AT(g, F, y)}
    if Q:
        want.update({2: oracle.field_B(g, cpos, qv), 3: oracle.apply_BT(g, cpos, y),
                     4: oracle.apply_C(g, cpos, x), 5: oracle.apply_CT(g, cpos, qv)})
    ins = {0: x, 1: y, 2: qv, 3: y, 4: x, 5: qv}
    t = B.build_tree(verts, tris, cpos, params)
    errs = {}
    for prec in precs:
        for op in want:
            got = host(B.fmm_matvec(t, op, prec, dev(ins[op])))
            errs[(op, prec)] = rel_l2(got, want[op])
    return t, errs


def test_no_charges():
    """Q = 0: panel operators still match; solve, energies and the adjoint
    give zeros."""
    B = lib()
    p = synth.born(3)
    cpos = np.zeros((0, 3))
    t, errs = _ops_vs_dense(B, p.verts, p.tris, cpos, B.Params())
    print(f"[edges] no charges {errs}", flush=True)
    assert max(errs.values()) <= 1e-5
    q = dev(np.zeros(0))
    x, info = B.solve_bem(t, q, tol=1e-6, precision=B.FP64)
    assert np.all(host(x) == 0.0) and info.converged
    assert B.solvation_energy(t, q, x, precision=B.FP64) == 0.0
    assert B.bibee_energy(t, q, kind=B.BIBEE_CFA, precision=B.FP32) == 0.0
    dq, dpos, _ = B.adjoint_grad(t, q, x, tol=1e-6, precision=B.FP64)
    assert host(dq).size == 0 and host(dpos).size == 0


def test_single_panel():
    """One panel: K' has only its zero diagonal, so A = (1 - f/2) I, and the
    charge operators reduce to one direct term."""
    B = lib()
    verts = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.2, 0.9, 0.0]])
    tris = np.array([[0, 1, 2]], np.int32)
    cpos = np.array([[0.3, 0.3, 1.5], [-0.4, 0.2, -0.7]])
    t, errs = _ops_vs_dense(B, verts, tris, cpos, B.Params())
    print(f"[edges] single panel {errs}", flush=True)
    assert max(e for (op, pr), e in errs.items() if pr == 0) <= 1e-14
    assert max(e for (op, pr), e in errs.items() if pr == 1) <= 1e-6
    xv = np.array([2.5])
    for prec in (0, 1):
        got = host(B.fmm_matvec(t, 0, prec, dev(xv)))
        assert got[0] == pytest.approx((1 - F / 2) * 2.5, rel=1e-15)


@pytest.mark.parametrize("keep,ncrit", [(997, 16), (4093, 32), (61, 8)])
def test_ragged_panel_counts(keep, ncrit):
    """A random subset of a mesh: leaves, P2P chunks, M2L tiles and the scan
    blocks all end part-full."""
    B = lib()
    p = synth.blobby(4)
    rng = np.random.default_rng(keep)
    sel = np.sort(rng.choice(p.n_panels, size=keep, replace=False))
    cpos = p.charge_pos[: 1 + keep % 13]
    t, errs = _ops_vs_dense(B, p.verts, p.tris[sel], cpos, B.Params(ncrit=ncrit))
    print(f"[edges] ragged keep={keep} L={t.info['leaf_level']} {errs}", flush=True)
    assert max(errs.values()) <= 1e-5


def test_expansion_orders():
    """p = 1 (monopole only) to the maximum p = 11: every order runs, the FMM
    error falls with p, and p >= 10 meets the 1e-5 matvec bar.  FP32 runs
    every operator at every order too (the kernels for orders other than
    10, and 8 column tiles at p = 11): its error is the FP64 one plus FP32
    rounding."""
    B = lib()
    p = synth.blobby(5)
    errs, errs32 = {}, {}
    for order in (1, 4, 8, 10, 11):
        t, e = _ops_vs_dense(B, p.verts, p.tris, p.charge_pos[:50], B.Params(p=order, ncrit=32))
        errs[order] = e[(0, 0)]
        errs32[order] = {op: (e[(op, 1)], e[(op, 0)]) for op in range(6)}
        B.tree_destroy(t)
    print(f"[edges] orders {errs}", flush=True)
    print(f"[edges] orders fp32 (fp32, fp64) {errs32}", flush=True)
    assert errs[1] > errs[4] > errs[8] > errs[10] >= 0.5 * errs[11]
    assert errs[10] <= 1e-5 and errs[11] <= 1e-5
    for order, per_op in errs32.items():
        for op, (e32, e64) in per_op.items():
            assert e32 <= e64 + 2e-6, (order, op, e32, e64)


def test_theta_extremes():
    """The smallest and largest accepted theta (0.3: a large near stencil and
    operator table; 1.0: few near leaves, loosely separated far pairs)
    against theta = 0.5: the error grows with theta.  FP32 at each theta:
    the FP64 error plus FP32 rounding."""
    B = lib()
    p = synth.kirkwood(4, n_charges=20)
    errs, noff, gap32 = {}, {}, {}
    for theta in (0.3, 0.5, 1.0):
        t, e = _ops_vs_dense(B, p.verts, p.tris, p.charge_pos, B.Params(theta=theta, ncrit=16))
        errs[theta] = max(v for (op, pr), v in e.items() if pr == 0)
        gap32[theta] = max(e[(op, 1)] - e[(op, 0)] for op in range(6))
        noff[theta] = t.info["n_offsets"]
        B.tree_destroy(t)
    print(f"[edges] theta errors {errs} offsets {noff} fp32 excess {gap32}", flush=True)
    assert errs[0.3] < errs[0.5] < errs[1.0]
    assert errs[0.3] <= 1e-7 and errs[0.5] <= 1e-5 and errs[1.0] <= 5e-2
    assert max(gap32.values()) <= 2e-6


def test_set_charges_limits():
    """bemfmm_set_charges keeps the tree: charges pushed to 0.9/1000 of a
    leaf side beyond their leaf boxes are accepted and every charge operator
    still matches the dense oracle at the moved positions; a charge moved
    0.1 side beyond its box is rejected (EINVAL) and leaves the charges as
    they were."""
    B = lib()
    p = synth.differentiation(4)
    g = oracle.geometry(p.verts, p.tris)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params())
    lo, hi, sL = leaf_boxes(t, p.charge_pos)
    rng = np.random.default_rng(12)
    x = rng.normal(size=p.n_panels)
    before = host(B.fmm_matvec(t, B.OP_C, B.FP64, dev(x)))
    bad = p.charge_pos.copy()
    bad[7, 0] = hi[7, 0] + 0.1 * sL
    with pytest.raises(B.BemfmmError) as ei:
        B.set_charges(t, dev(bad))
    assert ei.value.code == 1
    np.testing.assert_array_equal(host(B.fmm_matvec(t, B.OP_C, B.FP64, dev(x))), before)
    # every charge to just outside one face of its box
    moved = p.charge_pos.copy()
    axis = rng.integers(3, size=p.n_charges)
    side = rng.integers(2, size=p.n_charges)
    k = np.arange(p.n_charges)
    moved[k, axis] = np.where(side == 1, hi[k, axis] + 0.9e-3 * sL, lo[k, axis] - 0.9e-3 * sL)
    B.set_charges(t, dev(moved))
    qv, y = rng.normal(size=p.n_charges), rng.normal(size=p.n_panels)
    want = {B.OP_B: oracle.field_B(g, moved, qv), B.OP_BT: oracle.apply_BT(g, moved, y),
            B.OP_C: oracle.apply_C(g, moved, x), B.OP_CT: oracle.apply_CT(g, moved, qv)}
    ins = {B.OP_B: qv, B.OP_BT: y, B.OP_C: x, B.OP_CT: qv}
    for prec in (0, 1):
        for op, w in want.items():
            e = rel_l2(host(B.fmm_matvec(t, op, prec, dev(ins[op]))), w)
            print(f"[set_charges] op={op} prec={prec} err={e:.2e}", flush=True)
            assert e <= 1e-5
