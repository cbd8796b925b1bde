"""Parity at the benchmark's full sizes, in the launch configuration that
bench.py times (p = 10, theta = 0.5, ncrit = 64): sampled outputs that the
oracle computes one by one, energies where the dense oracle is affordable,
finite differences on the differentiation workload, and invariances."""
import numpy as np
import pytest

import oracle
import synth
from oracle import lpb as OL
from oracle import panel_integrals as PI

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


def _sub(g, rows):
    return oracle.Geometry(g.c[rows], g.n[rows], g.a[rows])


def test_crowded_full_sampled_rows():
    """Crowded system (512 molecules, 10,485,760 panels, 512,000 charges):
    all six operators on sampled rows (panel rows through a sub-geometry of
    the sampled targets, charge rows through the sampled charges); then the
    plain FP64 and the FP32-refined solves to 1e-6 agree in energy and the
    refined solution's residual holds on sampled dense rows.  The dense
    energy itself is out of reach here (parity partly unpinned, bounded by
    the sampled rows)."""
    errs, t = _sampled_rows("crowded-512x-L5", lambda: synth.crowded(), 128, 4)
    for prec in (0, 1):
        assert errs[prec][0] <= 1e-5 and errs[prec][1] <= 1e-5
    B = lib()
    p = synth.crowded()
    g = oracle.geometry(p.verts, p.tris)
    rng = np.random.default_rng(41)
    prow = np.sort(rng.choice(p.n_panels, size=96, replace=False))
    qrow = np.sort(rng.choice(p.n_charges, size=96, replace=False))
    x, qv = rng.normal(size=p.n_panels), rng.normal(size=p.n_charges)
    sub = _sub(g, prow)
    want = {B.OP_B: oracle.field_B(sub, p.charge_pos, qv), B.OP_CT: oracle.apply_CT(sub, p.charge_pos, qv),
            B.OP_C: oracle.apply_C(g, p.charge_pos[qrow], x), B.OP_BT: oracle.apply_BT(g, p.charge_pos[qrow], x)}
    ins = {B.OP_B: qv, B.OP_CT: qv, B.OP_C: x, B.OP_BT: x}
    rows = {B.OP_B: prow, B.OP_CT: prow, B.OP_C: qrow, B.OP_BT: qrow}
    for prec in (1, 0):
        for op, w in want.items():
            got = host(B.fmm_matvec(t, op, prec, dev(ins[op])))[rows[op]]
            e = rel_l2(got, w)
            print(f"    crowded op={op} prec={prec} err={e:.2e}", flush=True)
            assert e <= 1e-5
    x64, i64 = B.solve_bem(t, dev(p.q), tol=1e-6, maxit=300, precision=0)
    x32, i32 = B.solve_bem(t, dev(p.q), tol=1e-6, maxit=300, precision=2)
    e64 = B.solvation_energy(t, dev(p.q), x64)
    e32 = B.solvation_energy(t, dev(p.q), x32)
    print(f"[crowded-solve] fp64 {e64:.8f} ({i64.iters} it, {i64.seconds:.3f} s) refined {e32:.8f} "
          f"({i32.iters} it, {i32.outer_iters} outer, {i32.seconds:.3f} s)", flush=True)
    assert i64.converged and i32.converged
    assert abs(e32 - e64) <= 1e-5 * abs(e64)
    rhs = F * oracle.field_B(sub, p.charge_pos, p.q)
    r = oracle.apply_A(g, F, host(x32), rows=prow) - rhs
    assert np.linalg.norm(r) <= 1e-5 * np.linalg.norm(rhs)


def test_blobby_full_bibee_and_solve():
    """BIBEE energies at 1.31M panels (CFA, P and the +1/2 scale factor) vs
    the dense oracle (B q and C x are N x Q sums); the FP32-refined solve
    reaches 1e-6 and agrees with the FP64 solve."""
    B = lib()
    p = synth.blobby(8)
    g = oracle.geometry(p.verts, p.tris)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params())
    for kind, name in ((B.BIBEE_CFA, "cfa"), (B.BIBEE_P, "p"), (B.BIBEE_PLUS_HALF, "plus_half")):
        want = oracle.bibee_energy(g, p.charge_pos, p.q, EPS_IN, EPS_OUT, name)
        got32 = B.bibee_energy(t, dev(p.q), kind, 1)
        got64 = B.bibee_energy(t, dev(p.q), kind, 0)
        print(f"[full-bibee] {name} want={want:.8f} fp32={got32:.8f} fp64={got64:.8f}", flush=True)
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
    """dG/dq and dG/dr at the level-7 differentiation workload (327,680
    panels, 2000 charges) vs central differences (h = 1e-4 e and 1e-4 A) on
    20 seeded components, on a frozen tree, for the FP64 and the
    FP32-refined gradients.  The differences use FP64 solves to 1e-12.

    Error budget of a difference, relative to the largest gradient entry:
    dG is quadratic in q, so the charge differences are exact but for the
    solve (a residual tau moves dG by about tau |dG|, giving tau |dG| / h =
    5e-6 absolute against entries of order 100-1000); the position
    differences add h^2 |d3 dG| / 6, about (h / d)^2 = 1e-8 relative for a
    charge d >= 1 A from the nearest panel; the adjoint's FMM operators differ
    from the transposes of the forward's by the FMM error (about 1e-8).  The
    refined gradient adds its solves' tolerance (1e-9).  Bound: 1e-6 for
    both, against the gradient's largest entry of each kind."""
    B = lib()
    p = synth.differentiation(7)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params())
    q = p.q.copy()
    pos = p.charge_pos.copy()

    def energy(qv, pv):
        B.set_charges(t, dev(pv))
        x, _ = B.solve_bem(t, dev(qv), tol=1e-12, maxit=400, precision=0)
        return B.solvation_energy(t, dev(qv), x)

    B.set_charges(t, dev(pos))
    grads = {}
    for prec, tol in ((0, 1e-11), (2, 1e-9)):
        x, _ = B.solve_bem(t, dev(q), tol=tol, maxit=400, precision=prec)
        dq, dpos, _ = B.adjoint_grad(t, dev(q), x, tol=tol, maxit=400, precision=prec)
        grads[prec] = (host(dq), host(dpos))
    rng = np.random.default_rng(50)
    comps = rng.choice(p.n_charges * 4, size=20, replace=False)
    h = 1e-4
    worst = {0: [0.0, 0.0], 2: [0.0, 0.0]}
    for c in comps:
        k, d = divmod(int(c), 4)
        if d == 3:
            qp = q.copy(); qp[k] += h
            qm = q.copy(); qm[k] -= h
            fd = (energy(qp, pos) - energy(qm, pos)) / (2 * h)
            for prec, (dq, _) in grads.items():
                worst[prec][0] = max(worst[prec][0], abs(dq[k] - fd) / np.abs(dq).max())
        else:
            pp = pos.copy(); pp[k, d] += h
            pm = pos.copy(); pm[k, d] -= h
            fd = (energy(q, pp) - energy(q, pm)) / (2 * h)
            for prec, (_, dpos) in grads.items():
                worst[prec][1] = max(worst[prec][1], abs(dpos[k, d] - fd) / np.abs(dpos).max())
    B.set_charges(t, dev(pos))
    print(f"[fd] worst err vs max |grad|: fp64 dq={worst[0][0]:.2e} dpos={worst[0][1]:.2e}; "
          f"refined dq={worst[2][0]:.2e} dpos={worst[2][1]:.2e}", flush=True)
    for prec in (0, 2):
        assert worst[prec][0] <= 1e-6 and worst[prec][1] <= 1e-6


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


def test_blobby_full_nearquad_sampled_rows():
    """Near quadrature (nu = 2) on the surface the bench's extension rows
    time it on (blobby L8, 1.31M panels, about 15M close pairs): sampled
    rows of A and A^T against the dense oracle's rows plus the
    exact-minus-one-point corrections of those rows and columns, found by
    the oracle's own radius search."""
    B = lib()
    p = synth.blobby(8)
    g = oracle.geometry(p.verts, p.tris)
    nu = 2.0
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params(near_quad=nu))
    assert t.info["n_nearquad_pairs"] > 10 * p.n_panels
    rng = np.random.default_rng(6)
    x = rng.normal(size=p.n_panels)
    rows = np.sort(rng.choice(p.n_panels, size=128, replace=False))
    corr = PI.kprime_correction_of(g, p.verts, p.tris, nu, rows, side="row")
    corrT = PI.kprime_correction_of(g, p.verts, p.tris, nu, rows, side="col")
    want = oracle.apply_A(g, F, x, rows=rows) - F * PI.apply_correction(corr, x, g.N)[rows]
    wantT = oracle.apply_AT(g, F, x, rows=rows) - F * PI.apply_correction(corrT, x, g.N, transpose=True)[rows]
    for prec in (0, 1):
        e = rel_l2(host(B.fmm_matvec(t, 0, prec, dev(x)))[rows], want)
        eT = rel_l2(host(B.fmm_matvec(t, 1, prec, dev(x)))[rows], wantT)
        print(f"[full-nq] blobby-L8 nu={nu} prec={prec} close pairs of the rows {len(corr[0])} / {len(corrT[0])} "
              f"A err={e:.2e} A^T err={eT:.2e}", flush=True)
        assert e <= 1e-5 and eT <= 1e-5
    B.tree_destroy(t)


def test_blobby_full_lpb_sampled_rows():
    """The screened (linearised Poisson-Boltzmann) product on the surface
    the bench's extension rows time it on (blobby L8, 2,621,440 unknowns,
    kappa = 0.125/A): sampled rows of both halves against the dense
    oracle's rows (its self integrals taken for every panel)."""
    B = lib()
    p = synth.blobby(8)
    g = oracle.geometry(p.verts, p.tris)
    kappa = 0.125
    S = OL.LPB(g, p.verts, p.tris, p.eps_in, p.eps_out, kappa)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params())
    N = p.n_panels
    z = np.random.default_rng(7).normal(size=2 * N)
    y = host(B.lpb_matvec(t, kappa, dev(z)))
    rows = np.sort(np.random.default_rng(8).choice(N, size=48, replace=False))
    wu, wv = [], []
    for i in rows:
        Muu, Muv, Mvu, Mvv = S.rows(i, i + 1)
        wu.append(Muu[0] @ z[:N] + Muv[0] @ z[N:])
        wv.append(Mvu[0] @ z[:N] + Mvv[0] @ z[N:])
    eu, ev = rel_l2(y[rows], np.array(wu)), rel_l2(y[N + rows], np.array(wv))
    print(f"[full-lpb] blobby-L8 kappa={kappa} err_u={eu:.2e} err_v={ev:.2e}", flush=True)
    assert eu <= 1e-5 and ev <= 1e-5
    B.tree_destroy(t)
