"""Near quadrature (bemfmm_params.near_quad = nu): K' entries of close panel
pairs (|c_i - c_j| < nu rho_j) take the exact integral over the flat source
panel.  Compared with the oracle's near-quadrature operator
(oracle.panel_integrals), which is pinned by quadrature and closed forms:

* the close-pair count equals the oracle's (bit-exact);
* the correction itself (product with near_quad minus product without, on
  the same tree otherwise) equals the oracle's -f * Delta x to FP64 rounding,
  for A and A^T, in both precisions;
* the whole A and A^T products meet the matvec bar (1e-5 relative L2);
* solves and energies (Born, Kirkwood L4) meet the energy bar (1e-5 FP64,
  1e-4 refined) against the oracle's LAPACK solve of the same operator;
* a radius that could reach beyond the near field is refused (EINVAL).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import dev, host, lib, rel_l2, requires_gpu
from oracle import panel_integrals as PI

pytestmark = [pytest.mark.gpu, requires_gpu]

F = 1.0 - 4.0 / 80.0


@pytest.mark.parametrize("name,make,nu", [("born-L3", lambda: synth.born(3), 3.0),
                                          ("blobby-L4", lambda: synth.blobby(4), 2.5),
                                          ("kirkwood-L4", lambda: synth.kirkwood(4), 4.0)])
def test_nearquad_operators(name, make, nu):
    B = lib()
    p = make()
    g = oracle.geometry(p.verts, p.tris)
    corr = PI.kprime_correction(g, p.verts, p.tris, nu)
    t0 = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params(ncrit=32))
    t1 = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params(ncrit=32, near_quad=nu))
    assert t1.info["n_nearquad_pairs"] == len(corr[0]) and t0.info["n_nearquad_pairs"] == 0
    x = np.random.default_rng(9).normal(size=p.n_panels)
    dcorr = {B.OP_A: -F * PI.apply_correction(corr, x, g.N), B.OP_AT: -F * PI.apply_correction(corr, x, g.N, transpose=True)}
    want = {B.OP_A: PI.apply_A_nq(g, F, x, corr), B.OP_AT: PI.apply_AT_nq(g, F, x, corr)}
    for prec in (B.FP64, B.FP32):
        for op in (B.OP_A, B.OP_AT):
            y0 = host(B.fmm_matvec(t0, op, prec, dev(x)))
            y1 = host(B.fmm_matvec(t1, op, prec, dev(x)))
            e_corr = rel_l2(y1 - y0, dcorr[op])
            e_full = rel_l2(y1, want[op])
            print(f"[nearquad] {name} nu={nu} op={op} prec={prec} pairs={len(corr[0])} "
                  f"corr_err={e_corr:.2e} full_err={e_full:.2e}", flush=True)
            assert e_corr <= 1e-12
            assert e_full <= 1e-5
    B.tree_destroy(t0)
    B.tree_destroy(t1)


@pytest.mark.parametrize("name,make,nu,exact", [
    ("born-L3", lambda: synth.born(3), 2.0, lambda p: oracle.closed_forms.born(1.0, 2.0, 4.0, 80.0)),
    ("kirkwood-L4", lambda: synth.kirkwood(4), 2.0,
     lambda p: oracle.closed_forms.sphere_energy(p.charge_pos, p.q, 20.0, 4.0, 80.0))])
def test_nearquad_solve_energy(name, make, nu, exact):
    B = lib()
    p = make()
    g = oracle.geometry(p.verts, p.tris)
    corr = PI.kprime_correction(g, p.verts, p.tris, nu)
    xo = PI.solve_nq(g, p.charge_pos, p.q, 4.0, 80.0, corr)
    dGo = oracle.solvation_energy(g, p.charge_pos, p.q, xo, 4.0)
    x1, _ = oracle.solve(g, p.charge_pos, p.q, 4.0, 80.0, tol=1e-12)
    dG1 = oracle.solvation_energy(g, p.charge_pos, p.q, x1, 4.0)
    ref = exact(p)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params(ncrit=32, near_quad=nu))
    q = dev(p.q)
    for prec, tol in ((B.FP64, 1e-5), (B.FP32_REFINED, 1e-4)):
        xs, info = B.solve_bem(t, q, tol=1e-10, maxit=300, precision=prec)
        dG = B.solvation_energy(t, q, xs, precision=B.FP64)
        print(f"[nearquad-energy] {name} nu={nu} prec={prec} gpu={dG:.8f} oracle={dGo:.8f} "
              f"one-point={dG1:.8f} closed-form={ref:.8f} err_nq={(dGo - ref) / ref:+.4%} "
              f"err_1pt={(dG1 - ref) / ref:+.4%}", flush=True)
        assert abs(dG - dGo) <= tol * abs(dGo)
    B.tree_destroy(t)


def test_nearquad_radius_beyond_near_field_is_refused():
    B = lib()
    p = synth.blobby(4)
    with pytest.raises(B.BemfmmError) as ei:
        B.build_tree(p.verts, p.tris, p.charge_pos, B.Params(ncrit=1, near_quad=16.0))
    assert ei.value.code == 1
    assert "near field" in str(ei.value)
