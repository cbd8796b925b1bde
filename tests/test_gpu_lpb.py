"""Linearised Poisson-Boltzmann (screened solvent) on the GPU against the
dense oracle (oracle/lpb.py, pinned by the screened Born ion, Kirkwood's
screened series and the Poisson limit):

* a tree whose leaves are all near each other (no far field): the near
  field of both kernels, the exact self terms and the diagonal, to FP64
  rounding;
* full operators (Laplace and screened far fields by FMM, p = 10) on three
  surfaces and two screening lengths: the matvec bar, 1e-5 relative L2, on
  each half (u rows and v rows);
* solves and energies (Born ion, Kirkwood sphere L4, blobby L4) against the
  oracle's LAPACK solve of the same discrete system: 1e-5;
* arguments out of range are refused (EINVAL).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import dev, host, lib, rel_l2, requires_gpu
from oracle import lpb as OL

pytestmark = [pytest.mark.gpu, requires_gpu]


def _oracle(p, kappa):
    g = oracle.geometry(p.verts, p.tris)
    return OL.LPB(g, p.verts, p.tris, p.eps_in, p.eps_out, kappa)


@pytest.mark.parametrize("kappa", [0.4, 6.0])
def test_lpb_all_near_tree_matches_oracle(kappa):
    """One leaf, so the product is the near field, the self terms and the
    diagonal alone.  kappa r spans about [0.12, 1.6] at 0.4 and [1.8, 24]
    at 6 (e^{-kappa r} then runs down to 2^-34, through every entry of the
    exponential's table); rounding-level agreement either way."""
    B = lib()
    p = synth.born(2)                                   # 320 panels
    S = _oracle(p, kappa)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params(ncrit=4096))
    assert t.info["n_far_pairs"] == 0
    z = np.random.default_rng(3).normal(size=2 * p.n_panels)
    y = host(B.lpb_matvec(t, kappa, dev(z)))
    want = S.apply(z)
    e = rel_l2(y, want)
    print(f"[lpb] all-near kappa={kappa} err={e:.2e}", flush=True)
    assert e <= 1e-12
    B.tree_destroy(t)


@pytest.mark.parametrize("name,make,kappa", [("born-L3", lambda: synth.born(3), 0.1),
                                             ("kirkwood-L4", lambda: synth.kirkwood(4), 0.125),
                                             ("blobby-L4", lambda: synth.blobby(4), 0.5)])
def test_lpb_operator_matches_oracle(name, make, kappa):
    B = lib()
    p = make()
    S = _oracle(p, kappa)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params(ncrit=32))
    N = p.n_panels
    z = np.random.default_rng(4).normal(size=2 * N)
    y = host(B.lpb_matvec(t, kappa, dev(z)))
    want = S.apply(z)
    eu, ev = rel_l2(y[:N], want[:N]), rel_l2(y[N:], want[N:])
    print(f"[lpb] {name} kappa={kappa} leaf_level={t.info['leaf_level']} far_pairs={t.info['n_far_pairs']} "
          f"err_u={eu:.2e} err_v={ev:.2e}", flush=True)
    assert eu <= 1e-5 and ev <= 1e-5
    # deterministic: the same product twice is bitwise the same
    np.testing.assert_array_equal(host(B.lpb_matvec(t, kappa, dev(z))), y)
    B.tree_destroy(t)


@pytest.mark.parametrize("name,make,kappa", [("born-L3", lambda: synth.born(3), 0.1),
                                             ("kirkwood-L4", lambda: synth.kirkwood(4), 0.125),
                                             ("blobby-L4", lambda: synth.blobby(4), 0.3)])
def test_lpb_solve_energy_matches_oracle(name, make, kappa):
    B = lib()
    p = make()
    S = _oracle(p, kappa)
    uvo = S.solve(p.charge_pos, p.q)
    dGo = S.energy(p.charge_pos, p.q, uvo)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params(ncrit=32))
    q = dev(p.q)
    uv, info = B.lpb_solve(t, q, kappa, tol=1e-10, maxit=400, restart=60)
    dG = B.lpb_energy(t, q, uv)
    e_uv = rel_l2(host(uv), uvo)
    print(f"[lpb-energy] {name} kappa={kappa} gpu={dG:.8f} oracle={dGo:.8f} rel={abs(dG - dGo) / abs(dGo):.2e} "
          f"uv_err={e_uv:.2e} iters={info.iters} resid={info.rel_residual:.1e}", flush=True)
    assert info.converged and info.rel_residual <= 1e-10
    assert abs(dG - dGo) <= 1e-5 * abs(dGo)
    assert e_uv <= 1e-5
    B.tree_destroy(t)


def test_lpb_rejects_bad_arguments():
    B = lib()
    p = synth.born(2)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params())
    z = dev(np.zeros(2 * p.n_panels))
    for kappa in (0.0, -1.0, float("nan"), 1e4):
        with pytest.raises(B.BemfmmError) as ei:
            B.lpb_matvec(t, kappa, z)
        assert ei.value.code == 1
    B.tree_destroy(t)
