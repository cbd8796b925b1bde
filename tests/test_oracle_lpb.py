"""Pins of the linearised Poisson-Boltzmann oracle (oracle/lpb.py):

* kappa = 0: the formulation reduces to the Poisson model, and its energy
  equals the (separately pinned) Poisson oracle's on the same mesh;
* the screened Born ion closed form, approached at first order under
  refinement of the sphere (L2 -> L4), for two screening lengths;
* Kirkwood's screened sphere series for off-centre charges, approached
  under refinement;
* the screened series itself: its recurrence for k_n'/k_n against
  scipy.special.spherical_kn, its kappa = 0 and n = 0 special cases;
* the two self integrals against an adaptive quadrature of the polar
  integral, and their small-kappa limits (a_i kappa / 4 pi and
  kappa^2 / 8 pi times the exact flat-triangle potential at the centroid);
* the dense solve solves the assembled system, and apply() is its product.
"""
import numpy as np
import pytest
from scipy import integrate
from scipy.special import spherical_kn

import oracle
import synth
from oracle import closed_forms as cf
from oracle import lpb
from oracle import panel_integrals as PI


def _energy(p, kappa):
    g = oracle.geometry(p.verts, p.tris)
    S = lpb.LPB(g, p.verts, p.tris, p.eps_in, p.eps_out, kappa)
    uv = S.solve(p.charge_pos, p.q)
    return S.energy(p.charge_pos, p.q, uv)


@pytest.mark.parametrize("make", [lambda: synth.born(3), lambda: synth.kirkwood(3)])
def test_zero_screening_is_the_poisson_model(make):
    p = make()
    g = oracle.geometry(p.verts, p.tris)
    x, _ = oracle.solve(g, p.charge_pos, p.q, p.eps_in, p.eps_out, tol=1e-13, maxit=2000)
    want = oracle.solvation_energy(g, p.charge_pos, p.q, x, p.eps_in)
    assert _energy(p, 0.0) == pytest.approx(want, rel=1e-10)


@pytest.mark.parametrize("kappa", [0.1, 0.5])
def test_screened_born_converges(kappa):
    exact = cf.born_screened(1.0, 2.0, 4.0, 80.0, kappa)
    errs = [abs(_energy(synth.born(L), kappa) - exact) / abs(exact) for L in (2, 3, 4)]
    assert errs[0] > errs[1] > errs[2]
    assert 2.0 < errs[0] / errs[1] < 3.5 and 2.0 < errs[1] / errs[2] < 3.5
    assert errs[2] < 0.01


def test_screened_kirkwood_converges():
    kappa = 0.125
    p3, p2 = synth.kirkwood(3), synth.kirkwood(2)
    exact = cf.sphere_energy_lpb(p3.charge_pos, p3.q, 20.0, 4.0, 80.0, kappa)
    unscreened = cf.sphere_energy(p3.charge_pos, p3.q, 20.0, 4.0, 80.0)
    e2 = abs(_energy(p2, kappa) - exact) / abs(exact)
    e3 = abs(_energy(p3, kappa) - exact) / abs(exact)
    assert e3 < e2 / 3 and e3 < 0.08
    # the salt effect is resolved: the screened energy differs from the
    # unscreened one by more than the discretisation error at L3
    assert abs(exact - unscreened) / abs(exact) > 0.02


def test_screened_series_special_cases():
    x = 2.5
    n = np.arange(25)
    ref = x * spherical_kn(n, x, derivative=True) / spherical_kn(n, x)
    np.testing.assert_allclose(cf._lpb_lambda(24, x), ref, rtol=1e-13, atol=1e-13)
    pos = np.array([[3.0, 1.0, 2.0], [-5.0, 2.0, 1.0], [0.5, -7.0, 4.0]])
    q = np.array([1.0, -1.0, 0.5])
    assert cf.sphere_energy_lpb(pos, q, 20.0, 4.0, 80.0, 0.0) == pytest.approx(
        cf.sphere_energy(pos, q, 20.0, 4.0, 80.0), rel=1e-14)
    assert cf.sphere_energy_lpb(pos, q, 20.0, 4.0, 80.0, 1e-9) == pytest.approx(
        cf.sphere_energy(pos, q, 20.0, 4.0, 80.0), rel=1e-7)
    for k in (0.05, 0.3):
        assert cf.sphere_energy_lpb(np.zeros((1, 3)), [1.0], 2.0, 4.0, 80.0, k) == pytest.approx(
            cf.born_screened(1.0, 2.0, 4.0, 80.0, k), rel=1e-14)


def test_self_integrals():
    p = synth.born(2)
    g = oracle.geometry(p.verts, p.tris)
    V = p.verts[p.tris]
    kappa = 0.7
    Vs, Ds = lpb.self_integrals(p.verts, p.tris, g.c, kappa)
    # adaptive quadrature of the polar integral of h and of -h'/R (r dr dtheta)
    h = lambda s: -np.expm1(-kappa * s) / (4 * np.pi * s)
    hp_over = lambda s: (kappa * s * np.exp(-kappa * s) + np.expm1(-kappa * s)) / (4 * np.pi * s ** 3)  # h'/s
    for i in (0, 17, 101):
        c = g.c[i]
        tot_v = tot_d = 0.0
        for e in range(3):
            a, b = V[i][e], V[i][(e + 1) % 3]
            t = (b - a) / np.linalg.norm(b - a)
            foot = a + np.dot(c - a, t) * t
            P = np.linalg.norm(c - foot)
            ta, tb = np.arctan2(np.dot(a - foot, t), P), np.arctan2(np.dot(b - foot, t), P)
            fv = lambda th: integrate.quad(lambda s: h(s) * s, 0, P / np.cos(th), epsabs=0, epsrel=1e-13)[0]
            fd = lambda th: integrate.quad(lambda s: -hp_over(s) * s, 0, P / np.cos(th), epsabs=0,
                                           epsrel=1e-13)[0]
            tot_v += integrate.quad(fv, ta, tb, epsabs=0, epsrel=1e-12)[0]
            tot_d += integrate.quad(fd, ta, tb, epsabs=0, epsrel=1e-12)[0]
        assert Vs[i] == pytest.approx(tot_v, rel=1e-10)
        assert Ds[i] == pytest.approx(tot_d, rel=1e-8)
    # small-kappa limits, approached linearly in kappa
    S = np.array([PI.triangle_potential(V[i], g.c[i][None])[0] for i in range(len(V))])
    dev = []
    for k in (1e-3, 1e-5):
        Vk, Dk = lpb.self_integrals(p.verts, p.tris, g.c, k)
        dev.append((np.max(np.abs(Vk / k / (g.a / (4 * np.pi)) - 1)), np.max(np.abs(Dk / k ** 2 / (S / (8 * np.pi)) - 1))))
    dev = np.array(dev)
    assert np.all(dev[1] < 2e-6)
    np.testing.assert_allclose(dev[0] / dev[1], 100.0, rtol=0.01)


def test_solve_and_apply_are_consistent():
    p = synth.born(2)
    g = oracle.geometry(p.verts, p.tris)
    S = lpb.LPB(g, p.verts, p.tris, 4.0, 80.0, 0.3)
    M = S.assemble()
    uv = S.solve(p.charge_pos, p.q)
    b = S.rhs(p.charge_pos, p.q)
    assert np.linalg.norm(M @ uv - b) <= 1e-12 * np.linalg.norm(b)
    z = np.random.default_rng(2).normal(size=2 * g.N)
    np.testing.assert_allclose(S.apply(z), M @ z, rtol=1e-13, atol=1e-13 * np.linalg.norm(M @ z))
