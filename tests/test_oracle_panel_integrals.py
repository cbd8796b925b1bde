"""Pins of the exact flat-triangle integrals (oracle/panel_integrals.py),
each by something other than the edge/solid-angle formulas themselves:

* an adaptive polar quadrature of S around the foot of the point
  (scipy.integrate.quad of the radial integral in closed form);
* the closed form at the centroid of an equilateral triangle,
  S = sqrt(3) a ln(2 + sqrt(3)) (the same polar integral done by hand);
* Gauss's law for the solid angle on a closed icosahedron with outward
  normals: -4 pi inside (every face is seen from its back), 0 outside,
  -2 pi at the centroid of a face (its own face: the principal value 0);
* central differences of S for grad S;
* the far-field limit: S and grad S tend to those of a point source of
  strength area at the centroid, with an error O((size/d)^2);
* the near-quadrature K' entries against brute-force subdivision quadrature
  of the panel integral.
"""
import numpy as np
import pytest
from scipy import integrate

import oracle
import synth
from oracle import panel_integrals as PI

RNG = np.random.default_rng(1234)


def _random_triangle(rng):
    while True:
        v = rng.normal(size=(3, 3))
        n = np.cross(v[1] - v[0], v[2] - v[0])
        # reasonably shaped: area not tiny against the longest edge squared
        e = max(np.linalg.norm(v[(k + 1) % 3] - v[k]) for k in range(3))
        if np.linalg.norm(n) > 0.3 * e * e:
            return v


def _polar_S(v, r):
    """S by polar integration around the foot of r in the plane of T: each
    edge (a, b) contributes the signed sector from a to b, in which the ray
    of angle phi meets the edge at in-plane distance rho(phi), and the radial
    integral of rho' / sqrt(rho'^2 + h^2) is sqrt(rho^2 + h^2) - |h|."""
    n = np.cross(v[1] - v[0], v[2] - v[0])
    n /= np.linalg.norm(n)
    h = float(np.dot(r - v[0], n))
    foot = r - h * n
    e1 = (v[1] - v[0]) / np.linalg.norm(v[1] - v[0])
    e2 = np.cross(n, e1)
    P = [np.array([np.dot(x - foot, e1), np.dot(x - foot, e2)]) for x in v]
    total = 0.0
    for k in range(3):
        A, Bv = P[k], P[(k + 1) % 3]
        cr = A[0] * Bv[1] - A[1] * Bv[0]
        if abs(cr) < 1e-15:
            continue
        phiA = np.arctan2(A[1], A[0])
        dphi = np.arctan2(cr, np.dot(A, Bv))
        D = Bv - A

        def integrand(t):
            u = np.array([np.cos(phiA + t), np.sin(phiA + t)])
            rho = (A[0] * D[1] - A[1] * D[0]) / (u[0] * D[1] - u[1] * D[0])
            return np.sqrt(rho * rho + h * h) - abs(h)

        val, _ = integrate.quad(integrand, 0.0, dphi, epsabs=1e-14, epsrel=1e-13, limit=200)
        total += val
    return total


@pytest.mark.parametrize("case", range(12))
def test_potential_matches_polar_quadrature(case):
    rng = np.random.default_rng(100 + case)
    v = _random_triangle(rng)
    c = v.mean(axis=0)
    n = np.cross(v[1] - v[0], v[2] - v[0])
    n /= np.linalg.norm(n)
    pts = [c + 0.3 * n, c - 0.05 * n, c + rng.normal(size=3), c + 3.0 * rng.normal(size=3),
           v[0] + 0.2 * (v[1] - v[0]) + 0.1 * (v[2] - v[0]),              # in-plane inside
           v[0] - 0.4 * (v[1] - v[0]) - 0.3 * (v[2] - v[0])]              # in-plane outside
    got = PI.triangle_potential(v, np.array(pts))
    want = np.array([_polar_S(v, p) for p in pts])
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=0)


def test_equilateral_centroid_closed_form():
    for a in (0.5, 1.0, 2.7):
        v = np.array([[0, 0, 0], [a, 0, 0], [a / 2, a * np.sqrt(3) / 2, 0.0]])
        c = v.mean(axis=0)
        assert PI.triangle_potential(v, c[None])[0] == pytest.approx(np.sqrt(3) * a * np.log(2 + np.sqrt(3)),
                                                                      rel=1e-14)


def test_solid_angle_gauss_law_on_icosahedron():
    V, F = synth.icosphere(0)
    V = V * 2.0
    Ws = lambda r: sum(PI.solid_angle(V[f], r[None])[0] for f in F)
    for r in RNG.uniform(-0.8, 0.8, size=(5, 3)):            # inside (inradius of the icosahedron ~1.51)
        assert Ws(r) == pytest.approx(-4 * np.pi, rel=1e-13)
    for r in RNG.normal(size=(5, 3)) * 10 + 10:               # outside
        assert abs(Ws(r)) < 1e-12
    c = V[F[3]].mean(axis=0)                                   # on a face: -2 pi (own face: 0)
    assert PI.solid_angle(V[F[3]], c[None])[0] == 0.0
    assert Ws(c) == pytest.approx(-2 * np.pi, rel=1e-12)
    # just outside that face the own face adds +2 pi: the total jumps to 0
    n = np.cross(V[F[3]][1] - V[F[3]][0], V[F[3]][2] - V[F[3]][0])
    assert abs(Ws(c + 1e-9 * n / np.linalg.norm(n))) < 1e-6


@pytest.mark.parametrize("case", range(6))
def test_gradient_matches_central_differences(case):
    rng = np.random.default_rng(200 + case)
    v = _random_triangle(rng)
    c = v.mean(axis=0)
    pts = c + rng.normal(size=(4, 3)) * np.array([[0.4], [1.0], [2.0], [5.0]])
    g = PI.triangle_grad(v, pts)
    h = 1e-5
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (PI.triangle_potential(v, pts + e) - PI.triangle_potential(v, pts - e)) / (2 * h)
        np.testing.assert_allclose(g[:, k], fd, rtol=1e-6, atol=1e-9)


def test_far_field_tends_to_point_source():
    v = _random_triangle(np.random.default_rng(7))
    c = v.mean(axis=0)
    area = 0.5 * np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))
    d = np.random.default_rng(8).normal(size=3)
    d /= np.linalg.norm(d)
    errs = []
    for dist in (10.0, 20.0, 40.0, 80.0, 160.0):
        r = c + dist * d
        S = PI.triangle_potential(v, r[None])[0]
        G = PI.triangle_grad(v, r[None])[0]
        S0 = area / dist
        G0 = -area * (r - c) / dist ** 3
        errs.append((abs(S - S0) / S0, np.linalg.norm(G - G0) / np.linalg.norm(G0)))
    errs = np.array(errs)
    # the dipole moment about the centroid vanishes: the error falls as
    # (size/d)^2, a factor 4 per doubling of d once the next order has died out
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios > 3.5) and np.all(ratios < 5.5)
    assert np.all(np.abs(ratios[-1] - 4.0) < 0.35)


def _brute_panel_grad(v, r, k=8):
    """grad of the integral over T of 1/|r - r'| by the centroid rule on 4^k
    congruent sub-triangles."""
    n = 2 ** k
    area = 0.5 * np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))
    e1, e2 = (v[1] - v[0]) / n, (v[2] - v[0]) / n
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = i + j < n
    base = v[0] + i[keep][:, None] * e1 + j[keep][:, None] * e2
    up = base + (e1 + e2) / 3.0
    keep2 = (i + j < n - 1)
    base2 = v[0] + i[keep2][:, None] * e1 + j[keep2][:, None] * e2
    down = base2 + 2.0 * (e1 + e2) / 3.0
    pts = np.concatenate([up, down])
    d = r - pts
    R = np.linalg.norm(d, axis=1)
    return -(area / len(pts)) * np.sum(d / R[:, None] ** 3, axis=0)


def test_near_quadrature_kprime_against_subdivision():
    p = synth.born(2)                       # 320 panels, R = 2
    g = oracle.geometry(p.verts, p.tris)
    rows, cols, delta = PI.kprime_correction(g, p.verts, p.tris, 3.0)
    assert len(rows) > 0 and np.all(rows != cols)
    V = p.verts[p.tris]
    pick = np.random.default_rng(3).choice(len(rows), size=25, replace=False)
    for k in pick:
        i, j = rows[k], cols[k]
        exact = np.dot(g.n[i], _brute_panel_grad(V[j], g.c[i])) / (4 * np.pi)
        d = g.c[i] - g.c[j]
        point = -g.a[j] * np.dot(g.n[i], d) / (4 * np.pi * np.linalg.norm(d) ** 3)
        assert delta[k] == pytest.approx(exact - point, rel=2e-4, abs=1e-8 * abs(point))


def test_near_quadrature_operator_transpose_and_born():
    """A^T of the near-quadrature operator is the transpose of its A, and
    the Born ion stays within discretisation error of the closed form (the
    exact close-pair integrals move it from +2.0% to about +2.6%)."""
    p = synth.born(3)
    g = oracle.geometry(p.verts, p.tris)
    corr = PI.kprime_correction(g, p.verts, p.tris, 2.0)
    rng = np.random.default_rng(4)
    x, y = rng.normal(size=g.N), rng.normal(size=g.N)
    f = 0.95
    assert np.dot(y, PI.apply_A_nq(g, f, x, corr)) == pytest.approx(np.dot(x, PI.apply_AT_nq(g, f, y, corr)),
                                                                     rel=1e-12)
    xs = PI.solve_nq(g, p.charge_pos, p.q, 4.0, 80.0, corr)
    dG = oracle.solvation_energy(g, p.charge_pos, p.q, xs, 4.0)
    born = oracle.closed_forms.born(1.0, 2.0, 4.0, 80.0)
    assert 0.01 < (dG - born) / born < 0.04
    # the solve is a solve: residual of the near-quadrature operator
    r = PI.apply_A_nq(g, f, xs, corr) - f * oracle.field_B(g, p.charge_pos, p.q)
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(xs)


@pytest.mark.parametrize("side", ["row", "col"])
def test_near_quadrature_correction_of_given_panels(side):
    """The restricted search (large meshes: only the pairs of some target or
    source panels) finds exactly the entries of the full correction list in
    those rows or columns, with the same values."""
    p = synth.born(3)
    g = oracle.geometry(p.verts, p.tris)
    rows, cols, delta = PI.kprime_correction(g, p.verts, p.tris, 3.0)
    panels = np.sort(np.random.default_rng(5).choice(g.N, size=60, replace=False))
    r2, c2, d2 = PI.kprime_correction_of(g, p.verts, p.tris, 3.0, panels, side=side)
    keep = np.isin(rows if side == "row" else cols, panels)
    assert keep.sum() > 60
    np.testing.assert_array_equal(r2, rows[keep])
    np.testing.assert_array_equal(c2, cols[keep])
    np.testing.assert_array_equal(d2, delta[keep])
