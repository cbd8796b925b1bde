"""Pins of the FP64 dense oracle against closed forms, invariants, library
solves and brute force (CPU only).

Born ion and Kirkwood sphere: closed-form solutions of the Section 2.1
model; BIBEE sphere series: eq. CFA applied analytically; CFA upper bound:
Section 2.2; Gauss law for the induced charge; GMRES against a LAPACK solve
of the explicitly assembled A; the adjoint against central finite
differences."""
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import closed_forms as cf

EPS_IN, EPS_OUT = 4.0, 80.0
F = 1.0 - EPS_IN / EPS_OUT


def _load_golden(golden_dir, name):
    rows = []
    with open(os.path.join(golden_dir, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return np.array(rows)


def test_triangle_geometry_golden(golden_dir):
    rows = _load_golden(golden_dir, "triangle_geometry.txt")
    for r in rows:
        verts = r[:9].reshape(3, 3)
        g = oracle.geometry(verts, np.array([[0, 1, 2]], dtype=np.int32))
        np.testing.assert_allclose(g.c[0], r[9:12], rtol=0, atol=1e-15)
        np.testing.assert_allclose(g.n[0], r[12:15], rtol=0, atol=1e-15)
        assert g.a[0] == pytest.approx(r[15], rel=1e-15)


def test_geometry_rejects_bad_mesh():
    v = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0.0]])
    with pytest.raises(ValueError):
        oracle.geometry(v, np.array([[0, 1, 2]], dtype=np.int32))   # zero area
    with pytest.raises(ValueError):
        oracle.geometry(v, np.array([[0, 1, 3]], dtype=np.int32))   # index out of range


def test_icosphere_outward_and_area():
    for L in (1, 2, 3):
        v, t = synth.icosphere(L)
        g = oracle.geometry(v, t)
        assert np.all(np.einsum("ij,ij->i", g.n, g.c) > 0)
    # total area converges to 4 pi from below
    areas = [oracle.geometry(*synth.icosphere(L)).a.sum() for L in (2, 3, 4)]
    errs = [4 * np.pi - a for a in areas]
    assert all(e > 0 for e in errs) and errs[0] > 3.5 * errs[1] > 3.5 * 3.5 * errs[2] * 0.9


@pytest.mark.parametrize("L,bound", [(2, 0.06), (3, 0.025), (4, 0.01)])
def test_born_converges(L, bound):
    p = synth.born(L)
    g = oracle.geometry(p.verts, p.tris)
    x, info = oracle.solve(g, p.charge_pos, p.q, EPS_IN, EPS_OUT, tol=1e-11)
    assert info.converged
    dG = oracle.solvation_energy(g, p.charge_pos, p.q, x, EPS_IN)
    ex = cf.born(1.0, 2.0, EPS_IN, EPS_OUT)
    assert ex == pytest.approx(-19.7160625, rel=1e-12)
    assert 0 < (dG - ex) / ex < bound


def test_born_error_decreases_first_order():
    ex = cf.born(1.0, 2.0, EPS_IN, EPS_OUT)
    errs = []
    for L in (2, 3, 4):
        p = synth.born(L)
        g = oracle.geometry(p.verts, p.tris)
        x, _ = oracle.solve(g, p.charge_pos, p.q, EPS_IN, EPS_OUT, tol=1e-11)
        errs.append(abs(oracle.solvation_energy(g, p.charge_pos, p.q, x, EPS_IN) - ex))
    assert errs[0] / errs[1] > 2.0 and errs[1] / errs[2] > 2.0


def test_gauss_law_induced_charge():
    """Total induced charge -> -f sum q (exact in the continuum)."""
    vals = []
    for L in (2, 3, 4):
        p = synth.born(L)
        g = oracle.geometry(p.verts, p.tris)
        x, _ = oracle.solve(g, p.charge_pos, p.q, EPS_IN, EPS_OUT, tol=1e-11)
        vals.append(float((g.a * x).sum()))
    errs = [abs(v + F) for v in vals]
    assert errs[2] < errs[1] < errs[0] and errs[2] < 0.01


def test_cfa_exact_for_born_and_bounds():
    ex = cf.born(1.0, 2.0, EPS_IN, EPS_OUT)
    errs = []
    for L in (2, 3, 4):
        p = synth.born(L)
        g = oracle.geometry(p.verts, p.tris)
        errs.append(abs(oracle.bibee_energy(g, p.charge_pos, p.q, EPS_IN, EPS_OUT, "cfa") - ex) / abs(ex))
    # O(h^2): about 4x per level
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0
    # the continuum CFA for a centred charge equals Born exactly
    assert cf.sphere_energy(np.zeros((1, 3)), [1.0], 2.0, EPS_IN, EPS_OUT, "cfa") == pytest.approx(ex, rel=1e-14)


def test_kirkwood_series_and_bibee_bounds():
    errs, errs_cfa = [], []
    for L in (2, 3, 4):
        p = synth.kirkwood(L, n_charges=20)
        g = oracle.geometry(p.verts, p.tris)
        x, _ = oracle.solve(g, p.charge_pos, p.q, EPS_IN, EPS_OUT, tol=1e-11)
        dG = oracle.solvation_energy(g, p.charge_pos, p.q, x, EPS_IN)
        ex = cf.sphere_energy(p.charge_pos, p.q, 20.0, EPS_IN, EPS_OUT, "exact")
        cfa = oracle.bibee_energy(g, p.charge_pos, p.q, EPS_IN, EPS_OUT, "cfa")
        pp = oracle.bibee_energy(g, p.charge_pos, p.q, EPS_IN, EPS_OUT, "p")
        exc = cf.sphere_energy(p.charge_pos, p.q, 20.0, EPS_IN, EPS_OUT, "cfa")
        exp_ = cf.sphere_energy(p.charge_pos, p.q, 20.0, EPS_IN, EPS_OUT, "p")
        errs.append(abs(dG - ex) / abs(ex))
        errs_cfa.append(abs(cfa - exc) / abs(exc))
        # BIBEE/P <= BEM <= BIBEE/CFA (Section 2.2: CFA is an upper bound)
        assert pp <= dG <= cfa
        assert exp_ <= ex <= exc
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.03
    assert errs_cfa[0] > errs_cfa[1] > errs_cfa[2] and errs_cfa[2] < 0.01


@pytest.mark.parametrize("kind", ["cfa", "p", "plus_half"])
def test_bibee_variants_sphere_series(kind):
    """Each BIBEE variant of Section 2.2 (the principal-value operator
    replaced by -1/2, 0 or +1/2 times the identity) against its own sphere
    series: the discrete energy converges at O(h^2), about 4x per level.  A
    wrong scale (say 1 - f in place of 1 - f/2) is off by a factor of ten."""
    errs = []
    for L in (2, 3, 4):
        p = synth.kirkwood(L, n_charges=20)
        g = oracle.geometry(p.verts, p.tris)
        got = oracle.bibee_energy(g, p.charge_pos, p.q, EPS_IN, EPS_OUT, kind)
        want = cf.sphere_energy(p.charge_pos, p.q, 20.0, EPS_IN, EPS_OUT, kind)
        errs.append(abs(got - want) / abs(want))
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0
    assert errs[2] < 0.01


def test_bibee_series_ordering_and_born():
    """Continuum series: the n = 0 term of the CFA series is the Born term
    (CFA exact for a centred charge), and the variants order as
    plus_half <= P <= exact <= CFA for charges inside a sphere."""
    p = synth.kirkwood(3, n_charges=20)
    e = {k: cf.sphere_energy(p.charge_pos, p.q, 20.0, EPS_IN, EPS_OUT, k) for k in ("cfa", "p", "plus_half", "exact")}
    assert e["plus_half"] <= e["p"] <= e["exact"] <= e["cfa"]
    born = cf.born(1.0, 2.0, EPS_IN, EPS_OUT)
    assert cf.sphere_energy(np.zeros((1, 3)), [1.0], 2.0, EPS_IN, EPS_OUT, "exact") == pytest.approx(born, rel=1e-14)


def test_binding_composition_on_one_sphere():
    """Binding (Section 4.4): with protein, inhibitor and complex sharing one
    spherical surface (charges A, B and A + B), dG_bind is the cross term of
    the reaction-field series, K q_A^T M q_B, for the full BEM and for every
    BIBEE variant; the discrete result converges to it with the mesh."""
    rng = np.random.default_rng(7)
    for kind, key in (("bem", "exact"), ("cfa", "cfa"), ("p", "p")):
        errs = []
        for L in (3, 4):
            p = synth.kirkwood(L, n_charges=12)
            a, b = p.charge_pos[:6], p.charge_pos[6:]
            qa, qb = p.q[:6], p.q[6:] + rng.uniform(-0.1, 0.1, 6)
            mol = lambda pos, q: (p.verts, p.tris, pos, q)  # noqa: E731
            bind, c, pe, ie = oracle.binding_energy(mol(np.vstack([a, b]), np.concatenate([qa, qb])), mol(a, qa),
                                                    mol(b, qb), EPS_IN, EPS_OUT, method=kind)
            assert bind == pytest.approx(c - pe - ie, rel=1e-12, abs=1e-12)
            both = cf.sphere_energy(np.vstack([a, b]), np.concatenate([qa, qb]), 20.0, EPS_IN, EPS_OUT, key)
            want = both - cf.sphere_energy(a, qa, 20.0, EPS_IN, EPS_OUT, key) - \
                cf.sphere_energy(b, qb, 20.0, EPS_IN, EPS_OUT, key)
            errs.append(abs(bind - want) / abs(want))
        assert errs[1] < errs[0] and errs[1] < 0.05, (kind, errs)


def test_gmres_matches_lapack():
    p = synth.kirkwood(3, n_charges=20)
    g = oracle.geometry(p.verts, p.tris)
    A = oracle.assemble_A(g, F)
    b = F * oracle.field_B(g, p.charge_pos, p.q)
    xs = np.linalg.solve(A, b)
    for restart in (0, 3):
        x, info = oracle.gmres(g, F, b, tol=1e-13, restart=restart, maxit=200)
        assert info.converged
        assert np.abs(x - xs).max() <= 1e-10 * np.abs(xs).max()
    # transpose solve
    y, info = oracle.gmres(g, F, b, tol=1e-13, transpose=True)
    np.testing.assert_allclose(y, np.linalg.solve(A.T, b), rtol=0, atol=1e-10 * np.abs(y).max())


def test_operator_transposes():
    """<A x, y> = <x, A^T y>, <C x, q> = <x, C^T q>, <B q, y> = <q, B^T y>."""
    rng = np.random.default_rng(5)
    p = synth.blobby(3)
    g = oracle.geometry(p.verts, p.tris)
    x = rng.normal(size=g.N); y = rng.normal(size=g.N); q = p.q
    Am = oracle.assemble_A(g, F)
    np.testing.assert_allclose(oracle.apply_A(g, F, x), Am @ x, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(oracle.apply_AT(g, F, y), Am.T @ y, rtol=1e-12, atol=1e-12)
    lhs = oracle.apply_C(g, p.charge_pos, x) @ q
    rhs = x @ oracle.apply_CT(g, p.charge_pos, q)
    assert lhs == pytest.approx(rhs, rel=1e-12)
    lhs = oracle.field_B(g, p.charge_pos, q) @ y
    rhs = q @ oracle.apply_BT(g, p.charge_pos, y)
    assert lhs == pytest.approx(rhs, rel=1e-12)
    rows = np.array([0, 7, g.N - 1])
    np.testing.assert_allclose(oracle.apply_A(g, F, x, rows=rows), (Am @ x)[rows], rtol=1e-13)


def _energy(g, pos, q):
    x, info = oracle.solve(g, pos, q, EPS_IN, EPS_OUT, tol=1e-13, maxit=300)
    return oracle.solvation_energy(g, pos, q, x, EPS_IN), x


def test_adjoint_vs_finite_differences():
    p = synth.blobby(2)
    g = oracle.geometry(p.verts, p.tris)
    q = p.q[:12].copy(); pos = p.charge_pos[:12].copy()
    dG, x = _energy(g, pos, q)
    dq, dpos, y, info = oracle.adjoint_grad(g, pos, q, x, EPS_IN, EPS_OUT, tol=1e-13)
    assert info.converged
    h = 1e-4
    for i in (0, 5, 11):
        qp = q.copy(); qp[i] += h; qm = q.copy(); qm[i] -= h
        fd = (_energy(g, pos, qp)[0] - _energy(g, pos, qm)[0]) / (2 * h)
        assert dq[i] == pytest.approx(fd, rel=1e-7, abs=1e-9)
        for d in (0, 2):
            pp = pos.copy(); pp[i, d] += h; pm = pos.copy(); pm[i, d] -= h
            fd = (_energy(g, pp, q)[0] - _energy(g, pm, q)[0]) / (2 * h)
            assert dpos[i, d] == pytest.approx(fd, rel=1e-5, abs=1e-7)


def test_adjoint_vs_explicit_inverse():
    p = synth.blobby(2)
    g = oracle.geometry(p.verts, p.tris)
    A = oracle.assemble_A(g, F)
    Q = p.q.shape[0]
    B = np.stack([oracle.field_B(g, p.charge_pos[k:k + 1], [1.0]) for k in range(40)], axis=1)
    C = np.stack([oracle.apply_C(g, p.charge_pos[:40], np.eye(g.N)[j]) for j in range(g.N)], axis=1)
    q = p.q[:40]
    M = oracle.kappa(EPS_IN) * C @ np.linalg.solve(A, F * B)
    x, _ = oracle.solve(g, p.charge_pos[:40], q, EPS_IN, EPS_OUT, tol=1e-13)
    dq, _, _, _ = oracle.adjoint_grad(g, p.charge_pos[:40], q, x, EPS_IN, EPS_OUT, tol=1e-13)
    np.testing.assert_allclose(dq, (M + M.T) @ q, rtol=1e-9, atol=1e-9 * np.abs(dq).max())
    assert Q >= 40


def test_born_gradient_closed_form():
    """Born: d dG/dq = 2 dG / q; centred charge feels no force (mesh symmetry)."""
    p = synth.born(3)
    g = oracle.geometry(p.verts, p.tris)
    dG, x = _energy(g, p.charge_pos, p.q)
    dq, dpos, _, _ = oracle.adjoint_grad(g, p.charge_pos, p.q, x, EPS_IN, EPS_OUT, tol=1e-13)
    assert dq[0] == pytest.approx(2 * dG, rel=1e-10)
    assert np.abs(dpos).max() < 1e-9
