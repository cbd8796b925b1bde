"""Binding energy (Section 4.4, eq. binding-free-energy-estimate) through
bemfmm_binding_energy: two molecules as the "complex" (two closed surfaces,
all charges), each alone as the parts; compared with the dense oracle's
three energies for the full BEM and every BIBEE variant, and the
interaction term vanishing as the molecules separate."""
import numpy as np
import pytest

import oracle
import synth

from gpu_common import requires_gpu, lib

pytestmark = [pytest.mark.gpu, requires_gpu]


def _pair(d):
    a = synth.blobby(3)
    b = synth.kirkwood(3, R=8.0, n_charges=10, r_max=6.0)
    shift = np.array([d, 0.0, 0.0])
    V = np.concatenate([a.verts, b.verts + shift])
    T = np.concatenate([a.tris, b.tris + a.verts.shape[0]]).astype(np.int32)
    P = np.concatenate([a.charge_pos, b.charge_pos + shift])
    Q = np.concatenate([a.q, b.q])
    from paper_1007_4591_amd.binding import Molecule
    return (Molecule(V, T, P, Q), Molecule(a.verts, a.tris, a.charge_pos, a.q),
            Molecule(b.verts + shift, b.tris, b.charge_pos + shift, b.q))


def _dense(m):
    g = oracle.geometry(m.verts, m.tris)
    x, _ = oracle.solve(g, m.charge_pos, m.q, 4.0, 80.0, tol=1e-10)
    return oracle.solvation_energy(g, m.charge_pos, m.q, x, 4.0)


def test_binding_matches_dense():
    from paper_1007_4591_amd.binding import binding_energy
    B = lib()
    c, p, i = _pair(40.0)
    got = binding_energy(c, p, i, method="bem", params=B.Params(ncrit=16), tol=1e-9, precision=0)
    want = {k: _dense(m) for k, m in (("complex", c), ("protein", p), ("inhibitor", i))}
    want["binding"] = want["complex"] - want["protein"] - want["inhibitor"]
    print(f"[binding] got={got} want={want}", flush=True)
    for k in ("complex", "protein", "inhibitor"):
        assert abs(got[k] - want[k]) <= 1e-5 * abs(want[k])
    assert abs(got["binding"] - want["binding"]) <= 1e-5 * abs(want["complex"])


@pytest.mark.parametrize("method", ["cfa", "p", "plus_half"])
def test_binding_bibee_matches_dense(method):
    from paper_1007_4591_amd.binding import binding_energy
    B = lib()
    c, p, i = _pair(40.0)
    for prec, tol in ((0, 1e-5), (1, 1e-4)):
        got = binding_energy(c, p, i, method=method, params=B.Params(ncrit=16), precision=prec)
        want = oracle.binding_energy(*[(m.verts, m.tris, m.charge_pos, m.q) for m in (c, p, i)], 4.0, 80.0,
                                     method=method)
        print(f"[binding-{method}] prec={prec} got={got} want={want}", flush=True)
        for k, w in zip(("binding", "complex", "protein", "inhibitor"), want):
            assert abs(got[k] - w) <= tol * abs(want[1])


def test_binding_rejects_bad_method():
    B = lib()
    a = synth.born(2)
    t = B.build_tree(a.verts, a.tris, a.charge_pos, B.Params())
    with pytest.raises(B.BemfmmError):
        B.binding_energy(t, a.q, t, a.q, t, a.q, method=4)
    # one tree for all three parts: complex - 2 x itself = -dG
    out = B.binding_energy(t, a.q, t, a.q, t, a.q, method=B.ENERGY_BIBEE_CFA, precision=0)
    assert out["binding"] == pytest.approx(-out["complex"], rel=1e-12)


def test_binding_vanishes_with_separation():
    from paper_1007_4591_amd.binding import binding_energy
    B = lib()
    vals = []
    for d in (35.0, 70.0, 140.0):
        c, p, i = _pair(d)
        vals.append(abs(binding_energy(c, p, i, method="cfa", params=B.Params(ncrit=16))["binding"]))
    assert vals[0] > vals[1] > vals[2]
