"""GPU tree build vs the oracle's definitions, bit for bit (integer work):
Morton keys, stable order, cells of every level, leaf-level near lists and
M2L pairs of every level (Section 2.3 hierarchy and lists, Section 3.1
Morton order)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import tree as OT

from gpu_common import requires_gpu, lib

pytestmark = [pytest.mark.gpu, requires_gpu]

CASES = [
    ("born-L3", lambda: synth.born(3), 64, 0.5, OT.MAC_THETA),
    ("kirkwood-L4", lambda: synth.kirkwood(4), 16, 0.5, OT.MAC_THETA),
    ("blobby-L4-t07", lambda: synth.blobby(4), 16, 0.7, OT.MAC_THETA),
    ("blobby-L4-adj", lambda: synth.blobby(4), 8, 0.5, OT.MAC_ADJACENT),
    ("crowded-2x2x2-L2", lambda: synth.crowded(n_side=2, level=2, n_charges=50), 16, 0.5, OT.MAC_THETA),
]


@pytest.mark.parametrize("name,make,ncrit,theta,mac", CASES, ids=[c[0] for c in CASES])
def test_tree_matches_oracle(name, make, ncrit, theta, mac):
    B = lib()
    p = make()
    print(f"[tree] {name} N={p.n_panels} Q={p.n_charges}", flush=True)
    g = oracle.geometry(p.verts, p.tris)
    ot = OT.build(g.c, p.charge_pos, ncrit=ncrit, theta=theta, mac=mac, max_pairs_level=20000)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params(p=10, ncrit=ncrit, theta=theta, mac=mac))
    ex = B.tree_export(t)
    inf = ex["info"]
    assert inf["leaf_level"] == ot.L
    np.testing.assert_allclose(inf["lo"], ot.lo, rtol=0, atol=0)
    assert inf["side"] == ot.side
    np.testing.assert_array_equal(ex["panel_perm"], ot.panel_perm)
    np.testing.assert_array_equal(ex["panel_key"].astype(np.int64), ot.panel_key)
    np.testing.assert_array_equal(ex["charge_perm"], ot.charge_perm)
    np.testing.assert_array_equal(ex["charge_key"].astype(np.int64), ot.charge_key)
    lev = ex["cell_level"]
    gidx = {}
    for l in range(ot.L + 1):
        sel = np.nonzero(lev == l)[0]
        np.testing.assert_array_equal(ex["cell_key"][sel].astype(np.int64), ot.cell_key[l])
        rng = ex["cell_range"][sel]
        np.testing.assert_array_equal(rng[:, 0], ot.cell_pb[l])
        np.testing.assert_array_equal(rng[:, 1], ot.cell_pe[l])
        np.testing.assert_array_equal(rng[:, 2], ot.cell_qb[l])
        np.testing.assert_array_equal(rng[:, 3], ot.cell_qe[l])
        gidx[l] = sel
        if l > 0:
            par = ex["cell_parent"][sel] - gidx[l - 1][0]
            np.testing.assert_array_equal(par, ot.cell_parent[l])
    # leaf near lists (CSR, sources increasing)
    L = ot.L
    near = ot.near[L]
    ptr = ex["near_ptr"]
    src = ex["near_idx"]
    tgt = np.repeat(np.arange(ptr.shape[0] - 1), np.diff(ptr))
    np.testing.assert_array_equal(np.stack([tgt, src], axis=1), near)
    # far pairs of every level
    fp = ex["far_pairs"]
    for l in range(1, L + 1):
        sel = fp[:, 0] == l
        np.testing.assert_array_equal(fp[sel][:, 1:], ot.far[l])
    assert inf["n_far_pairs"] == sum(ot.far[l].shape[0] for l in range(1, L + 1))


def test_tree_rejects_bad_input():
    B = lib()
    v = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0.0]])
    with pytest.raises(B.BemfmmError):
        B.build_tree(v, np.array([[0, 1, 2]], np.int32), np.zeros((1, 3)))
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0.0]])
    with pytest.raises(B.BemfmmError):
        B.build_tree(v, np.array([[0, 1, 3]], np.int32), np.zeros((1, 3)))
    with pytest.raises(B.BemfmmError):
        B.build_tree(v, np.array([[0, 1, 2]], np.int32), np.array([[np.nan, 0, 0]]))
    with pytest.raises(B.BemfmmError):
        B.build_tree(v, np.array([[0, 1, 2]], np.int32), np.zeros((1, 3)), B.Params(p=0))
    with pytest.raises(B.BemfmmError):
        B.build_tree(v, np.array([[0, 1, 2]], np.int32), np.zeros((1, 3)), B.Params(theta=0.1))
