"""bemfmm_set_charges_noalloc against bemfmm_set_charges.

Two trees are built identically; one moves its charges with the allocating
entry point, the other with the allocation-free one (staging in the
library's fixed device array).  Every charge product of the two trees must
then be bitwise equal, in both precisions, and match the dense oracle at the
moved positions to the matvec bar (1e-5 relative L2).  Two calls in a row,
the second on a tree with fewer charges, after a rejected call that leaves
the shared error word set; a tree with more charges than the array holds is
refused with EINVAL and left unchanged."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import dev, host, leaf_boxes, lib, rel_l2, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

OPS = ("B", "BT", "C", "CT")


def _moved(tree, pos, seed):
    """Each charge to a random point of its leaf box, a fifth of them to
    just outside one face (by 0.5/1000 of the leaf side)."""
    lo, hi, sL = leaf_boxes(tree, pos)
    rng = np.random.default_rng(seed)
    m = lo + rng.uniform(0.05, 0.95, size=pos.shape) * sL
    k = np.nonzero(rng.uniform(size=len(pos)) < 0.2)[0]
    axis = rng.integers(3, size=len(k))
    up = rng.integers(2, size=len(k)) == 1
    m[k, axis] = np.where(up, hi[k, axis] + 0.5e-3 * sL, lo[k, axis] - 0.5e-3 * sL)
    return m


def _products(B, t, ins):
    ops = {"B": B.OP_B, "BT": B.OP_BT, "C": B.OP_C, "CT": B.OP_CT}
    return {(name, prec): host(B.fmm_matvec(t, ops[name], prec, dev(ins[name])))
            for name in OPS for prec in (B.FP64, B.FP32)}


def _check_pair(B, p, seed):
    g = oracle.geometry(p.verts, p.tris)
    ta = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params())
    tb = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params())
    moved = _moved(ta, p.charge_pos, seed)
    pos_dev = dev(moved)
    B.set_charges(ta, pos_dev)
    B.set_charges_noalloc(tb, pos_dev)
    rng = np.random.default_rng(seed + 1)
    qv, y = rng.normal(size=p.n_charges), rng.normal(size=p.n_panels)
    ins = {"B": qv, "BT": y, "C": y, "CT": qv}
    ra, rb = _products(B, ta, ins), _products(B, tb, ins)
    want = {"B": oracle.field_B(g, moved, qv), "BT": oracle.apply_BT(g, moved, y),
            "C": oracle.apply_C(g, moved, y), "CT": oracle.apply_CT(g, moved, qv)}
    for (name, prec), a in ra.items():
        e = rel_l2(rb[(name, prec)], want[name])
        print(f"[noalloc] Q={p.n_charges} op={name} prec={prec} err={e:.2e}", flush=True)
        np.testing.assert_array_equal(rb[(name, prec)], a)
        assert e <= 1e-5
    return ta, tb, moved


def test_noalloc_matches_set_charges_twice():
    B = lib()
    big = synth.differentiation(4)            # 5,120 panels, 2,000 charges
    ta, tb, moved = _check_pair(B, big, 21)
    # a rejected call: one charge far outside its leaf; the error word in the
    # shared array is left set and the tree keeps the positions it had
    lo, hi, sL = leaf_boxes(tb, big.charge_pos)
    bad = moved.copy()
    bad[3, 1] = hi[3, 1] + 0.2 * sL
    x = np.random.default_rng(5).normal(size=big.n_panels)
    before = host(B.fmm_matvec(tb, B.OP_C, B.FP64, dev(x)))
    with pytest.raises(B.BemfmmError) as ei:
        B.set_charges_noalloc(tb, dev(bad))
    assert ei.value.code == 1
    np.testing.assert_array_equal(host(B.fmm_matvec(tb, B.OP_C, B.FP64, dev(x))), before)
    B.tree_destroy(ta)
    B.tree_destroy(tb)
    # the second call, on a smaller input (fewer charges and panels)
    small = synth.kirkwood(level=3, n_charges=100)
    ta, tb, _ = _check_pair(B, small, 22)
    B.tree_destroy(ta)
    B.tree_destroy(tb)


def test_noalloc_refuses_more_charges_than_its_array():
    B = lib()
    p = synth.born(2)
    n = 699_041                                # one more than the array holds
    rng = np.random.default_rng(7)
    d = rng.normal(size=(n, 3))
    pos = d / np.linalg.norm(d, axis=1, keepdims=True) * (1.5 * rng.uniform(size=(n, 1)) ** (1 / 3))
    t = B.build_tree(p.verts, p.tris, pos, B.Params())
    qv = rng.normal(size=n)
    before = host(B.fmm_matvec(t, B.OP_B, B.FP64, dev(qv)))
    with pytest.raises(B.BemfmmError) as ei:
        B.set_charges_noalloc(t, dev(pos))
    assert ei.value.code == 1
    assert "699040" in str(ei.value)
    np.testing.assert_array_equal(host(B.fmm_matvec(t, B.OP_B, B.FP64, dev(qv))), before)
    B.set_charges(t, dev(pos))                 # the allocating entry point takes it
    np.testing.assert_array_equal(host(B.fmm_matvec(t, B.OP_B, B.FP64, dev(qv))), before)
    B.tree_destroy(t)
