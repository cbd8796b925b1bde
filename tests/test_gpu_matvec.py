"""GPU FMM products vs the FP64 dense oracle (Section 2.1 operators, Section
2.3 fast summation), element by element, plus stage-level checks of the
expansions against their definitions."""
import numpy as np
import pytest

import oracle
import synth
from oracle import harmonics as H
from oracle import tree as OT

from gpu_common import requires_gpu, lib, dev, host, rel_l2

pytestmark = [pytest.mark.gpu, requires_gpu]
EPS_IN, EPS_OUT = 4.0, 80.0
F = 1.0 - EPS_IN / EPS_OUT


def dense_ops(p, g, x, qv, y):
    """Oracle results of the six operators."""
    return {
        0: oracle.apply_A(g, F, x),
        1: oracle.apply_AT(g, F, y),
        2: oracle.field_B(g, p.charge_pos, qv),
        3: oracle.apply_BT(g, p.charge_pos, y),
        4: oracle.apply_C(g, p.charge_pos, x),
        5: oracle.apply_CT(g, p.charge_pos, qv),
    }


def _inputs(p, seed=7):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=p.n_panels)
    y = rng.normal(size=p.n_panels)
    qv = rng.normal(size=p.n_charges)
    return x, y, qv


def _run_all(B, t, x, y, qv, prec):
    ins = {0: x, 1: y, 2: qv, 3: y, 4: x, 5: qv}
    return {op: host(B.fmm_matvec(t, op, prec, dev(ins[op]))) for op in range(6)}


@pytest.mark.parametrize("prec,tol_direct", [(0, 1e-12), (1, 2e-6)])
def test_direct_limit_matches_dense(prec, tol_direct):
    """A tree with one level (ncrit huge) has no far field: the FMM is the
    direct sum, so FP64 must equal the dense oracle to rounding."""
    B = lib()
    p = synth.kirkwood(3, n_charges=30)
    g = oracle.geometry(p.verts, p.tris)
    x, y, qv = _inputs(p)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params(ncrit=100000))
    assert t.info["n_far_pairs"] == 0
    got = _run_all(B, t, x, y, qv, prec)
    want = dense_ops(p, g, x, qv, y)
    for op in range(6):
        print(f"[direct] prec={prec} op={op} err={rel_l2(got[op], want[op]):.3e}", flush=True)
        assert rel_l2(got[op], want[op]) <= tol_direct, op


CASES = [
    ("born-L3", lambda: synth.born(3), 32),
    ("kirkwood-L4-20q", lambda: synth.kirkwood(4, n_charges=20), 32),
    ("blobby-L5", lambda: synth.blobby(5), 32),
]


@pytest.mark.parametrize("name,make,ncrit", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", [0, 1])
def test_fmm_operators_match_dense(name, make, ncrit, prec):
    """Every operator at p = 10, theta = 0.5: relative L2 error <= 1e-5."""
    B = lib()
    p = make()
    g = oracle.geometry(p.verts, p.tris)
    x, y, qv = _inputs(p)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params(ncrit=ncrit))
    print(f"[fmm] {name} prec={prec} L={t.info['leaf_level']} far={t.info['n_far_pairs']}", flush=True)
    got = _run_all(B, t, x, y, qv, prec)
    want = dense_ops(p, g, x, qv, y)
    for op in range(6):
        e = rel_l2(got[op], want[op])
        print(f"    op={op} rel_l2={e:.3e}", flush=True)
        assert e <= 1e-5, (op, e)


def test_fmm_deterministic():
    B = lib()
    p = synth.blobby(4)
    x, _, _ = _inputs(p)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params(ncrit=16))
    a = host(B.fmm_matvec(t, 0, 1, dev(x)))
    b = host(B.fmm_matvec(t, 0, 1, dev(x)))
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("order", [10, 8])
@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 2e-6)])
def test_expansions_match_definitions(prec, tol, order):
    """Multipole expansions of every cell (P2M at the leaves, M2M above)
    equal the definition M_n^m = sum w conj(R_n^m(y - X)) applied directly
    to the cell's sources (M2M is exact), element by element.  p = 10 runs
    the P2M compiled for that order, p = 8 the generic one."""
    B = lib()
    p = synth.blobby(4)
    g = oracle.geometry(p.verts, p.tris)
    rng = np.random.default_rng(3)
    x = rng.normal(size=p.n_panels)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params(ncrit=16, p=order))
    B.fmm_matvec(t, 0, prec, dev(x))
    Mg = B.debug_expansions(t, prec, 0)
    ex = B.tree_export(t)
    lo, side = np.array(ex["info"]["lo"]), ex["info"]["side"]
    lev = ex["cell_level"]
    w = g.a * x
    perm = ex["panel_perm"]
    L = ex["info"]["leaf_level"]
    checked = 0
    for l in range(2, L + 1):
        sel = np.nonzero(lev == l)[0]
        s = side / (1 << l)
        for c in sel[:: max(1, len(sel) // 12)]:
            k = OT.deinterleave(np.array([ex["cell_key"][c]], dtype=np.int64), l)[0]
            X = lo + (k + 0.5) * s
            b, e = ex["cell_range"][c][:2]
            if e == b:
                continue
            idx = perm[b:e]
            want = H.p2m(g.c[idx], w[idx], X, s, order)
            scale = np.abs(want).max()
            err = np.abs(Mg[c] - want).max() / scale
            assert err <= tol, (l, c, err)
            checked += 1
    assert checked > 10


@pytest.mark.parametrize("prec", [0, 1])
def test_near_and_far_fields(prec):
    """P2P near field equals the direct sum over the near leaves (to
    rounding); the L2P far field equals the exact sum over all other sources
    to within the truncation error."""
    B = lib()
    p = synth.blobby(4)
    g = oracle.geometry(p.verts, p.tris)
    rng = np.random.default_rng(11)
    x = rng.normal(size=p.n_panels)
    t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params(ncrit=16))
    B.fmm_matvec(t, 0, prec, dev(x))
    with pytest.raises(B.BemfmmError):  # not recorded
        B.debug_fields(t, prec, p.n_panels)
    B.debug_record(t, True)
    y_rec = host(B.fmm_matvec(t, 0, prec, dev(x)))
    near, far = B.debug_fields(t, prec, p.n_panels)
    B.debug_record(t, False)
    # recording changes nothing in the product itself
    np.testing.assert_array_equal(y_rec, host(B.fmm_matvec(t, 0, prec, dev(x))))
    ex = B.tree_export(t)
    perm = ex["panel_perm"]
    L = ex["info"]["leaf_level"]
    lev = ex["cell_level"]
    leaf_rng = ex["cell_range"][lev == L]
    ptr, idx = ex["near_ptr"], ex["near_idx"]
    leaf_of = np.zeros(p.n_panels, dtype=np.int64)
    for li, (b, e, _, _) in enumerate(leaf_rng):
        leaf_of[perm[b:e]] = li
    w = g.a * x
    Kall = oracle.apply_Kp(g, x)
    tgts = rng.choice(p.n_panels, size=40, replace=False)
    for i in tgts:
        li = leaf_of[i]
        srcs = np.concatenate([perm[leaf_rng[s][0]:leaf_rng[s][1]] for s in idx[ptr[li]:ptr[li + 1]]])
        srcs = srcs[srcs != i]
        d = g.c[i] - g.c[srcs]
        r = np.linalg.norm(d, axis=1)
        want_near = -np.sum(w[srcs] * (d @ g.n[i]) / r ** 3) / (4 * np.pi)
        want_far = Kall[i] - want_near
        tol_n = 1e-12 if prec == 0 else 2e-6
        assert abs(near[i] - want_near) <= tol_n * np.abs(Kall).max(), i
        assert abs(far[i] - want_far) <= 1e-6 * np.abs(Kall).max(), i


def test_rebuild_after_destroy_reuses_memory_bitwise():
    """Device blocks of a destroyed tree are reused by the next builds (a
    smaller tree in between, then the same one); results must be bitwise
    those of the first build, also after the cache has been emptied."""
    B = lib()
    big, small = synth.blobby(5), synth.kirkwood(3, n_charges=30)
    x = _inputs(big)[0]
    xs = _inputs(small)[0]
    gs = oracle.geometry(small.verts, small.tris)
    outs = []
    for stage in ("first", "after-small", "after-release"):
        t = B.build_tree(big.verts, big.tris, big.charge_pos, B.Params())
        outs.append([host(B.fmm_matvec(t, 0, prec, dev(x))) for prec in (0, 1)])
        B.tree_destroy(t)
        ts = B.build_tree(small.verts, small.tris, small.charge_pos, B.Params(ncrit=16))
        e = rel_l2(host(B.fmm_matvec(ts, 0, 0, dev(xs))), oracle.apply_A(gs, F, xs))
        print(f"[rebuild] {stage} small-tree err={e:.3e}", flush=True)
        assert e <= 1e-5
        B.tree_destroy(ts)
        if stage == "after-small":
            B.release_cache()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


def test_switches_do_not_change_results(monkeypatch):
    """The near field run concurrently (forked at any point of the upward
    pass, or after M2L) or after the multipole passes gives bitwise the same
    products (the switches change scheduling, not arithmetic).  The FP32 M2L
    on FP32 MFMA gives bitwise the same products with persistent or one-tile
    workgroups; the split-bf16 M2L (the default for A and A^T at p = 10)
    differs from it by FP32 rounding only; the products from or to charges
    and the FP64 products do not use it."""
    B = lib()
    p = synth.blobby(5)
    x, y, qv = _inputs(p)
    outs = {}
    cases = {"base": ("1", "1", "-1", "1"), "in_line": ("0", "1", "-1", "1"),
             "fork0": ("1", "1", "0", "1"), "fork1": ("1", "1", "1", "1"), "fork2": ("1", "1", "2", "1"),
             "fork3": ("1", "1", "3", "1"), "fp32_mfma": ("1", "1", "-1", "0"), "per_tile": ("1", "0", "-1", "1")}
    for name, (conc, pers, fork, split) in cases.items():
        monkeypatch.setenv("BEMFMM_CONCURRENT_P2P", conc)
        monkeypatch.setenv("BEMFMM_M2L_PERSISTENT", pers)
        monkeypatch.setenv("BEMFMM_FORK_AT", fork)
        monkeypatch.setenv("BEMFMM_M2L_SPLIT", split)
        t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params())
        outs[name] = {prec: _run_all(B, t, x, y, qv, prec) for prec in (0, 1)}
        B.tree_destroy(t)
    ref = outs["base"]
    for name in ("in_line", "fork0", "fork1", "fork2", "fork3"):
        for prec in (0, 1):
            for op in range(6):
                assert np.array_equal(outs[name][prec][op], ref[prec][op]), (name, prec, op)
    for prec in (0, 1):
        for op in range(6):
            assert np.array_equal(outs["per_tile"][prec][op], outs["fp32_mfma"][prec][op]), (prec, op)
            if prec == 0 or op >= 2:
                assert np.array_equal(outs["fp32_mfma"][prec][op], ref[prec][op]), (prec, op)
            else:
                d = rel_l2(ref[prec][op], outs["fp32_mfma"][prec][op])
                print(f"  op {op}: split-bf16 vs FP32 MFMA M2L, rel L2 {d:.2e}", flush=True)
                assert d <= 1e-6, (op, d)


def test_persistent_m2l_matches_per_tile_at_full_size(monkeypatch):
    """At the bench surface (1.31M panels) the M2L is large enough to run
    persistent in both precisions (and the near field forks after M2M); the
    one-tile-per-workgroup kernels give bitwise the same products as the
    persistent ones on FP32 MFMA, and the split-bf16 M2L agrees with them to
    FP32 rounding."""
    B = lib()
    p = synth.blobby(8)
    x = np.random.default_rng(9).normal(size=p.n_panels)
    outs = {}
    for pers, split in (("1", "0"), ("0", "0"), ("1", "1")):
        monkeypatch.setenv("BEMFMM_M2L_PERSISTENT", pers)
        monkeypatch.setenv("BEMFMM_M2L_SPLIT", split)
        t = B.build_tree(p.verts, p.tris, p.charge_pos, B.Params())
        assert t.info["n_m2l_panel_pairs"] > 32 * 256 * 256
        outs[pers + split] = [host(B.fmm_matvec(t, op, prec, dev(x))) for op in (0, 1) for prec in (0, 1)]
        B.tree_destroy(t)
    for a, b in zip(outs["10"], outs["00"]):
        assert np.array_equal(a, b)
    for k, (a, b) in enumerate(zip(outs["11"], outs["10"])):
        if k % 2 == 0:  # FP64
            assert np.array_equal(a, b)
        else:
            d = rel_l2(a, b)
            print(f"  split-bf16 vs FP32 MFMA M2L, op {k // 2}: rel L2 {d:.2e}", flush=True)
            assert d <= 1e-6
