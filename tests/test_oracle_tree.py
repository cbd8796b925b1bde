"""Pins of the oracle's tree definitions: hand-worked Morton keys, the MAC
stencils (counted by hand), and the near/far partition property: for every
leaf target, near leaves plus the far cells of all its ancestors' levels
cover every source cell exactly once (Section 2.3: near domain by direct
sum, far domain by expansions)."""
import os

import numpy as np
import pytest

import synth
import oracle
from oracle import tree as T


def test_morton_golden(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "morton_keys.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    rows = np.array(rows, dtype=np.int64)
    np.testing.assert_array_equal(T.interleave(rows[:, :3]), rows[:, 3])
    np.testing.assert_array_equal(T.deinterleave(rows[:, 3], 10), rows[:, :3])


def test_theta_stencil_counts():
    r = np.arange(-7, 8)
    o = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    near = ~T.mac_far(o, 0.5, T.MAC_THETA)
    # |o|^2 <= 12: 1+6+12+8+6+24+24+12+30+24+24+8 = 179 cells; (2,2,2) is a tie -> near
    assert near.sum() == 179
    assert not T.mac_far(np.array([2, 2, 2]), 0.5, T.MAC_THETA)
    assert T.mac_far(np.array([3, 2, 0]), 0.5, T.MAC_THETA)
    # far offsets reachable from near parents: o = 2 O + d - c, O near, c, d in {0,1}^3
    R = np.arange(-3, 4)
    O = np.stack(np.meshgrid(R, R, R, indexing="ij"), axis=-1).reshape(-1, 3)
    O = O[~T.mac_far(O, 0.5, T.MAC_THETA)]
    bits = np.array([[i >> 2 & 1, i >> 1 & 1, i & 1] for i in range(8)])
    offs = set()
    for Ov in O:
        for c in bits:
            for d in bits:
                ov = 2 * Ov + d - c
                if T.mac_far(ov, 0.5, T.MAC_THETA):
                    offs.add(tuple(ov))
    assert len(offs) == 1740
    # adjacency rule: children of the parent's neighbours that are not adjacent
    adj = set()
    O1 = O[np.abs(O).max(axis=1) <= 1]
    for Ov in O1:
        for c in bits:
            for d in bits:
                ov = 2 * Ov + d - c
                if np.abs(ov).max() > 1:
                    adj.add(tuple(ov))
    assert len(adj) == 7 ** 3 - 27 == 316


def _check_partition(tr, src_cells_of_level):
    """Every (leaf target, leaf source) pair is covered exactly once: by a
    near pair at level L or by a far pair of their ancestors at some level."""
    L = tr.L
    C = tr.cell_key[L].shape[0]
    anc = [np.arange(C)]
    for l in range(L, 0, -1):
        anc.append(tr.cell_parent[l][anc[-1]])
    anc = anc[::-1]  # anc[l][leaf] = ancestor at level l
    cover = np.zeros((C, C), dtype=np.int64)
    nr = tr.near[L]
    cover[nr[:, 0], nr[:, 1]] += 1
    for l in range(1, L + 1):
        fp = tr.far[l]
        if fp.shape[0] == 0:
            continue
        hit = np.zeros((tr.cell_key[l].shape[0],) * 2, dtype=np.int64)
        hit[fp[:, 0], fp[:, 1]] = 1
        cover += hit[anc[l][:, None], anc[l][None, :]]
    assert np.all(cover == 1)


@pytest.mark.parametrize("mac,theta", [(T.MAC_THETA, 0.5), (T.MAC_THETA, 0.7), (T.MAC_ADJACENT, 0.5)])
def test_lists_partition(mac, theta):
    p = synth.blobby(4)
    g = oracle.geometry(p.verts, p.tris)
    tr = T.build(g.c, p.charge_pos, ncrit=16, theta=theta, mac=mac)
    assert tr.L >= 3
    _check_partition(tr, None)


def test_tree_invariants():
    p = synth.kirkwood(4)
    g = oracle.geometry(p.verts, p.tris)
    tr = T.build(g.c, p.charge_pos, ncrit=32)
    # the leaf level's mean occupancy is the closest to ncrit (log scale)
    L = tr.L
    occ = [g.N / np.unique(tr.panel_key >> (3 * (10 - l))).shape[0] for l in range(11)]
    dist = [abs(np.log(o / 32)) for o in occ]
    assert dist[L] <= min(dist[L - 1], dist[L + 1]) + 1e-12
    assert occ[L] <= 2 * 32 * 1.0001 or occ[L + 1] < 32 / 4
    # sorted keys; ranges tile the sorted arrays; charges too
    assert np.all(np.diff(tr.panel_key) >= 0)
    for l in range(L + 1):
        pb, pe = tr.cell_pb[l], tr.cell_pe[l]
        assert pb[0] == 0 and pe[-1] == g.N and np.all(pb[1:] == pe[:-1])
        qb, qe = tr.cell_qb[l], tr.cell_qe[l]
        assert qb[0] == 0 and qe[-1] == p.q.shape[0] and np.all(qb[1:] == qe[:-1])
        assert np.all((pe - pb) + (qe - qb) > 0)
    # points lie inside their leaf cells
    s = tr.side / (1 << L)
    ctr = tr.cell_centre(L)
    cell_of = np.repeat(np.arange(ctr.shape[0]), tr.cell_pe[L] - tr.cell_pb[L])
    rel = g.c[tr.panel_perm] - ctr[cell_of]
    assert np.abs(rel).max() <= 0.5 * s * (1 + 1e-12)
    # per-target lists equal the all-pairs lists
    near_t = tr.near[L]
    for t in (0, 5, ctr.shape[0] - 1):
        ns, fs = T.lists_for_targets(tr, L, [t], 0.5, T.MAC_THETA)[0]
        np.testing.assert_array_equal(ns, near_t[near_t[:, 0] == t, 1])
        np.testing.assert_array_equal(fs, tr.far[L][tr.far[L][:, 0] == t, 1])
