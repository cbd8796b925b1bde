"""Octree, Morton keys and interaction lists by their definitions.

TEST INFRASTRUCTURE ONLY.

Section 2.3 builds the spatial hierarchy by recursive 8-way subdivision down
to a leaf level, finds near and far domains of each cell on the tree, and
Section 3.1 orders leaf boxes by Morton index.  This module states those
definitions in plain numpy (with brute-force pair tests), for bit-exact
comparison with the GPU tree build.  The readings below are where the paper
is silent:

* Root cube: lo = componentwise minimum over panel centroids and charge
  positions, ext = largest extent over the three axes (1 if zero),
  side = ext * (1 + 2**-20), so that every point quantises strictly inside.
* Keys: 10 bits per axis, k_d = clamp(floor((x_d - lo_d) * (1024 / side)), 0, 1023),
  interleaved as bit 3b+2 = x bit b, 3b+1 = y bit b, 3b = z bit b (30-bit key).
* Order: points stably sorted by key (ties keep input order).
* Leaf level L: with m_l = N / (number of non-empty panel cells at level l),
  let l* be the smallest level (0..10) with m_l <= ncrit (10 if none); L is
  l* - 1 if m_{l*-1} is closer to ncrit on a log scale (m_{l*-1} m_{l*} <
  ncrit^2, compared exactly as N^2 < ncrit^2 c_{l*-1} c_{l*}), else l*.
  On a surface the occupancy drops about 4x per level, so this keeps the
  mean leaf occupancy within a factor of 2 of ncrit.  Uniform-depth sparse tree:
  cells at level l are the distinct level-l prefixes (key >> 3(10-l)) of
  panels and charges together, in increasing order.
* MAC between two same-level cells with integer offset o (source minus
  target, in cell units): THETA rule -- far iff 3 < theta^2 |o|^2 (box
  half-diagonals R = sqrt(3) s/2, far iff 2R < theta |d|); ADJACENT rule
  (the paper's: interaction list = children of the parent's neighbours that
  are not adjacent) -- far iff max |o_d| > 1.
* Lists: near_0 = {(root, root)}.  For l >= 1, a pair (t, s) whose parents
  are near at level l-1 is near at level l if the MAC rejects it and far
  (an M2L pair) if it accepts it.  P2P pairs are the near pairs at level L.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

LMAX = 10
MAC_THETA = 0
MAC_ADJACENT = 1


def bounding_cube(points: np.ndarray):
    """(lo[3], side) of the root cube."""
    lo = points.min(axis=0)
    hi = points.max(axis=0)
    ext = float((hi - lo).max())
    if ext == 0.0:
        ext = 1.0
    side = ext * (1.0 + 2.0 ** -20)
    return lo.astype(np.float64), side


def quantise(points: np.ndarray, lo: np.ndarray, side: float) -> np.ndarray:
    inv = 1024.0 / side
    k = np.floor((points - lo[None, :]) * inv)
    return np.clip(k, 0, 1023).astype(np.int64)


def interleave(k: np.ndarray) -> np.ndarray:
    """30-bit Morton key from (n,3) integer coordinates, bit by bit."""
    key = np.zeros(k.shape[0], dtype=np.int64)
    for b in range(LMAX):
        key |= ((k[:, 0] >> b) & 1) << (3 * b + 2)
        key |= ((k[:, 1] >> b) & 1) << (3 * b + 1)
        key |= ((k[:, 2] >> b) & 1) << (3 * b)
    return key


def deinterleave(key: np.ndarray, bits: int) -> np.ndarray:
    """(n,3) integer coordinates from keys with ``bits`` bits per axis."""
    key = np.asarray(key, dtype=np.int64)
    k = np.zeros((key.shape[0], 3), dtype=np.int64)
    for b in range(bits):
        k[:, 0] |= ((key >> (3 * b + 2)) & 1) << b
        k[:, 1] |= ((key >> (3 * b + 1)) & 1) << b
        k[:, 2] |= ((key >> (3 * b)) & 1) << b
    return k


def mac_far(o: np.ndarray, theta: float, mac: int) -> np.ndarray:
    o = np.asarray(o, dtype=np.int64)
    if mac == MAC_THETA:
        d2 = (o * o).sum(axis=-1).astype(np.float64)
        return 3.0 < theta * theta * d2
    return np.abs(o).max(axis=-1) > 1


@dataclass
class Tree:
    lo: np.ndarray
    side: float
    L: int
    panel_key: np.ndarray      # sorted 30-bit keys of panels
    panel_perm: np.ndarray     # sorted position -> input index
    charge_key: np.ndarray
    charge_perm: np.ndarray
    cell_key: list = field(default_factory=list)   # per level: prefixes (increasing)
    cell_pb: list = field(default_factory=list)    # panel ranges [pb, pe)
    cell_pe: list = field(default_factory=list)
    cell_qb: list = field(default_factory=list)    # charge ranges [qb, qe)
    cell_qe: list = field(default_factory=list)
    cell_parent: list = field(default_factory=list)
    near: list = field(default_factory=list)       # per level: (n,2) pairs (t, s), target-major
    far: list = field(default_factory=list)        # per level: (n,2) pairs (t, s), target-major

    def cell_coords(self, l):
        return deinterleave(self.cell_key[l], l)

    def cell_centre(self, l):
        s = self.side / (1 << l)
        return self.lo[None, :] + (self.cell_coords(l) + 0.5) * s


def choose_level(panel_key: np.ndarray, ncrit: int) -> int:
    N = int(panel_key.shape[0])
    counts = [int(np.unique(panel_key >> (3 * (LMAX - l))).shape[0]) for l in range(LMAX + 1)]
    for l in range(0, LMAX + 1):
        if N <= ncrit * counts[l]:  # mean occupancy N / c_l <= ncrit
            if l > 0 and N * N < ncrit * ncrit * counts[l - 1] * counts[l]:
                return l - 1
            return l
    return LMAX


def build(centroids: np.ndarray, charge_pos: np.ndarray, ncrit: int = 64, theta: float = 0.5,
          mac: int = MAC_THETA, lists: bool = True, max_pairs_level: int = 6000) -> Tree:
    """The whole tree; ``lists`` computes near/far pairs by brute force over
    all cell pairs of a level (levels with more than ``max_pairs_level``
    cells are skipped and left as None)."""
    pts = np.concatenate([centroids, charge_pos], axis=0)
    lo, side = bounding_cube(pts)
    pk = interleave(quantise(centroids, lo, side))
    qk = interleave(quantise(charge_pos, lo, side)) if charge_pos.shape[0] else np.zeros(0, np.int64)
    pperm = np.argsort(pk, kind="stable")
    qperm = np.argsort(qk, kind="stable")
    pk = pk[pperm]
    qk = qk[qperm]
    L = choose_level(pk, ncrit)
    T = Tree(lo, side, L, pk, pperm, qk, qperm)
    for l in range(L + 1):
        sh = 3 * (LMAX - l)
        keys = np.unique(np.concatenate([pk >> sh, qk >> sh]))
        T.cell_key.append(keys)
        T.cell_pb.append(np.searchsorted(pk >> sh, keys, side="left"))
        T.cell_pe.append(np.searchsorted(pk >> sh, keys, side="right"))
        T.cell_qb.append(np.searchsorted(qk >> sh, keys, side="left"))
        T.cell_qe.append(np.searchsorted(qk >> sh, keys, side="right"))
        if l == 0:
            T.cell_parent.append(np.full(keys.shape[0], -1, dtype=np.int64))
        else:
            T.cell_parent.append(np.searchsorted(T.cell_key[l - 1], keys >> 3))
    if lists:
        _lists(T, theta, mac, max_pairs_level)
    return T


def _lists(T: Tree, theta, mac, max_cells):
    T.near = [np.array([[0, 0]], dtype=np.int64)]
    T.far = [np.zeros((0, 2), dtype=np.int64)]
    for l in range(1, T.L + 1):
        C = T.cell_key[l].shape[0]
        if C > max_cells or T.near[l - 1] is None:
            T.near.append(None)
            T.far.append(None)
            continue
        k = T.cell_coords(l)
        par = T.cell_parent[l]
        pn = T.near[l - 1]
        Cp = T.cell_key[l - 1].shape[0]
        parent_near = np.zeros((Cp, Cp), dtype=bool)
        parent_near[pn[:, 0], pn[:, 1]] = True
        t_idx, s_idx = np.meshgrid(np.arange(C), np.arange(C), indexing="ij")
        t_idx = t_idx.ravel(); s_idx = s_idx.ravel()
        cand = parent_near[par[t_idx], par[s_idx]]
        t_idx = t_idx[cand]; s_idx = s_idx[cand]
        far = mac_far(k[s_idx] - k[t_idx], theta, mac)
        T.near.append(np.stack([t_idx[~far], s_idx[~far]], axis=1))
        T.far.append(np.stack([t_idx[far], s_idx[far]], axis=1))


def lists_for_targets(T: Tree, l: int, targets: np.ndarray, theta, mac):
    """Near and far partners (sorted source indices) of the given level-l
    targets, by the same definition, computed target by target by walking up
    the ancestors (for levels too large for the all-pairs form)."""
    out = []
    for t in np.asarray(targets):
        near_src, far_src = _partners(T, l, int(t), theta, mac)
        out.append((near_src, far_src))
    return out


def _partners(T, l, t, theta, mac):
    # near set of the target's ancestors, top-down, restricted to candidates
    anc = [t]
    for lv in range(l, 0, -1):
        anc.append(int(T.cell_parent[lv][anc[-1]]))
    anc = anc[::-1]  # anc[lv] = ancestor at level lv
    near_prev = np.array([0], dtype=np.int64)
    far = np.zeros(0, dtype=np.int64)
    for lv in range(1, l + 1):
        par = T.cell_parent[lv]
        cand = np.nonzero(np.isin(par, near_prev))[0]
        k = T.cell_coords(lv)
        fm = mac_far(k[cand] - k[anc[lv]][None, :], theta, mac)
        far = cand[fm]
        near_prev = cand[~fm]
    return near_prev, far
