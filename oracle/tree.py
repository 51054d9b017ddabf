"""Hierarchical partition of the points (oracle, integer work).  Test infrastructure only.

The paper's first FMM step is a hierarchical tree partition of the domain (section 1,
the list of FMM steps), with groups of points and their neighbour groups (section 4,
eq. 38: G_b and N_a).  The paper does not fix the tree; this module writes out the
definition the library uses, so that the device tree can be compared with it bit for bit:

* Root: the bounding cube of the points.  lo_k = min_i x_ik, ext = max_k (max_i x_ik - lo_k),
  computed in FP64 from the stored values (ext = 1 if all points coincide).
* Quantisation with B = floor(63/d) bits per coordinate:
  q_k = min(floor((x_k - lo_k) * (2^B / ext)), 2^B - 1), in FP64.
* Morton key: bit b of q_k goes to bit b*d + k of a 64-bit key.
* Order: stable sort by key (ties keep input order); perm[i] = input index of sorted point i.
* Boxes at level l are the distinct key prefixes key >> (d (B - l)).  The root exists; a box
  at level l >= 1 exists iff its parent is split; a box is split iff it exists, l < maxlev,
  and (l < min_level or it holds more than n_max points).  Existing, unsplit boxes are leaves.
  Leaves partition the sorted points into consecutive ranges.
* Near list U(a) of a leaf a: every leaf b (any level, a included) whose closed box meets
  the closed box of a.  Computed here by brute force over all leaf pairs.
* Coarse cell of a leaf: its ancestor's Morton index at the coarse level l_c (leaves are
  never coarser than l_c, because min_level = l_c forces the split).

Pinned by: Morton interleave against a bit-by-bit loop, the partition and symmetry of
the near lists, the geometric adjacency brute force itself, and the pair-cover identity
(near + far + pruned = N^2 ordered pairs) in tests/test_oracle_tree.py.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def bits_per_dim(d: int) -> int:
    return 63 // d


def root_cube(points):
    x = np.asarray(points)
    lo = x.min(axis=0).astype(np.float64)
    hi = x.max(axis=0).astype(np.float64)
    ext = float(np.max(hi - lo))
    if not ext > 0.0:
        ext = 1.0
    return lo, ext


def quantize(points, lo, ext, B: int) -> np.ndarray:
    scale = (2.0 ** B) / ext
    t = (np.asarray(points).astype(np.float64) - lo) * scale
    q = np.floor(t).astype(np.int64)
    return np.clip(q, 0, (1 << B) - 1)


def morton(q: np.ndarray, B: int) -> np.ndarray:
    n, d = q.shape
    key = np.zeros(n, dtype=np.uint64)
    for b in range(B):
        for k in range(d):
            bit = ((q[:, k] >> b) & 1).astype(np.uint64)
            key |= bit << np.uint64(b * d + k)
    return key


def deinterleave(prefix: np.ndarray, d: int, nbits: int) -> np.ndarray:
    """Integer coordinates (n, d) of Morton prefixes with nbits bits per coordinate."""
    prefix = np.asarray(prefix, dtype=np.uint64)
    out = np.zeros((prefix.shape[0], d), dtype=np.int64)
    for b in range(nbits):
        for k in range(d):
            out[:, k] |= (((prefix >> np.uint64(b * d + k)) & np.uint64(1)).astype(np.int64)) << b
    return out


@dataclass
class Tree:
    d: int
    B: int
    lo: np.ndarray
    ext: float
    keys: np.ndarray          # sorted Morton keys (uint64)
    perm: np.ndarray          # perm[i] = input index of the i-th sorted point
    leaf_begin: np.ndarray    # (nleaves + 1,)
    leaf_level: np.ndarray    # (nleaves,)
    leaf_prefix: np.ndarray   # (nleaves,) Morton prefix at the leaf's level
    nlevels: int              # number of levels that hold boxes (deepest level + 1)

    @property
    def nleaves(self) -> int:
        return int(self.leaf_level.shape[0])

    def leaf_box(self):
        """Closed boxes of the leaves in finest-level integer units: (lo, hi) each (nleaves, d)."""
        lev = self.leaf_level.astype(np.int64)
        c = np.stack([deinterleave(self.leaf_prefix[i:i + 1], self.d, int(lev[i]))[0]
                      for i in range(self.nleaves)]) if self.nleaves else np.zeros((0, self.d), np.int64)
        size = (np.int64(1) << (self.B - lev))[:, None]
        lo = c * size
        return lo, lo + size

    def coarse_cell(self, lc: int) -> np.ndarray:
        """Morton index at level lc of each leaf's ancestor (requires leaf_level >= lc)."""
        assert np.all(self.leaf_level >= lc)
        sh = (self.d * (self.leaf_level.astype(np.int64) - lc)).astype(np.uint64)
        return (self.leaf_prefix >> sh).astype(np.int64)


def build(points, n_max: int, max_level: int = 64, min_level: int = 0) -> Tree:
    x = np.asarray(points)
    n, d = x.shape
    B = bits_per_dim(d)
    lo, ext = root_cube(x)
    keys = morton(quantize(x, lo, ext, B), B)
    perm = np.argsort(keys, kind="stable")
    sk = keys[perm]
    maxlev = min(max_level, B)
    starts_all, levels_all, prefix_all = [], [], []
    split_prev = None
    box_prev = None
    nlev = 0
    for lev in range(0, maxlev + 1):
        prefix = sk >> np.uint64(d * (B - lev))
        head = np.ones(n, dtype=bool)
        head[1:] = prefix[1:] != prefix[:-1]
        start = np.nonzero(head)[0]
        count = np.diff(np.append(start, n))
        box_of_point = np.cumsum(head) - 1
        if lev == 0:
            exists = np.ones(start.shape[0], dtype=bool)
        else:
            parent = box_prev[start]
            exists = split_prev[parent]
        if not exists.any():
            break
        nlev = lev + 1
        split = exists & (lev < maxlev) & ((lev < min_level) | (count > n_max))
        leaf = exists & ~split
        starts_all.append(start[leaf])
        levels_all.append(np.full(int(leaf.sum()), lev, dtype=np.int64))
        prefix_all.append(prefix[start[leaf]])
        split_prev, box_prev = split, box_of_point
    st = np.concatenate(starts_all)
    order = np.argsort(st, kind="stable")
    st = st[order]
    lv = np.concatenate(levels_all)[order]
    pf = np.concatenate(prefix_all)[order]
    return Tree(d, B, lo, ext, sk, perm.astype(np.int64), np.append(st, n).astype(np.int64),
                lv.astype(np.int64), pf.astype(np.uint64), nlev)


def near_lists(tree: Tree):
    """CSR near lists: (ptr, idx) with idx sorted ascending per leaf.  Brute force over pairs."""
    lo, hi = tree.leaf_box()
    ptr = [0]
    idx = []
    for a in range(tree.nleaves):
        ok = np.all((lo[a] <= hi) & (lo <= hi[a]), axis=1)
        nb = np.nonzero(ok)[0]
        idx.append(nb)
        ptr.append(ptr[-1] + nb.shape[0])
    return np.asarray(ptr, dtype=np.int64), (np.concatenate(idx) if idx else np.zeros(0, np.int64)).astype(np.int64)


def coarse_cell_coords(cells: np.ndarray, d: int, lc: int) -> np.ndarray:
    return deinterleave(np.asarray(cells, dtype=np.uint64), d, lc)
