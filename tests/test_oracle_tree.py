"""Pins of the oracle tree (integer work) -- CPU only."""
import numpy as np
import pytest

from oracle import tree as T
from workloads import mixed_points, uniform_points


def test_morton_matches_bit_loop():
    rng = np.random.default_rng(0)
    for d in (2, 3, 5):
        B = T.bits_per_dim(d)
        q = rng.integers(0, 1 << B, size=(50, d))
        keys = T.morton(q, B)
        for i in range(50):
            k = 0
            for b in range(B):
                for c in range(d):
                    if (int(q[i, c]) >> b) & 1:
                        k += 1 << (b * d + c)
            assert int(keys[i]) == k
        assert np.array_equal(T.deinterleave(keys, d, B), q)


def test_quantize_range_and_clamp():
    x = uniform_points(1000, 3, 1)
    lo, ext = T.root_cube(x)
    B = T.bits_per_dim(3)
    q = T.quantize(x, lo, ext, B)
    assert q.min() >= 0 and q.max() <= (1 << B) - 1
    # the point on the far face is clamped into the last cell
    i = np.argmax(x[:, 0] - lo[0])
    if x[i, 0] - lo[0] == ext:
        assert q[i, 0] == (1 << B) - 1


@pytest.mark.parametrize("d,n,nmax", [(2, 3000, 40), (3, 5000, 64)])
def test_leaves_partition_and_split_rule(d, n, nmax):
    x = mixed_points(n, d, 3, 4, 0.01)
    tr = T.build(x, nmax, min_level=2)
    lb = tr.leaf_begin
    assert lb[0] == 0 and lb[-1] == n and np.all(np.diff(lb) > 0)
    counts = np.diff(lb)
    assert np.all((counts <= nmax) | (tr.leaf_level == tr.B))
    assert np.all(tr.leaf_level >= 2)
    # the parent of every leaf above the forced levels held more than nmax points
    for a in range(tr.nleaves):
        lev = int(tr.leaf_level[a])
        if lev <= 2:
            continue
        pp = tr.leaf_prefix[a] >> np.uint64(d)
        pref = tr.keys >> np.uint64(d * (tr.B - lev + 1))
        assert int((pref == pp).sum()) > nmax
    # perm is the stable argsort of the keys
    assert np.all(np.diff(tr.keys.astype(np.float64)) >= 0)
    assert np.array_equal(np.sort(tr.perm), np.arange(n))


def test_near_lists_symmetric_and_uniform_count():
    x = uniform_points(4096, 2, 1)
    tr = T.build(x, 10 ** 9, max_level=3, min_level=3)    # uniform depth-3 quadtree
    assert tr.nleaves == 64 and np.all(tr.leaf_level == 3)
    ptr, idx = T.near_lists(tr)
    cnt = np.diff(ptr)
    c = T.deinterleave(tr.leaf_prefix, 2, 3)
    inner = np.all((c > 0) & (c < 7), axis=1)
    assert np.all(cnt[inner] == 9)
    edge = np.sum((c == 0) | (c == 7), axis=1)
    assert np.all(cnt[edge == 1] == 6) and np.all(cnt[edge == 2] == 4)
    pairs = {(a, int(b)) for a in range(tr.nleaves) for b in idx[ptr[a]:ptr[a + 1]]}
    assert all((b, a) in pairs for (a, b) in pairs)
    assert all((a, a) in pairs for a in range(tr.nleaves))


def test_adaptive_near_lists_geometry():
    x = mixed_points(4000, 3, 9, 3, 0.01)
    tr = T.build(x, 50, min_level=1)
    ptr, idx = T.near_lists(tr)
    lo, hi = tr.leaf_box()
    # independent float check: touching closed boxes <=> gap of zero in every coordinate
    for a in range(0, tr.nleaves, 7):
        gap = np.maximum(0, np.maximum(lo - hi[a], lo[a] - hi)).max(axis=1)
        assert np.array_equal(np.nonzero(gap == 0)[0], idx[ptr[a]:ptr[a + 1]])


def test_no_pair_closer_than_cutoff_is_dropped():
    """Every pair closer than R_cut is near or inside the coarse stencil (pair cover)."""
    x = mixed_points(3000, 3, 4, 3, 0.01)
    lc, r = 3, 1
    tr = T.build(x, 60, min_level=lc)
    lo, ext = T.root_cube(x)
    w = ext / 2 ** lc
    rcut = 0.999 * (r * w)          # stencil radius r keeps all pairs with gap < r*w
    cc = T.coarse_cell_coords(tr.coarse_cell(lc), 3, lc)
    pc = np.repeat(cc, np.diff(tr.leaf_begin), axis=0)
    xs = x[tr.perm]
    for i in range(0, 3000, 37):
        dist = np.sqrt(((xs - xs[i]) ** 2).sum(1))
        close = dist < rcut
        inside = np.all(np.abs(pc - pc[i]) <= r, axis=1)
        assert np.all(inside[close])
