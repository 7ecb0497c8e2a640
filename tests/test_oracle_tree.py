"""Pins of the oracle's quadtree and interaction lists (no GPU).

The lists are checked against the property that makes an FMM exact up to
truncation: every (target leaf, source leaf) pair is accounted for exactly
once, and every far route is well separated.
"""
import numpy as np
import pytest

from oracle import tree as T
from vp_workloads import generators as gen


def _clustered(seed, n_uniform=1500, n_a=1500, n_b=600):
    rng = np.random.default_rng(seed)
    pts = np.concatenate([rng.normal(0.3, 0.02, (n_a, 2)), rng.uniform(-1, 1, (n_uniform, 2)),
                          rng.normal(-0.5, 0.005, (n_b, 2))])
    return np.clip(pts, -0.999, 0.999), rng


def test_morton_key_matches_quadrant_descent():
    """The top 2l key bits are the quadrant path of recursive halving."""
    rng = np.random.default_rng(0)
    x = rng.uniform(-1, 1, 200)
    y = rng.uniform(-1, 1, 200)
    k = T.morton_key(T.quantise(x, -1.0, 2.0), T.quantise(y, -1.0, 2.0))
    for i in range(200):
        lo_x, lo_y, side = -1.0, -1.0, 2.0
        path = 0
        for lev in range(12):
            side /= 2
            bx = int(x[i] >= lo_x + side)
            by = int(y[i] >= lo_y + side)
            lo_x += bx * side
            lo_y += by * side
            path = (path << 2) | (by << 1) | bx
        assert int(k[i]) >> (2 * (T.LBITS - 12)) == path


def test_quantise_edges():
    q = T.quantise(np.array([-1.0, 1.0, 0.0, -3.0, 7.0]), -1.0, 2.0)
    assert list(q) == [0, (1 << 30) - 1, 1 << 29, 0, (1 << 30) - 1]


@pytest.mark.parametrize("case", ["uniform", "clustered_self", "clustered_targets"])
def test_tree_invariants_and_coverage(case):
    if case == "uniform":
        wl = gen.config0()
        x, y, tx, ty, ml = wl.x, wl.y, None, None, 64
    else:
        pts, rng = _clustered(1)
        x, y = pts[:, 0], pts[:, 1]
        ml = 24
        if case == "clustered_targets":
            t = rng.uniform(-1, 1, (400, 2))
            tx, ty = t[:, 0], t[:, 1]
        else:
            tx = ty = None
    tr = T.build_tree(x, y, tx, ty, root=(-1.0, -1.0, 2.0), max_leaf=ml)
    leaf = tr.leaf
    # leaves partition the sorted points; counts respect max_leaf
    lb = np.nonzero(leaf)[0]
    order = np.lexsort((tr.src_end[lb], tr.src_begin[lb]))
    sb, se = tr.src_begin[lb][order], tr.src_end[lb][order]
    assert sb[0] == 0 and se[-1] == x.shape[0] and np.all(sb[1:] == se[:-1])
    assert np.all(se - sb <= ml) and np.all(tr.tgt_end[lb] - tr.tgt_begin[lb] <= ml)
    # points lie in their box's closed square
    x0, y0, side = tr.root
    for b in lb[:: max(1, lb.size // 50)]:
        cx, cy, h = T.box_center(tr, b)
        idx = tr.src_perm[tr.src_begin[b]:tr.src_end[b]]
        assert np.all(np.abs(x[idx] - cx) <= h / 2 + 1e-15) and np.all(np.abs(y[idx] - cy) <= h / 2 + 1e-15)
    # children: contiguous, next level, ranges partition the parent's
    for b in np.nonzero(~leaf)[0]:
        c0, nc = tr.child_begin[b], tr.nchild[b]
        ch = np.arange(c0, c0 + nc)
        assert np.all(tr.parent[ch] == b) and np.all(tr.level[ch] == tr.level[b] + 1)
        assert tr.src_begin[ch[0]] == tr.src_begin[b] and tr.src_end[ch[-1]] == tr.src_end[b]
    # Morton order inside each level
    for l in range(tr.nlevels):
        s = slice(tr.level_begin[l], tr.level_begin[l + 1])
        keys = T.morton_key(tr.ix[s], tr.iy[s])
        assert np.all(np.diff(keys.astype(np.int64)) > 0)
    # coverage: each (target leaf, source leaf) pair exactly once
    lists = T.all_lists(tr)
    cnt, leaves = T.coverage_counts(tr, lists)
    sub = cnt[np.ix_(leaves, leaves)]
    assert sub.min() == 1 and sub.max() == 1
    if case != "uniform":
        assert lists["W"][1].size > 0 and lists["X"][1].size > 0


def test_list_symmetries_and_separation():
    pts, _ = _clustered(2)
    tr = T.build_tree(pts[:, 0], pts[:, 1], root=(-1.0, -1.0, 2.0), max_leaf=16)
    L = T.all_lists(tr)

    def pairs(name):
        p, v = L[name]
        return {(b, int(a)) for b in range(tr.nbox) for a in v[p[b]:p[b + 1]]}

    U, V, W, X = (pairs(k) for k in "UVWX")
    assert U == {(a, b) for (b, a) in U}
    assert V == {(a, b) for (b, a) in V}
    assert X == {(a, b) for (b, a) in W}
    # separation: V boxes are at least one box side apart (Chebyshev gap);
    # W/X pairs at least one side of the smaller box apart.
    for (b, a) in list(V)[:2000] + list(W)[:2000]:
        l = max(tr.level[a], tr.level[b])
        ax0 = tr.ix[a] << (l - tr.level[a]); ax1 = (tr.ix[a] + 1) << (l - tr.level[a])
        ay0 = tr.iy[a] << (l - tr.level[a]); ay1 = (tr.iy[a] + 1) << (l - tr.level[a])
        bx0 = tr.ix[b] << (l - tr.level[b]); bx1 = (tr.ix[b] + 1) << (l - tr.level[b])
        by0 = tr.iy[b] << (l - tr.level[b]); by1 = (tr.iy[b] + 1) << (l - tr.level[b])
        gap = max(ax0 - bx1, bx0 - ax1, ay0 - by1, by0 - ay1)
        assert gap >= 1


def test_uniform_v_list_count_and_offsets():
    """In a uniform tree every interior box has 27 V-list boxes at offsets
    within [-3,3]^2 outside [-1,1]^2."""
    wl = gen.config0()
    tr = T.build_tree(wl.x, wl.y, root=wl.root, max_leaf=64)
    L = T.all_lists(tr)
    p, v = L["V"]
    assert v.size == 6900
    for b in range(tr.level_begin[4], tr.level_begin[5]):
        if 2 <= tr.ix[b] <= 13 and 2 <= tr.iy[b] <= 13:
            lst = v[p[b]:p[b + 1]]
            assert lst.size == 27
            off = np.stack([tr.ix[lst] - tr.ix[b], tr.iy[lst] - tr.iy[b]], 1)
            assert np.all(np.abs(off).max(1) >= 2) and np.all(np.abs(off).max(1) <= 3)
