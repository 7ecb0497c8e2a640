"""Plain quadtree and interaction lists -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's cpu_baseline leg may import
this module.  It shares no code with the GPU library.

The paper evaluates its target-independent smooth sum with a point FMM
(Section 1 synopsis; Section 3.2 after eq. Tk_smooth_quad, where the
modified weights J^k w_j make the sum FMM-compatible) but does not describe
the tree.  What follows is the reading the GPU library implements: the
adaptive quadtree and the U, V, W, X lists of the classical adaptive FMM,
each written here by its definition (brute force over candidate boxes),
with no traversal tricks.

Tree
  * root square (x0, y0, side); every point is quantised to a 2^30 x 2^30
    grid: q = clamp(floor(((v - v0) / side) * 2^30), 0, 2^30 - 1), computed
    in float64 in exactly that order;
  * Morton key: bit b of qx goes to bit 2b, bit b of qy to bit 2b+1;
  * points are sorted by key, ties by original index (a stable sort);
  * the root is level 0; a box is split when it holds more than max_leaf
    sources or more than max_leaf targets and its level is below max_level;
    its children are the non-empty quadrants (sources + targets > 0),
    visited in quadrant order (x bit, then y bit);
  * boxes are numbered level by level, each level in Morton order.

Lists (adjacent = the closed squares intersect)
  U(b), leaf b : leaves a adjacent to b (b itself included)
  V(b), any b  : boxes a on b's level, not adjacent to b, whose parent is
                 adjacent to b's parent
  W(b), leaf b : boxes a finer than b, not adjacent to b, whose parent is
                 adjacent to b
  X(b), any b  : leaves a coarser than b, not adjacent to b, adjacent to
                 b's parent
"""
from __future__ import annotations

import dataclasses

import numpy as np

LBITS = 30


def quantise(v, v0, side):
    """q = clamp(floor(((v - v0) / side) * 2^30), 0, 2^30 - 1) as int64."""
    t = (np.asarray(v, dtype=np.float64) - v0) / side
    t = t * float(1 << LBITS)
    q = np.floor(t)
    q = np.clip(q, 0, (1 << LBITS) - 1)
    return q.astype(np.int64)


def morton_key(qx, qy):
    """Interleave: bit b of qx -> bit 2b, bit b of qy -> bit 2b+1 (one bit at a time)."""
    qx = np.asarray(qx, dtype=np.uint64)
    qy = np.asarray(qy, dtype=np.uint64)
    k = np.zeros_like(qx)
    for b in range(LBITS):
        k |= ((qx >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
        k |= ((qy >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b + 1)
    return k


def stable_sort_by_key(keys):
    """Permutation sorting keys ascending, equal keys kept in index order."""
    idx = np.arange(keys.shape[0])
    return np.lexsort((idx, keys))


@dataclasses.dataclass
class Tree:
    root: tuple
    max_leaf: int
    max_level: int
    src_perm: np.ndarray      # sorted position -> original source index
    tgt_perm: np.ndarray      # sorted position -> original target index
    src_keys: np.ndarray      # sorted keys
    tgt_keys: np.ndarray
    level: np.ndarray         # per box
    ix: np.ndarray
    iy: np.ndarray
    parent: np.ndarray        # -1 for the root
    child_begin: np.ndarray   # index of first child, children contiguous
    nchild: np.ndarray
    src_begin: np.ndarray
    src_end: np.ndarray
    tgt_begin: np.ndarray
    tgt_end: np.ndarray
    level_begin: np.ndarray   # boxes of level l are level_begin[l]..level_begin[l+1]

    @property
    def nbox(self):
        return int(self.level.shape[0])

    @property
    def leaf(self):
        return self.nchild == 0

    @property
    def nlevels(self):
        return int(self.level_begin.shape[0]) - 1


def build_tree(x, y, tx=None, ty=None, root=(-1.0, -1.0, 2.0), max_leaf=64, max_level=LBITS):
    """Build the quadtree over sources (x, y) and targets (tx, ty) (None: the sources)."""
    x0, y0, side = root
    sk = morton_key(quantise(x, x0, side), quantise(y, y0, side))
    sp = stable_sort_by_key(sk)
    sk = sk[sp]
    if tx is None:
        tk, tp = sk, sp
    else:
        tk = morton_key(quantise(tx, x0, side), quantise(ty, y0, side))
        tp = stable_sort_by_key(tk)
        tk = tk[tp]
    ns_all, nt_all = sk.shape[0], tk.shape[0]

    level, ix, iy, parent, sb, se, tb, te = ([] for _ in range(8))
    child_begin, nchild = [], []
    level_begin = [0]
    # level 0
    cur = [(0, 0, -1, 0, ns_all, 0, nt_all)]
    lev = 0
    while cur:
        nxt = []
        base = len(level)
        for (bix, biy, par, s0, s1, t0, t1) in cur:
            level.append(lev)
            ix.append(bix)
            iy.append(biy)
            parent.append(par)
            sb.append(s0)
            se.append(s1)
            tb.append(t0)
            te.append(t1)
        # decide splits, in Morton order of this level
        next_base = base + len(cur)
        for k, (bix, biy, par, s0, s1, t0, t1) in enumerate(cur):
            ns, nt = s1 - s0, t1 - t0
            split = (ns > max_leaf or nt > max_leaf) and lev < max_level
            if not split:
                child_begin.append(-1)
                nchild.append(0)
                continue
            shift = 2 * (LBITS - lev - 1)
            prefix = _prefix(bix, biy, lev) << 2
            first = next_base + len(nxt)
            cnt = 0
            for c in range(4):
                lo = np.uint64((prefix | c) << shift)
                hi = np.uint64(((prefix | c) + 1) << shift)
                cs0 = s0 + int(np.searchsorted(sk[s0:s1], lo, side="left"))
                cs1 = s0 + int(np.searchsorted(sk[s0:s1], hi, side="left"))
                ct0 = t0 + int(np.searchsorted(tk[t0:t1], lo, side="left"))
                ct1 = t0 + int(np.searchsorted(tk[t0:t1], hi, side="left"))
                if (cs1 - cs0) + (ct1 - ct0) > 0:
                    nxt.append((2 * bix + (c & 1), 2 * biy + (c >> 1), base + k, cs0, cs1, ct0, ct1))
                    cnt += 1
            child_begin.append(first)
            nchild.append(cnt)
        level_begin.append(len(level))
        cur = nxt
        lev += 1
    a = lambda v: np.asarray(v, dtype=np.int64)
    return Tree(root=root, max_leaf=max_leaf, max_level=max_level, src_perm=a(sp), tgt_perm=a(tp),
                src_keys=sk, tgt_keys=tk, level=a(level), ix=a(ix), iy=a(iy), parent=a(parent),
                child_begin=a(child_begin), nchild=a(nchild), src_begin=a(sb), src_end=a(se),
                tgt_begin=a(tb), tgt_end=a(te), level_begin=a(level_begin))


def _prefix(ix, iy, lev):
    """Morton key prefix (2*lev bits) of box (ix, iy) on level lev."""
    k = 0
    for b in range(lev):
        k |= ((ix >> b) & 1) << (2 * b)
        k |= ((iy >> b) & 1) << (2 * b + 1)
    return k


def adjacent(tree, a, b):
    """Closed squares of boxes a and b (arrays broadcast) intersect."""
    a = np.asarray(a)
    b = np.asarray(b)
    L = np.maximum(tree.level[a], tree.level[b])
    sa = L - tree.level[a]
    sb_ = L - tree.level[b]
    ax0 = tree.ix[a] << sa
    ax1 = (tree.ix[a] + 1) << sa
    ay0 = tree.iy[a] << sa
    ay1 = (tree.iy[a] + 1) << sa
    bx0 = tree.ix[b] << sb_
    bx1 = (tree.ix[b] + 1) << sb_
    by0 = tree.iy[b] << sb_
    by1 = (tree.iy[b] + 1) << sb_
    return (ax0 <= bx1) & (bx0 <= ax1) & (ay0 <= by1) & (by0 <= ay1)


def lists_for(tree, b):
    """(U, V, W, X) of box b by definition, each sorted ascending (U, W empty for non-leaves)."""
    allb = np.arange(tree.nbox)
    lv = tree.level
    leaf = tree.leaf
    adj_b = adjacent(tree, allb, np.full(tree.nbox, b))
    U = W = np.zeros(0, dtype=np.int64)
    if leaf[b]:
        U = allb[leaf & adj_b]
        par = tree.parent
        has_par = par >= 0
        padj = np.zeros(tree.nbox, dtype=bool)
        padj[has_par] = adjacent(tree, par[has_par], np.full(has_par.sum(), b))
        W = allb[(lv > lv[b]) & ~adj_b & padj]
    V = X = np.zeros(0, dtype=np.int64)
    pb = tree.parent[b]
    if pb >= 0:
        same = (lv == lv[b]) & ~adj_b & (tree.parent >= 0)
        cand = allb[same]
        if cand.size:
            ok = adjacent(tree, tree.parent[cand], np.full(cand.size, pb))
            V = cand[ok]
        cand = allb[leaf & (lv < lv[b]) & ~adj_b]
        if cand.size:
            ok = adjacent(tree, cand, np.full(cand.size, pb))
            X = cand[ok]
    return U, V, W, X


def all_lists(tree):
    """Lists for every box: dict name -> (ptr[int64 nbox+1], idx[int64])."""
    out = {k: ([0], []) for k in "UVWX"}
    for b in range(tree.nbox):
        for name, lst in zip("UVWX", lists_for(tree, b)):
            p, v = out[name]
            v.extend(lst.tolist())
            p.append(len(v))
    return {k: (np.asarray(p, dtype=np.int64), np.asarray(v, dtype=np.int64)) for k, (p, v) in out.items()}


def ancestors_or_self(tree, b):
    out = []
    while b >= 0:
        out.append(int(b))
        b = int(tree.parent[b])
    return out


def coverage_counts(tree, lists=None):
    """For every (target leaf t, source leaf s): how many list routes account for it.

    Routes: s in U(t); an ancestor-or-self of s in W(t); a pair (B, A) with B
    an ancestor-or-self of t, A an ancestor-or-self of s and A in V(B); s in
    X(B) for an ancestor-or-self B of t.  A correct FMM counts every pair
    exactly once.  Returns a dense [nbox, nbox] count matrix (leaf rows/cols).
    """
    if lists is None:
        lists = all_lists(tree)
    nb = tree.nbox
    cnt = np.zeros((nb, nb), dtype=np.int64)
    leaves = np.nonzero(tree.leaf)[0]
    # descendant leaves of every box
    desc = {int(b): [] for b in range(nb)}
    for s in leaves:
        for a in ancestors_or_self(tree, s):
            desc[a].append(int(s))

    def L(name, b):
        p, v = lists[name]
        return v[p[b]:p[b + 1]]

    for t in leaves:
        for s in L("U", t):
            cnt[t, s] += 1
        for a in L("W", t):
            for s in desc[int(a)]:
                cnt[t, s] += 1
        for B in ancestors_or_self(tree, t):
            for A in L("V", B):
                for s in desc[int(A)]:
                    cnt[t, s] += 1
            for s in L("X", B):
                cnt[t, s] += 1
    return cnt, leaves


def box_center(tree, b):
    x0, y0, side = tree.root
    h = side / float(1 << int(tree.level[b]))
    return x0 + (tree.ix[b] + 0.5) * h, y0 + (tree.iy[b] + 0.5) * h, h
