"""What an order-p FMM computes on a uniform quadtree -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's cpu_baseline leg may import
this module.  It shares no code with the GPU library.

The paper hands its smooth sum (Section 3.2, eq. Tk_smooth_quad, with the
Green's function of Section 2.1) to a point FMM without fixing the order.
An FMM that keeps p+1 coefficients is an approximation of the direct sum;
what it computes exactly (up to rounding) has a plain definition when the
tree is uniform (only U and V lists):

  u(t) = near(t) + sum over boxes A that contain t, level >= 2,
                   sum over V in V(A) of  Re-part potential at t of
                   Loc_p[ Mul_p(V) ; about c_A ]

  * near(t): the direct sum over the sources of the leaves adjacent to the
    leaf of t (its U list), a zero-distance pair contributing nothing;
  * Mul_p(V): the multipole coefficients A_0..A_p of the sources in V about
    its centre (oracle.expansions.multipole: shifting child multipoles up
    reproduces them exactly, since A_k of the parent depends only on A_j,
    j <= k, of the children);
  * Loc_p[phi; about c]: the first p+1 Taylor coefficients about c of the
    truncated multipole field phi(z) = A_0 log(z - c_V) + sum_k A_k (s_V/(z - c_V))^k,
    written out below from the derivatives of log and of negative powers;
    shifting a degree-p local polynomial to a child is exact, so evaluating
    the ancestor's polynomial at t is the same number.

Scaled coefficients as in oracle.expansions: the local about c with box side
s is phi(z) = sum_l B_l ((z - c)/s)^l; the potential is -(1/2pi) Re phi.
"""
from __future__ import annotations

from math import comb

import numpy as np

from . import expansions as OE
from . import tree as OT

INV_4PI = 1.0 / (4.0 * np.pi)


def _binomials(p, K):
    """C[l, k] = C(k+l-1, l) for l = 0..p, k = 1..K (column 0 unused), as floats."""
    key = (p, K)
    if key not in _BINOM:
        C = np.zeros((p + 1, K + 1))
        for l in range(p + 1):
            for k in range(1, K + 1):
                C[l, k] = float(comb(k + l - 1, l))
        _BINOM[key] = C
    return _BINOM[key]


_BINOM = {}


def local_of_multipole(A, cV, sV, cA, sA, p):
    """Taylor coefficients about cA (scaled by sA^l), l = 0..p, of
    phi(z) = A_0 log(z - cV) + sum_{k=1..K} A_k (sV / (z - cV))^k.

    A: [nbatch, K+1] complex.  With d = cA - cV, u = sV/d, v = sA/d:
      l = 0 : phi(cA) = A_0 log d + sum_k A_k u^k
      l >= 1: (1/l!) d^l/dz^l log(z - cV) at cA = (-1)^(l-1) / (l d^l)
              (1/l!) d^l/dz^l (z - cV)^-k at cA  = (-1)^l C(k+l-1, l) d^(-k-l)
    each multiplied by sA^l, so B_l = A_0 (-1)^(l-1) v^l / l
    + sum_k A_k (-1)^l C(k+l-1, l) u^k v^l.  Returns [nbatch, p+1] complex.
    """
    A = np.atleast_2d(np.asarray(A, dtype=np.complex128))
    K = A.shape[1] - 1
    d = complex(cA - cV)
    u = sV / d  # source scale over distance
    v = sA / d  # target scale over distance
    l = np.arange(p + 1)
    k = np.arange(K + 1)
    sign = np.where(l % 2 == 0, 1.0, -1.0)
    # T[l, k] for k >= 1; column 0 holds the log term's coefficients
    T = sign[:, None] * _binomials(p, K) * (u ** k)[None, :] * (v ** l)[:, None]
    T[:, 0] = 0.0
    T[1:, 0] = -sign[1:] * v ** l[1:] / l[1:]
    B = A @ T.T
    B[:, 0] = A[:, 0] * np.log(d) + A[:, 1:] @ (u ** k[1:])
    return B


def evaluate_uniform(x, y, w, f, root, max_leaf, p):
    """The order-p FMM value at every node (targets = nodes), for a tree
    without W or X lists.  Returns [nbatch, n] in the caller's order."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    f = np.atleast_2d(np.asarray(f, dtype=np.float64))
    tr = OT.build_tree(x, y, root=root, max_leaf=max_leaf)
    lists = OT.all_lists(tr)
    for k in "WX":
        if lists[k][1].size:
            raise ValueError("evaluate_uniform needs a tree without W and X lists")
    perm = tr.src_perm
    z = (x + 1j * y)[perm]
    q = (np.asarray(w)[None, :] * f)[:, perm]
    nb = f.shape[0]
    out = np.zeros((nb, x.size))
    up, ui = lists["U"]
    vp_, vi = lists["V"]
    # multipoles of every box of level >= 2 from its own sources
    mult = {}
    for b in range(tr.nbox):
        if tr.level[b] < 2:
            continue
        cx, cy, h = OT.box_center(tr, b)
        sl = slice(tr.src_begin[b], tr.src_end[b])
        mult[b] = OE.multipole(z[sl], q[:, sl], cx + 1j * cy, h, p)
    # local polynomial of every box: its V list's truncated multipole fields
    loc = {}
    for b in range(tr.nbox):
        if tr.level[b] < 2:
            continue
        cx, cy, h = OT.box_center(tr, b)
        Bsum = np.zeros((nb, p + 1), dtype=np.complex128)
        for a in vi[vp_[b]:vp_[b + 1]]:
            ax, ay, ha = OT.box_center(tr, a)
            Bsum += local_of_multipole(mult[a], ax + 1j * ay, ha, cx + 1j * cy, h, p)
        loc[b] = (Bsum, cx + 1j * cy, h)
    for b in np.nonzero(tr.leaf)[0]:
        sl = slice(tr.src_begin[b], tr.src_end[b])
        zt = z[sl]
        if zt.size == 0:
            continue
        # near field by the definition
        idx = np.concatenate([np.arange(tr.src_begin[a], tr.src_end[a]) for a in ui[up[b]:up[b + 1]]])
        dz = zt[:, None] - z[idx][None, :]
        r2 = dz.real ** 2 + dz.imag ** 2
        with np.errstate(divide="ignore"):
            g = np.where(r2 > 0, -INV_4PI * np.log(np.where(r2 > 0, r2, 1.0)), 0.0)
        u = q[:, idx] @ g.T
        # far field: the local polynomials of the leaf and its ancestors
        for a in OT.ancestors_or_self(tr, int(b)):
            if tr.level[a] < 2:
                break
            Bsum, c, h = loc[a]
            u = u + OE.eval_local(Bsum, c, h, zt)
        out[:, perm[sl]] = u
    return out
