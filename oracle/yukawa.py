"""Modified Helmholtz (Yukawa) volume potential by definition -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's cpu_baseline leg may import
this module.  It shares no code with the GPU library.

Section 2.1 gives the Green's function of L = -Delta + lambda^2 in the form
G(r, r0) = (lambda^2 / 2 pi) K_0(lambda |r - r0|) (K_0 the modified Bessel
function of the second kind), and the smooth rule of Section 3.2
(eq. Tk_smooth_quad) is the same point sum with this G; Section 5 runs the
modified Helmholtz experiment with lambda^2 = 100.  The oracle is that sum
written out with scipy's K_0 (float64), plus the correction rows:

  u_b(t_i) = sum_{j: r_j != t_i} (lambda^2 / 2 pi) K_0(lambda |r_j - t_i|) w_j f_b[j]
             + sum_k C[i, k] f_b[k],

and its transpose (G is symmetric).  A pair at zero distance contributes
nothing, as for the Laplace kernel.  The sums run over sources in chunks
(numpy's pairwise summation), over targets in parallel threads.
"""
from __future__ import annotations

import concurrent.futures as cf
import os

import numpy as np
from scipy.special import k0

from . import direct

_CHUNK = 4096


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


def green(r, lam):
    """(lambda^2 / 2 pi) K_0(lambda r); r = 0 gives 0 (the excluded pair)."""
    r = np.asarray(r, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        g = (lam * lam / (2.0 * np.pi)) * k0(lam * np.where(r > 0, r, 1.0))
    return np.where(r > 0, g, 0.0)


def smooth(x, y, w, f, lam, tx=None, ty=None, tidx=None):
    """s_b(t_i) = sum_j G(r_j, t_i) w_j f_b[j]; [nbatch, m] or [nbatch, len(tidx)]."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    q = np.atleast_2d(np.asarray(f, dtype=np.float64)) * np.asarray(w, dtype=np.float64)[None, :]
    if tx is None:
        tx, ty = x, y
    tx = np.asarray(tx, dtype=np.float64)
    ty = np.asarray(ty, dtype=np.float64)
    if tidx is not None:
        tx, ty = tx[tidx], ty[tidx]
    out = np.zeros((q.shape[0], tx.size))

    def block(i0):
        i1 = min(tx.size, i0 + 256)
        acc = np.zeros((q.shape[0], i1 - i0))
        for j0 in range(0, x.size, _CHUNK):
            j1 = min(x.size, j0 + _CHUNK)
            r = np.hypot(tx[i0:i1, None] - x[None, j0:j1], ty[i0:i1, None] - y[None, j0:j1])
            acc += q[:, j0:j1] @ green(r, lam).T
        out[:, i0:i1] = acc

    with cf.ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(block, range(0, tx.size, 256)))
    return out


def evaluate(wl, lam, tidx=None):
    """Smooth sum plus correction rows at the targets of a workload."""
    u = smooth(wl.x, wl.y, wl.w, wl.f, lam, wl.tx, wl.ty, tidx)
    if wl.rowptr is not None:
        u = u + direct.csr(wl.rowptr, wl.col, wl.val, wl.f, tidx=tidx)
    return u


def evaluate_adjoint(wl, g, lam, sidx=None):
    """Transpose: d_b(r_j) = w_j sum_i G(r_j, t_i) g_b[i] + sum_i C[i, j] g_b[i]."""
    tx, ty = (wl.x, wl.y) if wl.tx is None else (wl.tx, wl.ty)
    # G is symmetric: the sum over targets at the nodes, then the weights
    s = smooth(tx, ty, np.ones(np.asarray(tx).size), g, lam, wl.x, wl.y, sidx)
    wsel = wl.w if sidx is None else wl.w[sidx]
    d = s * wsel[None, :]
    if wl.rowptr is not None:
        d = d + direct.csr_adjoint(wl.rowptr, wl.col, wl.val, g, wl.n, sidx)
    return d
