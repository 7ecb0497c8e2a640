"""Oversampled box quadrature by definition -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's cpu_baseline leg may import
this module.  It shares no code with the GPU library.

Section 4.2 (eq. fk_basis, eq. Tnm) represents the density on a box by its
tensor-product Chebyshev interpolant of order p, fixed by the values at the
tensor product of the roots of T_p (the interpolation nodes I_{B,p}), and
evaluates the smooth quadrature at the roots of T_q, q >= p (the upsampled
nodes I_{B,q}), mirroring the oversampling map O_{p,q} of Section 3.2 (next
to eq. vals_to_coeffs: values to coefficients, then the expansion's values at
the finer nodes).  The oracle follows those two steps literally in 1D:

  C_p = V_p^{-1},  V_p[i, n] = T_n(x_i)   (values at the p roots -> coefficients)
  O_1 = W_q C_p,   W_q[j, n] = T_n(y_j)   (coefficients -> values at the q roots)

and the box map is the tensor product O = O_1 (x) O_1 acting on values
ordered node a = jy * p + jx (x fastest); the sources of the smooth sum are
the q x q nodes with the density O f_p there, the targets are the p x p
nodes, and the correction columns index the p x p density values:

  u_b(t_i) = sum_j G(r_j, t_i) w_j (O f_b)_j + sum_k C[i, k] f_b[k].

(Sources and targets are distinct sets: a root of T_p is never a root of
T_q for even q = 2p, cos((4i+2) pi / 2q) against cos((2j+1) pi / 2q).)
"""
from __future__ import annotations

import numpy as np

from . import direct


def cheb_roots(n: int) -> np.ndarray:
    """Roots of T_n on [-1, 1], ascending: -cos((2i+1) pi / (2n))."""
    i = np.arange(n)
    return -np.cos((2 * i + 1) * np.pi / (2 * n))


def cheb_vandermonde(x: np.ndarray, n: int) -> np.ndarray:
    """V[i, k] = T_k(x_i), k = 0..n-1, by the three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    V = np.zeros((x.size, n))
    V[:, 0] = 1.0
    if n > 1:
        V[:, 1] = x
    for k in range(2, n):
        V[:, k] = 2 * x * V[:, k - 1] - V[:, k - 2]
    return V


def oversampling_1d(p: int, q: int) -> np.ndarray:
    """[q, p]: values at the p roots of T_p -> the degree < p interpolant's
    values at the q roots of T_q (values to coefficients, coefficients to
    values)."""
    Vp = cheb_vandermonde(cheb_roots(p), p)
    Wq = cheb_vandermonde(cheb_roots(q), p)
    return Wq @ np.linalg.solve(Vp, np.eye(p))


def oversampling_box(p: int, q: int) -> np.ndarray:
    """[q*q, p*p] tensor-product map, node a = jy * n + jx on both sides."""
    O1 = oversampling_1d(p, q)
    return np.kron(O1, O1)


def upsample(f_p, nbox: int, p: int, q: int) -> np.ndarray:
    """Per box O f: f_p [nbatch, nbox * p^2] -> [nbatch, nbox * q^2]."""
    f_p = np.atleast_2d(np.asarray(f_p, dtype=np.float64))
    O = oversampling_box(p, q)
    nb = f_p.shape[0]
    return (f_p.reshape(nb, nbox, p * p) @ O.T).reshape(nb, nbox * q * q)


def upsample_adjoint(v_q, nbox: int, p: int, q: int) -> np.ndarray:
    """O^T per box: [nbatch, nbox * q^2] -> [nbatch, nbox * p^2]."""
    v_q = np.atleast_2d(np.asarray(v_q, dtype=np.float64))
    O = oversampling_box(p, q)
    nb = v_q.shape[0]
    return (v_q.reshape(nb, nbox, q * q) @ O).reshape(nb, nbox * p * p)


def evaluate(wl, tidx=None):
    """u at the p-node targets of an oversampled box workload (see
    vp_workloads.generators.oversampled_grid): [nbatch, m] or [nbatch, len(tidx)]."""
    f_q = upsample(wl.f, wl.nbox, wl.p_interp, wl.q_interp)
    u = direct.smooth(wl.x, wl.y, wl.w, f_q, wl.tx, wl.ty, tidx=tidx)
    if wl.rowptr is not None:
        u = u + direct.csr(wl.rowptr, wl.col, wl.val, wl.f, tidx=tidx)
    return u


def evaluate_adjoint(wl, g):
    """The transpose of evaluate: df = O^T (w * V^T g) + C^T g, [nbatch, m]."""
    g = np.atleast_2d(np.asarray(g, dtype=np.float64))
    v = direct.smooth_adjoint(wl.x, wl.y, wl.w, g, wl.tx, wl.ty)
    df = upsample_adjoint(v, wl.nbox, wl.p_interp, wl.q_interp)
    if wl.rowptr is not None:
        df = df + direct.csr_adjoint(wl.rowptr, wl.col, wl.val, g, wl.m)
    return df
