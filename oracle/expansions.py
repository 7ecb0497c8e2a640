"""Multipole and local expansion coefficients by definition -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's cpu_baseline leg may import
this module.  It shares no code with the GPU library.

The paper hands its smooth sum (Section 3.2, eq. Tk_smooth_quad) to a point
FMM without fixing the expansions.  For the 2D Laplace kernel of Section 2.1,
G(r, r0) = -(1/2pi) log|r - r0| = -(1/2pi) Re log(z0 - z) in complex
notation, so a potential is u(z0) = -(1/2pi) Re phi(z0) with
phi(z0) = sum_j q_j log(z0 - z_j).  The GPU library stores coefficients
scaled by the box side s; their plain definitions are:

  multipole about c (valid for |z0 - c| > max |z_j - c|):
      phi(z0) = A_0 log(z0 - c) + sum_{k>=1} A_k (s / (z0 - c))^k
      A_0 = sum_j q_j,   A_k = -(1/k) sum_j q_j ((z_j - c)/s)^k

  local about c (valid for |z0 - c| < min |z_j - c|):
      phi(z0) = sum_{l>=0} B_l ((z0 - c)/s)^l
      B_0 = sum_j q_j log(c - z_j),   B_l = -(1/l) sum_j q_j (s/(z_j - c))^l

Both follow from the power series of log(1 - x).  Only Re phi matters, so
the branch of the complex logarithm in A_0 / B_0 terms is immaterial.
Arrays: points complex [ns]; charges [nbatch, ns]; coefficients
[nbatch, p+1] complex.
"""
from __future__ import annotations

import numpy as np

INV_2PI = 1.0 / (2.0 * np.pi)


def _q2(q):
    q = np.asarray(q, dtype=np.float64)
    return q[None, :] if q.ndim == 1 else q


def multipole(z, q, c, s, p):
    """A_0 = sum q, A_k = -(1/k) sum q ((z - c)/s)^k, k = 1..p."""
    q = _q2(q)
    w = (np.asarray(z, dtype=np.complex128) - c) / s
    A = np.zeros((q.shape[0], p + 1), dtype=np.complex128)
    A[:, 0] = q.sum(axis=1)
    pw = np.ones_like(w)
    for k in range(1, p + 1):
        pw = pw * w
        A[:, k] = -(q * pw[None, :]).sum(axis=1) / k
    return A


def local(z, q, c, s, p):
    """B_0 = sum q log(c - z), B_l = -(1/l) sum q (s/(z - c))^l, l = 1..p."""
    q = _q2(q)
    z = np.asarray(z, dtype=np.complex128)
    B = np.zeros((q.shape[0], p + 1), dtype=np.complex128)
    B[:, 0] = (q * np.log(c - z)[None, :]).sum(axis=1)
    iw = s / (z - c)
    pw = np.ones_like(iw)
    for l in range(1, p + 1):
        pw = pw * iw
        B[:, l] = -(q * pw[None, :]).sum(axis=1) / l
    return B


def eval_multipole(A, c, s, zt):
    """u(z0) = -(1/2pi) Re[A_0 log(z0 - c) + sum_k A_k (s/(z0 - c))^k]: [nbatch, nt]."""
    A = np.atleast_2d(A)
    zt = np.asarray(zt, dtype=np.complex128)
    d = zt - c
    phi = A[:, :1] * np.log(d)[None, :]
    iw = s / d
    pw = np.ones_like(iw)
    for k in range(1, A.shape[1]):
        pw = pw * iw
        phi = phi + A[:, k:k + 1] * pw[None, :]
    return -INV_2PI * phi.real


def eval_local(B, c, s, zt):
    """u(z0) = -(1/2pi) Re sum_l B_l ((z0 - c)/s)^l: [nbatch, nt]."""
    B = np.atleast_2d(B)
    w = (np.asarray(zt, dtype=np.complex128) - c) / s
    phi = np.zeros((B.shape[0], w.shape[0]), dtype=np.complex128)
    for l in range(B.shape[1] - 1, -1, -1):
        phi = phi * w[None, :] + B[:, l:l + 1]
    return -INV_2PI * phi.real


def eval_local_grad(B, c, s, zt):
    """Gradient of eval_local in (x0, y0): [nbatch, 2, nt].

    For analytic phi = U + iV, dU/dx = Re phi', dU/dy = -Im phi'.
    """
    B = np.atleast_2d(B)
    w = (np.asarray(zt, dtype=np.complex128) - c) / s
    dphi = np.zeros((B.shape[0], w.shape[0]), dtype=np.complex128)
    for l in range(B.shape[1] - 1, 0, -1):
        dphi = dphi * w[None, :] + l * B[:, l:l + 1]
    dphi = dphi / s
    return -INV_2PI * np.stack([dphi.real, -dphi.imag], axis=1)
