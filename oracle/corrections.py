"""Own-cell singular corrections by definition -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's cpu_baseline leg may import
this module.  It shares no code with the GPU library.

Section 4.1 (eqs. maptri_singular_quad, singcorr_inner_prod) and Section 4.2
(eqs. mapbox_singular_quad, Vkhat_box): near a target the smooth rule is
replaced, cell by cell, by the exact integral of G against the cell's
polynomial interpolant of f.  For a cell mapped affinely from a reference
cell (r = o + A zeta; the box [-1, 1]^2 with tensor degree < p, or the simplex
xi, eta >= 0, xi + eta <= 1 with total degree < p), nodes r_j = o + A zeta_j
and smooth weights w_j = |det A| wref_j, a target r_i that is one of the
cell's own nodes gets

    S_ij = integral over the cell of G(r, r_i) l_j(r) dA(r)
    C_ij = S_ij - [j != i] G(r_j, r_i) w_j

(l_j: the Lagrange basis of the interpolation space on the nodes), so that
sum_j (smooth + C) f_j is the integral of G times the interpolant.  The
interpolant expressed through coefficients (V a = f) and the basis
integrals, as the paper writes it, is the same linear map.

How it is computed here (plain and slow): polar coordinates about the
target in physical space; for each edge the angle runs between its corners
and the radius to R(theta) on the edge.  With rho = R s,

    int_0^R log(rho) g(rho) rho drho = R^2 [log R int_0^1 s g ds + int_0^1 s log s g ds],

where g is the (polynomial) interpolant along the ray: the first integral by
Gauss-Legendre (exact), the second by a tanh-sinh rule (the double
exponential substitution of Takahasi and Mori, which absorbs the log at s = 0),
and the angle by scipy's adaptive vector quadrature.  The Lagrange basis comes
from an orthogonal basis of the space (Legendre products for boxes, the
collapsed-coordinate Jacobi basis for triangles) and an inverse Vandermonde in
40-digit arithmetic (mpmath).
"""
from __future__ import annotations

import functools

import mpmath
import numpy as np
from numpy.polynomial import legendre as L
from scipy.integrate import quad_vec
from scipy.special import eval_jacobi, eval_legendre

BOX, TRIANGLE = 0, 1
REF_VERTS = {
    BOX: np.array([[-1.0, -1.0], [1.0, -1.0], [1.0, 1.0], [-1.0, 1.0]]),
    TRIANGLE: np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]),
}


def basis_degrees(shape, p):
    """(a, b) degree pairs of the basis of the space (tensor, or total degree < p)."""
    if shape == BOX:
        return [(a, b) for a in range(p) for b in range(p)]
    return [(a, b) for a in range(p) for b in range(p - a)]


def basis_values(shape, p, xi, eta):
    """phi_n(xi, eta) for every basis function n: [len(xi), N].  Boxes: products
    of Legendre polynomials; triangles: the orthogonal basis on the simplex in
    collapsed coordinates (Koornwinder's construction, Section 4.1),
    P_a(2 xi / (1 - eta) - 1) (1 - eta)^a P_b^(2a+1, 0)(2 eta - 1)."""
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    eta = np.atleast_1d(np.asarray(eta, dtype=np.float64))
    if shape == BOX:
        Px = L.legvander(xi, p - 1)
        Py = L.legvander(eta, p - 1)
        return np.stack([Px[:, a] * Py[:, b] for (a, b) in basis_degrees(shape, p)], axis=1)
    t = 1.0 - eta
    c = np.where(t > 0, (2.0 * xi + eta - 1.0) / np.where(t > 0, t, 1.0), 0.0)
    y = 2.0 * eta - 1.0
    return np.stack([eval_legendre(a, c) * t ** a * eval_jacobi(b, 2 * a + 1, 0, y)
                     for (a, b) in basis_degrees(shape, p)], axis=1)


@functools.lru_cache(maxsize=16)
def _inverse_vandermonde(shape, p, ref_key):
    ref = np.array(ref_key).reshape(-1, 2)
    V = basis_values(shape, p, ref[:, 0], ref[:, 1])
    mpmath.mp.dps = 40
    Vi = mpmath.inverse(mpmath.matrix(V.tolist()))
    return np.array([[float(Vi[r, c]) for c in range(Vi.cols)] for r in range(Vi.rows)])


def lagrange_values(shape, p, ref, xi, eta):
    """l_j(xi, eta): [len(xi), N] for the nodes ref [N, 2] (reference coordinates)."""
    Vi = _inverse_vandermonde(shape, p, tuple(np.asarray(ref, dtype=np.float64).ravel()))
    return basis_values(shape, p, xi, eta) @ Vi


def _tanh_sinh(h=1.0 / 16, tmax=3.6):
    """Nodes and weights of the tanh-sinh rule on [0, 1]."""
    t = np.arange(-tmax, tmax + h / 2, h)
    a = 0.5 * np.pi * np.sinh(t)
    x = 0.5 * (1.0 + np.tanh(a))
    w = 0.5 * h * 0.5 * np.pi * np.cosh(t) / np.cosh(a) ** 2
    keep = (x > 0.0) & (x < 1.0)
    return x[keep], w[keep]


_TS_X, _TS_W = _tanh_sinh()


def _ray_integrals(shape, p, ref, Ainv, o, target, theta, edge_pt, edge_n):
    """The integrand over the angle: sum over basis j of the radial integral
    along the ray at angle theta (vector [N])."""
    e = np.array([np.cos(theta), np.sin(theta)])
    R = float(edge_n @ (edge_pt - target)) / float(edge_n @ e)
    deg = (2 * (p - 1) if shape == BOX else p - 1) + 1
    sg, wg = np.polynomial.legendre.leggauss(deg // 2 + 2)
    sg, wg = 0.5 * (sg + 1.0), 0.5 * wg

    def lag(s):
        r = target[None, :] + (R * s)[:, None] * e[None, :]
        z = (r - o[None, :]) @ Ainv.T
        return lagrange_values(shape, p, ref, z[:, 0], z[:, 1])

    smooth = (wg * sg) @ lag(sg)
    logpart = (_TS_W * _TS_X * np.log(_TS_X)) @ lag(_TS_X)
    return R * R * (np.log(R) * smooth + logpart)


def s_row(shape, p, ref, o, A, i, tol=1e-15):
    """S_i. = integral of G(r, r_i) l_j(r) over the cell r = o + A zeta, for
    target node i (it does not depend on o); absolute tolerance of the angular
    quadrature: tol times the cell's area times 1 + |log| of its size."""
    ref = np.asarray(ref, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    # G depends on r - r_i only (Section 4.2, eq. Vkhat_box): the integral is
    # that over the cell translated to o = 0, where no coordinate carries the
    # cell's offset (which would cancel in r - o and lose digits)
    o = np.zeros(2)
    Ainv = np.linalg.inv(A)
    J = abs(np.linalg.det(A))
    epsabs = tol * J * (1.0 + abs(0.5 * np.log(J)))
    target = o + A @ ref[i]
    verts = o[None, :] + REF_VERTS[shape] @ A.T
    if np.linalg.det(A) < 0:  # keep the vertices counter-clockwise
        verts = verts[::-1]
    total = np.zeros(len(ref))
    nv = len(verts)
    for k in range(nv):
        va, vb = verts[k], verts[(k + 1) % nv]
        ta = np.arctan2(*(va - target)[::-1])
        tb = np.arctan2(*(vb - target)[::-1])
        if tb < ta:
            tb += 2.0 * np.pi
        t_edge = vb - va
        n = np.array([t_edge[1], -t_edge[0]])
        res, _ = quad_vec(lambda th: _ray_integrals(shape, p, ref, Ainv, o, target, th, va, n), ta, tb,
                          epsabs=epsabs, epsrel=1e-14, limit=400)
        total += res
    return -total / (2.0 * np.pi)


def block(shape, p, ref, wref, o, A, rows=None):
    """Correction block C [N, N] (rows: only those target rows, others zero)."""
    ref = np.asarray(ref, dtype=np.float64)
    wref = np.asarray(wref, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    N = len(ref)
    r = ref @ A.T  # relative to the cell origin (only differences enter)
    J = abs(np.linalg.det(A))
    C = np.zeros((N, N))
    for i in (range(N) if rows is None else rows):
        C[i] = s_row(shape, p, ref, o, A, i)
        d = np.hypot(r[:, 0] - r[i, 0], r[:, 1] - r[i, 1])
        smooth = np.where(np.arange(N) != i, -np.log(np.where(d > 0, d, 1.0)) / (2.0 * np.pi) * J * wref, 0.0)
        C[i] -= smooth
    return C


# ---------------------------------------------------------------------------
# closed forms used as pins
# ---------------------------------------------------------------------------
def rect_log_integral(a, b):
    """int_0^a int_0^b log sqrt(x^2 + y^2) dy dx (a, b > 0)."""
    return 0.5 * (a * b * (np.log(a * a + b * b) - 3.0) + a * a * np.arctan(b / a) + b * b * np.arctan(a / b))


def box_log_integral(x0, x1, y0, y1, t):
    """int over [x0,x1]x[y0,y1] of log|r - t| dA, t inside."""
    return sum(rect_log_integral(a, b) for a in (t[0] - x0, x1 - t[0]) for b in (t[1] - y0, y1 - t[1]))


def polygon_log_integral(verts, t):
    """int over the convex polygon (counter-clockwise vertices) of log|r - t| dA, t inside:
    per edge, with d its distance from t and psi the angle from the foot of the
    perpendicular, the antiderivative (d^2/2)[tan psi (log d - log cos psi - 3/2) + psi]."""
    total = 0.0
    nv = len(verts)
    for k in range(nv):
        va, vb = np.asarray(verts[k], float), np.asarray(verts[(k + 1) % nv], float)
        e = (vb - va) / np.linalg.norm(vb - va)
        foot = va + e * float(e @ (t - va))
        d = np.linalg.norm(foot - t)
        pa, pb = float(e @ (va - foot)), float(e @ (vb - foot))
        H = lambda s: 0.5 * d * d * (np.tan(np.arctan2(s, d)) * (np.log(d) - np.log(np.cos(np.arctan2(s, d))) - 1.5)
                                     + np.arctan2(s, d))
        total += H(pb) - H(pa)
    return total


def polygon_log_integral_many(verts, t):
    """polygon_log_integral for many (polygon, target) pairs at once:
    verts [M, nv, 2] (counter-clockwise), t [M, 2] -> [M]."""
    verts = np.asarray(verts, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    total = np.zeros(len(t))
    nv = verts.shape[1]
    for k in range(nv):
        va, vb = verts[:, k], verts[:, (k + 1) % nv]
        e = vb - va
        e = e / np.linalg.norm(e, axis=1)[:, None]
        foot = va + e * np.sum(e * (t - va), axis=1)[:, None]
        d = np.linalg.norm(foot - t, axis=1)
        pa, pb = np.sum(e * (va - foot), axis=1), np.sum(e * (vb - foot), axis=1)

        def H(s):
            psi = np.arctan2(s, d)
            return 0.5 * d * d * (np.tan(psi) * (np.log(d) - np.log(np.cos(psi)) - 1.5) + psi)
        total += H(pb) - H(pa)
    return total
