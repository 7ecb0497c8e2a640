"""Pins of oracle.corrections (own-cell singular corrections, Section 4.1 eq.
singcorr_inner_prod and Section 4.2 eq. mapbox_singular_quad) against facts the
mathematics fixes; CPU only.  A dropped log R term, a wrong Jacobian, a
misplaced radius, a wrong basis or a smooth term left on the diagonal fails
one of them.
"""
import mpmath
import numpy as np
import pytest

from oracle import corrections as CO

G_SCALE = -1.0 / (2.0 * np.pi)


def gl_box_pattern(p=8):
    x, w = np.polynomial.legendre.leggauss(p)
    ref = np.array([(a, b) for a in x for b in x])
    wref = np.array([wa * wb for wa in w for wb in w])
    return ref, wref


def lattice_triangle_pattern(p=9, shrink=0.9):
    lat = np.array([(i / (p - 1), j / (p - 1)) for i in range(p) for j in range(p - i)])
    ref = 1.0 / 3.0 + shrink * (lat - 1.0 / 3.0)
    # interpolatory smooth weights: the integrals of the Lagrange basis
    V = CO.basis_values(CO.TRIANGLE, p, ref[:, 0], ref[:, 1])
    xg, wg = np.polynomial.legendre.leggauss(20)
    u, v = np.meshgrid(0.5 * (xg + 1), 0.5 * (xg + 1), indexing="ij")
    ww = np.outer(0.5 * wg, 0.5 * wg)
    xi, eta = (u * (1 - v)).ravel(), v.ravel()  # Duffy map of the unit square onto the simplex
    jac = (ww * (1 - v)).ravel()
    ints = jac @ CO.basis_values(CO.TRIANGLE, p, xi, eta)
    wref = np.linalg.solve(V.T, ints)
    return ref, wref


@pytest.mark.parametrize("h,o", [(1.0, (0.0, 0.0)), (0.0390625, (0.3, -0.2)), (3.0, (-5.0, 2.0))])
def test_box_row_sums_closed_form(h, o):
    """sum_j S_ij = int_box G(r, r_i) dA (the Lagrange basis sums to one),
    against the closed form of int log r over rectangles."""
    ref, _ = gl_box_pattern()
    A = h * np.eye(2)
    for i in (9, 36):
        S = CO.s_row(CO.BOX, 8, ref, o, A, i)
        t = np.asarray(o) + A @ ref[i]
        exact = G_SCALE * CO.box_log_integral(o[0] - h, o[0] + h, o[1] - h, o[1] + h, t)
        assert abs(S.sum() - exact) <= 1e-14 * max(abs(exact), h * h)


@pytest.mark.parametrize("tri", [
    [[0.1, 0.2], [0.5, 0.25], [0.2, 0.6]],
    [[1.29, 0.0], [1.30, 0.0], [1.2999, 0.0031]],      # a thin boundary-band triangle
    [[0.0, 0.0], [0.0, 1.0], [1.0, 0.0]],               # clockwise (negative determinant)
])
def test_triangle_row_sums_closed_form(tri):
    tri = np.array(tri)
    ref, _ = lattice_triangle_pattern()
    o, A = tri[0], np.stack([tri[1] - tri[0], tri[2] - tri[0]], axis=1)
    ccw = tri if np.linalg.det(A) > 0 else tri[::-1]
    for i in (8, 44):
        S = CO.s_row(CO.TRIANGLE, 9, ref, o, A, i)
        t = o + A @ ref[i]
        exact = G_SCALE * CO.polygon_log_integral(ccw, t)
        scale = abs(np.linalg.det(A)) * max(1.0, abs(np.log(np.linalg.norm(A[:, 0]))))
        assert abs(S.sum() - exact) <= 1e-13 * scale


def test_polygon_closed_form_matches_rectangles():
    """The per-edge closed form on a square reproduces the rectangle formula."""
    sq = np.array([[-1.0, -1.0], [1.0, -1.0], [1.0, 1.0], [-1.0, 1.0]])
    for t in ([0.1, -0.3], [0.9, 0.95], [-0.99, 0.0]):
        t = np.array(t)
        assert abs(CO.polygon_log_integral(sq, t) - CO.box_log_integral(-1, 1, -1, 1, t)) <= 1e-14


def _mp_lagrange_1d(nodes, a, x):
    v = mpmath.mpf(1)
    for k, xk in enumerate(nodes):
        if k != a:
            v *= (x - xk) / (nodes[a] - xk)
    return v


def test_box_entries_brute_force():
    """Single entries S_ij on a box by 2D tanh-sinh in 20-digit arithmetic over
    the four rectangles meeting at the target (tensor Lagrange basis written
    out as products)."""
    p = 8
    ref, _ = gl_box_pattern(p)
    x1d = [mpmath.mpf(v) for v in np.polynomial.legendre.leggauss(p)[0]]
    h = 0.25
    o = np.array([0.5, -0.5])
    mpmath.mp.dps = 20
    for i, j in ((27, 36),):
        S = CO.s_row(CO.BOX, p, ref, o, h * np.eye(2), i)
        ai, bi = divmod(i, p)
        aj, bj = divmod(j, p)
        tx, ty = x1d[ai], x1d[bi]
        f = lambda X, Y: (mpmath.log(h * mpmath.sqrt((X - tx) ** 2 + (Y - ty) ** 2))
                          * _mp_lagrange_1d(x1d, aj, X) * _mp_lagrange_1d(x1d, bj, Y))
        ref_val = -h * h / (2 * mpmath.pi) * mpmath.quad(f, [-1, tx, 1], [-1, ty, 1])
        assert abs(S[j] - float(ref_val)) <= 1e-13 * h * h, (i, j, S[j], float(ref_val))


def test_triangle_polynomial_reproduction_brute_force():
    """sum_j S_ij P(r_j) = int_T G(r, r_i) P(r) dA for P of total degree 8 in
    the reference coordinates, the right side by 2D tanh-sinh (20 digits)
    over the three sub-triangles at the target, each mapped from the unit
    square (apex at u = 0)."""
    p = 9
    ref, _ = lattice_triangle_pattern(p)
    tri = np.array([[0.1, 0.2], [0.5, 0.25], [0.2, 0.6]])
    o, A = tri[0], np.stack([tri[1] - tri[0], tri[2] - tri[0]], axis=1)
    J = abs(np.linalg.det(A))
    P = lambda xi, eta: xi ** 2 * eta ** 3 - 0.5 * xi ** 7 + eta ** 8 + 0.3 * xi * eta
    mpmath.mp.dps = 20
    corners = [mpmath.matrix([0, 0]), mpmath.matrix([1, 0]), mpmath.matrix([0, 1])]
    Am = mpmath.matrix(A.tolist())
    for i in (40,):
        S = CO.s_row(CO.TRIANGLE, p, ref, o, A, i)
        lhs = float(S @ P(ref[:, 0], ref[:, 1]))
        z0 = mpmath.matrix([ref[i, 0], ref[i, 1]])
        total = mpmath.mpf(0)
        for k in range(3):
            Pk, Qk = corners[k], corners[(k + 1) % 3]
            d0, d1 = Pk - z0, Qk - Pk
            cross = abs(d0[0] * d1[1] - d0[1] * d1[0])

            def f(u, v):
                d = d0 + v * d1
                z = z0 + u * d
                rphys = Am * (u * d)
                r = mpmath.sqrt(rphys[0] ** 2 + rphys[1] ** 2)
                return mpmath.log(r) * P(z[0], z[1]) * u * cross
            total += mpmath.quad(f, [0, 1], [0, 1])
        rhs = float(-J / (2 * mpmath.pi) * total)
        assert abs(lhs - rhs) <= 1e-13 * J, (i, lhs, rhs)


def test_box_scaling_law():
    """S(h) = h^2 S(1) - (h^2 log h / 2 pi) int l_j, and int l_j is the
    Gauss-Legendre product weight (the tensor pattern integrates its own
    interpolants exactly)."""
    ref, wref = gl_box_pattern()
    for i in (19,):
        S1 = CO.s_row(CO.BOX, 8, ref, (0.0, 0.0), np.eye(2), i)
        for h in (0.01, 7.0):
            Sh = CO.s_row(CO.BOX, 8, ref, (2.0, 1.0), h * np.eye(2), i)
            pred = h * h * S1 - h * h * np.log(h) / (2 * np.pi) * wref
            assert np.max(np.abs(Sh - pred)) <= 1e-14 * h * h * max(1.0, abs(np.log(h)))


def test_box_mirror_symmetry_and_smooth_diagonal():
    """Mirroring xi -> -xi maps node (a, b) to (p-1-a, b) and leaves S
    invariant; the correction keeps the whole diagonal (the smooth rule skips
    the self pair) and subtracts G w_j off it."""
    p = 8
    ref, wref = gl_box_pattern(p)
    h = 0.5
    C = CO.block(CO.BOX, p, ref, wref, (0.0, 0.0), h * np.eye(2), rows=[3, (p - 1 - 0) * p + 3])
    i, im = 3, (p - 1) * p + 3
    perm = np.array([((p - 1 - a) * p + b) for a in range(p) for b in range(p)])
    S_i = CO.s_row(CO.BOX, p, ref, (0.0, 0.0), h * np.eye(2), i)
    S_im = CO.s_row(CO.BOX, p, ref, (0.0, 0.0), h * np.eye(2), im)
    assert np.max(np.abs(S_im[perm] - S_i)) <= 1e-15
    assert C[i, i] == pytest.approx(S_i[i], rel=0, abs=1e-18)
    d = np.hypot(*(h * (ref - ref[i])).T)
    off = np.arange(p * p) != i
    assert np.max(np.abs((S_i - C[i])[off] - (-np.log(d[off]) / (2 * np.pi) * h * h * wref[off]))) <= 1e-17
