"""Pins of the CPU oracle's direct sums against facts fixed by the paper and by
the mathematics (no GPU).  Each test would fail on a plausible slip in the
oracle: a wrong 1/(2 pi) factor, a sign, a transposed index, a dropped
correction term, a wrong weight convention.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.sparse
from scipy.special import exp1

from oracle import direct
from vp_workloads import generators as gen


def _rand_nodes(n, seed, lo=-1.0, hi=1.0):
    rng = np.random.default_rng(seed)
    x = rng.uniform(lo, hi, n)
    y = rng.uniform(lo, hi, n)
    w = rng.uniform(0.1, 1.0, n)
    return x, y, w, rng


def test_mpmath_brute_force_tiny():
    """30-digit brute force of s(t) = sum_j -(1/2pi) log|r_j - t| w_j f_j (Section 2.1 G)."""
    x, y, w, rng = _rand_nodes(40, 1)
    f = rng.standard_normal(40)
    tx = rng.uniform(-2, 2, 6)
    ty = rng.uniform(-2, 2, 6)
    got = direct.smooth(x, y, w, f, tx, ty)[0]
    mpmath.mp.dps = 30
    for i in range(6):
        acc = mpmath.mpf(0)
        for j in range(40):
            d = mpmath.sqrt((mpmath.mpf(x[j]) - tx[i]) ** 2 + (mpmath.mpf(y[j]) - ty[i]) ** 2)
            acc += -mpmath.log(d) / (2 * mpmath.pi) * mpmath.mpf(w[j]) * mpmath.mpf(f[j])
        ref = float(acc)
        assert abs(got[i] - ref) <= 1e-15 * max(1.0, abs(ref))


def _square_closed_form(tx, ty, a=-1.0, b=1.0):
    """-(1/4pi) int_{[a,b]^2} log((x-tx)^2 + (y-ty)^2) dA by the antiderivative
    F(x,y) = x y log(x^2+y^2) - 3xy + x^2 atan(y/x) + y^2 atan(x/y)."""

    def F(X, Y):
        return X * Y * math.log(X * X + Y * Y) - 3 * X * Y + X * X * math.atan(Y / X) + Y * Y * math.atan(X / Y)

    x0, x1, y0, y1 = a - tx, b - tx, a - ty, b - ty
    return -(F(x1, y1) - F(x0, y1) - F(x1, y0) + F(x0, y0)) / (4 * math.pi)


def test_unit_density_square_closed_form():
    """f = 1 on [-1,1]^2: the smooth rule (8x8 GL per box, weights summing to the
    box area) reproduces the closed-form log potential of the square at targets
    well outside it.  Pins G's normalisation and the weight convention."""
    x, y, w = gen.uniform_grid(16)
    f = np.ones_like(x)
    tx = np.array([1.7, 0.37, -1.31, 2.9, -2.2, 1.45])
    ty = np.array([0.3, -2.2, 1.9, -0.13, -2.6, 1.52])
    got = direct.smooth(x, y, w, f, tx, ty)[0]
    ref = np.array([_square_closed_form(a, b) for a, b in zip(tx, ty)])
    assert np.max(np.abs(got - ref)) <= 2e-14 * np.max(np.abs(ref))


def test_scaling_law():
    """Scaling all positions by 2 adds exactly -(log 2 / 2pi) sum_{j != i} w_j f_j."""
    x, y, w, rng = _rand_nodes(300, 2)
    f = rng.standard_normal(300)
    u = direct.smooth(x, y, w, f)[0]
    us = direct.smooth(2 * x, 2 * y, w, f)[0]
    tot = np.sum(w * f) - w * f  # excludes the self pair
    ref = u - math.log(2.0) / (2 * math.pi) * tot
    assert np.max(np.abs(us - ref)) <= 1e-13 * np.max(np.abs(u))


def test_translation_invariance_and_linearity():
    x, y, w, rng = _rand_nodes(250, 3)
    f1 = rng.standard_normal(250)
    f2 = rng.standard_normal(250)
    u1 = direct.smooth(x, y, w, f1)[0]
    u2 = direct.smooth(x, y, w, f2)[0]
    ush = direct.smooth(x + 0.5, y - 0.25, w, f1)[0]
    assert np.max(np.abs(ush - u1)) <= 1e-13 * np.max(np.abs(u1))
    ulin = direct.smooth(x, y, w, np.stack([0.3 * f1 - 1.7 * f2]))[0]
    assert np.max(np.abs(ulin - (0.3 * u1 - 1.7 * u2))) <= 1e-13 * np.max(np.abs(ulin))
    # batched evaluation equals separate ones
    ub = direct.smooth(x, y, w, np.stack([f1, f2]))
    assert np.array_equal(ub[0], u1) and np.array_equal(ub[1], u2)


def test_far_field_moments():
    """Far away, s(t) = -(1/2pi)[M0 log|t| - Re sum_k M_k / (k t^k)], M_k = sum w f z^k."""
    x, y, w, rng = _rand_nodes(200, 4)
    f = rng.standard_normal(200)
    z = x + 1j * y
    q = w * f
    th = rng.uniform(0, 2 * np.pi, 5)
    for R in (1e2, 1e4):
        t = R * np.exp(1j * th)
        got = direct.smooth(x, y, w, f, t.real, t.imag)[0]
        ser = np.sum(q) * np.log(np.abs(t))
        for k in range(1, 12):
            ser = ser - (np.sum(q * z ** k) / (k * t ** k)).real
        ref = -ser / (2 * np.pi)
        assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_narrow_gaussian_newton_potential():
    """A radial Gaussian exp(-rho^2/sigma^2) has the Newton potential
    -(sigma^2/2)[log rho + E1(rho^2/sigma^2)/2]; with sigma = 0.06 centred in
    [-1,1]^2 the truncation at the square is below 1e-100, so the discrete rule
    must match it at targets off the Gaussian's support."""
    x, y, w = gen.uniform_grid(32)
    sig = 0.06
    c = (0.0625, -0.0625)
    f = np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2) / sig ** 2)
    tx = np.array([0.7, -0.55, 0.3, 1.6, -2.5])
    ty = np.array([0.2, 0.6, -0.8, 1.1, 0.4])
    got = direct.smooth(x, y, w, f, tx, ty)[0]
    rho = np.hypot(tx - c[0], ty - c[1])
    ref = -(sig ** 2 / 2) * (np.log(rho) + 0.5 * exp1(rho ** 2 / sig ** 2))
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_self_pair_and_zero_distance_excluded():
    x, y, w, rng = _rand_nodes(100, 5)
    f = rng.standard_normal(100)
    u_self = direct.smooth(x, y, w, f)[0]
    # same targets passed explicitly: identical (the zero-distance pair is dropped)
    u_expl = direct.smooth(x, y, w, f, x.copy(), y.copy())[0]
    assert np.array_equal(u_self, u_expl)
    # dropping node i by hand gives the same value at target i
    i = 17
    keep = np.arange(100) != i
    ui = direct.smooth(x[keep], y[keep], w[keep], f[keep], x[i:i + 1], y[i:i + 1])[0, 0]
    assert abs(ui - u_self[i]) <= 1e-15 * max(1.0, abs(ui))


def _rand_csr(m, n, nnz_per_row, seed):
    rng = np.random.default_rng(seed)
    rowptr = np.arange(0, m * nnz_per_row + 1, nnz_per_row, dtype=np.int64)
    col = np.concatenate([np.sort(rng.choice(n, nnz_per_row, replace=False)) for _ in range(m)]).astype(np.int32)
    val = rng.standard_normal(m * nnz_per_row)
    return rowptr, col, val


def test_csr_against_scipy():
    m, n = 120, 90
    rowptr, col, val = _rand_csr(m, n, 7, 6)
    rng = np.random.default_rng(7)
    f = rng.standard_normal((3, n))
    g = rng.standard_normal((3, m))
    C = scipy.sparse.csr_matrix((val, col, rowptr), shape=(m, n))
    got = direct.csr(rowptr, col, val, f)
    assert np.allclose(got, (C @ f.T).T, rtol=0, atol=1e-13)
    gotT = direct.csr_adjoint(rowptr, col, val, g, n)
    assert np.allclose(gotT, (C.T @ g.T).T, rtol=0, atol=1e-13)
    sel = np.array([3, 50, 119])
    assert np.array_equal(direct.csr(rowptr, col, val, f, sel), got[:, sel])


@pytest.mark.parametrize("self_targets", [True, False])
def test_adjoint_dot_product(self_targets):
    """<g, A f> = <A^T g, f> for the full map (smooth + correction)."""
    x, y, w, rng = _rand_nodes(150, 8)
    if self_targets:
        tx = ty = None
        m = 150
    else:
        m = 70
        tx = rng.uniform(-1.2, 1.2, m)
        ty = rng.uniform(-1.2, 1.2, m)
    rowptr, col, val = _rand_csr(m, 150, 5, 9)
    f = rng.standard_normal((2, 150))
    g = rng.standard_normal((2, m))
    Af = direct.evaluate(x, y, w, f, rowptr, col, val, tx, ty)
    ATg = direct.evaluate_adjoint(x, y, w, g, rowptr, col, val, tx, ty)
    for b in range(2):
        lhs = np.dot(g[b], Af[b])
        rhs = np.dot(ATg[b], f[b])
        assert abs(lhs - rhs) <= 1e-13 * (np.abs(g[b]) @ np.abs(Af[b]))
    # a subset of source indices picks the same values
    sel = np.array([0, 77, 149])
    sub = direct.evaluate_adjoint(x, y, w, g, rowptr, col, val, tx, ty, sidx=sel)
    assert np.allclose(sub, ATg[:, sel], rtol=0, atol=1e-15 * np.max(np.abs(ATg)))


def test_target_gradient_central_difference():
    x, y, w, rng = _rand_nodes(300, 10)
    f = rng.standard_normal((2, 300))
    tx = rng.uniform(-0.9, 0.9, 8)
    ty = rng.uniform(-0.9, 0.9, 8)
    gr = direct.smooth_grad(x, y, w, f, tx, ty)
    h = 1e-6
    dx = (direct.smooth(x, y, w, f, tx + h, ty) - direct.smooth(x, y, w, f, tx - h, ty)) / (2 * h)
    dy = (direct.smooth(x, y, w, f, tx, ty + h) - direct.smooth(x, y, w, f, tx, ty - h)) / (2 * h)
    scale = np.max(np.abs(gr))
    assert np.max(np.abs(gr[:, 0] - dx)) <= 1e-6 * scale
    assert np.max(np.abs(gr[:, 1] - dy)) <= 1e-6 * scale


def test_generators_weights_and_layout():
    x, y, w = gen.uniform_grid(16)
    assert x.shape == (16384,)
    assert abs(w.sum() - 4.0) < 1e-13
    # each box's 64 nodes lie in that box and its weights sum to its area
    h = 2.0 / 16
    b = 37
    ix, iy = b % 16, b // 16
    xs, ys = x[64 * b:64 * b + 64], y[64 * b:64 * b + 64]
    assert xs.min() > -1 + ix * h and xs.max() < -1 + (ix + 1) * h
    assert ys.min() > -1 + iy * h and ys.max() < -1 + (iy + 1) * h
    assert abs(w[64 * b:64 * b + 64].sum() - h * h) < 1e-15
    wl = gen.config0()
    assert wl.rowptr[-1] == 64 * 16384 and wl.col.dtype == np.int32
    assert np.all(wl.col[64 * 100:64 * 101] == np.arange(64 * (100 // 64), 64 * (100 // 64) + 64))
    wl2 = gen.config0()
    assert np.array_equal(wl.f, wl2.f) and np.array_equal(wl.val, wl2.val)
