"""Pins of oracle.oversample (the box oversampling map O_{p,q} and the
oversampled smooth sum) against facts the mathematics fixes; CPU only.

Each would fail on a plausible slip: a wrong node set or ordering, an
interpolant of the wrong degree, a transposed tensor product, a wrong
quadrature weight, the correction applied to the upsampled values instead of
the density values, a missing O^T in the adjoint.
"""
import math

import numpy as np

from oracle import direct
from oracle import oversample as OS
from vp_workloads import generators as gen


def _lagrange(xs, xt):
    """L[j, i] = prod_{k != i} (xt_j - xs_k) / (xs_i - xs_k): the Lagrange
    basis written out (a different route from the oracle's coefficients)."""
    L = np.ones((xt.size, xs.size))
    for i in range(xs.size):
        for k in range(xs.size):
            if k != i:
                L[:, i] *= (xt - xs[k]) / (xs[i] - xs[k])
    return L


def test_nodes_are_chebyshev_roots():
    for n in (1, 2, 8, 16):
        r = OS.cheb_roots(n)
        assert np.all(np.diff(r) > 0)
        # T_n(x) = cos(n acos x) vanishes at every node
        assert np.max(np.abs(np.cos(n * np.arccos(r)))) < 1e-13
        assert np.allclose(r, gen.chebyshev_roots(n), rtol=0, atol=0)


def test_1d_map_reproduces_degree_below_p_only():
    p, q = 8, 16
    O1 = OS.oversampling_1d(p, q)
    xp, xq = OS.cheb_roots(p), OS.cheb_roots(q)
    for k in range(p):
        assert np.max(np.abs(O1 @ xp ** k - xq ** k)) < 1e-13
    # degree p is outside the interpolant's space
    assert np.max(np.abs(O1 @ xp ** p - xq ** p)) > 1e-3
    assert np.max(np.abs(O1.sum(axis=1) - 1.0)) < 1e-14


def test_1d_map_equals_lagrange_basis_and_identity():
    for p, q in ((8, 16), (5, 10), (3, 7), (6, 6)):
        O1 = OS.oversampling_1d(p, q)
        L = _lagrange(OS.cheb_roots(p), OS.cheb_roots(q))
        assert np.max(np.abs(O1 - L)) < 1e-13
    assert np.max(np.abs(OS.oversampling_1d(8, 8) - np.eye(8))) < 1e-14


def test_box_map_tensor_order():
    # node a = jy * n + jx (x fastest): x^a y^b with a, b < p is reproduced,
    # which fails if the Kronecker factors or the node order were swapped for
    # a polynomial of different degree in x and y
    p, q = 8, 16
    O = OS.oversampling_box(p, q)
    rp, rq = OS.cheb_roots(p), OS.cheb_roots(q)
    xp, yp = np.tile(rp, p), np.repeat(rp, p)
    xq, yq = np.tile(rq, q), np.repeat(rq, q)
    for a, b in ((0, 0), (7, 0), (0, 7), (3, 5), (7, 7)):
        assert np.max(np.abs(O @ (xp ** a * yp ** b) - xq ** a * yq ** b)) < 1e-12
    f = np.exp(xp) * np.cos(2 * yp)
    err = np.max(np.abs(O @ f - np.exp(xq) * np.cos(2 * yq)))
    assert 1e-8 < err < 1e-3  # a smooth function: interpolation error of degree 8, not exact


def test_fejer_weights_integrate_degree_below_q():
    for n in (1, 2, 7, 16):
        w, x = gen.fejer_weights(n), gen.chebyshev_roots(n)
        for k in range(n):
            exact = 0.0 if k % 2 else 2.0 / (k + 1)
            assert abs(np.dot(w, x ** k) - exact) < 1e-14
        assert np.all(w > 0)


def test_unit_density_far_field_closed_form():
    """f = 1 (interpolated exactly) on [-1,1]^2 as 4x4 boxes: the oversampled
    rule reproduces the closed-form log potential of the square at targets
    outside it (the antiderivative of the log kernel)."""
    wl = gen.config5(nbox_side=4, csr_seed=None, sample_seed=None)
    f = np.ones((1, wl.m))
    fq = OS.upsample(f, wl.nbox, 8, 16)
    assert np.max(np.abs(fq - 1.0)) < 1e-13
    tx = np.array([1.7, -1.4, 2.5, 0.3])
    ty = np.array([0.2, 1.9, -2.1, -1.35])
    got = direct.smooth(wl.x, wl.y, wl.w, fq, tx, ty)[0]

    def F(X, Y):
        return X * Y * math.log(X * X + Y * Y) - 3 * X * Y + X * X * math.atan(Y / X) + Y * Y * math.atan(X / Y)

    for i in range(tx.size):
        x0, x1, y0, y1 = -1 - tx[i], 1 - tx[i], -1 - ty[i], 1 - ty[i]
        ref = -(F(x1, y1) - F(x0, y1) - F(x1, y0) + F(x0, y0)) / (4 * math.pi)
        assert abs(got[i] - ref) < 1e-11 * abs(ref)


def test_evaluate_is_the_definition_and_adjoint_dot():
    wl = gen.config5(nbox_side=2, f_seeds=(3, 4), csr_seed=5, sample_seed=None)
    u = OS.evaluate(wl)
    # the definition spelled out with an explicit block-diagonal matrix
    O = OS.oversampling_box(8, 16)
    Ofull = np.kron(np.eye(wl.nbox), O)
    fq = wl.f @ Ofull.T
    dz = (wl.tx[:, None] - wl.x[None, :]) ** 2 + (wl.ty[:, None] - wl.y[None, :]) ** 2
    G = -np.log(dz) / (4 * np.pi)
    C = np.zeros((wl.m, wl.m))
    for i in range(wl.m):
        C[i, wl.col[wl.rowptr[i]:wl.rowptr[i + 1]]] += wl.val[wl.rowptr[i]:wl.rowptr[i + 1]]
    ref = (fq * wl.w) @ G.T + wl.f @ C.T
    assert np.max(np.abs(u - ref)) < 1e-13 * np.max(np.abs(ref))
    # the correction acts on the density values, not on the upsampled ones
    assert np.max(np.abs(u - OS.evaluate(gen.config5(nbox_side=2, f_seeds=(3, 4), csr_seed=None,
                                                       sample_seed=None)))) > 1e-6
    g = np.random.default_rng(9).standard_normal(u.shape)
    df = OS.evaluate_adjoint(wl, g)
    assert abs(np.sum(g * u) - np.sum(df * wl.f)) < 1e-12 * abs(np.sum(g * u))
    ref_adj = ((g @ G) * wl.w) @ Ofull + g @ C
    assert np.max(np.abs(df - ref_adj)) < 1e-13 * np.max(np.abs(ref_adj))


def test_targets_and_sources_are_distinct():
    wl = gen.config5(nbox_side=2, csr_seed=None, sample_seed=None)
    d2 = (wl.tx[:, None] - wl.x[None, :]) ** 2 + (wl.ty[:, None] - wl.y[None, :]) ** 2
    assert d2.min() > 1e-6
