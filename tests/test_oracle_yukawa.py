"""Pins of oracle.yukawa (the modified Helmholtz volume potential, Green's
function (lambda^2 / 2 pi) K_0(lambda r) of Section 2.1) against facts the
mathematics fixes; CPU only.  Each would fail on a plausible slip: a missing
lambda^2, K_0 of lambda^2 r or of r, a transposed sum, the self pair kept.
"""
import math

import mpmath
import numpy as np
from scipy.special import iv, kv

from oracle import direct
from oracle import yukawa as Y
from vp_workloads import generators as gen


def _cloud(n, seed, lo=-1.0, hi=1.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, n), rng.uniform(lo, hi, n), rng.uniform(0.1, 1.0, n), rng


def test_mpmath_brute_force_tiny():
    x, y, w, rng = _cloud(30, 1)
    f = rng.standard_normal(30)
    tx, ty = rng.uniform(-2, 2, 5), rng.uniform(-2, 2, 5)
    lam = 7.0
    got = Y.smooth(x, y, w, f, lam, tx, ty)[0]
    mpmath.mp.dps = 30
    for i in range(5):
        acc = mpmath.mpf(0)
        for j in range(30):
            r = mpmath.sqrt((mpmath.mpf(x[j]) - tx[i]) ** 2 + (mpmath.mpf(y[j]) - ty[i]) ** 2)
            acc += lam ** 2 / (2 * mpmath.pi) * mpmath.besselk(0, lam * r) * mpmath.mpf(w[j]) * mpmath.mpf(f[j])
        assert abs(got[i] - float(acc)) <= 1e-14 * max(abs(float(acc)), 1e-30)


def test_small_lambda_limit_is_the_laplace_potential():
    # K_0(x) = -log(x/2) - gamma + O(x^2 log x): (1/lambda^2) u_lambda approaches
    # the Laplace potential minus (log(lambda/2) + gamma) / (2 pi) sum_{j != i} w_j f_j
    x, y, w, rng = _cloud(400, 2)
    f = rng.standard_normal(400)
    lam = 1e-5
    uy = Y.smooth(x, y, w, f, lam)[0] / lam ** 2
    ul = direct.smooth(x, y, w, f)[0]
    tot = np.sum(w * f) - w * f  # the self pair is excluded in both
    ref = ul - (math.log(lam / 2) + np.euler_gamma) / (2 * math.pi) * tot
    assert np.max(np.abs(uy - ref)) <= 1e-7 * np.max(np.abs(ref))


def test_far_field_addition_theorem():
    # a cluster about c and a far target: the Graf expansion
    # K_0(lam |z - z_j|) = sum_n K_n(lam rho) I_n(lam rho_j) cos(n (theta - theta_j))
    rng = np.random.default_rng(3)
    c = 0.2 - 0.1j
    zj = c + 0.2 * (rng.uniform(-1, 1, 50) + 1j * rng.uniform(-1, 1, 50))
    q = rng.standard_normal(50)
    lam = 4.0
    zt = c + 1.1 * np.exp(1j * np.array([0.3, 1.9, 3.5, 5.0]))
    d, dj = zt - c, zj - c
    ser = np.zeros(zt.size)
    for n in range(0, 40):
        mult = 1.0 if n == 0 else 2.0
        a = np.sum(q * iv(n, lam * np.abs(dj)) * np.exp(-1j * n * np.angle(dj)))
        ser += mult * np.real(a * kv(n, lam * np.abs(d)) * np.exp(1j * n * np.angle(d)))
    ser *= lam ** 2 / (2 * np.pi)
    got = Y.smooth(zj.real, zj.imag, np.ones(50), q, lam, zt.real, zt.imag)[0]
    assert np.max(np.abs(got - ser)) <= 1e-13 * np.max(np.abs(ser))


def test_whole_plane_integral_of_the_kernel():
    # int_{R^2} (lambda^2 / 2 pi) K_0(lambda r) dA = 1: f = 1 on [-1.5, 1.5]^2 with
    # lambda = 12 (tail beyond the square ~ e^{-18}) at targets near the centre;
    # the smooth box rule carries an error from the log singularity there
    x, y, w = gen.uniform_grid(48, lo=-1.5, hi=1.5)
    f = np.ones_like(x)
    tx, ty = np.array([0.01, -0.013]), np.array([0.017, 0.004])
    u = Y.smooth(x, y, w, f, 12.0, tx, ty)[0]
    assert np.max(np.abs(u - 1.0)) < 2e-3


def test_self_pair_excluded_and_adjoint_dot():
    x, y, w = gen.uniform_grid(4)
    rng = np.random.default_rng(5)
    f = rng.standard_normal((2, x.size))
    cell_ptr = np.arange(0, x.size + 1, 64, dtype=np.int64)
    rowptr, col, val = gen.own_cell_csr(cell_ptr, 6)
    wl = gen.Workload(name="t", x=x, y=y, w=w, f=f, tx=None, ty=None, rowptr=rowptr, col=col, val=val,
                      root=(-1.0, -1.0, 2.0), sample=None, meta={})
    lam = 10.0
    u = Y.evaluate(wl, lam)
    # definition with an explicit matrix, the diagonal removed
    r = np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :])
    G = np.where(r > 0, lam ** 2 / (2 * np.pi) * kv(0, lam * np.where(r > 0, r, 1.0)), 0.0)
    C = np.zeros((x.size, x.size))
    for i in range(x.size):
        C[i, col[rowptr[i]:rowptr[i + 1]]] += val[rowptr[i]:rowptr[i + 1]]
    ref = (f * w) @ G.T + f @ C.T
    assert np.max(np.abs(u - ref)) <= 1e-13 * np.max(np.abs(ref))
    g = rng.standard_normal(u.shape)
    d = Y.evaluate_adjoint(wl, g, lam)
    assert abs(np.sum(g * u) - np.sum(d * f)) <= 1e-12 * abs(np.sum(g * u))
