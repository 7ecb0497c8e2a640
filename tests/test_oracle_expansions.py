"""Pins of the oracle's expansion definitions against its direct sums (no GPU).

The multipole and local series are truncated power series of log(1 - x);
their error at ratio rho = r/R is bounded by sum|q| rho^(p+1)/((p+1)(1-rho)).
"""
import numpy as np

from oracle import direct
from oracle import expansions as E


def _cluster(seed, n=80, c=0.1 + 0.2j, s=0.25):
    rng = np.random.default_rng(seed)
    z = c + s * (rng.uniform(-0.5, 0.5, n) + 1j * rng.uniform(-0.5, 0.5, n))
    w = rng.uniform(0.1, 1.0, n)
    f = rng.standard_normal((2, n))
    return z, w, f, c, s


def test_multipole_far_evaluation():
    z, w, f, c, s = _cluster(0)
    q = w[None, :] * f
    p = 20
    A = E.multipole(z, q, c, s, p)
    th = np.linspace(0, 2 * np.pi, 9)[:-1]
    R = 3.0 * s
    zt = c + R * np.exp(1j * th)
    got = E.eval_multipole(A, c, s, zt)
    ref = direct.smooth(z.real, z.imag, w, f, zt.real, zt.imag)
    rho = (np.sqrt(0.5) * s) / R
    bound = np.abs(q).sum(1).max() * rho ** (p + 1) / ((p + 1) * (1 - rho)) / (2 * np.pi)
    assert np.max(np.abs(got - ref)) <= bound
    assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_local_near_evaluation_and_gradient():
    z, w, f, c, s = _cluster(1)
    q = w[None, :] * f
    p = 24
    cl = c + 3.0 * s  # expansion centre well away from the cluster
    B = E.local(z, q, cl, s, p)
    rng = np.random.default_rng(2)
    zt = cl + 0.5 * s * (rng.uniform(-0.5, 0.5, 10) + 1j * rng.uniform(-0.5, 0.5, 10))
    got = E.eval_local(B, cl, s, zt)
    ref = direct.smooth(z.real, z.imag, w, f, zt.real, zt.imag)
    assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))
    g = E.eval_local_grad(B, cl, s, zt)
    gref = direct.smooth_grad(z.real, z.imag, w, f, zt.real, zt.imag)
    assert np.max(np.abs(g - gref)) <= 1e-10 * np.max(np.abs(gref))


def test_multipole_of_union_is_sum_of_shifted_parts():
    """Coefficients are linear in the charges: splitting a set changes nothing."""
    z, w, f, c, s = _cluster(3)
    q = w[None, :] * f
    A = E.multipole(z, q, c, s, 12)
    A1 = E.multipole(z[:30], q[:, :30], c, s, 12)
    A2 = E.multipole(z[30:], q[:, 30:], c, s, 12)
    assert np.allclose(A, A1 + A2, rtol=0, atol=1e-14)
