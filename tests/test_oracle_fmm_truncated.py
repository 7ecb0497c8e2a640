"""Pins of oracle.fmm_truncated (what an order-p FMM computes on a uniform
tree) against independent code and the direct sum; CPU only."""
import numpy as np

from oracle import direct
from oracle import expansions as OE
from oracle import fmm_truncated as FT
from vp_workloads import generators as gen


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_single_charge_at_centre_equals_local_series():
    # a charge at the source centre has the exact multipole [q, 0, ...]; the
    # Taylor coefficients of q log(z - c_V) about c_A are those of the local
    # series of that charge (expansions.local, written independently)
    q = np.array([[0.7], [-1.3]])
    cV, cA, s = 0.1 - 0.2j, 0.6 + 0.3j, 0.125
    A = np.zeros((2, 21), dtype=np.complex128)
    A[:, 0] = q[:, 0]
    got = FT.local_of_multipole(A, cV, s, cA, s, 20)
    ref = OE.local(np.array([cV]), q, cA, s, 20)
    # B_0 = q log(c_A - c_V): equal up to the branch (only Re phi matters)
    assert np.allclose(got[:, 0].real, ref[:, 0].real, rtol=1e-15, atol=1e-15)
    assert _rel(got[:, 1:], ref[:, 1:]) <= 1e-14


def test_high_order_multipole_field_matches_local_of_charges():
    # a cluster in a box of side s around c_V, target box two boxes right and
    # one up: the local of its 60-term multipole field agrees with the local
    # series of the charges themselves (tail (0.71/2.24)^61, far below rounding)
    rng = np.random.default_rng(2)
    s = 0.25
    cV, cA = 0.0 + 0.0j, 2 * s + 1j * s
    z = cV + s * (rng.uniform(-0.5, 0.5, 40) + 1j * rng.uniform(-0.5, 0.5, 40))
    q = rng.standard_normal((3, 40))
    A = OE.multipole(z, q, cV, s, 60)
    got = FT.local_of_multipole(A, cV, s, cA, s, 12)
    ref = OE.local(z, q, cA, s, 12)
    assert np.allclose(got[:, 0].real, ref[:, 0].real, rtol=1e-13, atol=1e-14)
    assert _rel(got[:, 1:], ref[:, 1:]) <= 1e-12


def test_wrong_binomial_would_fail():
    # the l = 1, k = 1 entry: d/dz (s/(z - c))  * s_A = -s s_A / d^2
    A = np.zeros((1, 2), dtype=np.complex128)
    A[0, 1] = 1.0
    d = 0.5 + 0.25j
    got = FT.local_of_multipole(A, 0.0, 0.1, d, 0.2, 1)
    assert np.isclose(got[0, 1], -0.1 * 0.2 / d ** 2, rtol=1e-15)
    assert np.isclose(got[0, 0], 0.1 / d, rtol=1e-15)


def _grid8():
    x, y, w = gen.uniform_grid(8)  # 8x8 boxes of 8x8 nodes, leaf level 3
    f, _ = gen.gaussian_sum_density(x, y, 5)
    return x, y, w, f[None, :]


def test_high_order_matches_direct_sum():
    x, y, w, f = _grid8()
    ref = direct.smooth(x, y, w, f)
    got = FT.evaluate_uniform(x, y, w, f, (-1.0, -1.0, 2.0), 64, 40)
    assert _rel(got, ref) <= 1e-13


def test_truncation_error_decreases_with_order():
    x, y, w, f = _grid8()
    ref = direct.smooth(x, y, w, f)
    errs = [_rel(FT.evaluate_uniform(x, y, w, f, (-1.0, -1.0, 2.0), 64, p), ref) for p in (4, 8, 16)]
    # a real approximation (not the direct sum) that converges geometrically
    assert errs[0] > 1e-6
    assert errs[0] > 10 * errs[1] > 100 * errs[2]
