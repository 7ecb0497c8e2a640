"""GPU generation of own-cell singular corrections (vp_correction_blocks;
Section 4.1 eq. singcorr_inner_prod, Section 4.2 eq. mapbox_singular_quad)
against the CPU oracle (oracle.corrections), through the C ABI.

Tolerance: rows of a block agree with the oracle to 2e-13 of the row's
largest entry (the two integrate the same singular integrals by different
rules: Duffy rays with exact u moments and graded v panels, against polar
coordinates with tanh-sinh radii and adaptive angles; measured up to 9e-14).  At the full size of
the star workload's 4,096 boundary triangles, every row is checked against a
property that holds at any size: its entries plus the smooth weights sum to
the closed-form integral of G over the cell (the Lagrange basis sums to one).
"""
import numpy as np
import pytest

from oracle import corrections as CO
from vp_workloads import generators as gen

pytestmark = pytest.mark.gpu
G_SCALE = -1.0 / (2.0 * np.pi)


def _vp():
    import torch  # noqa: F401
    from paper_2203_05933_amd import vp
    return vp


def _dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _smooth_rows(ref, wref, o, A):
    """G(r_j, r_i) |det A| wref_j off the diagonal, [N, N]."""
    r = o[None, :] + ref @ A.T
    d = np.hypot(r[:, None, 0] - r[None, :, 0], r[:, None, 1] - r[None, :, 1])
    np.fill_diagonal(d, 1.0)
    g = G_SCALE * np.log(d) * abs(np.linalg.det(A)) * wref[None, :]
    np.fill_diagonal(g, 0.0)
    return g


def test_box_blocks_match_oracle():
    vp = _vp()
    xi, eta, w = gen.gauss_legendre_box_nodes(8)
    ref = np.stack([xi, eta], 1)
    cells = [((0.3, -0.2), 1.0 / 256), ((-4.0, 2.5), 0.7)]
    maps = gen.cell_maps([c[0] for c in cells], [h * np.eye(2) for _, h in cells])
    C = _host(vp.correction_blocks("box", 8, xi, eta, w, _dev(maps)))
    assert C.shape == (2, 64, 64)
    for k, (o, h) in enumerate(cells):
        Co = CO.block(CO.BOX, 8, ref, w, o, h * np.eye(2), rows=[0, 27, 63])
        for i in (0, 27, 63):
            err = np.max(np.abs(C[k, i] - Co[i])) / np.max(np.abs(Co[i]))
            print(f"box h={h} row {i}: rel {err:.2e}")
            assert err <= 2e-13


@pytest.mark.parametrize("which", ["band0", "band_last", "skinny", "clockwise"])
def test_triangle_blocks_match_oracle(which):
    vp = _vp()
    xi, eta, w = gen.triangle_lattice_pattern(9)
    ref = np.stack([xi, eta], 1)
    band = gen.star_band_triangles()
    tri = {"band0": band[0], "band_last": band[-1],
           "skinny": np.array([[0.0, 0.0], [1.0, 0.02], [0.3, 0.05]]),
           "clockwise": np.array([[0.2, 0.1], [0.1, 0.4], [0.6, 0.3]])}[which]
    maps = gen.triangle_maps(tri[None])
    C = _host(vp.correction_blocks("triangle", 9, xi, eta, w, _dev(maps)))[0]
    o, A = maps[0, :2], maps[0, 2:].reshape(2, 2)
    rows = [0, 44]
    Co = CO.block(CO.TRIANGLE, 9, ref, w, o, A, rows=rows)
    for i in rows:
        err = np.max(np.abs(C[i] - Co[i])) / np.max(np.abs(Co[i]))
        print(f"triangle {which} row {i}: rel {err:.2e}")
        assert err <= 2e-13


def test_star_band_triangles_full_size_row_sums():
    """All 4,096 boundary-band triangles of the star workload (45 nodes
    each): every row's singular integrals (correction plus smooth terms)
    sum to the closed-form integral of G over the triangle."""
    vp = _vp()
    xi, eta, w = gen.triangle_lattice_pattern(9)
    ref = np.stack([xi, eta], 1)
    tris = gen.star_band_triangles()
    maps = gen.triangle_maps(tris)
    C = _host(vp.correction_blocks("triangle", 9, xi, eta, w, _dev(maps)))
    assert C.shape == (4096, 45, 45) and np.all(np.isfinite(C))
    A = maps[:, 2:].reshape(-1, 2, 2)
    o = maps[:, :2]
    targets = o[:, None, :] + np.einsum("kab,nb->kna", A, ref)       # [4096, 45, 2]
    J = np.abs(np.linalg.det(A))
    d = np.linalg.norm(targets[:, :, None, :] - targets[:, None, :, :], axis=3)
    idx = np.arange(45)
    d[:, idx, idx] = 1.0
    smooth = G_SCALE * np.log(d) * (J[:, None, None] * w[None, None, :])
    smooth[:, idx, idx] = 0.0
    S_sum = (C + smooth).sum(axis=2)                                 # [4096, 45]
    ccw = tris.copy()
    flip = np.linalg.det(A) < 0
    ccw[flip] = ccw[flip][:, ::-1]
    exact = G_SCALE * CO.polygon_log_integral_many(np.repeat(ccw, 45, axis=0), targets.reshape(-1, 2))
    err = np.abs(S_sum.ravel() - exact) / (J.repeat(45) * (1.0 + np.abs(np.log(np.sqrt(J.repeat(45))))))
    print(f"4096 band triangles: max row-sum error {err.max():.2e} (units of area x log size)")
    assert err.max() <= 1e-13


def test_box_levels_full_blocks_row_sums_and_repeatability():
    """The 8 x 8 Gauss-Legendre box pattern at the star workload's three box
    levels: every row against the closed form of int log r over rectangles;
    a second call gives the same bits."""
    vp = _vp()
    xi, eta, w = gen.gauss_legendre_box_nodes(8)
    ref = np.stack([xi, eta], 1)
    hs = [2.6 / 2 ** (lvl + 1) for lvl in (7, 8, 9)]
    maps = gen.cell_maps(np.zeros((3, 2)), [h * np.eye(2) for h in hs])
    md = _dev(maps)
    C = _host(vp.correction_blocks("box", 8, xi, eta, w, md))
    C2 = _host(vp.correction_blocks("box", 8, xi, eta, w, md))
    assert np.array_equal(C, C2)
    for k, h in enumerate(hs):
        S_sum = (C[k] + _smooth_rows(ref, w, np.zeros(2), h * np.eye(2))).sum(axis=1)
        exact = np.array([G_SCALE * CO.box_log_integral(-h, h, -h, h, h * ref[i]) for i in range(64)])
        err = np.max(np.abs(S_sum - exact)) / (h * h * (1 + abs(np.log(h))))
        print(f"box h={h}: max row-sum error {err:.2e}")
        assert err <= 1e-13


def test_edge_cases():
    """No cells (nothing to do), one node per cell (p = 1: the block is the
    cell's whole integral of G at its centre), and a singular map rejected."""
    import torch
    vp = _vp()
    xi, eta, w = gen.gauss_legendre_box_nodes(8)
    empty = vp.correction_blocks("box", 8, xi, eta, w, torch.zeros((0, 6), dtype=torch.float64, device="cuda:0"))
    assert empty.shape == (0, 64, 64)
    h = 0.3
    C = _host(vp.correction_blocks("box", 1, [0.0], [0.0], [4.0], _dev(gen.cell_maps([[1.0, 1.0]], [h * np.eye(2)]))))
    exact = G_SCALE * CO.box_log_integral(1 - h, 1 + h, 1 - h, 1 + h, np.array([1.0, 1.0]))
    assert abs(C[0, 0, 0] - exact) <= 1e-14 * h * h
    xt, yt, wt = gen.triangle_lattice_pattern(1)
    Ct = _host(vp.correction_blocks("triangle", 1, xt, yt, wt, _dev(gen.triangle_maps(gen.star_band_triangles()[:1]))))
    tri = gen.star_band_triangles()[0]
    cen = tri.mean(axis=0)
    ex_t = G_SCALE * CO.polygon_log_integral(tri, cen)
    assert abs(Ct[0, 0, 0] - ex_t) <= 1e-13 * abs(ex_t)
    bad = gen.cell_maps([[0.0, 0.0]], [np.array([[1.0, 2.0], [0.5, 1.0]])])
    with pytest.raises(vp.VPError) as e:
        vp.correction_blocks("box", 8, xi, eta, w, _dev(bad))
    assert e.value.status == vp.VP_EINVAL
