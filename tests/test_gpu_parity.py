"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Tolerances: rel_inf = max|u - u*| / max|u*| <= 1e-12 in the FP64 form and
<= 1e-6 in the FP32-bulk form (the accuracy targets of the workloads);
integer/index results (tree, permutations, lists) must match exactly.
"""
import numpy as np
import pytest

from oracle import direct
from oracle import expansions as OE
from oracle import tree as OT
from vp_workloads import generators as gen

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-6


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


def relinf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _clustered(seed, n_uniform=1500, n_a=1500, n_b=600):
    rng = np.random.default_rng(seed)
    pts = np.concatenate([rng.normal(0.3, 0.02, (n_a, 2)), rng.uniform(-1, 1, (n_uniform, 2)),
                          rng.normal(-0.5, 0.005, (n_b, 2))])
    pts = np.clip(pts, -0.999, 0.999)
    w = rng.uniform(0.1, 1.0, pts.shape[0]) / pts.shape[0]
    f = rng.standard_normal((1, pts.shape[0]))
    return pts[:, 0].copy(), pts[:, 1].copy(), w, f, rng


@pytest.fixture(scope="module")
def c0():
    return gen.config0()


# ---------------------------------------------------------------------------
# a0: tree, permutations and lists (integer work, exact)
# ---------------------------------------------------------------------------
def _compare_tree(plan, tr, self_targets):
    assert np.array_equal(plan.get_array("src_perm"), tr.src_perm)
    assert np.array_equal(plan.get_array("src_keys").astype(np.uint64), tr.src_keys)
    if not self_targets:
        assert np.array_equal(plan.get_array("tgt_perm"), tr.tgt_perm)
    assert np.array_equal(plan.get_array("level_begin"), tr.level_begin)
    box = plan.get_array("box").reshape(-1, 10)
    ref = np.stack([tr.level, tr.ix, tr.iy, tr.parent, tr.child_begin, tr.nchild, tr.src_begin,
                    tr.src_end, tr.tgt_begin, tr.tgt_end], axis=1)
    assert box.shape == ref.shape
    assert np.array_equal(box, ref)
    lists = OT.all_lists(tr)
    for k in "UVWX":
        p, v = lists[k]
        assert np.array_equal(plan.get_array(k + "_ptr"), p), k
        assert np.array_equal(plan.get_array(k + "_idx"), v), k


@pytest.mark.parametrize("case", ["uniform", "clustered_self", "clustered_targets"])
def test_tree_and_lists_match_oracle(case, c0):
    vp = _vp()
    if case == "uniform":
        x, y, w, tx, ty, ml, root = c0.x, c0.y, c0.w, None, None, 64, c0.root
    else:
        x, y, w, f, rng = _clustered(1)
        ml, root = 24, (-1.0, -1.0, 2.0)
        if case == "clustered_targets":
            t = rng.uniform(-1, 1, (400, 2))
            tx, ty = t[:, 0].copy(), t[:, 1].copy()
        else:
            tx = ty = None
    plan = vp.Plan(x, y, w, tx, ty, max_leaf=ml, root=root)
    tr = OT.build_tree(x, y, tx, ty, root=root, max_leaf=ml)
    _compare_tree(plan, tr, tx is None)
    if tx is not None:
        # separate targets: the pairwise kernel serves every U-list pair, and its
        # work count is targets of the leaf times sources of the neighbour
        p, v = OT.all_lists(tr)["U"]
        nt = tr.tgt_end - tr.tgt_begin
        ns = tr.src_end - tr.src_begin
        pairs = sum(int(nt[b]) * int(ns[v[p[b]:p[b + 1]]].sum()) for b in range(tr.nbox))
        assert plan.info()["near_pairs"] == pairs
    plan.close()


# ---------------------------------------------------------------------------
# full evaluations
# ---------------------------------------------------------------------------
def test_eval_config0_fp64(c0):
    vp = _vp()
    plan = vp.Plan(c0.x, c0.y, c0.w, rowptr=c0.rowptr, col=c0.col, val=c0.val, order=30, root=c0.root)
    u = _host(plan.eval(_dev(c0.f)))
    ref = direct.evaluate(c0.x, c0.y, c0.w, c0.f, c0.rowptr, c0.col, c0.val)
    err = relinf(u, ref)
    print(f"config0 fp64 p=30 rel_inf={err:.3e}")
    assert err <= TOL64
    # determinism: a second run is bitwise identical
    u2 = _host(plan.eval(_dev(c0.f)))
    assert np.array_equal(u, u2)
    plan.close()


def test_multipoles_and_locals_match_definitions(c0):
    """P2M/M2M are exact up to rounding; the downward pass reproduces the local
    expansion of each leaf's far sources within the truncation error."""
    vp = _vp()
    p = 30
    plan = vp.Plan(c0.x, c0.y, c0.w, order=p, root=c0.root)
    plan.eval(_dev(c0.f))
    M = plan.get_array("multipole").reshape(-1, 2 * (p + 1))
    L = plan.get_array("local").reshape(-1, 2 * (p + 1))
    tr = OT.build_tree(c0.x, c0.y, root=c0.root, max_leaf=64)
    z = (c0.x + 1j * c0.y)[tr.src_perm]
    q = (c0.w * c0.f[0])[tr.src_perm]
    worst = 0.0
    for b in range(tr.level_begin[2], tr.nbox, 7):
        cx, cy, h = OT.box_center(tr, b)
        sl = slice(tr.src_begin[b], tr.src_end[b])
        A = OE.multipole(z[sl], q[sl], cx + 1j * cy, h, p)[0]
        got = M[b, :p + 1] + 1j * M[b, p + 1:]
        worst = max(worst, np.max(np.abs(got - A)) / np.max(np.abs(A)))
    assert worst <= 1e-13, worst
    # locals of leaves vs far-source definition, compared as potentials at the leaf's nodes
    lists = OT.all_lists(tr)
    leaves = np.nonzero(tr.leaf)[0]
    worst = 0.0
    for b in leaves[::11]:
        up, ui = lists["U"]
        near = np.zeros(c0.n, dtype=bool)
        for a in ui[up[b]:up[b + 1]]:
            near[tr.src_begin[a]:tr.src_end[a]] = True
        far = ~near
        cx, cy, h = OT.box_center(tr, b)
        zt = z[tr.src_begin[b]:tr.src_end[b]]
        ref = direct.smooth(z.real[far], z.imag[far], np.ones(far.sum()), q[far][None, :], zt.real, zt.imag)[0]
        Bg = L[b, :p + 1] + 1j * L[b, p + 1:]
        got = OE.eval_local(Bg, cx + 1j * cy, h, zt)[0]
        worst = max(worst, np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    assert worst <= 1e-12, worst
    plan.close()


@pytest.mark.parametrize("targets", [False, True])
def test_eval_adaptive_tree(targets):
    vp = _vp()
    x, y, w, f, rng = _clustered(3)
    tx = ty = None
    if targets:
        t = rng.uniform(-1, 1, (700, 2))
        tx, ty = t[:, 0].copy(), t[:, 1].copy()
    plan = vp.Plan(x, y, w, tx, ty, order=30, max_leaf=32, root=(-1.0, -1.0, 2.0))
    info = plan.info()
    assert info["list_len"][2] > 0 and info["list_len"][3] > 0  # W and X lists in use
    u = _host(plan.eval(_dev(f)))
    ref = direct.smooth(x, y, w, f, tx, ty)
    err = relinf(u, ref)
    print(f"adaptive targets={targets} rel_inf={err:.3e} W={info['list_len'][2]} X={info['list_len'][3]}")
    assert err <= TOL64
    plan.close()


def test_adaptive_tree_sixteen_densities():
    """An adaptive tree with 16 densities: the matrix-core M2M takes one
    parent's 16 densities per wave, and parents with fewer than four
    children read the multipole array's zero block for the absent ones;
    the M2L's absent sources read the same block.  Forward and adjoint
    against the oracle, every density."""
    vp = _vp()
    x, y, w, _, rng = _clustered(11)
    f = rng.standard_normal((16, x.shape[0]))
    plan = vp.Plan(x, y, w, order=30, max_leaf=32, nbatch=16, root=(-1.0, -1.0, 2.0))
    info = plan.info()
    assert info["list_len"][2] > 0 and info["list_len"][3] > 0  # W and X lists in use
    u = _host(plan.eval(_dev(f)))
    ref = direct.smooth(x, y, w, f)
    err = max(relinf(u[b], ref[b]) for b in range(16))
    g = rng.standard_normal((16, x.shape[0]))
    d = _host(plan.eval_adjoint(_dev(g)))
    dref = direct.smooth_adjoint(x, y, w, g)
    aerr = max(relinf(d[b], dref[b]) for b in range(16))
    print(f"adaptive tree, 16 densities: rel_inf {err:.3e}, adjoint {aerr:.3e}")
    assert err <= TOL64
    assert aerr <= TOL64
    plan.close()


def test_adjoint_config0(c0):
    vp = _vp()
    plan = vp.Plan(c0.x, c0.y, c0.w, rowptr=c0.rowptr, col=c0.col, val=c0.val, order=30, root=c0.root)
    g = np.random.default_rng(5).standard_normal((1, c0.n))
    d = _host(plan.eval_adjoint(_dev(g)))
    ref = direct.evaluate_adjoint(c0.x, c0.y, c0.w, g, c0.rowptr, c0.col, c0.val)
    err = relinf(d, ref)
    print(f"adjoint rel_inf={err:.3e}")
    assert err <= TOL64
    u = _host(plan.eval(_dev(c0.f)))
    lhs, rhs = float(np.dot(g[0], u[0])), float(np.dot(d[0], c0.f[0]))
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(g[0]) @ np.abs(u[0]))
    plan.close()


def test_adjoint_separate_targets():
    vp = _vp()
    x, y, w, f, rng = _clustered(4)
    t = rng.uniform(-1, 1, (500, 2))
    plan = vp.Plan(x, y, w, t[:, 0].copy(), t[:, 1].copy(), order=30, max_leaf=32, root=(-1.0, -1.0, 2.0))
    g = rng.standard_normal((1, 500))
    d = _host(plan.eval_adjoint(_dev(g)))
    ref = direct.smooth_adjoint(x, y, w, g, t[:, 0], t[:, 1])
    assert relinf(d, ref) <= TOL64
    plan.close()


def test_grad_targets():
    vp = _vp()
    x, y, w = gen.uniform_grid(16)
    f, _ = gen.gaussian_sum_density(x, y, 41)
    rng = np.random.default_rng(43)
    t = rng.uniform(-0.95, 0.95, (512, 2))
    plan = vp.Plan(x, y, w, t[:, 0].copy(), t[:, 1].copy(), order=30, root=(-1.0, -1.0, 2.0))
    gr = _host(plan.eval_grad_targets(_dev(f[None, :])))
    ref = direct.smooth_grad(x, y, w, f, t[:, 0], t[:, 1])
    err = relinf(gr, ref)
    print(f"grad rel_inf={err:.3e}")
    assert err <= TOL64
    plan.close()


@pytest.mark.parametrize("nbatch", [3, 5])
def test_batched_densities(c0, nbatch):
    """Several densities in one evaluation (5: the near tables and the cell
    correction take their several-density forms)."""
    vp = _vp()
    fs = np.stack([gen.gaussian_sum_density(c0.x, c0.y, s)[0] for s in range(30, 30 + nbatch)])
    plan = vp.Plan(c0.x, c0.y, c0.w, rowptr=c0.rowptr, col=c0.col, val=c0.val, order=30, nbatch=nbatch,
                   root=c0.root)
    u = _host(plan.eval(_dev(fs)))
    ref = direct.evaluate(c0.x, c0.y, c0.w, fs, c0.rowptr, c0.col, c0.val)
    for b in range(nbatch):
        assert relinf(u[b], ref[b]) <= TOL64
    g = np.random.default_rng(8).standard_normal((nbatch, c0.n))
    d = _host(plan.eval_adjoint(_dev(g)))
    dref = direct.evaluate_adjoint(c0.x, c0.y, c0.w, g, c0.rowptr, c0.col, c0.val)
    for b in range(nbatch):
        assert relinf(d[b], dref[b]) <= TOL64
    plan.close()


@pytest.mark.parametrize("mode", ["fp32", "split", "fp64", "fp32_scaled", "fp64_scaled"])
def test_fp32_bulk_form(c0, mode):
    vp = _vp()
    plan = vp.Plan(c0.x, c0.y, c0.w, rowptr=c0.rowptr, col=c0.col, val=c0.val, order=14, precision="fp32",
                   m2l_mode=mode, root=c0.root)
    u = _host(plan.eval(_dev(c0.f)))
    ref = direct.evaluate(c0.x, c0.y, c0.w, c0.f, c0.rowptr, c0.col, c0.val)
    err = relinf(u, ref)
    print(f"fp32-bulk m2l={mode} p=14 rel_inf={err:.3e}")
    assert err <= TOL32
    plan.close()


@pytest.mark.parametrize("order", [1, 4, 15, 16, 30, 47, 60])
def test_every_order_matches_truncated_fmm_oracle(c0, order):
    """At every expansion order the plan accepts (1..60; here the two ends
    and the orders where the padded column size changes: 16, 32, 48, 64 rows,
    with extra padding rows at orders 4 and 16), both M2L forms give what an
    order-p FMM computes by definition on this uniform tree
    (oracle.fmm_truncated: direct near field plus the truncated Taylor
    coefficients of every V-list box's truncated multipole field), to
    rounding; at p >= 30 that is also the direct sum to 1e-12."""
    from oracle import fmm_truncated as FT
    vp = _vp()
    ref_p = FT.evaluate_uniform(c0.x, c0.y, c0.w, c0.f, c0.root, 64, order)
    res = []
    for mode, waves in (("fp64", 0), ("fp64_scaled", 0), ("fp64_scaled", 1)):
        plan = vp.Plan(c0.x, c0.y, c0.w, order=order, m2l_mode=mode, root=c0.root, m2l_waves=waves)
        u = _host(plan.eval(_dev(c0.f)))
        res.append((plan.get_array("local"), u))
        err = relinf(u, ref_p)
        print(f"order {order} m2l={mode} waves={waves or 4}: vs order-p FMM oracle {err:.2e}")
        assert err <= 1e-13
        plan.close()
    (l1, u1), (l2, u2), (l3, u3) = res
    assert relinf(l2, l1) <= 1e-13 and relinf(l3, l1) <= 1e-13
    assert relinf(u2, u1) <= 1e-13 and relinf(u3, u1) <= 1e-13
    if order >= 30:
        ref = direct.smooth(c0.x, c0.y, c0.w, c0.f)
        assert relinf(u2, ref) <= TOL64


@pytest.mark.parametrize("precision,order,tol", [("fp64", 30, TOL64), ("fp32", 14, TOL32)])
def test_autotuned_m2l(c0, precision, order, tol):
    """The plan-time autotuner picks a valid M2L kernel form, waves per tile
    and stream mode for the precision; the evaluation still meets the oracle
    tolerance, and a second plan of the same geometry takes the cached
    choices without timing."""
    vp = _vp()
    ref = direct.evaluate(c0.x, c0.y, c0.w, c0.f, c0.rowptr, c0.col, c0.val)
    infos = []
    for _ in range(2):
        plan = vp.Plan(c0.x, c0.y, c0.w, rowptr=c0.rowptr, col=c0.col, val=c0.val, order=order,
                       precision=precision, autotune=True, root=c0.root)
        info = plan.info()
        infos.append(info)
        assert info["m2l_mode"] in ((4, 1) if precision == "fp64" else (5, 2, 3, 4)), info["m2l_mode"]
        assert info["m2l_waves"] in (1, 2, 4) and info["table_waves"] in (1, 2, 4) and info["one_stream"] in (0, 1)
        u = _host(plan.eval(_dev(c0.f)))
        err = relinf(u, ref)
        print(f"autotuned {precision}: m2l mode {info['m2l_mode']}, waves {info['m2l_waves']}/"
              f"{info['table_waves']}, one stream {info['one_stream']}, tuned {info['tuned']} "
              f"({info['tune_ms']:.0f} ms), rel_inf={err:.3e}")
        assert err <= tol
        plan.close()
    assert infos[1]["tuned"] == 2
    for k in ("m2l_mode", "m2l_waves", "table_waves", "one_stream"):
        assert infos[0][k] == infos[1][k]


@pytest.mark.parametrize("precision,order,tol", [("fp64", 30, TOL64), ("fp32", 14, TOL32)])
def test_two_waves_per_tile(c0, precision, order, tol):
    """The two-wave and one-wave variants of the M2L and near-table kernels
    (the autotuner's other choices: two waves sharing a tile; one wave per
    M2L tile, four tiles per workgroup; one near-table wave over two tiles)
    against the oracle and the four-wave default."""
    vp = _vp()
    ref = direct.evaluate(c0.x, c0.y, c0.w, c0.f, c0.rowptr, c0.col, c0.val)
    out = {}
    for waves in (4, 2, 1):
        for mode in (("fp64_scaled", "fp64") if precision == "fp64" else ("fp32_scaled", "split")):
            plan = vp.Plan(c0.x, c0.y, c0.w, rowptr=c0.rowptr, col=c0.col, val=c0.val, order=order,
                           precision=precision, m2l_mode=mode, m2l_waves=waves, table_waves=waves, root=c0.root)
            assert plan.info()["m2l_waves"] == waves and plan.info()["table_waves"] == waves
            out[(waves, mode)] = u = _host(plan.eval(_dev(c0.f)))
            err = relinf(u, ref)
            print(f"{precision} {mode} {waves} waves: rel_inf={err:.3e}")
            assert err <= tol
            plan.close()
    for mode in {m for _, m in out}:
        for waves in (2, 1):
            assert relinf(out[(waves, mode)], out[(4, mode)]) <= (1e-14 if precision == "fp64" else 1e-7)


def test_autotuned_leaf_size(c0):
    """VP_FLAG_AUTOTUNE_LEAF builds the plan with 64- and 16-point leaves and
    keeps the faster one; either meets the oracle tolerance."""
    vp = _vp()
    plan = vp.Plan(c0.x, c0.y, c0.w, rowptr=c0.rowptr, col=c0.col, val=c0.val, order=30, autotune=True,
                   autotune_leaf=True, root=c0.root)
    info = plan.info()
    assert info["max_leaf"] in (64, 16) and info["tuned"] in (1, 2)
    u = _host(plan.eval(_dev(c0.f)))
    err = relinf(u, direct.evaluate(c0.x, c0.y, c0.w, c0.f, c0.rowptr, c0.col, c0.val))
    print(f"leaf autotune: max_leaf {info['max_leaf']}, rel_inf={err:.3e}")
    assert err <= TOL64
    plan.close()
    # 16-point leaves forced: the 8x8 box rule splits into congruent 4x4 quadrants
    plan = vp.Plan(c0.x, c0.y, c0.w, rowptr=c0.rowptr, col=c0.col, val=c0.val, order=30, max_leaf=16, root=c0.root)
    info = plan.info()
    u = _host(plan.eval(_dev(c0.f)))
    err = relinf(u, direct.evaluate(c0.x, c0.y, c0.w, c0.f, c0.rowptr, c0.col, c0.val))
    print(f"16-point leaves: p2p mode {info['p2p_mode_used']}, table leaves {info['table_leaves']}, rel_inf={err:.3e}")
    assert err <= TOL64
    plan.close()


@pytest.mark.parametrize("precision,order", [("fp64", 30), ("fp32", 14)])
def test_one_stream_matches_two_streams(c0, precision, order):
    """VP_FLAG_ONE_STREAM runs the correction and the near field on the plan's
    stream in sequence; every kernel computes the same sums in the same
    order, so forward and adjoint results are bitwise identical to the
    overlapped default, and both meet the oracle tolerance."""
    vp = _vp()
    out = []
    for one in (False, True):
        plan = vp.Plan(c0.x, c0.y, c0.w, rowptr=c0.rowptr, col=c0.col, val=c0.val, order=order,
                       precision=precision, one_stream=one, root=c0.root)
        out.append((_host(plan.eval(_dev(c0.f))), _host(plan.eval_adjoint(_dev(c0.f)))))
        plan.close()
    (u2, a2), (u1, a1) = out
    assert np.array_equal(u1, u2)
    assert np.array_equal(a1, a2)
    ref = direct.evaluate(c0.x, c0.y, c0.w, c0.f, c0.rowptr, c0.col, c0.val)
    assert relinf(u1, ref) <= (TOL64 if precision == "fp64" else TOL32)


@pytest.mark.parametrize("nbatch", [1, 2, 3, 5])
def test_correction_general_csr(nbatch):
    """A correction matrix that is not run-structured: rows of 0 to 150 entries
    (empty rows, rows longer than one 64-entry pass), unsorted random
    columns, with separate targets; forward and adjoint against the oracle."""
    vp = _vp()
    rng = np.random.default_rng(11 + nbatch)
    n, m = 900, 700
    x = rng.uniform(-1, 1, n)
    y = rng.uniform(-1, 1, n)
    w = rng.uniform(0.1, 1, n) / n
    tx = rng.uniform(-1, 1, m)
    ty = rng.uniform(-1, 1, m)
    lens = rng.integers(0, 151, m)
    lens[::7] = 0
    rowptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = rng.integers(0, n, int(rowptr[-1])).astype(np.int32)
    val = rng.standard_normal(int(rowptr[-1]))
    f = rng.standard_normal((nbatch, n))
    plan = vp.Plan(x, y, w, tx, ty, rowptr, col, val, order=30, max_leaf=32, nbatch=nbatch, root=(-1.0, -1.0, 2.0))
    assert plan.info()["corr_cells"] == 0  # not run-structured: the row kernel applies C
    u = _host(plan.eval(_dev(f)))
    ref = direct.evaluate(x, y, w, f, rowptr, col, val, tx, ty)
    assert max(relinf(u[b], ref[b]) for b in range(nbatch)) <= TOL64
    g = rng.standard_normal((nbatch, m))
    d = _host(plan.eval_adjoint(_dev(g)))
    dref = direct.evaluate_adjoint(x, y, w, g, rowptr, col, val, tx, ty)
    assert max(relinf(d[b], dref[b]) for b in range(nbatch)) <= TOL64
    plan.close()


@pytest.mark.parametrize("nbatch", [1, 3, 16])
def test_correction_cells(nbatch):
    """A block-diagonal correction (cells of 1 to 64 nodes, each row's columns
    its own cell's nodes, plus a few empty rows), which the plan applies
    cell by cell in both directions; forward and adjoint against the oracle."""
    vp = _vp()
    rng = np.random.default_rng(31 + nbatch)
    sizes = rng.integers(1, 65, 40)
    n = int(sizes.sum())
    x = rng.uniform(-1, 1, n)
    y = rng.uniform(-1, 1, n)
    w = rng.uniform(0.1, 1, n) / n
    lens, cols, start = [], [], 0
    for k, sz in enumerate(sizes):
        empty = k % 9 == 4  # a cell whose rows have no entries
        for _ in range(sz):
            lens.append(0 if empty else sz)
            if not empty:
                cols.extend(range(start, start + sz))
        start += sz
    rowptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.asarray(cols, dtype=np.int32)
    val = rng.standard_normal(col.size)
    f = rng.standard_normal((nbatch, n))
    plan = vp.Plan(x, y, w, rowptr=rowptr, col=col, val=val, order=30, max_leaf=32, nbatch=nbatch,
                   root=(-1.0, -1.0, 2.0))
    assert plan.info()["corr_cells"] == len(sizes)  # the cell kernel applies C
    u = _host(plan.eval(_dev(f)))
    ref = direct.evaluate(x, y, w, f, rowptr, col, val)
    assert max(relinf(u[b], ref[b]) for b in range(nbatch)) <= TOL64
    g = rng.standard_normal((nbatch, n))
    d = _host(plan.eval_adjoint(_dev(g)))
    dref = direct.evaluate_adjoint(x, y, w, g, rowptr, col, val)
    assert max(relinf(d[b], dref[b]) for b in range(nbatch)) <= TOL64
    plan.close()


@pytest.mark.parametrize("nbatch", [1, 4, 16])
def test_correction_shared_blocks(nbatch):
    """Cells whose value blocks repeat (the box corrections of one box size are
    one table, Section 4): a cell with a block identical bit for bit to an
    earlier cell's reads that cell's copy, also from an odd value offset onto
    an even one; a block that differs in one bit of one value keeps its own.
    One density (grouped apply and two-rows-per-load path), 4 (matrix cores) and 16; forward and
    adjoint against the oracle."""
    vp = _vp()
    rng = np.random.default_rng(97 + nbatch)
    blocks = {k: rng.standard_normal(sz * sz) for k, sz in ((0, 64), (1, 64), (2, 45))}
    near = blocks[0].copy()
    near[1000] = np.nextafter(near[1000], np.inf)  # one bit away from block 0
    blocks[3] = near
    # (nodes, block) of each square cell, in order; the 45-node cells move the
    # values after them to odd offsets
    # with one density, block 1's 21 cells go to the grouped matrix-core apply
    # (a full group of 16 and one of 5), the others stay cell by cell
    order = [(64, 0), (64, 0), (64, 1), (64, 3), (45, 2), (64, 0), (64, 1), (45, 2), (30, None)]
    order += [(64, 1)] * 10 + [(45, None)] + [(64, 1)] * 9
    n = sum(sz for sz, _ in order)
    x = rng.uniform(-1, 1, n)
    y = rng.uniform(-1, 1, n)
    w = rng.uniform(0.1, 1, n) / n
    lens, cols, vals, start = [], [], [], 0
    for sz, b in order:
        for _ in range(sz):
            lens.append(sz)
            cols.extend(range(start, start + sz))
        vals.append(blocks[b] if b is not None else rng.standard_normal(sz * sz))
        start += sz
    rowptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.asarray(cols, dtype=np.int32)
    val = np.concatenate(vals)
    f = rng.standard_normal((nbatch, n))
    plan = vp.Plan(x, y, w, rowptr=rowptr, col=col, val=val, order=30, max_leaf=32, nbatch=nbatch,
                   root=(-1.0, -1.0, 2.0))
    info = plan.info()
    assert info["corr_cells"] == len(order)
    assert info["corr_shared_cells"] == 23  # 2 of block 0, 20 of block 1, 1 of block 2
    assert info["corr_groups"] == (2 if nbatch == 1 else 0)  # block 1's 21 cells: 16 + 5
    assert info["corr_values_read"] == val.size - 22 * 64 * 64 - 45 * 45
    u = _host(plan.eval(_dev(f)))
    ref = direct.evaluate(x, y, w, f, rowptr, col, val)
    assert max(relinf(u[b], ref[b]) for b in range(nbatch)) <= TOL64
    g = rng.standard_normal((nbatch, n))
    d = _host(plan.eval_adjoint(_dev(g)))
    dref = direct.evaluate_adjoint(x, y, w, g, rowptr, col, val)
    assert max(relinf(d[b], dref[b]) for b in range(nbatch)) <= TOL64
    plan.close()


@pytest.mark.parametrize("nbatch", [1, 2])
def test_correction_cells_64_columns(nbatch):
    """Cells of 64 columns, the two-rows-per-load path of the cell apply
    (one density, values 16-byte aligned; one such cell has only 20 rows, a
    partial batch of 16), next to cells where it does not apply: a 45-node
    cell shifts the later cells' values to odd offsets.  Forward and adjoint
    against the oracle."""
    vp = _vp()
    rng = np.random.default_rng(71 + nbatch)
    # (first row, rows, first column, columns) of each cell, in row order;
    # values start at even offsets up to the 45-node cell, at odd ones after it
    cells = []
    start = 0
    for sz in (64, 64):
        cells.append((start, sz, start, sz))
        start += sz
    cells.append((start, 20, start, 64))  # 20 rows over 64 columns
    cells.append((start + 20, 44, start + 20, 44))
    start += 64
    for sz in (45, 64, 64):
        cells.append((start, sz, start, sz))
        start += sz
    n = start
    x = rng.uniform(-1, 1, n)
    y = rng.uniform(-1, 1, n)
    w = rng.uniform(0.1, 1, n) / n
    lens, cols = [], []
    for r0, nr, c0, nc in cells:
        for _ in range(nr):
            lens.append(nc)
            cols.extend(range(c0, c0 + nc))
    rowptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    col = np.asarray(cols, dtype=np.int32)
    val = rng.standard_normal(col.size)
    f = rng.standard_normal((nbatch, n))
    plan = vp.Plan(x, y, w, rowptr=rowptr, col=col, val=val, order=30, max_leaf=32, nbatch=nbatch,
                   root=(-1.0, -1.0, 2.0))
    assert plan.info()["corr_cells"] == len(cells)
    u = _host(plan.eval(_dev(f)))
    ref = direct.evaluate(x, y, w, f, rowptr, col, val)
    assert max(relinf(u[b], ref[b]) for b in range(nbatch)) <= TOL64
    g = rng.standard_normal((nbatch, n))
    d = _host(plan.eval_adjoint(_dev(g)))
    dref = direct.evaluate_adjoint(x, y, w, g, rowptr, col, val)
    assert max(relinf(d[b], dref[b]) for b in range(nbatch)) <= TOL64
    plan.close()


@pytest.mark.parametrize("n", [1, 2, 5, 63, 64, 65])
def test_small_inputs(n):
    vp = _vp()
    rng = np.random.default_rng(n)
    x = rng.uniform(-1, 1, n)
    y = rng.uniform(-1, 1, n)
    w = rng.uniform(0.1, 1, n)
    f = rng.standard_normal((1, n))
    plan = vp.Plan(x, y, w, order=20)
    u = _host(plan.eval(_dev(f)))
    ref = direct.smooth(x, y, w, f)
    if n == 1:
        assert np.all(u == 0.0)
    else:
        assert relinf(u, ref) <= TOL64
    plan.close()


def test_duplicate_points_and_deep_tree():
    """Coincident nodes: zero-distance pairs contribute nothing; the tree stops at max_level."""
    vp = _vp()
    rng = np.random.default_rng(9)
    x = rng.uniform(-1, 1, 300)
    y = rng.uniform(-1, 1, 300)
    x[100:110] = x[5]
    y[100:110] = y[5]
    w = rng.uniform(0.1, 1, 300)
    f = rng.standard_normal((1, 300))
    plan = vp.Plan(x, y, w, order=30, max_leaf=4, max_level=12)
    u = _host(plan.eval(_dev(f)))
    ref = direct.smooth(x, y, w, f)
    assert relinf(u, ref) <= TOL64
    plan.close()


def test_targets_on_nodes():
    """Separate targets placed exactly on source nodes: the zero-distance pair
    contributes nothing (the pairwise logarithm returns exactly 0 there), in
    the forward and the adjoint evaluation and for several densities."""
    vp = _vp()
    x, y, w, f, rng = _clustered(12)
    n = x.size
    on = rng.choice(n, 300, replace=False)
    t = np.concatenate([np.stack([x[on], y[on]], 1), rng.uniform(-1, 1, (200, 2))])
    tx, ty = t[:, 0].copy(), t[:, 1].copy()
    fs = np.concatenate([f, rng.standard_normal((2, n))])
    plan = vp.Plan(x, y, w, tx, ty, order=30, max_leaf=32, nbatch=3, root=(-1.0, -1.0, 2.0))
    u = _host(plan.eval(_dev(fs)))
    ref = direct.smooth(x, y, w, fs, tx, ty)
    assert np.all(np.isfinite(u))
    assert max(relinf(u[b], ref[b]) for b in range(3)) <= TOL64
    g = rng.standard_normal((3, t.shape[0]))
    d = _host(plan.eval_adjoint(_dev(g)))
    dref = direct.smooth_adjoint(x, y, w, g, tx, ty)
    assert max(relinf(d[b], dref[b]) for b in range(3)) <= TOL64
    plan.close()


# ---------------------------------------------------------------------------
# congruent-leaf path (near-field tables, pattern P2M/L2P) vs pairwise path
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision,order,tol", [("fp64", 30, TOL64), ("fp32", 14, TOL32)])
def test_tables_match_pairwise_and_oracle(c0, precision, order, tol):
    vp = _vp()
    ref = direct.evaluate(c0.x, c0.y, c0.w, c0.f, c0.rowptr, c0.col, c0.val)
    out = {}
    for mode in ("tables", "pairwise"):
        plan = vp.Plan(c0.x, c0.y, c0.w, rowptr=c0.rowptr, col=c0.col, val=c0.val, order=order,
                       precision=precision, p2p_mode=mode, root=c0.root)
        info = plan.info()
        assert info["p2p_mode_used"] == (2 if mode == "tables" else 1)
        if mode == "tables":
            assert info["table_leaves"] == 256 and info["near_pairs"] == 0
        u = _host(plan.eval(_dev(c0.f)))
        err = relinf(u, ref)
        print(f"{precision} p={order} {mode}: rel_inf={err:.3e}")
        assert err <= tol
        out[mode] = u
        g = np.random.default_rng(6).standard_normal((1, c0.n))
        d = _host(plan.eval_adjoint(_dev(g)))
        dref = direct.evaluate_adjoint(c0.x, c0.y, c0.w, g, c0.rowptr, c0.col, c0.val)
        assert relinf(d, dref) <= tol
        plan.close()
    if precision == "fp64":
        assert relinf(out["tables"], out["pairwise"]) <= 1e-13


def test_tables_on_adaptive_star_subset():
    """Pattern leaves at several levels next to non-pattern (triangle) leaves."""
    vp = _vp()
    wl = gen.config1()
    # keep a window of the domain so the oracle stays cheap
    keep = (np.abs(wl.x - 0.9) < 0.25) & (np.abs(wl.y) < 0.25)
    x, y, w, f = wl.x[keep], wl.y[keep], wl.w[keep], wl.f[:, keep]
    plan = vp.Plan(x, y, w, order=30, root=wl.root)
    info = plan.info()
    assert info["p2p_mode_used"] == 2 and info["table_leaves"] > 0 and info["near_pairs"] > 0
    u = _host(plan.eval(_dev(f)))
    ref = direct.smooth(x, y, w, f)
    err = relinf(u, ref)
    print(f"star window n={x.size} table_leaves={info['table_leaves']} rel_inf={err:.3e}")
    assert err <= TOL64
    plan.close()


def test_tables_match_pairwise_with_x_lists():
    """An adaptive window with X lists (leaves next to finer leaves): the
    congruent-leaf path (near tables, pattern P2M/L2P and the quadrant
    matrices for the virtual children of pattern X-list sources) against the
    general path (pairwise near field, VALU P2M of every quadrant)."""
    vp = _vp()
    wl = gen.config1()
    keep = (np.abs(wl.x - 0.9) < 0.25) & (np.abs(wl.y) < 0.25)
    x, y, w, f = wl.x[keep], wl.y[keep], wl.w[keep], wl.f[:, keep]
    out = {}
    for mode in ("tables", "pairwise"):
        plan = vp.Plan(x, y, w, order=30, p2p_mode=mode, root=wl.root)
        info = plan.info()
        assert info["list_len"][3] > 0
        out[mode] = _host(plan.eval(_dev(f)))
        plan.close()
    d = relinf(out["tables"], out["pairwise"])
    print(f"star window: tables vs pairwise {d:.2e}")
    assert d <= 1e-13


@pytest.mark.parametrize("case", ["c0_1", "c0_3", "c0_251_leaves", "star_window"])
def test_one_wave_tables(c0, case):
    """The one-wave near-table kernel (one operator load for two 16-column
    tiles) against the four-wave kernel and the oracle, forward and adjoint:
    one density (charges one density per row) and three (density-fastest
    charges, tiles straddling leaves), 251 table leaves with two densities
    (five leaves moved off the node pattern: the last 32-column group is
    ragged), and an adaptive window whose table leaves sit on several levels."""
    vp = _vp()
    if case == "c0_251_leaves":
        x, y = c0.x.copy(), c0.y.copy()
        rng = np.random.default_rng(78)
        for b in (3, 60, 128, 199, 250):
            sl = slice(64 * b, 64 * b + 64)
            x[sl] += 4e-13 * (2.0 / 16) * rng.choice([-1.0, 1.0], 64)
            y[sl] += 4e-13 * (2.0 / 16) * rng.choice([-1.0, 1.0], 64)
        w = c0.w
        f = np.stack([gen.gaussian_sum_density(x, y, s)[0] for s in (60, 61)])
        rowptr, col, val, root = c0.rowptr, c0.col, c0.val, c0.root
    elif case == "star_window":
        wl = gen.config1()
        keep = (np.abs(wl.x - 0.9) < 0.25) & (np.abs(wl.y) < 0.25)
        x, y, w, f = wl.x[keep], wl.y[keep], wl.w[keep], wl.f[:, keep]
        rowptr = col = val = None
        root = wl.root
    else:
        nb = int(case.split("_")[1])
        x, y, w = c0.x, c0.y, c0.w
        f = np.stack([gen.gaussian_sum_density(x, y, s)[0] for s in range(50, 50 + nb)])
        rowptr, col, val, root = c0.rowptr, c0.col, c0.val, c0.root
    out, adj = {}, {}
    g = np.random.default_rng(79).standard_normal(f.shape)
    for tw in (4, 1):
        plan = vp.Plan(x, y, w, rowptr=rowptr, col=col, val=val, order=30, nbatch=f.shape[0], root=root,
                       table_waves=tw)
        info = plan.info()
        assert info["table_waves"] == tw and info["p2p_mode_used"] == 2
        if case == "c0_251_leaves":
            assert info["table_leaves"] == 251
        out[tw] = _host(plan.eval(_dev(f)))
        adj[tw] = _host(plan.eval_adjoint(_dev(g)))
        plan.close()
    ref = direct.evaluate(x, y, w, f, rowptr, col, val) if rowptr is not None else direct.smooth(x, y, w, f)
    err = relinf(out[1], ref)
    d = relinf(out[1], out[4])
    da = relinf(adj[1], adj[4])
    print(f"one-wave tables {case}: rel_inf={err:.3e}, vs four waves {d:.2e} (adjoint {da:.2e})")
    assert err <= TOL64
    assert d <= 1e-14 and da <= 1e-14


@pytest.mark.parametrize("nbatch", [16, 32])
def test_l2p_from_parents(c0, nbatch):
    """With 16k densities on a uniform grid the deepest level's pattern leaves
    take their far field from the parents' local expansions (the L2L into
    that level folded into the L2P matrices): forward against the oracle,
    and the adjoint (which keeps the plain L2L) on the same plan."""
    vp = _vp()
    fs = np.stack([gen.gaussian_sum_density(c0.x, c0.y, s)[0] for s in range(70, 70 + nbatch)])
    plan = vp.Plan(c0.x, c0.y, c0.w, rowptr=c0.rowptr, col=c0.col, val=c0.val, order=30, nbatch=nbatch,
                   root=c0.root)
    assert plan.info()["l2p_from_parents"] == 1
    u = _host(plan.eval(_dev(fs)))
    ref = direct.evaluate(c0.x, c0.y, c0.w, fs, c0.rowptr, c0.col, c0.val)
    errs = [relinf(u[b], ref[b]) for b in range(nbatch)]
    print(f"l2p from parents, {nbatch} densities: max rel_inf {max(errs):.3e}")
    assert max(errs) <= TOL64
    g = np.random.default_rng(71).standard_normal((nbatch, c0.n))
    d = _host(plan.eval_adjoint(_dev(g)))
    dref = direct.evaluate_adjoint(c0.x, c0.y, c0.w, g, c0.rowptr, c0.col, c0.val)
    assert max(relinf(d[b], dref[b]) for b in range(nbatch)) <= TOL64
    # forward evaluations write only the density-fastest charges here; the
    # target gradients (pairwise near field) need the other copy, and the next
    # forward evaluation goes back to one copy
    idx = gen.sample_indices(c0.n, 512, 72)
    gr = _host(plan.eval_grad_targets(_dev(fs)))
    gref = direct.smooth_grad(c0.x, c0.y, c0.w, fs, tidx=idx)
    gerr = relinf(gr[:, :, idx], gref)
    print(f"target gradients after a one-copy forward evaluation: rel_inf {gerr:.3e}")
    assert gerr <= TOL64
    assert np.array_equal(_host(plan.eval(_dev(fs))), u)
    plan.close()
    # one density: the plain path
    p1 = vp.Plan(c0.x, c0.y, c0.w, rowptr=c0.rowptr, col=c0.col, val=c0.val, order=30, root=c0.root)
    assert p1.info()["l2p_from_parents"] == 0
    p1.close()


@pytest.mark.parametrize("case", ["shared", "shared_3_densities", "shared_fp32", "reordered_box", "per_entry"])
def test_corrections_folded_into_tables(c0, case):
    """Own-cell corrections that are one shared block on congruent leaves
    (Section 4: the correction depends on the box shape only) are folded into
    the near tables' self slot for forward evaluations.  The fold is declined
    when one box lists its nodes in another order (its rows and columns of the
    shared block meet the nodes in another order) or when the values differ
    per cell.  Forward and adjoint against the oracle either way."""
    vp = _vp()
    nb = 3 if case == "shared_3_densities" else 16
    fp32 = case == "shared_fp32"
    x, y, w, val = c0.x.copy(), c0.y.copy(), c0.w.copy(), c0.val
    if case == "reordered_box":
        sl = slice(64 * 37, 64 * 38)
        p = np.random.default_rng(81).permutation(64)
        x[sl], y[sl], w[sl] = x[sl][p], y[sl][p], w[sl][p]
    elif case == "per_entry":
        val = c0.val + 1e-3 * np.random.default_rng(82).standard_normal(c0.val.shape)
    fs = np.stack([gen.gaussian_sum_density(x, y, s)[0] for s in range(90, 90 + nb)])
    # (one-wave tables: the density-fastest charge copy, which with 16 densities the
    # charge pass writes together with the leaf multipoles)
    plan = vp.Plan(x, y, w, rowptr=c0.rowptr, col=c0.col, val=val, order=14 if fp32 else 30, nbatch=nb,
                   precision="fp32" if fp32 else "fp64", root=c0.root, table_waves=1)
    info = plan.info()
    # (the finish from the parents' expansions: FP64 with a multiple of 16 densities)
    assert info["l2p_from_parents"] == (1 if nb == 16 and not fp32 else 0)
    assert info["corr_one_block"] == (0 if case == "per_entry" else 1)
    assert info["corr_folded"] == (1 if case.startswith("shared") else 0)
    plan.set_timing(True)
    u = _host(plan.eval(_dev(fs)))
    tim = plan.timing()["ms"]
    plan.set_timing(False)
    assert tim["corr"] == 0.0 if info["corr_folded"] else tim["corr"] > 0.0
    # leaf multipoles formed in the charge pass with 16 densities
    assert (tim["p2m_pat"] == 0.0) == (nb == 16) and tim["charge"] > 0.0
    ref = direct.evaluate(x, y, w, fs, c0.rowptr, c0.col, val)
    err = max(relinf(u[b], ref[b]) for b in range(nb))
    g = np.random.default_rng(83).standard_normal((nb, c0.n))
    d = _host(plan.eval_adjoint(_dev(g)))
    dref = direct.evaluate_adjoint(x, y, w, g, c0.rowptr, c0.col, val)
    derr = max(relinf(d[b], dref[b]) for b in range(nb))
    print(f"corrections {case}: folded={info['corr_folded']} forward rel_inf {err:.3e}, adjoint {derr:.3e}")
    tol = TOL32 if fp32 else TOL64
    assert err <= tol and derr <= tol
    # repeated forward evaluations agree bit for bit (u is written, not accumulated)
    assert np.array_equal(_host(plan.eval(_dev(fs))), u)
    plan.close()


@pytest.mark.parametrize("band", ["inside", "outside"])
def test_tables_with_nodes_off_pattern(c0, band):
    """Leaves whose nodes deviate from the node pattern.  The near-field
    tables take a leaf when its box-relative coordinates agree with the
    pattern to 8 units in the last place of the root square's coordinates
    (8 * 2^-52 * (R/h + 1) box units, R = 1, h = 1/8 here); the tables use the
    pattern's coordinates.  Inside that band (0.4 of it) the leaves stay on
    the tables and the result still meets the oracle at 1e-12; at 4e-13 box
    units (outside it) they go to the pairwise kernel, which uses their own
    coordinates."""
    vp = _vp()
    h = 2.0 / 16
    tol_box = 8 * 2.0 ** -52 * (1.0 / h + 1.0)
    delta = (0.4 * tol_box if band == "inside" else 4e-13) * h
    x, y = c0.x.copy(), c0.y.copy()
    rng = np.random.default_rng(77)
    moved = [5, 77, 130, 200, 255]  # user box numbers (box 0 is the first leaf in Morton order)
    for b in moved:
        sl = slice(64 * b, 64 * b + 64)
        x[sl] += delta * rng.choice([-1.0, 1.0], 64)
        y[sl] += delta * rng.choice([-1.0, 1.0], 64)
    plan = vp.Plan(x, y, c0.w, rowptr=c0.rowptr, col=c0.col, val=c0.val, order=30, root=c0.root)
    info = plan.info()
    assert info["p2p_mode_used"] == 2
    assert info["table_leaves"] == (256 if band == "inside" else 256 - len(moved))
    u = _host(plan.eval(_dev(c0.f)))
    ref = direct.evaluate(x, y, c0.w, c0.f, c0.rowptr, c0.col, c0.val)
    err = relinf(u, ref)
    print(f"nodes off pattern ({band}, {delta / h:.1e} box units): table leaves {info['table_leaves']}, "
          f"rel_inf={err:.3e}")
    assert err <= TOL64
    plan.close()
