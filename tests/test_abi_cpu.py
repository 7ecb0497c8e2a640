"""The C-ABI library loads, exports every symbol include/vp.h declares, and
rejects invalid arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2203_05933_amd import vp
    return vp, vp.load_library()


def test_exports_match_header():
    vp, lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "vp.h")).read()
    declared = set(re.findall(r"\b(vp_[a-z_]+)\s*\(", hdr))
    assert declared == set(vp.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_options_struct_layout():
    vp, lib = _lib()
    o = vp.default_options()
    assert (o.order, o.max_leaf, o.nbatch, o.precision) == (30, 64, 1, 0)
    assert ctypes.sizeof(vp.Options) == 8 * 4 + 3 * 8 + 8 + 4 + 4 + 8 + 4 + 4
    assert (o.kernel, o.lam) == (0, 0.0)


def _plan(lib, vp, x, y, w, n, tx=None, ty=None, m=None, rowptr=None, col=None, val=None, **opt):
    o = vp.default_options()
    for k, v in opt.items():
        setattr(o, k, v)
    h = ctypes.c_void_p()
    p = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    st = lib.vp_plan(p(x), p(y), p(w), n, p(tx), p(ty), n if m is None else m, p(rowptr), p(col), p(val),
                     ctypes.byref(o), ctypes.byref(h))
    return st, h, lib.vp_last_error(None).decode()


@pytest.mark.parametrize("case", ["n0", "nan", "m_mismatch", "rowptr0", "rowptr_dec", "col_range",
                                  "order", "nbatch", "leaf", "fp32_mode", "flags", "root_node",
                                  "root_target", "kernel", "lambda0", "lambda_nan", "tile_waves",
                                  "table_waves"])
def test_plan_rejects_invalid(case):
    vp, lib = _lib()
    x = np.linspace(0, 1, 8)
    y = np.linspace(0, 1, 8)[::-1].copy()
    w = np.ones(8)
    rowptr = np.arange(0, 17, 2, dtype=np.int64)
    col = np.zeros(16, dtype=np.int32)
    val = np.ones(16)
    kw = {}
    n = 8
    if case == "n0":
        n = 0
    elif case == "nan":
        x = x.copy(); x[3] = np.nan
    elif case == "rowptr0":
        rowptr = rowptr + 1
    elif case == "rowptr_dec":
        rowptr = rowptr.copy(); rowptr[4] = 1
    elif case == "col_range":
        col = col.copy(); col[5] = 8
    elif case == "order":
        kw["order"] = 0
    elif case == "nbatch":
        kw["nbatch"] = 65
    elif case == "leaf":
        kw["max_leaf"] = 0
    elif case == "fp32_mode":
        kw["m2l_mode"] = 2  # FP32 M2L with precision FP64
    elif case == "flags":
        kw["flags"] = 4  # unknown bit
    elif case == "kernel":
        kw["kernel"] = 2
    elif case == "tile_waves":
        kw["m2l_waves"] = 3
    elif case == "table_waves":
        kw["table_waves"] = 3
    elif case == "lambda0":
        kw["kernel"], kw["lam"] = 1, 0.0
    elif case == "lambda_nan":
        kw["kernel"], kw["lam"] = 1, float("nan")
    if case in ("root_node", "root_target"):
        # a given root square must hold every node and target: [0, 1]^2 holds
        # the nodes, and one point leaves it by one ulp
        o = vp.default_options()
        o.root[0], o.root[1], o.root[2] = 0.0, 0.0, 1.0
        tx, ty = x.copy(), y.copy()
        if case == "root_node":
            x = x.copy(); x[7] = np.nextafter(1.0, 2.0)
        else:
            ty[2] = np.nextafter(0.0, -1.0)
        kw["root"] = o.root
        st, h, msg = _plan(lib, vp, x, y, w, n, tx=tx, ty=ty, m=8, rowptr=rowptr, col=col, val=val, **kw)
        assert "outside the root square" in msg, msg
    elif case == "m_mismatch":
        st, h, msg = _plan(lib, vp, x, y, w, n, m=7, rowptr=rowptr, col=col, val=val)
    else:
        st, h, msg = _plan(lib, vp, x, y, w, n, rowptr=rowptr, col=col, val=val, **kw)
    assert st == vp.VP_EINVAL, (st, msg)
    assert h.value is None
    assert len(msg) > 0


def test_null_plan_calls():
    vp, lib = _lib()
    assert lib.vp_eval(None, None, None) == vp.VP_EINVAL
    assert lib.vp_eval_adjoint(None, None, None) == vp.VP_EINVAL
    assert lib.vp_eval_grad_targets(None, None, None) == vp.VP_EINVAL
    assert lib.vp_destroy(None) == vp.VP_OK
    assert lib.vp_set_stream(None, None) == vp.VP_EINVAL
    assert b"NULL" in lib.vp_last_error(None)


@pytest.mark.parametrize("case", ["null_os", "p_gt_q", "q_big", "no_targets", "in_overlap", "in_range",
                                  "out_cover", "out_overlap", "col_range"])
def test_plan_oversampled_rejects_invalid(case):
    """vp_plan_oversampled checks the box layout before touching a device."""
    from vp_workloads import generators as gen
    vp, lib = _lib()
    wl = gen.config5(nbox_side=2, csr_seed=3, sample_seed=None)
    p, q, nbox = 8, 16, wl.nbox
    ins = np.arange(nbox, dtype=np.int64) * p * p
    outs = np.arange(nbox, dtype=np.int64) * q * q
    n_in, n, m = wl.m, wl.n, wl.m
    tx, ty, col = wl.tx, wl.ty, wl.col.copy()
    pp, qq = p, q
    if case == "p_gt_q":
        pp, qq = 9, 8
    elif case == "q_big":
        qq = 33
    elif case == "no_targets":
        tx = ty = None
    elif case == "in_overlap":
        ins = ins.copy(); ins[1] = ins[0] + 1
    elif case == "in_range":
        ins = ins.copy(); ins[-1] = n_in - 1
    elif case == "out_cover":
        n = n - 1
    elif case == "out_overlap":
        outs = outs.copy(); outs[2] = outs[1]
    elif case == "col_range":
        col[5] = n_in
    os_ = vp.Oversampling(pp, qq, nbox, n_in, ins.ctypes.data, outs.ctypes.data)
    h = ctypes.c_void_p()
    ptr = lambda a: None if a is None else np.ascontiguousarray(a).ctypes.data_as(ctypes.c_void_p)
    o = vp.default_options()
    st = lib.vp_plan_oversampled(ptr(wl.x), ptr(wl.y), ptr(wl.w), n, ptr(tx), ptr(ty), m, ptr(wl.rowptr), ptr(col),
                                 ptr(wl.val), None if case == "null_os" else ctypes.byref(os_), ctypes.byref(o),
                                 ctypes.byref(h))
    msg = lib.vp_last_error(None).decode()
    assert st == vp.VP_EINVAL, (st, msg)
    assert h.value is None
    assert len(msg) > 0


@pytest.mark.parametrize("case", ["fp32", "pairwise"])
def test_yukawa_unsupported_forms(case):
    """The modified Helmholtz kernel runs in float64 with near-field tables:
    the other forms are refused before touching a device."""
    vp, lib = _lib()
    x = np.linspace(0, 1, 8)
    y = np.linspace(0, 1, 8)[::-1].copy()
    w = np.ones(8)
    kw = {"kernel": 1, "lam": 10.0}
    if case == "fp32":
        kw["precision"] = 1
    else:
        kw["p2p_mode"] = 1
    st, h, msg = _plan(lib, vp, x, y, w, 8, **kw)
    assert st == vp.VP_EUNSUPPORTED, (st, msg)
    assert h.value is None


@pytest.mark.parametrize("case", ["shape", "order0", "order_big", "null_ref", "outside_box", "outside_tri",
                                  "duplicate", "ncell_neg", "null_maps", "ok_box", "ok_tri"])
def test_correction_blocks_host_checks(case):
    """vp_correction_blocks checks the pattern (and, with no cells, returns
    before any device call)."""
    from vp_workloads import generators as gen
    vp, lib = _lib()
    xb, yb, wb = gen.gauss_legendre_box_nodes(4)
    xt, yt, wt = gen.triangle_lattice_pattern(5)
    shape, p, x, y, w, ncell, maps = 0, 4, xb, yb, wb, 0, None
    expect = vp.VP_EINVAL
    if case == "shape":
        shape = 2
    elif case == "order0":
        p = 0
    elif case == "order_big":
        p, expect = 9, vp.VP_EUNSUPPORTED
        x = y = w = np.zeros(81)
    elif case == "null_ref":
        x = None
    elif case == "outside_box":
        x = xb.copy()
        x[3] = 1.0
    elif case == "outside_tri":
        shape, p, x, y, w = 1, 5, xt.copy(), yt, wt
        x[0] = -1e-12
    elif case == "duplicate":
        shape, p, x, y, w = 1, 5, xt.copy(), yt.copy(), wt
        x[1], y[1] = x[0], y[0]
    elif case == "ncell_neg":
        ncell = -1
    elif case == "null_maps":
        ncell = 3
    elif case == "ok_box":
        expect = vp.VP_OK
    elif case == "ok_tri":
        shape, p, x, y, w, expect = 1, 5, xt, yt, wt, vp.VP_OK
    p_ = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(ctypes.c_void_p)
    st = lib.vp_correction_blocks(shape, p, p_(x), p_(y), p_(w), ncell, maps, None, None)
    assert st == expect, (st, lib.vp_last_error(None))
    if expect != vp.VP_OK:
        assert len(lib.vp_last_error(None)) > 0
