"""GPU parity of the oversampled box rule (vp_plan_oversampled) against the
CPU oracle (oracle.oversample), through the C ABI.

The density is given at 8 x 8 Chebyshev-root nodes per box (the targets),
the smooth rule sits at 16 x 16 Chebyshev-root nodes (the sources; the
paper's twofold oversampling q = 2p), the library builds the interpolation
map itself.  Tolerances: rel_inf <= 1e-12 (float64), <= 1e-6 (FP32-bulk).
"""
import numpy as np
import pytest

from oracle import direct
from oracle import oversample as OS
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


def _layout(wl, in_start=None):
    p, q = wl.p_interp, wl.q_interp
    return dict(p=p, q=q, n_in=wl.n_in,
                in_start=np.arange(wl.nbox, dtype=np.int64) * p * p if in_start is None else in_start,
                out_start=np.arange(wl.nbox, dtype=np.int64) * q * q)


def _plan(vp, wl, **kw):
    return vp.Plan(wl.x, wl.y, wl.w, wl.tx, wl.ty, wl.rowptr, wl.col, wl.val, nbatch=wl.nbatch, root=wl.root,
                   oversampling=kw.pop("oversampling", None) or _layout(wl), **kw)


@pytest.fixture(scope="module")
def small():
    return gen.config5(nbox_side=8, f_seeds=(3, 4, 5), csr_seed=6, sample_seed=None)


def test_forward_all_targets(small):
    vp = _vp()
    plan = _plan(vp, small, order=30)
    info = plan.info()
    assert (info["os_p"], info["os_q"], info["n_in"]) == (8, 16, small.m)
    u = _host(plan.eval(_dev(small.f)))
    ref = OS.evaluate(small)
    err = relinf(u, ref)
    print(f"oversampled 8x8 boxes, 3 densities: rel_inf={err:.3e}")
    assert err <= TOL64
    plan.close()


def test_adjoint_and_dot_product(small):
    vp = _vp()
    plan = _plan(vp, small, order=30)
    g = np.random.default_rng(8).standard_normal((small.nbatch, small.m))
    df = _host(plan.eval_adjoint(_dev(g)))
    ref = OS.evaluate_adjoint(small, g)
    err = relinf(df, ref)
    u = _host(plan.eval(_dev(small.f)))
    dot = abs(np.sum(g * u) - np.sum(df * small.f)) / abs(np.sum(g * u))
    print(f"oversampled adjoint rel_inf={err:.3e}, dot test {dot:.2e}")
    assert err <= TOL64
    assert dot <= 1e-12
    plan.close()


def test_box_blocks_in_any_order(small):
    """The density values of box b may sit anywhere (here the boxes' blocks
    in reverse order): the same values give the same potentials."""
    vp = _vp()
    nb, p2 = small.nbox, 64
    rev = (nb - 1 - np.arange(nb, dtype=np.int64)) * p2
    f_rev = small.f.reshape(small.nbatch, nb, p2)[:, ::-1, :].reshape(small.nbatch, -1).copy()
    # the correction columns follow the values: column k of box b moves with it
    blk = small.col // p2
    col_rev = ((nb - 1 - blk) * p2 + small.col % p2).astype(np.int32)
    plan = vp.Plan(small.x, small.y, small.w, small.tx, small.ty, small.rowptr, col_rev, small.val,
                   nbatch=small.nbatch, root=small.root, oversampling=_layout(small, in_start=rev))
    u = _host(plan.eval(_dev(f_rev)))
    err = relinf(u, OS.evaluate(small))
    print(f"reversed box blocks: rel_inf={err:.3e}")
    assert err <= TOL64
    plan.close()


def test_fp32_bulk_form(small):
    vp = _vp()
    plan = _plan(vp, small, order=14, precision="fp32")
    u = _host(plan.eval(_dev(small.f)))
    err = relinf(u, OS.evaluate(small))
    print(f"oversampled fp32-bulk p=14: rel_inf={err:.3e}")
    assert err <= TOL32
    plan.close()


def test_target_gradient(small):
    vp = _vp()
    plan = _plan(vp, small, order=30)
    gr = _host(plan.eval_grad_targets(_dev(small.f)))
    fq = OS.upsample(small.f, small.nbox, 8, 16)
    ref = direct.smooth_grad(small.x, small.y, small.w, fq, small.tx, small.ty)
    err = relinf(gr, ref)
    print(f"oversampled target gradient rel_inf={err:.3e}")
    assert err <= TOL64
    plan.close()


def test_noalloc_matches_eval(small):
    import torch
    vp = _vp()
    plan = _plan(vp, small, order=30)
    fd = _dev(small.f)
    ref = _host(plan.eval(fd))
    out = torch.empty((small.nbatch, small.m), dtype=torch.float64, device="cuda:0")
    got = _host(plan.eval_noalloc(fd, out))
    assert relinf(got, ref) <= TOL64
    plan.close()


def test_full_size_sampled():
    """64 x 64 boxes: 262,144 targets, 1,048,576 sources, checked on 4,096
    sampled targets against the oracle."""
    vp = _vp()
    wl = gen.config5()
    plan = _plan(vp, wl, order=30)
    u = _host(plan.eval(_dev(wl.f)))[:, wl.sample]
    ref = OS.evaluate(wl, tidx=wl.sample)
    err = relinf(u, ref)
    print(f"oversampled 64x64 boxes on {wl.sample.size} targets: rel_inf={err:.3e}")
    assert err <= TOL64
    plan.close()
