"""GPU parity of the modified Helmholtz kernel (G = lambda^2/2pi K_0(lambda r),
Section 2.1) against the CPU oracle (oracle.yukawa), through the C ABI.

The library evaluates it on uniform grids of congruent 64-point leaves by
fixed matrices per level (near tables, pattern P2M / L2P, M2M, M2L, L2L) on
the matrix cores.  Tolerance: rel_inf <= 1e-12 at p = 30 (float64).
"""
import numpy as np
import pytest

from oracle import yukawa as Y
from vp_workloads import generators as gen

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


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


def _grid(nside, seeds, csr_seed=7):
    x, y, w = gen.uniform_grid(nside)
    f = np.stack([gen.gaussian_sum_density(x, y, s)[0] for s in seeds])
    rowptr = col = val = None
    if csr_seed is not None:
        cell_ptr = np.arange(0, x.size + 1, 64, dtype=np.int64)
        rowptr, col, val = gen.own_cell_csr(cell_ptr, csr_seed, cell_class=np.zeros(nside * nside, np.int64))
    return gen.Workload(name=f"yukawa{nside}", x=x, y=y, w=w, f=f, tx=None, ty=None, rowptr=rowptr, col=col,
                        val=val, root=(-1.0, -1.0, 2.0), sample=None, meta={})


def _plan(vp, wl, lam, order=30):
    return vp.Plan(wl.x, wl.y, wl.w, rowptr=wl.rowptr, col=wl.col, val=wl.val, order=order, nbatch=wl.nbatch,
                   root=wl.root, kernel="yukawa", lam=lam)


@pytest.mark.parametrize("lam", [1.0, 10.0, 40.0])
def test_forward_16x16_all_targets(lam):
    """16 x 16 boxes (16,384 nodes), every target, lambda from the nearly
    Laplace regime to a kernel that decays within a few boxes."""
    vp = _vp()
    wl = _grid(16, [0])
    plan = _plan(vp, wl, lam)
    info = plan.info()
    assert info["kernel"] == 1 and info["lam"] == lam
    u = _host(plan.eval(_dev(wl.f)))
    ref = Y.evaluate(wl, lam)
    err = relinf(u, ref)
    print(f"yukawa lambda={lam} 16x16 boxes: rel_inf={err:.3e}")
    assert err <= TOL64
    plan.close()


def test_batched_densities_and_adjoint():
    vp = _vp()
    wl = _grid(8, [1, 2, 3])
    lam = 10.0
    plan = _plan(vp, wl, lam)
    u = _host(plan.eval(_dev(wl.f)))
    assert relinf(u, Y.evaluate(wl, lam)) <= TOL64
    g = np.random.default_rng(4).standard_normal(u.shape)
    df = _host(plan.eval_adjoint(_dev(g)))
    ref = Y.evaluate_adjoint(wl, g, lam)
    err = relinf(df, ref)
    dot = abs(np.sum(g * u) - np.sum(df * wl.f)) / abs(np.sum(g * u))
    print(f"yukawa adjoint rel_inf={err:.3e}, dot test {dot:.2e}")
    assert err <= TOL64
    assert dot <= 1e-12
    plan.close()


def test_orders_converge():
    """The FMM error falls with the order and meets the bar at p = 30."""
    vp = _vp()
    wl = _grid(16, [5], csr_seed=None)
    lam = 10.0
    ref = Y.evaluate(wl, lam)
    errs = {}
    for p in (10, 20, 30):
        plan = _plan(vp, wl, lam, order=p)
        errs[p] = relinf(_host(plan.eval(_dev(wl.f))), ref)
        plan.close()
    print("yukawa errors by order:", {k: f"{v:.2e}" for k, v in errs.items()})
    assert errs[10] > errs[20] > errs[30] or errs[20] <= TOL64
    assert errs[30] <= TOL64


def test_large_grid_sampled():
    """64 x 64 boxes (262,144 nodes), 1,024 sampled targets."""
    vp = _vp()
    wl = _grid(64, [6])
    lam = 10.0
    plan = _plan(vp, wl, lam)
    u = _host(plan.eval(_dev(wl.f)))
    idx = gen.sample_indices(wl.n, 1024, 160)
    err = relinf(u[:, idx], Y.evaluate(wl, lam, tidx=idx))
    print(f"yukawa 64x64 boxes on 1024 targets: rel_inf={err:.3e}")
    assert err <= TOL64
    plan.close()


def test_unsupported_tree_and_gradient():
    vp = _vp()
    # an adaptive tree (leaves on several levels) is outside this build
    rng = np.random.default_rng(9)
    pts = np.clip(np.concatenate([rng.uniform(-1, 1, (3000, 2)), rng.normal(0.3, 0.01, (1000, 2))]), -0.99, 0.99)
    with pytest.raises(vp.VPError) as e:
        vp.Plan(pts[:, 0].copy(), pts[:, 1].copy(), np.ones(4000), kernel="yukawa", lam=10.0)
    assert e.value.status == vp.VP_EUNSUPPORTED
    wl = _grid(8, [1], csr_seed=None)
    plan = _plan(vp, wl, 10.0)
    with pytest.raises(vp.VPError) as e:
        plan.eval_grad_targets(_dev(wl.f))
    assert e.value.status == vp.VP_EUNSUPPORTED
    plan.close()
