"""vp_eval_noalloc (the evaluation with its workspace in the library's static
device array) against vp_eval, through the C ABI.

Two calls in a row on different plans, the second with a smaller input, then
the first plan again (so the static array holds a smaller plan's leftovers
when the larger one reuses it), each compared with vp_eval on the same plan
and inputs to the float64 bar (rel_inf <= 1e-12; the kernels and their order
are the same, so the results agree to the bit in practice).  A plan whose
workspace exceeds the static array is rejected with VP_EINVAL.
"""
import numpy as np
import pytest

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


def _grid(nside, seeds, csr_seed, precision="fp64", order=30, table_waves=0, shared=False):
    vp = _vp()
    x, y, w = gen.uniform_grid(nside)
    f = np.stack([gen.gaussian_sum_density(x, y, s)[0] for s in seeds])
    cell_ptr = np.arange(0, x.shape[0] + 1, 64, dtype=np.int64)
    cls = np.zeros(nside * nside, dtype=np.int64) if shared else None
    rowptr, col, val = gen.own_cell_csr(cell_ptr, csr_seed, cell_class=cls)
    plan = vp.Plan(x, y, w, rowptr=rowptr, col=col, val=val, order=order, nbatch=len(seeds),
                   precision=precision, root=(-1.0, -1.0, 2.0), table_waves=table_waves)
    return plan, f


def _compare(plan, f, label):
    import torch
    fd = _dev(f)
    ref = _host(plan.eval(fd))
    out = torch.full((plan.nbatch, plan.m), float("nan"), dtype=torch.float64, device="cuda:0")
    got = _host(plan.eval_noalloc(fd, out))
    err = relinf(got, ref)
    print(f"{label}: n={plan.n} nbatch={plan.nbatch} noalloc bytes={plan.info()['noalloc_bytes']} "
          f"rel_inf vs vp_eval={err:.3e} bitwise={np.array_equal(got, ref)}", flush=True)
    assert np.all(np.isfinite(got))
    assert err <= TOL64
    return err


def test_noalloc_matches_eval_two_calls():
    big, f_big = _grid(16, [0], 1)                 # 16,384 nodes, one density
    small, f_small = _grid(8, [3, 4], 5)           # 4,096 nodes, two densities
    assert small.info()["noalloc_bytes"] < big.info()["noalloc_bytes"]
    _compare(big, f_big, "first call (16x16 boxes)")
    _compare(small, f_small, "second call, smaller input (8x8 boxes)")
    _compare(big, f_big, "first plan again")
    big.close()
    small.close()


def test_noalloc_one_wave_tables():
    """The one-wave near-table kernel with several densities reads a
    density-fastest copy of the charges, which the static array also holds."""
    plan, f = _grid(8, [11, 12, 13], 14, table_waves=1)
    assert plan.info()["table_waves"] == 1
    _compare(plan, f, "one-wave tables, three densities, 8x8 boxes")
    plan.close()


def test_noalloc_fp32_bulk_form():
    plan, f = _grid(8, [7], 8, precision="fp32", order=14)
    _compare(plan, f, "fp32-bulk 8x8 boxes")
    plan.close()


@pytest.mark.parametrize("nb", [3, 16])
def test_noalloc_folded_corrections(nb):
    """One shared correction block on congruent boxes: forward evaluations
    apply it inside the near tables and write the output without reading it
    (the output buffer starts as NaN here)."""
    plan, f = _grid(8, list(range(20, 20 + nb)), 21, shared=True)
    assert plan.info()["corr_folded"] == 1
    _compare(plan, f, f"folded corrections, {nb} densities, 8x8 boxes")
    plan.close()


def test_noalloc_rejects_oversized_plan():
    vp = _vp()
    import torch
    plan, f = _grid(128, [0, 1, 2, 3], 9)  # 1,048,576 nodes x 4 densities
    need = plan.info()["noalloc_bytes"]
    assert need > (64 << 20)
    out = torch.empty((plan.nbatch, plan.m), dtype=torch.float64, device="cuda:0")
    with pytest.raises(vp.VPError) as e:
        plan.eval_noalloc(_dev(f), out)
    assert e.value.status == vp.VP_EINVAL
    assert "exceeds the static workspace" in str(e.value)
    # the plan stays usable
    u = _host(plan.eval(_dev(f)))
    assert np.all(np.isfinite(u))
    plan.close()
