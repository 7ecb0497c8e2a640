#!/usr/bin/env python3
"""Benchmark of the volume-potential evaluation hot path on one MI355X.

Workload (default): the star-shaped domain r = 1 + 0.3 cos 5 theta with an
adaptive box quadtree and a boundary band of triangles, 1,488,064 nodes,
targets = nodes, own-cell correction matrix, one density, FMM order p = 30
in float64.  A step is one full evaluation u = V f + C f (charges, upward
pass, M2L, downward pass, near field, far-field evaluation, correction and
un-permutation) with inputs resident in HBM; the plan (tree, lists,
operators) is built once beforehand, as the paper excludes set-up from its
timings.  The FP32-bulk form (p = 14) is measured on the same workload and
reported alongside.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mpoints/s volume-potential eval at rel err 1e-12 (FP64) vs 1e-6 (FP32 form)"
FP64_VECTOR_TFLOPS = 78.6   # MI355X published peak, FP64 vector
FP64_MFMA_TFLOPS = 78.6     # MI355X published peak, FP64 matrix (dense)
FP32_MFMA_TFLOPS = 157.3    # MI355X published peak, FP32 matrix (dense)
P2P_FLOPS_PER_PAIR = 27     # 2 differences, 3 for r^2, 20 for log(r^2), 2 for the update


# HBM bytes per launch of the star-workload kernels, from two rocprofv3 --pmc
# runs (FETCH_SIZE, then WRITE_SIZE) of this script, each scaled by what the
# counter reads for a plain 1 GiB device copy in the same run (FETCH_SIZE
# reads half the bytes, WRITE_SIZE all of them).  Valid only for the kernel
# sources they were taken on: the digest below covers every file of the
# library's source directory, and any change there turns traffic into null.
TRAFFIC_DIGEST = "d5945a711f0af58975d4e3526ade1f21f08edad5678cf3540973a3551c72dcd3"
TRAFFIC_WORKLOAD = "star_adaptive"
TRAFFIC = {  # stage -> (read bytes, written bytes) per launch, FP64 p = 30, one density
    "corr": (83605134, 11912327),  # k_corr_group + k_corr_cells
    "m2l": (250839465, 18844963),  # k_m2l_scaled, levels from the split level on
    "p2p": (92101604, 3547276),
}


def source_digest():
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2203_05933_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(stage, workload_name, order, nbatch):
    """Counter-measured HBM bytes per launch, or None when they do not apply."""
    if stage not in TRAFFIC or workload_name != TRAFFIC_WORKLOAD or order != 30 or nbatch != 1:
        return None
    if source_digest() != TRAFFIC_DIGEST:
        return None
    r, w = TRAFFIC[stage]
    return r + w


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(name):
    from vp_workloads import generators as gen
    if name == "star":
        return gen.config1()
    if name == "uniform128":
        return gen.config2()
    if name == "uniform16":
        return gen.config0()
    if name == "uniform256x16":
        return gen.config3()
    raise SystemExit(f"unknown workload {name}")


def time_evals(plan, f, u, steps, warmup):
    """Wall-clock time of `steps` evaluations (no per-stage events inside),
    then the same number of evaluations with per-stage HIP events on the
    plan's stream for the stage breakdown and the roofline."""
    import torch
    for _ in range(warmup):
        plan.eval(f, out=u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.eval(f, out=u)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.set_timing(True)
    for _ in range(steps):
        plan.eval(f, out=u)
    tim = plan.timing()
    plan.set_timing(False)
    return dt, tim


def stage_roofline(plan, tim, precision, stage, workload_name=None):
    """Roofline record of one single-kernel stage, or None when the stage has no model."""
    rec = _stage_roofline(plan, tim, precision, stage)
    if rec is not None and precision == "fp64":
        info = plan.info()
        rec["traffic"] = measured_traffic(stage, workload_name, info["order"], info["nbatch"])
        rec["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)"
    return rec


def _stage_roofline(plan, tim, precision, stage):
    info = plan.info()
    n = max(tim["evals"], 1)
    avg_s = tim["ms"][stage] / n / 1e3
    if avg_s <= 0:
        return None
    P = info["order"] + 1
    nb = info["nbatch"]
    if stage == "p2p":
        flops = info["near_pairs"] * nb * P2P_FLOPS_PER_PAIR
        return {"bound": "alu", "achieved": flops / avg_s / 1e12, "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": flops / avg_s / 1e12 / FP64_VECTOR_TFLOPS, "traffic": None, "kernel": "k_p2p",
                "avg_ms": avg_s * 1e3,
                "work": f"{info['near_pairs']} pairs x {nb} densities x {P2P_FLOPS_PER_PAIR} flops"}
    if stage == "m2l":
        # the "m2l" stage times the launch over the levels from split_level on;
        # the levels below run in the "coarse" stage on the third stream
        nv = info["m2l_translations"] - info["m2l_coarse_translations"]
        tile_ops = info["m2l_tile_ops"] - info["m2l_coarse_tile_ops"]
        scaled = info["m2l_mode"] in (4, 5)
        fp64_core = info["m2l_mode"] in (1, 4)
        per = 4 * P * P + 12 * P if scaled else 8 * P * P
        flops = nv * nb * per
        peak = FP64_MFMA_TFLOPS if fp64_core else FP32_MFMA_TFLOPS
        form = "2 real P x P products + 2 complex scalings" if scaled else "real 2P x 2P product"
        # matrix-core flops the launch issues: per (16-column tile, offset) two real
        # PQ x PQ products (scaled form) or one PD x PD product
        PQ = (P + 15) // 16 * 16
        PDm = (max(2 * P + 1, P + PQ) + 15) // 16 * 16  # rows per expansion column
        issued = tile_ops * (64 * PQ * PQ if scaled else 32 * PDm * PDm)
        return {"bound": "mfma", "achieved": flops / avg_s / 1e12, "peak": peak, "unit": "TFLOP/s",
                "frac": flops / avg_s / 1e12 / peak, "traffic": None,
                "kernel": "k_m2l_scaled" if scaled else "k_translate_split", "avg_ms": avg_s * 1e3,
                "issued_tflops": issued / avg_s / 1e12,
                "work": f"{nv} translations (V lists and X-list virtual children, levels >= {info['split_level']}) "
                        f"x {nb} densities x {per} flops ({form}, P={P}); {tile_ops} tile products issued"}
    if stage == "corr":
        nnz, m, n_, cells = info["nnz"], info["m"], info["n"], info["corr_cells"]
        if cells > 0:
            # distinct values (cells with an identical block read one copy); per cell:
            # first row, run start, value offset, two row pointers; f read once, outputs written
            nval, shared = info["corr_values_read"], info["corr_shared_cells"]
            bytes_ = nval * 8 + cells * (4 + 4 + 8 + 16) + m * 8 * nb + n_ * 8 * nb
            kern, what = "k_corr_cells", (f"{nval} distinct values of {nnz} x 8 B ({shared} of {cells} cells "
                                          f"share an identical block) + {cells} cell records")
            if info["corr_groups"] > 0:
                # one density: cells of a repeated block go 16 at a time through one matrix-core product
                kern = "k_corr_group + k_corr_cells"
                what += f", {info['corr_groups']} groups of up to 16 cells"
        else:
            bytes_ = nnz * 8 + (m + 1) * 8 + m * 4 + m * 8 * nb + n_ * 8 * nb
            kern, what = "k_corr", f"{nnz} values x 8 B + row pointers and runs"
        return {"bound": "hbm", "achieved": bytes_ / avg_s / 1e9, "peak": 8000.0, "unit": "GB/s",
                "frac": bytes_ / avg_s / 1e9 / 8000.0, "traffic": None, "kernel": kern,
                "avg_ms": avg_s * 1e3, "work": f"{what}, f read once, {nb} output rows written",
                # every value the kernel loads, shared blocks included (those come from the caches)
                "values_loaded_gbs": nnz * 8 / avg_s / 1e9}
    return None


def roofline(plan, tim, precision, workload_name=None):
    """Roofline record of the single-kernel stage with the largest device time."""
    recs = {}
    for st in ("m2l", "p2p", "corr"):
        r = stage_roofline(plan, tim, precision, st, workload_name)
        if r is not None:
            recs[st] = r
    stage = max(recs, key=lambda k: recs[k]["avg_ms"])
    return stage, recs[stage], recs


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="star", choices=["star", "uniform128", "uniform16", "uniform256x16"])
    ap.add_argument("--order", type=int, default=30)
    ap.add_argument("--order-fp32", type=int, default=14)
    ap.add_argument("--max-leaf", type=int, default=64)
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-bulk form")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle (cpu_baseline and errors)")
    ap.add_argument("--no-one-stream", action="store_true",
                    help="skip the one-stream run (per-stage times without the second stream's overlap)")
    ap.add_argument("--cpu-sample", type=int, default=12288, help="targets the oracle evaluates")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the timed loops, run one plain device copy (y = 2 x) of this many MiB read and "
                         "written, as the calibration kernel for hardware byte counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported by this build "
              "(the evaluation is single-device; see the design notes on sharding).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2203_05933_amd import vp

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log(f"[bench] generating workload {args.workload}")
    wl = workload(args.workload)
    nb = wl.nbatch
    log(f"[bench] n={wl.n} m={wl.m} nbatch={nb} nnz={0 if wl.rowptr is None else int(wl.rowptr[-1])}")

    f = torch.tensor(wl.f, dtype=torch.float64, device="cuda:0")
    u = torch.empty((nb, wl.m), dtype=torch.float64, device="cuda:0")

    t0 = time.perf_counter()
    plan = vp.Plan(wl.x, wl.y, wl.w, wl.tx, wl.ty, wl.rowptr, wl.col, wl.val, order=args.order,
                   max_leaf=args.max_leaf, nbatch=nb, precision="fp64", root=wl.root)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    info = plan.info()
    log(f"[bench] fp64 plan {plan_ms:.0f} ms: boxes={info['nbox']} leaves={info['nleaf']} "
        f"levels={info['nlevels']} lists={info['list_len']} near_pairs={info['near_pairs']}")
    dt, tim = time_evals(plan, f, u, args.steps, args.warmup)
    ms_per_step = dt / args.steps * 1e3
    value = wl.m * nb / (dt / args.steps) / 1e6
    log(f"[bench] fp64: {ms_per_step:.3f} ms/eval, {value:.1f} Mpoints/s; stages(ms/eval)="
        + json.dumps({k: round(v / max(tim['evals'], 1), 4) for k, v in tim["ms"].items()}))
    stage, roof, roofs = roofline(plan, tim, "fp64", wl.name)
    u64 = u.clone()

    one = None
    if not args.no_one_stream:
        # the same evaluation with every kernel on one stream: stage times
        # without contention from the overlapped second stream
        plan1 = vp.Plan(wl.x, wl.y, wl.w, wl.tx, wl.ty, wl.rowptr, wl.col, wl.val, order=args.order,
                        max_leaf=args.max_leaf, nbatch=nb, precision="fp64", one_stream=True, root=wl.root)
        u1 = torch.empty_like(u)
        dt1, tim1 = time_evals(plan1, f, u1, args.steps, args.warmup)
        one = {"ms_per_step": dt1 / args.steps * 1e3,
               "stages_ms": {k: v / max(tim1["evals"], 1) for k, v in tim1["ms"].items()},
               "stage_rooflines": {st: r for st in ("m2l", "p2p", "corr")
                                   if (r := _stage_roofline(plan1, tim1, "fp64", st)) is not None}}
        log(f"[bench] fp64 one stream: {one['ms_per_step']:.3f} ms/eval; stages(ms/eval)="
            + json.dumps({k: round(v, 4) for k, v in one["stages_ms"].items()}))
        plan1.close()
        del u1

    out32 = None
    forms32 = {}
    if not args.no_fp32:
        # FP32-bulk form: the default (scaled M2L in FP32) and the split hi/lo FP32
        # M2L products (T_hi M_hi + T_hi M_lo + T_lo M_hi per offset)
        for name, mode, desc in (("fp32_scaled", "auto", "fp32 mfma, scaled form"),
                                 ("split_hi_lo", "split", "split hi/lo fp32 mfma, per-offset operators")):
            plan32 = vp.Plan(wl.x, wl.y, wl.w, wl.tx, wl.ty, wl.rowptr, wl.col, wl.val, order=args.order_fp32,
                             max_leaf=args.max_leaf, nbatch=nb, precision="fp32", m2l_mode=mode, root=wl.root)
            u32 = torch.empty_like(u)
            dt32, tim32 = time_evals(plan32, f, u32, args.steps, args.warmup)
            v32 = wl.m * nb / (dt32 / args.steps) / 1e6
            forms32[name] = ({"value": v32, "ms_per_step": dt32 / args.steps * 1e3, "order": args.order_fp32,
                              "m2l": desc,
                              "stages_ms": {k: v / max(tim32["evals"], 1) for k, v in tim32["ms"].items()},
                              "speedup_vs_fp64": v32 / value}, u32)
            log(f"[bench] fp32-bulk ({name}): {dt32 / args.steps * 1e3:.3f} ms/eval, {v32:.1f} Mpoints/s")
            plan32.close()
        out32 = forms32["fp32_scaled"][0]
        out32["split_hi_lo"] = forms32["split_hi_lo"][0]
    cpu = None
    rel64 = rel32 = None
    if not args.no_cpu:
        from oracle import direct
        sample = wl.sample if wl.sample is not None else np.arange(wl.m)
        if args.cpu_sample > len(sample):
            # a larger seeded draw, so that the timed oracle run is 10-30 s of CPU work
            from vp_workloads import generators as gen
            sample = gen.sample_indices(wl.m, args.cpu_sample, 110)
        sample = sample[: args.cpu_sample]
        log(f"[bench] oracle on {len(sample)} sampled targets x {wl.n} nodes ({direct.num_threads()} threads)")
        t0 = time.perf_counter()
        ref = direct.evaluate(wl.x, wl.y, wl.w, wl.f, wl.rowptr, wl.col, wl.val, wl.tx, wl.ty, tidx=sample)
        tc = time.perf_counter() - t0
        cpu = {"value": len(sample) * nb / tc / 1e6, "unit": "Mpoints/s", "cores": direct.num_threads(),
               "kind": "oracle",
               "sample": f"{len(sample)} seeded targets of the same workload against all {wl.n} nodes "
                         f"(direct float64 sum with compensated summation + CSR row), {tc:.1f} s"}
        got = u64.cpu().numpy()[:, sample]
        rel64 = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        for name, (rec32, u32) in forms32.items():
            got32 = u32.cpu().numpy()[:, sample]
            rec32["rel_err"] = float(np.max(np.abs(got32 - ref)) / np.max(np.abs(ref)))
        if out32 is not None:
            rel32 = out32["rel_err"]
        log(f"[bench] rel_inf err fp64={rel64:.3e} fp32={rel32}")

    if args.copy_mib > 0:
        n_el = args.copy_mib * (1 << 20) // 8
        src = torch.ones(n_el, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {args.copy_mib} MiB read, {args.copy_mib} MiB written")
        del src, dst

    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.n} nodes, targets=nodes, {nb} density, p={args.order} float64, "
                               f"max_leaf={args.max_leaf}", "n": wl.n, "m": wl.m, "nbatch": nb,
                   "order": args.order, "nnz": int(info["nnz"]), "parallelism": "single GPU"},
        "rel_err": rel64,
        "plan_ms": plan_ms,
        "stages_ms": {k: v / max(tim["evals"], 1) for k, v in tim["ms"].items()},
        "dominant_stage": stage,
        "roofline": roof,
        "stage_rooflines": roofs,
        "one_stream": one,
        "fp32_form": out32,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
