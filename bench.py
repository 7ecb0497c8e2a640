#!/usr/bin/env python3
"""Benchmark of the volume-potential evaluation hot path on one MI355X.

Headline workload: the batched uniform grid -- 256 x 256 boxes on [-1,1]^2
with an 8x8 Gauss-Legendre rule per box (4,194,304 nodes), 16 seeded
Gaussian-sum densities evaluated in one launch, targets = nodes, own-cell
correction matrix (64 values per row; every box carries the same 64 x 64
block, as the box corrections of one box size form one table), FMM order
p = 30 in float64.  The FP32-bulk form (p = 14) is measured on the same
workload beside it.  A step is one full evaluation u = V f + C f (charges,
upward pass, M2L, downward pass, near field, far-field evaluation,
correction and un-permutation) with inputs resident in HBM; the plan (tree,
lists, operators) is built once beforehand, as the paper excludes set-up
from its timings.

Secondary records in the same JSON line (skipped with --no-secondary):
  * uniform128: 128 x 128 boxes (1,048,576 nodes, one density), FP64 p = 30
    beside FP32-bulk p = 14 (scaled and split hi/lo M2L), each with its error
    against the oracle on 4,096 sampled targets;
  * star: the adaptive star-shaped domain (1,488,064 nodes), FP64 and
    FP32-bulk, with errors against the oracle;
  * per_entry_correction: the headline grid with every correction value
    drawn on its own (no shared block), FP64, with the correction apply's
    rate against the HBM peak;
  * oversampled: 64 x 64 boxes with the density at 8 x 8 Chebyshev nodes
    per box (262,144 targets) and the smooth rule at 16 x 16 Chebyshev
    nodes (1,048,576 sources; the paper's twofold oversampling), FP64 and
    FP32-bulk, with errors against the oracle on 4,096 sampled targets.

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
HBM_GBS = 8000.0            # MI355X published HBM3E bandwidth
P2P_FLOPS_PER_PAIR = 27     # 2 differences, 3 for r^2, 20 for log(r^2), 2 for the update
GOLDEN_C3 = os.path.join(ROOT, "tests", "golden", "c3_sample_smooth.npy")
C3_NAME = "uniform256x256_gl8_b16"


# HBM bytes per launch of the headline's kernels, from two rocprofv3 --pmc
# runs (FETCH_SIZE, then WRITE_SIZE) of this script, each scaled by what the
# counter reads for a plain device copy of known size in the same run.  Valid
# only for the kernel sources they were taken on: each stage carries a digest
# of the sources that define its kernel, its launch and its schedule (whole
# headers, and the named functions of the .hip files), and a change there
# turns that stage's traffic into null.
TRAFFIC_WORKLOAD = C3_NAME
TRAFFIC = {  # stage -> (read bytes, written bytes, digest) per launch, FP64 p = 30, 16 densities
    "m2l": (1290221129, 671401433, "d00f38b54b6ec641cbf5cb7e92ea87521ccf424f0a66e987f8907d6ae5fd505d"),
    "tables": (1974325726, 538012040, "bd118e83c8dff3329c22b16d59a72776756f0e10d248f76bcdc9e1bf909b3110"),
}
CSRC = os.path.join(ROOT, "paper_2203_05933_amd", "csrc")
STAGE_SOURCES = {
    "m2l": (["vp_m2l_scaled.hpp", "vp_translate.hpp", "vp_internal.hpp"],
            {"vp_fmm.hip": ["build_schedules", "tile_order_by_work", "launch_m2l", "m2l_scaled",
                            "launch_m2l_scaled"]}),
    "tables": (["vp_translate.hpp", "vp_internal.hpp", "vp_near.hip"],
               {"vp_fmm.hip": ["launch_tables", "run_tables", "tile_order_by_work", "prepare_charges"]}),
    "corr": (["vp_translate.hpp", "vp_internal.hpp"],
             {"vp_fmm.hip": ["correction_apply", "launch_fixed_apply", "build_cells"]}),
}


def _function_text(src, name):
    """The text of the first definition of function `name` in src (signature
    to the matching closing brace)."""
    import re
    m = re.search(r"\n[^\n;]*\b" + re.escape(name) + r"\([^;{]*\)\s*\{", src)
    if not m:
        raise KeyError(name)
    i = src.index("{", m.end() - 1)
    depth = 0
    for j in range(i, len(src)):
        depth += {"{": 1, "}": -1}.get(src[j], 0)
        if depth == 0:
            return src[m.start():j + 1]
    raise KeyError(name)


def stage_digest(stage):
    import hashlib
    files, funcs = STAGE_SOURCES[stage]
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    for f, names in funcs.items():
        with open(os.path.join(CSRC, f)) as fh:
            src = fh.read()
        for n in names:
            h.update((f + ":" + n).encode() + _function_text(src, n).encode())
    return h.hexdigest()


def measured_traffic(stage, workload_name, order):
    """Counter-measured HBM bytes per launch, or None when they do not apply."""
    if stage not in TRAFFIC or workload_name != TRAFFIC_WORKLOAD or order != 30:
        return None
    r, w, digest = TRAFFIC[stage]
    if stage_digest(stage) != digest:
        return None
    return r + w


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(name, shared_blocks=True):
    from vp_workloads import generators as gen
    if name == "star":
        return gen.config1()
    if name == "uniform128":
        return gen.config2()
    if name == "uniform16":
        return gen.config0()
    if name == "uniform256x16":
        return gen.config3(shared_blocks=shared_blocks)
    if name == "oversampled64":
        return gen.config5()
    if name == "yukawa128":
        return gen.config6()
    raise SystemExit(f"unknown workload {name}")


# ----------------------------------------------------------------------------
# timing
# ----------------------------------------------------------------------------
def time_evals(plan, f, u, steps, warmup):
    """Wall-clock time of `steps` evaluations (no per-stage events inside),
    then the same number of evaluations with per-stage HIP events recorded on
    the stream each stage runs on, for the stage breakdown and the roofline."""
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


def oversampling_layout(wl):
    """Box layout of an oversampled workload (None for the others)."""
    import numpy as np
    if not hasattr(wl, "p_interp"):
        return None
    p, q = wl.p_interp, wl.q_interp
    return dict(p=p, q=q, n_in=wl.n_in, in_start=np.arange(wl.nbox, dtype=np.int64) * p * p,
                out_start=np.arange(wl.nbox, dtype=np.int64) * q * q)


def make_plan(wl, order, precision, m2l_mode="auto", one_stream=False, max_leaf=64, tune=False, tune_leaf=False,
              m2l_waves=0, table_waves=0):
    """A plan of the workload; tune: the plan-time autotuner (M2L form and
    waves per tile, near-table waves, streams), tune_leaf: also the leaf size."""
    from paper_2203_05933_amd import vp
    lam = wl.meta.get("lambda")
    kern = dict(kernel="yukawa", lam=lam) if lam else {}
    return vp.Plan(wl.x, wl.y, wl.w, wl.tx, wl.ty, wl.rowptr, wl.col, wl.val, order=order, max_leaf=max_leaf,
                   nbatch=wl.nbatch, precision=precision, m2l_mode=m2l_mode, one_stream=one_stream, root=wl.root,
                   oversampling=oversampling_layout(wl), autotune=tune and m2l_mode == "auto",
                   autotune_leaf=tune_leaf and m2l_mode == "auto", m2l_waves=m2l_waves, table_waves=table_waves,
                   **kern)


def tuned_choices(info):
    """The knobs an evaluation runs with (the autotuner's choices when tuned)."""
    from paper_2203_05933_amd import vp
    names = {v: k for k, v in vp.M2L_MODES.items()}
    return {"m2l_mode": names.get(info["m2l_mode"], info["m2l_mode"]), "m2l_waves": info["m2l_waves"],
            "table_waves": info["table_waves"], "one_stream": bool(info["one_stream"]), "max_leaf": info["max_leaf"],
            "tuned": {0: "defaults", 1: "timed at plan time", 2: "from the tuning cache"}[info["tuned"]],
            "tune_ms": info["tune_ms"],
            # own-cell corrections applied inside the near tables' self slot (no correction pass)
            "corrections_folded": bool(info["corr_folded"])}


def run_form(wl, f, order, precision, steps, warmup, m2l_mode="auto", one_stream=False, label="", tune=True,
             tune_leaf=False):
    """Plan (autotuned unless the M2L mode is given), time and return
    (record, result tensor, plan info, stage timing, plan)."""
    import torch
    t0 = time.perf_counter()
    plan = make_plan(wl, order, precision, m2l_mode, one_stream, tune=tune, tune_leaf=tune_leaf)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    u = torch.empty((wl.nbatch, wl.m), dtype=torch.float64, device="cuda:0")
    dt, tim = time_evals(plan, f, u, steps, warmup)
    ms = dt / steps * 1e3
    value = wl.m * wl.nbatch / (dt / steps) / 1e6
    info = plan.info()
    stages = {k: v / max(tim["evals"], 1) for k, v in tim["ms"].items()}
    rec = {"value": value, "ms_per_step": ms, "order": order, "precision": precision, "plan_ms": plan_ms,
           "m2l_mode": info["m2l_mode"], "choices": tuned_choices(info), "stages_ms": stages}
    log(f"[bench] {label} {precision} p={order}: plan {plan_ms:.0f} ms, {ms:.3f} ms/eval, {value:.1f} Mpoints/s; "
        "stages(ms/eval)=" + json.dumps({k: round(v, 4) for k, v in stages.items()}))
    return rec, u, info, tim, plan


# ----------------------------------------------------------------------------
# roofline records
# ----------------------------------------------------------------------------
def stage_roofline(info, tim, stage, workload_name=None):
    """Roofline record of one single-kernel stage, or None when the stage has no model."""
    n = max(tim["evals"], 1)
    avg_s = tim["ms"][stage] / n / 1e3
    if avg_s <= 0:
        return None
    P = info["order"] + 1
    nb = info["nbatch"]
    fp64 = info["precision"] == 0
    rec = None
    if (stage == "p2p" and info["near_pairs"] == 0) or (stage == "tables" and info["table_pairs"] == 0):
        return None  # the stage did no work in this plan
    if stage == "p2p":
        flops = info["near_pairs"] * nb * P2P_FLOPS_PER_PAIR
        rec = {"bound": "alu", "achieved": flops / avg_s / 1e12, "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
               "kernel": "k_p2p",
               "work": f"{info['near_pairs']} pairs x {nb} densities x {P2P_FLOPS_PER_PAIR} flops"}
    elif stage == "tables":
        # near-field tables: one multiply-add per (target, source) pair and density, FP64 matrix cores
        flops = info["table_pairs"] * nb * 2
        one_wave = info["table_waves"] == 1 and info["table_pattern"] <= 64
        rec = {"bound": "mfma", "achieved": flops / avg_s / 1e12, "peak": FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
               "kernel": "k_tables_ct (near-field tables, one wave over two tiles)" if one_wave
               else "k_translate_split (near-field tables)",
               "work": f"{info['table_pairs']} table pairs x {nb} densities x 2 flops"}
    elif stage == "m2l":
        # the "m2l" stage times the launch over the levels from split_level on;
        # the levels below run in the "coarse" stage on the third stream
        nv = info["m2l_translations"] - info["m2l_coarse_translations"]
        tile_ops = info["m2l_tile_ops"] - info["m2l_coarse_tile_ops"]
        # the modified Helmholtz kernel runs the per-offset real 2P x 2P operators
        scaled = info["m2l_mode"] in (4, 5) and info.get("kernel", 0) == 0
        fp64_core = info["m2l_mode"] in (1, 4) or info.get("kernel", 0) == 1
        per = 4 * P * P + 12 * P if scaled else 8 * P * P
        flops = nv * nb * per
        peak = FP64_MFMA_TFLOPS if fp64_core else FP32_MFMA_TFLOPS
        form = "2 real P x P products + 2 complex scalings" if scaled else "real 2P x 2P product"
        # matrix-core flops the launch issues: per (16-column tile, offset) two real
        # PQ x PQ products (scaled form) or one PD x PD product
        PQ = (P + 15) // 16 * 16
        PDm = (max(2 * P + 1, P + PQ) + 15) // 16 * 16  # rows per expansion column
        issued = tile_ops * (64 * PQ * PQ if scaled else 32 * PDm * PDm)
        rec = {"bound": "mfma", "achieved": flops / avg_s / 1e12, "peak": peak, "unit": "TFLOP/s",
               "kernel": ("k_m2l_wave" if info["m2l_waves"] == 1 else "k_m2l_scaled") if scaled
               else "k_translate_split", "issued_tflops": issued / avg_s / 1e12,
               "work": f"{nv} translations (V lists and X-list virtual children, levels >= {info['split_level']}) "
                       f"x {nb} densities x {per} flops ({form}, P={P}); {tile_ops} tile products issued"}
    elif stage == "corr":
        nnz, m, n_, cells = info["nnz"], info["m"], info["n"], info["corr_cells"]
        if cells > 0:
            # distinct values (cells with an identical block read one copy); per cell:
            # first row, run start, value offset, two row pointers; f read once, outputs written
            nval, shared = info["corr_values_read"], info["corr_shared_cells"]
            bytes_ = nval * 8 + cells * (4 + 4 + 8 + 16) + m * 8 * nb + n_ * 8 * nb
            kern, what = "k_corr_cells", (f"{nval} distinct values of {nnz} x 8 B ({shared} of {cells} cells "
                                          f"share an identical block) + {cells} cell records")
            if info["corr_one_block"]:
                kern = "k_fixed_apply (one shared 64 x 64 block over every (cell, density) column)"
            elif info["corr_groups"] > 0:
                kern = "k_corr_group + k_corr_cells"
                what += f", {info['corr_groups']} groups of up to 16 cells"
        else:
            bytes_ = nnz * 8 + (m + 1) * 8 + m * 4 + m * 8 * nb + n_ * 8 * nb
            kern, what = "k_corr", f"{nnz} values x 8 B + row pointers and runs"
        rec = {"bound": "hbm", "achieved": bytes_ / avg_s / 1e9, "peak": HBM_GBS, "unit": "GB/s", "kernel": kern,
               "work": f"{what}, f read once, {nb} output rows written",
               # every value the kernel loads, shared blocks included (those come from the caches)
               "values_loaded_gbs": nnz * 8 / avg_s / 1e9}
    if rec is None:
        return None
    rec["frac"] = rec["achieved"] / rec["peak"]
    rec["avg_ms"] = avg_s * 1e3
    rec["traffic"] = measured_traffic(stage, workload_name, info["order"]) if fp64 else None
    if rec["traffic"] is not None:
        rec["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)"
    return rec


def rooflines(info, tim, workload_name=None):
    """(dominant stage, its record, all records): the modelled single-kernel
    stage with the largest device time is the dominant one."""
    recs = {}
    for st in ("m2l", "tables", "p2p", "corr"):
        r = stage_roofline(info, tim, st, workload_name)
        if r is not None:
            recs[st] = r
    stage = max(recs, key=lambda k: recs[k]["avg_ms"])
    return stage, recs[stage], recs


# ----------------------------------------------------------------------------
# oracle (test infrastructure: reference values and the cpu_baseline leg)
# ----------------------------------------------------------------------------
def reference(wl):
    """Oracle values at the workload's sampled targets: [nbatch, nsample].  The
    headline grid's smooth sums are stored (tests/golden, written by a script
    that calls the oracle only); the correction rows are added here."""
    import numpy as np
    from oracle import direct
    if wl.name.startswith(C3_NAME) and os.path.exists(GOLDEN_C3):
        smooth = np.load(GOLDEN_C3)
        assert smooth.shape == (wl.nbatch, wl.sample.size)
        return smooth + direct.csr(wl.rowptr, wl.col, wl.val, wl.f, tidx=wl.sample)
    if hasattr(wl, "p_interp"):
        from oracle import oversample
        return oversample.evaluate(wl, tidx=wl.sample)
    if wl.meta.get("lambda"):
        from oracle import yukawa
        return yukawa.evaluate(wl, wl.meta["lambda"], tidx=wl.sample)
    return direct.evaluate(wl.x, wl.y, wl.w, wl.f, wl.rowptr, wl.col, wl.val, wl.tx, wl.ty, tidx=wl.sample)


def rel_err(u, ref, sample):
    import numpy as np
    got = u.cpu().numpy()[:, sample]
    return float(max(np.max(np.abs(got[b] - ref[b])) / np.max(np.abs(ref[b])) for b in range(ref.shape[0])))


def cpu_baseline(wl, count):
    """The oracle timed on the host's cores on `count` seeded targets of the
    workload (all nodes, all densities)."""
    from oracle import direct
    from vp_workloads import generators as gen
    sample = gen.sample_indices(wl.m, count, 110)
    log(f"[bench] oracle on {len(sample)} sampled targets x {wl.n} nodes x {wl.nbatch} densities "
        f"({direct.num_threads()} threads)")
    t0 = time.perf_counter()
    direct.evaluate(wl.x, wl.y, wl.w, wl.f, wl.rowptr, wl.col, wl.val, wl.tx, wl.ty, tidx=sample)
    tc = time.perf_counter() - t0
    return {"value": len(sample) * wl.nbatch / tc / 1e6, "unit": "Mpoints/s", "cores": direct.num_threads(),
            "kind": "oracle",
            "sample": f"{len(sample)} seeded targets (seed 110) of the same workload against all {wl.n} nodes and "
                      f"{wl.nbatch} densities (direct float64 sum with compensated summation + CSR row), {tc:.1f} s"}


# ----------------------------------------------------------------------------
# secondary records
# ----------------------------------------------------------------------------
def serialized_roofline(wl, f, order, precision, rec, roof, steps, warmup):
    """The roofline of a three-stream plan's dominant stage from a one-stream
    pass of the same kernels (with three streams the stage times include the
    other streams' kernels); returns (stage, roofline) and keeps the overlapped
    record in rec["roofline_overlapped"]."""
    import torch
    ch = rec["choices"]
    p1 = make_plan(wl, order, precision, m2l_mode=ch["m2l_mode"], one_stream=True, max_leaf=ch["max_leaf"],
                   m2l_waves=ch["m2l_waves"], table_waves=ch["table_waves"])
    u1 = torch.empty((wl.nbatch, wl.m), dtype=torch.float64, device="cuda:0")
    _, tim1 = time_evals(p1, f, u1, steps, warmup)
    rec["roofline_overlapped"] = roof
    stage, roof1, _ = rooflines(p1.info(), tim1, wl.name)
    rec["roofline_source"] = "serialized pass (one stream, the same kernels)"
    p1.close()
    return stage, roof1


def precision_pair(name, steps, warmup, order, order32, with_cpu):
    """FP64 beside the FP32-bulk form (scaled and split hi/lo M2L) on one workload."""
    import torch
    wl = workload(name)
    f = torch.tensor(wl.f, dtype=torch.float64, device="cuda:0")
    ref = reference(wl) if with_cpu else None
    if hasattr(wl, "p_interp"):
        desc = (f"{wl.name}: {wl.m} targets (density at {wl.p_interp}x{wl.p_interp} Chebyshev nodes per box), "
                f"{wl.n} sources ({wl.q_interp}x{wl.q_interp} per box), {wl.nbatch} density")
    else:
        desc = f"{wl.name}: {wl.n} nodes, targets=nodes, {wl.nbatch} density"
    out = {"workload": desc, "n": wl.n, "m": wl.m, "nbatch": wl.nbatch}
    forms = (("fp64", order, "fp64", "auto"), ("fp32_scaled", order32, "fp32", "auto"),
             ("fp32_split_hi_lo", order32, "fp32", "split"))
    base = None
    for key, p, prec, mode in forms:
        rec, u, info, tim, plan = run_form(wl, f, p, prec, steps, warmup, mode, label=wl.name)
        stage, roof, _ = rooflines(info, tim, wl.name)
        plan.close()
        if not rec["choices"]["one_stream"]:
            stage, roof = serialized_roofline(wl, f, p, prec, rec, roof, steps, warmup)
        rec["dominant_stage"] = stage
        rec["roofline"] = roof
        if ref is not None:
            rec["rel_err"] = rel_err(u, ref, wl.sample)
            rec["rel_err_targets"] = int(wl.sample.size)
        if base is None:
            base = rec["value"]
        else:
            rec["speedup_vs_fp64"] = rec["value"] / base
        out[key] = rec
        del u
    return out


def yukawa_record(steps, warmup, order, with_cpu):
    """The modified Helmholtz kernel (lambda = 10) on the 128 x 128-box grid, FP64."""
    import torch
    wl = workload("yukawa128")
    f = torch.tensor(wl.f, dtype=torch.float64, device="cuda:0")
    rec, u, info, tim, plan = run_form(wl, f, order, "fp64", steps, warmup, label=wl.name)
    rec["workload"] = (f"{wl.name}: {wl.n} nodes, targets=nodes, {wl.nbatch} density, "
                       f"G = lambda^2/(2 pi) K0(lambda r), lambda = {wl.meta['lambda']:g}")
    stage, roof, _ = rooflines(info, tim, wl.name)
    rec["dominant_stage"] = stage
    rec["roofline"] = roof
    if with_cpu:
        rec["rel_err"] = rel_err(u, reference(wl), wl.sample)
        rec["rel_err_targets"] = int(wl.sample.size)
    plan.close()
    return rec


def correction_generation_record(steps, warmup, with_cpu):
    """Own-cell singular corrections generated on the device: the star
    workload's 4,096 boundary-band triangles (45-node pattern, total degree
    < 9) and its three box levels (8 x 8 Gauss-Legendre), one call each."""
    import numpy as np
    import torch
    from paper_2203_05933_amd import vp
    from vp_workloads import generators as gen
    xt, yt, wt = gen.triangle_lattice_pattern(9)
    tris = gen.star_band_triangles()
    tmaps = torch.tensor(gen.triangle_maps(tris), dtype=torch.float64, device="cuda:0")
    xb, yb, wb = gen.gauss_legendre_box_nodes(8)
    hs = [2.6 / 2 ** (lvl + 1) for lvl in (7, 8, 9)]
    bmaps = torch.tensor(gen.cell_maps(np.zeros((3, 2)), [h * np.eye(2) for h in hs]), dtype=torch.float64,
                         device="cuda:0")
    out = torch.empty((len(tris), 45, 45), dtype=torch.float64, device="cuda:0")
    for _ in range(max(warmup, 1)):
        vp.correction_blocks("triangle", 9, xt, yt, wt, tmaps, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        vp.correction_blocks("triangle", 9, xt, yt, wt, tmaps, out)
    torch.cuda.synchronize()
    tri_ms = (time.perf_counter() - t0) / steps * 1e3
    t0 = time.perf_counter()
    for _ in range(steps):
        vp.correction_blocks("box", 8, xb, yb, wb, bmaps)
    torch.cuda.synchronize()
    box_ms = (time.perf_counter() - t0) / steps * 1e3
    rec = {"workload": "star boundary band: 4,096 straight triangles x 45 nodes (total degree < 9); "
                       "3 box sizes x 64 nodes (8 x 8 Gauss-Legendre)",
           "triangles_ms_per_call": tri_ms, "triangle_blocks_per_s": len(tris) / (tri_ms * 1e-3),
           "triangle_rows_per_s": len(tris) * 45 / (tri_ms * 1e-3),
           "boxes_ms_per_call": box_ms, "unit": "blocks/s",
           "note": "one vp_correction_blocks call: host rule tables, map checks, kernel, stream synchronised"}
    log(f"[bench] correction generation: 4096 triangles {tri_ms:.2f} ms/call "
        f"({rec['triangle_blocks_per_s']:.0f} blocks/s), 3 box sizes {box_ms:.2f} ms/call")
    if with_cpu:
        from oracle import corrections as CO
        ref = np.stack([xt, yt], 1)
        m = gen.triangle_maps(tris[:1])[0]
        t0 = time.perf_counter()
        CO.block(CO.TRIANGLE, 9, ref, wt, m[:2], m[2:].reshape(2, 2), rows=[0, 22])
        row_s = (time.perf_counter() - t0) / 2
        rec["cpu_baseline"] = {"value": 1.0 / (45 * row_s), "unit": "blocks/s", "cores": 1, "kind": "oracle",
                               "sample": "2 rows of one band triangle's 45-row block (oracle.corrections), "
                                         f"{2 * row_s:.1f} s, scaled to a block"}
    return rec


def per_entry_correction(steps, warmup, order, with_cpu):
    """The headline grid with every correction value drawn on its own."""
    import torch
    wl = workload("uniform256x16", shared_blocks=False)
    f = torch.tensor(wl.f, dtype=torch.float64, device="cuda:0")
    rec, u, info, tim, plan = run_form(wl, f, order, "fp64", steps, warmup, label="per-entry correction")
    stage, roof, recs = rooflines(info, tim, wl.name)
    rec["workload"] = (f"{wl.name}: {wl.n} nodes x {wl.nbatch} densities, {info['nnz']} correction values each "
                       "drawn on its own")
    rec["corr_apply"] = recs.get("corr")
    rec["dominant_stage"] = stage
    if with_cpu:
        rec["rel_err"] = rel_err(u, reference(wl), wl.sample)
    plan.close()
    del u
    # one stream: the apply without the other streams beside it
    plan1 = make_plan(wl, order, "fp64", one_stream=True)
    u1 = torch.empty((wl.nbatch, wl.m), dtype=torch.float64, device="cuda:0")
    _, tim1 = time_evals(plan1, f, u1, steps, warmup)
    rec["corr_apply_one_stream"] = stage_roofline(plan1.info(), tim1, "corr", wl.name)
    plan1.close()
    return rec


# ----------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform256x16",
                    choices=["uniform256x16", "star", "uniform128", "uniform16", "oversampled64", "yukawa128"])
    ap.add_argument("--order", type=int, default=30)
    ap.add_argument("--order-fp32", type=int, default=14)
    ap.add_argument("--max-leaf", type=int, default=64)
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-bulk form")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle (cpu_baseline and errors)")
    ap.add_argument("--no-secondary", action="store_true", help="skip the secondary records")
    ap.add_argument("--no-one-stream", action="store_true",
                    help="skip the serialized pass (every kernel on one stream): the roofline then comes from the "
                         "overlapped run, whose kernel durations include contention")
    ap.add_argument("--cpu-sample", type=int, default=256, help="targets the timed oracle evaluates")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the timed loops, run one plain device copy (y = 2 x) of this many MiB read and "
                         "written, as the calibration kernel for hardware byte counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported by this build "
              "(the evaluation is single-device; see the design notes on sharding).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2203_05933_amd import vp  # noqa: F401  (fails loudly without libvp.so)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log(f"[bench] generating workload {args.workload}")
    wl = workload(args.workload)
    nb = wl.nbatch
    log(f"[bench] n={wl.n} m={wl.m} nbatch={nb} nnz={0 if wl.rowptr is None else int(wl.rowptr[-1])}")
    f = torch.tensor(wl.f, dtype=torch.float64, device="cuda:0")

    rec64, u64, info, tim, plan = run_form(wl, f, args.order, "fp64", args.steps, args.warmup, label="headline",
                                           tune_leaf=True)
    log(f"[bench] headline plan choices: {json.dumps(rec64['choices'])}")
    value, ms_per_step = rec64["value"], rec64["ms_per_step"]
    stage, roof, roofs = rooflines(info, tim, wl.name)
    plan.close()

    # The serialized pass: the same evaluation with every kernel on one
    # stream, timed the same way (warm-up, wall-clock loop, then the loop with
    # per-stage HIP events).  The three-stream run overlaps the kernels, so
    # its per-stage durations include contention; the roofline is taken from
    # this pass, whose per-stage durations are the kernels' own (its last
    # `steps` launches of each kernel are the event-timed ones).
    one = None
    roofs_overlapped = roofs
    if not args.no_one_stream:
        ch = rec64["choices"]  # the same kernels as the headline plan, every one on one stream
        plan1 = make_plan(wl, args.order, "fp64", m2l_mode=ch["m2l_mode"], one_stream=True, max_leaf=ch["max_leaf"],
                          m2l_waves=ch["m2l_waves"], table_waves=ch["table_waves"])
        u1 = torch.empty_like(u64)
        dt1, tim1 = time_evals(plan1, f, u1, args.steps, args.warmup)
        inf1 = plan1.info()
        stage, roof, roofs = rooflines(inf1, tim1, wl.name)
        one = {"ms_per_step": dt1 / args.steps * 1e3,
               "stages_ms": {k: v / max(tim1["evals"], 1) for k, v in tim1["ms"].items()}}
        log(f"[bench] fp64 one stream: {one['ms_per_step']:.3f} ms/eval")
        plan1.close()
        del u1
    log(f"[bench] dominant stage {stage}: {roof['kernel']} {roof['avg_ms']:.3f} ms, frac {roof['frac']:.3f}")

    forms32 = {}
    if not args.no_fp32:
        # FP32-bulk: the scaled M2L in FP32 (default) and the split hi/lo FP32
        # products per offset (T_hi M_hi + T_hi M_lo + T_lo M_hi)
        for key, mode, desc in (("fp32_scaled", "auto", "autotuned FP32-bulk form (M2L form, waves, streams, leaf)"),
                                ("split_hi_lo", "split", "split hi/lo fp32 mfma, per-offset operators")):
            r32, u32, inf32, tim32, plan32 = run_form(wl, f, args.order_fp32, "fp32", args.steps, args.warmup,
                                                      mode, label="headline", tune_leaf=True)
            r32["m2l"] = desc
            r32["speedup_vs_fp64"] = r32["value"] / value
            st32, roof32, _ = rooflines(inf32, tim32, wl.name)
            plan32.close()
            if key == "fp32_scaled" and not r32["choices"]["one_stream"] and not args.no_one_stream:
                # the roofline from a serialized pass, as for FP64
                st32, roof32 = serialized_roofline(wl, f, args.order_fp32, "fp32", r32, roof32, args.steps,
                                                   args.warmup)
            r32["dominant_stage"] = st32
            r32["roofline"] = roof32
            forms32[key] = (r32, u32)

    cpu = None
    rel64 = None
    if not args.no_cpu:
        ref = reference(wl)
        rel64 = rel_err(u64, ref, wl.sample)
        for key, (r32, u32) in forms32.items():
            r32["rel_err"] = rel_err(u32, ref, wl.sample)
        log(f"[bench] rel_inf err on {wl.sample.size} targets x {nb} densities: fp64={rel64:.3e} "
            + " ".join(f"{k}={r['rel_err']:.3e}" for k, (r, _) in forms32.items()))
        cpu = cpu_baseline(wl, args.cpu_sample)
    out32 = None
    if forms32:
        out32 = forms32["fp32_scaled"][0]
        out32["split_hi_lo"] = forms32["split_hi_lo"][0]
    del forms32

    secondary = None
    if not args.no_secondary:
        secondary = {}
        del u64
        torch.cuda.empty_cache()
        secondary["per_entry_correction"] = per_entry_correction(args.steps, args.warmup, args.order, not args.no_cpu)
        torch.cuda.empty_cache()
        secondary["uniform128_precision"] = precision_pair("uniform128", args.steps, args.warmup, args.order,
                                                           args.order_fp32, not args.no_cpu)
        torch.cuda.empty_cache()
        secondary["star"] = precision_pair("star", args.steps, args.warmup, args.order, args.order_fp32,
                                           not args.no_cpu)
        torch.cuda.empty_cache()
        secondary["oversampled"] = precision_pair("oversampled64", args.steps, args.warmup, args.order,
                                                  args.order_fp32, not args.no_cpu)
        torch.cuda.empty_cache()
        secondary["yukawa"] = yukawa_record(args.steps, args.warmup, args.order, not args.no_cpu)
        secondary["correction_generation"] = correction_generation_record(args.steps, args.warmup, not args.no_cpu)

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
        "config": {"workload": f"{wl.name}: {wl.n} nodes x {nb} densities, targets=nodes, p={args.order} float64, "
                               f"max_leaf={rec64['choices']['max_leaf']} (autotuned among {args.max_leaf} and "
                               f"{args.max_leaf // 4}), own-cell correction (one shared 64x64 box block)",
                   "n": wl.n, "m": wl.m, "nbatch": nb, "order": args.order, "nnz": int(info["nnz"]),
                   "parallelism": "single GPU"},
        "rel_err": rel64,
        "rel_err_targets": None if rel64 is None else f"{wl.sample.size} sampled targets x {nb} densities",
        "plan_ms": rec64["plan_ms"],
        "autotuned": rec64["choices"],
        "stages_ms": rec64["stages_ms"],
        "dominant_stage": stage,
        "roofline": roof,
        "roofline_source": ("serialized pass (one stream): per-stage HIP events over its timed loop"
                            if one is not None else "three-stream run: per-stage HIP events (include contention)"),
        "stage_rooflines": roofs,
        "stage_rooflines_overlapped": roofs_overlapped,
        "one_stream": one,
        "fp32_form": out32,
        "cpu_baseline": cpu,
        "secondary": secondary,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
