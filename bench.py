#!/usr/bin/env python
"""Shifted band-solve throughput of the FEAST filter on one MI355X.

A step is one filter sweep over the whole workload: for every slice and
every Gauss-Legendre node, the band LU of z_j I - B, the solves with the
slice's start block (A x = y and A^H x = y), FP64 refinement to
||y - A x|| / ||y|| <= 1e-10 (complex64 path), and the weighted node sum
Q_i = sum_j [w_j x_j + conj(w_j) xh_j].  One right-hand-side column is one
column of one shifted system in one direction.

Default workload: complex Hermitian band n=16384, b=64, 16 equal-width
slices of [-50, 50] x 8 nodes = 128 shifted systems, m0_i =
max(ceil(1.5 m_i), m_i + 10) columns per slice with m_i the exact inertia
count.  The reported value is the complex64 + FP64-refinement path; the
plain FP64 path is measured the same way and reported beside it.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# workloads whose slices are placed by exact inertia: (slices, lowest
# eigenvalues covered, slices per filter group -- the factors of one group's
# systems and its buffers stay well inside the 288 GB of HBM)
PLANNED = {"cplx-n65536-b128": (64, 25600, 32)}
# band sections above this order are sampled on the CPU by a leading section
CPU_SECTION = 8192

PEAK_FP32_MFMA = 157.3e12   # MI355X dense FP32 matrix, flop/s
PEAK_FP64 = 78.6e12         # MI355X FP64 (vector and matrix), flop/s
PEAK_HBM = 8.0e12           # bytes/s
METRIC = "shifted band-solve RHS-cols/s, FP32+refine vs FP64, at resid ≤1e-10"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="cplx-n16384-b64")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 path")
    p.add_argument("--tune-log", default=None, metavar="PATH",
                   help="append the autotuner's time of every solve variant to PATH")
    p.add_argument("--no-e2e", action="store_true",
                   help="skip the end-to-end FEAST runs (all slices to convergence)")
    p.add_argument("--cpu-cols", type=int, default=256, help="columns in the CPU sample")
    p.add_argument("--group", type=int, default=0, metavar="SLICES",
                   help="slices per filter group of a planned workload (default: its table entry)")
    p.add_argument("--eig-out", default=None, metavar="PATH",
                   help="write the end-to-end eigenvalues and residuals of both precisions "
                        "(.npz)")
    p.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                   help="after the timed region, run one plain device copy of MIB MiB "
                        "(calibrates the HBM byte counters of a profiler run)")
    return p.parse_args()


# Sources of the block-solve and residual kernels: HBM byte counts recorded under profiles/
# are reported as roofline traffic only while these files are unchanged.
SOLVE_SOURCES = ["solve_kernel.h", "solve_f32.hip", "solve_f64.hip", "solve.hip", "solve_job.h",
                 "fb_internal.h"]


def solve_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in SOLVE_SOURCES:
        with open(os.path.join(ROOT, "paper_2012_00506_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(workload: str, name: str, precision: int):
    """HBM bytes per launch of the block-solve (complex64) or FP64 residual
    kernel from the committed counter summary of this workload, if taken on
    the current sources."""
    path = os.path.join(ROOT, "profiles", f"solve-resid_{workload}_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    key = {"solve": "solve_c64" if precision == 1 else None, "resid": "resid"}.get(name)
    ent = rec.get(key) if key else None
    if not ent or rec.get("source_sha256") != solve_source_hash():
        return None
    return ent["hbm_bytes_per_launch"]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_system(args):
    """One shifted system of the sample in one worker process: band LU and
    its N and H solves of the worker's columns (oracle, numpy)."""
    name, z, col0, ncols = args
    from threadpoolctl import threadpool_limits
    from oracle import bandlu
    import synth
    cfg = synth.CONFIGS[name]
    cfg_ab = cfg.matrix()
    n = cfg.n
    if n > CPU_SECTION:  # the leading principal section; times scale with n
        n = CPU_SECTION
        cfg_ab = cfg_ab[:, :n].copy()
        for d in range(1, cfg_ab.shape[0]):
            cfg_ab[d, n - d:] = 0
    Y = synth.rhs_block(n, ncols, cfg.seed, cfg.complex_, col0=col0)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        F = bandlu.shifted_band_lu(cfg_ab, z)
        t1 = time.perf_counter()
        bandlu.lu_solve(F, Y)
        bandlu.lu_solve_h(F, Y)
        t2 = time.perf_counter()
    scale = cfg.n / n
    return (t1 - t0) * scale, (t2 - t1) * scale


def cpu_baseline(cfg, m0_mean, ncols, slices):
    """The CPU oracle on a bounded sample, on all host cores: one worker
    process per core, each factoring one shifted system of the workload (the
    nodes of the middle slice, then of further slices) and solving ncols N
    and ncols H columns with it.  Throughput = all columns solved / wall time,
    with each worker's per-system time scaled to the workload's columns per
    system (2 mean m0): t_sys = t_LU + 2 m0 t_col."""
    import multiprocessing as mp
    from oracle import quadrature
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 16))
    tasks = []
    k = len(slices) // 2
    while len(tasks) < cores:
        lo, hi = slices[k % len(slices)]
        z, _ = quadrature.contour(lo, hi, 8)
        for zj in z:
            if len(tasks) < cores:
                tasks.append((cfg.name, complex(zj), 64 * len(tasks), ncols))
        k += 1
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        times = pool.map(_cpu_system, tasks)
    wall = time.perf_counter() - t0
    cols_sys = 2.0 * m0_mean
    t_sys = [t_lu + cols_sys * t_sol / (2 * ncols) for t_lu, t_sol in times]
    value = cores * cols_sys / (sum(t_sys) / len(t_sys))
    t_lu = sum(t for t, _ in times) / len(times)
    t_sol = sum(t for _, t in times) / len(times)
    return {"value": value, "unit": "RHS-cols/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": (("" if cfg.n <= CPU_SECTION else
                        f"leading n={CPU_SECTION} sections (times scaled by {cfg.n // CPU_SECTION}) "
                        "of ") +
                       f"{cores} shifted systems of the workload (n={cfg.n}, b={cfg.b}), one per "
                       f"core in parallel processes: oracle band LU {t_lu:.2f} s + {ncols} N and "
                       f"{ncols} H column solves {t_sol:.2f} s each (mean), {wall:.1f} s wall; "
                       f"per-system time scaled to {cols_sys:.0f} columns per system")}


def progress(msg: str) -> None:
    """One line on stderr per finished leg (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_path(fb, groups, steps, warmup, cols_per_step, stream=None):
    """Time the filter sweep: a step applies every group's filter (F, Y, Q)
    once, in order."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()

    def sweep():
        return [F(Y, Q, stream=s) for F, Y, Q in groups]

    # verification pass (not timed): every column's FP64 residual <= 1e-10
    for F, _, _ in groups:
        F.with_resid = True
    rs = sweep()
    torch.cuda.synchronize()
    worst = max(float(np.max(r.resid)) for r in rs)
    passes = max(int(np.max(r.passes)) for r in rs)
    for F, _, _ in groups:
        F.with_resid = False
    for _ in range(warmup):
        sweep()
    torch.cuda.synchronize()
    fb.profile_enable(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(s)
    for _ in range(steps):
        sweep()
    ev1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = fb.profile_read()
    fb.profile_enable(False)
    ms_step = 1e3 * wall / steps
    return {"ms_per_step": ms_step, "value": cols_per_step / (ms_step / 1e3),
            "max_resid": worst, "ir_passes": passes, "prof": prof,
            "event_ms_per_step": ev0.elapsed_time(ev1) / steps}


def band_norm1(ab) -> float:
    """||B||_1 of the Hermitian band (LAPACK lower storage): the largest
    column sum of |B(i, j)| over the full matrix."""
    a = np.abs(np.asarray(ab))
    b1, n = a.shape
    col = a[0].copy()
    for d in range(1, b1):
        col[: n - d] += a[d, : n - d]   # B(j+d, j) in column j
        col[d:] += a[d, : n - d]        # conj(B(j, j-d)) in column j
    return float(col.max())


def run_e2e(fb, B, cfg, lo, hi, counts, m0, precision, nrm1):
    """FEAST on every slice of the workload to convergence, from the seeded
    start blocks, with the per-class kernel time breakdown."""
    import torch
    import synth
    Y = [synth.rhs_block_device(cfg.n, m, cfg.seed * 1000 + i, cfg.complex_)
         for i, m in enumerate(m0)]
    Y = [y.contiguous().t().contiguous().t() if y.stride(0) != 1 else y for y in Y]
    torch.cuda.synchronize()
    fb.profile_enable(True)
    t0 = time.perf_counter()
    res = fb.feast_band_slice(B, lo, hi, Y, m_expected=counts, precision=precision,
                              ir_tol=1e-10 if precision else 1e-12)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = fb.profile_read()
    fb.profile_enable(False)
    mres = max(float(r.resid[: r.m_found].max()) for r in res if r.m_found)
    lam = np.concatenate([r.lam for r in res])
    rel = np.concatenate([r.resid[: r.m_found] for r in res])
    del Y
    torch.cuda.empty_cache()
    return {"precision": "c64+f64 refinement" if precision else "f64", "seconds": wall,
            "per_eigenpair": eigenpair_errors(lam, rel, nrm1), "_lam": lam, "_res": rel,
            "iters": [r.iters for r in res], "info": [r.info for r in res],
            "eigenpairs": int(sum(r.m_found for r in res)),
            "counts_match": bool(all(r.m_found == int(c) for r, c in zip(res, counts))),
            "max_resid": mres,
            # a Ritz value with residual ||B x - l x||_2 = r (||x|| = 1) lies
            # within r of an eigenvalue of the Hermitian B
            "eig_err_bound_max": mres * nrm1,
            "breakdown_ms": {k: round(v[1], 3) for k, v in prof.items() if v[0]},
            "launches": {k: v[0] for k, v in prof.items() if v[0]}}


def kato_temple(lam, res_abs):
    """Per Ritz pair (lam_i, residual r_i = ||B x_i - lam_i x_i||, ||x_i|| = 1)
    a bound on its distance to an eigenvalue of the Hermitian B: r_i^2 / d_i
    (Kato-Temple) when the neighbouring Ritz values, widened by their own
    residuals, leave a gap d_i > r_i on both sides, else r_i.  The outermost
    pairs of the computed range take r_i (a neighbour beyond it is unknown)."""
    o = np.argsort(lam)
    l, r = lam[o], res_abs[o]
    out = r.copy()
    for k in range(1, len(l) - 1):
        d = min(l[k] - l[k - 1] - r[k - 1], l[k + 1] - l[k] - r[k + 1])
        if d > r[k]:
            out[k] = min(r[k], r[k] ** 2 / d)
    b = np.empty_like(out)
    b[o] = out
    return b


def eigenpair_errors(lam, rel, nrm1):
    """Per-eigenpair error figures relative to ||B||_1: the residual, the
    residual bound on the eigenvalue error and the Kato-Temple bound, each as
    max / 99th percentile / median over the pairs."""
    kt = kato_temple(lam, rel * nrm1) / nrm1

    def q(v):
        return {"max": float(np.max(v)), "p99": float(np.percentile(v, 99)),
                "median": float(np.median(v))}
    o = np.argsort(lam)
    inner = kt[o][1:-1] if len(lam) > 2 else kt
    return {"pairs": int(len(lam)), "resid_rel": q(rel), "eig_err_bound_rel": q(rel),
            "kato_temple_rel": q(kt), "kato_temple_rel_max_inner": float(np.max(inner))}


def bound_via_reference(lam, res_abs, lam_ref, res_ref_abs, nrm1):
    """Per Ritz value of one run (ascending order), the smaller of its own
    Kato-Temple bound and |lam - lam_ref| plus the bound of the reference
    run's Ritz value of the same rank: the reference value lies within its
    bound of an eigenvalue, so lam lies within the sum of it.  Both runs hold
    the same eigenpairs (exact counts).  Relative to ||B||_1."""
    o, oref = np.argsort(lam), np.argsort(lam_ref)
    own = kato_temple(lam, res_abs)[o]
    ref = kato_temple(lam_ref, res_ref_abs)[oref]
    d = np.abs(lam[o] - lam_ref[oref])
    return np.minimum(own, d + ref) / nrm1


def roofline(prof, precision, workload):
    name, (L, ms, work) = max(prof.items(), key=lambda kv: kv[1][1])
    if L == 0 or ms <= 0:
        return None
    achieved = work / (ms / 1e3)
    if name == "solve":
        peak = PEAK_FP32_MFMA if precision == 1 else PEAK_FP64
        bound = "mfma"
    elif name == "resid":   # FP64 MFMA products
        peak, bound = PEAK_FP64, "mfma"
    elif name in ("bandmm", "inertia"):
        peak, bound = PEAK_FP64, "alu"
    else:
        peak = PEAK_FP32_MFMA if precision == 1 else PEAK_FP64
        bound = "mfma"
    return {"kernel": name, "bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12,
            "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": recorded_traffic(workload, name, precision),
            "launches": L, "avg_launch_ms": ms / L, "work_per_launch_flop": work / L}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by slices; see the design notes)", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    import paper_2012_00506_amd as fb
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(3)
    cfg = synth.CONFIGS[args.workload]
    t_setup = time.perf_counter()
    ab = cfg.matrix()
    B = fb.DeviceBand.from_band(ab)
    if cfg.slices:
        slices = list(cfg.slices)
        group = len(slices)
    else:  # equal-count slices of the lowest nev eigenvalues, by exact inertia
        K, nev, group = PLANNED[cfg.name]
        if args.group > 0:
            group = args.group
        bounds, _, _ = fb.slice_plan(B, K, "equal_count", nev=nev)
        slices = [(float(bounds[i]), float(bounds[i + 1])) for i in range(K)]
    edges = [slices[0][0]] + [s[1] for s in slices]
    neg, _, _ = fb.band_inertia(B, edges)
    counts = np.diff(neg)
    m0 = [max(math.ceil(1.5 * int(c)), int(c) + 10) for c in counts]
    lo = [s[0] for s in slices]
    hi = [s[1] for s in slices]
    Y = [synth.rhs_block_device(cfg.n, m, cfg.seed * 1000 + i, cfg.complex_)
         for i, m in enumerate(m0)]
    Y = [y.contiguous().t().contiguous().t() if y.stride(0) != 1 else y for y in Y]
    Q = [fb.colmajor(cfg.n, m, Y[0].dtype) for m in m0]
    n_nodes = 8
    ndir = 2 if cfg.complex_ else 1
    cols_per_step = float(sum(m0) * n_nodes * ndir)
    setup_s = time.perf_counter() - t_setup
    spans = [(g, min(g + group, len(slices))) for g in range(0, len(slices), group)]

    def groups(**kw):
        """One filter per group of slices (the whole sweep when it fits),
        sharing one workspace."""
        gs = [(fb.FeastFilter(B, lo[a:b], hi[a:b], m0[a:b], n_nodes=n_nodes, **kw), Y[a:b],
               Q[a:b]) for a, b in spans]
        # sized for the verification pass (which also keeps residuals) and the
        # timed passes (without them the waves are planned differently)
        need = 0
        for F, y, q in gs:
            for wr in (False, True):
                F.with_resid = wr
                need = max(need, F.workspace_bytes(y, q))
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
        for F, _, _ in gs:
            F._ws = ws
        return gs

    # tune the block-solve kernel for both precisions on this shape (not timed):
    # the systems of a sweep (at most as many as fit beside their buffers),
    # enough columns that each variant fills the GPU several times over as
    # the sweep's launches do
    tuned = {}
    nsys_t, m_t = min(len(m0) * n_nodes, 128), 512
    if cfg.n > 32768:
        nsys_t, m_t = 64, 256
    for prec in (1, 0):
        v, ms = fb.autotune(B, prec, nsys=nsys_t, m=m_t, cache_path=args.tune_log)
        tuned["c64" if prec else "c128"] = {"variant": v, "ms": ms}
        progress(f"autotune {'c64' if prec else 'c128'}: variant {v}, {ms:.1f} ms")

    res = {}
    G = groups(precision=1, ir_tol=1e-10, ir_max=6)
    res["fp32ir"] = run_path(fb, G, args.steps, args.warmup, cols_per_step)
    progress(f"complex64 + refinement: {res['fp32ir']['ms_per_step']:.1f} ms/step")
    del G
    torch.cuda.empty_cache()
    # the same sweep replayed from HIP graphs on a stream of its own
    gs = torch.cuda.Stream()
    G = groups(precision=1, ir_tol=1e-10, ir_max=6, graph=True)
    res["fp32ir_graph"] = run_path(fb, G, args.steps, args.warmup, cols_per_step, stream=gs)
    progress(f"complex64 + refinement, graph: {res['fp32ir_graph']['ms_per_step']:.1f} ms/step")
    del G
    torch.cuda.empty_cache()
    if not args.no_fp64:
        G = groups(precision=0)
        res["fp64"] = run_path(fb, G, args.steps, args.warmup, cols_per_step)
        progress(f"FP64 batched: {res['fp64']['ms_per_step']:.1f} ms/step")
        del G
        torch.cuda.empty_cache()
        if len(spans) == 1:
            # the plain FP64 path: one launch sequence per slice, no batching
            G = groups(precision=0, batched=False)
            res["fp64_plain"] = run_path(fb, G, args.steps, args.warmup, cols_per_step)
            progress(f"FP64 plain: {res['fp64_plain']['ms_per_step']:.1f} ms/step")
            del G
            torch.cuda.empty_cache()

    main_ = res["fp32ir"]
    out = {
        "metric": METRIC,
        "value": main_["value"],
        "unit": "RHS-cols/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 LU+solves, f64 residual/refinement",
        "data": "synthetic",
        "config": {"workload": cfg.name, "n": cfg.n, "b": cfg.b, "complex": cfg.complex_,
                   "slices": len(slices), "nodes": n_nodes, "systems": len(slices) * n_nodes,
                   "slices_per_filter_launch_group": group,
                   "m0": m0, "rhs_cols_per_step": cols_per_step, "ir_tol": 1e-10,
                   "parallelism": "single GPU"},
        "roofline": roofline(main_["prof"], 1, cfg.name),
        # every timed kernel class against its own peak (the dominant one is "roofline")
        "roofline_by_kernel": {k: roofline({k: v}, 1, cfg.name)
                               for k, v in main_["prof"].items() if v[0]},
        "fp32ir": {k: v for k, v in main_.items() if k != "prof"},
        "kernels_fp32ir": {k: {"launches": v[0], "ms": v[1], "flop": v[2]}
                           for k, v in main_["prof"].items() if v[0]},
        "setup_s": setup_s,
    }
    if "fp64" in res:
        r64 = res["fp64"]
        out["fp64"] = {k: v for k, v in r64.items() if k != "prof"}
        out["fp64"]["roofline"] = roofline(r64["prof"], 0, cfg.name)
        out["kernels_fp64"] = {k: {"launches": v[0], "ms": v[1], "flop": v[2]}
                               for k, v in r64["prof"].items() if v[0]}
        out["fp32ir_over_fp64"] = main_["value"] / r64["value"]
        if "fp64_plain" in res:
            rp = res["fp64_plain"]
            out["fp64_plain"] = {k: v for k, v in rp.items() if k != "prof"}
            out["fp32ir_over_fp64_plain"] = main_["value"] / rp["value"]
        else:
            out["fp64_plain"] = "not run: the sweep is split into filter groups"
    rg = res["fp32ir_graph"]
    out["fp32ir_graph"] = {k: v for k, v in rg.items() if k != "prof"}
    out["graph_over_direct"] = rg["value"] / main_["value"]
    out["solve_variants"] = tuned
    if args.calib_copy:
        nel = args.calib_copy * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = {"read": nel * 4, "write": nel * 4}
        del src, dst
    if not args.no_e2e:
        del Y, Q
        torch.cuda.empty_cache()
        nrm1 = band_norm1(ab)
        out["e2e"] = []
        for prec in (1, 0):
            out["e2e"].append(run_e2e(fb, B, cfg, lo, hi, counts, m0, prec, nrm1))
            progress(f"end to end {out['e2e'][-1]['precision']}: {out['e2e'][-1]['seconds']:.2f} s")
        lam1, lam0 = out["e2e"][0]["_lam"], out["e2e"][1]["_lam"]
        if len(lam1) == len(lam0):
            # the same eigenpairs in both precisions (every count is exact):
            # per-eigenpair difference of the eigenvalues, relative to ||B||_1
            d = np.abs(np.sort(lam1) - np.sort(lam0)) / nrm1
            out["e2e_c64_vs_f64_eig_rel"] = {"max": float(d.max()),
                                            "p99": float(np.percentile(d, 99)),
                                            "median": float(np.median(d))}
            # the complex64 run's eigenvalues certified through the FP64 run's
            via = bound_via_reference(lam1, out["e2e"][0]["_res"] * nrm1, lam0,
                                      out["e2e"][1]["_res"] * nrm1, nrm1)
            out["e2e"][0]["per_eigenpair"]["eig_err_bound_via_f64_rel_max"] = float(via.max())
        if args.eig_out:
            np.savez(args.eig_out, lam_c64=lam1, res_c64=out["e2e"][0]["_res"], lam_f64=lam0,
                     res_f64=out["e2e"][1]["_res"], norm1=nrm1)
        for e in out["e2e"]:
            del e["_lam"], e["_res"]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, float(np.mean(m0)), args.cpu_cols, slices)
        progress(f"CPU oracle: {out['cpu_baseline']['value']:.0f} RHS-cols/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
