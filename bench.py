#!/usr/bin/env python3
"""Throughput of the CLAK-Eig hot path on one MI355X: GLS cells per second.

A step is one pass of the per-block pipeline (genotype ingest and centring
statistics, rotation by Z^T, grid contraction, Schur solve) over every SNP block
of the workload, with the genotypes already resident in HBM.  The per-cohort
set-up (eigendecomposition of Phi, covariate and trait preparation) runs once
before timing and is reported separately.

Prints ONE JSON line.  Defaults: the single-trait workload n=1000, p=4
(p_L=3), m=10^6 SNPs in blocks of 10^4, mixed precision.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "c1": (1, "single-trait GWAS n=1000 p=4 m=1e6 (blocks of 1e4) t=1"),
    "c2": (2, "multi-trait GWAS n=1000 p=4 m=1e5 (blocks of 1e4) t=1000"),
    "c0": (0, "single-trait GWAS n=256 p=4 m=2000 t=1"),
    "c4": (4, "large multi-trait GWAS n=1e4 p=9 m=2e6 (blocks of 2e4) t=1000"),
    "c3": (3, "8 uneven cohorts n=500..4000 p=4 m=5e4 each (blocks of 1e4) t=10..2000, one batch launch"),
}
C3_BLOCK = 10_000
PEAK = {"mixed": (5000.0, "int8 dense MFMA, 5.0 POP/s"), "fp64": (78.6, "FP64 dense MFMA, 78.6 TFLOP/s")}
GRID_PRODUCTS = 10  # int8 digit products the grid kernel issues per algorithmic product


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c1")
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--m", type=int, default=None, help="override the number of SNPs (a multiple of the block)")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64-path comparison run")
    ap.add_argument("--eager", action="store_true",
                    help="call clak_run_block per block on one stream instead of the block pipeline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c2", action="store_true",
                    help="skip the multi-trait sub-record (n=1000, p=4, m=1e5, t=1000) of the default run")
    ap.add_argument("--host-genotypes", action="store_true",
                    help="keep the genotypes in pinned host memory: the ingest kernel reads them over PCIe "
                         "(end-to-end rate with the host link; not the HBM-resident headline)")
    ap.add_argument("--stage-genotypes", action="store_true",
                    help="plan flag CLAK_STAGE_GENOTYPES: copy-engine staging of every block before the ingest")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip clak_autotune_pipeline (launch parameters timed on a pipelined pass over the first "
                         "blocks before the timed region)")
    ap.add_argument("--tuning", default=None,
                    help="fixed launch parameters instead of the autotuner, as rot_cfg:C,rot_rg:R,grid_tt:T,grid_xt:X "
                         "(0: built-in; a profile of a tuned run repeats its choice this way)")
    ap.add_argument("--tune-blocks", type=int, default=4, help="blocks of the autotuner's pipelined passes")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file, read and appended to (default: a temporary copy of the library's "
                         "tuning database for gfx950, so shapes it lists are not timed again)")
    ap.add_argument("--retune", action="store_true", help="time every shape, ignoring the tuning database")
    ap.add_argument("--bed", action="store_true",
                    help="also time the out-of-core scan: the genotypes written as a PLINK 1 binary file (2-bit "
                         "rows) in the temp directory, read by the library's reader thread into pinned buffers "
                         "and streamed through the pipeline (disk/page cache -> host -> PCIe -> GPU)")
    ap.add_argument("--bed-depth", type=int, default=8, help="pinned buffers of the file reader")
    ap.add_argument("--pval", action="store_true",
                    help="also write the two-sided Wald p-value of every cell (fused in the Schur epilogue)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target duration of the oracle sample")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run one plain device-to-device copy of this many bytes (reference for the "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def upload_genotypes(w, m, torch, host=False):
    """(m, n) uint8 genotypes on the GPU (or in pinned host memory), generated block by block on the host."""
    G = torch.empty((m, w.n), dtype=torch.uint8, pin_memory=True) if host else \
        torch.empty((m, w.n), dtype=torch.uint8, device="cuda")
    chunk = 100_000
    for s0 in range(0, m, chunk):
        c = min(chunk, m - s0)
        G[s0:s0 + c].copy_(torch.from_numpy(w.genotypes(s0, c)))
    return G


def block_list(G, b, se, block, pv=None):
    m = G.shape[0]
    if pv is None:
        return [(G[s0:s0 + block], b[:, s0:s0 + block], se[:, s0:s0 + block]) for s0 in range(0, m, block)]
    return [(G[s0:s0 + block], b[:, s0:s0 + block], se[:, s0:s0 + block], None, pv[:, s0:s0 + block])
            for s0 in range(0, m, block)]


class Pass:
    """One step: every block of the workload, through the block pipeline
    (ingest of the next blocks on a side stream overlapped with block b,
    blocks alternating between two compute streams) or per-block calls."""

    def __init__(self, clak, plan, G, b, se, block, eager, pv=None):
        self.clak, self.plan, self.eager = clak, plan, eager
        self.blocks = block_list(G, b, se, block, pv)
        self.pipe = None if eager else clak.clak_pipeline_create(plan.handle, self.blocks)

    def __call__(self):
        if self.pipe is None:
            for blk in self.blocks:
                self.clak.clak_run_block(self.plan.handle, *blk)
        else:
            self.clak.clak_pipeline_launch(self.pipe)

    def close(self):
        if self.pipe is not None:
            self.clak.clak_pipeline_destroy(self.pipe)
            self.pipe = None


TUNING_DB = os.path.join(ROOT, "paper_1207_2169_amd", "tuning", "gfx950.txt")


def tune_cache_path(args):
    """The cache file the autotuner reads and appends to: --tune-cache, else a
    temporary copy of the library's tuning database (lines written by
    clak_autotune_pipeline on an MI355X), or none with --retune."""
    if args.tune_cache or args.retune:
        return args.tune_cache
    import shutil
    import tempfile
    fd, path = tempfile.mkstemp(prefix="clak_tuning_", suffix=".txt")
    os.close(fd)
    if os.path.exists(TUNING_DB):
        shutil.copyfile(TUNING_DB, path)
    import atexit
    atexit.register(os.remove, path)
    args.tune_cache = path
    return path


def tune(clak, handle, G, b, se, block, args):
    """Launch parameters for the plan: the fixed ones of --tuning, else
    clak_autotune_pipeline over the first --tune-blocks blocks (a pipelined
    pass per candidate), which takes them from the cache file when it lists
    the shape.  Returns "fixed", "database" or "timed"."""
    if args.tuning:
        clak.clak_plan_set_tuning(handle, *tuning_tuple(dict(p.split(":") for p in args.tuning.split(","))))
        return "fixed"
    path = tune_cache_path(args)
    size = os.path.getsize(path) if path and os.path.exists(path) else -1
    nb = max(1, min(args.tune_blocks, G.shape[0] // block))
    clak.clak_autotune_pipeline(handle, block_list(G[:nb * block], b[:, :nb * block], se[:, :nb * block], block),
                                cache_path=path)
    grew = path is None or not os.path.exists(path) or os.path.getsize(path) != size
    return "timed" if grew else "database"


def make_plan(clak, torch, w, block, precision, flags=0):
    prec = clak.CLAK_PREC_MIXED if precision == "mixed" else clak.CLAK_PREC_FP64
    plan = clak.Plan(w.n, w.pL, w.t, block, prec, flags)
    t = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    clak.clak_set_kinship(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Phi)).cuda())
    t1 = time.perf_counter()
    clak.clak_set_covariates(plan.handle, torch.from_numpy(np.ascontiguousarray(w.XL.T)).cuda().t())
    t2 = time.perf_counter()
    Y = torch.from_numpy(np.ascontiguousarray(w.Y.T)).cuda().t()
    # variance components of every trait by REML (timed only: the scan below
    # uses the h2, s2 the phenotypes were drawn with, as the CPU baseline does)
    if not flags & clak.CLAK_CHOL:
        clak.clak_estimate_vc(plan.handle, Y, clak.CLAK_VC_REML)
    t3 = time.perf_counter()
    clak.clak_set_traits(plan.handle, Y, torch.from_numpy(w.h2).cuda(), torch.from_numpy(w.s2).cuda())
    t4 = time.perf_counter()
    t.update(eig_ms=(t1 - t0) * 1e3, covariates_ms=(t2 - t1) * 1e3, vc_reml_ms=(t3 - t2) * 1e3,
             traits_ms=(t4 - t3) * 1e3)
    return plan, t


def timed_steps(clak, torch, plan, G, b, se, block, steps, warmup, eager, pv=None):
    """(ms per step over the timed steps, per-stage kernel times).

    The step time comes from HIP events around `steps` passes (pipeline
    launches unless eager).  The per-stage times come from the library's stage
    profiler, which brackets every stage's kernel with HIP events on the
    stream that kernel runs on (its events add a few microseconds between
    launches, so the step time is taken from a first timed region without it):
    a second region of the same length runs the pipeline as the first did
    (CLAK_PROFILE_PIPELINED: per stage the mean launch duration as the
    pipeline overlaps it, and the busy time, the union of its launches'
    intervals, which never exceeds the step), a third, shorter one runs every
    kernel alone (CLAK_PROFILE_SERIAL: isolated launch durations)."""
    run = Pass(clak, plan, G, b, se, block, eager, pv)
    try:
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(steps):
            run()
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        clak.clak_plan_set_profiling(plan.handle, clak.CLAK_PROFILE_PIPELINED)
        ev0.record()
        for _ in range(steps):
            run()
        ev1.record()
        pipe = clak.clak_plan_get_profile(plan.handle)
        busy = clak.clak_plan_get_busy(plan.handle)
        torch.cuda.synchronize()
        ms_prof = ev0.elapsed_time(ev1) / steps  # the profiled passes' own step time (events add host work)
        serial_steps = max(1, min(steps, 3))
        clak.clak_plan_set_profiling(plan.handle, clak.CLAK_PROFILE_SERIAL)
        for _ in range(serial_steps):
            run()
        alone = clak.clak_plan_get_profile(plan.handle)
        clak.clak_plan_set_profiling(plan.handle, clak.CLAK_PROFILE_OFF)
    finally:
        run.close()
    prof = {}
    for k, (tot, n) in pipe.items():
        prof[k] = {"launches_per_step": n / steps,
                   "mean_launch_ms": tot / n if n else 0.0,        # in the pipeline (overlapped)
                   "busy_ms_per_step": busy[k] / steps,            # union of the launch intervals
                   "busy_share": busy[k] / steps / ms_prof,         # of the profiled pass's wall time
                   "isolated_launch_ms": alone[k][0] / alone[k][1] if alone[k][1] else 0.0}
    return ms, prof


KERNELS = {("rotate", "mixed"): ("k_rot_i8", "k_mixed.hip"), ("grid", "mixed"): ("k_grid_ring", "k_grid.hip"),
           ("rotate", "fp64"): ("k_rot64", "k_fp64.hip"), ("grid", "fp64"): ("k_grid64", "k_fp64.hip")}


def stage_kernel(stage, precision, pL, tuning):
    """(kernel name, source file) of a stage's launches: the mixed grid runs
    the one-pass ring kernel for p_L <= 3 unless the tuner picked a two-stage
    tile (grid_tt 32 or 64), which runs k_grid32."""
    if stage == "grid" and precision == "mixed" and (pL > 3 or (tuning and tuning.get("grid_tt"))):
        return ("k_grid32", "k_mixed.hip")
    return KERNELS.get((stage, precision))


TUNING_KEYS = ("rot_cfg", "rot_rg", "grid_tt", "grid_xt")


def tuning_tuple(tuning):
    """The four launch parameters (0: built-in) of a tuning dict, or of None."""
    return tuple(int((tuning or {}).get(k, 0)) for k in TUNING_KEYS)


def committed_traffic(stage, precision, pL, workload, tuning):
    """HBM bytes per launch of the stage's kernel from the committed rocprofv3
    summaries (FETCH_SIZE / WRITE_SIZE scaled by a 1 GiB copy), or None when
    none was taken from the current kernel source with this run's launch
    parameters (a line "tuning=builtin" stands for all four at 0)."""
    import glob
    import hashlib
    key = stage_kernel(stage, precision, pL, tuning)
    if key is None:
        return None
    kernel, src = key
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_1207_2169_amd", "csrc", src), "rb").read()).hexdigest()[:16]
    want = tuning_tuple(tuning)
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if "traffic_bytes_per_launch=" not in line:
                continue
            kv = dict(tok.split("=", 1) for tok in line.split() if "=" in tok)
            if kv.get("workload") != workload or kv.get("kernel") != kernel or kv.get("sha256_16") != sha:
                continue
            tv = kv.get("tuning", "builtin")
            got = (0, 0, 0, 0) if tv == "builtin" else tuning_tuple(dict(p.split(":") for p in tv.split(",")))
            if got == want:
                return float(kv["traffic_bytes_per_launch"])
    return None


def stage_flops(stage, w, block):
    """Algorithmic flops of one launch of a stage on a full block."""
    if stage == "rotate":
        f = 2.0 * w.n * w.n * block
        if w.t == 1:  # single trait: the linear sums (extra row tile) and d^T (x o x)
            f += 2.0 * w.n * block * (w.pL + 1) + 3.0 * w.n * block
        return f
    if stage == "grid":
        return 2.0 * w.n * block * w.t * (w.pL + 2)
    return None


def roofline(prof, w, block, precision, workload, tuning, ms_step):
    """Roofline of the stage that does the most work per step (launches per
    step x its isolated launch duration: where two streams overlap kernels,
    each is stretched by the other, so their in-pipeline busy times do not
    tell which does more work).

    achieved = algorithmic flops of one launch x launches per step / the
    stage's busy time per step.  The busy time is the stage's share of a
    pipelined profiled pass (the union of its launch intervals over that
    pass's wall time: the time during which at least one of its kernels ran)
    times the unprofiled step, so it never exceeds the step.  Beside it: the
    mean launch duration in the pipeline (what a rocprofv3 kernel trace of the
    same passes averages) and the isolated one."""
    dom = max((k for k in prof if prof[k]["launches_per_step"] > 0),
              key=lambda k: prof[k]["launches_per_step"] * prof[k]["isolated_launch_ms"])
    d = prof[dom]
    flops = stage_flops(dom, w, block)
    if flops is None:
        return None
    peak, peak_name = PEAK[precision]
    # the stage's share of the profiled pass, applied to the unprofiled step
    # (the profiler's events stretch the profiled pass; the share is what it
    # measures without that bias), per launch
    per_launch = d["busy_share"] * ms_step / d["launches_per_step"]
    achieved = flops / (per_launch * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": committed_traffic(dom, precision, w.pL, workload, tuning),
            "kernel": (stage_kernel(dom, precision, w.pL, tuning) or (dom,))[0], "avg_launch_ms": per_launch,
            "launches_per_step": d["launches_per_step"],
            "basis": "in-pipeline busy time per launch: the share of a pipelined profiled pass during which at "
                     "least one launch of the kernel ran (union of its launch intervals, HIP events on each launch's "
                     "own stream) x the unprofiled step time / launches per step",
            "busy_share_of_step": d["busy_share"],
            "mean_launch_ms_in_pipeline": d["mean_launch_ms"], "isolated_launch_ms": d["isolated_launch_ms"],
            "frac_isolated": flops / (d["isolated_launch_ms"] * 1e-3) / 1e12 / peak if d["isolated_launch_ms"] else None,
            "peak_source": peak_name}
    if precision == "mixed" and dom == "rotate":
        roof["issued_int8_ops_frac"] = 4 * achieved / peak  # four digit planes of Z^T per product
    if precision == "mixed" and dom == "grid":
        roof["issued_int8_ops_frac"] = GRID_PRODUCTS * achieved / peak  # digit products per algorithmic product
    return roof


def parity_sample(w, b_gpu, se_gpu, n_traits=20, n_snps=500, seed=8):
    """eps_b, eps_SE of the GPU outputs against the oracle on n_traits random
    traits x n_snps random SNPs of the workload (every pair), with the oracle's
    time on the host."""
    import oracle
    rng = np.random.default_rng(seed)
    traits = np.sort(rng.choice(w.t, min(n_traits, w.t), replace=False))
    snps = np.sort(rng.choice(w.m, min(n_snps, w.m), replace=False))
    ii, jj = np.meshgrid(np.arange(snps.size), traits, indexing="ij")
    G = np.concatenate([w.genotypes(int(s), 1) for s in snps]).T.astype(np.float64)
    t0 = time.perf_counter()
    rb, rv, rf = oracle.gls_cells(w.Phi, w.XL, G, w.Y, w.h2, w.s2, ii.ravel(), jj.ravel())
    dt = time.perf_counter() - t0
    rse = np.sqrt(rv[:, -1, -1])
    gb = b_gpu[jj.ravel(), snps[ii.ravel()]].astype(np.float64)
    gse = se_gpu[jj.ravel(), snps[ii.ravel()]].astype(np.float64)
    ok = rf == 0
    return {"eps_b": float(np.max(np.abs(gb[ok] - rb[ok, -1]) / rse[ok])),
            "eps_se": float(np.max(np.abs(gse[ok] - rse[ok]) / rse[ok])), "cells_checked": int(ok.sum()),
            "sample": f"{traits.size} random traits x {snps.size} random SNPs", "oracle_s": dt,
            "oracle_threads": oracle.threads()}


def cpu_baseline(w, b_gpu, se_gpu, target_s):
    """The oracle on a bounded sample of the same workload, timed on the host."""
    import oracle
    rng = np.random.default_rng(7)
    traits = rng.choice(w.t, size=min(w.t, 2), replace=False)

    def run(ncell):
        snp = rng.choice(w.m, size=ncell, replace=ncell > w.m)  # small workloads: cells repeat
        tr = np.resize(traits, ncell)
        uniq, inv = np.unique(snp, return_inverse=True)
        G = np.concatenate([w.genotypes(int(s), 1) for s in uniq]).T.astype(np.float64)
        t0 = time.perf_counter()
        rb, rv, rf = oracle.gls_cells(w.Phi, w.XL, G, w.Y, w.h2, w.s2, inv, tr)
        dt = time.perf_counter() - t0
        return snp, tr, rb, np.sqrt(rv[:, -1, -1]), rf, dt

    n_cells = 2000
    while True:
        snp, tr, rb, rse, rf, dt = run(n_cells)
        if dt >= 0.5 * target_s or n_cells >= 2_000_000:
            break
        n_cells = int(min(2_000_000, n_cells * max(2.0, min(50.0, target_s / max(dt, 1e-3)))))
    gb = b_gpu[tr, snp].astype(np.float64)
    gse = se_gpu[tr, snp].astype(np.float64)
    ok = rf == 0
    eps_b = float(np.max(np.abs(gb[ok] - rb[ok, -1]) / rse[ok]))
    eps_se = float(np.max(np.abs(gse[ok] - rse[ok]) / rse[ok]))
    return {
        "value": n_cells / dt,
        "unit": "cells/s",
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": f"{n_cells} random (SNP, trait) cells over {len(traits)} trait(s) of the same workload, "
                  f"per-trait Cholesky of M_j included; {dt:.1f} s on {platform.processor() or 'host'}",
    }, {"eps_b": eps_b, "eps_se": eps_se, "cells_checked": int(ok.sum())}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the grid shards over SNP blocks and "
              "trait groups with one broadcast of Z; only the one-GPU shard is implemented and measured here", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1207_2169_amd import clak
    from synth import make_workload

    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "c3":
        return run_cohorts(args, clak, torch)
    cfg, wname = WORKLOADS[args.workload]
    kw = {} if args.m is None else {"m": args.m}
    log(f"[bench] generating workload {args.workload}: {wname}")
    w = make_workload(cfg, **kw)
    block = w.block
    m = w.m
    G = upload_genotypes(w, m, torch, host=args.host_genotypes)
    b = torch.empty((w.t, m), dtype=torch.float32, device="cuda")
    se = torch.empty_like(b)
    pv = torch.empty_like(b) if args.pval else None
    log(f"[bench] n={w.n} p_L={w.pL} m={m} t={w.t} block={block} precision={args.precision}"
        + (" genotypes in pinned host memory" if args.host_genotypes else ""))

    plan, setup = make_plan(clak, torch, w, block, args.precision,
                            clak.CLAK_STAGE_GENOTYPES if (args.host_genotypes or args.stage_genotypes) else 0)
    tuning = None
    if not args.no_tune:
        t0 = time.perf_counter()
        source = tune(clak, plan.handle, G, b, se, block, args)
        setup["autotune_ms"] = (time.perf_counter() - t0) * 1e3
        tuning = dict(zip(TUNING_KEYS, clak.clak_plan_get_tuning(plan.handle)), source=source)
        log(f"[bench] tuned launch parameters {tuning}")
    ms, prof = timed_steps(clak, torch, plan, G, b, se, block, args.steps, args.warmup, args.eager, pv)
    cells = m * w.t
    log(f"[bench] {ms:.3f} ms/step, {cells / ms * 1e3:.4e} cells/s; stages {prof}")
    roof = roofline(prof, w, block, args.precision, args.workload, tuning, ms)
    out = {
        "metric": "GLS cells/sec (SNP x trait) at n=1000, p=4; mixed precision vs FP64",
        "value": cells / (ms * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8" if args.precision == "mixed" else "f64",
        "data": "synthetic (seeded generators; genotypes " + ("in pinned host memory, copied block by block over "
                "PCIe by the copy engine on the ingest stream)" if args.host_genotypes else "resident in HBM)"),
        "config": {"workload": wname, "n": w.n, "p_L": w.pL, "p": w.pL + 1, "m": m, "t": w.t, "block": block,
                   "precision": args.precision, "parallelism": "single GPU", "tuning": tuning,
                   "outputs": "b, SE, p-value" if args.pval else "b, SE"},
        "roofline": roof,
        "stage_busy_ms_per_step": {k: v["busy_ms_per_step"] for k, v in prof.items()},
        "launch": "per-block clak_run_block calls, one stream" if args.eager else
                  "clak_pipeline_launch: ingest on a side stream overlapped with rotation",
        "setup_ms": setup,
    }
    b_h = b.cpu().numpy()
    se_h = se.cpu().numpy()

    if not args.no_compare and args.precision == "mixed":
        plan.close()
        torch.cuda.empty_cache()
        p64, _ = make_plan(clak, torch, w, block, "fp64")
        ms64, prof64 = timed_steps(clak, torch, p64, G, b, se, block, max(1, min(args.steps, 3)), 1, args.eager,
                                   pv)
        p64.close()
        out["fp64_plain"] = {"value": cells / (ms64 * 1e-3), "ms_per_step": ms64,
                             "stage_busy_ms_per_step": {k: v["busy_ms_per_step"] for k, v in prof64.items()},
                             "roofline": roofline(prof64, w, block, "fp64", args.workload, None, ms64)}
        out["mixed_over_fp64"] = ms64 / ms
        log(f"[bench] FP64 plain path: {ms64:.3f} ms/step")

    if not args.no_compare and w.t == 1:
        # the single-trait CLAK-Chol route on the same inputs (cross-check and
        # comparison; the headline line above is CLAK-Eig)
        torch.cuda.empty_cache()
        pc, setup_c = make_plan(clak, torch, w, block, args.precision, clak.CLAK_CHOL)
        bc, sc = torch.empty_like(b), torch.empty_like(se)
        if not args.no_tune:
            tune(clak, pc.handle, G, bc, sc, block, args)
        msc, profc = timed_steps(clak, torch, pc, G, bc, sc, block, args.steps, args.warmup, args.eager, pv)
        pc.close()
        zc = (bc.double() - b.double()).abs() / se.double()
        out["clak_chol"] = {"value": cells / (msc * 1e-3), "ms_per_step": msc,
                            "stage_busy_ms_per_step": {k: v["busy_ms_per_step"] for k, v in profc.items()},
                            "setup_ms": {k: v for k, v in setup_c.items() if k != "vc_reml_ms"},
                            "max_abs_diff_vs_eig_in_se_units": float(zc.max().item())}
        log(f"[bench] CLAK-Chol: {msc:.3f} ms/step, max |b_chol - b_eig| / SE = {zc.max().item():.3e}")

    if args.bed:
        import tempfile

        from synth import write_bed
        path = os.path.join(tempfile.gettempdir(), f"clak_bench_{os.getpid()}.bed")
        t0 = time.perf_counter()
        nbytes = write_bed(path, w, m)
        log(f"[bench] wrote {nbytes / 1e6:.0f} MB of 2-bit genotype rows in {time.perf_counter() - t0:.1f} s")
        try:
            torch.cuda.empty_cache()
            pb, _ = make_plan(clak, torch, w, block, args.precision,
                              clak.CLAK_STAGE_GENOTYPES if args.stage_genotypes else 0)
            if not args.no_tune:
                tune(clak, pb.handle, G, b, se, block, args)
            bb, sb = torch.empty_like(b), torch.empty_like(se)

            h = clak.clak_bed_open(path, w.n, m, block, args.bed_depth)
            try:
                clak.clak_bed_scan(h, pb.handle, bb, sb)  # warm: the file is now in the page cache
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                reps = max(1, min(args.steps, 5))
                for _ in range(reps):
                    clak.clak_bed_scan(h, pb.handle, bb, sb)
                msb = (time.perf_counter() - t0) / reps * 1e3
            finally:
                clak.clak_bed_close(h)
            pb.close()
            same = bool(torch.equal(torch.nan_to_num(bb), torch.nan_to_num(b))) if args.precision == "mixed" \
                and args.no_compare else None
            out["ooc_bed"] = {"value": cells / (msb * 1e-3), "unit": "cells/s", "ms_per_step": msb,
                              "file_bytes": nbytes, "reader_depth": args.bed_depth, "reps": reps,
                              "bitwise_equal_to_resident_run": same,
                              "staged_by_copy_engine": bool(args.stage_genotypes),
                              "note": "host wall clock per scan of the whole file (reader opened once); file in "
                                      "the host page cache; 2-bit rows from pinned host buffers over PCIe"}
            log(f"[bench] out-of-core 2-bit file scan: {msb:.3f} ms/step, {cells / msb * 1e3:.4e} cells/s")
        finally:
            os.remove(path)

    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        cb, err = cpu_baseline(w, b_h, se_h, args.cpu_seconds)
        out["cpu_baseline"] = cb
        out["parity_sample"] = err
    if args.workload == "c1" and not args.no_c2 and args.m is None:
        del G, b, se, pv
        torch.cuda.empty_cache()
        out["c2"] = multi_trait_record(args, clak, torch)
    print(json.dumps(out), flush=True)


def multi_trait_record(args, clak, torch):
    """The multi-trait workload (n=1000, p=4, m=1e5 in blocks of 1e4,
    t=1000: the configuration the metric is quoted on for many traits) timed
    like the headline: its rate, its dominant kernel's roofline, and the
    oracle's agreement on 20 random traits x 500 random SNPs."""
    from synth import make_workload
    cfg, wname = WORKLOADS["c2"]
    log(f"[bench] multi-trait sub-record: {wname}")
    w = make_workload(cfg)
    G = upload_genotypes(w, w.m, torch)
    b = torch.empty((w.t, w.m), dtype=torch.float32, device="cuda")
    se = torch.empty_like(b)
    plan, setup = make_plan(clak, torch, w, w.block, args.precision)
    tuning = None
    if not args.no_tune:
        source = tune(clak, plan.handle, G, b, se, w.block, args)
        tuning = dict(zip(TUNING_KEYS, clak.clak_plan_get_tuning(plan.handle)), source=source)
    ms, prof = timed_steps(clak, torch, plan, G, b, se, w.block, args.steps, args.warmup, args.eager)
    plan.close()
    cells = w.m * w.t
    log(f"[bench] multi-trait: {ms:.3f} ms/step, {cells / ms * 1e3:.4e} cells/s")
    rec = {"workload": wname, "value": cells / (ms * 1e-3), "unit": "cells/s", "ms_per_step": ms,
           "steps": args.steps, "warmup": args.warmup, "dtype": "i8" if args.precision == "mixed" else "f64",
           "config": {"n": w.n, "p_L": w.pL, "p": w.pL + 1, "m": w.m, "t": w.t, "block": w.block,
                      "precision": args.precision, "tuning": tuning},
           "roofline": roofline(prof, w, w.block, args.precision, "c2", tuning, ms),
           "stage_busy_ms_per_step": {k: v["busy_ms_per_step"] for k, v in prof.items()},
           "setup_ms": setup}
    rec["parity_sample"] = parity_sample(w, b.cpu().numpy(), se.cpu().numpy())
    log(f"[bench] multi-trait parity {rec['parity_sample']}")
    del G, b, se
    torch.cuda.empty_cache()
    return rec


def run_cohorts(args, clak, torch):
    """The batched configuration: eight cohorts of uneven n and t, each a plan
    with its own kinship eigendecomposition, submitted as one clak_batch
    launch (rounds of one SNP block per cohort, each round one launch per
    kernel over all cohorts).  A step is one launch over all cohorts."""
    from synth import cohort_workloads
    _, wname = WORKLOADS["c3"]
    log(f"[bench] generating workload c3: {wname}")
    ws = cohort_workloads(m=args.m or 50_000)
    plans, blocks, outs, setup = [], [], [], {}
    for w in ws:
        G = upload_genotypes(w, w.m, torch)
        b = torch.empty((w.t, w.m), dtype=torch.float32, device="cuda")
        se = torch.empty_like(b)
        plan, st = make_plan(clak, torch, w, C3_BLOCK, args.precision)
        if not args.no_tune:
            tune(clak, plan.handle, G, b, se, C3_BLOCK, args)
        for k, v in st.items():
            setup[k] = setup.get(k, 0.0) + v
        plans.append(plan)
        blocks.append(block_list(G, b, se, C3_BLOCK))
        outs.append((G, b, se))
        log(f"[bench]   cohort n={w.n} t={w.t} m={w.m}")
    handles = [p.handle for p in plans]
    batch = clak.clak_batch_create(handles, blocks)
    batch_info = clak.clak_batch_get_info(batch)
    try:
        for _ in range(args.warmup):
            clak.clak_batch_launch(batch)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(args.steps):
            clak.clak_batch_launch(batch)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        for h in handles:
            clak.clak_plan_set_profiling(h, clak.CLAK_PROFILE_PIPELINED)
        for _ in range(args.steps):
            clak.clak_batch_launch(batch)
        profs = [clak.clak_plan_get_profile(h) for h in handles]
        busys = [clak.clak_plan_get_busy(h) for h in handles]
        for h in handles:
            clak.clak_plan_set_profiling(h, clak.CLAK_PROFILE_OFF)
    finally:
        clak.clak_batch_destroy(batch)
    cells = sum(w.m * w.t for w in ws)
    log(f"[bench] {ms:.3f} ms/step, {cells / ms * 1e3:.4e} cells/s over {len(ws)} cohorts")
    # the cohorts' kernels run concurrently, so the roofline takes all the
    # algorithmic MFMA work of a step (rotations and grid contractions of
    # every cohort) over the step's wall time
    flops = sum(2.0 * w.n * w.n * w.m + 2.0 * w.n * w.m * w.t * (w.pL + 2) for w in ws)
    peak, peak_name = PEAK[args.precision]
    achieved = flops / (ms * 1e-3) / 1e12
    out = {
        "metric": "GLS cells/sec (SNP x trait), batched uneven cohorts; mixed precision",
        "value": cells / (ms * 1e-3), "unit": "cells/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i8" if args.precision == "mixed" else "f64",
        "data": "synthetic (seeded generators; genotypes resident in HBM)",
        "config": {"workload": wname, "cohorts": [{"n": w.n, "t": w.t, "m": w.m} for w in ws], "block": C3_BLOCK,
                   "precision": args.precision, "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None, "kernel": "k_rot_i8 + k_grid_ring (all cohorts)",
                     "basis": "rotation and grid flops of all cohorts per step / wall time of the step",
                     "peak_source": peak_name},
        "stage_launch_ms_summed_over_cohorts": {k: sum(p[k][0] for p in profs) / args.steps for k in profs[0]},
        "stage_busy_ms_per_cohort": [{k: v / args.steps for k, v in bz.items()} for bz in busys],
        "launch": ("clak_batch_launch: rounds of one block per cohort, each round one launch per kernel over all "
                   "cohorts (costliest first), on three streams" if batch_info[0] else
                   "clak_batch_launch: rounds of one block per cohort, per-cohort launches, on three streams"),
        "batch": {"batched": batch_info[0], "rounds": batch_info[1], "streams": batch_info[2]},
        "setup_ms": setup,
    }
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline (largest cohort)")
        wl = max(range(len(ws)), key=lambda c: ws[c].n)
        cb, err = cpu_baseline(ws[wl], outs[wl][1].cpu().numpy(), outs[wl][2].cpu().numpy(), args.cpu_seconds)
        out["cpu_baseline"] = cb
        out["parity_sample"] = err
    for p in plans:
        p.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
