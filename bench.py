"""Benchmark of the batched pentadiagonal solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Default workload ``hyperdiff``: 1-D hyperdiffusion, backward Euler,
A = I + 50*D4 with N = 4096, 65536 independent systems (C^0 uniform[-1, 1),
seed 2), factor once, every step solves A C^{k+1} = C^k in place.  A step is
one full solve of all 65536 systems; inputs are resident in HBM before the
timed region.  Prints one JSON line.

The same line carries a ``configs`` object with every other configuration,
each timed in this run and followed by its status check (a single-pass wait
that ran out makes the run fail): the plain N=256 solve, the 2-D
Cahn-Hilliard run, the precision comparison (FP64 sweeps against FP32
right-hand-side streams with 0 and 1 refinement steps, N=8192, 131072
right-hand sides, sigma in {1, 1e2, 1e4}), the 48-matrix group run,
periodic Crank-Nicolson, per-system matrices against rocSPARSE, and the copy
ceiling.  ``--headline-only`` skips them.

Other workloads (for tuning runs): ``plain`` (N=256, 256 RHS), ``precision``
(all three sigma), ``shape`` (any n / batch), ``copy`` (device copy),
``group`` (48 matrices, 200 graph-captured steps, persistent launch vs one
solve per matrix), ``cahn2d`` (2-D split-implicit Cahn-Hilliard, 1024^2 x 32),
``periodic`` (periodic Crank-Nicolson hyperdiffusion, N=4096, 65536 systems),
``rewrite`` (a matrix per system refactored every call, against rocSPARSE's
batched pentadiagonal QR solver).
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RHS-solves/s and HBM GB/s (% peak), FP32+refine vs FP64 at rel resid 1e-12"
PEAK_HBM_GBS = 8000.0
BYTES_PER_UNKNOWN_FP64 = 16  # read f once, write x once


SCHEDULE_NAMES = {1: "lane", 2: "partitioned", 3: "tile", 4: "onepass"}


# kernel source file of each schedule (the counters go stale when it changes)
SCHEDULE_SOURCES = {"lane": ("sweep.hip",), "partitioned": ("sweep.hip",), "tile": ("tile.hip",),
                    "onepass": ("onepass.hip", "lookback.h")}


def kernel_source_hash(names) -> str:
    """Hash of the kernel sources with comments and blank lines removed, so
    that a comment-only edit keeps the counters taken on the same code."""
    h = hashlib.sha256()
    for name in (names,) if isinstance(names, str) else names:
        with open(os.path.join(ROOT, "paper_1807_07382_amd", "csrc", name)) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        lines = (re.sub(r"//.*", "", line).rstrip() for line in text.splitlines())
        h.update("\n".join(line for line in lines if line).encode())
    return h.hexdigest()[:16]


def traffic_for(kernel: str, workload: str, sources=None):
    """HBM bytes moved by one step (all kernels of one step) from the
    committed rocprofv3 counter summary, if it was taken on the current kernel
    sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(f"{kernel}@{workload}")
    if sources is None:
        sources = SCHEDULE_SOURCES["".join(c for c in kernel if not c.isdigit())]
    if not rec or rec.get("source_hash") != kernel_source_hash(sources):
        return None
    return rec.get("bytes_per_step")


def cpu_baseline_hyperdiff(n, sigma, C0, budget_s=12.0):
    """The oracle (as it is) on the host cores, on a bounded column sample."""
    import oracle
    from oracle import workloads  # noqa: F401
    cols = 8192
    sample = np.ascontiguousarray(C0[:, :cols])
    dg = oracle.assemble_d4(n, sigma)
    fac = oracle.factor(dg)
    X = sample.copy()
    oracle.solve_inplace(dg, fac, X)  # warm-up
    steps = 0
    t0 = time.perf_counter()
    while True:
        oracle.solve_inplace(dg, fac, X)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return dict(value=cols * steps / el, unit="RHS-solves/s", cores=oracle.threads(),
                kind="oracle",
                sample=f"{cols} of the {C0.shape[1]} systems (N={n}), {steps} backward-Euler "
                       f"steps, {el:.1f} s, OpenMP over systems; factorisation excluded")


def run_hyperdiff(args, torch):
    from paper_1807_07382_amd import inputs
    from paper_1807_07382_amd import pentbatch as pb
    import oracle
    from oracle import workloads

    cfg = inputs.HYPERDIFF
    n, sigma, batch = cfg["n"], cfg["sigma"], cfg["batch"]
    w = inputs.hyperdiff()
    C0 = w["C0"]
    probe = np.array([0, 1, 63, 64, 4095, 31337, batch - 1])
    probe0 = C0[:, probe].copy()
    T = torch.from_numpy(C0).cuda()
    stream = torch.cuda.current_stream()
    # factorisation (excluded from the timed steps, as in the paper): the
    # first call also loads the library's device code; the second is the
    # cost of a factorisation (allocation, assembly, the serial recurrence,
    # the sweep and segment tables, one synchronisation)
    t_fac0 = time.perf_counter()
    pb.Plan.factor_d4(n, sigma).close()
    fac_cold_s = time.perf_counter() - t_fac0
    t_fac0 = time.perf_counter()
    plan = pb.Plan.factor_d4(n, sigma)
    fac_s = time.perf_counter() - t_fac0
    if args.schedule:
        kind, seg = (int(x) for x in args.schedule.split(","))
        plan.set_schedule(kind, seg)
    sched = plan.schedule_for(batch)
    for _ in range(args.warmup):
        plan.solve_(T, stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        plan.solve_(T, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    plan.check()  # raises if a single-pass wait ran out (its values would be NaN)
    # parity of the probe systems after all warmup + timed steps
    X = T[:, torch.from_numpy(probe).cuda()].cpu().numpy()
    ref = workloads.hyperdiffusion(n, sigma, probe0, args.warmup + args.steps)
    err = float(np.max(np.max(np.abs(X - ref), axis=0) / np.max(np.abs(ref), axis=0)))
    plan.close()
    ms_step = ms / args.steps
    solves_s = batch * args.steps / (ms / 1e3)
    alg_bytes = BYTES_PER_UNKNOWN_FP64 * n * batch
    achieved = alg_bytes / (ms_step / 1e3) / 1e9
    sched_name = SCHEDULE_NAMES[sched[0]] + (f"{sched[1]}" if sched[0] in (2, 4) else "")
    tr = traffic_for(sched_name, "hyperdiff")
    out = dict(
        metric=METRIC, value=solves_s, unit="RHS-solves/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=ms_step, higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload="hyperdiff", n=n, systems=batch, sigma=sigma,
                    implicit_steps=args.steps, layout="interleaved (batch-fastest)",
                    parallelism="single GPU", schedule=sched_name),
        roofline=dict(bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS, unit="GB/s",
                      frac=achieved / PEAK_HBM_GBS,
                      traffic=tr),
        row_updates_per_s=solves_s * n,
        factor_ms=fac_s * 1e3,
        factor_first_call_ms=fac_cold_s * 1e3,
        parity=dict(probe_systems=len(probe), max_rel_err_vs_oracle=err),
    )
    del T
    torch.cuda.empty_cache()
    if not args.headline_only:
        out["configs"] = all_configs(args, torch)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_hyperdiff(n, sigma, C0)
    return out


def _sub(args, **kw):
    ns = argparse.Namespace(**vars(args))
    ns.schedule = ""
    for k, v in kw.items():
        setattr(ns, k, v)
    return ns


def _roof(r):
    rf = r.get("roofline")
    if not rf:
        return None
    return {k: rf[k] for k in ("achieved", "frac", "traffic") if k in rf}


def all_configs(args, torch):
    """Every other configuration of the benchmark set, compact: the small
    plain solve, the 2-D Cahn-Hilliard run, the precision comparison at the
    three sigmas, the 48-matrix group run, periodic Crank-Nicolson, per-system
    matrices against rocSPARSE, and the copy ceiling measured in the same
    run.  Each timed loop is followed by the handle's status check."""
    res = {}
    r = run_plain(_sub(args, steps=200, warmup=5), torch)
    res["plain"] = dict(us_per_solve=r["ms_per_step"] * 1e3, solves_per_s=r["value"],
                        schedule=r["config"]["schedule"], parity=r["parity"])
    r = run_cahn2d(_sub(args, steps=50, warmup=2), torch)
    res["cahn2d"] = dict(steps=r["steps"], ms_per_step=r["ms_per_step"], solves_per_s=r["value"],
                         roofline=_roof(r), parity=r["parity"])
    prec = {}
    for sg in (1.0, 1e2, 1e4):
        prec[f"sigma={sg:g}"] = precision_compare(torch, sg)
    # HBM bytes of one FP32-stream solve (k = 0) at N = 8192 x 131072 from the
    # committed counters, against its 12 B per unknown
    prec["fp32_stream_refine0_traffic"] = traffic_for("onepass64_f32", "precision",
                                                      ("onepass.hip", "lookback.h"))
    prec["note"] = ("FP32 is the storage precision of the right-hand-side stream; the factors, "
                    "every operation and x are FP64, so the k=0 solve already has FP64 accuracy "
                    "(same eta as the FP64 solve) and is the form that beats FP64 (12 instead of "
                    "16 B per unknown); a correction adds a second pass over x")
    res["precision"] = prec
    r = run_group(_sub(args, steps=200, warmup=1), torch)
    res["group"] = dict(graph_steps=r["steps"], ms_per_step=r["ms_per_step"],
                        solves_per_s=r["value"], roofline=_roof(r),
                        unknowns_per_step=r["config"]["unknowns_per_step"],
                        kernel_variant=r["config"]["kernel_variant"],
                        max_rel_err_vs_oracle=r["persistent"]["max_rel_err_vs_oracle"],
                        per_matrix_ms_per_step=r["per_matrix"]["ms_per_step"],
                        speedup_of_persistent=r["per_matrix"]["speedup_of_persistent"])
    r = run_periodic(_sub(args, steps=100, warmup=3), torch)
    res["periodic"] = dict(ms_per_step=r["ms_per_step"], solves_per_s=r["value"],
                           form=r["config"]["form"], roofline=_roof(r), parity=r["parity"],
                           other_form=r["other_form"])
    r = run_rewrite(_sub(args, steps=20, warmup=2), torch)
    g = r["rocsparse_gpsv"] or {}
    res["rewrite"] = dict(ms_per_step=r["ms_per_step"], solves_per_s=r["value"],
                          roofline_56B=_roof(r), roofline_104B=r["kernel_plan_roofline"],
                          parity=r["parity"],
                          rocsparse_gpsv_ms_with_restore=g.get("ms_per_step_with_restore"),
                          rocsparse_gpsv_ms_solve_only=g.get("ms_solve_only"),
                          speedup_over_rocsparse=g.get("speedup_of_rewrite"))
    res["hyperdiff_tiled_layout"] = tiled_layout(torch)
    res["copy_ceiling"] = copy_ceiling(torch)
    return res


def tiled_layout(torch, steps=50):
    """The hyperdiffusion solve (N = 4096, 65536 systems) with each
    64-system tile its own contiguous interleaved block (pent_solve_tiled):
    ms per solve, and the bits of every system against the ordinary layout
    after one solve."""
    import ctypes
    from paper_1807_07382_amd import inputs
    from paper_1807_07382_amd import pentbatch as pb
    n, batch, sigma = inputs.HYPERDIFF["n"], inputs.HYPERDIFF["batch"], inputs.HYPERDIFF["sigma"]
    g = torch.Generator(device="cuda")
    g.manual_seed(2)
    F = torch.empty((n, batch), dtype=torch.float64, device="cuda").uniform_(-1, 1, generator=g)
    T = F.reshape(n, batch // 64, 64).permute(1, 0, 2).contiguous()
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    L = pb.lib()
    with pb.Plan.factor_d4(n, sigma) as plan:
        def solve():
            st = L.pent_solve_tiled(plan.handle, ctypes.c_void_p(T.data_ptr()), batch, 64, n * 64, sp)
            if st != pb.OK:
                raise pb.PentError(st, "solve_tiled")
        solve()
        plan.solve_(F, stream)
        torch.cuda.synchronize()
        same = bool(torch.equal(T.permute(1, 0, 2).reshape(n, batch), F))
        ms = _timed(torch, stream, solve, steps)
        plan.check()
    gbs = BYTES_PER_UNKNOWN_FP64 * n * batch / (ms / 1e3) / 1e9
    del F, T
    torch.cuda.empty_cache()
    return dict(ms_per_solve=ms, solves_per_s=batch / (ms / 1e3), achieved_GBs=gbs,
                frac=gbs / PEAK_HBM_GBS, bits_equal_interleaved=same)


def copy_ceiling(torch, reps=20):
    """Read+write bandwidth of plain copies of the hyperdiffusion state (2
    GiB, FP64) in this run: torch's device copy, the library's copy through
    the single pass's blocks (64 systems x 64 rows per wave, four waves down
    the rows, in place), and the same copy with other workgroup shapes."""
    from paper_1807_07382_amd import inputs
    from paper_1807_07382_amd import pentbatch as pb
    n, batch = inputs.HYPERDIFF["n"], inputs.HYPERDIFF["batch"]
    src = torch.empty((n, batch), dtype=torch.float64, device="cuda").uniform_()
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    nbytes = 2 * src.numel() * 8
    out = {}
    dst.copy_(src)
    ms = _timed(torch, stream, lambda: dst.copy_(src), reps)
    out["torch_copy_GBs"] = nbytes / (ms / 1e3) / 1e9
    pb.stream_copy(dst, dst, stream)
    ms = _timed(torch, stream, lambda: pb.stream_copy(dst, dst, stream), reps)
    out["single_pass_blocks_GBs"] = nbytes / (ms / 1e3) / 1e9
    # the same copy with other workgroup shapes (tiles side by side x waves
    # down): what the block shape alone does to the bandwidth on this layout
    for ta, wd in ((1, 2), (2, 2), (2, 1), (4, 1)):
        pb.stream_copy_shaped(dst, dst, ta, wd, stream)
        ms = _timed(torch, stream, lambda: pb.stream_copy_shaped(dst, dst, ta, wd, stream), reps)
        out[f"blocks_{ta}_across_{wd}_down_GBs"] = nbytes / (ms / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return out


def _timed(torch, stream, fn, reps):
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(reps):
        fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps


def precision_compare(torch, sigma, reps=10, seed=4):
    """FP64 sweeps against FP32 right-hand-side streams (FP64 arithmetic,
    0 and 1 refinement steps) on the precision workload: N=8192, 131072
    right-hand sides uniform[-1, 1) rounded to FP32 (drawn on the device from
    a seeded generator).  Reports solves/s, algorithmic bytes per unknown of
    the schedule in use, the largest device backward error and the largest
    error against the oracle on sampled systems."""
    from paper_1807_07382_amd import inputs
    from paper_1807_07382_amd import pentbatch as pb
    import oracle
    n, m = inputs.PRECISION["n"], inputs.PRECISION["batch"]
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    F64src = torch.empty((n, m), dtype=torch.float64, device="cuda").uniform_(-1, 1, generator=g)
    F32 = F64src.float()
    del F64src
    F64 = F32.double()
    X = torch.empty((n, m), dtype=torch.float64, device="cuda")
    eta = torch.empty(m, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    cols = torch.arange(0, m, m // 16, device="cuda")
    f_sample = F32[:, cols].double().cpu().numpy()
    ref = oracle.solve(oracle.assemble_d4(n, sigma), f_sample)
    out = dict(workload="precision", n=n, systems=m, sigma=sigma)
    with pb.Plan.factor_d4(n, sigma) as plan:
        # bytes per unknown of one solve: the single pass reads f once, the
        # partitioned sweep twice; x is written once (FP64)
        one = plan.schedule_for(m)[0] == 4
        solve64, solve32 = (16, 12) if one else (24, 16)
        # one correction: fused on the single pass (f and x in, x read again
        # and written: 4 + 8 + 8 + 8), else residual (f, x in; r out: 20) +
        # correction solve + x += d (24)
        refine1 = solve32 + (28 if one else 20 + solve64 + 24)
        out["schedule"] = "single pass" if one else "partitioned"
        nbytes = plan.mixed_workspace_size(m, 1, True)
        work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")

        def rel_err(T):
            Xs = T[:, cols].cpu().numpy()
            return float(np.max(np.max(np.abs(Xs - ref), axis=0) / np.max(np.abs(ref), axis=0)))

        # FP64: out-of-place solve X = A^{-1} F64 (copy + in-place solve would add a pass)
        ms64 = _timed(torch, stream, lambda: plan.solve_mixed(F64, X, work=work, stream=stream), reps)
        plan.solve_mixed(F64, X, eta=eta, work=work, stream=stream)
        torch.cuda.synchronize()
        out["fp64"] = dict(ms=ms64, solves_per_s=m / (ms64 / 1e3), bytes_per_unknown=solve64,
                           max_eta=float(eta.max()), max_rel_err_vs_oracle=rel_err(X))
        for k in (0, 1):
            ms = _timed(torch, stream,
                        lambda: plan.solve_mixed(F32, X, refine_steps=k, work=work, stream=stream),
                        reps)
            plan.solve_mixed(F32, X, refine_steps=k, eta=eta, work=work, stream=stream)
            torch.cuda.synchronize()
            out[f"fp32_stream_refine{k}"] = dict(
                ms=ms, solves_per_s=m / (ms / 1e3), bytes_per_unknown=solve32 if k == 0 else refine1,
                max_eta=float(eta.max()), max_rel_err_vs_oracle=rel_err(X),
                speedup_vs_fp64=ms64 / ms)
        plan.check()
    del F32, F64, X, work
    torch.cuda.empty_cache()
    return out


def run_precision(args, torch):
    from paper_1807_07382_amd import inputs
    res = [precision_compare(torch, s) for s in inputs.PRECISION["sigmas"]]
    best = res[1]["fp32_stream_refine0"]
    return dict(metric=METRIC, value=best["solves_per_s"], unit="RHS-solves/s", n_gpus=1,
                steps=10, warmup=0, ms_per_step=best["ms"], higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="f32-stream/f64", data="synthetic",
                config=dict(workload="precision", n=inputs.PRECISION["n"],
                            systems=inputs.PRECISION["batch"]),
                per_sigma=res)


def run_group(args, torch):
    """48 matrices I + sigma_k*D4 (sigma_k, N_k, R_k log-uniform, seed 5),
    every step solves all of them in place (backward Euler); 200 steps are
    captured into one HIP graph.  Persistent single launch per step (kernel
    variant autotuned) against one solve per matrix (schedules autotuned)."""
    from paper_1807_07382_amd import inputs
    from paper_1807_07382_amd import pentbatch as pb
    from oracle import workloads
    steps = args.steps if args.steps != 100 else inputs.GROUP["steps"]
    mats = inputs.group()
    plans = [pb.Plan.factor_d4(F.shape[0], sg) for sg, F in mats]
    # each matrix's block with its rows padded to whole 128-byte lines (ld a
    # multiple of 16 doubles; PENT_GROUP_LD_PAD overrides, for comparisons),
    # so no 64-system row segment straddles a line it only partly uses
    pad = int(os.environ.get("PENT_GROUP_LD_PAD", "16"))
    Ts = []
    for _, F in mats:
        ld = (F.shape[1] + pad - 1) // pad * pad
        T = torch.zeros((F.shape[0], ld), dtype=torch.float64, device="cuda")
        T[:, :F.shape[1]].copy_(torch.from_numpy(F))
        Ts.append(T[:, :F.shape[1]])
    probe = [(k, np.unique([0, F.shape[1] - 1])) for k, (_, F) in enumerate(mats)]
    init = [T.clone() for T in Ts]
    unknowns = sum(F.shape[0] * F.shape[1] for _, F in mats)
    systems = sum(F.shape[1] for _, F in mats)
    g = pb.Group(plans)
    variant, tune_ms = g.autotune(Ts)
    for p, (_, F) in zip(plans, mats):
        p.autotune(F.shape[1])
    s = torch.cuda.Stream()
    res = {}
    for mode in (pb.GROUP_FP64, pb.GROUP_PER_MATRIX):
        for T, I in zip(Ts, init):
            T.copy_(I)
        torch.cuda.synchronize()
        graph = g.capture(Ts, steps=steps, mode=mode, stream=s)
        graph.launch(stream=s)                     # warm-up replay
        s.synchronize()
        for T, I in zip(Ts, init):
            T.copy_(I)
        torch.cuda.synchronize()
        ms = _timed(torch, s, lambda: graph.launch(stream=s), 1)
        g.check()
        # parity: the state after one replay (= steps implicit steps)
        errs = []
        for k, cols in probe:
            sigma, F = mats[k]
            ref = workloads.group_run([(sigma, np.ascontiguousarray(F[:, cols]))], steps)[0]
            X = Ts[k][:, torch.from_numpy(cols).cuda()].cpu().numpy()
            den = np.maximum(np.max(np.abs(ref), axis=0), 1e-300)
            errs.append(float(np.max(np.max(np.abs(X - ref), axis=0) / den)))
        graph.close()
        res[mode] = dict(ms=ms, max_rel_err_vs_oracle=max(errs))
    g.close()
    ms_step = res[pb.GROUP_FP64]["ms"] / steps
    gbs = BYTES_PER_UNKNOWN_FP64 * unknowns / (ms_step / 1e3) / 1e9
    return dict(metric=METRIC, value=systems * steps / (res[pb.GROUP_FP64]["ms"] / 1e3), unit="RHS-solves/s",
                n_gpus=1, steps=steps, warmup=1, ms_per_step=ms_step, higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
                config=dict(workload="group", matrices=len(mats), unknowns_per_step=unknowns,
                            systems=systems, graph_steps=steps, kernel_variant=variant,
                            layout=f"interleaved per matrix, ld rounded up to a multiple of {pad}"),
                roofline=dict(bound="hbm", achieved=gbs, peak=PEAK_HBM_GBS, unit="GB/s",
                              frac=gbs / PEAK_HBM_GBS,
                              traffic=traffic_for("group_onepass64", "group",
                                                  ("onepass.hip", "lookback.h"))
                              if variant == 1 else None),
                persistent=res[pb.GROUP_FP64],
                per_matrix=dict(res[pb.GROUP_PER_MATRIX],
                                ms_per_step=res[pb.GROUP_PER_MATRIX]["ms"] / steps,
                                speedup_of_persistent=res[pb.GROUP_PER_MATRIX]["ms"] / res[pb.GROUP_FP64]["ms"]))


def run_cahn2d(args, torch):
    """2-D split-implicit Cahn-Hilliard: 1024 x 1024 grid, 32 instances,
    sigma = 200, 50 steps; every step = 32768 x sweeps (system-major, the
    explicit stencil formed inside the sweep kernel) and 32768 y sweeps
    (batch-fastest), N = 1024."""
    from paper_1807_07382_amd import inputs
    from paper_1807_07382_amd import pentbatch as pb
    from oracle import workloads
    w = inputs.cahn2d()
    n, ninst, sigma = w["nx"], w["ninst"], w["sigma"]
    steps = args.steps if args.steps != 100 else inputs.CAHN2D["steps"]
    h = 1.0 / n
    gam = w["gammas"]
    dt = torch.from_numpy(sigma * h ** 4 / gam).cuda()
    C0 = torch.from_numpy(w["C0"]).cuda()
    C = C0.clone()
    R = torch.empty_like(C)
    stream = torch.cuda.current_stream()
    plan = pb.Plan.factor_d4(n, sigma)
    for _ in range(args.warmup):
        pb.ch2d_step(plan, plan, C, R, dt, h, stream)
    C.copy_(C0)
    ms = _timed(torch, stream, lambda: pb.ch2d_step(plan, plan, C, R, dt, h, stream), steps)
    plan.check()
    # parity of one instance after `steps` steps
    sub = np.ascontiguousarray(w["C0"][:, :1, :])
    ref = workloads.ch_run(sub, gam[:1], sigma, steps)
    err = float(np.max(np.abs(C[:, :1, :].cpu().numpy() - ref)) / np.max(np.abs(ref)))
    plan.close()
    points = n * n * ninst
    # two passes: x sweeps (C in, the explicit term formed in the kernel,
    # R out) and y sweeps (R in, C out)
    alg = 2 * BYTES_PER_UNKNOWN_FP64 * points
    gbs = alg / (ms / 1e3) / 1e9
    return dict(metric=METRIC, value=2 * n * ninst / (ms / 1e3), unit="RHS-solves/s", n_gpus=1,
                steps=steps, warmup=args.warmup, ms_per_step=ms, higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
                config=dict(workload="cahn2d", grid=[n, n], instances=ninst, sigma=sigma),
                roofline=dict(bound="hbm", achieved=gbs, peak=PEAK_HBM_GBS, unit="GB/s",
                              frac=gbs / PEAK_HBM_GBS,
                              traffic=traffic_for("ch2d", "cahn2d",
                                                  ("onepass.hip", "lookback.h", "ch2d.hip"))),
                parity=dict(instance=0, max_rel_err_vs_oracle=err))


def run_plain(args, torch):
    from paper_1807_07382_amd import inputs
    from paper_1807_07382_amd import pentbatch as pb
    w = inputs.plain()
    n, sigma, F = w["n"], w["sigma"], w["F"]
    T = torch.from_numpy(F).cuda()
    stream = torch.cuda.current_stream()
    plan = pb.Plan.factor_d4(n, sigma)
    if args.schedule:
        kind, seg = (int(x) for x in args.schedule.split(","))
        plan.set_schedule(kind, seg)
    for _ in range(args.warmup):
        plan.solve_(T, stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        plan.solve_(T, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    plan.check()
    sched = plan.schedule_for(F.shape[1])
    X = T.cpu().numpy()
    plan.close()
    import oracle
    ref = oracle.solve(oracle.assemble_d4(n, sigma), F)
    for _ in range(args.warmup + args.steps - 1):
        ref = oracle.solve(oracle.assemble_d4(n, sigma), ref)
    err = float(np.max(np.max(np.abs(X - ref), axis=0) / np.max(np.abs(ref), axis=0)))
    ms_step = ms / args.steps
    return dict(metric=METRIC, value=F.shape[1] / (ms_step / 1e3), unit="RHS-solves/s",
                n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=ms_step,
                higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
                data="synthetic", config=dict(workload="plain", n=n, systems=F.shape[1],
                                              sigma=sigma,
                                              schedule=SCHEDULE_NAMES[sched[0]] +
                                              (f"{sched[1]}" if sched[0] in (2, 4) else "")),
                parity=dict(systems=F.shape[1], solves=args.warmup + args.steps,
                            max_rel_err_vs_oracle=err))


def run_copy(args, torch):
    """Plain device-to-device copy of a buffer the size of the hyperdiffusion
    state (torch's copy kernel): the attainable-bandwidth reference, and the
    known-size kernel the HBM counters are scaled by."""
    from paper_1807_07382_amd import inputs
    n, batch = inputs.HYPERDIFF["n"], inputs.HYPERDIFF["batch"]
    src = torch.empty((n, batch), dtype=torch.float64, device="cuda").uniform_()
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        dst.copy_(src)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    nbytes = 2 * src.numel() * 8
    return dict(metric="device copy bandwidth", value=nbytes / (ms_step / 1e3) / 1e9,
                unit="GB/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
                ms_per_step=ms_step, bytes_per_launch=nbytes, higher_is_better=True,
                dtype="f64", data="synthetic",
                config=dict(workload="copy", elements=src.numel()))


def run_shape(args, torch):
    """One solve of ``--batch`` systems of size ``--n`` (I + sigma*D4),
    batch-fastest, repeated ``--steps`` times in place (tuning sweeps)."""
    from paper_1807_07382_amd import pentbatch as pb
    n, batch, sigma = args.n, args.batch, args.sigma
    T = torch.empty((n, batch), dtype=torch.float64, device="cuda").uniform_(-1, 1)
    stream = torch.cuda.current_stream()
    plan = pb.Plan.factor_d4(n, sigma)
    if args.schedule:
        kind, seg = (int(x) for x in args.schedule.split(","))
        plan.set_schedule(kind, seg)
    for _ in range(args.warmup):
        plan.solve_(T, stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        plan.solve_(T, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    plan.check()
    plan.close()
    gbs = BYTES_PER_UNKNOWN_FP64 * n * batch / (ms_step / 1e3) / 1e9
    return dict(metric=METRIC, value=batch / (ms_step / 1e3), unit="RHS-solves/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=ms_step,
                higher_is_better=True, dtype="f64", data="synthetic",
                config=dict(workload="shape", n=n, systems=batch, sigma=sigma,
                            schedule=args.schedule or "auto"),
                roofline=dict(bound="hbm", achieved=gbs, peak=PEAK_HBM_GBS, unit="GB/s",
                              frac=gbs / PEAK_HBM_GBS, traffic=None))


def run_periodic(args, torch):
    """Periodic hyperdiffusion with Crank-Nicolson (the paper's benchmark
    scheme, Sec. 2.3): N = 4096, sigma = 50, 65536 systems; a step is the
    explicit half R = 2C - AC and the bordered periodic solve A C' = R."""
    from paper_1807_07382_amd import inputs
    from paper_1807_07382_amd import pentbatch as pb
    from oracle import cyclic
    w = inputs.periodic()
    n, sigma, batch = w["n"], w["sigma"], w["C0"].shape[1]
    steps = args.steps
    probe = np.array([0, 1, 63, 64, 4095, 31337, batch - 1])
    C = torch.from_numpy(w["C0"]).cuda()
    R = torch.empty_like(C)
    stream = torch.cuda.current_stream()
    cy = pb.Cyclic.factor_d4(n, sigma)
    state = {"C": C, "R": R}

    def step():
        state["C"], state["R"] = cy.cn_steps_(state["C"], 1, state["R"], stream)

    form = cy.schedule_for(batch, cn=True)
    for _ in range(args.warmup):
        step()
    ms = _timed(torch, stream, step, steps)
    cy.check()
    X = state["C"][:, torch.from_numpy(probe).cuda()].cpu().numpy()
    ref = cyclic.cn_run(sigma, w["C0"][:, probe], args.warmup + steps)
    err = float(np.max(np.max(np.abs(X - ref), axis=0) / np.max(np.abs(ref), axis=0)))
    # the other form of the same step, for comparison (same data, timing only)
    other = 1 if form[0] == 2 else 2
    cy.set_schedule(other, 64)
    step()
    ms_other = _timed(torch, stream, step, max(5, steps // 5))
    cy.check()
    cy.close()
    names = {1: "stencil, E-solve, update (three passes)", 2: "single pass"}
    alg = BYTES_PER_UNKNOWN_FP64 * n * batch  # one CN step: read C once, write C' once
    gbs = alg / (ms / 1e3) / 1e9
    return dict(metric=METRIC, value=batch / (ms / 1e3), unit="RHS-solves/s", n_gpus=1,
                steps=steps, warmup=args.warmup, ms_per_step=ms, higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
                config=dict(workload="periodic", n=n, systems=batch, sigma=sigma,
                            scheme="Crank-Nicolson, periodic (bordering)",
                            form=names[form[0]], seg_rows=form[1]),
                other_form=dict(form=names[other], ms_per_step=ms_other),
                roofline=dict(bound="hbm", achieved=gbs, peak=PEAK_HBM_GBS, unit="GB/s",
                              frac=gbs / PEAK_HBM_GBS,
                              traffic=traffic_for("cyc_onepass64", "periodic",
                                                  ("cyclic.hip", "lookback.h"))
                              if form == (2, 64) else None),
                parity=dict(probe_systems=len(probe), max_rel_err_vs_oracle=err,
                            oracle_steps=args.warmup + steps))


def _rocsparse_gpsv(torch):
    """rocSPARSE's batched pentadiagonal solver (QR, interleaved layout), the
    counterpart of the general batched solver the paper compares against;
    loaded with ctypes for the comparison only."""
    import ctypes
    L = ctypes.CDLL("librocsparse.so")
    h = ctypes.c_void_p()
    if L.rocsparse_create_handle(ctypes.byref(h)) != 0:
        raise RuntimeError("rocsparse_create_handle failed")
    L.rocsparse_set_stream(h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    P, I = ctypes.c_void_p, ctypes.c_int
    L.rocsparse_dgpsv_interleaved_batch_buffer_size.argtypes = [P, I, I, P, P, P, P, P, P, I, I,
                                                                ctypes.POINTER(ctypes.c_size_t)]
    L.rocsparse_dgpsv_interleaved_batch.argtypes = [P, I, I, P, P, P, P, P, P, I, I, P]
    return L, h


def run_rewrite(args, torch):
    """Per-system matrices refactored every call (the paper's refactor-every-
    step mode, Sec. 3): N = 1024, 65536 systems, system j = I + sigma_j D4
    with sigma_j log-uniform in [1e-2, 1e4]; one step = factor and solve all
    systems.  Compared with rocSPARSE dgpsv_interleaved_batch (QR), which
    overwrites its diagonals, so its step also restores them."""
    from paper_1807_07382_amd import inputs
    from paper_1807_07382_amd import pentbatch as pb
    import oracle
    cfg = inputs.REWRITE
    n, batch = cfg["n"], cfg["batch"]
    w = inputs.rewrite()
    sig = torch.from_numpy(w["sigma"]).cuda()
    ones = torch.ones((n, 1), dtype=torch.float64, device="cuda")
    diags = [ones * sig, ones * (-4.0 * sig), 1.0 + 6.0 * ones * sig, ones * (-4.0 * sig), ones * sig]
    F0 = torch.from_numpy(w["F"]).cuda()
    F = F0.clone()
    stream = torch.cuda.current_stream()
    work = torch.empty(pb.lib().pent_rewrite_workspace_size(n, batch), dtype=torch.uint8,
                       device="cuda")
    step = lambda: pb.solve_rewrite_(*diags, F, work=work, stream=stream)
    for _ in range(args.warmup):
        step()
    F.copy_(F0)
    ms = _timed(torch, stream, step, args.steps)
    # parity: one solve from F0 on sampled systems against the oracle
    F.copy_(F0)
    pb.solve_rewrite_(*diags, F, work=work, stream=stream, check=True)
    cols = np.array([0, 1, 63, 64, 4097, batch - 1])
    hd = [x[:, torch.from_numpy(cols).cuda()].cpu().numpy() for x in diags]
    ref = oracle.rewrite_solve(*hd, w["F"][:, cols])
    X = F[:, torch.from_numpy(cols).cuda()].cpu().numpy()
    err = float(np.max(np.max(np.abs(X - ref), axis=0) / np.max(np.abs(ref), axis=0)))
    # rocSPARSE gpsv on the same systems
    gpsv = None
    try:
        L, h = _rocsparse_gpsv(torch)
        import ctypes
        wk = [x.clone() for x in diags]
        # its convention: first two entries of ds, first of dl, last of du,
        # last two of dw are zero
        wk[0][:2] = 0.0
        wk[1][:1] = 0.0
        wk[3][-1:] = 0.0
        wk[4][-2:] = 0.0
        pristine = [x.clone() for x in wk]
        Fg = F0.clone()
        sz = ctypes.c_size_t(0)
        ptrs = [ctypes.c_void_p(x.data_ptr()) for x in wk]
        st = L.rocsparse_dgpsv_interleaved_batch_buffer_size(h, 0, n, *ptrs, ctypes.c_void_p(Fg.data_ptr()),
                                                             batch, batch, ctypes.byref(sz))
        buf = torch.empty(max(sz.value, 256), dtype=torch.uint8, device="cuda")

        def gstep():
            for x, y in zip(wk, pristine):
                x.copy_(y)
            L.rocsparse_dgpsv_interleaved_batch(h, 0, n, *ptrs, ctypes.c_void_p(Fg.data_ptr()), batch,
                                                batch, ctypes.c_void_p(buf.data_ptr()))

        def gsolve_only():
            L.rocsparse_dgpsv_interleaved_batch(h, 0, n, *ptrs, ctypes.c_void_p(Fg.data_ptr()), batch,
                                                batch, ctypes.c_void_p(buf.data_ptr()))

        gstep()
        torch.cuda.synchronize()
        Xg = Fg[:, torch.from_numpy(cols).cuda()].cpu().numpy()
        gerr = float(np.max(np.max(np.abs(Xg - ref), axis=0) / np.max(np.abs(ref), axis=0)))
        gms = _timed(torch, stream, gstep, max(3, args.steps // 5))
        gsolve_ms = _timed(torch, stream, gsolve_only, max(3, args.steps // 5))
        gpsv = dict(status=int(st), ms_per_step_with_restore=gms, ms_solve_only=gsolve_ms,
                    buffer_bytes=int(sz.value), max_rel_err_vs_oracle=gerr,
                    speedup_of_rewrite=gms / ms)
        L.rocsparse_destroy_handle(h)
    except (OSError, RuntimeError) as exc:
        gpsv = dict(error=str(exc))
    # the method's minimum: five diagonals and f read, x written (56 B per
    # unknown); the kernel's own plan also writes gamma, delta and g and reads
    # them back (104 B)
    alg = 56 * n * batch
    gbs = alg / (ms / 1e3) / 1e9
    gbs104 = 104 * n * batch / (ms / 1e3) / 1e9
    return dict(metric=METRIC, value=batch / (ms / 1e3), unit="RHS-solves/s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=ms, higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
                config=dict(workload="rewrite", n=n, systems=batch,
                            matrices="one per system, refactored every call"),
                roofline=dict(bound="hbm", achieved=gbs, peak=PEAK_HBM_GBS, unit="GB/s",
                              frac=gbs / PEAK_HBM_GBS, bytes_per_unknown=56,
                              traffic=traffic_for("rewrite_lane", "rewrite", ("rewrite.hip",))),
                kernel_plan_roofline=dict(bytes_per_unknown=104, achieved=gbs104,
                                          frac=gbs104 / PEAK_HBM_GBS),
                parity=dict(probe_systems=len(cols), max_rel_err_vs_oracle=err),
                rocsparse_gpsv=gpsv)


WORKLOADS = {"hyperdiff": run_hyperdiff, "periodic": run_periodic, "rewrite": run_rewrite, "plain": run_plain, "copy": run_copy,
             "shape": run_shape, "precision": run_precision, "group": run_group,
             "cahn2d": run_cahn2d}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="hyperdiff", choices=sorted(WORKLOADS))
    ap.add_argument("--schedule", default="", help="force kind,seg_rows (tuning)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--headline-only", action="store_true",
                    help="hyperdiff only: skip the other configurations (profiling runs)")
    ap.add_argument("--n", type=int, default=1024, help="shape workload: rows")
    ap.add_argument("--batch", type=int, default=32768, help="shape workload: systems")
    ap.add_argument("--sigma", type=float, default=200.0, help="shape workload: sigma")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path shards "
              "by systems with no exchange, see the design notes.", file=sys.stderr)
        return 2
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    out = WORKLOADS[args.workload](args, torch)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
