#!/usr/bin/env python3
"""Benchmark: stochastic-Galerkin KKT solves per second on one MI355X.

A step is one pass of the whole hot path over one batch: a preconditioned
FGMRES(30) solve to relative residual 1e-8 of every member of the batch
(block-diagonal Schur preconditioner with Chebyshev mass solves and the
hierarchical Gauss-Seidel sweep with multigrid inner solves).  The default
workload is the steady 128 x 128 problem (16,641 nodes, M = 6 random
variables, total degree P = 4, n_xi = 210, sigma = 0.3) with its beta sweep
{1e-2, 1e-4, 1e-6} solved as one batch of three members (seeded Gaussian-bump
targets).  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0   # MI355X HBM3E

WORKLOADS = {
    # name: (n, M, P, sigma, betas, n_t, seeds)
    "steady-128-M6-P4": dict(n=128, M=6, P=4, sigma=0.3, betas=(1e-2, 1e-4, 1e-6), n_t=1, seeds=(1, 2, 3)),
    "steady-16-M4-P3": dict(n=16, M=4, P=3, sigma=0.2, betas=(1e-2,), n_t=1, seeds=(0,)),
    "heat-64-M4-P3-nt32": dict(n=64, M=4, P=3, sigma=0.2, betas=(1e-3,), n_t=32, seeds=(4,)),
    "steady-512-M8-P3": dict(n=512, M=8, P=3, sigma=0.3, betas=(1e-2,), n_t=1, seeds=(5,)),
    # the largest shape the serving stream draws (n_xi = 495, 98 M unknowns)
    "steady-256-M8-P4": dict(n=256, M=8, P=4, sigma=0.3, betas=(1e-2,), n_t=1, seeds=(6,)),
}
DEFAULT = "steady-128-M6-P4"
# kernels timed with HIP events around every launch (sg_options.profile), with
# the algorithmic bytes each launch must move
PROF_KIND = {"kkt_apply": 1, "mg_down": 2, "arnoldi_dots": 3, "hgs_rhs": 4, "arnoldi_update": 5, "mg_tail": 6,
             "mass_cheb": 7, "mg_up": 8}
ARNOLDI = {"dcgs2": 0, "cgs2": 1}


# sources of the kernels whose HBM traffic is taken from a committed counter summary
TRAFFIC_SOURCES = ("paper_2512_23804_amd/csrc/kernels.hip", "paper_2512_23804_amd/csrc/solver.cpp",
                   "paper_2512_23804_amd/csrc/common.hpp")


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary (profiles/*_traffic_*.md: FETCH_SIZE and WRITE_SIZE scaled by a
    copy probe), or None when no summary covers this kernel and workload or the
    kernel sources changed since the counters were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic_*.md"))):
        kv = {}
        with open(path) as f:
            for line in f:
                if ":" in line and line[:1].isalpha():
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel") != kernel or kv.get("workload") != workload:
            continue
        h = hashlib.sha256()
        for src in TRAFFIC_SOURCES:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != kv.get("sources_sha256"):
            return None
        return float(kv["traffic_bytes_per_launch"])
    return None


def make_problems(sgl, sg_inputs, wl):
    probs = []
    for beta, seed in zip(wl["betas"], wl["seeds"]):
        if wl["n_t"] > 1:
            tgt = sg_inputs.moving_bump(wl["n"], wl["n_t"], 1.0, seed)
        else:
            tgt = sg_inputs.gaussian_bumps(wl["n"], seed)
        probs.append(sgl.ProblemData(wl["n"], wl["M"], wl["P"], wl["sigma"], beta, tgt, n_t=wl["n_t"], T=1.0))
    return probs


def timed_solves(torch, sgl, probs, opts, steps, warmup, stream, tuned=None, keep=None):
    """Time `steps` batched solves after `warmup` untimed ones; with `keep`,
    append the last solution (device tensor, members x KKT length)."""
    h = sgl.Handle(probs, opts, stream=stream)
    if tuned is not None:
        tuned.extend([list(r) for r in h.sizes.sweep_rows])
    x = torch.zeros(h.members * h.kkt_elems, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        h.solve(x)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        rc, info = h.solve(x)
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if keep is not None:
        keep.append(x.view(h.members, h.kkt_elems).clone())
    h.close()
    return dt, infos


def max_rel_diff(a, b):
    """max over members of ||a - b||_inf / ||b||_inf"""
    return max(float((a[i] - b[i]).abs().max() / b[i].abs().max()) for i in range(b.shape[0]))


def sg_apply_bandwidth(torch, sgl, probs, stream, min_bytes=1 << 30, reps=20):
    """Average duration of the SG operator apply (sg_apply_operator) with HIP
    events on the library's stream, rotating over enough input/output blocks
    that the working set exceeds the 256 MB last-level cache."""
    h = sgl.Handle(probs[:1], sgl.default_options(), stream=stream)
    blk = h.block_elems
    nbuf = max(2, int(np.ceil(min_bytes / (16 * blk))))
    xs = [torch.rand(blk, dtype=torch.float64, device="cuda") for _ in range(nbuf)]
    ys = [torch.empty(blk, dtype=torch.float64, device="cuda") for _ in range(nbuf)]
    with torch.cuda.stream(stream):
        for i in range(nbuf):
            h.apply_operator(xs[i], ys[i], stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for r in range(reps):
            for i in range(nbuf):
                h.apply_operator(xs[i], ys[i], stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / (reps * nbuf)
    s = h.sizes
    bytes_per = 8.0 * (2 * blk + (s.M + 1) * s.n * s.n)
    h.close()
    return dict(ms=ms, bytes=bytes_per, GBps=bytes_per / ms / 1e6, buffers=nbuf)


def serving_run(sgl, sg_inputs, num, rate, grids, precision):
    """Continuous-batching server (sg_submit / sg_poll) on a seeded Poisson
    stream of mixed-shape steady requests; latency is submit -> completion
    and includes the host <-> device copies of the request's arrays."""
    from math import comb
    reqs = sg_inputs.serving_stream(num, seed=7, rate_per_s=rate, grid_choices=grids)
    srv = sgl.Server(hbm_budget_bytes=0, max_slots=16)
    opts = sgl.default_options(rtol=1e-8, precision=precision)
    pending, converged = {}, 0
    t0 = time.perf_counter()

    def drain():
        nonlocal converged
        for t in list(pending):
            rc, info = srv.poll(t)
            if rc != sgl.SG_PENDING:
                converged += int(rc == sgl.SG_OK and info.converged == 1)
                del pending[t]          # releases the host output array

    for r in reqs:
        while time.perf_counter() - t0 < r["arrival"]:
            drain()
            time.sleep(0.0005)
        pd = sgl.ProblemData(r["n"], r["M"], r["P"], r["sigma"], r["beta"], sg_inputs.gaussian_bumps(r["n"], r["seed"]))
        out = np.empty(3 * comb(r["M"] + r["P"], r["P"]) * (r["n"] + 1) ** 2)
        pending[srv.submit(pd, out, opts)] = out
    while pending:
        drain()
        time.sleep(0.001)
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    return {"requests": num, "arrival_rate_per_s": rate, "grids": list(grids), "M_range": [4, 8],
            "P_range": [2, 4], "precision": {0: "fp64", 1: "fp32_refine", 2: "fp32_precond"}[precision],
            "converged": converged, "wall_s": wall, "solves_per_s": num / wall, "p50_ms": st["p50_ms"],
            "p99_ms": st["p99_ms"]}


def serving_sweep(sgl, sg_inputs, num, grids):
    """The same seeded request mix (shapes do not depend on the arrival rate)
    submitted all at once to measure the FP64 capacity, then as Poisson streams
    at half and one and a half times that capacity; each arrival pattern in
    FP64 and with FP32 refinement."""
    runs = []

    def one(rate, precision):
        r = serving_run(sgl, sg_inputs, num, rate, grids, precision)
        print(f"[serving] {r['precision']} rate {rate:.3g}/s: {r['converged']}/{num} converged, "
              f"{r['solves_per_s']:.2f} solves/s, p50 {r['p50_ms']:.0f} ms, p99 {r['p99_ms']:.0f} ms",
              file=sys.stderr, flush=True)
        runs.append(r)
        return r

    cap = one(float("inf"), 0)["solves_per_s"]
    one(float("inf"), 1)
    for f in (0.5, 1.5):
        for prec in (0, 1):
            one(f * cap, prec)
    return {"serving_sweep": {"requests": num, "grids": list(grids), "fp64_capacity_solves_per_s": cap,
                              "runs": runs}}


def cpu_baseline(wl, gpu_iters):
    """The oracle (plain FP64 numpy/scipy, single thread) timed on one
    preconditioned FGMRES iteration of the first member: one preconditioner
    application (Chebyshev + two hGS sweeps with multigrid) and one matricized
    KKT apply; scaled by the GPU run's iterations per solve."""
    from threadpoolctl import threadpool_limits

    import sg_inputs
    from oracle import kkt, precond

    with threadpool_limits(limits=1):
        if wl["n_t"] > 1:
            tgt = sg_inputs.moving_bump(wl["n"], wl["n_t"], 1.0, wl["seeds"][0])
        else:
            tgt = sg_inputs.gaussian_bumps(wl["n"], wl["seeds"][0])
        prob = kkt.Problem(n=wl["n"], M=wl["M"], P=wl["P"], sigma=wl["sigma"], beta=wl["betas"][0],
                           n_t=wl["n_t"], y_target=tgt)
        sg = kkt.setup(prob)
        inner = precond.make_inner(sg)
        r = kkt.rhs(sg)
        V = np.random.default_rng(0).standard_normal((15, r.size))
        reps, t0 = 0, time.perf_counter()
        while True:   # whole iterations until at least 10 s of CPU work
            z = precond.precond_apply(sg, r, inner)
            w = kkt.kkt_apply_matricized(sg, z)
            # Arnoldi work of an average iteration (15 basis vectors, two Gram-Schmidt passes)
            for _ in range(2):
                hcoef = V @ w
                w = w - V.T @ hcoef
            reps += 1
            if time.perf_counter() - t0 >= 10.0:
                break
        t_iter = (time.perf_counter() - t0) / reps
    per_solve = t_iter * gpu_iters
    return dict(value=1.0 / per_solve, unit="solves/s", cores=1, kind="oracle",
                sample=f"{reps} FGMRES iterations of the oracle on the first member at the workload size "
                       f"({t_iter:.2f} s each, single thread), scaled by {gpu_iters:.1f} iterations per solve")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--profile-kernel", default="auto", choices=["auto"] + sorted(PROF_KIND),
                    help="kernel reported as roofline (auto: the one with the largest measured total time)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=32, help="requests in the serving stream (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=30.0, help="Poisson arrival rate of the serving stream")
    ap.add_argument("--serve-grids", default="32,64", help="grid sizes n the serving stream draws from")
    ap.add_argument("--serve-sweep", action="store_true",
                    help="only run the mixed serving protocol (saturated capacity, then Poisson arrivals at "
                         "0.5x and 1.5x the FP64 capacity, FP64 and FP32 refinement) and print its JSON")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy a 1 GiB FP64 tensor three times (calibrates hardware byte counters) and exit")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP32 and single-solve comparisons")
    ap.add_argument("--no-graphs", action="store_true", help="launch every kernel directly (no HIP graph replay)")
    ap.add_argument("--sweep-rows", type=int, default=0, choices=[0, 2, 4, 8],
                    help="strip rows of the sweep kernels (0: autotuned)")
    ap.add_argument("--arnoldi", default="dcgs2", choices=sorted(ARNOLDI),
                    help="FGMRES orthogonalisation (delayed reorthogonalisation or Gram-Schmidt twice)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_probe:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 8 << 27, "copy_probe_bytes_written": 8 << 27, "copies": 3}))
        return

    import paper_2512_23804_amd as sgl
    import sg_inputs

    if args.serve_sweep:
        grids = tuple(int(g) for g in args.serve_grids.split(","))
        print(json.dumps(serving_sweep(sgl, sg_inputs, args.serve_requests, grids)), flush=True)
        return

    wl = WORKLOADS[args.workload]
    probs = make_problems(sgl, sg_inputs, wl)
    stream = torch.cuda.Stream()

    graphs = 0 if args.no_graphs else 1
    # headline: FP64 batch (the whole beta sweep) per step
    arn = ARNOLDI[args.arnoldi]
    opts = sgl.default_options(rtol=1e-8, use_graphs=graphs, arnoldi=arn, sweep_rows=args.sweep_rows)
    tuned = []
    x64 = []
    dt, infos = timed_solves(torch, sgl, probs, opts, args.steps, args.warmup, stream, tuned, keep=x64)
    nsolve = len(probs) * args.steps
    value = nsolve / dt
    iters = [i.iters for step in infos for i in step]
    rel = max(i.rel_res_true for step in infos for i in step)
    # per-kernel rooflines: one more solve of the same batch per kernel kind with
    # HIP events around every launch of that kernel on the library's stream
    # (event pairs serialise the stream a little, so these solves are not part
    # of the timed steps)
    kern = {}
    kinds = PROF_KIND if args.profile_kernel == "auto" else {args.profile_kernel: PROF_KIND[args.profile_kernel]}
    for name, kind in kinds.items():
        popt = sgl.default_options(rtol=1e-8, profile=kind, arnoldi=arn, sweep_rows=args.sweep_rows)
        _, pinfo = timed_solves(torch, sgl, probs, popt, 1, 0, stream)
        pms, pbytes, plaunch = pinfo[0][0].prof_ms, pinfo[0][0].prof_bytes, pinfo[0][0].prof_launches
        if plaunch == 0:
            continue
        ach = pbytes / pms / 1e6 if pms > 0 else 0.0
        kern[name] = {"ms_per_step": pms, "launches": plaunch, "avg_launch_ms": pms / plaunch,
                      "bytes_per_launch": pbytes / plaunch, "achieved_GBps": ach, "frac": ach / HBM_PEAK_GBPS}
    dom = args.profile_kernel if args.profile_kernel != "auto" else max(kern, key=lambda k: kern[k]["ms_per_step"])
    kd = kern[dom]
    out = {
        "metric": "KKT solves/s to rel-res 1e-8 (FP64 vs FP32+refine); SG apply HBM GB/s",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Gaussian-bump targets, cosine random field)",
        "config": {"workload": args.workload, "n": wl["n"], "M": wl["M"], "P": wl["P"], "sigma": wl["sigma"],
                   "betas": list(wl["betas"]), "n_t": wl["n_t"], "batch": len(probs), "restart": 30,
                   "rtol": 1e-8, "precision": "fp64", "graphs": bool(graphs),
                   "arnoldi": args.arnoldi, "sweep_rows_fp64": tuned[0]},
        "iterations": iters[: len(probs)],
        "max_rel_res": rel,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": kd["achieved_GBps"], "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": kd["achieved_GBps"] / HBM_PEAK_GBPS,
                     "traffic": measured_traffic(dom, args.workload),
                     "launches": kd["launches"], "avg_launch_ms": kd["avg_launch_ms"],
                     "bytes_per_launch": kd["bytes_per_launch"]},
        "kernels": kern,
    }
    if not args.no_extras:
        o32 = sgl.default_options(rtol=1e-8, precision=sgl.SG_PREC_FP32_REFINE, use_graphs=graphs,
                                  arnoldi=arn, sweep_rows=args.sweep_rows)
        x32 = []
        dt32, inf32 = timed_solves(torch, sgl, probs, o32, args.steps, 1, stream, keep=x32)
        out["fp32_refine"] = {"value": nsolve / dt32, "unit": "solves/s", "dtype": "f32 operator/preconditioner, "
                              "f64 Arnoldi and refinement", "iterations": [i.iters for i in inf32[0]],
                              "max_rel_res": max(i.rel_res_true for st in inf32 for i in st),
                              "max_rel_diff_vs_fp64": max_rel_diff(x32[0], x64[0])}
        opc = sgl.default_options(rtol=1e-8, precision=sgl.SG_PREC_FP32_PRECOND, use_graphs=graphs, arnoldi=arn,
                                  sweep_rows=args.sweep_rows)
        xpc = []
        dtp, infp = timed_solves(torch, sgl, probs, opc, args.steps, 1, stream, keep=xpc)
        out["fp32_precond"] = {"value": nsolve / dtp, "unit": "solves/s", "dtype": "f32 preconditioner, "
                               "f64 operator, Arnoldi and restarts", "iterations": [i.iters for i in infp[0]],
                               "max_rel_res": max(i.rel_res_true for st in infp for i in st),
                               "max_rel_diff_vs_fp64": max_rel_diff(xpc[0], x64[0])}
        del x32, xpc
        single = []
        t_single = 0.0
        for p in probs:
            sopt = sgl.default_options(rtol=1e-8, use_graphs=graphs, arnoldi=arn, sweep_rows=args.sweep_rows)
            dts, infs = timed_solves(torch, sgl, [p], sopt, 1, 1, stream)
            t_single += dts
            single.append(infs[0][0].iters)
        out["fp64_single"] = {"value": len(probs) / t_single, "unit": "solves/s", "iterations": single}
        out["sg_apply"] = sg_apply_bandwidth(torch, sgl, probs, stream)
        out["sg_apply"]["frac_of_hbm_peak"] = out["sg_apply"]["GBps"] / HBM_PEAK_GBPS
    if not args.no_extras and args.serve_requests > 0:
        grids = tuple(int(g) for g in args.serve_grids.split(","))
        out["serving"] = serving_run(sgl, sg_inputs, args.serve_requests, args.serve_rate, grids, 0)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, float(np.mean(iters)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
