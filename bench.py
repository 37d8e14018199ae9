#!/usr/bin/env python3
"""Benchmark: stochastic-Galerkin KKT solves per second on one MI355X.

A step is one pass of the whole hot path over one batch: a preconditioned
FGMRES(30) solve to relative residual 1e-8 of every member of the batch
(block-diagonal Schur preconditioner with Chebyshev mass solves and the
hierarchical Gauss-Seidel sweep with multigrid inner solves).  The default
workload is the largest single-GPU steady problem: 512 x 512 Q1 elements
(263,169 nodes), M = 8 random variables, total degree P = 3 (n_xi = 165),
sigma = 0.3, beta = 1e-2, about 130 M unknowns (seeded Gaussian-bump target).
Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
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

HBM_PEAK_GBPS = 8000.0   # MI355X HBM3E

WORKLOADS = {
    # name: (n, M, P, sigma, betas, n_t, seeds)
    "steady-128-M6-P4": dict(n=128, M=6, P=4, sigma=0.3, betas=(1e-2, 1e-4, 1e-6), n_t=1, seeds=(1, 2, 3)),
    "steady-16-M4-P3": dict(n=16, M=4, P=3, sigma=0.2, betas=(1e-2,), n_t=1, seeds=(0,)),
    "heat-64-M4-P3-nt32": dict(n=64, M=4, P=3, sigma=0.2, betas=(1e-3,), n_t=32, seeds=(4,)),
    "steady-512-M8-P3": dict(n=512, M=8, P=3, sigma=0.3, betas=(1e-2,), n_t=1, seeds=(5,)),
    # the largest shape the serving stream draws (n_xi = 495, 98 M unknowns)
    "steady-256-M8-P4": dict(n=256, M=8, P=4, sigma=0.3, betas=(1e-2,), n_t=1, seeds=(6,)),
    # Section 5's own workload: log-normal field (KL of the exponential covariance, correlation length 1
    # on [-1,1]^2), Hermite chaos m = 3, p = 3 (n_xi = 20, n_A = 84 terms), sigma = 0.2, gamma = 1,
    # indicator target, 32 x 32 elements, the beta sweep of its Table (deter beta)
    "lognormal-32-M3-P3": dict(n=32, M=3, P=3, sigma=0.2, betas=(1e-2, 1e-3, 1e-4, 1e-5), n_t=1, seeds=(0, 0, 0, 0),
                               field="lognormal", gamma=1.0),
    "lognormal-128-M3-P3": dict(n=128, M=3, P=3, sigma=0.2, betas=(1e-4,), n_t=1, seeds=(0,),
                                field="lognormal", gamma=1.0),
}
DEFAULT = "steady-512-M8-P3"
# kernels timed with HIP events around every launch (sg_options.profile), with
# the algorithmic bytes each launch must move
PROF_KIND = {"kkt_apply": 1, "mg_down": 2, "arnoldi_dots": 3, "hgs_rhs": 4, "arnoldi_update": 5, "mg_tail": 6,
             "mass_cheb": 7, "mg_up": 8}
ARNOLDI = {"dcgs2": 0, "cgs2": 1}


# the source text behind the Arnoldi passes whose HBM traffic is taken from a committed
# counter summary: the DCGS2 kernels and their launchers in kernels.hip, and the
# launch shape (blocks per member vector) in solver.cpp
TRAFFIC_REGIONS = (
    ("paper_2512_23804_amd/csrc/kernels.hip", "constexpr int kDotsU", "void k_dcgs_finish("),
    ("paper_2512_23804_amd/csrc/kernels.hip", "void launch_dcgs_dots(", "void launch_dcgs_finish("),
    ("paper_2512_23804_amd/csrc/solver.cpp", "nblk = ", "\n"),
)


def traffic_source_digest() -> str:
    """sha256 over the source regions in TRAFFIC_REGIONS (start marker up to,
    not including, the end marker)."""
    import hashlib
    h = hashlib.sha256()
    for src, start, end in TRAFFIC_REGIONS:
        with open(os.path.join(ROOT, src)) as f:
            text = f.read()
        i = text.index(start)
        j = text.index(end.encode().decode("unicode_escape"), i + len(start))
        h.update(text[i:j].encode())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary (profiles/*_traffic_*.md: FETCH_SIZE and WRITE_SIZE scaled by a
    copy probe), or None when no summary covers this kernel and workload or the
    kernel sources changed since the counters were taken."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic_*.md"))):
        kv = {}
        with open(path) as f:
            for line in f:
                if ":" in line and line[:1].isalpha():
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel") != kernel or kv.get("workload") != workload:
            continue
        if traffic_source_digest() != kv.get("sources_sha256"):
            return None
        return float(kv["traffic_bytes_per_launch"])
    return None


def make_problems(sgl, sg_inputs, wl):
    probs = []
    lognormal = wl.get("field") == "lognormal"
    for beta, seed in zip(wl["betas"], wl["seeds"]):
        if wl["n_t"] > 1:
            tgt = sg_inputs.moving_bump(wl["n"], wl["n_t"], 1.0, seed)
        elif lognormal:
            tgt = sg_inputs.indicator_target(wl["n"])
        else:
            tgt = sg_inputs.gaussian_bumps(wl["n"], seed)
        probs.append(sgl.ProblemData(wl["n"], wl["M"], wl["P"], wl["sigma"], beta, tgt, n_t=wl["n_t"], T=1.0,
                                     gamma=wl.get("gamma", 0.0),
                                     field=sgl.SG_FIELD_LOGNORMAL if lognormal else sgl.SG_FIELD_AFFINE))
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
    torch.cuda.synchronize()     # the inputs are written on torch's stream, read on `stream`
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


def serving_run(sgl, sg_inputs, num, rate, grids, precision, keep=None):
    """Continuous-batching server (sg_submit / sg_poll) on a seeded Poisson
    stream of mixed-shape steady requests; latency is submit -> completion
    and includes the host <-> device copies of the request's arrays.  With
    `keep` (a dict), each request's host solution is stored under its index."""
    from math import comb
    reqs = sg_inputs.serving_stream(num, seed=7, rate_per_s=rate, grid_choices=grids)
    srv = sgl.Server(hbm_budget_bytes=0, max_slots=16)
    opts = sgl.default_options(rtol=1e-8, precision=precision)
    pending, converged, worst = {}, 0, 0.0
    setup_ms, solve_ms, iters = [], [], []
    t0 = time.perf_counter()

    def drain():
        nonlocal converged, worst
        for t in list(pending):
            rc, info = srv.poll(t)
            if rc != sgl.SG_PENDING:
                ok = rc == sgl.SG_OK and info.converged == 1
                converged += int(ok)
                worst = max(worst, info.rel_res_true)
                setup_ms.append(info.t_setup_ms)
                solve_ms.append(info.t_solve_ms)
                iters.append(info.iters)
                i, out = pending.pop(t)
                if keep is not None and i % KEEP_EVERY == 0:
                    keep[i] = out

    for i, r in enumerate(reqs):
        while time.perf_counter() - t0 < r["arrival"]:
            drain()
            time.sleep(0.0005)
        pd = sgl.ProblemData(r["n"], r["M"], r["P"], r["sigma"], r["beta"], sg_inputs.gaussian_bumps(r["n"], r["seed"]))
        out = np.empty(3 * comb(r["M"] + r["P"], r["P"]) * (r["n"] + 1) ** 2)
        pending[srv.submit(pd, out, opts)] = (i, out)
    while pending:
        drain()
        time.sleep(0.001)
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    return {"path": "serving", "requests": num, "arrival_rate_per_s": rate, "grids": list(grids), "M_range": [4, 8],
            "P_range": [2, 4], "precision": {0: "fp64", 1: "fp32_refine", 2: "fp32_precond"}[precision],
            "converged": converged, "max_rel_res": worst, "wall_s": wall, "solves_per_s": converged / wall,
            "submitted_per_s": num / wall, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
            "mean_batch_setup_ms": float(np.mean(setup_ms)) if setup_ms else None,
            "mean_batch_solve_ms": float(np.mean(solve_ms)) if solve_ms else None,
            "mean_iterations": float(np.mean(iters)) if iters else None,
            "failed": converged < num}


def single_solve_run(torch, sgl, sg_inputs, num, grids, keep=None):
    """The plain FP64 single-solve path on the same seeded request mix: the
    requests, all queued at time zero, are solved one after another, each with
    its own handle (sg_setup + sg_solve on device buffers, no batching, no
    overlap); latency is from the start to the copy of its solution to host
    memory, as in the server."""
    reqs = sg_inputs.serving_stream(num, seed=7, rate_per_s=float("inf"), grid_choices=grids)
    opts = sgl.default_options(rtol=1e-8, use_graphs=0)
    lat, converged, worst = [], 0, 0.0
    t0 = time.perf_counter()
    for i, r in enumerate(reqs):
        pd = sgl.ProblemData(r["n"], r["M"], r["P"], r["sigma"], r["beta"], sg_inputs.gaussian_bumps(r["n"], r["seed"]))
        h = sgl.Handle(pd, opts)
        x = torch.zeros(h.kkt_elems, dtype=torch.float64, device="cuda")
        rc, info = h.solve(x)
        out = x.cpu().numpy()
        h.close()
        del x
        converged += int(rc == sgl.SG_OK and info[0].converged == 1)
        worst = max(worst, info[0].rel_res_true)
        lat.append(1000.0 * (time.perf_counter() - t0))
        if keep is not None and i % KEEP_EVERY == 0:
            keep[i] = out
    wall = time.perf_counter() - t0
    return {"path": "single_fp64", "requests": num, "arrival_rate_per_s": float("inf"), "grids": list(grids),
            "precision": "fp64", "converged": converged, "max_rel_res": worst, "wall_s": wall,
            "solves_per_s": converged / wall, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "failed": converged < num}


# the serving comparison keeps the host solutions of every KEEP_EVERY-th request
# (a 256 x 256, n_xi = 495 request's solution is 785 MB) for the FP32 / FP64 differences
KEEP_EVERY = 8


def _max_rel_diff_host(a: dict, b: dict) -> float:
    """max over the kept requests of ||a - b||_inf / ||b||_inf (host solutions)."""
    return max(float(np.max(np.abs(a[i] - b[i])) / np.max(np.abs(b[i]))) for i in b)


def serving_compare(torch, sgl, sg_inputs, num, grids):
    """The batched-serving comparison on one seeded mixed-shape request mix,
    every request queued at time zero (capacity): FP64 serving, FP32 operator
    and preconditioner with FP64 refinement in serving, and the plain FP64
    single-solve path.  Each FP32 result's max-norm difference from the FP64
    serving result of the same request is reported."""
    x64, x32, xs = {}, {}, {}
    runs = [serving_run(sgl, sg_inputs, num, float("inf"), grids, 0, keep=x64),
            serving_run(sgl, sg_inputs, num, float("inf"), grids, 1, keep=x32),
            single_solve_run(torch, sgl, sg_inputs, num, grids, keep=xs)]
    runs[1]["max_rel_diff_vs_fp64"] = _max_rel_diff_host(x32, x64)
    runs[2]["max_rel_diff_vs_fp64"] = _max_rel_diff_host(xs, x64)
    return {"requests": num, "grids": list(grids), "arrivals": "all at time zero",
            "differences_over": f"every {KEEP_EVERY}th request", "runs": runs,
            "fp32_refine_serving_over_single_fp64": runs[1]["solves_per_s"] / runs[2]["solves_per_s"],
            "fp64_serving_over_single_fp64": runs[0]["solves_per_s"] / runs[2]["solves_per_s"]}


def serving_sweep(torch, sgl, sg_inputs, num, grids):
    """The same seeded request mix (shapes do not depend on the arrival rate)
    submitted all at once to measure capacity (FP64 serving, FP32-refinement
    serving, plain FP64 single solves), then as Poisson streams at half and one
    and a half times the FP64 serving capacity, in both serving precisions."""
    cmp = serving_compare(torch, sgl, sg_inputs, num, grids)
    runs = list(cmp["runs"])
    for r in runs:
        print(f"[serving] {r['path']} {r['precision']} all at once: {r['converged']}/{num} converged, "
              f"{r['solves_per_s']:.2f} solves/s, p50 {r['p50_ms']:.0f} ms, p99 {r['p99_ms']:.0f} ms",
              file=sys.stderr, flush=True)
    cap = runs[0]["solves_per_s"]
    for f in (0.5, 1.5):
        for prec in (0, 1):
            r = serving_run(sgl, sg_inputs, num, f * cap, grids, prec)
            print(f"[serving] {r['precision']} rate {f * cap:.3g}/s: {r['converged']}/{num} converged, "
                  f"{r['solves_per_s']:.2f} solves/s, p50 {r['p50_ms']:.0f} ms, p99 {r['p99_ms']:.0f} ms",
                  file=sys.stderr, flush=True)
            runs.append(r)
    return {"serving_sweep": {"requests": num, "grids": list(grids), "fp64_capacity_solves_per_s": cap,
                              "runs": runs}}


# preconditioner variants (Section 5: Chebyshev-5 / Chebyshev-10 / direct mass
# solves with hGS-1; the truncations n_tau = 1 and m + 1; Algorithm 5 with N > 1)
# as sg_options overrides
PRECOND_VARIANTS = [
    ("cheb5 + hGS-1 (multigrid mean blocks)", {}),
    ("cheb10 + hGS-1", dict(cheb_steps=10)),
    ("exact mass + hGS-1", dict(cheb_steps=0)),
    ("cheb5 + hGS-1 (exact mean blocks)", dict(mean_solver=1)),
    ("exact mass + hGS-1 (exact mean blocks)", dict(cheb_steps=0, mean_solver=1)),
    ("cheb5 + Richardson N=2", dict(richardson_steps=2)),
    ("cheb5 + hGS-1, mean-based (r = 1)", dict(truncation_r=1)),
    ("hGSoc (Alg. 2-3; Alg. 4 on time steps), cheb5 level solves", dict(precond=1)),
]


def precond_variants(torch, sgl, sg_inputs, workload, steps, warmup):
    wl = WORKLOADS[workload]
    probs = make_problems(sgl, sg_inputs, wl)
    stream = torch.cuda.Stream()
    rows = []
    variants = list(PRECOND_VARIANTS)
    if wl.get("field") == "lognormal":
        # Section 5's three truncations n_tau = 1, m + 1, n_A with each mass-block variant
        variants = [(f"{mass} + hGS-1, n_tau = {name}", dict(truncation_r=r, **mo))
                    for mass, mo in (("cheb5", {}), ("cheb10", dict(cheb_steps=10)), ("exact mass", dict(cheb_steps=0)))
                    for name, r in (("1", 1), ("m+1", wl["M"] + 1), ("n_A", 0))]
        variants.append(("cheb5 + hGS-1 (exact mean blocks), n_tau = m+1", dict(truncation_r=wl["M"] + 1,
                                                                               mean_solver=1)))
        variants.append(("hGSoc (Alg. 2-3), n_tau = m+1", dict(truncation_r=wl["M"] + 1, precond=1)))
    for label, over in variants:
        print(f"[bench] variant {label}", file=sys.stderr, flush=True)
        opts = sgl.default_options(rtol=1e-8, **over)
        dt, infos = timed_solves(torch, sgl, probs, opts, steps, warmup, stream)
        last = infos[-1]
        rows.append({"variant": label, "options": over, "iterations": [i.iters for i in last],
                     "solves_per_s": steps * len(probs) / dt, "ms_per_step": 1000.0 * dt / steps,
                     "max_rel_res": max(i.rel_res_true for i in last),
                     "converged": all(i.converged == 1 for i in last)})
    return {"precond_variants": workload, "steps": steps, "rows": rows}


def paper_tables(torch, sgl, sg_inputs, grids, mean="direct"):
    """The grid of the paper's tables of sigma variations (Section 5): log-normal
    field with Hermite chaos, beta = 1e-4, gamma = 1, indicator target;
    n_xi = 20 (m = 3, p = 3), 70 (4, 4), 84 (6, 3); truncations n_tau = 1,
    m + 1, n_A; Chebyshev-5 or direct (sine-transform) mass solves with hGS-1,
    whose mean-block solves are direct as in the paper (exact sine-transform
    solves; `mean` = "multigrid" switches them to one V-cycle); sigma = 0.01,
    0.1, 0.4 as the three members of one batch.  One untimed solve, then one
    timed; the time per member is the batch's solve time over three.
    FGMRES(30) to relative residual 1e-8."""
    rows = []
    stream = torch.cuda.Stream()
    sigmas = (0.01, 0.1, 0.4)
    for n in grids:
        tgt = sg_inputs.indicator_target(n)
        for M, P in ((3, 3), (4, 4), (6, 3)):
            probs = [sgl.ProblemData(n, M, P, sg, 1e-4, tgt, gamma=1.0, field=sgl.SG_FIELD_LOGNORMAL)
                     for sg in sigmas]
            for mass, mo in (("cheb5", {}), ("direct", dict(cheb_steps=0))):
                for name, r in (("1", 1), ("m+1", M + 1), ("n_A", 0)):
                    print(f"[bench] paper table n={n} m={M} p={P} {mass} n_tau={name}", file=sys.stderr,
                          flush=True)
                    opts = sgl.default_options(rtol=1e-8, truncation_r=r,
                                               mean_solver=1 if mean == "direct" else 0, **mo)
                    dt, infos = timed_solves(torch, sgl, probs, opts, 1, 1, stream)
                    last = infos[-1]
                    rows.append({"n": n, "nodes": (n + 1) ** 2, "m": M, "p": P, "n_xi": math.comb(M + P, P),
                                 "mass": mass, "mean_blocks": mean, "n_tau": name, "sigma": list(sigmas),
                                 "iterations": [i.iters for i in last],
                                 "ms_per_solve": 1000.0 * dt / len(probs),
                                 "max_rel_res": max(i.rel_res_true for i in last),
                                 "converged": all(i.converged == 1 for i in last)})
                    print(json.dumps(rows[-1]), flush=True)
    return {"paper_tables": rows}


def paper_parabolic(torch, sgl, sg_inputs):
    """The settings of the paper's time-dependent tables (Section 5): log-normal
    field with Hermite chaos, gamma = 1, the indicator target at every time step,
    y_0 = 0, T = 1; Chebyshev-5 + hGS-1 with direct (sine-transform) mean-block
    solves; truncations n_tau = 1, m + 1, n_A; relative tolerances 1e-6 and
    1e-4; FGMRES(30).  Defaults m = p = 3, sigma = 0.2, beta = 1e-4, 32 x 32
    elements, n_t = 8; each table varies one of them (its values as the members
    of one batch where only sigma or beta change).  One untimed solve, then one
    timed; the time per member is the batch's solve time over its members."""
    base = dict(n=32, M=3, P=3, n_t=8, members=[(0.2, 1e-4)])
    tables = [("mesh", dict(base, n=nn)) for nn in (8, 16, 32, 64)]
    tables += [("beta", dict(base, members=[(0.2, b) for b in (1e-2, 1e-3, 1e-6)]))]
    tables += [("sigma", dict(base, members=[(sg, 1e-4) for sg in (0.01, 0.02, 0.05, 0.1, 0.2, 0.4)]))]
    tables += [("n_t", dict(base, n_t=nt)) for nt in (4, 16, 64)]
    tables += [("(m, p)", dict(base, M=M, P=P)) for M, P in ((4, 4), (6, 3))]
    stream = torch.cuda.Stream()
    rows = []
    for table, c in tables:
        tgt = np.tile(sg_inputs.indicator_target(c["n"]), (c["n_t"], 1))
        probs = [sgl.ProblemData(c["n"], c["M"], c["P"], sg, b, tgt, gamma=1.0, n_t=c["n_t"], T=1.0,
                                 field=sgl.SG_FIELD_LOGNORMAL) for sg, b in c["members"]]
        for tol in (1e-6, 1e-4):
            for name, r in (("1", 1), ("m+1", c["M"] + 1), ("n_A", 0)):
                print(f"[bench] paper parabolic {table}: n={c['n']} m={c['M']} p={c['P']} n_t={c['n_t']} "
                      f"tol={tol:g} n_tau={name}", file=sys.stderr, flush=True)
                opts = sgl.default_options(rtol=tol, truncation_r=r, mean_solver=1, max_iter=600)
                dt, infos = timed_solves(torch, sgl, probs, opts, 1, 1, stream)
                last = infos[-1]
                rows.append({"table": table, "n": c["n"], "m": c["M"], "p": c["P"], "n_t": c["n_t"],
                             "members": [list(mb) for mb in c["members"]], "tol": tol, "n_tau": name,
                             "iterations": [i.iters for i in last], "ms_per_solve": 1000.0 * dt / len(probs),
                             "converged": all(i.converged == 1 for i in last)})
                print(json.dumps(rows[-1]), flush=True)
    return {"paper_parabolic": rows}


def cpu_baseline(wl, gpu_iters):
    """The oracle (plain FP64 numpy/scipy, BLAS threaded over every core this
    process may use) timed on the first member at the workload size.

    When one oracle FGMRES iteration (one preconditioner application: the
    Chebyshev mass blocks and two hGS sweeps with multigrid inner solves; one
    matricized KKT apply; the Gram-Schmidt work of an average Arnoldi step)
    takes a few seconds, whole iterations are timed for about 10 s.  At sizes
    where one iteration takes longer, its parts are timed once each (one KKT
    apply, the mass blocks, one hGS sweep counted twice, the Schur mass
    product, Gram-Schmidt on 4 vectors scaled to 15) and summed: a projected
    iteration.  Either way the per-iteration time is scaled by the GPU run's
    iterations per solve."""
    from threadpoolctl import threadpool_limits

    import sg_inputs
    from oracle import kkt, precond

    cores = len(os.sched_getaffinity(0))
    with threadpool_limits(limits=cores):
        if wl["n_t"] > 1:
            tgt = sg_inputs.moving_bump(wl["n"], wl["n_t"], 1.0, wl["seeds"][0])
        else:
            tgt = sg_inputs.gaussian_bumps(wl["n"], wl["seeds"][0])
        prob = kkt.Problem(n=wl["n"], M=wl["M"], P=wl["P"], sigma=wl["sigma"], beta=wl["betas"][0],
                           n_t=wl["n_t"], y_target=tgt)
        sg = kkt.setup(prob)
        inner = precond.make_inner(sg)
        r = kkt.rhs(sg)
        t0 = time.perf_counter()
        w = kkt.kkt_apply_matricized(sg, r)
        t_kkt = time.perf_counter() - t0
        if t_kkt < 2.0:
            V = np.random.default_rng(0).standard_normal((15, r.size))
            reps, t0 = 0, time.perf_counter()
            while True:   # whole iterations until at least 10 s of CPU work
                z = precond.precond_apply(sg, r, inner)
                w = kkt.kkt_apply_matricized(sg, z)
                for _ in range(2):          # Arnoldi work of an average iteration (15 basis vectors)
                    hcoef = V @ w
                    w = w - V.T @ hcoef
                reps += 1
                if time.perf_counter() - t0 >= 10.0:
                    break
            t_iter = (time.perf_counter() - t0) / reps
            sample = (f"{reps} whole FGMRES iterations of the oracle on the first member at the workload size "
                      f"({t_iter:.2f} s each, {cores} threads), scaled by {gpu_iters:.1f} iterations per solve")
            kind = "oracle"
        else:
            Ry, Ru, Rl = kkt.split(sg, r)
            t0 = time.perf_counter()
            if prob.steady:
                precond.kkt_cheb(sg, Ry, 5)
                precond.kkt_cheb(sg, Ru, 5)
            else:
                for t in range(prob.n_t):
                    precond.kkt_cheb(sg, Ry[t], 5)
                    precond.kkt_cheb(sg, Ru[t], 5)
            t_cheb = time.perf_counter() - t0
            R0 = Rl if prob.steady else Rl[0]
            t0 = time.perf_counter()
            V1 = precond.hgs(sg, R0, inner, prob.M + 1)
            t_hgs = (time.perf_counter() - t0) * (1 if prob.steady else prob.n_t)
            t0 = time.perf_counter()
            kkt.mass_apply(sg, V1)
            t_mass = (time.perf_counter() - t0) * (1 if prob.steady else prob.n_t)
            V = np.random.default_rng(0).standard_normal((4, r.size))
            t0 = time.perf_counter()
            for _ in range(2):
                hcoef = V @ w
                w = w - V.T @ hcoef
            t_gs = (time.perf_counter() - t0) * 15.0 / 4.0
            del V
            t_iter = t_kkt + t_cheb + 2 * t_hgs + t_mass + t_gs
            sample = (f"projected: one oracle FGMRES iteration on the first member at the workload size, from its "
                      f"parts timed once each with {cores} threads (KKT apply {t_kkt:.1f} s, mass blocks "
                      f"{t_cheb:.1f} s, 2 x hGS sweep {t_hgs:.1f} s, Schur mass product {t_mass:.1f} s, "
                      f"Gram-Schmidt {t_gs:.1f} s; {t_iter:.1f} s per iteration), scaled by {gpu_iters:.1f} "
                      f"iterations per solve")
            kind = "oracle"
    per_solve = t_iter * gpu_iters
    return dict(value=1.0 / per_solve, unit="solves/s", cores=cores, kind=kind, sample=sample,
                projected=t_kkt >= 2.0, s_per_iteration=t_iter)


def residual_check(wl, x_canonical, reported, nrows=10000, seed=17):
    """The oracle's check of a GPU solution: the FP64 residual b - K x on
    `nrows` seeded random rows of the explicit KKT system (every block), the
    norm estimate sqrt(N/S sum r_i^2) / ||b|| against the solver's reported
    relative residual, and the largest sampled |r_i| / ||b||."""
    import sg_inputs
    from oracle import fem, kkt

    if wl["n_t"] > 1:
        tgt = sg_inputs.moving_bump(wl["n"], wl["n_t"], 1.0, wl["seeds"][0])
    else:
        tgt = sg_inputs.gaussian_bumps(wl["n"], wl["seeds"][0])
    prob = kkt.Problem(n=wl["n"], M=wl["M"], P=wl["P"], sigma=wl["sigma"], beta=wl["betas"][0],
                       n_t=wl["n_t"], y_target=tgt)
    sg = kkt.setup(prob)
    nt = max(wl["n_t"], 1)
    V = np.asarray(x_canonical).reshape(3, nt, sg.n_xi, -1)
    blocks = [fem.extract(V[i], wl["n"]) for i in range(3)]
    if prob.steady:
        blocks = [b[0] for b in blocks]
    x = np.concatenate([b.reshape(-1) for b in blocks])
    del V, blocks
    b = kkt.rhs(sg)
    rows = np.sort(np.random.default_rng(seed).choice(b.size, size=min(nrows, b.size), replace=False))
    r = b[rows] - kkt.kkt_rows(sg, x, rows)
    bn = float(np.linalg.norm(b))
    est = float(np.sqrt(b.size / rows.size * np.sum(r * r))) / bn
    return {"rows": int(rows.size), "seed": seed, "unknowns": int(b.size), "estimated_rel_res": est,
            "reported_rel_res": reported, "max_sampled_abs_res_over_norm_b": float(np.max(np.abs(r))) / bn,
            "ok": bool(est <= 3.0 * max(reported, 1e-16) and np.max(np.abs(r)) / bn <= 1e-8)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--profile-kernel", default="auto", choices=["auto"] + sorted(PROF_KIND),
                    help="kernel reported as roofline (auto: the one with the largest measured total time)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=256,
                    help="requests of the serving comparison (all queued at time zero; 0: skip)")
    ap.add_argument("--serve-grids", default="32,64,128,256", help="grid sizes n the request mix draws from")
    ap.add_argument("--paper-tables", action="store_true",
                    help="iterations and time per solve on the grid of the paper's tables of sigma variations "
                         "(log-normal field, n_xi = 20 / 70 / 84, n_tau = 1 / m+1 / n_A, Chebyshev-5 or direct "
                         "mass solves, sigma = 0.01 / 0.1 / 0.4), one JSON line per setting")
    ap.add_argument("--paper-parabolic", action="store_true",
                    help="iterations and time per solve on the settings of the paper's time-dependent tables "
                         "(log-normal field; mesh, beta, sigma, n_t and (m, p) variations; tolerances 1e-6 and "
                         "1e-4; n_tau = 1 / m+1 / n_A), one JSON line per setting")
    ap.add_argument("--paper-grids", default="16,32,64,128", help="element counts per side for --paper-tables")
    ap.add_argument("--paper-mean", default="direct", choices=["direct", "multigrid"],
                    help="mean-block solves for --paper-tables")
    ap.add_argument("--serve-sweep", action="store_true",
                    help="only run the mixed serving protocol (capacity of FP64 serving, FP32-refinement "
                         "serving and plain FP64 single solves, then Poisson arrivals at 0.5x and 1.5x the "
                         "FP64 serving capacity) and print its JSON")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy a 1 GiB FP64 tensor three times (calibrates hardware byte counters) and exit")
    ap.add_argument("--kernel-probe", choices=["apply", "kkt", "precond"],
                    help="only apply the SG operator, the KKT matrix or the preconditioner (FP64, one vector of the "
                         "workload's first problem, strips of --sweep-rows or autotuned) --probe-reps times after one "
                         "warm-up, and exit (the kernels' hardware counters are taken on this)")
    ap.add_argument("--probe-reps", type=int, default=5)
    ap.add_argument("--probe-options", default="{}",
                    help='sg_options overrides for --kernel-probe as JSON, e.g. \'{"mean_solver": 1}\'')
    ap.add_argument("--precond-variants", action="store_true",
                    help="iterations and solves/s of the preconditioner variants of Section 5 on --workload "
                         "(Chebyshev 5/10 or exact mass solves; multigrid or exact mean-block solves; "
                         "Richardson steps; truncation)")
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

    if args.kernel_probe:
        wl = WORKLOADS[args.workload]
        h = sgl.Handle(make_problems(sgl, sg_inputs, wl)[:1],
                       sgl.default_options(sweep_rows=args.sweep_rows, **json.loads(args.probe_options)))
        per = h.block_elems if args.kernel_probe == "apply" else h.kkt_elems
        x = torch.rand(per, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        fn = {"apply": h.apply_operator, "kkt": h.apply_kkt, "precond": h.precond_apply}[args.kernel_probe]
        fn(x, y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.probe_reps):
            fn(x, y)
        torch.cuda.synchronize()
        print(json.dumps({"kernel_probe": args.kernel_probe, "workload": args.workload, "reps": args.probe_reps,
                          "options": json.loads(args.probe_options),
                          "ms_per_apply": 1000.0 * (time.perf_counter() - t0) / args.probe_reps,
                          "sweep_rows": [list(r) for r in h.sizes.sweep_rows]}))
        h.close()
        return

    if args.precond_variants:
        print(json.dumps(precond_variants(torch, sgl, sg_inputs, args.workload, args.steps, args.warmup)), flush=True)
        return
    if args.paper_parabolic:
        paper_parabolic(torch, sgl, sg_inputs)
        return
    if args.paper_tables:
        paper_tables(torch, sgl, sg_inputs, tuple(int(g) for g in args.paper_grids.split(",")), args.paper_mean)
        return

    grids = tuple(int(g) for g in args.serve_grids.split(","))
    if args.serve_sweep:
        print(json.dumps(serving_sweep(torch, sgl, sg_inputs, args.serve_requests, grids)), flush=True)
        return

    def say(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    wl = WORKLOADS[args.workload]
    probs = make_problems(sgl, sg_inputs, wl)
    stream = torch.cuda.Stream()

    graphs = 0 if args.no_graphs else 1
    # headline: FP64 batch (the whole beta sweep) per step
    arn = ARNOLDI[args.arnoldi]
    opts = sgl.default_options(rtol=1e-8, use_graphs=graphs, arnoldi=arn, sweep_rows=args.sweep_rows)
    tuned = []
    x64 = []
    say(f"headline {args.workload}: {args.warmup} warmup + {args.steps} timed FP64 solves")
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
    say("per-kernel event timing")
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
        # the library's model of every member's algorithmic HBM bytes (sg_solve_info.bytes_moved),
        # over the timed steps' wall time: the whole solve's average bandwidth
        "solve_model": {"bytes_per_step": sum(i.bytes_moved for i in infos[-1]),
                        "GBps": sum(i.bytes_moved for step in infos for i in step) / dt / 1e9,
                        "frac_of_hbm_peak": sum(i.bytes_moved for step in infos for i in step) / dt / 1e9
                        / HBM_PEAK_GBPS},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": kd["achieved_GBps"], "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": kd["achieved_GBps"] / HBM_PEAK_GBPS,
                     "traffic": measured_traffic(dom, args.workload),
                     "launches": kd["launches"], "avg_launch_ms": kd["avg_launch_ms"],
                     "bytes_per_launch": kd["bytes_per_launch"]},
        "kernels": kern,
    }
    if not args.no_extras:
        say("SG operator apply bandwidth")
        out["sg_apply"] = sg_apply_bandwidth(torch, sgl, probs, stream)
        out["sg_apply"]["frac_of_hbm_peak"] = out["sg_apply"]["GBps"] / HBM_PEAK_GBPS
        hk = sgl.Handle(probs, sgl.default_options(), stream=stream)
        b = torch.zeros(hk.members * hk.kkt_elems, dtype=torch.float64, device="cuda")
        hk.rhs(b)
        bnorm = b.view(hk.members, -1).norm(dim=1)

        def residual_gap(xa, xb):
            """max over members of ||K (xa - xb)|| / ||b||: how far apart two
            solutions are in the residual norm the solver stops on."""
            d = (xa - xb).reshape(-1).contiguous()
            kd_ = torch.empty_like(d)
            torch.cuda.synchronize()     # d is formed on torch's stream, the library reads it on `stream`
            hk.apply_kkt(d, kd_, stream=stream)
            torch.cuda.synchronize()
            return float((kd_.view(hk.members, -1).norm(dim=1) / bnorm).max())

        for label, prec, basis32, dtype in (
                ("fp32_refine", sgl.SG_PREC_FP32_REFINE, 1,
                 "inner cycles: f32 storage of operator input/output, preconditioner and Arnoldi basis, f64 stiffness "
                 "and Arnoldi sums; f64 residual and refinement"),
                ("fp32_refine_f64_basis", sgl.SG_PREC_FP32_REFINE, 0,
                 "inner cycles: f32 storage of operator input/output and preconditioner, f64 Arnoldi basis; f64 "
                 "residual and refinement"),
                ("fp32_precond", sgl.SG_PREC_FP32_PRECOND, 1,
                 "f32 preconditioner, f64 operator, Arnoldi and restarts")):
            say(f"{label}: {args.steps} timed solves")
            o = sgl.default_options(rtol=1e-8, precision=prec, use_graphs=graphs, arnoldi=arn,
                                    sweep_rows=args.sweep_rows, basis_fp32=basis32)
            xk = []
            dtk, infk = timed_solves(torch, sgl, probs, o, args.steps, 1, stream, keep=xk)
            out[label] = {"value": nsolve / dtk, "unit": "solves/s", "dtype": dtype,
                          "iterations": [i.iters for i in infk[0]],
                          "outer_refinements": [i.outer_refinements for i in infk[0]],
                          "max_rel_res": max(i.rel_res_true for st in infk for i in st),
                          "max_rel_diff_vs_fp64": max_rel_diff(xk[0], x64[0]),
                          "max_residual_gap_vs_fp64": residual_gap(xk[0], x64[0])}
            del xk
        hk.close()
        say("plain FP64 single solves")
        single = []
        t_single = 0.0
        for p in probs:
            sopt = sgl.default_options(rtol=1e-8, use_graphs=graphs, arnoldi=arn, sweep_rows=args.sweep_rows)
            dts, infs = timed_solves(torch, sgl, [p], sopt, 1, 1, stream)
            t_single += dts
            single.append(infs[0][0].iters)
        out["fp64_single"] = {"value": len(probs) / t_single, "unit": "solves/s", "iterations": single}
    if not args.no_extras and args.serve_requests > 0:
        say(f"serving comparison: {args.serve_requests} requests on grids {grids}")
        out["serving"] = serving_compare(torch, sgl, sg_inputs, args.serve_requests, grids)
    xsol = x64[0][0].cpu().numpy()
    del x64
    if not args.no_cpu_baseline:
        say("CPU baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(wl, float(np.mean(iters)))
        say("oracle residual check of the FP64 solution on sampled KKT rows")
        out["residual_check"] = residual_check(wl, xsol, infos[-1][0].rel_res_true)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
