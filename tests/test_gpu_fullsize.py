"""GPU parity at the benchmark workloads' full sizes, on the problems, batch and
options that bench.py times (its WORKLOADS table), through the C ABI.

* applies: every output entry of the batched KKT apply (and of the
  preconditioner where the oracle finishes in seconds) against the oracle,
  FP64 within 1e-12 and FP32 within 1e-5 of the reference's max-norm;
* solves: the FP64 true residual ||b - K x|| / ||b|| of each member's GPU
  solution, recomputed by the oracle's own KKT apply, meets the 1e-8
  stopping tolerance and matches the residual the solver reports.
"""
import os
import sys

import numpy as np
import pytest

from _helpers import canonical_to_kkt, kkt_to_canonical, make_case, rel_max
from oracle import kkt, precond

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402  (the workload table bench.py times)


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _members(name):
    wl = bench.WORKLOADS[name]
    return [make_case(wl["n"], wl["M"], wl["P"], wl["sigma"], beta, 0.0, wl["n_t"], 1.0, seed)
            for beta, seed in zip(wl["betas"], wl["seeds"])]


def _handle(cases, **opt):
    import paper_2512_23804_amd as sgl
    return sgl.Handle([sgl.ProblemData(**kw) for _, kw in cases], sgl.default_options(**opt))


@pytest.mark.parametrize("name", ["steady-128-M6-P4", "heat-64-M4-P3-nt32", "steady-512-M8-P3", "steady-256-M8-P4"])
def test_fullsize_applies(name):
    _need_gpu()
    _say(f"full-size applies {name}")
    cases = _members(name)
    sgs = [kkt.setup(p) for p, _ in cases]
    h = _handle(cases)
    rng = np.random.default_rng(3)
    xs = [rng.uniform(-1, 1, size=kkt.rhs(sg).size) for sg in sgs]
    xd = torch.from_numpy(np.concatenate([kkt_to_canonical(sg, x) for sg, x in zip(sgs, xs)])).cuda()
    with_precond = bench.WORKLOADS[name]["n"] <= 128      # the oracle's hGS beyond 128 x 128 takes minutes
    outs = {}
    for dt in (torch.float64, torch.float32):
        xi = xd.to(dt)
        y = torch.zeros_like(xi)
        h.apply_kkt(xi, y)
        outs[("kkt", dt)] = y
        if with_precond:
            z = torch.zeros_like(xi)
            h.precond_apply(xi, z)
            outs[("pc", dt)] = z
    torch.cuda.synchronize()
    E = h.kkt_elems
    for i, (sg, x) in enumerate(zip(sgs, xs)):
        refs = {"kkt": kkt.kkt_apply_matricized(sg, x)}
        if with_precond:
            refs["pc"] = precond.precond_apply(sg, x, precond.make_inner(sg))
        for (what, dt), out in outs.items():
            got = canonical_to_kkt(sg, out[i * E:(i + 1) * E].double().cpu().numpy())
            err = rel_max(got, refs[what])
            assert err < (1e-12 if dt == torch.float64 else 1e-5), (name, i, what, dt, err)


@pytest.mark.parametrize("precision", [0, 1, 2], ids=["fp64", "fp32_refine", "fp32_precond"])
@pytest.mark.parametrize("name", sorted(bench.WORKLOADS))
def test_fullsize_solve_true_residual(name, precision):
    """Each member's GPU solution at the benchmark size, in every precision
    mode: the oracle's FP64 residual ||b - K x|| / ||b|| <= 1e-8 and within 1%
    of the residual the solver reports."""
    _need_gpu()
    _say(f"full-size solve {name} precision={precision}")
    cases = _members(name)
    h = _handle(cases, rtol=1e-8, precision=precision)
    x = torch.zeros(h.members * h.kkt_elems, dtype=torch.float64, device="cuda")
    rc, infos = h.solve(x)
    torch.cuda.synchronize()
    assert rc == 0
    X = x.cpu().numpy()
    E = h.kkt_elems
    for i, (prob, _) in enumerate(cases):
        sg = kkt.setup(prob)
        xi = canonical_to_kkt(sg, X[i * E:(i + 1) * E])
        b = kkt.rhs(sg)
        rel = np.linalg.norm(b - kkt.kkt_apply_matricized(sg, xi)) / np.linalg.norm(b)
        assert rel <= 1e-8, (name, i, rel)
        assert abs(rel - infos[i].rel_res_true) <= 1e-2 * rel + 1e-12, (name, i, rel, infos[i].rel_res_true)
