"""GPU tests of the continuous-batching server (sg_server_* / sg_submit / sg_poll).

Requests of mixed shapes arrive over time; requests that arrive while others
run are admitted as slots and memory free up and same-shape requests are solved
as one batch.  Every result must equal (bit for bit) the result of solving that
request alone with the same options.
"""
import sys
import time
from math import comb

import numpy as np
import pytest

import sg_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    import paper_2512_23804_amd as sgl
    return sgl


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _kkt_len(n, M, P):
    return 3 * comb(M + P, P) * (n + 1) ** 2


def _wait(srv, tickets, timeout=120.0):
    sgl = _lib()
    t0 = time.time()
    res = {}
    pending = set(tickets)
    while pending and time.time() - t0 < timeout:
        for t in list(pending):
            rc, info = srv.poll(t)
            if rc != sgl.SG_PENDING:
                res[t] = (rc, info)
                pending.discard(t)
        time.sleep(0.002)
    assert not pending, f"{len(pending)} requests did not finish"
    return res


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_server_results_equal_alone(precision):
    _need_gpu()
    sgl = _lib()
    _say(f"serving mix precision={precision}")
    reqs = sg_inputs.serving_stream(12, seed=7, rate_per_s=400.0, grid_choices=(16, 32), M_range=(2, 4),
                                    P_range=(2, 3))
    opts = sgl.default_options(rtol=1e-8, precision=precision)
    srv = sgl.Server(hbm_budget_bytes=0, max_slots=8)
    tickets, items = [], []
    t0 = time.time()
    for r in reqs:
        while time.time() - t0 < r["arrival"]:
            time.sleep(0.0005)
        pd = sgl.ProblemData(r["n"], r["M"], r["P"], r["sigma"], r["beta"], sg_inputs.gaussian_bumps(r["n"], r["seed"]))
        out = np.full(_kkt_len(r["n"], r["M"], r["P"]), np.nan)
        tickets.append(srv.submit(pd, out, opts))
        items.append((r, pd, out))
    res = _wait(srv, tickets)
    stats = srv.stats()
    srv.close()
    assert stats["completed"] == len(reqs) and stats["p99_ms"] >= stats["p50_ms"] > 0
    dev = torch.device("cuda:0")
    for t, (r, pd, out) in zip(tickets, items):
        rc, info = res[t]
        assert rc == sgl.SG_OK and info.converged == 1 and info.rel_res_true <= 1e-8
        assert info.latency_ms > 0
        h = sgl.Handle(pd, opts)
        x = torch.zeros(h.kkt_elems, dtype=torch.float64, device=dev)
        rca, infa = h.solve(x)
        assert rca == sgl.SG_OK and infa[0].iters == info.iters
        assert np.array_equal(x.cpu().numpy(), out), f"request {r} differs from its alone solve"
        h.close()


def test_server_cancel_and_admission():
    _need_gpu()
    sgl = _lib()
    _say("serving cancel/admission")
    srv = sgl.Server(hbm_budget_bytes=0, max_slots=1)
    big = sgl.ProblemData(64, 4, 3, 0.2, 1e-4, sg_inputs.gaussian_bumps(64, 1))
    small = sgl.ProblemData(16, 2, 2, 0.2, 1e-2, sg_inputs.gaussian_bumps(16, 2))
    out_big = np.zeros(_kkt_len(64, 4, 3))
    out_small = np.zeros(_kkt_len(16, 2, 2))
    t_big = srv.submit(big, out_big)
    t_small = srv.submit(small, out_small)         # waits for the only slot
    assert srv.cancel(t_small) == sgl.SG_OK
    res = _wait(srv, [t_big])
    assert res[t_big][0] == sgl.SG_OK
    rc, _ = srv.poll(t_small)
    assert rc == sgl.SG_ERR_CANCELLED
    assert srv.cancel(t_big) == sgl.SG_ERR_INVALID          # already finished
    assert srv.poll(987654)[0] == sgl.SG_ERR_UNKNOWN
    srv.close()
    # a request whose footprint can never fit the budget is rejected at submit
    tiny = sgl.Server(hbm_budget_bytes=1 << 20, max_slots=4)
    with pytest.raises(sgl.SGError) as e:
        tiny.submit(big, out_big)
    assert e.value.code == sgl.SG_ERR_NOMEM
    tiny.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_request_joins_running_batch(precision):
    """Two slots, three same-shape requests queued at once: a fast and a slow
    request run, the third waits; when the fast one ends, the third takes its
    slot in the running batch at the next restart boundary.  Every result
    equals its alone solve bit for bit."""
    _need_gpu()
    sgl = _lib()
    _say(f"serving join at restart precision={precision}")
    n, M, P = 32, 3, 2
    params = [(0.1, 1e-1, 11), (0.3, 1e-6, 12), (0.2, 1e-3, 13)]    # fast, slow (several cycles), joiner
    opts = sgl.default_options(rtol=1e-9, precision=precision, max_iter=600)
    srv = sgl.Server(hbm_budget_bytes=0, max_slots=2)
    tickets, items = [], []
    for sigma, beta, seed in params:
        pd = sgl.ProblemData(n, M, P, sigma, beta, sg_inputs.gaussian_bumps(n, seed))
        out = np.full(_kkt_len(n, M, P), np.nan)
        tickets.append(srv.submit(pd, out, opts))
        items.append((pd, out))
    res = _wait(srv, tickets)
    srv.close()
    infos = [res[t][1] for t in tickets]
    assert all(res[t][0] == sgl.SG_OK for t in tickets)
    assert [i.joined_batch for i in infos] == [0, 0, 1], [i.joined_batch for i in infos]
    assert infos[1].iters > infos[0].iters, [i.iters for i in infos]
    dev = torch.device("cuda:0")
    for (pd, out), info in zip(items, infos):
        h = sgl.Handle(pd, opts)
        x = torch.zeros(h.kkt_elems, dtype=torch.float64, device=dev)
        rca, infa = h.solve(x)
        assert rca == sgl.SG_OK and infa[0].iters == info.iters
        assert np.array_equal(x.cpu().numpy(), out)
        h.close()


def test_server_lognormal_requests_join_and_equal_alone():
    """Log-normal requests (Hermite chaos; each member's element couplings
    are rebuilt when a request takes a finished member's slot): every result
    equals its alone solve bit for bit."""
    _need_gpu()
    sgl = _lib()
    _say("serving log-normal requests")
    n, M, P = 16, 2, 2
    params = [(0.1, 1e-1, 1.0), (0.3, 1e-5, 0.5), (0.2, 1e-3, 2.0)]   # fast, slow, joiner (sigma, beta, corr)
    opts = sgl.default_options(rtol=1e-9, max_iter=600)
    srv = sgl.Server(hbm_budget_bytes=0, max_slots=2)
    tickets, items = [], []
    for sigma, beta, corr in params:
        pd = sgl.ProblemData(n, M, P, sigma, beta, sg_inputs.indicator_target(n), gamma=1.0,
                             field=sgl.SG_FIELD_LOGNORMAL, corr_len=corr)
        out = np.full(_kkt_len(n, M, P), np.nan)
        tickets.append(srv.submit(pd, out, opts))
        items.append((pd, out))
    res = _wait(srv, tickets)
    srv.close()
    infos = [res[t][1] for t in tickets]
    assert all(res[t][0] == sgl.SG_OK for t in tickets)
    assert infos[2].joined_batch == 1, [i.joined_batch for i in infos]
    dev = torch.device("cuda:0")
    for (pd, out), info in zip(items, infos):
        h = sgl.Handle(pd, opts)
        x = torch.zeros(h.kkt_elems, dtype=torch.float64, device=dev)
        rca, infa = h.solve(x)
        assert rca == sgl.SG_OK and infa[0].iters == info.iters
        assert np.array_equal(x.cpu().numpy(), out)
        h.close()
