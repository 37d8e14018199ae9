"""GPU parity at the limits the C ABI accepts.

* The largest grid, n = 4096 (16.8 M nodes per chaos column): the operator
  apply compared with the oracle's element-by-element whole-grid product on
  every node, and an FP64 solve whose KKT residual the oracle recomputes on
  every row (oracle/local.py; assembling the sparse matrices is not wanted at
  this size).
* The most modes (M = 16, the gather kernels), the highest degree (P = 8,
  nine degree levels in the hGS sweeps) and both at once at n = 8 (n_xi =
  153): operator, KKT and preconditioner applies and solves against the
  oracle, through the same checks as the main parity tests.
* A zero right-hand side: the solve starts converged (x = 0, no iterations),
  alone and beside a member with a nonzero target, which keeps its alone
  result bit for bit.

Tolerances: operator within 1e-12 of the oracle's max-norm; solutions within
1e-8 (the main parity tests' bars); the recomputed relative residual below
the solver's 1e-8.  At n = 4096 the residual itself carries a rounding floor:
the stiffness rows are O(1) combinations of the solution while ||b|| is a mass
product of size h^2 = 6e-8, so evaluating b - K x in FP64 leaves about
eps / h^2 ~ 4e-9 relative to ||b||; the oracle's and the library's figures
(different summation orders) are required to agree within 2.5e-9.
"""
from types import SimpleNamespace

import numpy as np
import pytest
import torch

from _helpers import make_case, rel_max, ring_is_zero
from oracle import basis, fem, kkt, local
from test_gpu_parity import test_kkt_apply as kkt_apply_case
from test_gpu_parity import test_operator_apply as operator_apply_case
from test_gpu_parity import test_precond_apply as precond_apply_case
from test_gpu_parity import test_solve_matches_direct as solve_case

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _handle(kws, **opt):
    import paper_2512_23804_amd as sgl
    return sgl.Handle([sgl.ProblemData(**kw) for kw in kws], sgl.default_options(**opt))


NMAX = 4096


def test_max_grid_operator_apply():
    dev = _dev()
    n, M, P, sigma = NMAX, 1, 1, 0.3
    _say(f"operator apply n={n} M={M} P={P}")
    _, kw = make_case(n, M, P, sigma, 1e-2)
    h = _handle([kw])
    nxi = h.sizes.n_xi
    X = np.random.default_rng(5).uniform(-1, 1, size=(1, 1, nxi, (n + 1) ** 2))
    Xd = torch.from_numpy(X).to(dev)
    Yd = torch.full_like(Xd, np.nan)
    h.apply_operator(Xd, Yd)
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy()
    del Xd, Yd
    assert ring_is_zero(Y, n)
    ref = local.operator(n, fem.cosine_modes(n, M, sigma), basis.triple_product_matrices(M, P), X[0, 0])
    assert rel_max(fem.extract(Y[0, 0], n), ref) < 1e-12


def test_max_grid_solve_residual():
    dev = _dev()
    n, M, P, sigma, beta = NMAX, 1, 1, 0.3, 1e-2
    _say(f"solve n={n} M={M} P={P}")
    prob, kw = make_case(n, M, P, sigma, beta)
    h = _handle([kw], rtol=1e-8)
    xd = torch.zeros(h.kkt_elems, dtype=torch.float64, device=dev)
    rc, info = h.solve(xd)
    torch.cuda.synchronize()
    assert rc == 0 and info[0].converged == 1
    reported = info[0].rel_res_true
    assert reported <= 1e-8
    nxi = h.sizes.n_xi
    V = xd.cpu().numpy().reshape(3, nxi, (n + 1) ** 2)
    del xd
    hg = kkt.h_gamma(SimpleNamespace(n_xi=nxi, prob=prob))
    ry, ru, rl, by = local.kkt_residual_steady(n, fem.cosine_modes(n, M, sigma), basis.triple_product_matrices(M, P),
                                               hg, beta, prob.y_target, V[0], V[1], V[2])
    rel = np.sqrt(np.sum(ry * ry) + np.sum(ru * ru) + np.sum(rl * rl)) / np.linalg.norm(by)
    _say(f"n={n}: {info[0].iters} iterations, reported {reported:.3e}, oracle {rel:.3e}")
    assert rel <= 1e-8
    assert abs(rel - reported) <= 2.5e-9


# n, M, P, sigma, beta, gamma, n_t
LIMIT_SHAPES = [
    (16, 16, 1, 0.2, 1e-2, 0.0, 1),     # M = 16: the most modes
    (16, 1, 8, 0.3, 1e-2, 0.3, 1),      # P = 8: the highest degree, nine degree levels
    (8, 16, 2, 0.2, 1e-3, 0.0, 1),      # both large: n_xi = 153
    (8, 16, 1, 0.2, 1e-2, 0.0, 3),      # M = 16, time-dependent
]


@pytest.mark.parametrize("shape", LIMIT_SHAPES)
def test_limit_shapes_applies(shape):
    operator_apply_case(shape)
    kkt_apply_case(shape)
    precond_apply_case(shape, 1)
    precond_apply_case(shape, 0)


@pytest.mark.parametrize("shape", LIMIT_SHAPES)
def test_limit_shapes_solve(shape):
    solve_case(shape, 0)


def test_zero_target_starts_converged():
    dev = _dev()
    n, M, P = 16, 3, 2
    _say("zero right-hand side")
    _, kw_zero = make_case(n, M, P, 0.2, 1e-2)
    kw_zero["y_target"] = np.zeros_like(kw_zero["y_target"])
    _, kw = make_case(n, M, P, 0.25, 1e-3, seed=2)
    h0 = _handle([kw_zero], rtol=1e-10)
    x0 = torch.full((h0.kkt_elems,), np.nan, dtype=torch.float64, device=dev)
    rc, info = h0.solve(x0)
    torch.cuda.synchronize()
    assert rc == 0 and info[0].converged == 1 and info[0].iters == 0 and info[0].rel_res_true == 0.0
    assert torch.all(x0 == 0).item()
    # beside a member with a target: that member's result is its alone result
    ha = _handle([kw], rtol=1e-10)
    xa = torch.zeros(ha.kkt_elems, dtype=torch.float64, device=dev)
    rca, ia = ha.solve(xa)
    hb = _handle([kw_zero, kw], rtol=1e-10)
    xb = torch.zeros(2 * hb.kkt_elems, dtype=torch.float64, device=dev)
    rcb, ib = hb.solve(xb)
    torch.cuda.synchronize()
    assert rca == 0 and rcb == 0
    half = xa.numel()
    assert torch.all(xb[:half] == 0).item()
    assert torch.equal(xb[half:], xa)
    assert ib[0].iters == 0 and ib[1].iters == ia[0].iters and ib[1].rel_res_true == ia[0].rel_res_true
