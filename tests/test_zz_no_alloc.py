"""GPU test of sg_precond_apply_noalloc, the preconditioner entry point that
allocates nothing (its scratch is the library's fixed device array), against
sg_precond_apply on the same handles and inputs, through the C ABI.

The two entry points run the same kernels in the same order, so their
outputs must be identical.  Two calls in a row on different handles, the
second with a smaller input, check that nothing the first call left in the
shared scratch array leaks into the second.
"""
import sys

import numpy as np
import pytest

from _helpers import make_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _handle(cases, **opt):
    import paper_2512_23804_amd as sgl
    probs = [sgl.ProblemData(**make_case(*c)[1]) for c in cases]
    return sgl.Handle(probs, sgl.default_options(**opt))


def _compare(h, dtype, seed):
    """sg_precond_apply and sg_precond_apply_noalloc on one seeded input
    (every member); the outputs start as different NaN-free garbage so that
    unwritten entries would show."""
    dev = _dev()
    g = torch.Generator(device="cpu").manual_seed(seed)
    n_el = h.members * h.kkt_elems
    r = torch.randn(n_el, generator=g, dtype=torch.float64).to(dev, dtype)
    z_ref = torch.full((n_el,), 7.0, dtype=dtype, device=dev)
    z_na = torch.full((n_el,), -3.0, dtype=dtype, device=dev)
    h.precond_apply(r, z_ref)
    h.precond_apply_noalloc(r, z_na)
    torch.cuda.synchronize()
    assert torch.isfinite(z_na).all()
    scale = float(z_ref.abs().max())
    err = float((z_na - z_ref).abs().max()) / scale
    assert err <= (1e-12 if dtype == torch.float64 else 1e-5), err
    assert torch.equal(z_na, z_ref)


# (n, M, P, sigma, beta, gamma, n_t) per member
BIG = [(32, 4, 3, 0.2, 1e-2, 0.0, 1), (32, 4, 3, 0.25, 1e-4, 0.5, 1)]
SMALL = [(16, 3, 2, 0.2, 1e-3, 0.0, 1)]
TIME = [(16, 2, 3, 0.3, 1e-3, 0.0, 4)]


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_noalloc_matches_precond_apply_two_calls(dtype):
    dt = torch.float64 if dtype == "fp64" else torch.float32
    _say(f"noalloc {dtype}: batch of 2 at 32x32, M=4, P=3")
    h1 = _handle(BIG)
    _compare(h1, dt, 1)
    _say(f"noalloc {dtype}: then one member at 16x16, M=3, P=2 (smaller)")
    h2 = _handle(SMALL)
    _compare(h2, dt, 2)
    _say(f"noalloc {dtype}: the first handle again")
    _compare(h1, dt, 3)
    h1.close()
    h2.close()


def test_noalloc_time_dependent_and_per_step_chebyshev():
    _say("noalloc: heat 16x16, n_t=4, 12 Chebyshev steps (per-step kernel and its buffers)")
    h = _handle(TIME, cheb_steps=12)
    _compare(h, torch.float64, 4)
    h.close()
    _say("noalloc: heat 16x16, n_t=4, 5 Chebyshev steps")
    h = _handle(TIME)
    _compare(h, torch.float64, 5)
    h.close()


def test_noalloc_rejects_sizes_beyond_the_scratch():
    import paper_2512_23804_amd as sgl
    dev = _dev()
    _say("noalloc: 256x256, M=4, P=4 needs more than the fixed scratch")
    h = _handle([(256, 4, 4, 0.2, 1e-2, 0.0, 1)])
    r = torch.ones(h.kkt_elems, dtype=torch.float64, device=dev)
    z = torch.full_like(r, 5.0)
    rc = h.precond_apply_noalloc(r, z, allow=(sgl.SG_OK, sgl.SG_ERR_NOMEM))
    torch.cuda.synchronize()
    assert rc == sgl.SG_ERR_NOMEM
    assert "fixed maximum" in sgl.lib.sg_last_error().decode()
    assert bool((z == 5.0).all())          # nothing was launched
    h.close()
    _say("noalloc: a call that fits still works after the rejection")
    h2 = _handle(SMALL)
    _compare(h2, torch.float64, 6)
    h2.close()


def test_noalloc_level_kernels_above_the_tail():
    """A 128 x 128 grid: the multigrid level kernels above the fused tail run,
    with the pre-smoothed iterate the down kernel stores for the up kernel
    carved from the fixed scratch like every other buffer (FP64, then FP32,
    then FP64 again on the same handle)."""
    _say("noalloc: 128x128, M=2, P=1 (multigrid level kernels)")
    h = _handle([(128, 2, 1, 0.25, 1e-3, 0.0, 1)])
    _compare(h, torch.float64, 7)
    _compare(h, torch.float32, 8)
    _compare(h, torch.float64, 9)
    h.close()
