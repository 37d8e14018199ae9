"""Test helpers: problem construction for both sides and layout conversion
between the oracle's interior blocks and the library's canonical layout."""
from __future__ import annotations

import numpy as np

import sg_inputs
from oracle import fem, kkt


def make_case(n, M, P, sigma, beta, gamma=0.0, n_t=1, T=1.0, seed=0, y0=False, kappa=None, field="affine",
              corr=1.0):
    """Return (oracle Problem, dict of library ProblemData kwargs) built from the
    same seeded inputs.  field="lognormal": the log-normal coefficient with
    Hermite chaos and, when steady, the indicator target of Section 5."""
    if field == "lognormal" and n_t <= 1:
        target = sg_inputs.indicator_target(n)
    elif n_t <= 1:
        target = sg_inputs.gaussian_bumps(n, seed)
    else:
        target = sg_inputs.moving_bump(n, n_t, T, seed)
    y0v = None
    if y0:
        y0v = sg_inputs.gaussian_bumps(n, seed + 100) * sg_inputs.unit_sine(n)
    prob = kkt.Problem(n=n, M=M, P=P, sigma=sigma, beta=beta, gamma=gamma, n_t=n_t, T=T,
                       y_target=target, kappa=kappa, y0=y0v, field=field, corr=corr)
    lib_kw = dict(n=n, M=M, P=P, sigma=sigma, beta=beta, y_target=target, gamma=gamma, n_t=n_t, T=T,
                  kappa=kappa, y0=y0v, field=1 if field == "lognormal" else 0, corr_len=corr)
    return prob, lib_kw


def block_to_canonical(B: np.ndarray, n: int) -> np.ndarray:
    """(..., n_int) interior arrays -> (..., (n+1)^2) full-grid arrays."""
    return fem.embed(B, n)


def canonical_to_block(V: np.ndarray, n: int) -> np.ndarray:
    return fem.extract(V, n)


def kkt_to_canonical(sg: kkt.SG, x: np.ndarray) -> np.ndarray:
    """Oracle flat KKT vector -> canonical [3][n_t][n_xi][(n+1)^2] flat array."""
    n = sg.prob.n
    parts = [block_to_canonical(b, n) for b in kkt.split(sg, x)]
    return np.concatenate([p.reshape(-1) for p in parts])


def canonical_to_kkt(sg: kkt.SG, v: np.ndarray) -> np.ndarray:
    n = sg.prob.n
    nt = max(sg.prob.n_t, 1)
    shp = (3, nt, sg.n_xi, (n + 1) ** 2)
    V = np.asarray(v).reshape(shp)
    blocks = [canonical_to_block(V[i], n) for i in range(3)]
    if sg.prob.steady:
        blocks = [b[0] for b in blocks]
    return np.concatenate([b.reshape(-1) for b in blocks])


def rel_max(a: np.ndarray, ref: np.ndarray) -> float:
    """max |a - ref| / max |ref| (element-wise comparison scaled by the reference's size)."""
    scale = np.max(np.abs(ref))
    return float(np.max(np.abs(a - ref)) / (scale if scale > 0 else 1.0))


def ring_is_zero(v: np.ndarray, n: int) -> bool:
    g = np.asarray(v).reshape(-1, n + 1, n + 1)
    return bool(np.all(g[:, 0, :] == 0) and np.all(g[:, -1, :] == 0) and np.all(g[:, :, 0] == 0)
                and np.all(g[:, :, -1] == 0))
