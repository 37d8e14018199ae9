"""Seeded synthetic inputs for the stochastic-Galerkin optimal-control solver.

This module is shared by the CPU oracle, the tests and the benchmark. It holds
no arithmetic of the method itself: it only draws seeded random numbers and
evaluates the target functions that define a workload at the grid nodes.

Grid convention (shared with the library's vector layout): the unit square
[0,1]^2 is split into n x n square Q1 elements, h = 1/n; node (ix, iy) sits at
(ix*h, iy*h) and has flat index iy*(n+1)+ix.

Workload recipes (the paper's experiments use a discontinuous quadrant target,
Section 5; the synthetic stand-ins here are seeded Gaussian-bump sums of the
same smooth-plus-localised character):
  * steady target: sum of `nbumps` Gaussian bumps, centres U(0.15,0.85)^2,
    widths U(0.05,0.15), amplitudes U(0.5,1.5);
  * moving target: one bump of width 0.1, amplitude 1, whose centre moves on a
    straight line from c0 to c1 (both U(0.2,0.8)^2) and is sampled at
    t_k = k*T/n_t, k = 1..n_t;
  * indicator target: 1 on [0,1/2]^2, else 0 (the paper's quadrant mapped to
    the unit square);
  * serving stream: request shapes and parameters drawn per the batched
    serving workload, with exponential inter-arrival gaps.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "node_coords",
    "gaussian_bumps",
    "moving_bump",
    "indicator_target",
    "random_block",
    "serving_stream",
    "field_modes",
]


def node_coords(n: int):
    """Return (x, y) arrays of length (n+1)^2 in flat node order iy*(n+1)+ix."""
    t = np.arange(n + 1, dtype=np.float64) / n
    y, x = np.meshgrid(t, t, indexing="ij")
    return x.reshape(-1), y.reshape(-1)


def _bumps(x, y, centres, widths, amps):
    out = np.zeros_like(x)
    for (cx, cy), s, a in zip(centres, widths, amps):
        out += a * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * s * s))
    return out


def gaussian_bumps(n: int, seed: int, nbumps: int = 4) -> np.ndarray:
    """Steady target: seeded sum of Gaussian bumps at the (n+1)^2 nodes (float64)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.15, 0.85, size=(nbumps, 2))
    widths = rng.uniform(0.05, 0.15, size=nbumps)
    amps = rng.uniform(0.5, 1.5, size=nbumps)
    x, y = node_coords(n)
    return _bumps(x, y, centres, widths, amps)


def moving_bump(n: int, n_t: int, T: float, seed: int) -> np.ndarray:
    """Time-dependent target: array [n_t][(n+1)^2] at t_k = k*T/n_t, k = 1..n_t."""
    rng = np.random.default_rng(seed)
    c0 = rng.uniform(0.2, 0.8, size=2)
    c1 = rng.uniform(0.2, 0.8, size=2)
    x, y = node_coords(n)
    out = np.empty((n_t, (n + 1) ** 2), dtype=np.float64)
    for k in range(1, n_t + 1):
        s = k / n_t
        c = c0 + s * (c1 - c0)
        out[k - 1] = _bumps(x, y, [c], [0.1], [1.0])
    return out


def indicator_target(n: int) -> np.ndarray:
    """1 on [0,1/2]^2 (closed), 0 elsewhere, at the (n+1)^2 nodes."""
    x, y = node_coords(n)
    return ((x <= 0.5) & (y <= 0.5)).astype(np.float64)


def random_block(shape, seed: int, dtype=np.float64) -> np.ndarray:
    """Uniform(-1,1) array of the given shape (operator-apply test inputs)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=shape).astype(dtype)


def serving_stream(num: int, seed: int, rate_per_s: float,
                   grid_choices=(32, 64, 128, 256), M_range=(4, 8), P_range=(2, 4),
                   sigma_range=(0.1, 0.3), beta_log10_range=(-6.0, -1.0)):
    """Draw `num` steady requests for the batched serving workload.

    Returns a list of dicts with keys n, M, P, sigma, beta, seed (target seed)
    and arrival (seconds since the stream start, Poisson process of the given
    rate).  Request i uses target seed 1000+i.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=num)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(num):
        n = int(rng.choice(grid_choices))
        M = int(rng.integers(M_range[0], M_range[1] + 1))
        P = int(rng.integers(P_range[0], P_range[1] + 1))
        sigma = float(rng.uniform(*sigma_range))
        beta = float(10.0 ** rng.uniform(*beta_log10_range))
        reqs.append(dict(n=n, M=M, P=P, sigma=sigma, beta=beta,
                         seed=1000 + i, arrival=float(arrivals[i])))
    return reqs


def field_modes(n: int, M: int, seed: int, amp: float = 0.6, mean: float = 1.3) -> np.ndarray:
    """Seeded per-element coefficient modes [M+1][n][n] (index [k][ey][ex],
    values at the element centroids) of an affine random field whose modes are
    not symmetric under x <-> y: mode 0 is the constant `mean`, mode k is
    w_k cos(a_k pi x + p_k) cos(b_k pi y + q_k) with integer wavenumbers
    a_k != b_k, random phases and weights w_k ~ k^-2, scaled so that
    sqrt(3) sum_k max|mode k| = amp * mean (amp < 1 keeps the field
    a = mean + sqrt(3) sum_k mode_k xi_k-type expansion positive for all xi)."""
    rng = np.random.default_rng(seed)
    t = (np.arange(n, dtype=np.float64) + 0.5) / n
    yc, xc = np.meshgrid(t, t, indexing="ij")
    out = np.empty((M + 1, n, n), dtype=np.float64)
    out[0] = mean
    peak = 0.0
    for k in range(1, M + 1):
        a = int(rng.integers(0, 4))
        b = int(rng.integers(0, 4))
        if b == a:
            b = a + 1
        px, py = rng.uniform(0.0, math.pi, size=2)
        out[k] = k ** -2.0 * np.cos(a * math.pi * xc + px) * np.cos(b * math.pi * yc + py)
        peak += np.max(np.abs(out[k]))
    out[1:] *= amp * mean / (math.sqrt(3.0) * peak)
    return out


def unit_sine(n: int) -> np.ndarray:
    """sin(pi x) sin(pi y) at the (n+1)^2 nodes (zero on the boundary)."""
    x, y = node_coords(n)
    return np.sin(math.pi * x) * np.sin(math.pi * y)


__all__.append("unit_sine")
