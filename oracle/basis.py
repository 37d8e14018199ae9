"""Stochastic basis: total-degree multi-indices and Legendre triple products.

Oracle (test infrastructure only).

Paper passages followed
  * Section 2.1: orthonormal gPC basis {psi_k}, psi_1 = 1, E[psi_k] = 0 for
    k > 1; dimension n_xi = C(m_xi + p, p) of the total-degree space.
  * Section 2.1: triple products h_{ljk} = E[psi_l psi_j psi_k], matrices
    H_l symmetric, H_1 = I.
  * Algorithm 1: the basis is ordered by polynomial degree so that degree d
    occupies the index range (C(m+d-1, d-1), C(m+d, d)].

Reading (the paper is silent): within one degree the multi-indices are in
descending lexicographic order, so e_1 precedes e_2 and (2,0,..) precedes
(1,1,0,..).  The chaos family is orthonormal Legendre on U(-1,1)^M
(psi_alpha = prod_m sqrt(2 alpha_m + 1) P_{alpha_m}(xi_m)) instead of the
paper's Hermite family; the affine coefficient then couples psi_alpha only to
psi_{alpha +- e_k}.
"""
from __future__ import annotations

from math import comb

import numpy as np
from numpy.polynomial import legendre as npleg


def _compositions_desc(total: int, parts: int):
    """All tuples of `parts` non-negative ints summing to `total`, in
    descending lexicographic order."""
    if parts == 1:
        yield (total,)
        return
    for first in range(total, -1, -1):
        for rest in _compositions_desc(total - first, parts - 1):
            yield (first,) + rest


def multi_indices(M: int, P: int) -> np.ndarray:
    """Total-degree multi-index set {alpha in N^M : |alpha| <= P}.

    Graded by degree (Algorithm 1's level ranges), descending lexicographic
    inside a degree.  Returns an int32 array of shape (n_xi, M).
    """
    rows = []
    for d in range(P + 1):
        rows.extend(_compositions_desc(d, M))
    out = np.array(rows, dtype=np.int32).reshape(-1, M)
    assert out.shape[0] == comb(M + P, P)
    return out


def level_offsets(M: int, P: int) -> np.ndarray:
    """offsets[d] = number of multi-indices of degree < d, d = 0..P+1.

    Degree d occupies columns offsets[d] .. offsets[d+1]-1, i.e. the range
    (C(m+d-1, d-1), C(m+d, d)] of Algorithm 1 in 0-based form."""
    return np.array([comb(M + d - 1, d - 1) if d > 0 else 0 for d in range(P + 2)],
                    dtype=np.int64)


def psi1d(deg: int, x: np.ndarray) -> np.ndarray:
    """Orthonormal Legendre polynomial sqrt(2 deg + 1) P_deg(x) for U(-1,1)."""
    c = np.zeros(deg + 1)
    c[deg] = 1.0
    return np.sqrt(2.0 * deg + 1.0) * npleg.legval(x, c)


def psi_eval(alpha: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """psi_alpha(xi) for points xi of shape (npts, M)."""
    xi = np.atleast_2d(xi)
    val = np.ones(xi.shape[0])
    for m, a in enumerate(alpha):
        val = val * psi1d(int(a), xi[:, m])
    return val


def _one_dim_moments(P: int):
    """1-D expectation tables under U(-1,1), by (P+2)-point Gauss-Legendre
    quadrature (exact for polynomial degree <= 2P+3):
      E1[a, b] = E[psi_a psi_b],  E3[a, b] = E[sqrt(3) xi psi_a psi_b]."""
    x, w = npleg.leggauss(P + 2)
    w = 0.5 * w                       # density of U(-1,1)
    V = np.stack([psi1d(a, x) for a in range(P + 1)])   # (P+1, q)
    E1 = (V * w) @ V.T
    E3 = (V * (w * np.sqrt(3.0) * x)) @ V.T
    return E1, E3


def triple_product_matrices(M: int, P: int, drop: float = 1e-13):
    """G_k = E[psi_{e_k} psi_alpha psi_beta] for k = 0..M (G_0 = E[psi_0 ...]).

    Section 2.1 (H_l with l = e_k).  The M-dimensional expectation factorises
    over the independent xi_m, so each entry is a product of 1-D
    Gauss-Legendre moments (tensor quadrature).  Entries below `drop` in
    magnitude are structural zeros (they come out at rounding level).
    Returns a list of M+1 dense float64 arrays (n_xi, n_xi).
    """
    A = multi_indices(M, P)
    E1, E3 = _one_dim_moments(P)
    n = A.shape[0]
    G = []
    # k = 0: psi_0 = 1, so the product of 1-D mass moments in every dimension.
    base = np.ones((n, n))
    for m in range(M):
        base = base * E1[np.ix_(A[:, m], A[:, m])]
    base[np.abs(base) < drop] = 0.0
    G.append(base)
    for k in range(M):
        g = np.ones((n, n))
        for m in range(M):
            tab = E3 if m == k else E1
            g = g * tab[np.ix_(A[:, m], A[:, m])]
        g[np.abs(g) < drop] = 0.0
        G.append(g)
    return G


def gl_nodes(npts: int) -> np.ndarray:
    """Gauss-Legendre nodes on [-1,1] (library routine; used by pins)."""
    return npleg.leggauss(npts)[0]
