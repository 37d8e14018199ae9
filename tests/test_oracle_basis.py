"""Pins of the oracle's stochastic basis (Section 2.1 of the paper) against
values the paper prints and facts of Legendre polynomials that do not depend
on the oracle's own formulas."""
import os
from math import comb

import numpy as np
import pytest
from scipy import integrate
from scipy.special import eval_legendre

from oracle import basis

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_basis_sizes.txt")


def _golden_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    return rows


@pytest.mark.parametrize("row", _golden_rows())
def test_basis_size_matches_paper(row):
    m, p, n_xi, n_a = row
    assert basis.multi_indices(m, p).shape == (n_xi, m)
    # the log-normal expansion size is the same counting at degree 2p
    assert basis.multi_indices(m, 2 * p).shape[0] == n_a


@pytest.mark.parametrize("M,P,n_xi", [(4, 3, 35), (6, 4, 210), (8, 3, 165), (4, 2, 15), (8, 4, 495)])
def test_workload_basis_sizes(M, P, n_xi):
    A = basis.multi_indices(M, P)
    assert A.shape[0] == n_xi
    # every multi-index distinct, total degree <= P
    assert len({tuple(a) for a in A}) == n_xi
    assert A.sum(axis=1).max() == P and A.min() >= 0


@pytest.mark.parametrize("M,P", [(3, 3), (4, 3), (6, 4)])
def test_level_ranges_follow_algorithm1(M, P):
    """Algorithm 1: degree d occupies (C(m+d-1, d-1), C(m+d, d)]."""
    A = basis.multi_indices(M, P)
    off = basis.level_offsets(M, P)
    deg = A.sum(axis=1)
    for d in range(P + 1):
        lo = comb(M + d - 1, d - 1) if d > 0 else 0
        hi = comb(M + d, d)
        assert off[d] == lo and off[d + 1] == hi
        assert np.all(deg[lo:hi] == d)
        assert hi - lo == comb(M + d - 1, d)


def test_within_degree_order_is_descending_lex():
    A = basis.multi_indices(2, 2)
    assert [tuple(a) for a in A] == [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]
    A = basis.multi_indices(3, 1)
    assert [tuple(a) for a in A] == [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]


@pytest.mark.parametrize("deg_a,deg_b", [(0, 0), (1, 1), (3, 3), (2, 4), (1, 2), (3, 4)])
def test_one_dim_moments_by_adaptive_quadrature(deg_a, deg_b):
    """Orthonormality and the xi-moment of the Legendre family, checked with
    scipy's adaptive quadrature of scipy's Legendre polynomials."""
    E1, E3 = basis._one_dim_moments(4)

    def f(x, w):
        return 0.5 * w(x) * np.sqrt(2 * deg_a + 1) * eval_legendre(deg_a, x) * \
            np.sqrt(2 * deg_b + 1) * eval_legendre(deg_b, x)

    m1 = integrate.quad(lambda x: f(x, lambda t: 1.0), -1, 1, epsabs=1e-14)[0]
    m3 = integrate.quad(lambda x: f(x, lambda t: np.sqrt(3.0) * t), -1, 1, epsabs=1e-14)[0]
    assert abs(E1[deg_a, deg_b] - m1) < 1e-13
    assert abs(E3[deg_a, deg_b] - m3) < 1e-13


@pytest.mark.parametrize("M,P", [(2, 3), (4, 3), (3, 4)])
def test_triple_products_structure(M, P):
    """H_1 = I (Section 2.1), H_l symmetric, and the affine field couples
    psi_alpha only to psi_{alpha +- e_k}: 2 C(M+P-1, P-1) nonzeros per G_k."""
    A = basis.multi_indices(M, P)
    G = basis.triple_product_matrices(M, P)
    n = A.shape[0]
    assert np.allclose(G[0], np.eye(n), atol=1e-14, rtol=0)
    for k in range(1, M + 1):
        Gk = G[k]
        assert np.max(np.abs(Gk - Gk.T)) < 1e-15
        nz = set(zip(*np.nonzero(Gk)))
        expect = set()
        for i in range(n):
            for j in range(n):
                d = A[j] - A[i]
                if np.abs(d).sum() == 1 and abs(d[k - 1]) == 1:
                    expect.add((i, j))
        assert nz == expect
        assert len(nz) == 2 * comb(M + P - 1, P - 1)


@pytest.mark.parametrize("M,P", [(1, 4), (2, 3), (3, 3), (4, 2)])
def test_g_spectrum_is_union_of_gauss_nodes(M, P):
    """Golub-Welsch: multiplication by xi_k = psi_{e_k}/sqrt(3) restricted to a
    chain alpha_k = 0..L is the Jacobi matrix of Legendre, whose eigenvalues are
    the (L+1)-point Gauss-Legendre nodes.  The total-degree set splits into
    chains with L = P - |alpha without k|."""
    A = basis.multi_indices(M, P)
    G = basis.triple_product_matrices(M, P)
    for k in range(1, M + 1):
        ev = np.sort(np.linalg.eigvalsh(G[k] / np.sqrt(3.0)))
        expect = []
        rest = {tuple(np.delete(a, k - 1)) for a in A}
        for r in rest:
            L = P - sum(r)
            expect.extend(basis.gl_nodes(L + 1))
        expect = np.sort(np.array(expect))
        assert ev.shape == expect.shape
        assert np.max(np.abs(ev - expect)) < 1e-13


def test_g_entries_against_monte_carlo():
    """E[psi_{e_k} psi_a psi_b] by plain Monte Carlo on U(-1,1)^M (loose)."""
    M, P = 2, 2
    A = basis.multi_indices(M, P)
    G = basis.triple_product_matrices(M, P)
    rng = np.random.default_rng(11)
    xi = rng.uniform(-1, 1, size=(400_000, M))
    psi = np.stack([basis.psi_eval(a, xi) for a in A])
    for k in range(1, M + 1):
        pk = np.sqrt(3.0) * xi[:, k - 1]
        mc = (psi * pk) @ psi.T / xi.shape[0]
        assert np.max(np.abs(mc - G[k])) < 0.03
