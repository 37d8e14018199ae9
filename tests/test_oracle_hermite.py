"""Pins of the log-normal / Hermite workload (oracle/hermite.py) against
quadrature, recurrences and the exponential it expands."""
from math import comb, factorial, sqrt

import numpy as np
import pytest
from numpy.polynomial import hermite_e as He
from scipy import integrate

import sg_inputs
from oracle import basis, hermite, kkt


def _he_norm(k, x):
    c = np.zeros(k + 1)
    c[k] = 1.0
    return He.hermeval(x, c) / sqrt(factorial(k))


def test_triple_products_by_gauss_hermite_quadrature():
    x, w = He.hermegauss(40)
    w = w / np.sqrt(2 * np.pi)
    for a in range(7):
        for b in range(5):
            for c in range(5):
                ref = float(np.sum(w * _he_norm(a, x) * _he_norm(b, x) * _he_norm(c, x)))
                assert abs(hermite.triple_1d(a, b, c) - ref) < 1e-11 * max(1.0, abs(ref)), (a, b, c)


def test_h_matrices_structure():
    M, P = 3, 2
    H = hermite.h_matrices(M, P)
    alpha = basis.multi_indices(M, P)
    nxi = alpha.shape[0]
    assert len(H) == comb(M + 2 * P, 2 * P) == hermite.coefficient_indices(M, P).shape[0]
    assert np.array_equal(H[0], np.eye(nxi))
    for Hl in H:
        assert np.array_equal(Hl, Hl.T)
    # linear terms: xi_k psi_n = sqrt(n+1) psi_{n+1} + sqrt(n) psi_{n-1} (three-term recurrence)
    index = {tuple(a): j for j, a in enumerate(alpha)}
    for k in range(M):
        Hk = H[1 + k]
        ref = np.zeros((nxi, nxi))
        for j, a in enumerate(alpha):
            up = list(a)
            up[k] += 1
            if tuple(up) in index:
                ref[j, index[tuple(up)]] = ref[index[tuple(up)], j] = sqrt(a[k] + 1)
        assert np.max(np.abs(Hk - ref)) < 1e-14
    # higher terms couple inside a degree level (e.g. 2 e_1 couples e_1 with e_1)
    lam = hermite.coefficient_indices(M, P)
    l2 = [i for i, l in enumerate(lam) if tuple(l) == (2, 0, 0)][0]
    assert abs(H[l2][1, 1] - hermite.triple_1d(2, 1, 1)) < 1e-15 and H[l2][1, 1] != 0.0


@pytest.mark.parametrize("corr", [1.0, 0.5])
def test_kl_1d_integral_equation_and_orthonormality(corr):
    pairs = hermite.kl_1d(5, corr)
    for p in pairs:
        theta = p[0]
        for s in (-0.7, 0.1, 0.9):
            lhs = integrate.quad(lambda t: np.exp(-abs(s - t) / corr) * hermite.kl_eval_1d(p, t), -1, 1, points=[s],
                                 epsabs=1e-13, epsrel=1e-12, limit=200)[0]
            assert abs(lhs - theta * hermite.kl_eval_1d(p, s)) < 1e-9
    for i, p in enumerate(pairs):
        for j, q in enumerate(pairs):
            v = integrate.quad(lambda t: hermite.kl_eval_1d(p, t) * hermite.kl_eval_1d(q, t), -1, 1,
                               epsabs=1e-13, limit=200)[0]
            assert abs(v - (1.0 if i == j else 0.0)) < 1e-10
    # the largest eigenvalues of a Nystrom discretisation of the kernel agree
    N = 2000
    t = -1 + (np.arange(N) + 0.5) * 2 / N
    K = np.exp(-np.abs(t[:, None] - t[None, :]) / corr) * (2 / N)
    ev = np.sort(np.linalg.eigvalsh(K))[::-1][:5]
    assert np.max(np.abs(ev - np.array([p[0] for p in pairs])) / ev) < 1e-3


def test_lognormal_expansion_converges_to_the_exponential():
    """sum_{|alpha| <= 2P} kappa_alpha psi_alpha(xi) approaches
    exp(sum_m f_m xi_m - sum_m f_m^2 / 2) (mean 1) as P grows."""
    M, sigma = 2, 0.3
    n = 4
    rng = np.random.default_rng(0)
    xis = rng.standard_normal((5, M))
    # element (1, 2) of the 4 x 4 grid: centre (2.5/4, 1.5/4) mapped to [-1, 1]^2
    x1, x2 = 2 * 2.5 / 4 - 1, 2 * 1.5 / 4 - 1
    f = hermite.kl_functions(M, sigma, 1.0, np.array([x1]), np.array([x2]))[:, 0]
    exact = np.exp(xis @ f - 0.5 * np.sum(f * f))
    errs = []
    for P in (1, 2, 3):
        kap = hermite.lognormal_modes(n, M, P, sigma)[:, 1, 2]
        lam = hermite.coefficient_indices(M, P)
        val = np.zeros(len(xis))
        for l, a in enumerate(lam):
            psi = np.ones(len(xis))
            for m in range(M):
                psi = psi * _he_norm(int(a[m]), xis[:, m])
            val += kap[l] * psi
        errs.append(np.max(np.abs(val - exact)))
    assert errs[1] < errs[0] and errs[2] < errs[1] and errs[2] < 1e-6, errs
    assert hermite.lognormal_modes(n, M, 2, sigma)[0].min() == 1.0        # mean coefficient kappa_1 = 1


def test_lognormal_kkt_solves():
    """The log-normal KKT system is nonsingular on a tiny grid, its SG
    stiffness is positive definite, and the direct solve has zero residual."""
    prob = kkt.Problem(n=8, M=2, P=2, sigma=0.2, beta=1e-2, gamma=1.0, y_target=sg_inputs.indicator_target(8),
                       field="lognormal")
    sg = kkt.setup(prob)
    assert len(sg.G) == comb(2 + 4, 4)
    A = kkt.A_kron(sg).toarray()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0
    x = kkt.solve_direct(sg)
    b = kkt.rhs(sg)
    assert np.linalg.norm(kkt.kkt_matrix(sg) @ x - b) <= 1e-12 * np.linalg.norm(b)
