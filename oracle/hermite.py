"""Log-normal coefficient with Hermite chaos (the paper's own workload).

Oracle (test infrastructure only).

Paper passages followed
  * Section 2.1: orthonormal Hermite chaos psi_alpha = prod_m He_{alpha_m}(xi_m)
    / sqrt(alpha_m!) in independent standard Gaussians; the solution space has
    total degree p (n_xi = C(m + p, p)) and the coefficient total degree 2p
    (n_A = C(m + 2p, 2p)); A = sum_l H_l (x) A_l with (H_l)_{jk} = E[psi_l
    psi_j psi_k].
  * Section 2.1, eq. (Czxy): f = f_0 + sum_i sqrt(theta_i) phi_i xi_i is the
    truncated Karhunen-Loeve expansion of a Gaussian field, (theta_i, phi_i)
    the eigenpairs of its covariance; the coefficient is exp(f) and its chaos
    coefficients follow Ghanem's formula.
  * Section 5: covariance sigma^2 exp(-|x1 - y1| / l1 - |x2 - y2| / l2) on
    [-1, 1]^2 with l1 = l2 = 1, mean coefficient kappa_1 = 1.

Readings:
  * The chaos coefficients come from the Hermite generating function:
    exp(sum_m f_m xi_m - f_m^2 / 2) = sum_alpha prod_m f_m^alpha_m / alpha_m!
    He_alpha_m(xi_m), so with kappa_1 = 1 (f_0 = -sum f_m^2 / 2)
    kappa_alpha(x) = prod_m f_m(x)^alpha_m / sqrt(alpha_m!).  The printed
    formula evaluates psi_i at xi - f, which gives (-f)^alpha: the field with
    xi -> -xi, equal in law; this oracle uses +f.
  * The square [-1, 1]^2 of Section 5 is mapped onto the unit square of the
    discretisation by x = 2 x' - 1; the coefficient at an element is its value
    at the element centre.
"""
from __future__ import annotations

from math import comb, factorial, sqrt

import numpy as np
from scipy.optimize import brentq

from . import basis


# ----------------------------------------------------------------------------
# Hermite triple products
# ----------------------------------------------------------------------------

def triple_1d(a: int, b: int, c: int) -> float:
    """E[psi_a psi_b psi_c] for orthonormal probabilists' Hermite polynomials
    psi_k = He_k / sqrt(k!): the classical closed form a! b! c! / ((s-a)!
    (s-b)! (s-c)!) for E[He_a He_b He_c] when s = (a+b+c)/2 is an integer not
    below max(a, b, c), zero otherwise, divided by sqrt(a! b! c!)."""
    if (a + b + c) % 2:
        return 0.0
    s = (a + b + c) // 2
    if s < max(a, b, c):
        return 0.0
    num = sqrt(factorial(a) * factorial(b) * factorial(c))
    return num / (factorial(s - a) * factorial(s - b) * factorial(s - c))


def coefficient_indices(M: int, P: int) -> np.ndarray:
    """Multi-indices of the coefficient expansion: total degree <= 2P, graded
    by degree (l = 0 is the mean, then the M linear terms, ...)."""
    return basis.multi_indices(M, 2 * P)


def h_matrices(M: int, P: int) -> list:
    """H_l, l = 0..n_A-1: (H_l)_{jk} = E[psi_l psi_j psi_k] over the degree-P
    solution basis (dense n_xi x n_xi arrays)."""
    alpha = basis.multi_indices(M, P)
    lam = coefficient_indices(M, P)
    nxi = alpha.shape[0]
    out = []
    for l in lam:
        H = np.zeros((nxi, nxi))
        for j in range(nxi):
            for k in range(j, nxi):
                v = 1.0
                for m in range(M):
                    v *= triple_1d(int(l[m]), int(alpha[j, m]), int(alpha[k, m]))
                    if v == 0.0:
                        break
                H[j, k] = H[k, j] = v
        out.append(H)
    assert len(out) == comb(M + 2 * P, 2 * P)
    return out


# ----------------------------------------------------------------------------
# Karhunen-Loeve eigenpairs of the separable exponential covariance
# ----------------------------------------------------------------------------

def kl_1d(count: int, corr: float = 1.0, a: float = 1.0):
    """The `count` largest eigenpairs of exp(-|s - t| / corr) on [-a, a]:
    theta = 2 c / (w^2 + c^2), c = 1 / corr, with w the roots of
    c - w tan(w a) = 0 (even eigenfunctions cos(w x) / sqrt(a + sin(2 w a) / (2 w)))
    and w + c tan(w a) = 0 (odd eigenfunctions sin(w x) / sqrt(a - sin(2 w a) / (2 w))).
    Returns a list of (theta, kind, w, norm) sorted by decreasing theta."""
    c = 1.0 / corr
    pairs = []
    eps = 1e-12
    k = 0
    while len(pairs) < 2 * count + 2:
        # even root in (k pi / a, (k + 1/2) pi / a)
        lo, hi = k * np.pi / a + eps, (k + 0.5) * np.pi / a - eps
        w = brentq(lambda w: c * np.cos(w * a) - w * np.sin(w * a), lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
        pairs.append((2 * c / (w * w + c * c), 0, w, 1.0 / np.sqrt(a + np.sin(2 * w * a) / (2 * w))))
        # odd root in ((k + 1/2) pi / a, (k + 1) pi / a)
        lo, hi = (k + 0.5) * np.pi / a + eps, (k + 1) * np.pi / a - eps
        w = brentq(lambda w: w * np.cos(w * a) + c * np.sin(w * a), lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
        pairs.append((2 * c / (w * w + c * c), 1, w, 1.0 / np.sqrt(a - np.sin(2 * w * a) / (2 * w))))
        k += 1
    pairs.sort(key=lambda p: -p[0])
    return pairs[:count]


def kl_eval_1d(pair, x: np.ndarray) -> np.ndarray:
    _, kind, w, nrm = pair
    return nrm * (np.cos(w * x) if kind == 0 else np.sin(w * x))


def kl_2d(M: int, sigma: float, corr: float = 1.0):
    """The M largest eigenpairs of sigma^2 exp(-|x1-y1|/corr - |x2-y2|/corr) on
    [-1, 1]^2: products of the 1-D pairs.  The unordered index pairs {i <= j}
    are sorted by decreasing eigenvalue and each expands to (i, j) then (j, i),
    so the two equal eigenvalues of a pair keep a fixed order whatever the
    rounding of the 1-D roots.  Returns [(theta, pair_x, pair_y)]."""
    one = kl_1d(M + 2, corr)
    und = [(sigma * sigma * one[i][0] * one[j][0], i, j) for i in range(len(one)) for j in range(i, len(one))]
    und.sort(key=lambda c: -c[0])
    out = []
    for theta, i, j in und:
        out.append((theta, one[i], one[j]))
        if i != j:
            out.append((theta, one[j], one[i]))
    return out[:M]


def kl_functions(M: int, sigma: float, corr: float, x1: np.ndarray, x2: np.ndarray) -> np.ndarray:
    """f_m(x) = sqrt(theta_m) phi_m(x) at points (x1, x2) of [-1, 1]^2; shape (M, npts)."""
    out = []
    for theta, px, py in kl_2d(M, sigma, corr):
        out.append(np.sqrt(theta) * kl_eval_1d(px, x1) * kl_eval_1d(py, x2))
    return np.array(out)


def lognormal_modes(n: int, M: int, P: int, sigma: float, corr: float = 1.0) -> np.ndarray:
    """Per-element chaos coefficients kappa_l, l = 0..n_A-1, of the log-normal
    field with mean 1 (shape (n_A, n, n), [ey][ex]): element centres of the
    n x n grid on the unit square mapped to [-1, 1]^2."""
    c = (np.arange(n) + 0.5) / n
    X1, X2 = np.meshgrid(2 * c - 1, 2 * c - 1)          # [ey][ex]
    f = kl_functions(M, sigma, corr, X1.ravel(), X2.ravel())
    lam = coefficient_indices(M, P)
    out = np.empty((lam.shape[0], n * n))
    for l, a in enumerate(lam):
        v = np.ones(n * n)
        for m in range(M):
            if a[m]:
                v = v * f[m] ** int(a[m]) / sqrt(factorial(int(a[m])))
        out[l] = v
    return out.reshape(-1, n, n)
