"""Numerical verification of the spectral bounds of Section 4 (Theorem
thm:approx, Lemma lem:lower_bound and the theta theorem, Theorem
thm:truncation, Lemma lem:lmin-sigY and the hGS bound) on tiny problems,
with dense operators built from their definitions (oracle/spectral.py)."""
import numpy as np
import pytest

import sg_inputs
from oracle import kkt, spectral


def _ops(n=4, M=2, P=2, nt=3, beta=1e-2, gamma=0.0, sigma=0.3, T=1.0):
    if nt <= 1:
        tgt = sg_inputs.gaussian_bumps(n, 0)
    else:
        tgt = sg_inputs.moving_bump(n, nt, T, 0)
    prob = kkt.Problem(n=n, M=M, P=P, sigma=sigma, beta=beta, gamma=gamma, n_t=nt, T=T, y_target=tgt)
    return spectral.TimeOperators(kkt.setup(prob))


CASES = [dict(beta=1e-2), dict(beta=1e-4), dict(beta=1e-4, gamma=0.5), dict(beta=1e-6),
         dict(nt=1, beta=1e-2), dict(nt=1, beta=1e-5, gamma=1.0), dict(n=8, M=3, P=2, nt=2, beta=1e-3)]
TOL = 1e-10


@pytest.mark.parametrize("case", CASES)
def test_schur_approximation_interval(case):
    """Theorem thm:approx: lambda(S-bar^{-1} S-exact) in [1/(2(1+alpha)), 1] with
    alpha = ((sqrt(k)+1)/(sqrt(k)-1))^2 - 1, k = cond(A_t); steady: [1/2, 1].
    Both are proven for gamma = 0.  For gamma > 0 the factor uses the scalar
    s^2 = (1+gamma)/beta while M_gamma = H^gamma (x) M carries 1 on the mean
    mode, so s^2 N W N^T exceeds the exact (1/beta) term by up to 1 + gamma
    there and the lower end can drop by that factor; steady: 1/(2(1+gamma))
    (the case gamma = 1, beta = 1e-5 reaches 0.33 < 1/2)."""
    T = _ops(**case)
    lo, hi = spectral.eig_ratio(T.S_exact(), T.S_of(T.Zbar()))
    k = T.kappa_At()
    alpha = ((np.sqrt(k) + 1) / (np.sqrt(k) - 1)) ** 2 - 1
    g = case.get("gamma", 0.0)
    assert hi <= 1 + TOL
    assert lo >= 1 / (2 * (1 + alpha) * (1 + g)) - TOL
    if case.get("nt", 3) == 1:
        assert lo >= 1 / (2 * (1 + g)) - TOL
        if g > 0:
            assert lo < 0.5          # the gamma = 0 interval does not carry over


@pytest.mark.parametrize("case", [c for c in CASES if c.get("nt", 3) > 1])
def test_theta_interval_and_bound(case):
    """Theorem after lem:lower_bound: (1-theta)^2 <= lambda(S-bar^{-1} S-tilde)
    <= (1+theta)^2, and theta <= sqrt(2 beta)/(sqrt(1+gamma)(1-1/mu) tau) kappa(M^1/2)
    when mu > 1."""
    T = _ops(**case)
    th = T.theta()
    lo, hi = spectral.eig_ratio(T.S_of(T.Zr(len(T.H))), T.S_of(T.Zbar()))
    assert (1 - th) ** 2 - TOL <= lo and hi <= (1 + th) ** 2 + TOL
    mu = T.mu()
    if mu > 1:
        assert th <= T.theta_bound(mu) + TOL


def test_lower_bound_lemma():
    """Lemma lem:lower_bound on a case where its condition mu > 1 holds
    (tau >> sqrt(beta)): lambda_min(S-tilde) >= (tau/beta)(1-1/mu)^2 lambda_min(M),
    and the identity sigma_min^2(N W^1/2) = lambda_min(M)/(1+gamma) of its proof."""
    import scipy.linalg as sla
    for gamma in (0.0, 0.5):
        T = _ops(beta=1e-6, gamma=gamma)
        mu = T.mu()
        assert mu > 1
        lmin_M = np.linalg.eigvalsh(T.M).min()
        St = T.S_of(T.Zr(len(T.H)))
        lam = np.linalg.eigvalsh(0.5 * (St + St.T)).min()
        assert lam >= (T.tau / T.sg.prob.beta) * (1 - 1 / mu) ** 2 * lmin_M * (1 - TOL)
        smin = np.linalg.svd(T.N @ sla.sqrtm(T.W).real, compute_uv=False)[-1]
        assert abs(smin ** 2 - lmin_M / (1 + gamma)) < 1e-10 * lmin_M


@pytest.mark.parametrize("case", CASES)
def test_truncation_bounds(case):
    """Theorem thm:truncation: with delta_r = sum_{l>r} ||H_l|| ||A-hat_l|| / lambda_min(A-hat_1),
    1 - delta_r <= lambda(Z_r^{-1} Z) <= 1 + delta_r for the factors Z = Z-tilde, and the
    Schur pair S_r = Z_r W Z_r, S = Z W Z in [(1-delta_r)^2, (1+delta_r)^2]."""
    T = _ops(**case)
    nA = len(T.H)
    Z = T.Zr(nA)
    S = T.S_of(Z)
    for r in range(1, nA + 1):
        d = T.delta_r(r)
        if d >= 1:
            continue
        lo, hi = spectral.eig_ratio(Z, T.Zr(r))
        assert 1 - d - TOL <= lo and hi <= 1 + d + TOL
        lo, hi = spectral.eig_ratio(S, T.S_of(T.Zr(r)))
        assert (1 - d) ** 2 - TOL <= lo and hi <= (1 + d) ** 2 + TOL


@pytest.mark.parametrize("case", CASES)
def test_hgs_lemma_and_factor_bound(case):
    """Lemma lem:lmin-sigY (lambda_min(I+Y+Y^T) >= 1 - Delta_r, sigma_max(Y) <=
    sum ||L_l|| rho_l <= Delta_r, rho_l <= ||kappa_l||_inf / kappa_0, ||L_l|| <= ||H_l||)
    and the factor bound 1 <= lambda(Z_r^{-1} Z_hGS) <= 1 + Delta_r^2/(1-Delta_r)."""
    T = _ops(**case)
    sg = T.sg
    nA = len(T.H)
    for r in range(2, nA + 1):
        D, rho = T.Delta_r(r)
        Y = T.Y(r)
        lmin = np.linalg.eigvalsh(np.eye(Y.shape[0]) + Y + Y.T).min()
        assert lmin >= 1 - D - TOL
        Ls = [np.linalg.norm(T.level_lower(T.H[l]), 2) for l in range(1, r)]
        assert all(Ll <= np.linalg.norm(T.H[l], 2) + TOL for Ll, l in zip(Ls, range(1, r)))
        smax = np.linalg.norm(Y, 2)
        assert smax <= sum(Ll * rho[l - 1] for Ll, l in zip(Ls, range(1, r))) + TOL <= D + 2 * TOL
        k0 = sg.kappa[0].min()
        for l in range(1, nA):
            assert rho[l - 1] <= np.abs(sg.kappa[l]).max() / k0 + TOL
        if D < 1:
            lo, hi = spectral.eig_ratio(T.Z_hgs(r), T.Zr(r))
            assert lo >= 1 - TOL and hi <= 1 + D * D / (1 - D) + TOL


def test_hgs_schur_pair_reading():
    """The printed bound for the Schur pair, 1 <= lambda(S_r^{-1} S_hGS) <=
    (1 + Delta_r^2/(1-Delta_r))^2, squares the factor bound; the upper end holds
    here but the lower end does not (the factors Z_hGS and Z_r do not commute
    with W), so only the factor bound above is asserted as a theorem and the
    Schur pair's measured range is recorded."""
    T = _ops(beta=1e-2)
    r = len(T.H)
    D, _ = T.Delta_r(r)
    lo, hi = spectral.eig_ratio(T.S_of(T.Z_hgs(r)), T.S_of(T.Zr(r)))
    assert hi <= (1 + D * D / (1 - D)) ** 2 + TOL
    assert 0.99 < lo < 1.0
