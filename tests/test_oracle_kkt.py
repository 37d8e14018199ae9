"""Pins of the oracle's KKT systems and direct solve against closed forms,
textbook equivalences and the paper's time-stepping equations."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import sg_inputs
from oracle import basis, fem, kkt


def _steady(n=8, M=2, P=2, sigma=0.2, beta=1e-2, gamma=0.0, target=None, seed=0):
    if target is None:
        target = sg_inputs.gaussian_bumps(n, seed)
    return kkt.setup(kkt.Problem(n=n, M=M, P=P, sigma=sigma, beta=beta, gamma=gamma, y_target=target))


def test_kkt_symmetric_and_direct_residual():
    sg = _steady(n=8, M=3, P=2, gamma=0.5)
    K = kkt.kkt_matrix(sg)
    assert abs(K - K.T).max() == 0.0
    x = kkt.solve_direct(sg)
    b = kkt.rhs(sg)
    assert np.linalg.norm(b - K @ x) / np.linalg.norm(b) < 1e-12
    assert kkt._backward_error(K, x, b) < 1e-15


def test_matricized_apply_equals_kronecker():
    """eq. (mat-vec): (G (x) K) vec(X) = vec(K X G^T)."""
    sg = _steady(n=8, M=3, P=3)
    X = sg_inputs.random_block((sg.n_xi, sg.n_int), 5)
    Y1 = kkt.operator_apply(sg, X)
    Y2 = (kkt.A_kron(sg) @ X.ravel()).reshape(X.shape)
    assert np.max(np.abs(Y1 - Y2)) < 1e-13 * np.max(np.abs(Y2))


@pytest.mark.parametrize("beta", [1e-2, 1e-4])
def test_deterministic_sine_closed_form(beta):
    """sigma = 0: the target s*sin(pi x)sin(pi y) gives the exact discrete
    solution y = s/(1 + beta mu^2) v, u = mu y, lambda = -beta u in chaos
    column 0, with K v = mu M v; all other chaos columns vanish."""
    n, s = 16, 1.7
    target = s * sg_inputs.unit_sine(n)
    sg = _steady(n=n, M=2, P=2, sigma=0.0, beta=beta, target=target)
    h = 1.0 / n
    k1 = (2 / h) * (1 - math.cos(math.pi * h))
    m1 = (h / 3) * (2 + math.cos(math.pi * h))
    mu = 2 * k1 / m1
    v = fem.extract(sg_inputs.unit_sine(n), n)
    Y, U, L = kkt.split(sg, kkt.solve_direct(sg))
    c = s / (1 + beta * mu * mu)
    assert np.max(np.abs(Y[0] - c * v)) < 1e-12
    assert np.max(np.abs(U[0] - mu * c * v)) < 1e-10 * mu
    assert np.max(np.abs(L[0] + beta * mu * c * v)) < 1e-12
    assert np.max(np.abs(Y[1:])) < 1e-13 and np.max(np.abs(U[1:])) < 1e-11


def _deterministic_kkt(n, coeff, beta, target):
    K = fem.restrict(fem.assemble_full(n, coeff, "stiffness"), n)
    Mf = fem.assemble_full(n, 1.0, "mass")
    Mi = fem.restrict(Mf, n)
    b = (Mf @ target)[fem.interior_index(n)]
    KKT = sp.bmat([[Mi, None, -K], [None, beta * Mi, Mi], [-K, Mi, None]], format="csc")
    m = Mi.shape[0]
    x = spla.spsolve(KKT, np.concatenate([b, np.zeros(2 * m)]))
    return x[:m], x[m:2 * m], x[2 * m:]


@pytest.mark.parametrize("P", [1, 2, 4])
def test_single_variable_sg_equals_gauss_collocation(P):
    """M = 1, gamma = 0: the SG system with the complete degree-P basis is
    diagonalised by the eigenvectors of the Jacobi matrix G_1/sqrt(3), so
    Y_i = sum_q w_q psi_i(xi_q) y_det(xi_q) over the (P+1)-point Gauss rule."""
    n, beta, sigma = 8, 1e-2, 0.5
    target = sg_inputs.gaussian_bumps(n, 7)
    sg = _steady(n=n, M=1, P=P, sigma=sigma, beta=beta, target=target)
    Y, U, L = kkt.split(sg, kkt.solve_direct(sg))
    x, w = np.polynomial.legendre.leggauss(P + 1)
    w = 0.5 * w
    kap = fem.cosine_modes(n, 1, sigma)
    Yc, Uc, Lc = np.zeros_like(Y), np.zeros_like(U), np.zeros_like(L)
    for xq, wq in zip(x, w):
        coeff = kap[0] + math.sqrt(3.0) * xq * kap[1]     # a(x, xi_q) = kappa_0 + kappa_1 psi_1(xi_q)
        yq, uq, lq = _deterministic_kkt(n, coeff, beta, target)
        for i in range(P + 1):
            psi = basis.psi1d(i, np.array([xq]))[0]
            Yc[i] += wq * psi * yq
            Uc[i] += wq * psi * uq
            Lc[i] += wq * psi * lq
    scale = np.max(np.abs(Y))
    assert np.max(np.abs(Y - Yc)) < 1e-12 * scale
    assert np.max(np.abs(U - Uc)) < 1e-10 * np.max(np.abs(U))
    assert np.max(np.abs(L - Lc)) < 1e-12 * np.max(np.abs(L))


def test_mean_converges_to_tensor_collocation_mean():
    """M = 2, gamma = 0: the SG mean approaches the tensor Gauss mean of the
    parametric solutions as P grows (the problem decouples per xi)."""
    n, beta, sigma = 8, 1e-2, 0.6
    target = sg_inputs.gaussian_bumps(n, 2)
    kap = fem.cosine_modes(n, 2, sigma)
    x, w = np.polynomial.legendre.leggauss(8)
    w = 0.5 * w
    mean_ref = 0.0
    for x1, w1 in zip(x, w):
        for x2, w2 in zip(x, w):
            coeff = kap[0] + math.sqrt(3.0) * (x1 * kap[1] + x2 * kap[2])
            mean_ref = mean_ref + w1 * w2 * _deterministic_kkt(n, coeff, beta, target)[0]
    errs = []
    for P in (1, 2, 3):
        sg = _steady(n=n, M=2, P=P, sigma=sigma, beta=beta, target=target)
        Y = kkt.split(sg, kkt.solve_direct(sg))[0]
        errs.append(np.max(np.abs(Y[0] - mean_ref)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3 * np.max(np.abs(mean_ref))


def _time_problem(n=8, M=2, P=2, nt=5, beta=1e-3, gamma=0.0, y0=True):
    target = sg_inputs.moving_bump(n, nt, 1.0, 4)
    y0v = sg_inputs.gaussian_bumps(n, 9) * sg_inputs.unit_sine(n) if y0 else None
    return kkt.setup(kkt.Problem(n=n, M=M, P=P, sigma=0.3, beta=beta, gamma=gamma, n_t=nt, y_target=target, y0=y0v))


def test_time_kkt_reproduces_backward_euler_sweeps():
    """Section 3, eq. (back Euler): the solved (y, u) satisfy
    (M + tau A) y_k = M y_{k-1} + tau M u_k step by step; the gradient row
    gives u_k = -lambda_k / (beta D_kk); the adjoint row, swept backward,
    L lambda_k = M lambda_{k+1} + tau D_kk (M_gamma y_k - M y_d,k)."""
    sg = _time_problem(gamma=0.3)
    p = sg.prob
    tau = p.tau
    Y, U, L = kkt.split(sg, kkt.solve_direct(sg))
    Mc = kkt.Mcal(sg)
    Lc = kkt.L_cal(sg).tocsc()
    lu = spla.splu(Lc)
    y_prev = np.zeros(sg.n_xi * sg.n_int)
    y_prev[:sg.n_int] = fem.extract(p.y0, p.n)
    scale = np.max(np.abs(Y))
    for t in range(p.n_t):
        y = lu.solve(Mc @ y_prev + tau * (Mc @ U[t].ravel()))
        assert np.max(np.abs(y - Y[t].ravel())) < 1e-11 * scale
        y_prev = y
    D = np.ones(p.n_t)
    D[0] = D[-1] = 0.5
    for t in range(p.n_t):
        assert np.max(np.abs(U[t] + L[t] / (p.beta * D[t]))) < 1e-9 * np.max(np.abs(U))
    Mg = kkt.Mgamma(sg)
    yt = np.reshape(p.y_target, (p.n_t, -1))
    lam_next = np.zeros(sg.n_xi * sg.n_int)
    lu_t = spla.splu(Lc.T.tocsc())
    for t in range(p.n_t - 1, -1, -1):
        load = np.zeros(sg.n_xi * sg.n_int)
        load[:sg.n_int] = (sg.Mfull @ yt[t])[fem.interior_index(p.n)]
        lam = lu_t.solve(Mc @ lam_next + tau * D[t] * (Mg @ Y[t].ravel() - load))
        assert np.max(np.abs(lam - L[t].ravel())) < 1e-11 * np.max(np.abs(L))
        lam_next = lam


def test_time_kkt_sigma_zero_stays_in_mean_column():
    sg = kkt.setup(kkt.Problem(n=8, M=2, P=2, sigma=0.0, beta=1e-2, n_t=3,
                               y_target=sg_inputs.moving_bump(8, 3, 1.0, 1)))
    Y, U, L = kkt.split(sg, kkt.solve_direct(sg))
    assert np.max(np.abs(Y[:, 1:])) < 1e-14 * np.max(np.abs(Y))
    assert np.max(np.abs(Y[:, 0])) > 0


def test_moments():
    sg = _steady(n=8, M=2, P=2, sigma=0.3)
    Y = kkt.split(sg, kkt.solve_direct(sg))[0]
    mean, var = kkt.moments(Y)
    assert np.array_equal(mean, Y[0])
    assert np.all(var >= 0) and np.max(var) > 0


@pytest.mark.parametrize("nt", [1, 4])
def test_matricized_kkt_apply_equals_explicit(nt):
    if nt == 1:
        sg = _steady(n=8, M=3, P=2, gamma=0.4)
    else:
        sg = _time_problem(n=8, M=2, P=2, nt=nt, gamma=0.4)
    K = kkt.kkt_matrix(sg)
    x = sg_inputs.random_block(K.shape[0], 3)
    ref = K @ x
    assert np.max(np.abs(kkt.kkt_apply_matricized(sg, x) - ref)) < 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("nt", [1, 4])
def test_kkt_rows_equal_explicit_matrix_rows(nt):
    """kkt_rows (sampled rows, used for the large-grid residual check) equals
    the explicit KKT matrix times x on those rows, every block and time step."""
    if nt == 1:
        sg = _steady(n=8, M=3, P=2, gamma=0.4)
    else:
        sg = _time_problem(n=8, M=2, P=2, nt=nt, gamma=0.4)
    K = kkt.kkt_matrix(sg)
    x = sg_inputs.random_block(K.shape[0], 4)
    rows = np.random.default_rng(5).choice(K.shape[0], size=600, replace=False)
    ref = (K @ x)[rows]
    assert np.max(np.abs(kkt.kkt_rows(sg, x, rows) - ref)) < 1e-13 * np.max(np.abs(ref))
