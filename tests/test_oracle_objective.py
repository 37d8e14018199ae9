"""Pins of the oracle against the optimisation problem itself.

The KKT systems in oracle/kkt.py are the first-order conditions of the
discrete objective of Section 2.1 (steady: tracking term, variance weight
gamma, control cost beta) and of Section 3 (trapezoidal time weights D).  The
tests below evaluate that objective with no help from the oracle's KKT
matrices: the random fields are reconstructed from their chaos coefficients
and integrated over xi by tensor Gauss-Legendre quadrature (exact for the
polynomial degrees involved), the variance is E[(y - E y)^2] computed the same
way, and the mass matrix is the tensor product of 1-D linear-element mass
matrices.  The oracle's direct solution must then be a stationary point of the
objective along every direction that keeps the state equation satisfied, and
the oracle's variance field must equal the quadrature variance.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.special import eval_legendre

import sg_inputs
from oracle import kkt


def _mass_full_1d_tensor(n):
    """Full-grid Q1 mass matrix as M1 (x) M1, M1 = the 1-D linear-element mass
    matrix on n uniform cells of [0,1] (diagonal 2h/3 inside, h/3 at the two
    ends, off-diagonal h/6); node index iy*(n+1)+ix."""
    h = 1.0 / n
    d = np.full(n + 1, 2.0 * h / 3.0)
    d[0] = d[-1] = h / 3.0
    M1 = sp.diags([np.full(n, h / 6.0), d, np.full(n, h / 6.0)], [-1, 0, 1], format="csr")
    return sp.kron(M1, M1, format="csr")


def _interior(n):
    i = np.arange(1, n)
    iy, ix = np.meshgrid(i, i, indexing="ij")
    return (iy * (n + 1) + ix).reshape(-1)


def _quadrature(alpha, P):
    """Tensor Gauss-Legendre rule for U(-1,1)^M with P+1 points per variable
    (exact for degree <= 2P+1 in each variable) and the values of every
    orthonormal Legendre product psi_alpha at its nodes: returns (w, Psi) with
    Psi[q, j] = psi_{alpha_j}(xi_q) and sum_q w_q = 1."""
    M = alpha.shape[1]
    x, w = np.polynomial.legendre.leggauss(P + 1)
    w = 0.5 * w
    pts = np.array(list(itertools.product(range(P + 1), repeat=M)))
    W = np.prod(w[pts], axis=1)
    Psi = np.ones((pts.shape[0], alpha.shape[0]))
    for m in range(M):
        xm = x[pts[:, m]]
        for j in range(alpha.shape[0]):
            a = int(alpha[j, m])
            Psi[:, j] *= np.sqrt(2 * a + 1) * eval_legendre(a, xm)
    return W, Psi


def _field_terms(Y, n, W, Psi, Mf, target_full=None):
    """E[(y - y_d)^T M (y - y_d)] and the integrated variance
    int Var(y) dx = E[(y - E y)^T M (y - E y)] of the field with chaos
    coefficients Y (n_xi, n_int), by quadrature over xi (y = 0 on the boundary)."""
    I = _interior(n)
    nodes = (n + 1) ** 2
    samples = Psi @ Y                                  # (nq, n_int): y(xi_q) at the interior nodes
    full = np.zeros((samples.shape[0], nodes))
    full[:, I] = samples
    mean = W @ full
    dev = full - mean[None, :]
    var_int = float(np.sum(W * np.einsum("qi,qi->q", dev, (Mf @ dev.T).T)))
    if target_full is None:
        return var_int
    e = full - target_full[None, :]
    track = float(np.sum(W * np.einsum("qi,qi->q", e, (Mf @ e.T).T)))
    return track, var_int


def _objective_steady(sg, x, W, Psi, Mf):
    """Section 2.1, eq. (problem-stoch) in discrete form:
    J = 1/2 E||y - y_d||_M^2 + gamma/2 int Var(y) + beta/2 E||u||_M^2."""
    p = sg.prob
    Y, U, _ = kkt.split(sg, x)
    track, var = _field_terms(Y, p.n, W, Psi, Mf, np.reshape(p.y_target, -1))
    uu = _field_terms(U, p.n, W, Psi, Mf, np.zeros((p.n + 1) ** 2))[0]
    return 0.5 * track + 0.5 * p.gamma * var + 0.5 * p.beta * uu


def _objective_time(sg, x, W, Psi, Mf):
    """Section 3 (discrete time objective with trapezoid weights D =
    diag(1/2, 1, ..., 1, 1/2) over the n_t unknown states):
    J = tau sum_t D_t [1/2 E||y_t - y_d,t||_M^2 + gamma/2 int Var(y_t) + beta/2 E||u_t||_M^2]."""
    p = sg.prob
    Y, U, _ = kkt.split(sg, x)
    D = np.ones(p.n_t)
    D[0] = D[-1] = 0.5
    yt = np.reshape(p.y_target, (p.n_t, -1))
    J = 0.0
    for t in range(p.n_t):
        track, var = _field_terms(Y[t], p.n, W, Psi, Mf, yt[t])
        uu = _field_terms(U[t], p.n, W, Psi, Mf, np.zeros((p.n + 1) ** 2))[0]
        J += p.tau * D[t] * (0.5 * track + 0.5 * p.gamma * var + 0.5 * p.beta * uu)
    return J


def _feasible_direction_steady(sg, seed):
    """(dy, du) with A dy = M du: a direction along which the state equation
    -A y + M u = 0 stays satisfied (random du, dy from a sparse solve)."""
    du = sg_inputs.random_block((sg.n_xi, sg.n_int), seed)
    rhs = kkt.Mcal(sg) @ du.ravel()
    dy = spla.spsolve(kkt.A_kron(sg).tocsc(), rhs).reshape(du.shape)
    return np.concatenate([dy.ravel(), du.ravel(), np.zeros(du.size)])


def _feasible_direction_time(sg, seed):
    """Backward Euler from a zero initial perturbation:
    (M + tau A) dy_t = M dy_{t-1} + tau M du_t (Section 3, eq. back Euler)."""
    p = sg.prob
    du = sg_inputs.random_block((p.n_t, sg.n_xi, sg.n_int), seed)
    Mc = kkt.Mcal(sg)
    lu = spla.splu((Mc + p.tau * kkt.A_kron(sg)).tocsc())
    dy = np.zeros_like(du)
    prev = np.zeros(sg.n_xi * sg.n_int)
    for t in range(p.n_t):
        prev = lu.solve(Mc @ prev + p.tau * (Mc @ du[t].ravel()))
        dy[t] = prev.reshape(sg.n_xi, sg.n_int)
    return np.concatenate([dy.ravel(), du.ravel(), np.zeros(du.size)])


CASES = [
    # n, M, P, sigma, beta, gamma, n_t
    (8, 2, 2, 0.3, 1e-2, 0.0, 1),
    (8, 2, 2, 0.3, 1e-2, 0.8, 1),
    (8, 3, 2, 0.4, 1e-3, 2.0, 1),
    (8, 2, 2, 0.3, 1e-2, 0.6, 4),
]


@pytest.mark.parametrize("case", CASES)
def test_direct_solution_is_stationary_for_the_objective(case):
    """Along any constraint-feasible direction d the objective J is a
    quadratic in the step, so (J(x* + d) - J(x* - d)) / 2 is its exact first
    derivative at x*; it must vanish relative to the curvature term
    (J(x* + d) + J(x* - d))/2 - J(x*) > 0.  A slip in H^gamma (gamma applied to
    the mean column, or not applied), in the time weights or in the tracking
    load moves the first derivative to the size of the curvature term."""
    n, M, P, sigma, beta, gamma, nt = case
    if nt <= 1:
        target = sg_inputs.gaussian_bumps(n, 3)
    else:
        target = sg_inputs.moving_bump(n, nt, 1.0, 5)
    sg = kkt.setup(kkt.Problem(n=n, M=M, P=P, sigma=sigma, beta=beta, gamma=gamma, n_t=nt, y_target=target))
    x = kkt.solve_direct(sg)
    W, Psi = _quadrature(sg.alpha, P)
    Mf = _mass_full_1d_tensor(n)
    J = (lambda v: _objective_steady(sg, v, W, Psi, Mf)) if nt <= 1 else \
        (lambda v: _objective_time(sg, v, W, Psi, Mf))
    for seed in (11, 12, 13):
        d = _feasible_direction_steady(sg, seed) if nt <= 1 else _feasible_direction_time(sg, seed)
        # scale the direction to the solution's size
        d *= np.max(np.abs(x[: x.size // 3])) / np.max(np.abs(d[: d.size // 3]))
        jp, jm, j0 = J(x + d), J(x - d), J(x)
        curv = 0.5 * (jp + jm) - j0
        slope = 0.5 * (jp - jm)
        assert curv > 0
        assert abs(slope) < 1e-9 * curv, (slope, curv)


def test_stationarity_detects_gamma_on_the_mean_column(monkeypatch):
    """The pin above is sharp: with gamma wrongly applied to chaos column 0
    as well (H^gamma = (1+gamma) I), the direct solution is no longer
    stationary for the objective."""
    n, M, P, sigma, beta, gamma = 8, 2, 2, 0.3, 1e-2, 0.8
    sg = kkt.setup(kkt.Problem(n=n, M=M, P=P, sigma=sigma, beta=beta, gamma=gamma,
                               y_target=sg_inputs.gaussian_bumps(n, 3)))
    monkeypatch.setattr(kkt, "h_gamma", lambda s: np.full(s.n_xi, 1.0 + s.prob.gamma))
    x = kkt.solve_direct(sg)
    W, Psi = _quadrature(sg.alpha, P)
    Mf = _mass_full_1d_tensor(n)
    d = _feasible_direction_steady(sg, 11)
    d *= np.max(np.abs(x[: x.size // 3])) / np.max(np.abs(d[: d.size // 3]))
    jp, jm, j0 = (_objective_steady(sg, v, W, Psi, Mf) for v in (x + d, x - d, x))
    assert abs(0.5 * (jp - jm)) > 1e-3 * (0.5 * (jp + jm) - j0)


@pytest.mark.parametrize("M,P", [(2, 2), (3, 3)])
def test_moments_variance_equals_quadrature(M, P):
    """Var[y](x) = E[y^2] - E[y]^2 of the reconstructed field, by quadrature
    over xi, equals the oracle's variance field node by node (orthonormal
    basis; Section 2.1, H^sigma)."""
    n = 8
    sg = kkt.setup(kkt.Problem(n=n, M=M, P=P, sigma=0.35, beta=1e-2, gamma=0.5,
                               y_target=sg_inputs.gaussian_bumps(n, 4)))
    Y = kkt.split(sg, kkt.solve_direct(sg))[0]
    mean, var = kkt.moments(Y)
    W, Psi = _quadrature(sg.alpha, P)
    samples = Psi @ Y
    m_q = W @ samples
    v_q = W @ (samples ** 2) - m_q ** 2
    assert np.max(np.abs(mean - m_q)) < 1e-13 * np.max(np.abs(m_q))
    assert np.max(np.abs(var - v_q)) < 1e-10 * np.max(v_q)
    # the integrated variance of the finite-element field, E[(y - E y)^T M (y - E y)]
    # by quadrature, is the paper's discrete variance term y^T (H^sigma (x) M) y
    Mf = _mass_full_1d_tensor(n)
    Mi = Mf[_interior(n)][:, _interior(n)]
    y_msigma_y = sum(float(Y[j] @ (Mi @ Y[j])) for j in range(1, sg.n_xi))
    assert abs(_field_terms(Y, n, W, Psi, Mf) - y_msigma_y) < 1e-12 * y_msigma_y
