"""Pins of the oracle's preconditioner pieces: Chebyshev semi-iteration,
geometric multigrid, hGS (Algorithm 1) and the Schur block."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from numpy.polynomial import chebyshev as C

import sg_inputs
from oracle import fem, fgmres, kkt, precond


@pytest.mark.parametrize("steps", [1, 2, 5, 10])
def test_cheb_mass_on_sine_mode_closed_form(steps):
    """On the sine eigenvector of diag(M)^{-1}M (eigenvalue mu), the
    Chebyshev semi-iteration from 0 has error factor
    T_k((1 - mu/g)/rho) / T_k(1/rho), g = 5/4, rho = 0.8 (Golub-Varga)."""
    n = 16
    h = 1.0 / n
    Mi = fem.restrict(fem.assemble_full(n, 1.0, "mass"), n)
    v = fem.extract(sg_inputs.unit_sine(n), n)
    m1 = (h / 3) * (2 + np.cos(np.pi * h))
    lam = m1 * m1                                    # M v = lam v
    mu = lam / (4 * h * h / 9)                       # diag(M)^{-1} M v = mu v
    g, rho = 1.25, 0.8
    x = precond.cheb_mass(Mi, v[None, :], steps)[0]
    err_factor = C.chebval((1 - mu / g) / rho, [0] * steps + [1]) / C.chebval(1 / rho, [0] * steps + [1])
    expect = (1 - err_factor) * v / lam
    assert np.max(np.abs(x - expect)) < 1e-13 * np.max(np.abs(expect))


def test_cheb_mass_converges():
    n = 8
    Mi = fem.restrict(fem.assemble_full(n, 1.0, "mass"), n)
    r = sg_inputs.random_block((3, (n - 1) ** 2), 1)
    exact = spla.spsolve(Mi.tocsc(), r.T).T
    e5 = np.max(np.abs(precond.cheb_mass(Mi, r, 5) - exact))
    e10 = np.max(np.abs(precond.cheb_mass(Mi, r, 10) - exact))
    assert e10 < 0.2 * e5 < 0.2 * np.max(np.abs(exact))


@pytest.mark.parametrize("n", [4, 8, 16])
@pytest.mark.parametrize("a,b", [(1.0, 0.0), (1.0, 10.0), (0.03, 1.3), (1.0, 1e3)])
def test_lambda_max_formula_against_eigensolver(n, a, b):
    K = fem.restrict(fem.assemble_full(n, 1.0, "stiffness"), n)
    Mm = fem.restrict(fem.assemble_full(n, 1.0, "mass"), n)
    A = (a * K + b * Mm).toarray()
    d = np.diag(A)
    ev = np.linalg.eigvalsh(A / np.sqrt(np.outer(d, d)))
    assert abs(precond.sine_lambda_max(n, a, b) - ev.max()) < 1e-13 * ev.max()


@pytest.mark.parametrize("nc", [4, 8])
def test_galerkin_coarse_operator_is_rediscretisation(nc):
    """Nested Q1 spaces: P^T A_h P equals the operator assembled on the coarse grid."""
    a, b = 0.7, 3.0
    nf = 2 * nc
    P = precond.prolongation_2d(nc)

    def op(m):
        K = fem.restrict(fem.assemble_full(m, 1.0, "stiffness"), m)
        Mm = fem.restrict(fem.assemble_full(m, 1.0, "mass"), m)
        return a * K + b * Mm
    G = (P.T @ op(nf) @ P).toarray()
    assert np.max(np.abs(G - op(nc).toarray())) < 1e-13


def test_prolongation_reproduces_bilinear_functions():
    """Bilinear interpolation is exact for x*y type functions (vanishing on the boundary)."""
    nc = 4
    f = lambda m: fem.extract(sg_inputs.node_coords(m)[0] * (1 - sg_inputs.node_coords(m)[0])
                              * sg_inputs.node_coords(m)[1], m)
    P = precond.prolongation_2d(nc)
    xc, yc = sg_inputs.node_coords(nc)
    xf, yf = sg_inputs.node_coords(2 * nc)
    # piecewise-bilinear function: interpolate g = x*y on each coarse cell exactly
    g_c = fem.extract(xc * yc * (xc < 1) * (yc < 1), nc)
    g_f = fem.extract(xf * yf * (xf < 1) * (yf < 1), 2 * nc)
    # x*y is bilinear, so away from the last coarse cells the interpolation is exact
    mask = fem.extract(((xf <= 1 - 1 / nc) & (yf <= 1 - 1 / nc)).astype(float), 2 * nc) > 0
    assert np.max(np.abs((P @ g_c - g_f)[mask])) < 1e-15


def test_smoother_polynomial_matches_three_term_recurrence():
    """The smoother's power-series q equals Chebyshev acceleration run with the
    classical three-term recurrence (Saad, Iterative Methods, Alg. 12.1)."""
    n, a, b = 8, 1.0, 5.0
    g = precond.GMG(n, a, b, 3, 3)
    A, Dinv = g.A[0], g.Dinv[0]
    lmax = precond.sine_lambda_max(n, a, b)
    lo, hi = 0.3 * lmax, 1.1 * lmax
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    rhs = sg_inputs.random_block(((n - 1) ** 2, 2), 4)
    x0 = sg_inputs.random_block(((n - 1) ** 2, 2), 5)
    # recurrence
    sig = theta / delta
    rho_old = 1.0 / sig
    x = x0.copy()
    d = Dinv[:, None] * (rhs - A @ x) / theta
    x = x + d
    for _ in range(2):
        rho = 1.0 / (2 * sig - rho_old)
        d = rho * rho_old * d + (2 * rho / delta) * Dinv[:, None] * (rhs - A @ x)
        x = x + d
        rho_old = rho
    y = g._smooth(0, x0, rhs, 0)
    assert np.max(np.abs(x - y)) < 1e-13 * np.max(np.abs(y))


@pytest.mark.parametrize("n", [16, 32])
@pytest.mark.parametrize("a,b", [(1.0, 10.0), (1.0, 1e3), (1 / 32, 1.3), (1.0, 0.0)])
def test_vcycle_contraction_and_symmetry(n, a, b):
    g = precond.GMG(n, a, b)
    A = g.A[0]
    N = A.shape[0]
    Vmat = g.apply(np.eye(N)).T                      # V-cycle as an explicit matrix
    assert np.max(np.abs(Vmat - Vmat.T)) < 1e-12 * np.max(np.abs(Vmat))
    E = np.eye(N) - Vmat @ A.toarray()
    # energy-norm contraction: spectral radius of the error propagator
    rho = np.max(np.abs(np.linalg.eigvals(E)))
    assert rho < 0.2


def _sg(n=8, M=3, P=3, sigma=0.3, beta=1e-2, gamma=0.0, nt=1):
    tgt = sg_inputs.gaussian_bumps(n, 1) if nt <= 1 else sg_inputs.moving_bump(n, nt, 1.0, 2)
    return kkt.setup(kkt.Problem(n=n, M=M, P=P, sigma=sigma, beta=beta, gamma=gamma, n_t=nt, y_target=tgt))


@pytest.mark.parametrize("nt", [1, 4])
@pytest.mark.parametrize("r", [1, 2, 4])
def test_hgs_equals_symmetric_gauss_seidel_factorisation(nt, r):
    """With exact inner solves, hGS is the inverse of
    (X_1 + X_r) X_1^{-1} (X_1 + X_r^T) (Section 4, the hGS bound), X_1 the
    level-diagonal part and X_r the strictly lower (lower-degree) part of Z_r.
    r = 1 reduces to the mean-based I (x) A1^{-1}."""
    sg = _sg(nt=nt)
    inner = precond.make_inner(sg, "exact")
    Z = precond.z_truncated(sg, r).toarray()
    ni = sg.n_int
    lvl = np.repeat(np.searchsorted(sg.offsets, np.arange(sg.n_xi), side="right") - 1, ni)
    X1 = np.where(lvl[:, None] == lvl[None, :], Z, 0.0)
    Xr = np.where(lvl[:, None] > lvl[None, :], Z, 0.0)
    Zh = (X1 + Xr) @ np.linalg.solve(X1, X1 + Xr.T)
    R = sg_inputs.random_block((sg.n_xi, ni), 8)
    V = precond.hgs(sg, R, inner, r)
    expect = np.linalg.solve(Zh, R.ravel()).reshape(R.shape)
    assert np.max(np.abs(V - expect)) < 1e-11 * np.max(np.abs(expect))
    if r == 1:
        a, b, _ = precond.mean_operator_coeffs(sg)
        A1 = (a * fem.restrict(fem.assemble_full(sg.prob.n, 1.0, "stiffness"), sg.prob.n) + b * sg.Mi).tocsc()
        assert np.max(np.abs(V - spla.spsolve(A1, R.T).T)) < 1e-12 * np.max(np.abs(V))


def test_z_truncated_full_equals_operator():
    """r = M+1 (steady): Z = A + sqrt((1+gamma)/beta) M-cal (eq. mathcalZ)."""
    sg = _sg(gamma=0.5)
    Z = precond.z_truncated(sg, sg.prob.M + 1)
    s = np.sqrt(1.5 / sg.prob.beta)
    assert abs(Z - (kkt.A_kron(sg) + s * kkt.Mcal(sg))).max() < 1e-12


def test_time_z_tilde_matches_paper_form():
    """eq. (another form of Ztilde): Z-tilde = tau sqrt((1+gamma)/beta) N + I (x) L, per time step."""
    sg = _sg(nt=4, gamma=0.2)
    p = sg.prob
    Z = precond.z_truncated(sg, p.M + 1)
    expect = p.tau * np.sqrt((1 + p.gamma) / p.beta) * kkt.Mcal(sg) + kkt.L_cal(sg)
    assert abs(Z - expect).max() < 1e-12


def test_schur_with_exact_mean_solves():
    """r = 1 with exact inner solves: S^{-1} = (I (x) A1^{-1}) M_gamma (I (x) A1^{-1})."""
    sg = _sg(gamma=0.4)
    inner = precond.make_inner(sg, "exact")
    R = sg_inputs.random_block((sg.n_xi, sg.n_int), 2)
    Zinv = lambda X: inner.apply(X)
    expect = Zinv(kkt.h_gamma(sg)[:, None] * kkt.mass_apply(sg, Zinv(R)))
    got = precond.schur_inverse(sg, R, inner, 1)
    assert np.max(np.abs(got - expect)) < 1e-13 * np.max(np.abs(expect))


def test_fgmres_minimal_residual_property():
    """GMRES minimises ||b - A x|| over the Krylov space: compare each iterate
    (no restart, identity preconditioner) with a least-squares solve over an
    explicitly formed Krylov basis."""
    rng = np.random.default_rng(0)
    n = 40
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) * 0.4
    b = rng.standard_normal(n)
    for k in (3, 7, 12):
        x, info = fgmres.fgmres(lambda v: A @ v, lambda v: v, b, tol=1e-30, restart=k, max_iter=k)
        Kry = np.stack([np.linalg.matrix_power(A, i) @ b for i in range(k)], axis=1)
        Q, _ = np.linalg.qr(Kry)
        y = np.linalg.lstsq(A @ Q, b, rcond=None)[0]
        assert abs(np.linalg.norm(b - A @ x) - np.linalg.norm(b - A @ Q @ y)) < 1e-10


def test_fgmres_solves_small_kkt_and_truncation_trend():
    """FGMRES with the block preconditioner reaches 1e-8; keeping the
    first-order modes (r = M+1) needs no more iterations than the mean-based
    r = 1 (the qualitative trend of Tables 1-4)."""
    sg = _sg(n=16, M=3, P=3, sigma=0.6)
    K = kkt.kkt_matrix(sg)
    b = kkt.rhs(sg)
    inner = precond.make_inner(sg)
    its = {}
    for r in (1, sg.prob.M + 1):
        x, info = fgmres.fgmres(lambda v: K @ v, lambda v: precond.precond_apply(sg, v, inner, r), b, 1e-8)
        assert info["converged"] and info["rel_res"] <= 1e-8
        its[r] = info["iters"]
    assert its[sg.prob.M + 1] <= its[1]


def _exact_schur_pair(sg, r_trunc):
    """(oracle S-approximation inverse as a dense matrix, exact Schur
    complement of the oracle's KKT matrix): the KKT matrix is
    [[A_bar, B^T], [B, 0]] with A_bar the (y, u) block, so the exact Schur
    complement of the adjoint block is B A_bar^{-1} B^T, whatever the scale the
    paper prints for it."""
    K = kkt.kkt_matrix(sg).toarray()
    m = K.shape[0] // 3
    S_exact = K[2 * m:, :2 * m] @ np.linalg.solve(K[:2 * m, :2 * m], K[2 * m:, :2 * m].T)
    inner = precond.make_inner(sg, "exact")
    shp = kkt.block_shape(sg)
    eye = np.eye(m)
    Sinv = np.array([precond.schur_inverse(sg, eye[i].reshape(shp), inner, r_trunc).ravel()
                     for i in range(m)]).T
    return Sinv, S_exact


@pytest.mark.parametrize("beta", [1e-2, 1e-4])
def test_steady_schur_approximation_spectrum(beta):
    """Steady, gamma = 0, deterministic field (so one hGS with exact inner
    solves is Z^{-1} exactly): S = Z M^{-1} Z with Z = A + M/sqrt(beta) is the
    matching approximation of S_exact = A M^{-1} A + M/beta, whose cross term
    (A M^{-1} M + M M^{-1} A)/sqrt(beta) = 2A/sqrt(beta) is positive definite,
    so the eigenvalues of S^{-1} S_exact lie in [1/2, 1] (eq. mathcalZ; the
    bound of Theorem thm:approx in its steady form).  A slip in the scale of
    either hGS, of the M_gamma product or of sqrt((1+gamma)/beta) leaves it."""
    sg = kkt.setup(kkt.Problem(n=4, M=2, P=2, sigma=0.0, beta=beta, y_target=sg_inputs.gaussian_bumps(4, 2)))
    Sinv, S_exact = _exact_schur_pair(sg, sg.prob.M + 1)
    ev = np.linalg.eigvals(Sinv @ S_exact)
    assert np.max(np.abs(ev.imag)) < 1e-10
    assert ev.real.min() >= 0.5 - 1e-10 and ev.real.max() <= 1.0 + 1e-10


@pytest.mark.parametrize("nt", [1, 8])
@pytest.mark.parametrize("gamma", [0.0, 0.5])
def test_schur_scale_in_the_small_beta_limit(gamma, nt):
    """Deterministic field, exact inner solves (so the hGS is Z^{-1} /
    Z-tilde^{-1} exactly).  Steady (eq. mathcalZ): for beta -> 0 both
    S_exact = A M_gamma^{-1} A + M/beta and S = Z M_gamma^{-1} Z are dominated
    by their 1/beta mass terms, M/beta and ((1+gamma)/beta) M M_gamma^{-1} M.
    Time-dependent: for beta -> 0 with tau fixed (tau >> sqrt(beta), the regime
    of Lemma lem:lower_bound) both the exact Schur complement
    B A_bar^{-1} B^T and S-tilde = (1/tau) Z-tilde (D (x) M_gamma)^{-1} Z-tilde
    are dominated by their (tau/beta) N (.)^{-1} N terms, which coincide up to
    the variance weight: on chaos column 0 (h^gamma = 1) the ratio is
    1/(1+gamma), on the other columns 1.  So the eigenvalues of
    S-tilde^{-1} S_exact approach {1/(1+gamma), 1}.  Reading: S-tilde carries
    the 1/tau of S-bar (eq. S hat); a tau^2, 1 or 1/tau in its place scales
    every eigenvalue by tau^{+-1} (here 8) and fails; in either form a slip of
    H^gamma in the middle factor moves the mean-column limit."""
    tgt = sg_inputs.gaussian_bumps(4, 2) if nt <= 1 else sg_inputs.moving_bump(4, nt, 1.0, 2)
    sg = kkt.setup(kkt.Problem(n=4, M=2, P=1, sigma=0.0, beta=1e-10, gamma=gamma, n_t=nt, y_target=tgt))
    Sinv, S_exact = _exact_schur_pair(sg, sg.prob.M + 1)
    ev = np.linalg.eigvals(Sinv @ S_exact)
    assert np.max(np.abs(ev.imag)) < 1e-8
    lo = 1.0 / (1.0 + gamma)
    assert ev.real.min() >= lo - 0.01 and ev.real.max() <= 1.0 + 1e-8
    if gamma > 0:
        # both limits are attained: the mean column and the fluctuation columns
        assert np.any(np.abs(ev.real - lo) < 0.01) and np.any(np.abs(ev.real - 1.0) < 0.01)


@pytest.mark.parametrize("nt", [1, 3])
def test_mass_blocks_invert_the_preconditioner_diagonal(nt):
    """The state and control blocks of the preconditioner approximate the
    inverses of the (1,1) and (2,2) blocks of eq. (stoch-prec) / eq. (precon
    for time): (tau D (x) H^gamma (x) M) and (tau beta D (x) H_1 (x) M) (steady:
    tau = D = 1).  With 60 Chebyshev steps the semi-iteration is exact to
    rounding, so applied to those blocks times v the preconditioner returns v.
    The block products are formed here from the interior mass matrix and
    H^gamma = diag(1, 1+gamma, ..., 1+gamma) written out, not from the
    oracle's KKT pieces; a slip of H^gamma <-> 1/H^gamma, beta <-> 1/beta or
    tau <-> 1/tau fails."""
    gamma, beta = 0.7, 3e-3
    n, M, P = 8, 2, 2
    target = sg_inputs.gaussian_bumps(n, 1) if nt <= 1 else sg_inputs.moving_bump(n, nt, 1.0, 3)
    sg = kkt.setup(kkt.Problem(n=n, M=M, P=P, sigma=0.3, beta=beta, gamma=gamma, n_t=nt, y_target=target,
                               T=0.6))
    Mi = fem.restrict(fem.assemble_full(n, 1.0, "mass"), n)
    hg = np.full(sg.n_xi, 1.0 + gamma)
    hg[0] = 1.0
    shp = kkt.block_shape(sg)
    vy = sg_inputs.random_block(shp, 21)
    vu = sg_inputs.random_block(shp, 22)
    if nt <= 1:
        ry = hg[:, None] * (Mi @ vy.T).T
        ru = beta * (Mi @ vu.T).T
    else:
        tau = 0.6 / nt
        D = np.ones(nt)
        D[0] = D[-1] = 0.5
        ry = np.stack([tau * D[t] * hg[:, None] * (Mi @ vy[t].T).T for t in range(nt)])
        ru = np.stack([tau * beta * D[t] * (Mi @ vu[t].T).T for t in range(nt)])
    rl = sg_inputs.random_block(shp, 23)
    r = np.concatenate([ry.ravel(), ru.ravel(), rl.ravel()])
    zy, zu, _ = kkt.split(sg, precond.precond_apply(sg, r, precond.make_inner(sg), cheb_steps=60))
    assert np.max(np.abs(zy - vy)) < 1e-12 and np.max(np.abs(zu - vu)) < 1e-12


def test_richardson_converges_to_truncated_z_solve():
    """Algorithm 5: N preconditioned Richardson steps with hGS (exact inner
    solves) approach Z_r^{-1} R, Z_r assembled independently as explicit
    Kronecker sums, geometrically; N = 1 is one hGS."""
    for r_trunc in (2, 3):
        prob = kkt.Problem(n=8, M=2, P=2, sigma=0.3, beta=1e-2, gamma=0.0, n_t=1, T=1.0,
                           y_target=sg_inputs.gaussian_bumps(8, 0))
        sg = kkt.setup(prob)
        inner = precond.make_inner(sg, "exact")
        R = np.random.default_rng(1).standard_normal((sg.n_xi, sg.Mi.shape[0]))
        ex = spla.spsolve(precond.z_truncated(sg, r_trunc).tocsc(), R.ravel()).reshape(R.shape)
        assert np.array_equal(precond.richardson(sg, R, inner, r_trunc, 1), precond.hgs(sg, R, inner, r_trunc))
        errs = [np.linalg.norm(precond.richardson(sg, R, inner, r_trunc, N) - ex) / np.linalg.norm(ex)
                for N in (1, 2, 3, 6)]
        assert errs[0] < 0.05 and errs[1] < 0.1 * errs[0] and errs[2] < 0.1 * errs[1] and errs[3] < 1e-11, errs


def test_exact_mass_solve():
    """cheb_steps = 0: the mass blocks by a direct solve; M applied to the
    result gives back the right-hand side, while 5 Chebyshev steps do not."""
    prob = kkt.Problem(n=8, M=2, P=2, sigma=0.3, beta=1e-2, gamma=0.0, n_t=1, T=1.0,
                       y_target=sg_inputs.gaussian_bumps(8, 0))
    sg = kkt.setup(prob)
    R = np.random.default_rng(2).standard_normal((4, sg.Mi.shape[0]))
    X = precond.kkt_cheb(sg, R, 0)
    assert np.max(np.abs((sg.Mi @ X.T).T - R)) < 1e-13 * np.max(np.abs(R))
    X5 = precond.kkt_cheb(sg, R, 5)
    assert np.max(np.abs((sg.Mi @ X5.T).T - R)) > 1e-6 * np.max(np.abs(R))
