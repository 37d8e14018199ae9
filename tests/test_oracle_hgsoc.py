"""Pins of the oracle's hGSoc preconditioner (Algorithms 2-3): the coupled
state/control/adjoint hierarchical Gauss-Seidel sweep over degree levels with
P-tilde = blkdiag(M, beta M, A-tilde_1) solves on each level.

The sweep is checked against the algebra it stands for, built independently
with explicit sparse matrices: one forward and one backward block
Gauss-Seidel sweep from zero on the KKT matrix split by degree levels
(level-diagonal blocks replaced by P-tilde, off-level couplings truncated to
the kept modes) equals (D + U)^{-1} D (D + L)^{-1}."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import sg_inputs
from oracle import fem, fgmres, kkt, precond


def _case(n, M, P, sigma, beta, gamma=0.0):
    prob = kkt.Problem(n=n, M=M, P=P, sigma=sigma, beta=beta, gamma=gamma, y_target=sg_inputs.gaussian_bumps(n, 0))
    return kkt.setup(prob)


def _ptilde_blocks(sg):
    a, b, _ = precond.mean_operator_coeffs(sg)
    K = fem.restrict(fem.assemble_full(sg.prob.n, 1.0, "stiffness"), sg.prob.n)
    return sg.Mi, sg.prob.beta * sg.Mi, (a * K + b * sg.Mi).tocsr()


@pytest.mark.parametrize("shape", [(8, 3, 3, 0.3, 1e-2, 0.0, 4), (8, 2, 4, 0.25, 1e-4, 0.5, 3),
                                   (8, 4, 2, 0.2, 1e-1, 0.0, 2), (4, 3, 2, 0.3, 1e-3, 0.0, 4)])
def test_hgsoc_equals_symmetric_block_gauss_seidel(shape):
    n, M, P, sigma, beta, gamma, r_trunc = shape
    sg = _case(n, M, P, sigma, beta, gamma)
    r = sg_inputs.random_block((3 * sg.n_xi * sg.n_int,), 3)
    z = precond.hgsoc(sg, r, precond.PtildeSolve(sg, "exact"), r_trunc)
    D, L, U = precond.hgsoc_matrix_form(sg, _ptilde_blocks(sg), r_trunc)
    x1 = spla.spsolve((D + L).tocsc(), r)
    zz = spla.spsolve((D + U).tocsc(), D @ x1)
    assert np.max(np.abs(z - zz)) < 1e-12 * np.max(np.abs(zz))


def test_hgsoc_splitting_reproduces_the_kkt_couplings():
    """D + L + U minus the level-diagonal P-tilde blocks plus the KKT's own
    level-diagonal blocks is the KKT matrix (all modes kept): the sweep sees
    exactly the KKT's off-level couplings."""
    sg = _case(8, 3, 2, 0.3, 1e-2)
    D, L, U = precond.hgsoc_matrix_form(sg, _ptilde_blocks(sg), sg.prob.M + 1)
    Kkkt = kkt.kkt_steady(sg)
    nxi, ni = sg.n_xi, sg.n_int
    lev = np.zeros(nxi, dtype=int)
    off = sg.offsets
    for d in range(len(off) - 1):
        lev[int(off[d]):int(off[d + 1])] = d
    levu = np.tile(np.repeat(lev, ni), 3)
    Kc = Kkkt.tocoo()
    same = levu[Kc.row] == levu[Kc.col]
    n3 = 3 * nxi * ni
    Kdiag = sp.csr_matrix((Kc.data[same], (Kc.row[same], Kc.col[same])), shape=(n3, n3))
    rebuilt = (Kdiag + L + U).toarray()
    assert np.max(np.abs(rebuilt - Kkkt.toarray())) < 1e-13 * abs(Kkkt).max()


def test_hgsoc_mean_based_is_ptilde():
    """r = 1 (no modes kept): every level is solved independently, so hGSoc is
    P-tilde^{-1} column by column."""
    sg = _case(8, 3, 2, 0.3, 1e-2)
    r = sg_inputs.random_block((3 * sg.n_xi * sg.n_int,), 5)
    pt = precond.PtildeSolve(sg, "exact")
    z = precond.hgsoc(sg, r, pt, 1)
    Ry, Ru, Rl = kkt.split(sg, r)
    Mb, bMb, A1 = _ptilde_blocks(sg)
    ref = [spla.spsolve(B.tocsc(), R.T).T for B, R in ((Mb, Ry), (bMb, Ru), (A1, Rl))]
    assert np.max(np.abs(z - np.concatenate([x.ravel() for x in ref]))) < 1e-12 * np.max(np.abs(z))


def test_hgsoc_flags_a_wrong_coupling_sign():
    """A plausible slip (adding instead of subtracting the state row's adjoint
    coupling, i.e. the sign of D) moves the result off the block Gauss-Seidel
    algebra by far more than rounding."""
    sg = _case(8, 3, 3, 0.3, 1e-2)
    r = sg_inputs.random_block((3 * sg.n_xi * sg.n_int,), 7)
    D, L, U = precond.hgsoc_matrix_form(sg, _ptilde_blocks(sg), sg.prob.M + 1)
    Dm, Lm, Um = D, -L, -U           # the mistake: couplings with the wrong sign
    x1 = spla.spsolve((Dm + Lm).tocsc(), r)
    wrong = spla.spsolve((Dm + Um).tocsc(), Dm @ x1)
    z = precond.hgsoc(sg, r, precond.PtildeSolve(sg, "exact"), sg.prob.M + 1)
    assert np.max(np.abs(z - wrong)) > 1e-3 * np.max(np.abs(z))


@pytest.mark.parametrize("gamma", [0.0, 0.5])
def test_hgsoc_schur_reading_equals_block_gauss_seidel(gamma):
    """With the Schur-type reading (the block-diagonal preconditioner
    restricted to each chaos column: h^gamma_j M, beta M, A-tilde_1
    (h^gamma_j M)^{-1} A-tilde_1) the sweep is the same block Gauss-Seidel
    algebra with those blocks on the diagonal."""
    sg = _case(8, 3, 3, 0.3, 1e-2, gamma)
    r = sg_inputs.random_block((3 * sg.n_xi * sg.n_int,), 9)
    z = precond.hgsoc(sg, r, precond.PtildeSolve(sg, "exact", adjoint="schur"), sg.prob.M + 1)
    Mb, bMb, A1 = _ptilde_blocks(sg)
    S = (A1 @ spla.spsolve(sg.Mi.tocsc(), A1.tocsc())).tocsr()
    hg = kkt.h_gamma(sg)
    D, L, U = precond.hgsoc_matrix_form(sg, (Mb, bMb, S), sg.prob.M + 1,
                                        col_weights=(hg, np.ones(sg.n_xi), 1.0 / hg))
    x1 = spla.spsolve((D + L).tocsc(), r)
    zz = spla.spsolve((D + U).tocsc(), D @ x1)
    assert np.max(np.abs(z - zz)) < 1e-10 * np.max(np.abs(zz))


def test_hgsoc_preconditioned_fgmres_converges():
    """FGMRES with hGSoc (Schur-type adjoint block; multigrid and Chebyshev
    solves inside, as on the GPU) reaches the direct solution; iteration
    counts are context only."""
    sg = _case(8, 3, 3, 0.3, 1e-2)
    b = kkt.rhs(sg)
    K = kkt.kkt_steady(sg)
    pt = precond.PtildeSolve(sg, "cheb", adjoint="schur")
    x, info = fgmres.fgmres(lambda v: K @ v, lambda v: precond.hgsoc(sg, v, pt, sg.prob.M + 1), b, tol=1e-10,
                            restart=30, max_iter=400)
    assert info["converged"]
    ref = kkt.solve_direct(sg)
    assert np.max(np.abs(x - ref)) < 1e-7 * np.max(np.abs(ref))


# ----------------------------------------------------------------------------
# Algorithm 4 (hGSoc-PINT): Algorithms 2-3 on every time step of the
# all-at-once system
# ----------------------------------------------------------------------------

def _time_case(n, M, P, sigma, beta, gamma, nt):
    prob = kkt.Problem(n=n, M=M, P=P, sigma=sigma, beta=beta, gamma=gamma, n_t=nt, T=1.0,
                       y_target=sg_inputs.moving_bump(n, nt, 1.0, 0))
    return kkt.setup(prob)


def _step_rows(sg, t):
    """Flat indices of time step t's unknowns in the all-at-once layout, in the
    order [Y | U | Lambda], chaos-major inside a block."""
    nt, nx, ni = sg.prob.n_t, sg.n_xi, sg.n_int
    blk = nt * nx * ni
    one = t * nx * ni + np.arange(nx * ni)
    return np.concatenate([one, blk + one, 2 * blk + one])


@pytest.mark.parametrize("gamma", [0.0, 0.5])
def test_hgsoc_pint_splitting_is_each_steps_kkt_block(gamma):
    """For every time step, the level-diagonal blocks of that step's rows of
    the all-at-once KKT matrix plus the splitting's off-level parts L + U
    (couplings scaled by tau) rebuild the step's block of the KKT matrix: the
    sweep sees the step's own couplings with the right scale and sign, and
    only the couplings to the neighbouring steps are left out."""
    sg = _time_case(8, 3, 2, 0.3, 1e-2, gamma, 3)
    Kt = kkt.kkt_time(sg).tocsr()
    nxi, ni = sg.n_xi, sg.n_int
    lev = np.zeros(nxi, dtype=int)
    off = sg.offsets
    for d in range(len(off) - 1):
        lev[int(off[d]):int(off[d + 1])] = d
    levu = np.tile(np.repeat(lev, ni), 3)
    n3 = 3 * nxi * ni
    a, b, _ = precond.mean_operator_coeffs(sg)
    K = fem.restrict(fem.assemble_full(sg.prob.n, 1.0, "stiffness"), sg.prob.n)
    for t in range(sg.prob.n_t):
        idx = _step_rows(sg, t)
        Ks = Kt[idx][:, idx].tocoo()
        same = levu[Ks.row] == levu[Ks.col]
        Kdiag = sp.csr_matrix((Ks.data[same], (Ks.row[same], Ks.col[same])), shape=(n3, n3))
        _, L, U = precond.hgsoc_matrix_form(sg, (sg.Mi, sg.Mi, (a * K + b * sg.Mi).tocsr()), sg.prob.M + 1,
                                            coupling=sg.prob.tau)
        rebuilt = (Kdiag + L + U).toarray()
        assert np.max(np.abs(rebuilt - Ks.toarray())) < 1e-13 * abs(Kt).max()


@pytest.mark.parametrize("shape", [(8, 3, 2, 0.3, 1e-2, 0.5, 3, 4), (8, 2, 3, 0.25, 1e-3, 0.0, 4, 2)])
def test_hgsoc_pint_equals_block_gauss_seidel_per_step(shape):
    """Each time step's part of Algorithm 4 is the symmetric block
    Gauss-Seidel algebra of that step's level-split system with the step's
    P-tilde blocks on the diagonal: tau D_tt h^gamma_j M, beta tau D_tt M and
    A-hat_1 (tau D_tt h^gamma_j M)^{-1} A-hat_1 (eq. A_hat), couplings scaled
    by tau."""
    n, M, P, sigma, beta, gamma, nt, r_trunc = shape
    sg = _time_case(n, M, P, sigma, beta, gamma, nt)
    p = sg.prob
    r = sg_inputs.random_block((3 * nt * sg.n_xi * sg.n_int,), 11)
    z = precond.hgsoc_pint(sg, r, precond.PtildeSolve(sg, "exact", adjoint="schur"), r_trunc)
    a, b, _ = precond.mean_operator_coeffs(sg)
    K = fem.restrict(fem.assemble_full(n, 1.0, "stiffness"), n)
    A1 = (a * K + b * sg.Mi).tocsr()
    S = (A1 @ spla.spsolve(sg.Mi.tocsc(), A1.tocsc())).tocsr()
    hg = kkt.h_gamma(sg)
    for t in range(nt):
        w = p.tau * (0.5 if t in (0, nt - 1) else 1.0)
        D, L, U = precond.hgsoc_matrix_form(sg, (sg.Mi, p.beta * sg.Mi, S), r_trunc,
                                            col_weights=(w * hg, w * np.ones(sg.n_xi), 1.0 / (w * hg)),
                                            coupling=p.tau)
        idx = _step_rows(sg, t)
        x1 = spla.spsolve((D + L).tocsc(), r[idx])
        zz = spla.spsolve((D + U).tocsc(), D @ x1)
        assert np.max(np.abs(z[idx] - zz)) < 1e-10 * np.max(np.abs(zz))


def test_hgsoc_pint_preconditioned_fgmres_converges():
    """FGMRES on the all-at-once KKT system with Algorithm 4 (Chebyshev and
    multigrid solves inside, as on the GPU) reaches the direct solution."""
    sg = _time_case(8, 3, 2, 0.3, 1e-2, 0.0, 3)
    b = kkt.rhs(sg)
    K = kkt.kkt_time(sg)
    pt = precond.PtildeSolve(sg, "cheb", adjoint="schur")
    x, info = fgmres.fgmres(lambda v: K @ v, lambda v: precond.hgsoc_pint(sg, v, pt, sg.prob.M + 1), b, tol=1e-10,
                            restart=30, max_iter=400)
    assert info["converged"]
    ref = kkt.solve_direct(sg)
    assert np.max(np.abs(x - ref)) < 1e-7 * np.max(np.abs(ref))
