"""Preconditioner pieces, written out with explicit sparse matrices.

Oracle (test infrastructure only).

Paper passages followed
  * Section 2.2, eq. (stoch-prec): block-diagonal preconditioner
    blkdiag(M_gamma, beta M, S); Section 2.2, eq. (mathcalZ):
    S = Z M_gamma^{-1} Z^T with Z = sum_l H_l (x) A-tilde_l,
    A-tilde_1 = A_1 + sqrt((1+gamma)/beta) M, so S^{-1} = Z^{-1} M_gamma Z^{-1}.
  * Section 2.2 and Section 5: the mass blocks are inverted approximately by
    Chebyshev semi-iteration (Golub & Varga), D = ((lmin+lmax)/2) diag(M) with
    eigenvalue bounds [1/4, 9/4] of diag(M)^{-1} M.
  * Algorithm 1 (hGS): symmetric block Gauss-Seidel over the degree levels,
    diagonal blocks A-tilde_1, off-diagonal products truncated to the modes in
    I_tau (eq. matvec-block).
  * Algorithm 5 (preconditioned Richardson): each Z^{-1} is N steps from a
    zero initial guess, x <- x + hGS(b - Z_r x); N = 1 (the paper's runs) is
    one hGS application.
  * Section 5: the mass blocks by Chebyshev semi-iteration (5 or 10 steps) or
    by a direct (Cholesky) factorisation of M.
  * Section 3.1, eq. (precon for time), eq. (Z hat approx), eq. (A_hat) and
    Algorithm 4: the time-dependent preconditioner
    blkdiag(tau D (x) M_gamma, tau beta D (x) M, S-tilde) with Z-tilde
    block-diagonal in time and A-hat_1 = (1 + tau sqrt((1+gamma)/beta)) M
    + tau A_1, A-hat_l = tau A_l.

Readings (the paper is silent or ambiguous):
  * Chebyshev recurrence: the textbook Golub-Varga weights omega_1 = 1,
    omega_2 = 1/(1 - rho^2/2), omega_{k+1} = 1/(1 - rho^2 omega_k / 4);
  * the Schur block applies hGS twice (one Richardson N = 1 step per Z^{-1})
    with the M_gamma multiply between them;
  * S-tilde carries the 1/tau of S-bar, so S-tilde^{-1} = tau Z-tilde^{-1}
    (D (x) M_gamma) Z-tilde^{-1};
  * truncation r keeps the modes k = 1..r-1 (r = 1 is the mean-based
    preconditioner, r = M+1 keeps every mode of the affine field, r = n_A
    every term of the log-normal field);
  * the A-tilde_1 / A-hat_1 solves inside hGS are either exact (sparse LU,
    the "ideal" preconditioner of the analysis) or one geometric-multigrid
    V-cycle (the solver's choice in place of the paper's direct solves); the
    multigrid is defined in class GMG below.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from numpy.polynomial import Chebyshev, Polynomial

from . import fem, kkt


# ----------------------------------------------------------------------------
# Chebyshev semi-iteration for the mass matrix
# ----------------------------------------------------------------------------

def cheb_mass(Mi: sp.spmatrix, R: np.ndarray, steps: int,
              lmin: float = 0.25, lmax: float = 2.25) -> np.ndarray:
    """Approximate M^{-1} applied to each row of R by `steps` Chebyshev
    semi-iterations from x = 0 (Golub-Varga recurrence, textbook weights)."""
    gam = 0.5 * (lmin + lmax)
    rho = (lmax - lmin) / (lmax + lmin)
    dinv = 1.0 / (gam * Mi.diagonal())
    R = np.atleast_2d(R)
    x_prev = np.zeros_like(R)
    x = R * dinv                                   # k = 1, omega_1 = 1
    omega = 1.0
    for k in range(1, steps):
        omega = 1.0 / (1.0 - 0.5 * rho * rho) if k == 1 else 1.0 / (1.0 - 0.25 * rho * rho * omega)
        r = R - (Mi @ x.T).T
        x_new = omega * (r * dinv + x - x_prev) + x_prev
        x_prev, x = x, x_new
    return x


# ----------------------------------------------------------------------------
# Geometric multigrid for a K + b M (constant coefficients)
# ----------------------------------------------------------------------------

def prolongation_1d(nc: int) -> sp.csr_matrix:
    """Linear interpolation from the nc-1 interior nodes of a 1-D grid with nc
    cells to the 2nc-1 interior nodes of its bisection (zero end values)."""
    nf = 2 * nc
    rows, cols, vals = [], [], []
    for I in range(1, nc):              # coarse interior node I at fine node 2I
        j = I - 1
        for fi, w in ((2 * I - 1, 0.5), (2 * I, 1.0), (2 * I + 1, 0.5)):
            rows.append(fi - 1)
            cols.append(j)
            vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf - 1, nc - 1))


def prolongation_2d(nc: int) -> sp.csr_matrix:
    """Bilinear interpolation = tensor product of 1-D linear interpolation
    (interior nodes, iy-major)."""
    p = prolongation_1d(nc)
    return sp.kron(p, p, format="csr")


def sine_lambda_max(n: int, a: float, b: float) -> float:
    """Largest eigenvalue of diag(A)^{-1} A for A = a K + b M on the interior
    of the uniform n x n Q1 grid.

    The unit-coefficient Q1 matrices are K = K1 (x) M1 + M1 (x) K1 and
    M = M1 (x) M1 with the 1-D P1 matrices K1 = tridiag(-1,2,-1)/h and
    M1 = h tridiag(1,4,1)/6, whose common eigenvectors are the discrete sines
    with eigenvalues (2/h)(1 - cos i pi h) and (h/3)(2 + cos i pi h); the
    diagonal of A is the constant a 8/3 + b 4h^2/9."""
    h = 1.0 / n
    th = np.arange(1, n) * np.pi * h
    k1 = (2.0 / h) * (1.0 - np.cos(th))
    m1 = (h / 3.0) * (2.0 + np.cos(th))
    lam = a * (np.outer(k1, m1) + np.outer(m1, k1)) + b * np.outer(m1, m1)
    diag = a * 8.0 / 3.0 + b * 4.0 * h * h / 9.0
    return float(lam.max() / diag)


class GMG:
    """One V-cycle of geometric multigrid for A = a K + b M on the n x n grid.

    Definition (the solver's choice; the paper factorises A-tilde_1 directly):
      * levels n, n/2, ..., n_c with n_c = min(n, 8) (n a power of two);
      * level operator a K_l + b M_l, assembled on each grid (for nested Q1
        with constant coefficients this equals the Galerkin product
        P^T A_{l+1} P);
      * prolongation P = bilinear interpolation, restriction R = P^T;
      * smoother: polynomial (Chebyshev) smoothing x <- x + q(B) D^{-1}(b - A x)
        with B = D^{-1} A, D = diag(A), whose error propagator is
        T_nu((theta - B)/delta) / T_nu(theta/delta) on [lo, hi] =
        [0.3, 1.1] * lambda_max(B); nu_pre steps before and nu_post after the
        coarse correction;
      * coarsest level solved exactly (dense inverse);
      * zero initial guess.
    """

    def __init__(self, n: int, a: float, b: float, nu_pre: int = 2, nu_post: int = 2,
                 n_coarse: int = 8):
        self.n, self.a, self.b = n, a, b
        self.nu_pre, self.nu_post = nu_pre, nu_post
        sizes = [n]
        while sizes[-1] > n_coarse:
            sizes.append(sizes[-1] // 2)
        self.sizes = sizes
        self.A, self.Dinv, self.q = [], [], []
        for m in sizes:
            K = fem.restrict(fem.assemble_full(m, 1.0, "stiffness"), m)
            Mm = fem.restrict(fem.assemble_full(m, 1.0, "mass"), m)
            A = (a * K + b * Mm).tocsr()
            self.A.append(A)
            self.Dinv.append(1.0 / A.diagonal())
            lmax = sine_lambda_max(m, a, b)
            self.q.append((self._smoother_poly(nu_pre, 0.3 * lmax, 1.1 * lmax),
                           self._smoother_poly(nu_post, 0.3 * lmax, 1.1 * lmax)))
        self.P = [prolongation_2d(m // 2) for m in sizes[:-1]]
        self.coarse_inv = np.linalg.inv(self.A[-1].toarray())

    @staticmethod
    def _smoother_poly(nu: int, lo: float, hi: float) -> np.ndarray:
        """Power-series coefficients of q with 1 - t q(t) = T_nu((theta-t)/delta)/T_nu(theta/delta)."""
        if nu == 0:
            return np.zeros(1)
        theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
        Tn = Chebyshev.basis(nu).convert(kind=Polynomial)
        z = Polynomial([theta / delta, -1.0 / delta])
        p = Polynomial([0.0])
        zp = Polynomial([1.0])
        for c in Tn.coef:
            p = p + c * zp
            zp = zp * z
        p = p / Tn(theta / delta)
        one_minus = Polynomial([1.0]) - p
        q, rem = divmod(one_minus, Polynomial([0.0, 1.0]))
        assert np.all(np.abs(rem.coef) < 1e-10 * np.max(np.abs(one_minus.coef)))
        return q.coef

    def _smooth(self, lvl: int, x: np.ndarray, b: np.ndarray, which: int) -> np.ndarray:
        coef = self.q[lvl][which]
        if len(coef) == 1 and coef[0] == 0.0:
            return x
        A, Dinv = self.A[lvl], self.Dinv[lvl]
        w = Dinv[:, None] * (b - A @ x)
        # Horner: q(B) w = c0 w + B (c1 w + B (c2 w + ...)), B = D^{-1} A
        y = coef[-1] * w
        for c in coef[-2::-1]:
            y = c * w + Dinv[:, None] * (A @ y)
        return x + y

    def _vcycle(self, lvl: int, b: np.ndarray) -> np.ndarray:
        if lvl == len(self.sizes) - 1:
            return self.coarse_inv @ b
        x = np.zeros_like(b)
        x = self._smooth(lvl, x, b, 0)
        r = b - self.A[lvl] @ x
        P = self.P[lvl]
        x = x + P @ self._vcycle(lvl + 1, P.T @ r)
        x = self._smooth(lvl, x, b, 1)
        return x

    def apply(self, B: np.ndarray) -> np.ndarray:
        """V-cycle applied to each row of B (shape (cols, n_int))."""
        B = np.atleast_2d(B)
        return self._vcycle(0, B.T).T


class ExactSolve:
    """Exact inverse of A = a K + b M (sparse LU with one step of iterative
    refinement, so the result is the exact solve to rounding), for the ideal
    preconditioner and the exact mean-block option."""

    def __init__(self, n: int, a: float, b: float):
        K = fem.restrict(fem.assemble_full(n, 1.0, "stiffness"), n)
        Mm = fem.restrict(fem.assemble_full(n, 1.0, "mass"), n)
        self.A = (a * K + b * Mm).tocsc()
        self.lu = spla.splu(self.A)

    def apply(self, B: np.ndarray) -> np.ndarray:
        B = np.ascontiguousarray(np.atleast_2d(B).T)
        X = self.lu.solve(B)
        X = X + self.lu.solve(np.ascontiguousarray(B - self.A @ X))
        return X.T


# ----------------------------------------------------------------------------
# hGS (Algorithm 1) and the Schur block
# ----------------------------------------------------------------------------

def mean_operator_coeffs(sg: kkt.SG):
    """(a, b, scale): A-tilde_1 = a K_unit + b M and the factor on the
    off-level products, steady (eq. mathcalZ) or time-dependent (eq. A_hat).

    The mean coefficient kappa_0 must be a constant c0, so K_0 = c0 K_unit."""
    p = sg.prob
    c0 = float(sg.kappa[0].reshape(-1)[0])
    s = np.sqrt((1.0 + p.gamma) / p.beta)
    if p.steady:
        return c0, s, 1.0
    tau = p.tau
    return tau * c0, 1.0 + tau * s, tau


def make_inner(sg: kkt.SG, mode: str = "gmg", nu_pre: int = 2, nu_post: int = 2):
    a, b, _ = mean_operator_coeffs(sg)
    if mode == "exact":
        return ExactSolve(sg.prob.n, a, b)
    return GMG(sg.prob.n, a, b, nu_pre, nu_post)


def hgs(sg: kkt.SG, R: np.ndarray, inner, r_trunc: int) -> np.ndarray:
    """Algorithm 1 applied to R (shape (n_xi, n_int)), zero initial guess.

    Levels d = 0..P are the degree blocks; sweep d = 0..P then P-1..0.  For
    level d: V_(d) = A1^{-1} [R_(d) - sum_{tau in I_tau} scale A_tau V_(other) H_tau]
    with the product taken over all columns outside level d (the E and F
    terms of eq. alg-hGS2), using the current V.  I_tau = modes 1..r-1."""
    off = sg.offsets
    P = len(off) - 2
    _, _, scale = mean_operator_coeffs(sg)
    modes = list(range(1, min(r_trunc, len(sg.G))))
    V = np.zeros_like(R)
    order = list(range(P + 1)) + list(range(P - 1, -1, -1))
    for d in order:
        lo, hi = int(off[d]), int(off[d + 1])
        B = R[lo:hi].copy()
        if modes:
            Vm = V.copy()
            Vm[lo:hi] = 0.0
            for k in modes:
                Gk = sg.G[k]
                # rows lo:hi of (G_k^T V) then K_k on the spatial index
                W = Gk[:, lo:hi].T @ Vm
                B -= scale * (sg.K[k] @ W.T).T
        V[lo:hi] = inner.apply(B)
    return V


def richardson(sg: kkt.SG, R: np.ndarray, inner, r_trunc: int, steps: int = 1) -> np.ndarray:
    """Algorithm 5: N = steps preconditioned Richardson steps on Z_r X = R
    (R, X of shape (n_xi, n_int)) from X = 0, each preconditioned by one hGS
    (Algorithm 1): X <- X + hGS(R - Z_r X)."""
    X = hgs(sg, R, inner, r_trunc)
    if steps > 1:
        Z = z_truncated(sg, r_trunc)
        for _ in range(steps - 1):
            res = R - (Z @ X.ravel()).reshape(R.shape)
            X = X + hgs(sg, res, inner, r_trunc)
    return X


def schur_inverse(sg: kkt.SG, R: np.ndarray, inner, r_trunc: int, richardson_steps: int = 1) -> np.ndarray:
    """Steady: S^{-1} r ~ Z^{-1} M_gamma Z^{-1} r with each Z^{-1} Richardson
    (one hGS for N = 1).  Time-dependent (R has a leading n_t axis): per step
    t, tau Z_t^{-1} (D_tt M_gamma) Z_t^{-1} r_t."""
    p = sg.prob
    hg = kkt.h_gamma(sg)[:, None]
    zinv = lambda B: richardson(sg, B, inner, r_trunc, richardson_steps)   # noqa: E731
    if p.steady:
        V = zinv(R)
        W = hg * kkt.mass_apply(sg, V)
        return zinv(W)
    nt, tau = p.n_t, p.tau
    D = np.ones(nt)
    D[0] = D[-1] = 0.5
    out = np.empty_like(R)
    for t in range(nt):
        V = zinv(R[t])
        W = D[t] * hg * kkt.mass_apply(sg, V)
        out[t] = tau * zinv(W)
    return out


def precond_apply(sg: kkt.SG, r: np.ndarray, inner=None, r_trunc: int | None = None,
                  cheb_steps: int = 5, richardson_steps: int = 1) -> np.ndarray:
    """Block-diagonal preconditioner of eq. (stoch-prec) / eq. (precon for time)
    applied to a flat KKT vector.  cheb_steps = 0: the mass blocks by a direct
    factorisation of M (the paper's Cholesky variant)."""
    p = sg.prob
    if inner is None:
        inner = make_inner(sg)
    if r_trunc is None:
        r_trunc = len(sg.G)
    Ry, Ru, Rl = kkt.split(sg, r)
    hg = kkt.h_gamma(sg)[:, None]
    if p.steady:
        Zy = kkt_cheb(sg, Ry, cheb_steps) / hg
        Zu = kkt_cheb(sg, Ru, cheb_steps) / p.beta
    else:
        nt, tau = p.n_t, p.tau
        D = np.ones(nt)
        D[0] = D[-1] = 0.5
        Zy = np.empty_like(Ry)
        Zu = np.empty_like(Ru)
        for t in range(nt):
            Zy[t] = kkt_cheb(sg, Ry[t], cheb_steps) / (tau * D[t] * hg)
            Zu[t] = kkt_cheb(sg, Ru[t], cheb_steps) / (p.beta * tau * D[t])
    Zl = schur_inverse(sg, Rl, inner, r_trunc, richardson_steps)
    return np.concatenate([Zy.ravel(), Zu.ravel(), Zl.ravel()])


def kkt_cheb(sg: kkt.SG, R: np.ndarray, steps: int) -> np.ndarray:
    """M^{-1} applied to the rows of R: Chebyshev with `steps` steps, or
    exactly (sparse Cholesky-equivalent LU of M) when steps == 0."""
    if steps == 0:
        Mc = sp.csc_matrix(sg.Mi)
        lu = spla.splu(Mc)
        B = np.ascontiguousarray(np.atleast_2d(R).T)
        X = lu.solve(B)
        return (X + lu.solve(np.ascontiguousarray(B - Mc @ X))).T
    return cheb_mass(sg.Mi, R, steps)


def z_truncated(sg: kkt.SG, r_trunc: int) -> sp.csr_matrix:
    """Explicit Z_r = I (x) A1 + scale sum_{k=1}^{r-1} G_k (x) K_k (eq. S_r)."""
    a, b, scale = mean_operator_coeffs(sg)
    n = sg.prob.n
    K = fem.restrict(fem.assemble_full(n, 1.0, "stiffness"), n)
    A1 = (a * K + b * sg.Mi).tocsr()
    Z = sp.kron(sp.identity(sg.n_xi), A1, format="csr")
    for k in range(1, min(r_trunc, len(sg.G))):
        Z = Z + scale * sp.kron(sp.csr_matrix(sg.G[k]), sg.K[k], format="csr")
    return Z.tocsr()


# ----------------------------------------------------------------------------
# hGSoc: hierarchical Gauss-Seidel on the coupled KKT system (Algorithms 2-3)
# ----------------------------------------------------------------------------

class PtildeSolve:
    """Solves with P-tilde = blkdiag(M, beta M, A-tilde_1) column by column
    (Section 2.3, the auxiliary block-diagonal matrix of Algorithms 2-3).

    mode "exact": sparse LU of M and A-tilde_1 (the paper factorises P-tilde
    once); mode "cheb": Chebyshev semi-iteration with `cheb_steps` steps for
    M (the mass solves of the block preconditioner) and one multigrid V-cycle
    for A-tilde_1 (the solver's choice).

    adjoint "literal": P-tilde = blkdiag(M, beta M, A-tilde_1) as printed.
    adjoint "schur": the block-diagonal preconditioner of eq. (stoch-prec)
    restricted to chaos column j: blkdiag(h^gamma_j M, beta M, A-tilde_1
    (h^gamma_j M)^{-1} A-tilde_1), the third block applied as A-tilde_1^{-1}
    h^gamma_j M A-tilde_1^{-1}.  The adjoint row of the level-diagonal KKT
    block has no entry on the adjoint itself, so A-tilde_1 alone does not
    approximate it (with it the coupled sweep stagnates; see the iteration
    counts)."""

    def __init__(self, sg: kkt.SG, mode: str = "cheb", cheb_steps: int = 5, nu_pre: int = 2, nu_post: int = 2,
                 adjoint: str = "literal"):
        self.sg, self.mode, self.cheb_steps, self.adjoint = sg, mode, cheb_steps, adjoint
        self.inner = make_inner(sg, "exact" if mode == "exact" else "gmg", nu_pre, nu_post)
        if mode == "exact":
            self.mlu = spla.splu(sg.Mi.tocsc())

    def mass_inv(self, R: np.ndarray) -> np.ndarray:
        R = np.atleast_2d(R)
        if self.mode == "exact":
            return self.mlu.solve(np.ascontiguousarray(R.T)).T
        return cheb_mass(self.sg.Mi, R, self.cheb_steps)

    def apply(self, BY: np.ndarray, BU: np.ndarray, BL: np.ndarray, lo: int = 0, hi: int | None = None,
              w: float = 1.0):
        """Rows of BY, BU, BL are the chaos columns lo..hi-1.  w scales the
        state and control mass blocks: 1 for the steady system, tau D_tt for
        time step t of the all-at-once system (whose mean block is A-hat_1,
        eq. A_hat)."""
        VL = self.inner.apply(BL)
        beta = self.sg.prob.beta
        if self.adjoint == "schur":
            hg = kkt.h_gamma(self.sg)[lo:hi if hi is not None else lo + np.atleast_2d(BL).shape[0]][:, None]
            VL = self.inner.apply(w * hg * kkt.mass_apply(self.sg, VL))
            return self.mass_inv(BY) / (w * hg), self.mass_inv(BU) / (w * beta), VL
        return self.mass_inv(BY) / w, self.mass_inv(BU) / (w * beta), VL


def _step_scalings(sg: kkt.SG, t: int | None):
    """(w, c): the state and control mass blocks of the level system are w
    (h^gamma M, beta M), and the KKT couplings between levels (the off-level
    part of A, and the control-adjoint mass) carry the factor c.  Steady: (1,
    1).  Time step t of eq. (KKT:stoch-time-dependent) without its couplings
    to the neighbouring steps: (tau D_tt, tau): state row tau D_tt M_gamma y -
    L lambda, control row beta tau D_tt M u + tau M lambda, adjoint row -L y +
    tau M u, with L = I (x) (M + tau A_1) + tau sum_{l>=2} H_l (x) A_l."""
    if t is None:
        return 1.0, 1.0
    p = sg.prob
    D = 0.5 if t in (0, p.n_t - 1) else 1.0
    return p.tau * D, p.tau


def hgsoc(sg: kkt.SG, r: np.ndarray, ptilde: PtildeSolve, r_trunc: int, t: int | None = None) -> np.ndarray:
    """Algorithms 2-3 applied to a flat steady KKT residual (zero initial
    guess), returning the flat preconditioned vector.

    The unknowns are swept level by level, degrees d = 0..P and back
    P-1..0; at level d the three blocks solve with P-tilde against the level's
    residual rows minus the KKT couplings to every other level, taken with
    the current values:
      state row    R^Y - C + D,   C = M V^Y [h^gamma off-level],  D = sum_tau A_tau V^L [h_tau],
      control row  R^U - E - F,   E = beta M V^U [h_1 off-level],  F = M V^L [h_1 off-level],
      adjoint row  R^L + G - H,   G = sum_tau A_tau V^Y [h_tau],   H = M V^U [h_1 off-level],
    tau over the kept modes I_tau (k = 1..r-1).  H^gamma and H_1 = I are
    diagonal, so C, E, F and H vanish; they are formed anyway from the
    off-level parts of those matrices."""
    p = sg.prob
    assert p.steady == (t is None), "steady system, or one time step t of the all-at-once system"
    w, c = _step_scalings(sg, t)
    if t is None:
        Ry, Ru, Rl = (b.copy() for b in kkt.split(sg, r))
    else:
        Ry, Ru, Rl = (b.copy() for b in r.reshape(3, sg.n_xi, sg.n_int))
    off = sg.offsets
    P = len(off) - 2
    modes = list(range(1, min(r_trunc, len(sg.G))))
    hg = np.diag(kkt.h_gamma(sg))
    H1 = np.eye(sg.n_xi)
    VY, VU, VL = np.zeros_like(Ry), np.zeros_like(Ru), np.zeros_like(Rl)
    order = list(range(P + 1)) + list(range(P - 1, -1, -1))
    for d in order:
        lo, hi = int(off[d]), int(off[d + 1])

        def others(V):
            W = V.copy()
            W[lo:hi] = 0.0
            return W

        def couple(Hm, V):
            # columns lo:hi of V_mat Hm, as rows: (Hm[:, lo:hi])^T applied to the chaos rows of V
            return Hm[:, lo:hi].T @ V

        Yo, Uo, Lo = others(VY), others(VU), others(VL)
        C = w * kkt.mass_apply(sg, couple(hg, Yo))
        E = w * p.beta * kkt.mass_apply(sg, couple(H1, Uo))
        F = c * kkt.mass_apply(sg, couple(H1, Lo))
        Hh = c * kkt.mass_apply(sg, couple(H1, Uo))
        D = np.zeros((hi - lo, Ry.shape[1]))
        G = np.zeros_like(D)
        for k in modes:
            D += c * (sg.K[k] @ couple(sg.G[k], Lo).T).T
            G += c * (sg.K[k] @ couple(sg.G[k], Yo).T).T
        by = Ry[lo:hi] - C + D
        bu = Ru[lo:hi] - E - F
        bl = Rl[lo:hi] + G - Hh
        VY[lo:hi], VU[lo:hi], VL[lo:hi] = ptilde.apply(by, bu, bl, lo, hi, w)
    return np.concatenate([VY.ravel(), VU.ravel(), VL.ravel()])


def hgsoc_pint(sg: kkt.SG, r: np.ndarray, ptilde: PtildeSolve, r_trunc: int) -> np.ndarray:
    """Algorithm 4 (hGSoc-PINT): Algorithms 2-3 applied to each time step's
    subvector of the all-at-once residual independently (see _step_scalings
    for the step's blocks; the mean block is A-hat_1), the results
    concatenated in the flat time-dependent layout [block][t][j][node]."""
    p = sg.prob
    assert not p.steady
    nt, nx, ni = p.n_t, sg.n_xi, sg.n_int
    R = r.reshape(3, nt, nx, ni)
    out = np.empty_like(R)
    for t in range(nt):
        z = hgsoc(sg, R[:, t].reshape(-1), ptilde, r_trunc, t)
        out[:, t] = z.reshape(3, nx, ni)
    return out.reshape(-1)


def hgsoc_matrix_form(sg: kkt.SG, ptilde_blocks: tuple, r_trunc: int, col_weights: tuple | None = None,
                      coupling: float = 1.0) -> tuple:
    """The matrices behind Algorithms 2-3 with exact P-tilde solves: the level
    splitting K_r = D + L + U of the KKT matrix with every level-diagonal
    block replaced by P-tilde (per chaos column) and the off-level couplings
    truncated to the kept modes; one forward and one backward block
    Gauss-Seidel sweep from zero then equal (D + U)^{-1} D (D + L)^{-1}.
    ptilde_blocks = (M, beta M, A-tilde_1) as sparse matrices, scaled per
    chaos column by col_weights = (w_Y, w_U, w_Lambda) when given; the
    off-level couplings -A are scaled by `coupling` (tau for a time step of
    the all-at-once system).  Returns (D, L, U) over the unknown order
    [Y | U | Lambda], chaos-major inside a block."""
    p = sg.prob
    nxi, ni = sg.n_xi, sg.n_int
    Mb, bMb, A1 = ptilde_blocks
    off = sg.offsets
    level = np.zeros(nxi, dtype=int)
    for d in range(len(off) - 1):
        level[int(off[d]):int(off[d + 1])] = d
    modes = list(range(1, min(r_trunc, len(sg.G))))
    I = sp.identity(nxi, format="csr")
    if col_weights is None:
        Dg = sp.block_diag([sp.kron(I, Mb), sp.kron(I, bMb), sp.kron(I, A1)], format="csr")
    else:
        Dg = sp.block_diag([sp.kron(sp.diags(w), B) for w, B in zip(col_weights, (Mb, bMb, A1))], format="csr")
    # off-level couplings of the KKT rows (state: -A Lambda; adjoint: -A Y)
    Aoff = None
    for k in modes:
        t = sp.kron(sp.csr_matrix(sg.G[k]), sg.K[k], format="csr")
        Aoff = t if Aoff is None else Aoff + t
    Z = sp.csr_matrix((nxi * ni, nxi * ni))
    if Aoff is None:
        Aoff = Z
    Koff = sp.bmat([[None, None, -coupling * Aoff], [None, Z, None], [-coupling * Aoff, None, None]], format="csr")
    # level of each unknown (row / column)
    lev = np.tile(np.repeat(level, ni), 3)
    Kc = Koff.tocoo()
    lower = lev[Kc.row] > lev[Kc.col]
    upper = lev[Kc.row] < lev[Kc.col]
    n3 = 3 * nxi * ni
    L = sp.csr_matrix((Kc.data[lower], (Kc.row[lower], Kc.col[lower])), shape=(n3, n3))
    U = sp.csr_matrix((Kc.data[upper], (Kc.row[upper], Kc.col[upper])), shape=(n3, n3))
    return Dg, L, U
