"""Stochastic-Galerkin matrices and the KKT systems, assembled explicitly.

Oracle (test infrastructure only).

Paper passages followed
  * Section 2.1, eq. (stoch-system): steady KKT
        [[M_gamma, 0, -A^T], [0, beta M, M^T], [-A, M, 0]] [y; u; lambda]
      = [M y_d; 0; g],
    with M_gamma = H^gamma (x) M, H^gamma = H_1 + gamma H^sigma,
    H^sigma = diag(0, 1, ..., 1), M = H_1 (x) M, A = sum_l H_l (x) A_l.
  * Section 2.2, eq. (mat-vec) and eq. (Zv): (V (x) W) vec(X) = vec(W X V^T);
    the operator apply in matricized form is sum_l A_l X H_l.
  * Section 3, eq. (back Euler), eq. (K_t for stochastic), eq. (CD) and
    eq. (KKT:stoch-time-dependent): all-at-once backward-Euler system with
    A_t = I (x) L - C (x) M, L = H_1 (x) (M + tau A_1) + tau sum_{l>=2} H_l (x) A_l,
    N = I (x) H_1 (x) M, C = subdiag(1), D = diag(1/2, 1, ..., 1, 1/2).

Vector layout: every block (state, control, adjoint) is an array of shape
(n_xi, n_int) -- row j holds the coefficients of psi_j on the interior nodes,
i.e. the column-major vec of the paper's matricized V-bar -- and time-dependent
blocks have a leading n_t axis.  Flattening in C order gives the paper's vec.

Readings (listed with the rest of the readings in the design notes):
  * y_d is the nodal interpolant of the target on all nodes and enters as
    (M_full y_d) restricted to interior rows in chaos column 0 (the exact
    gradient of 1/2 (y - y_d)^T M (y - y_d) with y = 0 on the boundary);
  * g = 0 (homogeneous Dirichlet); for a nonzero initial state the first
    constraint block is d_1 = -M y_0, the sign that backward Euler gives for
    the third block row -A_t y + tau N u = d;
  * the KKT blocks use A_l (not A-tilde) in eq. (stoch-system-m);
  * the time grid is t_k = k tau, k = 1..n_t, tau = T / n_t, and D applies to
    those n_t unknown states as printed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import basis, fem


@dataclass
class Problem:
    """Data of eq. (problem-stoch)/(pde-stoch) (steady, n_t <= 1) or of the
    time-dependent problem (n_t >= 2), with g = 0."""
    n: int
    M: int
    P: int
    sigma: float
    beta: float
    y_target: np.ndarray            # (n+1)^2, or (n_t, (n+1)^2) when n_t >= 2
    gamma: float = 0.0
    n_t: int = 1
    T: float = 1.0
    kappa: np.ndarray | None = None  # (M+1, n, n) per-element modes; None = cosine field
    y0: np.ndarray | None = None     # (n+1)^2 initial state (time-dependent only)
    field: str = "affine"            # "affine": Legendre chaos, sigma-scaled cosine (or kappa) modes;
                                     # "lognormal": Hermite chaos, log-normal field of Section 5
    corr: float = 1.0                # log-normal: correlation length on [-1, 1]^2

    @property
    def steady(self) -> bool:
        return self.n_t <= 1

    @property
    def tau(self) -> float:
        return self.T / self.n_t


@dataclass
class SG:
    """Assembled stochastic-Galerkin pieces of one problem."""
    prob: Problem
    alpha: np.ndarray                    # multi-indices (n_xi, M)
    offsets: np.ndarray                  # degree level offsets (P+2,)
    G: list                              # dense triple-product matrices H_l, l = 0..n_terms-1
    K: list                              # interior stiffness matrices A_l of the coefficient terms
    Mi: sp.csr_matrix                    # interior mass matrix
    Mfull: sp.csr_matrix                 # full-grid mass matrix
    kappa: np.ndarray                    # (n_terms, n, n): M+1 (affine) or n_A (log-normal)
    _cache: dict = field(default_factory=dict)

    @property
    def n_xi(self) -> int:
        return self.alpha.shape[0]

    @property
    def n_int(self) -> int:
        return (self.prob.n - 1) ** 2


def setup(prob: Problem) -> SG:
    """Build the basis, triple products and per-mode FE matrices (Section 2.1)."""
    n, M, P = prob.n, prob.M, prob.P
    alpha = basis.multi_indices(M, P)
    offsets = basis.level_offsets(M, P)
    if prob.field == "lognormal":
        from . import hermite
        G = hermite.h_matrices(M, P)
        kappa = hermite.lognormal_modes(n, M, P, prob.sigma, prob.corr)
    else:
        G = basis.triple_product_matrices(M, P)
        kappa = prob.kappa if prob.kappa is not None else fem.cosine_modes(n, M, prob.sigma)
    K = [fem.restrict(fem.assemble_full(n, kappa[k], "stiffness"), n) for k in range(len(G))]
    Mfull = fem.assemble_full(n, 1.0, "mass")
    Mi = fem.restrict(Mfull, n)
    return SG(prob, alpha, offsets, G, K, Mi, Mfull, np.asarray(kappa, dtype=np.float64))


# ----------------------------------------------------------------------------
# Matricized applies (eq. mat-vec / eq. Zv)
# ----------------------------------------------------------------------------

def operator_apply(sg: SG, X: np.ndarray) -> np.ndarray:
    """Y = sum_k K_k X G_k in the (n_xi, n_int) layout (eq. Zv with A_l).

    With rows of X holding the chaos columns, X_mat = X^T and
    (K X_mat G)^T = G^T X K^T = G X K (G, K symmetric)."""
    Y = np.zeros_like(X)
    for Gk, Kk in zip(sg.G, sg.K):
        Y += (Kk @ (Gk.T @ X).T).T
    return Y


def mass_apply(sg: SG, X: np.ndarray) -> np.ndarray:
    """Apply the interior mass matrix to every chaos row."""
    return (sg.Mi @ X.T).T


def h_gamma(sg: SG) -> np.ndarray:
    """Diagonal of H^gamma = H_1 + gamma H^sigma (Section 2.1)."""
    d = np.full(sg.n_xi, 1.0 + sg.prob.gamma)
    d[0] = 1.0
    return d


# ----------------------------------------------------------------------------
# Explicit Kronecker matrices
# ----------------------------------------------------------------------------

def A_kron(sg: SG) -> sp.csr_matrix:
    """A = sum_l H_l (x) A_l (Section 2.1)."""
    if "A" not in sg._cache:
        A = None
        for Gk, Kk in zip(sg.G, sg.K):
            term = sp.kron(sp.csr_matrix(Gk), Kk, format="csr")
            A = term if A is None else A + term
        sg._cache["A"] = A.tocsr()
    return sg._cache["A"]


def Mcal(sg: SG) -> sp.csr_matrix:
    """M-cal = H_1 (x) M (eq. def-Mcal)."""
    return sp.kron(sp.identity(sg.n_xi), sg.Mi, format="csr")


def Mgamma(sg: SG) -> sp.csr_matrix:
    """M_gamma = H^gamma (x) M."""
    return sp.kron(sp.diags(h_gamma(sg)), sg.Mi, format="csr")


def kkt_steady(sg: SG) -> sp.csr_matrix:
    """Steady KKT matrix of eq. (stoch-system)."""
    b = sg.prob.beta
    A = A_kron(sg)
    Mc = Mcal(sg)
    return sp.bmat([[Mgamma(sg), None, -A.T],
                    [None, b * Mc, Mc.T],
                    [-A, Mc, None]], format="csc")


def L_cal(sg: SG) -> sp.csr_matrix:
    """L = H_1 (x) (M + tau A_1) + tau sum_{l>=2} H_l (x) A_l (eq. K_t for stochastic)."""
    return (Mcal(sg) + sg.prob.tau * A_kron(sg)).tocsr()


def time_matrices(sg: SG):
    """A_t, N, C, D of eq. (K_t for stochastic) and eq. (CD)."""
    nt = sg.prob.n_t
    C = sp.diags(np.ones(nt - 1), -1, shape=(nt, nt), format="csr")
    D = np.ones(nt)
    D[0] = 0.5
    D[-1] = 0.5
    Mc = Mcal(sg)
    At = sp.kron(sp.identity(nt), L_cal(sg)) - sp.kron(C, Mc)
    N = sp.kron(sp.identity(nt), Mc)
    return At.tocsr(), N.tocsr(), C, D


def kkt_time(sg: SG) -> sp.csr_matrix:
    """Time-dependent KKT matrix of eq. (KKT:stoch-time-dependent)."""
    tau, b = sg.prob.tau, sg.prob.beta
    At, N, C, D = time_matrices(sg)
    Dg = sp.kron(sp.diags(D), Mgamma(sg))
    Dm = sp.kron(sp.diags(D), Mcal(sg))
    return sp.bmat([[tau * Dg, None, -At.T],
                    [None, b * tau * Dm, tau * N.T],
                    [-At, tau * N, None]], format="csc")


def kkt_matrix(sg: SG) -> sp.csc_matrix:
    return kkt_steady(sg) if sg.prob.steady else kkt_time(sg)


# ----------------------------------------------------------------------------
# Right-hand sides
# ----------------------------------------------------------------------------

def _target_load(sg: SG, yt_full: np.ndarray) -> np.ndarray:
    """(M_full y_d) on the interior rows (reading of the discrete target term)."""
    n = sg.prob.n
    return (sg.Mfull @ np.asarray(yt_full, dtype=np.float64))[fem.interior_index(n)]


def rhs(sg: SG) -> np.ndarray:
    """KKT right-hand side as a flat vector [b_y; b_u; b_lambda]."""
    p = sg.prob
    nx, ni = sg.n_xi, sg.n_int
    if p.steady:
        by = np.zeros((nx, ni))
        by[0] = _target_load(sg, np.reshape(p.y_target, -1))
        return np.concatenate([by.ravel(), np.zeros(nx * ni), np.zeros(nx * ni)])
    nt, tau = p.n_t, p.tau
    D = np.ones(nt)
    D[0] = D[-1] = 0.5
    yt = np.reshape(p.y_target, (nt, -1))
    by = np.zeros((nt, nx, ni))
    for t in range(nt):
        by[t, 0] = tau * D[t] * _target_load(sg, yt[t])
    bl = np.zeros((nt, nx, ni))
    if p.y0 is not None:
        y0i = fem.extract(np.asarray(p.y0, dtype=np.float64), p.n)
        bl[0, 0] = -(sg.Mi @ y0i)
    return np.concatenate([by.ravel(), np.zeros(nt * nx * ni), bl.ravel()])


def block_shape(sg: SG):
    p = sg.prob
    return (sg.n_xi, sg.n_int) if p.steady else (p.n_t, sg.n_xi, sg.n_int)


def split(sg: SG, x: np.ndarray):
    """Flat KKT vector -> (Y, U, Lambda) arrays in the block layout."""
    shp = block_shape(sg)
    m = int(np.prod(shp))
    return x[:m].reshape(shp), x[m:2 * m].reshape(shp), x[2 * m:].reshape(shp)


# ----------------------------------------------------------------------------
# Solve
# ----------------------------------------------------------------------------

def _nested_dissection(nx: int, ny: int, x0: int = 0, y0: int = 0) -> list:
    """Nested-dissection order of an nx x ny block of interior nodes (a fill-
    reducing ordering for the sparse factorisation; any order gives the same
    solution)."""
    if nx * ny <= 4:
        return [(x0 + i, y0 + j) for j in range(ny) for i in range(nx)]
    if nx >= ny:
        m = nx // 2
        return (_nested_dissection(m, ny, x0, y0) + _nested_dissection(nx - m - 1, ny, x0 + m + 1, y0)
                + [(x0 + m, y0 + j) for j in range(ny)])
    m = ny // 2
    return (_nested_dissection(nx, m, x0, y0) + _nested_dissection(nx, ny - m - 1, x0, y0 + m + 1)
            + [(x0 + i, y0 + m) for i in range(nx)])


def _reduced_system(sg: SG, b: np.ndarray):
    """Eliminate the control block exactly.

    Steady: the second block row gives u = (M^{-1} b_u - lambda)/beta, leaving
    the symmetric quasi-definite system
        [[M_gamma, -A], [-A, -M/beta]] [y; lambda] = [b_y; b_lambda - b_u/beta].
    Time-dependent: u = (D (x) M)^{-1} b_u/(beta tau) - (D^{-1} (x) I) lambda/beta and
        [[tau D (x) M_gamma, -A_t^T], [-A_t, -(tau/beta) D^{-1} (x) M]] [y; lambda]
      = [b_y; b_lambda - (D^{-1} (x) I) b_u/beta]."""
    p = sg.prob
    m = b.size // 3
    by, bu, bl = b[:m], b[m:2 * m], b[2 * m:]
    Mlu = spla.splu(sg.Mi.tocsc())
    ni = sg.n_int

    def minv(v):
        V = v.reshape(-1, ni)
        return np.stack([Mlu.solve(row) for row in V]).reshape(-1)

    if p.steady:
        R = sp.bmat([[Mgamma(sg), -A_kron(sg).T], [-A_kron(sg), -Mcal(sg) / p.beta]], format="csc")
        rb = np.concatenate([by, bl - bu / p.beta])

        def back(yl):
            lam = yl[m:]
            return np.concatenate([yl[:m], (minv(bu) - lam) / p.beta, lam])
        return R, rb, back
    tau = p.tau
    At, N, C, D = time_matrices(sg)
    dinv = np.repeat(1.0 / D, sg.n_xi * ni)
    R = sp.bmat([[tau * sp.kron(sp.diags(D), Mgamma(sg)), -At.T],
                 [-At, -(tau / p.beta) * sp.kron(sp.diags(1.0 / D), Mcal(sg))]], format="csc")
    rb = np.concatenate([by, bl - dinv * bu / p.beta])

    def back(yl):
        lam = yl[m:]
        u = dinv * minv(bu) / (p.beta * tau) - dinv * lam / p.beta
        return np.concatenate([yl[:m], u, lam])
    return R, rb, back


def _backward_error(K, x, b) -> float:
    """Normwise backward error ||b - K x||_inf / (||K||_inf ||x||_inf + ||b||_inf)."""
    r = b - K @ x
    knorm = abs(K).sum(axis=1).max()
    return float(np.max(np.abs(r)) / (knorm * np.max(np.abs(x)) + np.max(np.abs(b))))


def solve_direct(sg: SG, b: np.ndarray | None = None, check: float = 1e-15, max_refine: int = 4):
    """Exact discrete solution of the KKT system (the method's fixed point).

    The control block is eliminated exactly (``_reduced_system``), the
    quasi-definite remainder is factorised by sparse LU in a nested-dissection
    order of the spatial nodes, and the result is refined against the full KKT
    matrix until its normwise backward error is <= `check` (raises otherwise).
    The backward error, not the relative residual, is the attainable target:
    for small beta ||K|| ||x|| exceeds ||b|| by orders of magnitude."""
    K = kkt_matrix(sg)
    if b is None:
        b = rhs(sg)
    R, rb, back = _reduced_system(sg, b)
    n1 = sg.prob.n - 1
    ni = sg.n_int
    nblk = R.shape[0] // ni
    nodes = _nested_dissection(n1, n1)
    node_perm = np.array([iy * n1 + ix for ix, iy in nodes])
    perm = (np.arange(nblk)[None, :] * ni + node_perm[:, None]).reshape(-1)
    Rp = R[perm][:, perm].tocsc()
    lu = spla.splu(Rp, permc_spec="NATURAL", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))

    def reduced_solve(rhs_vec):
        z = np.empty_like(rhs_vec)
        z[perm] = lu.solve(rhs_vec[perm])
        return z

    x = back(reduced_solve(rb))
    eta = _backward_error(K, x, b)
    for _ in range(max_refine):
        if eta <= check:
            break
        _, rr, back_r = _reduced_system(sg, b - K @ x)
        x = x + back_r(reduced_solve(rr))
        eta = _backward_error(K, x, b)
    if eta > check:
        raise RuntimeError(f"direct KKT solve backward error {eta:.3e} above {check:.1e}")
    return x


def kkt_apply(sg: SG, x: np.ndarray) -> np.ndarray:
    """Explicit KKT matrix times a flat vector."""
    return kkt_matrix(sg) @ x


def kkt_apply_matricized(sg: SG, x: np.ndarray) -> np.ndarray:
    """KKT matrix times a flat vector in the matricized form of
    eq. (stoch-system-m) (steady) and of the time-dependent blocks, without
    forming any Kronecker product (for sizes where the explicit matrix is too
    large).  Uses A_l in all three block rows."""
    p = sg.prob
    Y, U, L = split(sg, x)
    hg = h_gamma(sg)[:, None]
    if p.steady:
        RY = hg * mass_apply(sg, Y) - operator_apply(sg, L)
        RU = p.beta * mass_apply(sg, U) + mass_apply(sg, L)
        RL = -operator_apply(sg, Y) + mass_apply(sg, U)
        return np.concatenate([RY.ravel(), RU.ravel(), RL.ravel()])
    nt, tau = p.n_t, p.tau
    D = np.ones(nt)
    D[0] = D[-1] = 0.5
    RY, RU, RL = np.empty_like(Y), np.empty_like(U), np.empty_like(L)
    for t in range(nt):
        ML = mass_apply(sg, L[t])
        MY = mass_apply(sg, Y[t])
        MU = mass_apply(sg, U[t])
        # (A_t^T lambda)_t = L lambda_t - M lambda_{t+1};  (A_t y)_t = L y_t - M y_{t-1}
        AtL = ML + tau * operator_apply(sg, L[t]) - (mass_apply(sg, L[t + 1]) if t + 1 < nt else 0.0)
        AtY = MY + tau * operator_apply(sg, Y[t]) - (mass_apply(sg, Y[t - 1]) if t > 0 else 0.0)
        RY[t] = tau * D[t] * hg * MY - AtL
        RU[t] = p.beta * tau * D[t] * MU + tau * ML
        RL[t] = -AtY + tau * MU
    return np.concatenate([RY.ravel(), RU.ravel(), RL.ravel()])


def moments(Y: np.ndarray):
    """Mean and variance fields of an SG expansion (orthonormal basis):
    E[y] = Y_0 and Var[y] = sum_{j>=1} Y_j^2 (Section 2.1, H^sigma)."""
    return Y[..., 0, :], np.sum(Y[..., 1:, :] ** 2, axis=-2)


def kkt_rows(sg: SG, x: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """Selected entries (K x)[rows] of the KKT matrix times a flat vector,
    from the explicit rows of the Kronecker blocks (Section 2.1, eq.
    (stoch-system); Section 3, eq. (KKT:stoch-time-dependent)), for sizes where
    neither the matrix nor a full apply is wanted.

    A flat row index addresses [block][t][j][i] (block 0 state, 1 control,
    2 adjoint; t only when time-dependent; chaos j; interior node i).  Row
    (j, i) of A = sum_k H_k (x) A_k applied to a block X is
    sum_k sum_j' h_{k j j'} (A_k[i, :] . X_j'), computed from the sampled
    spatial rows of every A_k and the matrices H_k."""
    p = sg.prob
    rows = np.asarray(rows, dtype=np.int64)
    Y, U, L = split(sg, x)
    if p.steady:                          # one time step, so both forms share the code below
        Y, U, L = Y[None], U[None], L[None]
    nt = Y.shape[0]
    nx, ni = sg.n_xi, sg.n_int
    blk = nt * nx * ni
    b = rows // blk
    rem = rows % blk
    i = rem % ni
    j = (rem // ni) % nx
    t = rem // (nx * ni)
    hg = h_gamma(sg)
    tau = 1.0 if p.steady else p.tau
    D = np.ones(nt)
    if not p.steady:
        D[0] = D[-1] = 0.5
    out = np.empty(rows.size)
    for blkid in range(3):
        s = np.flatnonzero(b == blkid)
        if s.size == 0:
            continue
        jj, ts = j[s], t[s]
        Ms = sg.Mi.tocsr()[i[s]]                     # sampled spatial rows of M and of every A_k
        Ks = [Kk.tocsr()[i[s]] for Kk in sg.K]

        def mass(F, dt=0):
            """(M F_{t+dt, j})_i, zero where t+dt leaves [0, n_t)."""
            tn = ts + dt
            ok = np.flatnonzero((tn >= 0) & (tn < nt))
            v = np.zeros(s.size)
            v[ok] = np.asarray(Ms[ok].multiply(F[tn[ok], jj[ok]]).sum(axis=1)).ravel()
            return v

        def stiff(F):
            """(A F_t)_{j,i} = sum_k sum_j' h_{k j j'} (A_k[i,:] . F_{t,j'})."""
            acc = np.zeros(s.size)
            for Gk, Kk in zip(sg.G, Ks):
                T = np.empty((s.size, nx))
                for tq in np.unique(ts):
                    m = np.flatnonzero(ts == tq)
                    T[m] = np.asarray(Kk[m] @ F[tq].T)
                acc += np.einsum("sq,qs->s", T, Gk[:, jj])
            return acc

        Dt = D[ts]
        if blkid == 0:
            # tau D_t M_gamma y_t - (A_t^T lambda)_t, (A_t^T lambda)_t = L lambda_t - M lambda_{t+1};
            # steady: M_gamma y - A lambda
            trans = mass(L) + tau * stiff(L) - mass(L, +1) if not p.steady else stiff(L)
            out[s] = tau * Dt * hg[jj] * mass(Y) - trans
        elif blkid == 1:
            out[s] = p.beta * tau * Dt * mass(U) + tau * mass(L)
        else:
            # -(A_t y)_t + tau M u_t, (A_t y)_t = L y_t - M y_{t-1}; steady: -A y + M u
            fwd = mass(Y) + tau * stiff(Y) - mass(Y, -1) if not p.steady else stiff(Y)
            out[s] = -fwd + tau * mass(U)
    return out
