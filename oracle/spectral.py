"""Numerical check of the spectral bounds of Section 4 on tiny problems.

Oracle (test infrastructure only).  Dense matrices, written from the
definitions in Sections 3-4:
  * eq. (K_t for stochastic): A_t = I (x) L - C (x) Mcal,  N = I (x) H_1 (x) M,
    L = H_1 (x) (M + tau A_1) + tau sum_{l>=2} H_l (x) A_l;  C = subdiagonal of
    ones, D = diag(1/2, 1, .., 1, 1/2) (eq. CD);
  * the exact Schur complement of the time-dependent KKT matrix,
    (1/tau) A_t W A_t^T + (tau/beta) N (D (x) Mcal)^{-1} N^T with
    W = (D (x) M_gamma)^{-1} (eq. time-exact-pre, read with tau/beta: R16);
  * S-bar = (1/tau) Z-bar W Z-bar^T, Z-bar = A_t + tau s N, s = sqrt((1+gamma)/beta)
    (eq. S hat);  Z-tilde = tau s N + I (x) L (eq. Z hat approx) and
    S-tilde = (1/tau) Z-tilde W Z-tilde (eq. S_tilde with the 1/tau of S-bar);
  * truncation: Z-tilde_r keeps H_l for l <= r (eq. S_r), S-tilde_r likewise;
  * hGS: Z_hGS = (X_1 + X_r) X_1^{-1} (X_1 + X_r^T), X_1 = I (x) H_1 (x) A-hat_1,
    X_r = I (x) sum_{l=2}^r L_l (x) A-hat_l with H_l = L_l + L_l^T split by
    degree level (L_l maps level d to level d+1), A-hat_1 = (1 + tau s) M + tau A_1,
    A-hat_l = tau A_l (l >= 2).

Index convention: l = 1 is the mean (chaos matrix G_0 = I, stiffness K_0),
l = k+1 is mode k (G_k, K_k).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import kkt


def _gen_eig(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Eigenvalues of B^{-1} A for symmetric A and SPD B (ascending)."""
    return sla.eigh(0.5 * (A + A.T), 0.5 * (B + B.T), eigvals_only=True)


def _sym_sqrt_inv(B: np.ndarray) -> np.ndarray:
    w, V = np.linalg.eigh(0.5 * (B + B.T))
    return (V / np.sqrt(w)) @ V.T


class TimeOperators:
    """Dense operators of Section 4 for one (small) problem.  A steady problem
    is the case n_t = 1 with tau = 1, D = I, C = 0 and no backward-Euler mass
    term in L (the steady-state remark of Section 4): then S-exact =
    A M_gamma^{-1} A + M / beta, S-bar = S-tilde = Z M_gamma^{-1} Z and
    A-hat_1 = A-tilde_1 = A_1 + s M."""

    def __init__(self, sg: kkt.SG):
        p = sg.prob
        self.sg = sg
        nt, tau = (1, 1.0) if p.steady else (p.n_t, p.tau)
        self.tau, self.nt = tau, nt
        self.s = np.sqrt((1.0 + p.gamma) / p.beta)
        M = sg.Mi.toarray()
        self.M = M
        nxi = sg.n_xi
        self.H = [np.asarray(G) for G in sg.G]                 # H_1 = G_0 = I, H_{k+1} = G_k
        self.A = [K.toarray() for K in sg.K]                  # A_1 = K_0, A_{k+1} = K_k
        hg = kkt.h_gamma(sg)
        self.Mcal = np.kron(np.eye(nxi), M)
        self.Mgam = np.kron(np.diag(hg), M)
        self.C = np.diag(np.ones(nt - 1), -1)
        self.D = np.eye(nt)
        if not p.steady:
            self.D[0, 0] = self.D[-1, -1] = 0.5
        m_t = 0.0 if p.steady else 1.0                         # backward-Euler mass
        self.L = np.kron(self.H[0], m_t * M + tau * self.A[0])
        for Hl, Al in zip(self.H[1:], self.A[1:]):
            self.L += tau * np.kron(Hl, Al)
        I = np.eye(nt)
        self.N = np.kron(I, self.Mcal)
        self.At = np.kron(I, self.L) - np.kron(self.C, self.Mcal)
        self.W = np.linalg.inv(np.kron(self.D, self.Mgam))
        self.Ahat = [(m_t + tau * self.s) * M + tau * self.A[0]] + [tau * Al for Al in self.A[1:]]

    def Zr(self, r: int) -> np.ndarray:
        """Z-tilde_r (r = n_A: Z-tilde)."""
        inner = np.kron(self.H[0], self.Ahat[0])
        for l in range(1, min(r, len(self.H))):
            inner = inner + np.kron(self.H[l], self.Ahat[l])
        return np.kron(np.eye(self.nt), inner)

    def S_of(self, Z: np.ndarray) -> np.ndarray:
        return (Z @ self.W @ Z.T) / self.tau

    def S_exact(self) -> np.ndarray:
        Winv_u = np.linalg.inv(np.kron(self.D, self.Mcal))
        return (self.At @ self.W @ self.At.T) / self.tau + (self.tau / self.sg.prob.beta) * (self.N @ Winv_u @ self.N.T)

    def Zbar(self) -> np.ndarray:
        return self.At + self.tau * self.s * self.N

    def level_lower(self, Hl: np.ndarray) -> np.ndarray:
        """L_l: the part of H_l mapping a degree level d to level d+1."""
        off = self.sg.offsets
        lev = np.zeros(Hl.shape[0], dtype=int)
        for d in range(len(off) - 1):
            lev[int(off[d]):int(off[d + 1])] = d
        return np.where(lev[:, None] > lev[None, :], Hl, 0.0)

    def Z_hgs(self, r: int) -> np.ndarray:
        I = np.eye(self.nt)
        X1 = np.kron(I, np.kron(self.H[0], self.Ahat[0]))
        Xr = np.zeros_like(X1)
        for l in range(1, min(r, len(self.H))):
            Xr += np.kron(I, np.kron(self.level_lower(self.H[l]), self.Ahat[l]))
        return (X1 + Xr) @ np.linalg.solve(X1, X1 + Xr.T)

    # --- the quantities of the bounds -------------------------------------
    def kappa_At(self) -> float:
        sv = np.linalg.svd(self.At, compute_uv=False)
        return float(sv[0] / sv[-1])

    def mu(self) -> float:
        """mu of eq. (mucond): tau s sigma_min(N W^1/2) / ||(I (x) L) W^1/2||_2."""
        Wh = sla.sqrtm(self.W).real
        smin = np.linalg.svd(self.N @ Wh, compute_uv=False)[-1]
        nrm = np.linalg.norm(np.kron(np.eye(self.nt), self.L) @ Wh, 2)
        return float(self.tau * self.s * smin / nrm)

    def theta(self) -> float:
        """theta = sup ||W^1/2 (C (x) Mcal)^T v|| / ||W^1/2 Z-tilde^T v||."""
        CM = np.kron(self.C, self.Mcal)
        Zt = self.Zr(len(self.H))
        num = CM @ self.W @ CM.T
        den = Zt @ self.W @ Zt.T
        return float(np.sqrt(max(_gen_eig(num, den).max(), 0.0)))

    def theta_bound(self, mu: float) -> float:
        g = self.sg.prob.gamma
        wM = np.linalg.eigvalsh(self.M)
        kap_half = np.sqrt(wM.max() / wM.min())
        return float(np.sqrt(2.0 * self.sg.prob.beta) / (np.sqrt(1.0 + g) * (1.0 - 1.0 / mu) * self.tau) * kap_half)

    def delta_r(self, r: int) -> float:
        nu = np.linalg.eigvalsh(self.Ahat[0]).min()
        tail = sum(np.linalg.norm(self.H[l], 2) * np.linalg.norm(self.Ahat[l], 2) for l in range(r, len(self.H)))
        return float(tail / nu)

    def Delta_r(self, r: int):
        """(Delta_r, rho_l list) of Lemma lmin-sigY."""
        Ah = _sym_sqrt_inv(self.Ahat[0])
        rho = [np.linalg.norm(Ah @ self.Ahat[l] @ Ah, 2) for l in range(1, len(self.H))]
        D = sum(np.linalg.norm(self.H[l], 2) * rho[l - 1] for l in range(1, min(r, len(self.H))))
        return float(D), rho

    def Y(self, r: int) -> np.ndarray:
        I = np.eye(self.nt)
        X1h = _sym_sqrt_inv(np.kron(I, np.kron(self.H[0], self.Ahat[0])))
        Xr = np.zeros((X1h.shape[0], X1h.shape[0]))
        for l in range(1, min(r, len(self.H))):
            Xr += np.kron(I, np.kron(self.level_lower(self.H[l]), self.Ahat[l]))
        return X1h @ Xr @ X1h


def eig_ratio(A: np.ndarray, B: np.ndarray):
    """(min, max) of the eigenvalues of B^{-1} A (A symmetric, B SPD)."""
    e = _gen_eig(A, B)
    return float(e.min()), float(e.max())


def eig_ratio_general(A: np.ndarray, B: np.ndarray):
    """(min, max) of the real parts of the eigenvalues of B^{-1} A (general A)."""
    e = np.linalg.eigvals(np.linalg.solve(B, A))
    return float(e.real.min()), float(e.real.max())
