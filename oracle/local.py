"""Element-by-element products on the whole grid, for sizes where assembling
the sparse matrices is not wanted (n up to 4096).

Oracle (test infrastructure only).

Paper passages followed
  * Section 2.1, eq. (gPC-A): (A_l x)_a = sum_e kappa_l(e) sum_b (K_e)_{ab} x_b
    with the Q1 element stiffness K_e, and (M x)_a = sum_e sum_b (M_e)_{ab} x_b;
    the SG operator applies sum_l H_l (x) A_l (eq. mat-vec / eq. Zv).
  * Section 2.1, eq. (stoch-system): the rows of the steady KKT system,
    [H^gamma (x) M, 0, -A^T; 0, beta H_1 (x) M, H_1 (x) M; -A, H_1 (x) M, 0].

Each product is the sum over the four element positions around a node and
the four corners of that element, taken on whole-grid arrays (one shifted
slice per element corner), with the element matrices of `fem.element_matrices`
and the grid conventions of `fem` (node (ix, iy) at flat index iy (n+1) + ix,
coefficients indexed [ey, ex], local corners (0,0), (1,0), (1,1), (0,1)).
Vectors enter in the full-grid layout; their boundary ring is zeroed first
(Dirichlet elimination), except for the target load, which uses the target's
boundary values as the full mass matrix does.
"""
from __future__ import annotations

import numpy as np

from . import fem

# element position (dx, dy) relative to the node: the node is the element's
# corner (ix - ex, iy - ey)
_ELEMS = [(-1, -1), (0, -1), (-1, 0), (0, 0)]
_LOCAL = [(0, 0), (1, 0), (1, 1), (0, 1)]


def _corner_index(cx: int, cy: int) -> int:
    return _LOCAL.index((cx, cy))


def _grid(v: np.ndarray, n: int, zero_ring: bool) -> np.ndarray:
    g = np.array(np.asarray(v, dtype=np.float64).reshape(n + 1, n + 1), copy=True)
    if zero_ring:
        g[0, :] = g[-1, :] = 0.0
        g[:, 0] = g[:, -1] = 0.0
    return g


def product(n: int, v: np.ndarray, which: str, coeff=None, zero_ring: bool = True) -> np.ndarray:
    """(E_c v) at every interior node, E the stiffness or mass of coefficient
    `coeff` ((n, n) per element, [ey, ex]; None for 1).  Returns an
    (n-1, n-1) array indexed [iy-1, ix-1]."""
    Ke, Me = fem.element_matrices(1.0 / n)
    E = Ke if which == "stiffness" else Me
    g = _grid(v, n, zero_ring)
    out = np.zeros((n - 1, n - 1))
    for dx, dy in _ELEMS:
        # element (ex, ey) = (ix + dx, iy + dy) for interior nodes ix, iy = 1..n-1
        ex0, ey0 = 1 + dx, 1 + dy
        a = _corner_index(-dx, -dy)               # the node's corner in that element
        acc = np.zeros((n - 1, n - 1))
        for b, (cx, cy) in enumerate(_LOCAL):
            # corner b of element (ex, ey) is node (ex + cx, ey + cy)
            sl = g[ey0 + cy: ey0 + cy + n - 1, ex0 + cx: ex0 + cx + n - 1]
            acc += E[a, b] * sl
        if coeff is not None:
            acc *= np.asarray(coeff)[ey0: ey0 + n - 1, ex0: ex0 + n - 1]
        out += acc
    return out


def operator(n: int, kappa: np.ndarray, G: list, X: np.ndarray) -> np.ndarray:
    """sum_l H_l (x) A_l applied to the chaos columns X ((n_xi, (n+1)^2),
    full grid): row j of the result is sum_l sum_j' (H_l)_{j j'} A_l X_j'.
    Returns (n_xi, (n-1)^2) interior values, iy-major."""
    nxi = X.shape[0]
    Y = np.zeros((nxi, (n - 1) ** 2))
    for l, Hl in enumerate(G):
        AX = np.stack([product(n, X[i], "stiffness", kappa[l]).reshape(-1) for i in range(nxi)])
        Y += Hl @ AX
    return Y


def mass(n: int, X: np.ndarray) -> np.ndarray:
    """M applied to every chaos column: (n_xi, (n-1)^2) interior values."""
    return np.stack([product(n, X[i], "mass").reshape(-1) for i in range(X.shape[0])])


def kkt_residual_steady(n: int, kappa: np.ndarray, G: list, hg: np.ndarray, beta: float, y_target: np.ndarray,
                        Y: np.ndarray, U: np.ndarray, L: np.ndarray):
    """b - K x of the steady KKT system for full-grid blocks Y, U, L ((n_xi,
    (n+1)^2) each): returns (r_y, r_u, r_lambda) on the interior nodes and
    the interior right-hand side b_y of the mean column (b_u = b_lambda = 0).

    Rows: r_y = b_y - (H^gamma (x) M) y + A lambda, r_u = -beta M u - M lambda,
    r_lambda = A y - M u, with b_y = M_full y_d in the mean column."""
    AY = operator(n, kappa, G, Y)
    AL = operator(n, kappa, G, L)
    MY, MU, ML = mass(n, Y), mass(n, U), mass(n, L)
    by = product(n, y_target, "mass", zero_ring=False).reshape(-1)
    ry = -hg[:, None] * MY + AL
    ry[0] += by
    ru = -beta * MU - ML
    rl = AY - MU
    return ry, ru, rl, by
