"""Q1 finite elements on the unit square.

Oracle (test infrastructure only).

Paper passages followed
  * Section 2.1, eq. (gPC-A): (A_l)_{ab} = int kappa_l grad phi_a . grad phi_b,
    all A_l share one sparsity pattern; mass M_{ab} = int phi_a phi_b.
  * Section 5: Q1 approximation on a uniform square mesh.

Readings (the paper is silent; it uses a third-party toolbox):
  * domain [0,1]^2 with n x n square elements, h = 1/n; node (ix, iy) has flat
    index iy*(n+1)+ix; element (ex, ey) has flat index ey*n+ex;
  * each coefficient mode kappa_l is taken constant per element, equal to its
    value at the element centroid, so element matrices are exact;
  * homogeneous Dirichlet data are imposed by eliminating the boundary nodes:
    the algebraic unknowns are the (n-1)^2 interior nodes in iy-major order.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

# Local node order on an element: (0,0), (1,0), (1,1), (0,1) (counter-clockwise).
_LOCAL = np.array([[0, 0], [1, 0], [1, 1], [0, 1]])


def _shape(xr, yr):
    """Bilinear shape functions and reference gradients at (xr, yr) in [0,1]^2."""
    N = np.array([(1 - xr) * (1 - yr), xr * (1 - yr), xr * yr, (1 - xr) * yr])
    dNx = np.array([-(1 - yr), (1 - yr), yr, -yr])
    dNy = np.array([-(1 - xr), -xr, xr, (1 - xr)])
    return N, dNx, dNy


def element_matrices(h: float):
    """Unit-coefficient Q1 element stiffness and mass on an h x h square.

    Computed by 2x2 Gauss-Legendre quadrature of the bilinear shape functions
    (exact for these bi-quadratic integrands).  Returns (Ke, Me), 4x4 each."""
    g = np.array([0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)])
    Ke = np.zeros((4, 4))
    Me = np.zeros((4, 4))
    for xr in g:
        for yr in g:
            N, dNx, dNy = _shape(xr, yr)
            w = 0.25 * h * h                      # weight * Jacobian (area h^2)
            # physical gradients: d/dx = (1/h) d/dxr
            gx, gy = dNx / h, dNy / h
            Ke += w * (np.outer(gx, gx) + np.outer(gy, gy))
            Me += w * np.outer(N, N)
    return Ke, Me


def element_nodes(n: int) -> np.ndarray:
    """Global node indices of each element's 4 local nodes, shape (n*n, 4)."""
    ex, ey = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ex = ex.reshape(-1)
    ey = ey.reshape(-1)
    cols = []
    for dx, dy in _LOCAL:
        cols.append((ey + dy) * (n + 1) + (ex + dx))
    return np.stack(cols, axis=1)


def assemble_full(n: int, coeff: np.ndarray | float, which: str) -> sp.csr_matrix:
    """Assemble the full-grid ((n+1)^2 square) stiffness or mass matrix.

    `coeff` is a per-element array (n, n) indexed [ey, ex] (or a scalar);
    `which` is "stiffness" or "mass" (mass ignores coeff unless given)."""
    h = 1.0 / n
    Ke, Me = element_matrices(h)
    E = Ke if which == "stiffness" else Me
    c = np.broadcast_to(np.asarray(coeff, dtype=np.float64), (n, n)).reshape(-1)
    nodes = element_nodes(n)
    rows = np.repeat(nodes, 4, axis=1).reshape(-1)
    cols = np.tile(nodes, (1, 4)).reshape(-1)
    vals = (c[:, None] * E.reshape(1, 16)).reshape(-1)
    N = (n + 1) ** 2
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def interior_index(n: int) -> np.ndarray:
    """Flat full-grid indices of the interior nodes, iy-major."""
    i = np.arange(1, n)
    iy, ix = np.meshgrid(i, i, indexing="ij")
    return (iy * (n + 1) + ix).reshape(-1)


def restrict(A: sp.spmatrix, n: int) -> sp.csr_matrix:
    """Interior rows and columns of a full-grid matrix (Dirichlet elimination)."""
    I = interior_index(n)
    return sp.csr_matrix(A.tocsr()[I][:, I])


def centroids(n: int):
    """Element centroid coordinates, arrays (n, n) indexed [ey, ex]."""
    t = (np.arange(n) + 0.5) / n
    yc, xc = np.meshgrid(t, t, indexing="ij")
    return xc, yc


def cosine_modes(n: int, M: int, sigma: float) -> np.ndarray:
    """Per-element coefficient modes of a(x, xi) = 1 + sigma sum_k k^-2
    cos(k pi x1) cos(k pi x2) xi_k, xi_k ~ U(-1,1).

    In the orthonormal Legendre basis xi_k = psi_{e_k} / sqrt(3), so the mode
    multiplying psi_{e_k} is sigma k^-2 cos cos / sqrt(3) (eq. KLE with an
    affine expansion).  Returns (M+1, n, n): index 0 is the mean (1)."""
    xc, yc = centroids(n)
    out = np.empty((M + 1, n, n))
    out[0] = 1.0
    for k in range(1, M + 1):
        out[k] = sigma * k ** -2.0 * np.cos(k * math.pi * xc) * np.cos(k * math.pi * yc) / math.sqrt(3.0)
    return out


def embed(v_int: np.ndarray, n: int) -> np.ndarray:
    """Interior vector(s) -> full-grid layout with a zero boundary ring.
    Accepts (..., (n-1)^2) and returns (..., (n+1)^2)."""
    v_int = np.asarray(v_int)
    out = np.zeros(v_int.shape[:-1] + ((n + 1) ** 2,))
    out[..., interior_index(n)] = v_int
    return out


def extract(v_full: np.ndarray, n: int) -> np.ndarray:
    """Full-grid vector(s) -> interior values (boundary ring dropped)."""
    return np.asarray(v_full)[..., interior_index(n)]
