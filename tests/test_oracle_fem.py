"""Pins of the oracle's Q1 finite elements against closed forms."""
import math

import numpy as np
import pytest

import sg_inputs
from oracle import fem


def test_element_matrices_closed_form():
    """Textbook bilinear element: stiffness (1/6)[4,-1,-2,-1;...] (h-independent
    in 2-D) and mass (h^2/36)[4,2,1,2;...] in counter-clockwise node order."""
    for h in (1.0, 0.25, 1 / 16):
        Ke, Me = fem.element_matrices(h)
        K_ref = np.array([[4, -1, -2, -1], [-1, 4, -1, -2], [-2, -1, 4, -1], [-1, -2, -1, 4]]) / 6.0
        M_ref = np.array([[4, 2, 1, 2], [2, 4, 2, 1], [1, 2, 4, 2], [2, 1, 2, 4]]) * h * h / 36.0
        assert np.max(np.abs(Ke - K_ref)) < 1e-15
        assert np.max(np.abs(Me - M_ref)) < 1e-15 * max(1.0, h * h)


@pytest.mark.parametrize("n", [4, 8, 16, 32])
def test_sine_mode_eigen_identity(n):
    """v = sin(pi x) sin(pi y) on the interior satisfies K v = mu_h M v and
    M v = m1^2 v with k1 = (2/h)(1 - cos pi h), m1 = (h/3)(2 + cos pi h),
    mu_h = 2 k1 / m1 (1-D P1 eigenvalues of the tensor-product Q1 matrices)."""
    h = 1.0 / n
    K = fem.restrict(fem.assemble_full(n, 1.0, "stiffness"), n)
    M = fem.restrict(fem.assemble_full(n, 1.0, "mass"), n)
    v = fem.extract(sg_inputs.unit_sine(n), n)
    k1 = (2.0 / h) * (1.0 - math.cos(math.pi * h))
    m1 = (h / 3.0) * (2.0 + math.cos(math.pi * h))
    assert np.max(np.abs(M @ v - m1 * m1 * v)) < 1e-15
    assert np.max(np.abs(K @ v - (2.0 * k1 / m1) * (M @ v))) < 1e-13


@pytest.mark.parametrize("n", [4, 16])
def test_mass_diagonal_and_total(n):
    h = 1.0 / n
    Mf = fem.assemble_full(n, 1.0, "mass")
    assert abs(Mf.sum() - 1.0) < 1e-14                       # integral of 1 over the square
    Mi = fem.restrict(Mf, n)
    assert np.allclose(Mi.diagonal(), 4 * h * h / 9, rtol=0, atol=1e-16)


def test_variable_coefficient_energy():
    """For the linear function v = x, grad v = (1, 0) and
    v^T K_c v = sum_e c_e |e| = h^2 sum_e c_e (full grid, no elimination)."""
    n = 8
    rng = np.random.default_rng(3)
    c = rng.uniform(0.5, 2.0, size=(n, n))
    K = fem.assemble_full(n, c, "stiffness")
    x, y = sg_inputs.node_coords(n)
    assert abs(x @ (K @ x) - c.sum() / n ** 2) < 1e-13
    assert abs(y @ (K @ y) - c.sum() / n ** 2) < 1e-13
    ones = np.ones((n + 1) ** 2)
    assert np.max(np.abs(K @ ones)) < 1e-13                   # constants in the kernel


def test_cosine_modes_and_coercivity():
    n, M, s = 16, 4, 0.2
    kap = fem.cosine_modes(n, M, s)
    xc, yc = fem.centroids(n)
    assert np.all(kap[0] == 1.0)
    k = 3
    assert abs(kap[k][2, 5] - s / 9 * math.cos(3 * math.pi * xc[2, 5]) * math.cos(3 * math.pi * yc[2, 5]) / math.sqrt(3)) < 1e-16
    # a = kappa_0 + sum_k kappa_k psi_{e_k}, psi_{e_k} = sqrt(3) xi_k in [-sqrt(3), sqrt(3)]
    amin = kap[0] - math.sqrt(3.0) * np.abs(kap[1:]).sum(axis=0)
    assert amin.min() > 1.0 - s * sum(j ** -2.0 for j in range(1, M + 1)) - 1e-14


def test_embed_extract_roundtrip():
    n = 8
    v = np.arange((n - 1) ** 2, dtype=float)
    full = fem.embed(v, n)
    assert full.shape == ((n + 1) ** 2,)
    assert np.all(full.reshape(n + 1, n + 1)[0] == 0) and np.all(full.reshape(n + 1, n + 1)[:, -1] == 0)
    assert np.array_equal(fem.extract(full, n), v)
