"""Pins of the oracle's element-by-element whole-grid products (oracle/local.py).

They are checked against the assembled sparse matrices of oracle/kkt.py (an
independent route through COO assembly and Dirichlet restriction) and against
facts of the Q1 discretisation that hold at any size: the constant-coefficient
stiffness annihilates linear functions at interior nodes, the mass row sums
are h^2, and the 9-point stencils of the unit-coefficient stiffness (8/3 at the
centre, -1/3 at the eight neighbours) and mass (h^2/36 [1 4 1; 4 16 4; 1 4 1]).
"""
import numpy as np
import pytest

import sg_inputs
from oracle import basis, fem, kkt, local


def _field(n, seed=3):
    # asymmetric per-element field (breaks the x <-> y symmetry of the cosine modes)
    rng = np.random.default_rng(seed)
    return 1.0 + 0.3 * rng.uniform(-1, 1, size=(n, n))


@pytest.mark.parametrize("n", [4, 8, 16])
def test_product_matches_assembled(n):
    rng = np.random.default_rng(n)
    v = rng.uniform(-1, 1, size=(n + 1) ** 2)
    c = _field(n)
    for which, coeff in [("stiffness", c), ("stiffness", None), ("mass", None)]:
        A = fem.assemble_full(n, 1.0 if coeff is None else coeff, which)
        ref = fem.restrict(A, n) @ fem.extract(v, n)
        got = local.product(n, v, which, coeff).reshape(-1)
        assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_stencils_and_invariants():
    n = 16
    h = 1.0 / n
    xs = np.arange(n + 1) * h
    X1, X2 = np.meshgrid(xs, xs)                    # [iy, ix]
    # constant-coefficient stiffness of a linear function vanishes at interior
    # nodes whose stencil stays off the zeroed ring
    lin = (2.0 * X1 - 3.0 * X2 + 0.5).reshape(-1)
    Kl = local.product(n, lin, "stiffness", zero_ring=False)
    assert np.max(np.abs(Kl)) < 1e-12
    # mass row sums: h^2 at every interior node
    ones = np.ones((n + 1) ** 2)
    assert np.allclose(local.product(n, ones, "mass", zero_ring=False), h * h, rtol=0, atol=1e-15)
    # single-node impulses give the two 9-point stencils
    e = np.zeros((n + 1, n + 1))
    e[5, 7] = 1.0
    Ks = local.product(n, e.reshape(-1), "stiffness")
    Ms = local.product(n, e.reshape(-1), "mass")
    ks = np.full((3, 3), -1.0 / 3.0)
    ks[1, 1] = 8.0 / 3.0
    ms = h * h / 36.0 * np.array([[1, 4, 1], [4, 16, 4], [1, 4, 1]], dtype=float)
    assert np.allclose(Ks[3:6, 5:8], ks, rtol=0, atol=1e-14)
    assert np.allclose(Ms[3:6, 5:8], ms, rtol=0, atol=1e-17)
    Ks[3:6, 5:8] = 0.0
    Ms[3:6, 5:8] = 0.0
    assert not np.any(Ks) and not np.any(Ms)


@pytest.mark.parametrize("case", [(8, 2, 2, 0.3, 1e-2, 0.0), (16, 3, 2, 0.2, 1e-3, 0.5)])
def test_operator_and_kkt_residual_match_assembled(case):
    n, M, P, sigma, beta, gamma = case
    tgt = sg_inputs.gaussian_bumps(n, 4)
    prob = kkt.Problem(n=n, M=M, P=P, sigma=sigma, beta=beta, gamma=gamma, y_target=tgt)
    sg = kkt.setup(prob)
    rng = np.random.default_rng(7)
    nxi = sg.n_xi
    full = rng.uniform(-1, 1, size=(3, nxi, (n + 1) ** 2))
    # the ring of the inputs is ignored by both sides
    Y, U, L = full
    ref_op = kkt.operator_apply(sg, fem.extract(Y, n))
    got_op = local.operator(n, sg.kappa, sg.G, Y)
    assert np.max(np.abs(got_op - ref_op)) <= 1e-13 * np.max(np.abs(ref_op))
    x = np.concatenate([fem.extract(B, n).reshape(-1) for B in full])
    r_ref = kkt.rhs(sg) - kkt.kkt_matrix(sg) @ x
    ry, ru, rl, by = local.kkt_residual_steady(n, sg.kappa, sg.G, kkt.h_gamma(sg), beta, tgt, Y, U, L)
    r = np.concatenate([ry.reshape(-1), ru.reshape(-1), rl.reshape(-1)])
    assert np.max(np.abs(r - r_ref)) <= 1e-13 * np.max(np.abs(r_ref))
    assert np.allclose(by, kkt.rhs(sg)[: (n - 1) ** 2], rtol=1e-14, atol=0)


def test_operator_with_basis_tables():
    # the operator from the basis module's triple products and fem's cosine
    # modes directly (the inputs the maximum-grid GPU test uses)
    n, M, P, sigma = 8, 1, 1, 0.3
    G = basis.triple_product_matrices(M, P)
    kap = fem.cosine_modes(n, M, sigma)
    prob = kkt.Problem(n=n, M=M, P=P, sigma=sigma, beta=1e-2, y_target=sg_inputs.gaussian_bumps(n, 0))
    sg = kkt.setup(prob)
    X = np.random.default_rng(2).uniform(-1, 1, size=(sg.n_xi, (n + 1) ** 2))
    assert np.allclose(local.operator(n, kap, G, X), kkt.operator_apply(sg, fem.extract(X, n)), rtol=0, atol=1e-13)
