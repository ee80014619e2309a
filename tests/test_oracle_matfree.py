"""Pins of the oracle's Q_p stiffness action (the definition the matrix-free fine operator is checked against)."""
import numpy as np
import pytest

import fixtures as F
from oracle.matfree import element_stiffness, gauss_01, stiffness_apply


def test_gauss_rule_integrates_monomials_exactly():
    for k in (2, 3, 4):
        g, w = gauss_01(k)
        for m in range(2 * k):
            assert abs(float(w @ g ** m) - 1.0 / (m + 1)) <= 1e-15


@pytest.mark.parametrize("a,b", [(1.0, 1.0), (0.5, 2.0), (3.0, 0.25)])
def test_q1_rectangle_closed_form(a, b):
    """Bilinear element on [0,a] x [0,b]: K = (b/a) M1 (x) K1 + (a/b) K1 (x) M1 with the 1D stiffness
    [[1,-1],[-1,1]] and mass [[1/3,1/6],[1/6,1/3]] (tensor order, x fastest); the unit square gives the textbook
    (1/6)[[4,-1,-1,-2], ...]."""
    corners = np.array([[0, 0], [a, 0], [0, b], [a, b]], dtype=float)
    K = element_stiffness(corners, 1)
    K1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
    M1 = np.array([[1 / 3, 1 / 6], [1 / 6, 1 / 3]])
    ref = (b / a) * np.kron(M1, K1) + (a / b) * np.kron(K1, M1)
    np.testing.assert_allclose(K, ref, rtol=0, atol=1e-14 * max(a / b, b / a))
    if a == b == 1.0:
        np.testing.assert_allclose(K, np.array([[4, -1, -1, -2], [-1, 4, -2, -1], [-1, -2, 4, -1],
                                                [-2, -1, -1, 4]]) / 6.0, atol=1e-15)


@pytest.mark.parametrize("d,N,p,jit,kap", [(2, 4, 3, 0.2, False), (2, 5, 1, 0.0, True), (3, 3, 2, 0.15, False),
                                           (3, 2, 3, 0.0, True), (2, 3, 2, 0.2, True)])
def test_matches_assembled_matrix(d, N, p, jit, kap):
    """The oracle's action equals the fixture's independently assembled Dirichlet stiffness matrix."""
    kappa = F.rng(7, F.PURPOSE_KAPPA).lognormal(0.0, 1.0, size=N ** d) if kap else None
    prob = F.structured_qp(d, N, p, jitter=jit, cfg=3, kappa=kappa)
    x = F.rng(7, F.PURPOSE_RHS).standard_normal(prob.n)
    y = stiffness_apply(prob.coords, prob.cells, p, x, kappa=kappa, constrained=prob.boundary,
                        cdiag=np.ones(prob.n))
    ref = prob.scipy() @ x
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("d,p", [(2, 3), (3, 2)])
def test_linear_energy_constants_and_symmetry(d, p):
    """No constraints: constants are in the kernel, a linear u has energy |grad u|^2 vol = |a|^2 (the unit
    domain), and the operator is symmetric."""
    N = 3
    prob = F.structured_qp(d, N, p, jitter=0.2, cfg=4, dirichlet=False)
    X = prob.coords
    one = np.ones(prob.n)
    assert np.abs(stiffness_apply(X, prob.cells, p, one)).max() <= 1e-12
    a = np.array([0.7, -1.3, 0.4][:d])
    u = X @ a + 0.25
    assert abs(float(u @ stiffness_apply(X, prob.cells, p, u)) - float(a @ a)) <= 1e-12
    g = F.rng(4, F.PURPOSE_RHS)
    v, w = g.standard_normal(prob.n), g.standard_normal(prob.n)
    lhs, rhs = v @ stiffness_apply(X, prob.cells, p, w), w @ stiffness_apply(X, prob.cells, p, v)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
