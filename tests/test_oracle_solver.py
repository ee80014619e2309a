"""Pins of the oracle's smoother, V-cycle, PCG and adjoint gradient (Section 5 Remarks on the smoother
and on the two-level error propagator; Section 6 smoother, coarse solver and stopping rule)."""
import numpy as np
import pytest
import scipy.sparse as sp

import fixtures as F
import oracle as O
from oracle.smoother import lanczos_start, lanczos_tridiagonal, sturm_max_eig


def _spd(n, seed, cond=50.0):
    g = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n)
    M = Q @ np.diag(ev) @ Q.T
    Dh = np.diag(g.uniform(0.5, 2.0, n))
    return Dh @ M @ Dh


def test_lanczos_start_vector_is_integer_defined():
    v = lanczos_start(3)
    assert v[0] == -0.5
    # 2654435761 / 2^32 is the fractional golden-ratio multiplier (Knuth's multiplicative hash)
    assert abs(v[1] - ((np.sqrt(5.0) - 1.0) / 2.0 - 0.5)) < 1e-8
    assert v[2] == ((2 * 2654435761) % 2 ** 32) / 2 ** 32 - 0.5


def test_sturm_bisection_matches_eigvalsh():
    g = np.random.default_rng(3)
    a = g.standard_normal(12)
    b = g.uniform(0.1, 1.0, 11)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    assert abs(sturm_max_eig(a, b) - np.linalg.eigvalsh(T)[-1]) < 1e-13


def test_lanczos_estimate_bounds_and_converges():
    A = _spd(40, 1)
    D = np.diag(A).copy()
    lam = np.max(np.linalg.eigvals(A / D[:, None]).real)
    est10 = O.lanczos_max_eig(sp.csr_matrix(A), D, 10)
    est40 = O.lanczos_max_eig(sp.csr_matrix(A), D, 40)
    assert est10 <= lam * (1 + 1e-12)
    assert est10 > 0.8 * lam
    assert abs(est40 - lam) < 1e-9 * lam


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_chebyshev_error_polynomial_closed_form(degree):
    """e_new = p(D^{-1}A) e with p(l) = T_K((theta - l)/delta) / T_K(theta/delta) (Chebyshev acceleration)."""
    A = _spd(30, 2)
    D = np.diag(A).copy()
    lam_hi = 1.1 * np.max(np.linalg.eigvals(A / D[:, None]).real)
    lam_lo = lam_hi / 30.0
    theta, delta = 0.5 * (lam_hi + lam_lo), 0.5 * (lam_hi - lam_lo)
    g = np.random.default_rng(4)
    xs = g.standard_normal(30)
    b = A @ xs
    x0 = g.standard_normal(30)
    x1 = O.chebyshev_apply(sp.csr_matrix(A), D, b, x0, lam_lo, lam_hi, degree)
    # eigen-decomposition of the D-symmetric operator D^{-1}A
    Dm = np.diag(1.0 / np.sqrt(D))
    w, U = np.linalg.eigh(Dm @ A @ Dm)
    T = np.polynomial.chebyshev.Chebyshev.basis(degree)
    pw = T((theta - w) / delta) / T(theta / delta)
    e0 = np.sqrt(D) * (xs - x0)
    e1_ref = U @ (pw * (U.T @ e0))
    np.testing.assert_allclose(np.sqrt(D) * (xs - x1), e1_ref, atol=1e-12 * np.abs(e0).max())


def _two_level(d=2, N=8, p=2, pc=1, leaf=24, pre=2, post=2, jitter=0.2):
    prob = F.structured_qp(d, N, p, jitter=jitter, cfg=2)
    h = O.build_hierarchy(prob.coords, prob.scipy(), coarse_degree=pc, leaf_size=leaf, max_levels=2,
                          pre_steps=pre, post_steps=post)
    return prob, h


def _B_matrix(h, n):
    return np.stack([O.vcycle(h, e) for e in np.eye(n)], axis=1)


def test_two_level_error_propagator():
    """I - B A = p(D^{-1}A)^post (I - P A_c^{-1} P^T A) p(D^{-1}A)^pre (Section 5 Remark on E, with
    pre-smoothing added; the smoother polynomial from the eigen-decomposition)."""
    prob, h = _two_level(pre=2, post=1)
    A = prob.scipy().toarray()
    n = A.shape[0]
    lv = h.levels[0]
    D = np.diag(A).copy()
    theta, delta = 0.5 * (lv.lam_hi + lv.lam_lo), 0.5 * (lv.lam_hi - lv.lam_lo)
    Dm = np.diag(1.0 / np.sqrt(D))
    w, U = np.linalg.eigh(Dm @ A @ Dm)
    T = np.polynomial.chebyshev.Chebyshev.basis(3)
    pw = T((theta - w) / delta) / T(theta / delta)
    S = np.diag(np.sqrt(1.0 / D)) @ U @ np.diag(pw) @ U.T @ np.diag(np.sqrt(D))   # p(D^{-1}A)
    P = h.levels[0].P.toarray()
    Ac = P.T @ A @ P
    Cc = np.eye(n) - P @ np.linalg.solve(Ac, P.T @ A)
    E_ref = np.linalg.matrix_power(S, 1) @ Cc @ np.linalg.matrix_power(S, 2)
    E = np.eye(n) - _B_matrix(h, n) @ A
    np.testing.assert_allclose(E, E_ref, atol=1e-10)


@pytest.mark.parametrize("levels", [2, 0])
def test_vcycle_symmetric_positive_definite(levels):
    prob = F.structured_qp(2, 10, 3, jitter=0.2, cfg=2)
    h = O.build_hierarchy(prob.coords, prob.scipy(), coarse_degree=2, leaf_size=40, max_levels=levels,
                          max_coarse_dofs=40)
    if levels == 0:
        assert len(h.levels) >= 3
    g = np.random.default_rng(7)
    for _ in range(3):
        x, y = g.standard_normal(prob.n), g.standard_normal(prob.n)
        Bx, By = O.vcycle(h, x), O.vcycle(h, y)
        assert abs(Bx @ y - x @ By) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(y)
        assert Bx @ x > 0


def test_vcycle_exact_on_worked_example():
    """p'=1 boxes whose points are their own box nodes: two-level B = A^{-1}; PCG converges in one step."""
    prob = F.structured_qp(2, 3, 1, dirichlet=False)
    A = (prob.scipy() + sp.identity(16)).tocsr()
    h = O.build_hierarchy(prob.coords, A, coarse_degree=1, leaf_size=4, max_levels=2)
    Bm = _B_matrix(h, 16)
    np.testing.assert_allclose(Bm, np.linalg.inv(A.toarray()), atol=1e-12)
    b = np.random.default_rng(0).standard_normal(16)
    x, k, conv, _, _ = O.pcg(h, b, rtol=1e-10)
    assert k == 1 and conv


def test_pcg_matches_direct_solve():
    w = F.workload(1)
    h = O.build_hierarchy(w.problem.coords, w.problem.scipy(), coarse_degree=1, leaf_size=64, max_levels=2,
                          pre_steps=1, post_steps=1)
    x, k, conv, hist, cond = O.pcg(h, w.rhs, rtol=1e-13)
    xs = np.linalg.solve(w.problem.scipy().toarray(), w.rhs)
    assert conv
    assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs)
    # the condition estimate approaches the spectrum of BA, which lies in (0, ...]
    Bm = _B_matrix(h, w.problem.n)
    ev = np.sort(np.linalg.eigvals(Bm @ w.problem.scipy().toarray()).real)
    assert cond <= ev[-1] / ev[0] * (1 + 1e-6)
    assert cond >= 0.9 * ev[-1] / ev[0]


def test_pcg_stop_rule_and_zero_rhs():
    w = F.workload(1)
    h = O.build_hierarchy(w.problem.coords, w.problem.scipy(), coarse_degree=1, leaf_size=64, max_levels=2)
    x, k, conv, hist, _ = O.pcg(h, np.zeros(w.problem.n))
    assert k == 0 and conv and np.all(x == 0)
    x, k, conv, hist, _ = O.pcg(h, w.rhs, rtol=1e-10)
    assert hist[k] <= 1e-10 * hist[0] and hist[k - 1] > 1e-10 * hist[0]
    x, k, conv, hist, _ = O.pcg(h, w.rhs, rtol=1e-10, maxit=2)
    assert not conv and k == 2


def test_coarse_degree_trend():
    """Section 6.1: enriching the coarse space (p'=1) needs far fewer iterations than p'=0."""
    prob = F.structured_qp(2, 32, 1)
    b = F.nodal_rhs(prob, np.ones(prob.n))
    its = []
    for pc in (0, 1):
        h = O.build_hierarchy(prob.coords, prob.scipy(), coarse_degree=pc, leaf_size=32, max_levels=2)
        its.append(O.pcg(h, b, rtol=1e-6)[1])
    assert its[1] < its[0]


def _cfg5_small(N=4):
    ncells = N ** 3
    kappa = np.exp(F.rng(5, F.PURPOSE_KAPPA).standard_normal(ncells))
    prob = F.structured_qp(3, N, 2, cfg=5, kappa=kappa, keep_ke=True)
    ut = F.smooth_target(prob.coords, 5)
    return prob, kappa, ut


def _direct(prob):
    def solve(kappa, rhs):
        A = O.assemble_kappa(prob.row_ptr, prob.col, prob.n, prob.cells, prob.Ke, kappa, prob.boundary)
        return np.linalg.solve(A.toarray(), rhs), A
    return solve


def test_assemble_kappa_matches_fixture():
    prob, kappa, _ = _cfg5_small()
    A = O.assemble_kappa(prob.row_ptr, prob.col, prob.n, prob.cells, prob.Ke, kappa, prob.boundary)
    np.testing.assert_allclose(A.data, prob.val, rtol=1e-13, atol=1e-15)


def test_adjoint_gradient_fd_and_euler_identity():
    prob, kappa, ut = _cfg5_small()
    b = prob.mass_rhs_weights
    solve = _direct(prob)
    L, g, u, lam = O.loss_and_gradient(solve, prob.cells, prob.Ke, kappa, b, ut, prob.boundary)
    # Euler identity: A is homogeneous of degree 1 in kappa on unconstrained DoFs
    assert abs(kappa @ g + (u - ut) @ u) <= 1e-10 * abs((u - ut) @ u)
    # central finite differences on a few cells
    for e in [0, 5, 17, 40, 63]:
        hk = 1e-4 * kappa[e]
        kp, km = kappa.copy(), kappa.copy()
        kp[e] += hk
        km[e] -= hk
        Lp = 0.5 * np.sum((solve(kp, b)[0] - ut) ** 2)
        Lm = 0.5 * np.sum((solve(km, b)[0] - ut) ** 2)
        fd = (Lp - Lm) / (2 * hk)
        assert abs(fd - g[e]) <= 1e-6 * max(abs(g[e]), 1e-3 * np.abs(g).max())


def test_adjoint_gradient_dense_formula():
    prob, kappa, ut = _cfg5_small(3)
    b = prob.mass_rhs_weights
    solve = _direct(prob)
    L, g, u, lam = O.loss_and_gradient(solve, prob.cells, prob.Ke, kappa, b, ut, prob.boundary)
    A = O.assemble_kappa(prob.row_ptr, prob.col, prob.n, prob.cells, prob.Ke, kappa, prob.boundary).toarray()
    for e in range(0, prob.cells.shape[0], 5):
        dA = np.zeros_like(A)
        c = prob.cells[e]
        for a in range(len(c)):
            for bb in range(len(c)):
                if not (prob.boundary[c[a]] or prob.boundary[c[bb]]):
                    dA[c[a], c[bb]] += prob.Ke[a, bb]
        du = -np.linalg.solve(A, dA @ u)
        assert abs((u - ut) @ du - g[e]) <= 1e-10 * max(1.0, abs(g[e]))


def test_pcg_batched_columns_match_direct_solves():
    """O12: independent PCG per right-hand side, each frozen on its own convergence.  Pinned against a dense
    direct solve of every column, a zero column (0 iterations, x = 0) and a scaled column (the stop rule is
    relative, so a scaled right-hand side takes the same iterations and gives the scaled solution)."""
    w = F.workload(1)
    A = w.problem.scipy()
    h = O.build_hierarchy(w.problem.coords, A, coarse_degree=1, leaf_size=64, max_levels=2,
                          pre_steps=1, post_steps=1)
    g = np.random.default_rng(11)
    b1 = g.standard_normal(w.problem.n)
    b1[w.problem.boundary] = 0.0
    Bm = np.stack([w.rhs, np.zeros(w.problem.n), 1e6 * w.rhs, b1])
    X, iters = O.pcg_batched(h, Bm, rtol=1e-13)
    Xs = np.linalg.solve(A.toarray(), Bm.T).T
    for j in (0, 2, 3):
        assert np.linalg.norm(X[j] - Xs[j]) <= 1e-11 * np.linalg.norm(Xs[j])
    assert iters[1] == 0 and np.all(X[1] == 0.0)
    assert iters[2] == iters[0] and iters[0] > 0
    np.testing.assert_allclose(X[2], 1e6 * X[0], rtol=0, atol=1e-9 * np.abs(X[2]).max())
