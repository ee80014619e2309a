"""Pins of the synthetic input generator (structured Q_p discretisations, paper Section 2)."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

import fixtures as F


@pytest.mark.parametrize("d,N,p,n_paper", [
    (2, 64, 1, 4225),      # structured square, Q1, 6 refinements (Section 6.1 table)
    (2, 32, 3, 9409),      # structured square, Q3, 5 refinements (Section 6.1 table)
    (3, 16, 1, 4913),      # structured cube, Q1, 4 refinements (Section 6.4 table)
    (3, 16, 2, 35937),     # structured cube, Q2, 4 refinements (Section 6.4 table)
])
def test_dof_counts_match_paper_tables(d, N, p, n_paper):
    prob = F.structured_qp(d, N, p)
    assert prob.n == n_paper


def test_large_dof_counts_formula():
    # Section 6.1 (Q3, 8 refinements) and Section 6.4 (Q2, 6 refinements) report these DoF counts;
    # the generator numbers the (pN+1)^d node grid.
    assert (3 * 256 + 1) ** 2 == 591361
    assert (2 * 64 + 1) ** 3 == 2146689


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_gll_basis_norm_identity(p):
    """Section 5 lemma on GLL Lagrange polynomials: ||psi_j||^2_{L2(-1,1)} = 2p/(2p+1) w_j."""
    nodes01 = F.gll_nodes(p)
    w = F.gll_weights(p)
    xg, wg = np.polynomial.legendre.leggauss(2 * p + 2)       # exact for degree 2p
    val, _ = F.lagrange_1d(nodes01, 0.5 * (xg + 1.0))
    norms = (val ** 2 * wg[:, None]).sum(axis=0)              # integral over [-1,1] in x
    np.testing.assert_allclose(norms, 2 * p / (2 * p + 1) * w, rtol=1e-13)
    # GLL weights integrate 1 exactly
    assert abs(w.sum() - 2.0) < 1e-14


def test_q1_unit_square_element_stiffness_closed_form():
    tab = F._reference_tables(2, 1)
    Xv = np.array([[[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0]]])
    K, M = F._element_matrices(Xv, tab)
    # textbook bilinear stiffness on the unit square, local order (0,0),(1,0),(0,1),(1,1)
    ref = np.array([[4, -1, -1, -2], [-1, 4, -2, -1], [-1, -2, 4, -1], [-2, -1, -1, 4]]) / 6.0
    np.testing.assert_allclose(K[0], ref, atol=1e-15)
    mref = np.array([[4, 2, 2, 1], [2, 4, 1, 2], [2, 1, 4, 2], [1, 2, 2, 4]]) / 36.0
    np.testing.assert_allclose(M[0], mref, atol=1e-15)


@pytest.mark.parametrize("d,N,p,jit", [(2, 6, 2, 0.0), (2, 5, 3, 0.2), (3, 3, 2, 0.0)])
def test_stiffness_symmetry_and_zero_row_sums(d, N, p, jit):
    prob = F.structured_qp(d, N, p, jitter=jit, cfg=2, dirichlet=False)
    A = prob.scipy()
    assert abs(A - A.T).max() == 0.0
    rs = np.asarray(A.sum(axis=1)).ravel()
    assert np.max(np.abs(rs)) < 1e-12 * abs(A).max()


def test_dirichlet_rows_are_identity_and_columns_dropped():
    prob = F.structured_qp(2, 4, 2)
    A = prob.scipy().tocsr()
    for i in np.flatnonzero(prob.boundary):
        row = A.getrow(i)
        assert row.nnz == 1 and row.indices[0] == i and row.data[0] == 1.0
    Ad = A.toarray()
    bi = np.flatnonzero(prob.boundary)
    off = Ad[np.ix_(~prob.boundary, bi)]
    assert np.all(off == 0.0)


def test_linear_energy_on_neumann_operator():
    """For u = a.x (exactly representable), u^T K u = |a|^2 area(Omega) = |a|^2 (jittered interior)."""
    prob = F.structured_qp(2, 6, 3, jitter=0.2, cfg=2, dirichlet=False)
    a = np.array([0.7, -1.3])
    u = prob.coords @ a
    e = u @ (prob.scipy() @ u)
    assert abs(e - a @ a) < 1e-12


@pytest.mark.parametrize("d,p,Ns", [(2, 1, [4, 8, 16]), (2, 2, [4, 8, 16]), (3, 2, [2, 4, 8])])
def test_manufactured_solution_convergence(d, p, Ns):
    """Section 6: u = prod sin(pi x_i) solves -Lap u = d pi^2 u; nodal error decays like h^{p+1}."""
    errs = []
    for N in Ns:
        prob = F.structured_qp(d, N, p)
        x = prob.coords
        u = np.prod(np.sin(np.pi * x), axis=1)
        f = d * np.pi ** 2 * u
        b = F.nodal_rhs(prob, f)
        uh = sla.spsolve(prob.scipy().tocsc(), b)
        errs.append(np.max(np.abs(uh - u)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > p + 1 - 0.35), (errs, rates)


def test_seeded_inputs_are_reproducible():
    a = F.rng(2, F.PURPOSE_RHS).standard_normal(5)
    b = F.rng(2, F.PURPOSE_RHS).standard_normal(5)
    assert np.array_equal(a, b)
    w1 = F.workload(1)
    w2 = F.workload(1)
    assert np.array_equal(w1.rhs, w2.rhs) and np.array_equal(w1.problem.val, w2.problem.val)
