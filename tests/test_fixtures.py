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


# ---- simplicial P_p stand-in meshes (the paper's simplicial experiments) -----------------------------------
@pytest.mark.parametrize("p", [1, 2, 3])
def test_simplicial_counts_and_element_matrices(p):
    """(pN+1)^2 lattice support points, 2N^2 triangles; element stiffness symmetric with zero row sums and
    exact energy |grad u|^2 area for linear u; element mass exact for u^2 of linear u (degree 2 <= 2p)."""
    N = 5
    prob = F.simplicial_pp(N, p, jitter=0.2, cfg=2, keep_ke=True, dirichlet=False)
    assert prob.n == (p * N + 1) ** 2 and prob.cells.shape == (2 * N * N, (p + 1) * (p + 2) // 2)
    Ke = prob.Ke
    assert np.abs(Ke - Ke.transpose(0, 2, 1)).max() <= 1e-12 * np.abs(Ke).max()
    assert np.abs(Ke.sum(axis=2)).max() <= 1e-11 * np.abs(Ke).max()
    a, b, c0 = 0.7, -1.3, 0.4
    x = prob.coords[prob.cells]                                     # (cells, nloc, 2)
    u = a * x[..., 0] + b * x[..., 1] + c0
    # the element's vertices: local nodes (0,0), (p,0), (0,p) in the (i, j) listing
    ij = F._simplex_reference(p)[0]
    iA = int(np.flatnonzero((ij[:, 0] == 0) & (ij[:, 1] == 0))[0])
    iB = int(np.flatnonzero((ij[:, 0] == p) & (ij[:, 1] == 0))[0])
    iC = int(np.flatnonzero((ij[:, 0] == 0) & (ij[:, 1] == p))[0])
    XA, XB, XC = x[:, iA], x[:, iB], x[:, iC]
    area = 0.5 * np.abs((XB - XA)[:, 0] * (XC - XA)[:, 1] - (XB - XA)[:, 1] * (XC - XA)[:, 0])
    energy = np.einsum("ci,cij,cj->c", u, Ke, u)
    np.testing.assert_allclose(energy, (a * a + b * b) * area, rtol=1e-11)
    M = prob.mass
    assert abs(M.sum() - 1.0) <= 1e-12                              # area of the unit square
    ug = a * prob.coords[:, 0] + b * prob.coords[:, 1] + c0
    # int_{[0,1]^2} (a x + b y + c)^2 dx dy in closed form
    exact = a * a / 3 + b * b / 3 + c0 * c0 + a * b / 2 + a * c0 + b * c0
    assert abs(ug @ (M @ ug) - exact) <= 1e-12


@pytest.mark.parametrize("p", [1, 2])
def test_simplicial_manufactured_solution_converges(p):
    """-Lap u = 2 pi^2 sin(pi x) sin(pi y) with homogeneous Dirichlet data: nodal max error O(h^{p+1})."""
    import scipy.sparse.linalg as spla
    errs = []
    for N in (8, 16):
        prob = F.simplicial_pp(N, p, jitter=0.0, cfg=2)
        ue = np.sin(np.pi * prob.coords[:, 0]) * np.sin(np.pi * prob.coords[:, 1])
        b = F.nodal_rhs(prob, 2 * np.pi ** 2 * ue)
        uh = spla.spsolve(prob.scipy().tocsc(), b)
        errs.append(np.abs(uh - ue).max())
    rate = np.log2(errs[0] / errs[1])
    assert rate >= p + 0.7, (errs, rate)
