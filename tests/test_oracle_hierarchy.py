"""Pins of the oracle's transfers and Galerkin operators (Section 4 transfer construction and composite
prolongation; Section 5 partition-of-unity remark; inherited operators A_i = P_i^T A P_i)."""
import numpy as np
import pytest
import scipy.sparse as sp

import fixtures as F
import oracle as O
from oracle.basis import box_basis_values, coarse_multi_index, box_node_points
from oracle.hierarchy import R3mgError


def _hier(d, N, p, pc, leaf, max_levels=0, max_coarse=2000, jitter=0.0, dirichlet=True, **kw):
    prob = F.structured_qp(d, N, p, jitter=jitter, cfg=2, dirichlet=dirichlet)
    A = prob.scipy()
    if not dirichlet:
        A = (A + sp.identity(prob.n)).tocsr()
    h = O.build_hierarchy(prob.coords, A, coarse_degree=pc, leaf_size=leaf, max_levels=max_levels,
                          max_coarse_dofs=max_coarse, **kw)
    return prob, h


def _composite(h, level):
    P = sp.identity(h.levels[0].A.shape[0], format="csr")
    for l in range(level):
        P = P @ h.levels[l].P
    return P.tocsr()


def _random_poly(d, pc, rng):
    """Random global polynomial in Q^{p'} (all monomials x^a y^b z^c with exponents <= p')."""
    mi = coarse_multi_index(d, pc)
    c = rng.standard_normal(mi.shape[0])

    def g(x):
        return np.sum(c[None, :] * np.prod(x[:, None, :] ** mi[None, :, :], axis=2), axis=1)
    return g


@pytest.mark.parametrize("d,N,p,pc,leaf,jit", [
    (2, 12, 2, 1, 16, 0.2), (2, 10, 3, 2, 32, 0.2), (2, 8, 3, 3, 40, 0.0), (3, 8, 2, 2, 256, 0.0),
    (3, 6, 2, 1, 48, 0.0), (2, 8, 2, 0, 24, 0.0)])
def test_polynomial_reproduction_all_levels(d, N, p, pc, leaf, jit):
    """P_l applied to the box-node values of a global g in Q^{p'} reproduces g at unconstrained points."""
    prob, h = _hier(d, N, p, pc, leaf, max_coarse=1, jitter=jit)
    g = _random_poly(d, pc, np.random.default_rng(1))
    free = ~h.constrained
    for lev in range(1, len(h.levels)):
        lv = h.levels[lev]
        nodes = np.concatenate([box_node_points(lv.lo[k], lv.hi[k], pc) for k in range(lv.lo.shape[0])])
        c = g(nodes) if pc > 0 else np.ones(lv.lo.shape[0])
        if pc == 0:
            g_ref = np.ones(prob.n)
        else:
            g_ref = g(prob.coords)
        v = _composite(h, lev) @ c
        np.testing.assert_allclose(v[free], g_ref[free], atol=1e-11 * max(1.0, np.abs(g_ref).max()))
        assert np.all(v[~free] == 0.0)


@pytest.mark.parametrize("pc", [0, 1, 2, 3])
def test_partition_of_unity(pc):
    """Section 5 remark: sum of all coarse functions = 1 on unconstrained DoFs (row sums of P)."""
    prob, h = _hier(2, 10, 3, pc, 40 if pc < 3 else 100, max_coarse=1)
    for lev in range(1, len(h.levels)):
        rs = np.asarray(_composite(h, lev).sum(axis=1)).ravel()
        np.testing.assert_allclose(rs[~h.constrained], 1.0, atol=1e-13)
        assert np.all(rs[h.constrained] == 0.0)


def test_p0_is_permutation_on_worked_example():
    """Each leaf's points are its p'=1 box nodes: P_{M-1} is a permutation (hand-derived example)."""
    prob = F.structured_qp(2, 3, 1, dirichlet=False)      # 4x4 node grid, i = ix + 4 iy
    A = (prob.scipy() + sp.identity(16)).tocsr()
    h = O.build_hierarchy(prob.coords, A, coarse_degree=1, leaf_size=4, max_levels=2)
    P = h.levels[0].P.toarray()
    assert P.shape == (16, 16)
    assert np.all(np.isclose(P, 0.0) | np.isclose(P, 1.0))
    np.testing.assert_allclose(P.sum(axis=0), 1.0)
    np.testing.assert_allclose(P.sum(axis=1), 1.0)
    assert np.all(np.diff(h.levels[0].P_indptr) == 4)      # all B entries stored, zeros included


def test_composite_equals_direct_evaluation():
    """P_i = P_{M-1} P~ ... P~ equals evaluating the level-i box basis at the fine points."""
    prob, h = _hier(2, 12, 2, 2, 40, max_coarse=1, jitter=0.2)
    free = ~h.constrained
    for lev in range(2, len(h.levels)):
        lv = h.levels[lev]
        own = h.tree.owner(lv.depth)
        direct = box_basis_values(prob.coords[free], lv.lo[own[free]], lv.hi[own[free]], h.pc)
        comp = _composite(h, lev)[free].toarray()
        B = h.B
        ref = np.zeros_like(comp)
        rows = np.arange(direct.shape[0])
        for q in range(B):
            ref[rows, own[free] * B + q] = direct[:, q]
        np.testing.assert_allclose(comp, ref, atol=1e-12)


def test_galerkin_p0_closed_form():
    """p'=0 (Nicolaides): A_c[K,K'] = sum of A_ij over unconstrained i in K, j in K'."""
    prob, h = _hier(2, 8, 2, 0, 12, max_levels=2)
    A = prob.scipy().toarray()
    own = h.owner
    free = ~h.constrained
    nb = h.levels[1].A.shape[0]
    ref = np.zeros((nb, nb))
    for i in np.flatnonzero(free):
        for j in np.flatnonzero(free):
            ref[own[i], own[j]] += A[i, j]
    np.testing.assert_allclose(h.levels[1].A.toarray(), ref, rtol=1e-13, atol=1e-13 * abs(ref).max())


def test_recursive_equals_composite_galerkin():
    """Inherited operators: A_i from the recursion equals P_i^T A P_i with the composite P_i."""
    prob, h = _hier(3, 6, 2, 1, 48, max_coarse=1)
    A = h.levels[0].A
    for lev in range(1, len(h.levels)):
        P = _composite(h, lev)
        ref = (P.T @ A @ P).toarray()
        got = h.levels[lev].A.toarray()
        np.testing.assert_allclose(got, ref, atol=1e-12 * abs(ref).max())


@pytest.mark.parametrize("pc", [1, 2])
def test_coarse_operators_spd_and_annihilate_constants(pc):
    """Neumann operator K (+I): coarse operators are SPD; with K alone, A_c kills the constants' coarse
    representation and reproduces the energy of linear functions (|a|^2 on the unit square)."""
    prob = F.structured_qp(2, 8, 2, jitter=0.2, cfg=2, dirichlet=False)
    K = prob.scipy()
    h = O.build_hierarchy(prob.coords, (K + sp.identity(prob.n)).tocsr(), coarse_degree=pc, leaf_size=20,
                          max_coarse_dofs=1)
    for lev in range(1, len(h.levels)):
        Ac = h.levels[lev].A.toarray()
        assert np.max(np.abs(Ac - Ac.T)) <= 1e-13 * np.abs(Ac).max()
        assert np.linalg.eigvalsh(Ac).min() > 0
        P = _composite(h, lev)
        Kc = (P.T @ K @ P).toarray()
        lv = h.levels[lev]
        nodes = np.concatenate([box_node_points(lv.lo[k], lv.hi[k], pc) for k in range(lv.lo.shape[0])])
        one = np.ones(nodes.shape[0])
        assert np.max(np.abs(Kc @ one)) < 1e-12
        a = np.array([0.3, -1.1])
        cl = nodes @ a
        assert abs(cl @ Kc @ cl - a @ a) < 1e-11


def test_block_pattern_is_box_adjacency():
    prob, h = _hier(2, 8, 2, 1, 24, max_levels=2)
    lv = h.levels[1]
    B = h.B
    Ad = lv.A.toarray()
    nb = lv.lo.shape[0]
    stored = np.zeros((nb, nb), dtype=bool)
    for K in range(nb):
        stored[K, lv.block_col[lv.block_ptr[K]:lv.block_ptr[K + 1]]] = True
    nz = np.abs(Ad).reshape(nb, B, nb, B).max(axis=(1, 3)) > 0
    assert np.all(stored >= nz)                     # every nonzero block is in the pattern
    A = prob.scipy().tocoo()
    own = np.where(h.constrained, -1, h.owner)
    ref = np.zeros((nb, nb), dtype=bool)
    m = (own[A.row] >= 0) & (own[A.col] >= 0)
    ref[own[A.row[m]], own[A.col[m]]] = True
    np.testing.assert_array_equal(stored, ref)


def test_errors_degenerate_and_not_unisolvent():
    # all points on a line: zero extent along y -> degenerate box for p' >= 1
    pts = np.stack([np.linspace(0, 1, 20), np.zeros(20)], axis=1)
    A = sp.identity(20, format="csr") * 2.0 - sp.eye(20, k=1) - sp.eye(20, k=-1)
    with pytest.raises(R3mgError) as e:
        O.build_hierarchy(pts, A.tocsr(), coarse_degree=1, leaf_size=5)
    assert e.value.code == "DEGENERATE_BOX"
    # too few points per box for p'=2 in 2D (B = 9 > leaf 4)
    prob = F.structured_qp(2, 6, 1, dirichlet=False)
    A = (prob.scipy() + sp.identity(prob.n)).tocsr()
    with pytest.raises(R3mgError) as e:
        O.build_hierarchy(prob.coords, A, coarse_degree=2, leaf_size=4)
    assert e.value.code == "NOT_UNISOLVENT"
    # enough points but only two distinct x values inside each box: Q^2 is not unisolvent
    xs = np.repeat([0.0, 1.0], 12)
    ys = np.tile(np.linspace(0, 1, 12), 2)
    pts = np.stack([xs, ys], axis=1)
    A = sp.identity(24, format="csr") * 3.0
    A = (A - 0.5 * sp.eye(24, k=1) - 0.5 * sp.eye(24, k=-1)).tocsr()
    with pytest.raises(R3mgError) as e:
        O.build_hierarchy(pts, A, coarse_degree=2, leaf_size=24, max_levels=2)
    assert e.value.code == "NOT_UNISOLVENT"
