"""Pins of the oracle's cell-based agglomeration (Section 4): the R-tree over cells, the boxes as bounding boxes
of the agglomerates' cells, and the unique first-come assignment of shared support points."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import fixtures as F
import oracle as O
from oracle.basis import box_node_points, coarse_multi_index
from oracle.hierarchy import R3mgError

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden_2x1():
    rec = {}
    for line in open(os.path.join(GOLDEN, "cells_2x1.txt")):
        if line.startswith("#") or not line.strip():
            continue
        key, *vals = line.split()
        rec[key] = np.array([float(v) for v in vals])
    return rec


def _mesh_2x1():
    coords = np.array([[ix / 2.0, iy] for iy in range(2) for ix in range(3)], dtype=np.float64)
    cells = np.array([[0, 1, 3, 4], [1, 2, 4, 5]])
    # SPD matrix on the node graph: Laplacian of the cell connectivity plus the identity (no constrained rows)
    A = sp.lil_matrix((6, 6))
    for c in cells:
        for i in c:
            for j in c:
                if i != j:
                    A[i, j] -= 1.0
                    A[i, i] += 1.0
    A = (A.tocsr() + sp.identity(6)).tocsr()
    A.sort_indices()
    return coords, cells, A


def test_worked_example_first_come_ownership():
    coords, cells, A = _mesh_2x1()
    g = _golden_2x1()
    tree = O.cell_rtree(coords, cells, 1)
    assert tree.depth == 1
    np.testing.assert_array_equal(tree.owner(1), g["owner"].astype(int))
    lo, hi = tree.boxes(coords, 1)
    np.testing.assert_array_equal(np.concatenate([lo[0], hi[0]]), g["box0"])
    np.testing.assert_array_equal(np.concatenate([lo[1], hi[1]]), g["box1"])
    # p' = 0: P_{M-1} is the ownership indicator and A_1 sums the entries between owned sets
    h = O.build_hierarchy(coords, A, coarse_degree=0, leaf_size=1, max_levels=2, cells=cells)
    own = g["owner"].astype(int)
    P = h.levels[0].P.toarray()
    np.testing.assert_array_equal(P, np.eye(2)[own])
    Ad = A.toarray()
    A1 = np.array([[Ad[np.ix_(own == a, own == b)].sum() for b in range(2)] for a in range(2)])
    np.testing.assert_allclose(h.levels[1].A.toarray(), A1, rtol=0, atol=1e-14)
    # p' = 1: agglomerate 1 keeps two points (x = 1 only) and cannot carry Q^1 (the Remark on parameters)
    with pytest.raises(R3mgError) as e:
        O.build_hierarchy(coords, A, coarse_degree=1, leaf_size=1, max_levels=2, cells=cells)
    assert e.value.code == "NOT_UNISOLVENT"


def _sequential_first_come(cells, node, n):
    """The paper's procedure written as a loop: visit the agglomerates in array order, each taking the support
    points of its cells that no earlier agglomerate took."""
    own = np.full(n, -1)
    for k in range(node.max() + 1):
        for c in np.flatnonzero(node == k):
            for i in cells[c]:
                if own[i] < 0:
                    own[i] = k
    return own


@pytest.mark.parametrize("d,N,p,leaf,jit", [(2, 12, 3, 4, 0.2), (2, 20, 1, 2, 0.0), (3, 6, 2, 2, 0.0)])
def test_cell_tree_invariants(d, N, p, leaf, jit):
    prob = F.structured_qp(d, N, p, jitter=jit, cfg=2)
    tree = O.cell_rtree(prob.coords, prob.cells, leaf)
    x = prob.coords
    for k in range(tree.depth + 1):
        node = tree.cell_node(k)
        own = tree.owner(k)
        np.testing.assert_array_equal(own, _sequential_first_come(prob.cells, node, prob.n))
        lo, hi = tree.boxes(x, k)
        # every box is the bounding box of its cells' points and contains its owned points
        for b in range(1 << k):
            pts = x[np.unique(prob.cells[node == b])]
            np.testing.assert_array_equal(lo[b], pts.min(axis=0))
            np.testing.assert_array_equal(hi[b], pts.max(axis=0))
        assert np.all(x >= lo[own] - 0.0) and np.all(x <= hi[own] + 0.0)
        # nested boxes and cell occupancy window of the bisection tree
        counts = np.bincount(node, minlength=1 << k)
        assert counts.max() - counts.min() <= 1
        if k > 0:
            plo, phi = tree.boxes(x, k - 1)
            par = np.arange(1 << k) >> 1
            assert np.all(lo >= plo[par]) and np.all(hi <= phi[par])


@pytest.mark.parametrize("d,N,p,pc,leaf", [(2, 16, 2, 1, 4), (2, 12, 3, 2, 8), (3, 6, 2, 1, 4)])
def test_cell_based_polynomial_reproduction_and_partition_of_unity(d, N, p, pc, leaf):
    """Every composite P_l of a cell-based hierarchy reproduces global Q^{p'} polynomials and sums to one at the
    unconstrained points (Section 5 partition-of-unity remark)."""
    prob = F.structured_qp(d, N, p, jitter=0.1 if d == 2 else 0.0, cfg=2)
    h = O.build_hierarchy(prob.coords, prob.scipy(), coarse_degree=pc, leaf_size=leaf, max_coarse_dofs=1,
                          skip_leaf_level=True, cells=prob.cells)
    mi = coarse_multi_index(d, pc)
    cf = np.random.default_rng(3).standard_normal(mi.shape[0])

    def g(z):
        return np.sum(cf[None, :] * np.prod(z[:, None, :] ** mi[None, :, :], axis=2), axis=1)
    free = ~h.constrained
    P = sp.identity(prob.n, format="csr")
    for lev in range(1, len(h.levels)):
        P = (P @ h.levels[lev - 1].P).tocsr()
        lv = h.levels[lev]
        nodes = np.concatenate([box_node_points(lv.lo[k], lv.hi[k], pc) for k in range(lv.lo.shape[0])])
        v = P @ g(nodes)
        np.testing.assert_allclose(v[free], g(prob.coords)[free], atol=1e-11 * max(1.0, np.abs(g(prob.coords)).max()))
        rs = np.asarray(P.sum(axis=1)).ravel()
        np.testing.assert_allclose(rs[free], 1.0, atol=1e-12)
