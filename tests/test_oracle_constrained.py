"""Pins of the oracle's constrained set (step O1).

Section 5 builds the coarse spaces through an interpolation into the discrete space with homogeneous Dirichlet
data, so every coarse function vanishes on the Dirichlet boundary.  The oracle reads the Dirichlet set off the
matrix: a row is constrained when every stored off-diagonal value in it is exactly 0.0 (identity rows and
columns of the eliminated boundary data).  The pins below compare that reading with the boundary the fixtures
know from the mesh itself (grid indices on the faces of the cube, or the edges of the triangulated square),
which owes nothing to the matrix values, and with hand-built rows.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import fixtures as F
from oracle.hierarchy import constrained_set


@pytest.mark.parametrize("make", [
    lambda: F.structured_qp(2, 12, 3, jitter=0.2, cfg=2),      # 2D Q3 jittered (the headline's element)
    lambda: F.structured_qp(3, 6, 2, cfg=3),                   # 3D Q2
    lambda: F.structured_qp(3, 4, 3, cfg=4),                   # 3D Q3
    lambda: F.simplicial_pp(6, 2, jitter=0.2, cfg=2),          # simplicial P2
], ids=["2d_q3_jitter", "3d_q2", "3d_q3", "simplex_p2"])
def test_constrained_set_equals_mesh_boundary(make):
    prob = make()
    c = constrained_set(prob.scipy())
    assert c.dtype == bool and c.shape == (prob.n,)
    np.testing.assert_array_equal(c, prob.boundary)
    # neither empty nor everything: a reading that marks no row, or every row, fails here
    assert 0 < int(c.sum()) < prob.n


@pytest.mark.parametrize("make", [
    lambda: F.structured_qp(2, 8, 2, cfg=2, dirichlet=False),
    lambda: F.structured_qp(3, 3, 2, cfg=3, dirichlet=False),
], ids=["2d_neumann", "3d_neumann"])
def test_no_dirichlet_rows_means_empty_constrained_set(make):
    prob = make()
    assert not constrained_set(prob.scipy()).any()


def test_explicit_zero_off_diagonals_are_constrained():
    """Hand case: a row whose only stored off-diagonals are explicit 0.0 is constrained; one nonzero
    off-diagonal makes a row unconstrained, however small; the diagonal value itself never matters."""
    indptr = np.array([0, 3, 5, 7, 8, 10])
    indices = np.array([0, 1, 3,   1, 2,   1, 2,   3,   4, 0])
    data = np.array([1.0, 0.0, 0.0,   7.0, 0.0,   0.0, 2.0,   0.0,   5.0, 1e-300])
    A = sp.csr_matrix((data, indices, indptr), shape=(5, 5))
    assert A.nnz == 10                              # the explicit zeros are stored, not dropped
    c = constrained_set(A)
    # row 0: stored off-diagonals (0,1), (0,3) both 0.0 -> constrained
    # row 1: off-diagonal (1,2) is 0.0 -> constrained (diagonal 7.0 is irrelevant)
    # row 2: off-diagonal (2,1) is 0.0 -> constrained
    # row 3: only its (zero) diagonal -> constrained
    # row 4: off-diagonal (4,0) = 1e-300 is nonzero -> unconstrained
    np.testing.assert_array_equal(c, [True, True, True, True, False])


def test_one_nonzero_off_diagonal_unconstrains_a_dirichlet_row():
    """Putting one nonzero off-diagonal back into a Dirichlet row makes exactly that row unconstrained."""
    prob = F.structured_qp(2, 6, 2, cfg=2)
    A = prob.scipy().tolil()
    i = int(np.flatnonzero(prob.boundary)[3])
    j = int(np.flatnonzero(~prob.boundary)[0])
    A[i, j] = -0.5
    c = constrained_set(A.tocsr())
    expect = prob.boundary.copy()
    expect[i] = False
    np.testing.assert_array_equal(c, expect)
