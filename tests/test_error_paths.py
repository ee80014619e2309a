"""Failure detection (no GPU needed): the library and the oracle reject an operator that is not symmetric
positive definite with R3MG_ERR_NOT_SPD / "NOT_SPD", and the library reports sizes beyond its int32 index range
as R3MG_ERR_OOM, each before touching anything.

Section 6's smoother is Jacobi-preconditioned Chebyshev, which divides by the diagonal, and its coarsest solve
is a direct factorisation, which fails on an indefinite coarse operator.  The oracle checks the diagonal of
every smoothed level and the Cholesky factorisation of the coarsest one; the library checks the fine-level
diagonal on the host at analysis (the coarse levels and the coarsest factorisation on the device at
r3mg_factor, covered by the GPU tests)."""
import ctypes as C

import numpy as np
import pytest
import scipy.sparse as sp

import fixtures as F
import oracle as O

P = pytest.importorskip("paper_2607_28235_amd")


def _cfg1():
    w = F.workload(1)
    return w.problem


def _with_diag(prob, i, value):
    A = prob.scipy().tolil()
    A[i, i] = value
    A = A.tocsr()
    A.sort_indices()
    return A


@pytest.mark.parametrize("value", [-1.0, 0.0])
def test_nonpositive_fine_diagonal_is_not_spd(value):
    prob = _cfg1()
    i = int(np.flatnonzero(~prob.boundary)[17])
    A = _with_diag(prob, i, value)
    with pytest.raises(O.R3mgError) as eo:
        O.build_hierarchy(prob.coords, A, coarse_degree=1, leaf_size=64, max_levels=2)
    assert eo.value.code == "NOT_SPD"
    with pytest.raises(P.R3mgError) as e:
        P.Hierarchy(prob.coords, A.indptr, A.indices, A.data,
                    P.Options(dim=2, coarse_degree=1, leaf_size=64, max_levels=2), factor=False)
    assert e.value.code == "NOT_SPD" and e.value.status == -4
    assert f"row {i}" in str(e.value)


def test_nonpositive_diagonal_of_a_constrained_row_is_not_spd():
    """A Dirichlet row keeps its diagonal entry (the identity row); zero there is rejected too."""
    prob = _cfg1()
    i = int(np.flatnonzero(prob.boundary)[5])
    A = _with_diag(prob, i, 0.0)
    assert O.hierarchy.constrained_set(A)[i]
    with pytest.raises(O.R3mgError) as eo:
        O.build_hierarchy(prob.coords, A, coarse_degree=1, leaf_size=64, max_levels=2)
    assert eo.value.code == "NOT_SPD"
    with pytest.raises(P.R3mgError) as e:
        P.Hierarchy(prob.coords, A.indptr, A.indices, A.data,
                    P.Options(dim=2, coarse_degree=1, leaf_size=64, max_levels=2), factor=False)
    assert e.value.code == "NOT_SPD"


def test_missing_diagonal_entry_is_not_spd():
    prob = _cfg1()
    A = prob.scipy().tocsr()
    i = int(np.flatnonzero(~prob.boundary)[3])
    keep = np.ones(A.nnz, dtype=bool)
    s, e = A.indptr[i], A.indptr[i + 1]
    keep[s + int(np.flatnonzero(A.indices[s:e] == i)[0])] = False
    rows = np.repeat(np.arange(prob.n), np.diff(A.indptr))[keep]
    B = sp.csr_matrix((A.data[keep], (rows, A.indices[keep])), shape=A.shape)
    B.sort_indices()
    assert B[i, i] == 0.0
    with pytest.raises(P.R3mgError) as err:
        P.Hierarchy(prob.coords, B.indptr, B.indices, B.data,
                    P.Options(dim=2, coarse_degree=1, leaf_size=64, max_levels=2), factor=False)
    assert err.value.code == "NOT_SPD"


def test_indefinite_coarsest_operator_is_not_spd_in_the_oracle():
    """A - sigma I on the unconstrained rows keeps a positive diagonal (sigma is half the smallest one) but is
    indefinite; with two levels the Galerkin coarsest operator P^T (A - sigma I) P is indefinite as well, and
    its Cholesky factorisation fails.  (The library takes the same decision in its device factorisation.)"""
    prob = _cfg1()
    A = prob.scipy()
    free = ~prob.boundary
    sigma = 0.5 * A.diagonal()[free].min()
    S = (A - sp.diags(sigma * free.astype(np.float64))).tocsr()
    S.sort_indices()
    assert np.all(S.diagonal() > 0)
    assert np.linalg.eigvalsh(S.toarray())[0] < 0
    with pytest.raises(O.R3mgError) as eo:
        O.build_hierarchy(prob.coords, S, coarse_degree=1, leaf_size=64, max_levels=2)
    assert eo.value.code == "NOT_SPD"
    assert "coarsest" in str(eo.value)
    # the host analysis accepts it (positive diagonal): the failure belongs to the numeric set-up
    h = P.Hierarchy(prob.coords, S.indptr, S.indices, S.data,
                    P.Options(dim=2, coarse_degree=1, leaf_size=64, max_levels=2), factor=False)
    h.close()


def test_nnz_beyond_int32_is_oom_before_reading_the_pattern():
    """row_ptr[n] >= 2^31 is reported as OOM (the index range of the device arrays) before any column index or
    value is read: the tiny arrays passed here would be read out of bounds otherwise."""
    L = P.lib()
    n = 4
    coords = np.zeros((n, 2))
    coords[:, 0] = np.arange(n)
    coords[:, 1] = np.arange(n) % 2
    row_ptr = np.array([0, 1, 2, 3, 1 << 31], dtype=np.int64)
    col = np.arange(n, dtype=np.int32)
    val = np.ones(n)
    o = P.Options(dim=2, coarse_degree=0, leaf_size=2)._c()
    h = C.c_void_p()
    st = L.r3mg_analyze(coords.ctypes.data_as(C.c_void_p), n, row_ptr.ctypes.data_as(C.c_void_p),
                        col.ctypes.data_as(C.c_void_p), val.ctypes.data_as(C.c_void_p), C.byref(o), C.byref(h))
    assert st == -5                       # R3MG_ERR_OOM
    assert not h.value                    # *out stays NULL
    assert b"int32" in L.r3mg_last_error()


def test_one_sided_coupling_is_not_spd():
    """An entry A_ij whose transpose A_ji is missing makes the coarse block pattern asymmetric; the library, which
    forms only the upper coarse blocks and mirrors them, rejects it at analysis as not symmetric."""
    prob = _cfg1()
    free = np.flatnonzero(~prob.boundary)
    i = int(free[0])
    dist = np.linalg.norm(prob.coords[free] - prob.coords[i], axis=1)
    j = int(free[int(np.argmax(dist))])
    A = prob.scipy().tolil()
    assert A[i, j] == 0 and A[j, i] == 0
    A[i, j] = -1e-3
    A = A.tocsr()
    A.sort_indices()
    with pytest.raises(P.R3mgError) as e:
        P.Hierarchy(prob.coords, A.indptr, A.indices, A.data,
                    P.Options(dim=2, coarse_degree=1, leaf_size=64, max_levels=2), factor=False)
    assert e.value.code == "NOT_SPD" and "not symmetric" in str(e.value)
