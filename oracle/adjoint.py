"""Adjoint gradient of a least-squares loss with respect to a per-cell coefficient (oracle; test
infrastructure only).

Not in the paper (its model problem is the Poisson equation of Section 2); this is the standard adjoint
method applied to -div(kappa grad u) = f discretised as in Section 2:

  A(kappa) = sum_e kappa_e K_e on unconstrained DoFs, identity rows/columns on the constrained set C;
  u = A^{-1} b;  L = 1/2 ||u - u_t||_2^2 over the nodal values;
  adjoint: A lambda = u - u_t (A symmetric, so the same operator and preconditioner serve both solves);
  g_e = dL/dkappa_e = -lambda_e^T K_e u_e, restricted to the unconstrained local DoFs of cell e.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def assemble_kappa(row_ptr, col, n, cells, Ke, kappa, constrained) -> sp.csr_matrix:
    """CSR values of A(kappa) on the given pattern (the pattern must contain every coupled pair)."""
    cells = np.asarray(cells, dtype=np.int64)
    nloc = cells.shape[1]
    shared = Ke.ndim == 2
    rows, cols, vals = [], [], []
    for a in range(nloc):
        for b in range(nloc):
            kab = Ke[a, b] if shared else Ke[:, a, b]
            rows.append(cells[:, a])
            cols.append(cells[:, b])
            vals.append(kappa * kab)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    keep = ~(constrained[rows] | constrained[cols])
    M = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n, n)).tocsr()   # sums duplicates
    M = (M + sp.diags(constrained.astype(np.float64))).tocoo()
    # place the values on the caller's pattern (pattern entries absent from M stay exact zeros)
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    r_of = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    pkeys = r_of * n + col
    mkeys = M.row.astype(np.int64) * n + M.col
    pos = np.searchsorted(pkeys, mkeys)
    if np.any(pos >= len(pkeys)) or np.any(pkeys[np.minimum(pos, len(pkeys) - 1)] != mkeys):
        raise ValueError("pattern misses a coupled pair")
    out = np.zeros(len(col))
    out[pos] = M.data
    return sp.csr_matrix((out, col, row_ptr), shape=(n, n))


def cell_gradient(cells, Ke, u, lam, constrained) -> np.ndarray:
    """g_e = -lambda_e^T K_e u_e over the unconstrained local DoFs of every cell."""
    cells = np.asarray(cells, dtype=np.int64)
    free = ~constrained[cells]
    ue = np.where(free, u[cells], 0.0)
    le = np.where(free, lam[cells], 0.0)
    if Ke.ndim == 2:
        return -np.einsum("ea,ab,eb->e", le, Ke, ue)
    return -np.einsum("ea,eab,eb->e", le, Ke, ue)


def loss_and_gradient(solve, cells, Ke, kappa, b, u_target, constrained):
    """solve(A, rhs) -> x is any SPD solver on A(kappa) (the oracle PCG in the tests)."""
    u, A = solve(kappa, b)
    res = u - u_target
    L = 0.5 * float(res @ res)
    lam, _ = solve(kappa, res)
    return L, cell_gradient(cells, Ke, u, lam, constrained), u, lam
