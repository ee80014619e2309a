"""Hierarchy set-up: constrained set, transfers, Galerkin operators, smoother and coarsest factor
(oracle; test infrastructure only).

Section 4: the level operators are inherited, A_i = P_i^T A P_i, with P_i the prolongation from level i to
the finest level, so only the prolongations have to be defined.  Point-based agglomeration: the fine
support points are split among the leaf boxes of the R-tree; the first coarse prolongation P_{M-1} evaluates,
at each owned fine support point, the Q^{p'}(B_K) basis of its box (nodal interpolation, which needs point
values only).  Between agglomerated levels the prolongation P~ is again the natural injection
Q^{p'}(parent box) -> Q^{p'}(child box), and P_i = P_{M-1} P~ ... P~ (composite product).  Remark on the
R-tree parameters and the following remark on heuristics: an agglomerate with too few (or badly placed)
support points makes the local interpolation fail -- reported here as an error, never repaired.
Section 6: the coarsest problem is solved with a sparse direct solver (MUMPS); this reading uses a dense
Cholesky factorisation, which is exact up to rounding.

Readings where the paper is silent:
  O1  constrained set C = rows whose stored off-diagonal entries are all exactly 0.0 (identity rows of the
      Dirichlet data); their rows of P_{M-1} are empty, so coarse functions vanish on the boundary, as the
      interpolation I_h^V of Section 5 enforces.
  O5  all B = (p'+1)^d entries of an owned unconstrained row are stored, exact zeros included.
      Unisolvence: the owned-unconstrained value matrix Phi_K of every leaf must have full column rank,
      tested by a Cholesky factorisation of Phi_K^T Phi_K with pivots > 1e-12 * max diagonal.
  O6  P~[C*B+q', G*B+q] = phi^G_q(y^C_{q'}) with y^C the box nodes of the child box C inside its parent G.
  O7  block (K,K') of A_{l+1} is stored (all B*B entries) iff some stored entry of A_l couples a row owned
      by K to a column owned by K'; both triangles are computed, symmetry is checked, never enforced.
Coarse numbering: box index (left to right) * B + q.  Level 0 keeps the caller's numbering.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .basis import box_basis_values, box_node_points
from .rtree import RTree, bisection_rtree, cell_rtree, select_levels
from .smoother import lanczos_max_eig


class R3mgError(RuntimeError):
    def __init__(self, code: str, msg: str):
        super().__init__(f"{code}: {msg}")
        self.code = code


@dataclasses.dataclass
class Level:
    A: sp.csr_matrix                      # level operator (level numbering)
    diag: np.ndarray
    lam_hi: float = 0.0
    lam_lo: float = 0.0
    P: Optional[sp.csr_matrix] = None     # prolongation from level l+1 to level l
    P_indptr: Optional[np.ndarray] = None  # explicit sparsity of P (zeros kept)
    P_indices: Optional[np.ndarray] = None
    P_data: Optional[np.ndarray] = None
    depth: int = -1                        # R-tree depth of the boxes that define this level (l >= 1)
    lo: Optional[np.ndarray] = None        # box MBRs of this level (l >= 1)
    hi: Optional[np.ndarray] = None
    block_ptr: Optional[np.ndarray] = None  # l >= 1: block sparsity (box rows -> box cols)
    block_col: Optional[np.ndarray] = None


@dataclasses.dataclass
class Hierarchy:
    d: int
    pc: int
    B: int
    levels: List[Level]
    chol: np.ndarray                        # lower Cholesky factor of the dense coarsest operator
    constrained: np.ndarray
    tree: RTree
    depths: List[int]
    owner: np.ndarray                       # leaf box of every fine point (-1 never: constrained own too)
    degree: int = 3
    pre: int = 2
    post: int = 2


def constrained_set(A: sp.csr_matrix) -> np.ndarray:
    """O1: rows whose stored off-diagonal values are all exactly zero."""
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    offd = (A.indices != rows) & (A.data != 0.0)
    has = np.zeros(n, dtype=bool)
    has[rows[offd]] = True
    return ~has


def _check_unisolvent(Phi_rows: np.ndarray, owner: np.ndarray, nbox: int, B: int):
    """O5 unisolvence test per box: Cholesky of G = Phi_K^T Phi_K with pivots > 1e-12 * max diag(G)."""
    srt = np.argsort(owner, kind="stable")
    cnt = np.bincount(owner, minlength=nbox)
    if np.any(cnt < B):
        k = int(np.flatnonzero(cnt < B)[0])
        raise R3mgError("NOT_UNISOLVENT", f"box {k} owns {cnt[k]} unconstrained points < {B}")
    off = np.concatenate([[0], np.cumsum(cnt)])
    G = np.empty((nbox, B, B))
    for k in range(nbox):
        Phi = Phi_rows[srt[off[k]:off[k + 1]]]
        G[k] = Phi.T @ Phi
    tol = 1e-12 * np.max(np.diagonal(G, axis1=1, axis2=2), axis=1)
    L = np.zeros_like(G)
    for j in range(B):                       # column-by-column Cholesky, all boxes at once
        piv = G[:, j, j] - np.einsum("kc,kc->k", L[:, j, :j], L[:, j, :j])
        bad = ~(piv > tol)
        if np.any(bad):
            k = int(np.flatnonzero(bad)[0])
            raise R3mgError("NOT_UNISOLVENT", f"box {k}: pivot {piv[k]:.3e} at column {j}")
        L[:, j, j] = np.sqrt(piv)
        for i in range(j + 1, B):
            L[:, i, j] = (G[:, i, j] - np.einsum("kc,kc->k", L[:, i, :j], L[:, j, :j])) / L[:, j, j]


def prolongation_fine(coords, constrained, owner, lo, hi, pc):
    """O4/O5: P_{M-1}; returns (indptr, indices, data) with B stored entries per unconstrained row."""
    n, d = coords.shape
    B = (pc + 1) ** d
    if pc >= 1 and np.any(hi <= lo):
        raise R3mgError("DEGENERATE_BOX", "a leaf box has zero extent along some axis")
    free = ~constrained
    vals = box_basis_values(coords[free], lo[owner[free]], hi[owner[free]], pc)      # (nfree, B)
    _check_unisolvent(vals, owner[free], lo.shape[0], B)
    counts = np.where(free, B, 0)
    indptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    indices = (owner[free][:, None] * B + np.arange(B)[None, :]).ravel().astype(np.int64)
    data = vals.ravel()
    return indptr, indices, data


def prolongation_coarse(lo_c, hi_c, lo_g, hi_g, parent, pc):
    """O6: P~ from level l+1 (parent boxes G) to level l (child boxes C)."""
    d = lo_c.shape[1]
    B = (pc + 1) ** d
    if pc >= 1 and (np.any(hi_c <= lo_c) or np.any(hi_g <= lo_g)):
        raise R3mgError("DEGENERATE_BOX", "a coarse box has zero extent along some axis")
    nc = lo_c.shape[0]
    rows_data = []
    for c in range(nc):
        g = parent[c]
        y = box_node_points(lo_c[c], hi_c[c], pc)                  # (B, d) child box nodes
        rows_data.append(box_basis_values(y, lo_g[g], hi_g[g], pc))  # (B, B): [q', q]
    data = np.concatenate([r.ravel() for r in rows_data])
    indptr = np.arange(nc * B + 1, dtype=np.int64) * B
    indices = (parent[:, None, None] * B + np.arange(B)[None, None, :]).repeat(B, axis=1).ravel()
    return indptr, indices.astype(np.int64), data


def block_pattern(A: sp.csr_matrix, row_box: np.ndarray, nbox: int):
    """O7 sparsity: box pairs linked by a stored entry of A (rows/cols with row_box < 0 ignored)."""
    coo = A.tocoo()
    rb = row_box[coo.row]
    cb = row_box[coo.col]
    keep = (rb >= 0) & (cb >= 0)
    key = np.unique(rb[keep].astype(np.int64) * nbox + cb[keep])
    br = key // nbox
    bc = key % nbox
    ptr = np.zeros(nbox + 1, dtype=np.int64)
    np.add.at(ptr, br + 1, 1)
    return np.cumsum(ptr), bc.astype(np.int64)


def build_hierarchy(coords, A: sp.csr_matrix, *, coarse_degree: int, leaf_size: int, max_levels: int = 0,
                    max_coarse_dofs: int = 2000, skip_leaf_level: bool = False, cheb_degree: int = 3,
                    pre_steps: int = 2, post_steps: int = 2, lanczos_steps: int = 10,
                    cheb_boost: float = 1.1, cheb_ratio: float = 30.0, cells=None) -> Hierarchy:
    """Section 4 set-up.  cells (ncells x nloc support-point indices) selects cell-based agglomeration
    (oracle.rtree.CellTree, leaf_size counting cells); point-based agglomeration otherwise."""
    coords = np.asarray(coords, dtype=np.float64)
    A = sp.csr_matrix(A, dtype=np.float64)
    n, d = coords.shape
    pc = coarse_degree
    B = (pc + 1) ** d
    if not (np.all(np.isfinite(coords)) and np.all(np.isfinite(A.data))):
        raise R3mgError("INVALID", "non-finite input")
    C = constrained_set(A)
    tree = bisection_rtree(coords, leaf_size) if cells is None else cell_rtree(coords, cells, leaf_size)
    depths = select_levels(tree, d, B, max_levels=max_levels, max_coarse_dofs=max_coarse_dofs,
                           skip_leaf_level=skip_leaf_level)
    levels: List[Level] = []

    # level 0 operator and P_{M-1}
    owner = tree.owner(depths[0])
    lo, hi = tree.boxes(coords, depths[0])
    ip, ix, dt = prolongation_fine(coords, C, owner, lo, hi, pc)
    nb = lo.shape[0]
    P0 = sp.csr_matrix((dt, ix, ip), shape=(n, nb * B))
    lv0 = Level(A=A, diag=A.diagonal().copy(), P=P0, P_indptr=ip, P_indices=ix, P_data=dt)
    levels.append(lv0)
    # level 0 -> 1 sparsity from the stored fine entries between unconstrained points
    row_box = np.where(C, -1, owner)
    bptr, bcol = block_pattern(A, row_box, nb)
    for li, dep in enumerate(depths):
        Af = levels[-1].A
        Pl = levels[-1].P
        Ac = (Pl.T @ (Af @ Pl)).tocsr()                      # A_{l+1} = P_l^T A_l P_l
        Ac.sort_indices()
        amax = np.max(np.abs(Ac.data)) if Ac.nnz else 0.0
        asym = abs(Ac - Ac.T).max() if Ac.nnz else 0.0
        if asym > 1e-13 * amax:
            raise R3mgError("NOT_SPD", f"Galerkin operator not symmetric ({asym:.3e})")
        lv = Level(A=Ac, diag=Ac.diagonal().copy(), depth=dep, lo=lo, hi=hi, block_ptr=bptr,
                   block_col=bcol)
        levels.append(lv)
        if li + 1 < len(depths):
            dep2 = depths[li + 1]
            lo2, hi2 = tree.boxes(coords, dep2)
            parent = np.arange(nb) >> (dep - dep2)
            ip, ix, dt = prolongation_coarse(lo, hi, lo2, hi2, parent, pc)
            nb2 = lo2.shape[0]
            lv.P = sp.csr_matrix((dt, ix, ip), shape=(nb * B, nb2 * B))
            lv.P_indptr, lv.P_indices, lv.P_data = ip, ix, dt
            # blocks of the next level: parents of the box pairs stored on this level
            brow = np.repeat(np.arange(nb), np.diff(bptr))
            key = np.unique(parent[brow] * nb2 + parent[bcol])
            cnt = np.zeros(nb2 + 1, dtype=np.int64)
            np.add.at(cnt, key // nb2 + 1, 1)
            bptr, bcol = np.cumsum(cnt), (key % nb2).astype(np.int64)
            lo, hi, nb = lo2, hi2, nb2
    # smoother set-up on every level but the coarsest (O8)
    for li, lv in enumerate(levels[:-1]):
        if np.any(lv.diag <= 0.0):
            raise R3mgError("NOT_SPD", f"non-positive diagonal on level {li}")
        lam = lanczos_max_eig(lv.A, lv.diag, lanczos_steps)
        lv.lam_hi = cheb_boost * lam
        lv.lam_lo = lv.lam_hi / cheb_ratio
    # dense coarsest factorisation (replaces the sparse direct solver)
    Ad = levels[-1].A.toarray()
    try:
        Lc = np.linalg.cholesky(Ad)
    except np.linalg.LinAlgError:
        raise R3mgError("NOT_SPD", "coarsest operator is not positive definite")
    return Hierarchy(d=d, pc=pc, B=B, levels=levels, chol=Lc, constrained=C, tree=tree, depths=depths,
                     owner=owner, degree=cheb_degree, pre=pre_steps, post=post_steps)


def coarsest_solve(h: Hierarchy, r: np.ndarray) -> np.ndarray:
    """z = A_L^{-1} r by forward and back substitution with the Cholesky factor."""
    y = sla.solve_triangular(h.chol, r, lower=True)
    return sla.solve_triangular(h.chol.T, y, lower=False)
