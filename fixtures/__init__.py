"""Seeded synthetic inputs: structured Q_p Lagrange discretisations of elliptic problems.

This module generates the *inputs* of the multilevel method (support-point coordinates, the assembled
stiffness matrix in CSR form, right-hand sides, cell connectivity and element matrices). It contains none
of the method's arithmetic: no agglomeration, no transfers, no Galerkin products, no smoothing and no
Krylov iteration. Both the FP64 CPU oracle and the HIP library consume what it returns.

Discretisation (paper Section 2, model problem and FE spaces):
  * domain [0,1]^d, N^d quadrilateral/hexahedral cells, optional seeded jitter of interior mesh vertices;
  * continuous Q_p tensor Lagrange elements on Gauss-Lobatto-Legendre (GLL) nodes (the analysis of
    Section 5 assumes GLL nodes on hypercubes), mapped through the multilinear cell map;
  * stiffness  K_e[a,b] = sum_q w_q |J_q| grad(phi_a).grad(phi_b), Gauss (p+1)^d quadrature;
  * homogeneous Dirichlet data on the whole boundary, imposed by identity rows and columns
    (constrained rows keep only their diagonal, entries in constrained columns are not stored);
  * DoF numbering lexicographic on the (pN+1)^d node grid, x fastest.

Random numbers: numpy Generator(PCG64(SeedSequence((cfg, purpose, j)))) with
purpose 0 = vertex jitter, 1 = right-hand side, 2 = kappa, 3 = adjoint target, 4 = FD cells.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

PURPOSE_JITTER, PURPOSE_RHS, PURPOSE_KAPPA, PURPOSE_TARGET, PURPOSE_FDCELLS = 0, 1, 2, 3, 4


def rng(cfg: int, purpose: int, j: int = 0) -> np.random.Generator:
    """Counter-free seeded generator shared by every consumer of the synthetic inputs."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence((cfg, purpose, j))))


# ----------------------------------------------------------------------------------------------
# 1D rules
# ----------------------------------------------------------------------------------------------
def gll_nodes(p: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre nodes of degree p mapped to [0,1] (endpoints plus roots of L_p')."""
    if p < 1:
        raise ValueError("p >= 1")
    if p == 1:
        return np.array([0.0, 1.0])
    if p == 2:
        return np.array([0.0, 0.5, 1.0])
    if p == 3:
        s = 1.0 / math.sqrt(5.0)
        return np.array([0.0, 0.5 * (1.0 - s), 0.5 * (1.0 + s), 1.0])
    c = np.zeros(p + 1)
    c[p] = 1.0
    inner = np.sort(np.polynomial.legendre.legroots(np.polynomial.legendre.legder(c)).real)
    return np.concatenate([[0.0], 0.5 * (inner + 1.0), [1.0]])


def gll_weights(p: int) -> np.ndarray:
    """GLL quadrature weights on [-1,1]: w_j = 2 / (p(p+1) L_p(xi_j)^2)."""
    x = 2.0 * gll_nodes(p) - 1.0
    c = np.zeros(p + 1)
    c[p] = 1.0
    lp = np.polynomial.legendre.legval(x, c)
    return 2.0 / (p * (p + 1) * lp * lp)


def gauss_rule(nq: int):
    """Gauss-Legendre rule with nq points on [0,1]."""
    x, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_1d(nodes: np.ndarray, s: np.ndarray):
    """Values and derivatives of the Lagrange basis on `nodes` at points `s`: (len(s), len(nodes))."""
    s = np.asarray(s, dtype=np.float64)
    k = len(nodes)
    val = np.ones((len(s), k))
    der = np.zeros((len(s), k))
    for j in range(k):
        others = [m for m in range(k) if m != j]
        denom = np.prod([nodes[j] - nodes[m] for m in others])
        for m in others:
            val[:, j] *= (s - nodes[m])
        val[:, j] /= denom
        for drop in others:
            t = np.ones(len(s))
            for m in others:
                if m != drop:
                    t *= (s - nodes[m])
            der[:, j] += t
        der[:, j] /= denom
    return val, der


# ----------------------------------------------------------------------------------------------
# Problem container
# ----------------------------------------------------------------------------------------------
@dataclasses.dataclass
class QpProblem:
    d: int
    N: int
    p: int
    coords: np.ndarray          # (n, d) float64, support points
    row_ptr: np.ndarray         # (n+1,) int64
    col: np.ndarray             # (nnz,) int32, ascending per row
    val: np.ndarray             # (nnz,) float64
    boundary: np.ndarray        # (n,) bool, Dirichlet-constrained support points
    cells: np.ndarray           # (ncells, (p+1)^d) int32 global DoF of each local node
    mass_rhs_weights: Optional[np.ndarray] = None   # b_i = int phi_i  (row sums of M), zero on boundary
    Ke: Optional[np.ndarray] = None                 # (nloc,nloc) shared or (ncells,nloc,nloc) per cell
    kappa: Optional[np.ndarray] = None              # (ncells,) per-cell coefficient used in `val`
    h: float = 0.0                                  # max cell diameter

    @property
    def n(self) -> int:
        return self.coords.shape[0]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def _local_offsets(d: int, p: int) -> np.ndarray:
    """(nloc, d) integer offsets of the local nodes, local index a = ax + (p+1) ay + (p+1)^2 az."""
    r = np.arange(p + 1)
    grids = np.meshgrid(*([r] * d), indexing="ij")           # grids[k] varies along axis k
    # we want x fastest: iterate az, ay, ax
    offs = np.stack([g.transpose(*reversed(range(d))).ravel() for g in grids], axis=1)
    return offs


def _reference_tables(d: int, p: int):
    nodes = gll_nodes(p)
    gq, gw = gauss_rule(p + 1)
    V1, D1 = lagrange_1d(nodes, gq)                           # (nq1, p+1)
    offs = _local_offsets(d, p)                               # (nloc, d)
    qoffs = _local_offsets(d, p)                              # quadrature multi-index, same shape
    nloc = offs.shape[0]
    nq = qoffs.shape[0]
    val = np.ones((nq, nloc))
    grad = np.ones((nq, nloc, d))
    wq = np.ones(nq)
    for k in range(d):
        vk = V1[qoffs[:, k]][:, offs[:, k]]                   # (nq, nloc)
        dk = D1[qoffs[:, k]][:, offs[:, k]]
        val *= vk
        wq *= gw[qoffs[:, k]]
        for m in range(d):
            grad[:, :, m] *= dk if m == k else vk
    # multilinear vertex shape functions and their reference gradients at the quadrature points
    voffs = _local_offsets(d, 1)                              # (2^d, d)
    V1v, D1v = lagrange_1d(np.array([0.0, 1.0]), gq)
    nv = voffs.shape[0]
    vval = np.ones((nq, nv))
    vgrad = np.ones((nq, nv, d))
    for k in range(d):
        vk = V1v[qoffs[:, k]][:, voffs[:, k]]
        dk = D1v[qoffs[:, k]][:, voffs[:, k]]
        vval *= vk
        for m in range(d):
            vgrad[:, :, m] *= dk if m == k else vk
    return dict(nodes=nodes, val=val, grad=grad, wq=wq, offs=offs, voffs=voffs,
                vval=vval, vgrad=vgrad, nloc=nloc, nq=nq)


def _element_matrices(Xv: np.ndarray, tab) -> tuple:
    """Stiffness and mass matrices for a chunk of multilinear cells. Xv: (c, 2^d, d) vertex coords."""
    J = np.einsum("cvi,qvk->cqik", Xv, tab["vgrad"])            # dx_i/dxi_k
    det = np.linalg.det(J)
    if np.any(det <= 0):
        raise ValueError("inverted cell")
    invJ = np.linalg.inv(J)                                    # dxi_k/dx_i = invJ[k,i]
    g = np.einsum("cqki,qak->cqai", invJ, tab["grad"])        # physical gradients
    wdet = det * tab["wq"][None, :]
    K = np.einsum("cq,cqai,cqbi->cab", wdet, g, g)
    M = np.einsum("cq,qa,qb->cab", wdet, tab["val"], tab["val"])
    # exact symmetry of the element matrices (einsum may sum the two triangles in different orders)
    K = 0.5 * (K + K.transpose(0, 2, 1))
    M = 0.5 * (M + M.transpose(0, 2, 1))
    return K, M


def structured_qp(d: int, N: int, p: int, *, jitter: float = 0.0, cfg: int = 0,
                  kappa: Optional[np.ndarray] = None, keep_ke: bool = False, dirichlet: bool = True,
                  chunk: int = 8192) -> QpProblem:
    """Assemble the Q_p stiffness matrix on [0,1]^d with N^d cells (optionally jittered vertices).

    jitter is a fraction of h = 1/N: every interior mesh vertex moves by U[-jitter h, jitter h] per
    component (seed purpose 0).  kappa (per cell) scales each element stiffness matrix.
    dirichlet=False leaves every support point unconstrained (pure Neumann operator, singular).
    """
    tab = _reference_tables(d, p)
    nloc, offs = tab["nloc"], tab["offs"]
    M1 = p * N + 1
    n = M1 ** d
    strides = np.array([M1 ** k for k in range(d)], dtype=np.int64)

    # mesh vertices
    Nv = N + 1
    vgrid = np.stack(np.meshgrid(*([np.arange(Nv)] * d), indexing="ij"), axis=-1)  # [i0,i1,..] -> idx
    vgrid = vgrid.transpose(*reversed(range(d)), d).reshape(-1, d)                 # x fastest
    vx = vgrid.astype(np.float64) / N
    if jitter > 0.0:
        g = rng(cfg, PURPOSE_JITTER)
        shift = g.uniform(-jitter / N, jitter / N, size=vx.shape)
        interior = np.all((vgrid > 0) & (vgrid < N), axis=1)
        vx[interior] += shift[interior]
    vstr = np.array([Nv ** k for k in range(d)], dtype=np.int64)

    # cells: x fastest
    cgrid = np.stack(np.meshgrid(*([np.arange(N)] * d), indexing="ij"), axis=-1)
    cgrid = cgrid.transpose(*reversed(range(d)), d).reshape(-1, d).astype(np.int64)
    ncells = cgrid.shape[0]
    cells = ((cgrid[:, None, :] * p + offs[None, :, :]) * strides).sum(-1).astype(np.int64)
    cell_verts = ((cgrid[:, None, :] + tab["voffs"][None, :, :]) * vstr).sum(-1)  # (ncells, 2^d)

    # support-point coordinates via the multilinear cell map (last writer wins; shared nodes agree)
    coords = np.empty((n, d))
    nodes = tab["nodes"]
    ref = np.stack([nodes[offs[:, k]] for k in range(d)], axis=1)              # (nloc, d)
    V1v, _ = lagrange_1d(np.array([0.0, 1.0]), nodes)                          # (p+1, 2)
    shp = np.ones((nloc, tab["voffs"].shape[0]))
    for k in range(d):
        shp *= V1v[offs[:, k]][:, tab["voffs"][:, k]]
    for c0 in range(0, ncells, chunk):
        c1 = min(ncells, c0 + chunk)
        Xv = vx[cell_verts[c0:c1]]                                              # (c, 2^d, d)
        coords[cells[c0:c1]] = np.einsum("av,cvi->cai", shp, Xv)
    del ref

    # boundary support points
    gidx = np.stack([(np.arange(n) // strides[k]) % M1 for k in range(d)], axis=1)
    boundary = np.any((gidx == 0) | (gidx == M1 - 1), axis=1)
    if not dirichlet:
        boundary[:] = False

    # stencil ("diagonal") storage: S[g, delta] for delta in [-p,p]^d, flat index with x fastest
    W = 2 * p + 1
    nst = W ** d
    dstr = np.array([W ** k for k in range(d)], dtype=np.int64)
    S = np.zeros((n, nst))
    Mw = np.zeros(n)                   # row sums of the mass matrix: int phi_i
    pat = np.zeros((n, nst), dtype=bool)
    delta_ab = (((offs[None, :, :] - offs[:, None, :]) + p) * dstr).sum(-1)   # (nloc, nloc)
    uniform = jitter == 0.0
    Ke_shared = None
    Ke_all = np.empty((ncells, nloc, nloc)) if (keep_ke and not uniform) else None
    if uniform:
        Xv = vx[cell_verts[:1]]
        K1, Mm1 = _element_matrices(Xv, tab)
        Ke_shared, Me_shared = K1[0], Mm1[0]
    h = 0.0
    for c0 in range(0, ncells, chunk):
        c1 = min(ncells, c0 + chunk)
        Xv = vx[cell_verts[c0:c1]]
        diam = np.max(np.linalg.norm(Xv[:, :, None, :] - Xv[:, None, :, :], axis=-1), axis=(1, 2))
        h = max(h, float(diam.max()))
        if uniform:
            K = None
        else:
            K, Mm = _element_matrices(Xv, tab)
            if Ke_all is not None:
                Ke_all[c0:c1] = K
        kap = None if kappa is None else kappa[c0:c1]
        cl = cells[c0:c1]
        for a in range(nloc):
            rows = cl[:, a]
            for b in range(nloc):
                dl = delta_ab[a, b]
                if uniform:
                    v = Ke_shared[a, b] if kap is None else Ke_shared[a, b] * kap
                    S[rows, dl] += v
                else:
                    v = K[:, a, b] if kap is None else K[:, a, b] * kap
                    S[rows, dl] += v
                pat[rows, dl] = True
            if uniform:
                Mw[rows] += Me_shared[a].sum()
            else:
                Mw[rows] += Mm[:, a, :].sum(axis=1)

    # Dirichlet: constrained rows keep the diagonal (1.0); constrained columns are dropped
    dvec = np.stack(np.meshgrid(*([np.arange(-p, p + 1)] * d), indexing="ij"), axis=-1)
    dvec = dvec.transpose(*reversed(range(d)), d).reshape(-1, d)            # (nst, d), x fastest
    dflat = (dvec * strides).sum(-1)
    center = int((p * dstr).sum())
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    cols_out, vals_out = [], []
    counts = np.empty(n, dtype=np.int64)
    rchunk = 1 << 18
    for r0 in range(0, n, rchunk):
        r1 = min(n, r0 + rchunk)
        m = pat[r0:r1].copy()
        rr = np.arange(r0, r1)
        colm = rr[:, None] + dflat[None, :]
        inb = np.all((gidx[r0:r1, None, :] + dvec[None, :, :] >= 0) &
                     (gidx[r0:r1, None, :] + dvec[None, :, :] < M1), axis=-1)
        m &= inb
        bc_row = boundary[r0:r1]
        colc = np.clip(colm, 0, n - 1)
        m &= ~boundary[colc]                                   # drop constrained columns
        m[bc_row, :] = False
        m[bc_row, center] = True                               # constrained rows: diagonal only
        vv = S[r0:r1].copy()
        vv[bc_row, center] = 1.0
        ri, di = np.nonzero(m)
        counts[r0:r1] = np.bincount(ri, minlength=r1 - r0)
        cols_out.append(colm[ri, di].astype(np.int32))
        vals_out.append(vv[ri, di])
    row_ptr[1:] = np.cumsum(counts)
    col = np.concatenate(cols_out)
    val = np.concatenate(vals_out)
    del S, pat
    Mw[boundary] = 0.0
    Ke = Ke_shared if uniform else Ke_all
    return QpProblem(d=d, N=N, p=p, coords=coords, row_ptr=row_ptr, col=col, val=val,
                     boundary=boundary, cells=cells.astype(np.int32), mass_rhs_weights=Mw,
                     Ke=Ke if keep_ke else None, kappa=kappa, h=h)


def mass_apply(d: int, N: int, p: int, f: np.ndarray, *, jitter: float = 0.0, cfg: int = 0,
               chunk: int = 8192) -> np.ndarray:
    """b = M f with the consistent Q_p mass matrix (Gauss (p+1)^d quadrature), unconstrained form.
    f may be (n,) or (k, n) for k right-hand sides at once."""
    tab = _reference_tables(d, p)
    offs = tab["offs"]
    M1 = p * N + 1
    strides = np.array([M1 ** k for k in range(d)], dtype=np.int64)
    Nv = N + 1
    vgrid = np.stack(np.meshgrid(*([np.arange(Nv)] * d), indexing="ij"), axis=-1)
    vgrid = vgrid.transpose(*reversed(range(d)), d).reshape(-1, d)
    vx = vgrid.astype(np.float64) / N
    if jitter > 0.0:
        g = rng(cfg, PURPOSE_JITTER)
        shift = g.uniform(-jitter / N, jitter / N, size=vx.shape)
        interior = np.all((vgrid > 0) & (vgrid < N), axis=1)
        vx[interior] += shift[interior]
    vstr = np.array([Nv ** k for k in range(d)], dtype=np.int64)
    cgrid = np.stack(np.meshgrid(*([np.arange(N)] * d), indexing="ij"), axis=-1)
    cgrid = cgrid.transpose(*reversed(range(d)), d).reshape(-1, d).astype(np.int64)
    ncells = cgrid.shape[0]
    cells = ((cgrid[:, None, :] * p + offs[None, :, :]) * strides).sum(-1)
    cell_verts = ((cgrid[:, None, :] + tab["voffs"][None, :, :]) * vstr).sum(-1)
    F2 = np.atleast_2d(f)
    b = np.zeros_like(F2, dtype=np.float64)
    uniform = jitter == 0.0
    if uniform:
        _, Mm1 = _element_matrices(vx[cell_verts[:1]], tab)
    for c0 in range(0, ncells, chunk):
        c1 = min(ncells, c0 + chunk)
        cl = cells[c0:c1]
        if uniform:
            be = np.einsum("ab,kcb->kca", Mm1[0], F2[:, cl])
        else:
            _, Mm = _element_matrices(vx[cell_verts[c0:c1]], tab)
            be = np.einsum("cab,kcb->kca", Mm, F2[:, cl])
        for a in range(cl.shape[1]):
            b[:, cl[:, a]] += be[:, :, a]
    return b if f.ndim == 2 else b[0]


# ----------------------------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    problem: QpProblem
    rhs: np.ndarray                 # (n,) or (nrhs, n)
    coarse_degree: int
    leaf_size: int
    max_levels: int
    max_coarse_dofs: int
    pre_steps: int
    post_steps: int
    extra: dict = dataclasses.field(default_factory=dict)
    skip_leaf_level: int = 0


def nodal_rhs(prob: QpProblem, f: np.ndarray, *, jitter: float = 0.0, cfg: int = 0) -> np.ndarray:
    """b = M f_h zeroed on constrained points (f given at the support points)."""
    if getattr(prob, "mass", None) is not None:    # simplicial problems carry their assembled mass matrix
        b = prob.mass @ f
    else:
        b = mass_apply(prob.d, prob.N, prob.p, f, jitter=jitter, cfg=cfg)
    b[prob.boundary] = 0.0
    return b


# ---------------------------------------------------------------------------------------------------------
# Simplicial P_p meshes (the paper's simplicial experiments use Lagrange elements of total degree p on
# uniformly spaced nodes): the unit square, N x N squares each split along the diagonal from (x, y) to
# (x+1, y+1) into two triangles, optional jitter of the interior vertices (the same vertices as structured_qp).
# ---------------------------------------------------------------------------------------------------------
def _simplex_reference(p: int):
    """Equispaced nodes (i/p, j/p), i + j <= p, of the reference triangle, the monomial coefficients of the
    Lagrange basis on them, and the exact reference stiffness blocks S_ab = int d_a phi_i d_b phi_j and mass
    int phi_i phi_j (monomial integrals int x^m y^n = m! n! / (m + n + 2)!)."""
    from math import factorial
    ij = [(i, j) for j in range(p + 1) for i in range(p + 1 - j)]
    mono = [(a, b) for b in range(p + 1) for a in range(p + 1 - b)]
    X = np.array([[i / p, j / p] for i, j in ij]) if p > 0 else np.zeros((1, 2))
    V = np.array([[x ** a * y ** b for a, b in mono] for x, y in X])
    Cf = np.linalg.inv(V)                                  # phi_i = sum_k Cf[k, i] x^a_k y^b_k
    m = len(mono)

    def integ(a, b):
        return factorial(a) * factorial(b) / factorial(a + b + 2)
    # monomial Gram matrices: <m_k, m_l>, <d_x m_k, d_x m_l>, ...
    G = np.array([[integ(a1 + a2, b1 + b2) for a2, b2 in mono] for a1, b1 in mono])

    def dmono(k, axis):
        a, b = mono[k]
        if axis == 0:
            return (a, max(a - 1, 0), b) if a > 0 else (0, 0, 0)
        return (b, a, max(b - 1, 0)) if b > 0 else (0, 0, 0)
    Gd = np.zeros((2, 2, m, m))
    for ax in range(2):
        for bx in range(2):
            for k in range(m):
                ck, ak, bk = dmono(k, ax)
                if ck == 0:
                    continue
                for l in range(m):
                    cl, al, bl = dmono(l, bx)
                    if cl == 0:
                        continue
                    Gd[ax, bx, k, l] = ck * cl * integ(ak + al, bk + bl)
    S = np.einsum("ki,abkl,lj->abij", Cf, Gd, Cf)
    Mref = Cf.T @ G @ Cf
    return np.array(ij), S, 0.5 * (Mref + Mref.T)


def simplicial_pp(N: int, p: int, *, jitter: float = 0.0, cfg: int = 0, dirichlet: bool = True,
                  keep_ke: bool = False) -> QpProblem:
    """P_p stiffness matrix on the triangulated unit square (2 N^2 triangles, (pN + 1)^2 support points on the
    lattice, numbered x fastest), Dirichlet rows as in structured_qp.  The returned problem also carries the
    assembled consistent mass matrix (`mass`) for right-hand sides."""
    import scipy.sparse as sp
    M1 = p * N + 1
    n = M1 * M1
    Nv = N + 1
    vx = np.stack(np.meshgrid(np.arange(Nv), np.arange(Nv), indexing="xy"), axis=-1).reshape(-1, 2) / N
    vgrid = np.rint(vx * N).astype(np.int64)
    if jitter > 0.0:
        g = rng(cfg, PURPOSE_JITTER)
        shift = g.uniform(-jitter / N, jitter / N, size=vx.shape)
        interior = np.all((vgrid > 0) & (vgrid < N), axis=1)
        vx = vx.copy()
        vx[interior] += shift[interior]
    ij, S, Mref = _simplex_reference(p)
    nloc = ij.shape[0]
    cx, cy = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    cx, cy = cx.ravel(), cy.ravel()
    v00, v10 = cy * Nv + cx, cy * Nv + cx + 1
    v01, v11 = (cy + 1) * Nv + cx, (cy + 1) * Nv + cx + 1
    tris, offs = [], []
    # T0 = (v00, v10, v11): lattice offset of node (i, j) = (i + j, j); T1 = (v00, v11, v01): (i, i + j)
    for verts, off in (((v00, v10, v11), np.stack([ij[:, 0] + ij[:, 1], ij[:, 1]], 1)),
                       ((v00, v11, v01), np.stack([ij[:, 0], ij[:, 0] + ij[:, 1]], 1))):
        tris.append(np.stack(verts, 1))
        lx = p * cx[:, None] + off[None, :, 0]
        ly = p * cy[:, None] + off[None, :, 1]
        offs.append(ly * M1 + lx)
    tv = np.concatenate(tris)                               # (2 N^2, 3) vertex indices
    cells = np.concatenate(offs).astype(np.int64)           # (2 N^2, nloc) support points
    ncells = tv.shape[0]
    XA, XB, XC = vx[tv[:, 0]], vx[tv[:, 1]], vx[tv[:, 2]]
    J = np.stack([XB - XA, XC - XA], axis=2)                 # (c, 2, 2): columns dX/dxi, dX/deta
    det = np.linalg.det(J)
    if np.any(det <= 0):
        raise ValueError("inverted triangle")
    Jinv = np.linalg.inv(J)
    Gm = np.einsum("cak,cbk->cab", Jinv, Jinv)              # J^-1 J^-T (grad_x = J^-T grad_xi)
    Ke = det[:, None, None] * np.einsum("cab,abij->cij", Gm, S)
    Ke = 0.5 * (Ke + Ke.transpose(0, 2, 1))                   # exact up to the basis' rounding: symmetrise
    Me = det[:, None, None] * Mref[None, :, :]
    coords = np.empty((n, 2))
    lam = ij / max(p, 1)
    coords[cells] = (XA[:, None, :] + lam[None, :, 0:1] * (XB - XA)[:, None, :] +
                     lam[None, :, 1:2] * (XC - XA)[:, None, :])
    rows = np.repeat(cells, nloc, axis=1).ravel()
    colsi = np.tile(cells, (1, nloc)).ravel()
    A = sp.csr_matrix((Ke.ravel(), (rows, colsi)), shape=(n, n))
    M = sp.csr_matrix((Me.ravel(), (rows, colsi)), shape=(n, n))
    A.sum_duplicates()
    M.sum_duplicates()
    gx, gy = np.arange(n) % M1, np.arange(n) // M1
    boundary = (gx == 0) | (gx == M1 - 1) | (gy == 0) | (gy == M1 - 1)
    if not dirichlet:
        boundary[:] = False
    if boundary.any():
        keep = ~boundary
        D = sp.diags(keep.astype(np.float64))
        A = (D @ A @ D + sp.diags(boundary.astype(np.float64))).tocsr()
        A.eliminate_zeros()
        # keep the constrained rows' diagonal even where the product removed it
        A = A.tocsr()
    A.sort_indices()
    Mw = np.asarray(M.sum(axis=1)).ravel()
    Mw[boundary] = 0.0
    h = float(np.max(np.linalg.norm(np.stack([XB - XA, XC - XB, XA - XC], 1), axis=2)))
    prob = QpProblem(d=2, N=N, p=p, coords=coords, row_ptr=A.indptr.astype(np.int64),
                     col=A.indices.astype(np.int32), val=A.data.astype(np.float64), boundary=boundary,
                     cells=cells.astype(np.int32), mass_rhs_weights=Mw, Ke=Ke if keep_ke else None, h=h)
    prob.mass = M.tocsr()
    return prob


def smooth_target(coords: np.ndarray, cfg: int = 5) -> np.ndarray:
    """u_t = sum_{j<4} a_j prod_a sin(pi m_{j,a} x_a), a_j ~ N(0, 0.05^2), m ~ U{1,2,3} (purpose 3)."""
    g = rng(cfg, PURPOSE_TARGET)
    d = coords.shape[1]
    a = g.normal(0.0, 0.05, size=4)
    m = g.integers(1, 4, size=(4, d))
    u = np.zeros(coords.shape[0])
    for j in range(4):
        t = np.full(coords.shape[0], a[j])
        for k in range(d):
            t *= np.sin(np.pi * m[j, k] * coords[:, k])
        u += t
    return u


def workload(cfg: int, *, scale: Optional[int] = None) -> Workload:
    """Build configuration `cfg` (1..5).  `scale` overrides N for reduced-size test instances."""
    if cfg == 1:
        N = scale or 16
        prob = structured_qp(2, N, 2, cfg=1)
        f = rng(1, PURPOSE_RHS).uniform(-1.0, 1.0, size=prob.n)
        b = nodal_rhs(prob, f, cfg=1)
        return Workload("2D Poisson Q2 16x16 (1,089 DoFs), p'=1, leaf 64, 2 levels, V(1,1)",
                        prob, b, 1, 64, 2, 2000, 1, 1)
    if cfg == 2:
        N = scale or 256
        prob = structured_qp(2, N, 3, jitter=0.2, cfg=2)
        f = rng(2, PURPOSE_RHS).standard_normal(prob.n)
        b = nodal_rhs(prob, f, jitter=0.2, cfg=2)
        return Workload("2D Poisson Q3 256x256 jittered (591,361 DoFs), p'=2, leaf 128, 4 levels, V(2,2)",
                        prob, b, 2, 128, 4, 2000, 2, 2)
    if cfg == 3:
        N = scale or 64
        prob = structured_qp(3, N, 2, cfg=3)
        f = rng(3, PURPOSE_RHS).standard_normal(prob.n)
        b = nodal_rhs(prob, f, cfg=3)
        return Workload("3D Poisson Q2 64^3 (2,146,689 DoFs), p'=2, leaf 256, <=2000 coarse, V(2,2)",
                        prob, b, 2, 256, 0, 2000, 2, 2, skip_leaf_level=1)
    if cfg == 4:
        N = scale or 48
        prob = structured_qp(3, N, 3, cfg=4)
        Fm = np.stack([rng(4, PURPOSE_RHS, j).standard_normal(prob.n) for j in range(16)])
        B = mass_apply(3, N, 3, Fm, cfg=4)
        B[:, prob.boundary] = 0.0
        return Workload("3D Poisson Q3 48^3 (3,048,625 DoFs), 16 RHS, p'=2, leaf 256",
                        prob, B, 2, 256, 0, 2000, 2, 2, skip_leaf_level=1)
    if cfg == 5:
        N = scale or 64
        ncells = N ** 3
        kappa = np.exp(rng(5, PURPOSE_KAPPA).standard_normal(ncells))
        prob = structured_qp(3, N, 2, cfg=5, kappa=kappa, keep_ke=True)
        b = prob.mass_rhs_weights.copy()
        ut = smooth_target(prob.coords, 5)
        fd = rng(5, PURPOSE_FDCELLS).choice(ncells, size=min(32, ncells), replace=False)
        return Workload("3D -div(kappa grad u)=1, Q2 64^3, lognormal kappa per cell",
                        prob, b, 2, 256, 0, 2000, 2, 2, extra=dict(target=ut, fd_cells=fd), skip_leaf_level=1)
    raise ValueError(cfg)


def uneven_batch_sizes():
    """Q2 meshes of the second batch: N in {16,21,25,30,34,39,43,48}."""
    return [16, 21, 25, 30, 34, 39, 43, 48]


def uneven_batch(sizes=None):
    """Second batch of the multi-RHS workload: independent 3D Q2 Poisson problems of different sizes, one seeded
    Gaussian nodal right-hand side each (purpose 1, j = problem index)."""
    out = []
    for j, N in enumerate(sizes or uneven_batch_sizes()):
        prob = structured_qp(3, N, 2, cfg=4)
        f = rng(4, PURPOSE_RHS, 100 + j).standard_normal(prob.n)
        out.append((prob, nodal_rhs(prob, f, cfg=4)))
    return out
