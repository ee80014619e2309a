"""Box-local coarse basis (oracle; test infrastructure only).

Section 4: the coarse functions of an agglomerate K are the basis of Q^{p'}(B_K) on the axis-aligned
bounding box B_K, injected into the fine space by nodal interpolation at the support points K owns
(Section 5, definition of the local coarse space V_i^c; p' = 0 gives the Nicolaides space).  The paper
does not fix the basis of Q^{p'}(B_K); Section 5's admissibility assumption asks for stable tensor-product
interpolation nodes on the box, so this reading takes tensor Lagrange polynomials on the GLL nodes of the
box: on [0,1], p'=1 -> {0,1}, p'=2 -> {0,1/2,1}, p'=3 -> {0,(1-1/sqrt5)/2,(1+1/sqrt5)/2,1}.

Local coordinates xi_a = (x_a - lo_a)/(hi_a - lo_a); phi_q(x) = prod_a l_{q_a}(xi_a) with the coarse index
q = q_0 + (p'+1) q_1 + (p'+1)^2 q_2.
"""
from __future__ import annotations

import math

import numpy as np


def box_nodes_1d(pc: int) -> np.ndarray:
    if pc == 0:
        return np.array([0.5])
    if pc == 1:
        return np.array([0.0, 1.0])
    if pc == 2:
        return np.array([0.0, 0.5, 1.0])
    if pc == 3:
        s = 1.0 / math.sqrt(5.0)
        return np.array([0.0, 0.5 * (1.0 - s), 0.5 * (1.0 + s), 1.0])
    raise ValueError("coarse degree p' must be in 0..3")


def lagrange_1d(nodes: np.ndarray, s: np.ndarray) -> np.ndarray:
    """l_j(s) = prod_{m != j} (s - t_m)/(t_j - t_m); returns (len(s), len(nodes))."""
    s = np.asarray(s, dtype=np.float64)
    k = len(nodes)
    out = np.ones((s.shape[0], k))
    if k == 1:
        return out
    for j in range(k):
        for m in range(k):
            if m != j:
                out[:, j] *= (s - nodes[m]) / (nodes[j] - nodes[m])
    return out


def coarse_multi_index(d: int, pc: int) -> np.ndarray:
    """(B, d) table of (q_0, q_1, q_2) for q = q_0 + (p'+1) q_1 + (p'+1)^2 q_2."""
    k = pc + 1
    B = k ** d
    q = np.arange(B)
    return np.stack([(q // (k ** a)) % k for a in range(d)], axis=1)


def box_basis_values(x: np.ndarray, lo: np.ndarray, hi: np.ndarray, pc: int) -> np.ndarray:
    """phi_q of the box [lo, hi] at points x (rows); returns (npts, B)."""
    x = np.atleast_2d(x)
    d = x.shape[1]
    mi = coarse_multi_index(d, pc)
    if pc == 0:
        return np.ones((x.shape[0], 1))
    nodes = box_nodes_1d(pc)
    vals = np.ones((x.shape[0], mi.shape[0]))
    for a in range(d):
        xi = (x[:, a] - lo[..., a]) / (hi[..., a] - lo[..., a])
        la = lagrange_1d(nodes, xi)                     # (npts, p'+1)
        vals *= la[:, mi[:, a]]
    return vals


def box_node_points(lo: np.ndarray, hi: np.ndarray, pc: int) -> np.ndarray:
    """Tensor GLL nodes y_q = lo + t_q * (hi - lo) of one box, (B, d), same q ordering."""
    d = lo.shape[0]
    mi = coarse_multi_index(d, pc)
    t = box_nodes_1d(pc)
    return lo[None, :] + t[mi] * (hi - lo)[None, :]
