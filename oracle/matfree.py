"""Q_p Laplace stiffness action on multilinear cells, written from its definition (test infrastructure).

TEST INFRASTRUCTURE ONLY: the oracle of the library's matrix-free fine operator.  It shares no code with it.

The operator is the stiffness matrix of the Poisson problem used in the paper's experiments (Section 6), on
continuous Q_p Lagrange elements (Section 2: the tensor Lagrange space on quadrilaterals and hexahedra) with the
Lagrange nodes at the Gauss-Lobatto points of each axis (the nodes the analysis of Section 5 assumes):

    (K_e)_ab = integral over cell e of grad phi_a . grad phi_b,

the cell being the image of [0,1]^d under the multilinear map of its 2^d corner nodes and the integral being
taken with the tensor Gauss-Legendre rule of p + 1 points per axis.  A = D (sum_e kappa_e K_e) D + diag(cd)
where D zeroes the constrained DoFs (their rows and columns) and cd is the diagonal kept on constrained rows.

Nothing here is blocked or factorised: every cell and Gauss point is visited explicitly, and each Gauss point adds
the outer product of the basis gradients.
"""
from __future__ import annotations

import numpy as np

from .basis import box_nodes_1d


def gauss_01(k: int):
    """Gauss-Legendre points and weights of k points on [0, 1] (numpy's rule on [-1, 1], mapped)."""
    x, w = np.polynomial.legendre.leggauss(k)
    return 0.5 * (x + 1.0), 0.5 * w


def _lagrange_1d(nodes: np.ndarray, s: float):
    """Values and derivatives at s of the Lagrange polynomials on `nodes`."""
    k = nodes.size
    val = np.ones(k)
    der = np.zeros(k)
    for i in range(k):
        for m in range(k):
            if m == i:
                continue
            val[i] *= (s - nodes[m]) / (nodes[i] - nodes[m])
        for j in range(k):
            if j == i:
                continue
            t = 1.0 / (nodes[i] - nodes[j])
            for m in range(k):
                if m != i and m != j:
                    t *= (s - nodes[m]) / (nodes[i] - nodes[m])
            der[i] += t
    return val, der


def element_stiffness(corners: np.ndarray, p: int) -> np.ndarray:
    """K_e of one cell from its 2^d corner coordinates (corner v at bit pattern v: bit a set = far side along
    axis a), local nodes in tensor order (x fastest)."""
    nv, d = corners.shape
    k = p + 1
    nodes = box_nodes_1d(p)
    g, w = gauss_01(k)
    nloc = k ** d
    multi = [tuple((a // k ** ax) % k for ax in range(d)) for a in range(nloc)]
    K = np.zeros((nloc, nloc))
    for qi in range(k ** d):
        qm = [(qi // k ** ax) % k for ax in range(d)]
        xi = np.array([g[m] for m in qm])
        wq = np.prod([w[m] for m in qm])
        # Jacobian of the multilinear map: J[i, c] = d x_i / d xi_c
        J = np.zeros((d, d))
        for v in range(nv):
            bits = [(v >> ax) & 1 for ax in range(d)]
            for c in range(d):
                dpsi = 1.0
                for ax in range(d):
                    if ax == c:
                        dpsi *= 1.0 if bits[ax] else -1.0
                    else:
                        dpsi *= xi[ax] if bits[ax] else 1.0 - xi[ax]
                J[:, c] += corners[v] * dpsi
        det = np.linalg.det(J)
        Jinv = np.linalg.inv(J)
        # reference gradients of every basis function at this Gauss point
        tabs = [_lagrange_1d(nodes, xi[ax]) for ax in range(d)]
        grads = np.zeros((nloc, d))
        for a, ma in enumerate(multi):
            for c in range(d):
                gv = 1.0
                for ax in range(d):
                    val, der = tabs[ax]
                    gv *= der[ma[ax]] if ax == c else val[ma[ax]]
                grads[a, c] = gv
        phys = grads @ Jinv                     # grad_x phi = J^-T grad_xi phi, stored as rows
        K += wq * abs(det) * (phys @ phys.T)    # all pairs (a, b) of this Gauss point's contribution
    return K


def stiffness_apply(coords: np.ndarray, cells: np.ndarray, p: int, x: np.ndarray, *, kappa=None,
                    constrained=None, cdiag=None) -> np.ndarray:
    """y = A x for the operator described in the module docstring.  cells: (ncells, (p+1)^d) in tensor order."""
    coords = np.asarray(coords, dtype=np.float64)
    n, d = coords.shape
    k = p + 1
    cons = np.zeros(n, dtype=bool) if constrained is None else np.asarray(constrained, dtype=bool)
    xf = np.where(cons, 0.0, x)
    y = np.zeros(n)
    corner_pos = [sum(((v >> ax) & 1) * p * k ** ax for ax in range(d)) for v in range(2 ** d)]
    for e in range(cells.shape[0]):
        c = cells[e]
        Ke = element_stiffness(coords[c[corner_pos]], p)
        kap = 1.0 if kappa is None else float(kappa[e])
        y[c] += kap * (Ke @ xf[c])
    y[cons] = 0.0
    if cdiag is not None:
        y[cons] = np.asarray(cdiag)[cons] * x[cons]
    return y
