"""FP64 CPU oracle for R3MG-C: PCG preconditioned by one V-cycle of an R-tree agglomeration hierarchy.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously-correct reference that the HIP
library is checked against.  Only the test-suite, the smoke entry point and the CPU-baseline leg of the
benchmark may import it; the product path never calls it and shares no code with it.

Every step follows the paper (Polverino, Feder, Heltai, "R3MG-C: a high-order algebraic-geometric
multilevel preconditioner for continuous finite element discretizations"):

  rtree.py      agglomeration of support points by a bisection R-tree      (Section 3, Definition of an
                R-tree of order (m,M); Section 4, point-based agglomeration; Section 6, level choice)
  basis.py      box-local Q^{p'} Lagrange basis on GLL nodes of the box    (Section 4; Section 5, local
                coarse space V_i^c and the admissibility assumption on stable box nodes)
  hierarchy.py  constrained set, prolongations P_{M-1} and P~, Galerkin operators A_i = P_i^T A P_i,
                smoother set-up, dense coarsest factorisation              (Section 4; Section 6)
  smoother.py   Lanczos eigenvalue estimate and Chebyshev-accelerated Jacobi (Section 5 Remark on the
                smoother; Section 6, smoother paragraph)
  solve.py      V-cycle and (batched) PCG                                  (Section 4, Section 5 Remark on
                the two-level error propagator, Section 6 stopping rule)
  adjoint.py    adjoint gradient of 1/2||u-u_t||^2 with respect to per-cell kappa (standard adjoint
                method; not in the paper)
  matfree.py    Q_p Laplace stiffness action cell by cell from its definition (the operator of Section 6,
                the reference of the matrix-free fine operator)

Readings where the paper is silent are listed in the module docstrings (bisection R-tree instead of the
Boost R*-tree, GLL box nodes, Chebyshev interval parameters, Lanczos start vector, stop rule form).
All arithmetic is float64.
"""
from .rtree import bisection_rtree, cell_rtree, select_levels, RTree, CellTree
from .basis import box_nodes_1d, box_basis_values
from .hierarchy import Hierarchy, build_hierarchy, R3mgError
from .smoother import lanczos_max_eig, sturm_max_eig, chebyshev_apply
from .solve import vcycle, pcg, pcg_batched
from .adjoint import assemble_kappa, cell_gradient, loss_and_gradient
from .matfree import element_stiffness, stiffness_apply

__all__ = [
    "bisection_rtree", "cell_rtree", "CellTree", "select_levels", "RTree", "box_nodes_1d", "box_basis_values", "Hierarchy",
    "build_hierarchy", "R3mgError", "lanczos_max_eig", "sturm_max_eig", "chebyshev_apply", "vcycle",
    "pcg", "pcg_batched", "assemble_kappa", "cell_gradient", "loss_and_gradient", "element_stiffness",
    "stiffness_apply",
]
