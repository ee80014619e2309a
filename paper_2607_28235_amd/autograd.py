"""Differentiable R3MG-C solve of -div(kappa grad u) = f with respect to a per-cell coefficient kappa.

Standard adjoint method (not in the paper, whose model problem is Poisson): the forward pass assembles
A(kappa) = sum_e kappa_e K_e on the GPU (deterministic gather), rebuilds the hierarchy numerically on the same
partition and transfers (Galerkin products, Lanczos bounds, coarsest factorisation) and solves A u = b by PCG.
The backward pass solves the adjoint system A lambda = dL/du with the same hierarchy (A is symmetric) and
forms g_e = -lambda_e^T K_e u_e per cell on the GPU.  Constrained (Dirichlet) rows are identity rows that do
not depend on kappa.  Every arithmetic step runs in libr3mg.so; this module only orders the calls.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from ._lib import Assembler, Hierarchy, Options


class AdjointPoisson:
    """Holds the hierarchy, the assembler and the device copies of the cell data for one mesh/pattern."""

    def __init__(self, coords: np.ndarray, row_ptr: np.ndarray, col: np.ndarray, val: np.ndarray,
                 cells: np.ndarray, Ke: np.ndarray, b: np.ndarray, options: Options, *, rtol: float = 1e-10,
                 maxit: int = 500, device: str = "cuda"):
        self.h = Hierarchy(coords, row_ptr, col, val, options)
        self.asm = Assembler(self.h, cells)
        self.cells = torch.from_numpy(np.ascontiguousarray(cells, dtype=np.int32)).to(device)
        Ke = np.ascontiguousarray(Ke, dtype=np.float64)
        nloc = cells.shape[1]
        self.ke_stride = 0 if Ke.ndim == 2 else nloc * nloc
        self.Ke = torch.from_numpy(Ke).to(device)
        self.b = torch.from_numpy(np.ascontiguousarray(b, dtype=np.float64)).to(device)
        self.vals = torch.empty(self.h.nnz, dtype=torch.float64, device=device)
        self.rtol, self.maxit = rtol, maxit
        self._kref = None     # the kappa tensor whose operator the hierarchy holds (kept alive on purpose:
        self._kver = -1       # a freed tensor's address may be handed to a different tensor)
        self.last_iters = (0, 0)

    def set_kappa(self, kappa: torch.Tensor):
        """Assemble A(kappa) and rebuild the hierarchy numerically, unless the hierarchy already holds the
        operator of this very tensor at its current version."""
        if kappa is self._kref and kappa._version == self._kver:
            return
        self.asm.assemble(kappa.detach().contiguous(), self.Ke, self.ke_stride, self.vals)
        self.h.update_values(self.vals)
        self._kref, self._kver = kappa, kappa._version

    def invalidate(self):
        self._kref, self._kver = None, -1

    def solve_field(self, rhs: torch.Tensor) -> torch.Tensor:
        x = torch.zeros_like(rhs)
        it, _, ok = self.h.pcg(rhs.contiguous(), x, rtol=self.rtol, maxit=self.maxit)
        if not ok:
            raise RuntimeError("PCG did not converge")
        return x, int(it[0])

    def __call__(self, kappa: torch.Tensor) -> torch.Tensor:
        return PoissonSolve.apply(kappa, self)


class PoissonSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kappa: torch.Tensor, op: AdjointPoisson):
        op.set_kappa(kappa)
        u, it = op.solve_field(op.b)
        ctx.op = op
        ctx.kappa = kappa            # the very object, so that backward can tell whether it is still assembled
        ctx.save_for_backward(kappa, u)
        op.last_iters = (it, op.last_iters[1])
        return u

    @staticmethod
    def backward(ctx, gu: torch.Tensor):
        kappa, u = ctx.saved_tensors
        op: AdjointPoisson = ctx.op
        op.set_kappa(ctx.kappa)             # the hierarchy must hold A(kappa) of this forward
        lam, it = op.solve_field(gu.contiguous())
        g = torch.empty_like(kappa)
        op.h.cell_grad(op.cells, op.Ke, op.ke_stride, u, lam, g)
        op.last_iters = (op.last_iters[0], it)
        return g, None
