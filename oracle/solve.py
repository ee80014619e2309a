"""V-cycle and preconditioned conjugate gradients (oracle; test infrastructure only).

Section 4: one multigrid V-cycle is used as the preconditioner of CG.  The paper lists the components
(Section 6: hierarchy, transfers, degree-3 Chebyshev-Jacobi smoother with 2 pre- and 2 post-steps, level
operators, direct coarsest solve) and the two-level error propagator E = (I - RA)(I - i_c A_c^{-1} i_c' A)
(Section 5 Remark).  The V-cycle below is the textbook symmetric multiplicative cycle built from them:

    B_L r = A_L^{-1} r
    B_l r: x = S^nu(r, 0); r_c = P_l^T (r - A_l x); x += P_l B_{l+1} r_c; x = S^nu(r, x).

PCG (Section 6): stop when the 2-norm of the recursive residual falls below tau.  The paper stops at
||r|| < 1e-9 or a 1e-6 reduction; the reading here is tau = max(rtol * ||r_0||, atol) with atol = 0 by
default.  The iteration count is the number of x-updates when the test first passes (0 if r_0 passes).
The condition estimate is the ratio of extreme eigenvalues of the Lanczos tridiagonal built from the CG
coefficients (the "Cond." column of the paper's tables).
"""
from __future__ import annotations

import numpy as np

from .hierarchy import Hierarchy, coarsest_solve
from .smoother import chebyshev_apply


def vcycle(h: Hierarchy, r: np.ndarray, level: int = 0) -> np.ndarray:
    lv = h.levels
    if level == len(lv) - 1:
        return coarsest_solve(h, r)
    L = lv[level]
    x = np.zeros_like(r)
    for _ in range(h.pre):
        x = chebyshev_apply(L.A, L.diag, r, x, L.lam_lo, L.lam_hi, h.degree)
    rc = L.P.T @ (r - L.A @ x)
    x = x + L.P @ vcycle(h, rc, level + 1)
    for _ in range(h.post):
        x = chebyshev_apply(L.A, L.diag, r, x, L.lam_lo, L.lam_hi, h.degree)
    return x


def _cg_condition(alphas, betas) -> float:
    k = len(alphas)
    if k == 0:
        return 1.0
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    ev = np.linalg.eigvalsh(T)
    return float(ev[-1] / ev[0])


def pcg(h: Hierarchy, b: np.ndarray, x0: np.ndarray = None, *, rtol: float = 1e-10, atol: float = 0.0,
        maxit: int = 500, precondition: bool = True):
    """Returns (x, iters, converged, residual_history, condition_estimate)."""
    A = h.levels[0].A
    x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
    r = b - A @ x
    nr = np.linalg.norm(r)
    tau = max(rtol * nr, atol)
    hist = [nr]
    if nr <= tau:
        return x, 0, True, hist, 1.0
    z = vcycle(h, r) if precondition else r.copy()
    p = z.copy()
    gamma = r @ z
    alphas, betas = [], []
    for k in range(1, maxit + 1):
        q = A @ p
        alpha = gamma / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        alphas.append(alpha)
        nr = np.linalg.norm(r)
        hist.append(nr)
        if nr <= tau:
            return x, k, True, hist, _cg_condition(alphas, betas)
        z = vcycle(h, r) if precondition else r.copy()
        gamma_new = r @ z
        beta = gamma_new / gamma
        betas.append(beta)
        p = z + beta * p
        gamma = gamma_new
    return x, maxit, False, hist, _cg_condition(alphas, betas)


def pcg_batched(h: Hierarchy, Bm: np.ndarray, *, rtol: float = 1e-10, atol: float = 0.0, maxit: int = 500):
    """Independent PCG per right-hand side (rows of Bm); each column is frozen once converged."""
    out = np.zeros_like(Bm)
    iters = np.zeros(Bm.shape[0], dtype=np.int64)
    for j in range(Bm.shape[0]):
        x, k, _, _, _ = pcg(h, Bm[j], rtol=rtol, atol=atol, maxit=maxit)
        out[j] = x
        iters[j] = k
    return out, iters
