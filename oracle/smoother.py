"""Chebyshev-accelerated Jacobi smoother and its Lanczos eigenvalue estimate (oracle; test infrastructure only).

Section 5 (Remark on the smoother) and Section 6 (smoother paragraph): the smoother is a degree-3
Chebyshev acceleration of Jacobi; on every level it uses the precomputed inverse diagonal and applications
of the level operator, and its parameters come from a Lanczos estimate of the spectrum.  Two pre- and two
post-smoothing steps are used.  Readings where the paper is silent:

  * Lanczos runs on D^{-1}A in the D-inner product for `steps` steps (default 10), from the integer-defined
    start vector v_i = ((i * 2654435761) mod 2^32) / 2^32 - 1/2, so that every implementation starts from the
    same vector; the largest Ritz value is found by Sturm-sequence bisection;
  * lambda_hi = boost * lambda_hat (boost 1.1), lambda_lo = lambda_hi / ratio (ratio 30);
  * one smoothing "step" is one degree-K application of the Chebyshev iteration on D^{-1}A (Saad,
    Iterative Methods for Sparse Linear Systems, Chebyshev acceleration algorithm), started from the
    current iterate.
"""
from __future__ import annotations

import numpy as np


def lanczos_start(n: int, index: np.ndarray = None) -> np.ndarray:
    """v_i = ((i * 2654435761) mod 2^32) / 2^32 - 1/2 for i = index (default 0..n-1)."""
    i = np.arange(n, dtype=np.uint64) if index is None else np.asarray(index, dtype=np.uint64)
    h = (i * np.uint64(2654435761)) % np.uint64(1 << 32)
    return h.astype(np.float64) / float(1 << 32) - 0.5


def lanczos_tridiagonal(A, diag: np.ndarray, steps: int, v0: np.ndarray):
    """Lanczos on M = D^{-1} A with <u,v>_D = sum D_i u_i v_i; returns (alpha, beta) of T_m."""
    alpha, beta = [], []
    v = v0 / np.sqrt(np.sum(diag * v0 * v0))
    v_prev = np.zeros_like(v)
    b_prev = 0.0
    for _ in range(steps):
        u = (A @ v) / diag - b_prev * v_prev
        a = np.sum(diag * u * v)
        u = u - a * v
        b = np.sqrt(np.sum(diag * u * u))
        alpha.append(a)
        if not (b > 0.0) or len(alpha) == steps:
            break
        beta.append(b)
        v_prev, v = v, u / b
        b_prev = b
    return np.array(alpha), np.array(beta)


def sturm_count(alpha: np.ndarray, beta: np.ndarray, x: float) -> int:
    """Number of eigenvalues of the symmetric tridiagonal (alpha; beta) strictly below x."""
    cnt = 0
    q = alpha[0] - x
    if q < 0:
        cnt += 1
    for k in range(1, len(alpha)):
        if q == 0.0:
            q = 1e-300
        q = alpha[k] - x - beta[k - 1] ** 2 / q
        if q < 0:
            cnt += 1
    return cnt


def sturm_max_eig(alpha: np.ndarray, beta: np.ndarray, tol: float = 1e-15) -> float:
    """Largest eigenvalue of the tridiagonal by bisection on the Sturm count, from Gershgorin bounds."""
    m = len(alpha)
    off = np.zeros(m)
    if m > 1:
        off[:-1] += np.abs(beta)
        off[1:] += np.abs(beta)
    lo = float(np.min(alpha - off))
    hi = float(np.max(alpha + off))
    for _ in range(200):
        if hi - lo <= tol * max(1.0, abs(hi)):
            break
        mid = 0.5 * (lo + hi)
        if sturm_count(alpha, beta, mid) == m:    # every eigenvalue below mid
            hi = mid
        else:
            lo = mid
    return hi


def lanczos_max_eig(A, diag: np.ndarray, steps: int = 10, index: np.ndarray = None) -> float:
    v0 = lanczos_start(A.shape[0], index)
    a, b = lanczos_tridiagonal(A, diag, steps, v0)
    return sturm_max_eig(a, b)


def chebyshev_apply(A, diag: np.ndarray, b: np.ndarray, x: np.ndarray, lam_lo: float, lam_hi: float,
                    degree: int) -> np.ndarray:
    """One degree-K Chebyshev-Jacobi application started from x; returns the new iterate."""
    theta = 0.5 * (lam_hi + lam_lo)
    delta = 0.5 * (lam_hi - lam_lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    x = x.copy()
    r = (b - A @ x) / diag
    d = r / theta
    for k in range(1, degree + 1):
        x = x + d
        if k < degree:
            r = r - (A @ d) / diag
            rho_new = 1.0 / (2.0 * sigma - rho)
            d = rho_new * rho * d + (2.0 * rho_new / delta) * r
            rho = rho_new
    return x
