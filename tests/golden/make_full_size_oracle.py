"""Write sampled oracle outputs of the full-size 3D workloads (test data for the -m gpu full-size parity tests).

The oracle needs minutes per solve at these sizes, too long to run inside the GPU test-suite, so this script
runs it once on the CPU and stores, for 1024 seeded indices, the values the GPU results are compared with, plus
the norms and counts those comparisons need:

  full_cfg3.json  3D Poisson Q2 64^3 (2,146,689 DoFs), p'=2, leaf 256, leaf level skipped, <= 2000 coarse DoFs,
                  V(2,2): level sizes; one V-cycle z = B b; PCG iterations to rtol 1e-10; the solution to rtol 1e-13.
  full_cfg5.json  -div(kappa grad u) = 1 on the same cube, lognormal kappa per cell: level sizes; u to rtol 1e-13;
                  the loss 1/2 ||u - u_t||^2; the adjoint gradient (adjoint solve to rtol 1e-13) at the 32 seeded
                  finite-difference cells and at 1024 seeded cells; its norm.

Only `fixtures` (the seeded inputs) and `oracle` are used.  Usage (about 10-20 minutes and 20 GB of memory):
    python tests/golden/make_full_size_oracle.py [cfg ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import fixtures as F  # noqa: E402
import oracle as O  # noqa: E402

NSAMPLE = 1024
SAMPLE_SEED = 20260   # seeds the sample indices only; the inputs come from the fixtures' own seeds


def log(*a):
    print("[golden]", *a, flush=True)


def sample(n: int, k: int = NSAMPLE) -> np.ndarray:
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n, size=k, replace=False))


def hierarchy(w):
    return O.build_hierarchy(w.problem.coords, w.problem.scipy(), coarse_degree=w.coarse_degree,
                             leaf_size=w.leaf_size, max_levels=w.max_levels, max_coarse_dofs=w.max_coarse_dofs,
                             pre_steps=w.pre_steps, post_steps=w.post_steps, skip_leaf_level=bool(w.skip_leaf_level))


def vals(x, idx):
    return [float(v) for v in np.asarray(x)[idx]]


def cfg3() -> dict:
    t0 = time.time()
    w = F.workload(3)
    prob = w.problem
    log(f"cfg3 inputs n={prob.n} nnz={prob.nnz} ({time.time() - t0:.0f}s)")
    h = hierarchy(w)
    log(f"cfg3 hierarchy levels {[lv.A.shape[0] for lv in h.levels]} ({time.time() - t0:.0f}s)")
    idx = sample(prob.n)
    z = O.vcycle(h, w.rhs)
    log(f"cfg3 V-cycle ({time.time() - t0:.0f}s)")
    _, k10, conv10, hist10, _ = O.pcg(h, w.rhs, rtol=1e-10)
    log(f"cfg3 PCG rtol 1e-10: {k10} iterations ({time.time() - t0:.0f}s)")
    x, k13, conv13, _, _ = O.pcg(h, w.rhs, rtol=1e-13)
    log(f"cfg3 PCG rtol 1e-13: {k13} iterations ({time.time() - t0:.0f}s)")
    assert conv10 and conv13
    return {"workload": w.name, "n": int(prob.n), "nnz": int(prob.nnz),
            "levels": [int(lv.A.shape[0]) for lv in h.levels], "idx": [int(i) for i in idx],
            "vcycle_z": vals(z, idx), "vcycle_z_norm": float(np.linalg.norm(z)),
            "iters_rtol_1e-10": int(k10), "residual_history_rtol_1e-10": [float(v) for v in hist10],
            "x_rtol_1e-13": vals(x, idx), "x_norm": float(np.linalg.norm(x)), "b_norm": float(np.linalg.norm(w.rhs))}


def cfg5() -> dict:
    t0 = time.time()
    w = F.workload(5)
    prob = w.problem
    ut = w.extra["target"]
    fd = np.asarray(w.extra["fd_cells"])
    kappa = np.exp(F.rng(5, F.PURPOSE_KAPPA).standard_normal(prob.cells.shape[0]))
    log(f"cfg5 inputs n={prob.n} cells={prob.cells.shape[0]} ({time.time() - t0:.0f}s)")
    h = hierarchy(w)
    log(f"cfg5 hierarchy levels {[lv.A.shape[0] for lv in h.levels]} ({time.time() - t0:.0f}s)")

    def solve(k, rhs):
        x, it, conv, _, _ = O.pcg(h, rhs, rtol=1e-13)
        assert conv
        log(f"cfg5 solve: {it} iterations ({time.time() - t0:.0f}s)")
        return x, None

    L, g, u, lam = O.loss_and_gradient(solve, prob.cells, prob.Ke, kappa, w.rhs, ut, prob.boundary)
    idx = sample(prob.n)
    cidx = sample(prob.cells.shape[0])
    return {"workload": w.name, "n": int(prob.n), "ncells": int(prob.cells.shape[0]),
            "levels": [int(lv.A.shape[0]) for lv in h.levels], "idx": [int(i) for i in idx],
            "u_rtol_1e-13": vals(u, idx), "u_norm": float(np.linalg.norm(u)), "loss": float(L),
            "fd_cells": [int(e) for e in fd], "grad_fd_cells": vals(g, fd),
            "cell_idx": [int(e) for e in cidx], "grad_cells": vals(g, cidx), "grad_norm": float(np.linalg.norm(g))}


def main(argv):
    which = [int(a) for a in argv] or [3, 5]
    for cfg in which:
        out = {3: cfg3, 5: cfg5}[cfg]()
        path = os.path.join(HERE, f"full_cfg{cfg}.json")
        with open(path, "w") as f:
            json.dump(out, f, separators=(",", ":"))
            f.write("\n")
        log(f"wrote {path} ({os.path.getsize(path)} bytes)")


if __name__ == "__main__":
    main(sys.argv[1:])
