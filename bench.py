"""Benchmark of the R3MG-C hot path on one MI355X.

Workload: 2D Poisson on the unit square, 256x256 quadrilaterals with seeded interior-vertex jitter of 0.2h,
continuous Q3 (769^2 = 591,361 DoFs), p'=2, leaf 128, 4 levels, V(2,2) Chebyshev-3 smoother, seeded Gaussian
nodal f, PCG to rtol 1e-10.  One step = one PCG solve from x0 = 0 with every input resident in HBM; the
headline runs the float32 V-cycle inside float64 CG, the plain float64 method is timed beside it.

Prints one JSON line (metric, value, ..., roofline, cpu_baseline).  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0     # MI355X HBM3E peak


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU (oracle) baseline leg")
    ap.add_argument("--scale", type=int, default=None, help="override N (cells per side) for quick runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import fixtures as F
    import paper_2607_28235_amd as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    t0 = time.time()
    w = F.workload(2, scale=args.scale)
    prob = w.problem
    log(f"inputs: n={prob.n} nnz={prob.nnz} ({time.time() - t0:.1f}s)")

    def make(fp32: int):
        o = P.Options(dim=2, coarse_degree=w.coarse_degree, leaf_size=w.leaf_size, max_levels=w.max_levels,
                      max_coarse_dofs=w.max_coarse_dofs, pre_steps=w.pre_steps, post_steps=w.post_steps,
                      vcycle_fp32=fp32)
        ta = time.time()
        h = P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o, factor=False)
        tb = time.time()
        h.factor()
        torch.cuda.synchronize()
        tc = time.time()
        return h, tb - ta, tc - tb

    h32, an32, fac32 = make(1)
    h64, an64, fac64 = make(0)
    log(f"setup fp32: analyze {an32:.2f}s factor {fac32:.2f}s; fp64: analyze {an64:.2f}s factor {fac64:.2f}s")
    info = h32.info()
    b = torch.from_numpy(w.rhs).to(dev)
    x = torch.zeros_like(b)

    def solve(h):
        x.zero_()
        it, rr, ok = h.pcg(b, x, rtol=1e-10, maxit=500)
        return int(it[0]), float(rr[0]), ok

    def timed(h, steps, warmup):
        for _ in range(warmup):
            solve(h)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        its = []
        for _ in range(steps):
            its.append(solve(h)[0])
        torch.cuda.synchronize()
        return (time.perf_counter() - ts) / steps, its

    t32, it32 = timed(h32, args.steps, args.warmup)
    x32 = x.cpu().numpy().copy()
    log(f"fp32 V-cycle: {t32 * 1e3:.3f} ms/solve, iters {it32[-1]}")
    t64, it64 = timed(h64, args.steps, args.warmup)
    x64 = x.cpu().numpy().copy()
    log(f"fp64 V-cycle: {t64 * 1e3:.3f} ms/solve, iters {it64[-1]}")

    # V-cycle time (hipEvents on torch's current stream, which the library launches on)
    r = torch.from_numpy(w.rhs).to(dev)
    z = torch.zeros_like(r)
    vc = {}
    for name, h in (("fp32", h32), ("fp64", h64)):
        for _ in range(3):
            h.vcycle(r, z)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 50
        e0.record()
        for _ in range(reps):
            h.vcycle(r, z)
        e1.record()
        e1.synchronize()
        vc[name] = e0.elapsed_time(e1) / reps
    lv_info = {"fp32": h32.info(), "fp64": h64.info()}

    def vcycle_bytes(inf, fp32):
        """Algorithmic bytes of one V-cycle: K(pre+post) operator applications per smoothed level (matrix,
        row pointers/block indices, 7 vector streams each), 4 transfer vector passes per level, the dense
        coarsest inverse (float64) and the entry/exit passes of the fine level."""
        K, nu = 3, w.pre_steps + w.post_steps
        s = 4 if fp32 else 8
        tot = 0.0
        for l, lv in enumerate(inf):
            if l < len(inf) - 1:
                tot += K * nu * lv["bytes_per_apply"]
                tot += 4 * lv["n"] * s
            else:
                tot += lv["n"] * lv["n"] * 8.0
        tot += 2 * prob.n * 8 + 3 * prob.n * s
        return tot

    vb = {k: vcycle_bytes(lv_info[k], k == "fp32") for k in vc}
    vgbs = {k: vb[k] / (vc[k] * 1e-3) / 1e9 for k in vc}
    log(f"V-cycle: fp32 {vc['fp32']:.3f} ms ({vgbs['fp32']:.0f} GB/s), fp64 {vc['fp64']:.3f} ms ({vgbs['fp64']:.0f} GB/s)")

    # dominant kernel: fused level-0 smoother step, timed live with hipEvents on the launch stream
    kms, kbytes = h32.time_smoother_kernel(0, 200)
    kgbs = kbytes / (kms * 1e-3) / 1e9
    per_level = []
    for l in range(len(info) - 1):
        ms_l, by_l = h32.time_smoother_kernel(l, 100)
        per_level.append({"level": l, "n": info[l]["n"], "nnz": info[l]["nnz"], "us_per_launch": ms_l * 1e3,
                          "bytes_per_launch": by_l, "GBps": by_l / (ms_l * 1e-3) / 1e9})
    log(f"level-0 fp32 smoother kernel: {kms * 1e3:.1f} us, {kgbs:.0f} GB/s")

    # CPU baseline: the FP64 oracle, same inputs, timed on the host cores
    cpu = None
    err = {}
    if not args.no_cpu:
        import oracle as O
        import threadpoolctl
        ta = time.time()
        ho = O.build_hierarchy(prob.coords, prob.scipy(), coarse_degree=w.coarse_degree, leaf_size=w.leaf_size,
                               max_levels=w.max_levels, max_coarse_dofs=w.max_coarse_dofs,
                               pre_steps=w.pre_steps, post_steps=w.post_steps)
        t_set = time.time() - ta
        ta = time.time()
        xo, ko, conv, _, _ = O.pcg(ho, w.rhs, rtol=1e-10)
        t_sol = time.time() - ta
        # sparse products run on one thread; the dense coarsest solves use the BLAS pool
        cores = max([d.get("num_threads", 1) for d in threadpoolctl.threadpool_info()] + [1])
        cpu = {"value": prob.n / t_sol, "unit": "DoF/s", "cores": cores, "kind": "oracle",
               "sample": f"one full FP64 oracle PCG solve of the same 591,361-DoF system (rtol 1e-10, {ko} "
                         f"iterations, {t_sol:.1f}s; oracle set-up {t_set:.1f}s excluded)",
               "iters": ko}
        err = {"fp32_vs_oracle": float(np.linalg.norm(x32 - xo) / np.linalg.norm(xo)),
               "fp64_vs_oracle": float(np.linalg.norm(x64 - xo) / np.linalg.norm(xo))}
        log(f"oracle: {t_sol:.1f}s solve, {ko} iters; errors {err}")

    out = {
        "metric": "DoF/s solved to rtol 1e-10 (FP32 V-cycle in FP64 CG)",
        "value": prob.n / t32,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 V-cycle / f64 CG",
        "data": "synthetic",
        "config": {"workload": w.name, "n": prob.n, "nnz": prob.nnz, "levels": len(info),
                   "level_sizes": [lv["n"] for lv in info], "rtol": 1e-10, "parallelism": "single GPU"},
        "iters_fp32": it32[-1],
        "iters_fp64": it64[-1],
        "fp64_value": prob.n / t64,
        "fp64_ms_per_step": t64 * 1e3,
        "speedup_fp32_over_fp64": t64 / t32,
        "setup_s": {"fp32": {"analyze": an32, "factor": fac32}, "fp64": {"analyze": an64, "factor": fac64}},
        "vcycle_ms": vc,
        "vcycle_GBps": vgbs,
        "vcycle_frac_of_peak": {k: v / PEAK_HBM_GBS for k, v in vgbs.items()},
        "smoother_kernel_per_level_fp32": per_level,
        "solution_rel_diff": err,
        "roofline": {"bound": "hbm", "achieved": kgbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": kgbs / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "k_level<float,1,false> (fine-level fused SpMV + Chebyshev step)",
                     "bytes_per_launch": kbytes, "us_per_launch": kms * 1e3},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
