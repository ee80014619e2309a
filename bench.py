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
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_fine_kernels_2d_q3_591k.md")


def recorded_traffic(kernel: str):
    """HBM bytes per launch of the fine-level fused kernel from the committed rocprofv3 --pmc summary (FETCH_SIZE
    and WRITE_SIZE scaled by a plain-copy calibration), or None if the kernel source changed since or the
    summary covers another row-block shape than the one this run chose."""
    import hashlib
    try:
        md = open(TRAFFIC_PROFILE).read()
        src = open(os.path.join(ROOT, "paper_2607_28235_amd", "csrc", "kernels.hip")).read()
    except OSError:
        return None
    i = src.find("// ==== fine-level row-block kernels ====")
    j = src.find("// ==== end of fine-level row-block kernels ====", i)
    if i < 0 or j < 0:
        return None
    h = hashlib.sha256(src[i:j].encode()).hexdigest()
    rec = dict(line.split(": ", 1) for line in md.splitlines() if ": " in line and not line.startswith("|"))
    key = f"traffic[{kernel}]"
    if rec.get("kernel_source_sha256", "").strip() != h or key not in rec:
        return None
    return float(rec[key])


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU (oracle) baseline leg")
    ap.add_argument("--scale", type=int, default=None, help="override N (cells per side) for quick runs")
    ap.add_argument("--workload", default="solve2d",
                    choices=["solve2d", "solve3d", "batch16", "uneven8", "adjoint", "replicate", "matfree"],
                    help="solve2d: the headline (591k-DoF Q3 square); batch16: 16-RHS block PCG on the 48^3 Q3 "
                         "cube; uneven8: 8 Q2 cubes of 16^3..48^3 in one graph; adjoint: kappa-gradient on 64^3 Q2")
    ap.add_argument("--fd-cells", type=int, default=32)
    ap.add_argument("--matfree", action="store_true",
                    help="batch16: also time the solves with the matrix-free fine operator")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (the HBM-counter calibration kernel)")
    ap.add_argument("--fine-kernel", type=int, default=-1,
                    help="pin the fine-level row-block shape (0..12; -1: chosen by timing at set-up), e.g. for "
                         "hardware-counter runs that must see one kernel")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU runs are not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload not in ("solve2d", "solve3d"):
        {"batch16": bench_batch16, "uneven8": bench_uneven8, "adjoint": bench_adjoint,
         "replicate": bench_replicate, "matfree": bench_matfree}[args.workload](args)
        return

    import torch
    import fixtures as F
    import paper_2607_28235_amd as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    t0 = time.time()
    w = F.workload(2 if args.workload == "solve2d" else 3, scale=args.scale)
    prob = w.problem
    log(f"inputs: n={prob.n} nnz={prob.nnz} ({time.time() - t0:.1f}s)")

    def make(fp32: int):
        o = P.Options(dim=prob.d, coarse_degree=w.coarse_degree, leaf_size=w.leaf_size, max_levels=w.max_levels,
                      max_coarse_dofs=w.max_coarse_dofs, pre_steps=w.pre_steps, post_steps=w.post_steps,
                      vcycle_fp32=fp32, skip_leaf_level=w.skip_leaf_level, fine_kernel=args.fine_kernel)
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
        """Mean time per solve over exactly `steps` solves (synchronised on both sides), and each solve's own
        wall time (every solve ends synchronised: the library reads its state back)."""
        for _ in range(warmup):
            solve(h)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        its, each = [], []
        for _ in range(steps):
            t1 = time.perf_counter()
            its.append(solve(h)[0])
            each.append(time.perf_counter() - t1)
        torch.cuda.synchronize()
        return (time.perf_counter() - ts) / steps, its, each

    def spread(each):
        a = np.asarray(each) * 1e3
        return {"median": float(np.median(a)), "min": float(a.min()), "max": float(a.max())}

    t32, it32, each32 = timed(h32, args.steps, args.warmup)
    x32 = x.cpu().numpy().copy()
    log(f"fp32 V-cycle: {t32 * 1e3:.3f} ms/solve ({spread(each32)}), iters {it32[-1]}")
    t64, it64, each64 = timed(h64, args.steps, args.warmup)
    x64 = x.cpu().numpy().copy()
    log(f"fp64 V-cycle: {t64 * 1e3:.3f} ms/solve ({spread(each64)}), iters {it64[-1]}")

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

    def apply_bytes(lv, l, s):
        """Algorithmic bytes of one operator application with the fused Chebyshev update: the matrix with a
        4-byte index per nonzero (CSR, fine level) or per stored B x B block (coarse levels), 4-byte row or
        block-row pointers, and 7 vector streams (u read, x read and written, rho read and written, D^-1, d)."""
        if l == 0:
            return lv["nnz"] * (s + 4) + 4 * (lv["n"] + 1) + 7 * lv["n"] * s
        B = (w.coarse_degree + 1) ** prob.d
        return lv["nnz"] * s + 4 * lv["nnz"] / (B * B) + 4 * (lv["nboxes"] + 1) + 7 * lv["n"] * s

    def vcycle_bytes(inf, fp32, stored):
        """Algorithmic bytes of one V-cycle: K(pre+post) operator applications per smoothed level (apply_bytes,
        or with stored=True the bytes of the storage format the library reports), 4 transfer vector passes per
        level, the dense coarsest inverse (float64) and the entry/exit passes of the fine level."""
        K, nu = 3, w.pre_steps + w.post_steps
        s = 4 if fp32 else 8
        tot = 0.0
        for l, lv in enumerate(inf):
            if l < len(inf) - 1:
                tot += K * nu * (lv["bytes_per_apply"] if stored else apply_bytes(lv, l, s))
                tot += 4 * lv["n"] * s
            else:
                tot += lv["n"] * lv["n"] * 8.0
        tot += 2 * prob.n * 8 + 3 * prob.n * s
        return tot

    vb = {k: vcycle_bytes(lv_info[k], k == "fp32", False) for k in vc}
    vgbs = {k: vb[k] / (vc[k] * 1e-3) / 1e9 for k in vc}
    vb_stored = {k: vcycle_bytes(lv_info[k], k == "fp32", True) for k in vc}
    log(f"V-cycle: fp32 {vc['fp32']:.3f} ms ({vgbs['fp32']:.0f} GB/s), fp64 {vc['fp64']:.3f} ms ({vgbs['fp64']:.0f} GB/s)")

    # dominant kernel: fused level-0 smoother step, timed live with hipEvents on the launch stream, back to back
    # as a smoothing sweep runs it, and alone after a 1 GiB pass that evicts the caches (HBM only)
    kms, kbytes = h32.time_smoother_kernel(0, 200)
    kms_cold, _ = h32.time_smoother_kernel(0, 40, flush_bytes=1 << 30)
    abytes = apply_bytes(info[0], 0, 4)
    kgbs = abytes / (kms * 1e-3) / 1e9
    kgbs_cold = abytes / (kms_cold * 1e-3) / 1e9
    per_level = []
    for l in range(len(info) - 1):
        ms_l, by_l = h32.time_smoother_kernel(l, 100)
        per_level.append({"level": l, "kernel": info[l]["kernel"], "n": info[l]["n"], "nnz": info[l]["nnz"],
                          "us_per_launch": ms_l * 1e3,
                          "bytes_per_launch": by_l, "GBps": by_l / (ms_l * 1e-3) / 1e9})
    log(f"level-0 fp32 smoother kernel: {kms * 1e3:.1f} us back to back, {kms_cold * 1e3:.1f} us from HBM; "
        f"{abytes / 1e6:.1f} MB algorithmic ({kbytes / 1e6:.1f} MB as stored): {kgbs:.0f} / {kgbs_cold:.0f} GB/s")

    # CPU baseline: the FP64 oracle, same inputs, timed on the host cores
    cpu = None
    err = {}
    if not args.no_cpu:
        import oracle as O
        import threadpoolctl
        ta = time.time()
        ho = O.build_hierarchy(prob.coords, prob.scipy(), coarse_degree=w.coarse_degree, leaf_size=w.leaf_size,
                               max_levels=w.max_levels, max_coarse_dofs=w.max_coarse_dofs,
                               pre_steps=w.pre_steps, post_steps=w.post_steps,
                               skip_leaf_level=bool(w.skip_leaf_level))
        t_set = time.time() - ta
        # repeat the whole solve until about 10 s of CPU work have been timed (one solve takes ~1 s)
        reps, t_tot = 0, 0.0
        while t_tot < 10.0 and reps < 30:
            ta = time.time()
            xo, ko, conv, _, _ = O.pcg(ho, w.rhs, rtol=1e-10)
            t_tot += time.time() - ta
            reps += 1
        t_sol = t_tot / reps
        # the reference solution of the accuracy check: the oracle solved to rtol 1e-13 (not timed)
        x_ref = O.pcg(ho, w.rhs, rtol=1e-13)[0]
        # sparse products run on one thread; the dense coarsest solves use the BLAS pool
        cores = max([d.get("num_threads", 1) for d in threadpoolctl.threadpool_info()] + [1])
        cpu = {"value": prob.n / t_sol, "unit": "DoF/s", "cores": cores, "kind": "oracle",
               "sample": f"{reps} full FP64 oracle PCG solves of the same {prob.n:,}-DoF system (rtol 1e-10, {ko} "
                         f"iterations, {t_tot:.1f}s in total, {t_sol:.2f}s each; oracle set-up {t_set:.1f}s "
                         f"excluded)",
               "iters": ko}
        err = {"fp32_vs_oracle_rtol1e-13": float(np.linalg.norm(x32 - x_ref) / np.linalg.norm(x_ref)),
               "fp64_vs_oracle_rtol1e-13": float(np.linalg.norm(x64 - x_ref) / np.linalg.norm(x_ref)),
               "fp32_vs_oracle_rtol1e-10": float(np.linalg.norm(x32 - xo) / np.linalg.norm(xo)),
               "fp64_vs_oracle_rtol1e-10": float(np.linalg.norm(x64 - xo) / np.linalg.norm(xo))}
        log(f"oracle: {t_sol:.1f}s solve, {ko} iters; errors {err}")

    out = {
        "metric": "DoF/s solved to rtol 1e-10 (FP32 V-cycle in FP64 CG)",
        "value": prob.n / t32,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t32 * 1e3,
        "ms_per_step_spread": spread(each32),
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
        "fp64_ms_per_step_spread": spread(each64),
        "speedup_fp32_over_fp64": t64 / t32,
        "setup_s": {"fp32": {"analyze": an32, "factor": fac32}, "fp64": {"analyze": an64, "factor": fac64}},
        "vcycle_ms": vc,
        "vcycle_GBps": vgbs,
        "vcycle_frac_of_peak": {k: v / PEAK_HBM_GBS for k, v in vgbs.items()},
        "vcycle_GBps_as_stored": {k: vb_stored[k] / (vc[k] * 1e-3) / 1e9 for k in vc},
        "smoother_kernel_per_level_fp32": per_level,
        "solution_rel_diff": err,
        "roofline": {"bound": "hbm", "achieved": kgbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": kgbs / PEAK_HBM_GBS,
                     "traffic": (recorded_traffic(info[0]["kernel"])
                                 if (args.workload == "solve2d" and args.scale is None) else None),
                     "kernel": info[0]["kernel"] + " (fine-level fused SpMV + Chebyshev step)",
                     "bytes_per_launch": abytes, "us_per_launch": kms * 1e3,
                     "bytes_per_launch_as_stored": kbytes,
                     "frac_as_stored": kbytes / (kms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                     "hbm_only": {"us_per_launch": kms_cold * 1e3, "achieved": kgbs_cold,
                                  "frac": kgbs_cold / PEAK_HBM_GBS,
                                  "method": "each launch timed alone after a 1 GiB read+write pass"}},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if args.copy_calibration:
        _copy_calibration(torch)


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    out = None
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - ts) / steps, out


def bench_batch16(args):
    """Block PCG over 16 seeded right-hand sides in lockstep (float32 V-cycle, float64 CG) on the 3D Q3 cube
    (48^3 cells, 3,048,625 DoFs), with the SpMM tiles chosen by the library's autotuner; compared with one
    right-hand side at a time on the same hierarchy."""
    import torch
    import fixtures as F
    import paper_2607_28235_amd as P
    t0 = time.time()
    w = F.workload(4, scale=args.scale)
    prob = w.problem
    log(f"inputs: n={prob.n} nnz={prob.nnz} 16 rhs ({time.time() - t0:.1f}s)")
    o = P.Options(dim=3, coarse_degree=2, leaf_size=256, max_coarse_dofs=2000, vcycle_fp32=1,
                  skip_leaf_level=w.skip_leaf_level)
    ta = time.time()
    h = P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o)
    torch.cuda.synchronize()
    t_setup = time.time() - ta
    info = h.info()
    log(f"setup {t_setup:.1f}s levels {[lv['n'] for lv in info]}")
    B = torch.from_numpy(w.rhs).to("cuda")
    X = torch.zeros_like(B)

    def solve16():
        X.zero_()
        return h.pcg(B, X, rtol=1e-10, maxit=500)
    t16, (it16, rr16, ok16) = _timed(solve16, args.steps, args.warmup)
    x1 = torch.zeros(prob.n, dtype=torch.float64, device="cuda")
    b0 = B[0].contiguous()

    def solve1():
        x1.zero_()
        return h.pcg(b0, x1, rtol=1e-10, maxit=500)
    t1, (it1, _, _) = _timed(solve1, args.steps, args.warmup)
    R = (B - 0).cpu().numpy()
    Xh = X.cpu().numpy()
    res = np.linalg.norm(R - (prob.scipy() @ Xh.T).T, axis=1) / np.linalg.norm(R, axis=1)
    log(f"16 rhs: {t16 * 1e3:.1f} ms ({16 * prob.n / t16:.3e} DoF/s), 1 rhs: {t1 * 1e3:.1f} ms")
    # dominant kernel: the fine-level fused smoother step for 16 columns (the tuned multi-RHS kernel), timed live
    # with hipEvents on the launch stream, back to back and alone after a 1 GiB pass that evicts the caches.
    # Algorithmic bytes: the matrix once with a 4-byte index per nonzero, row pointers, 7 vector streams of 16
    # float32 columns.
    kms, kbytes = h.time_smoother_kernel(0, 40, nrhs=16)
    kms_cold, _ = h.time_smoother_kernel(0, 10, flush_bytes=1 << 30, nrhs=16)
    abytes = info[0]["nnz"] * (4 + 4) + 4 * (prob.n + 1) + 7 * prob.n * 4 * 16
    kgbs, kgbs_cold = abytes / (kms * 1e-3) / 1e9, abytes / (kms_cold * 1e-3) / 1e9
    log(f"level-0 16-rhs fp32 smoother kernel: {kms * 1e3:.1f} us back to back, {kms_cold * 1e3:.1f} us from HBM; "
        f"{abytes / 1e6:.1f} MB algorithmic ({kbytes / 1e6:.1f} MB as stored): {kgbs:.0f} / {kgbs_cold:.0f} GB/s")
    roofline = {"bound": "hbm", "achieved": kgbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": kgbs / PEAK_HBM_GBS,
                "traffic": None, "kernel": "fine-level fused SpMV + Chebyshev step, 16 float32 columns",
                "bytes_per_launch": abytes, "us_per_launch": kms * 1e3, "bytes_per_launch_as_stored": kbytes,
                "frac_as_stored": kbytes / (kms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                "hbm_only": {"us_per_launch": kms_cold * 1e3, "achieved": kgbs_cold, "frac": kgbs_cold / PEAK_HBM_GBS,
                             "method": "each launch timed alone after a 1 GiB read+write pass"}}
    mf = None
    if args.matfree:
        # the same solves with the matrix-free fine operator (cell kernel looping over the 16 columns)
        ta = time.time()
        h.set_matrix_free(prob.cells, prob.p)
        t_att = time.time() - ta
        t16m, (it16m, _, ok16m) = _timed(solve16, args.steps, args.warmup)
        x16m = X.cpu().numpy()
        t1m, (it1m, _, _) = _timed(solve1, args.steps, args.warmup)
        resm = np.linalg.norm(R - (prob.scipy() @ x16m.T).T, axis=1) / np.linalg.norm(R, axis=1)
        mf = {"ms_16rhs": t16m * 1e3, "DoF_per_s_16rhs": 16 * prob.n / t16m, "iters": [int(i) for i in it16m],
              "all_converged": bool(ok16m), "max_true_relres": float(resm.max()), "ms_1rhs": t1m * 1e3,
              "speedup_over_csr_16rhs": t16 / t16m, "set_up_s": t_att,
              "solution_rel_diff_vs_csr": float(np.linalg.norm(x16m - Xh) / np.linalg.norm(Xh))}
        log(f"matrix-free: 16 rhs {t16m * 1e3:.1f} ms ({16 * prob.n / t16m:.3e} DoF/s), 1 rhs {t1m * 1e3:.1f} ms")
    print(json.dumps({
        "metric": "DoF/s solved to rtol 1e-10, 16 right-hand sides in lockstep (FP32 V-cycle in FP64 CG)",
        "value": 16 * prob.n / t16, "unit": "DoF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t16 * 1e3, "higher_is_better": True, "dtype": "f32 V-cycle / f64 CG",
        "config": {"workload": w.name, "n": prob.n, "nnz": prob.nnz, "nrhs": 16,
                   "level_sizes": [lv["n"] for lv in info]},
        "iters": [int(i) for i in it16], "max_true_relres": float(res.max()), "all_converged": bool(ok16),
        "single_rhs_ms": t1 * 1e3, "single_rhs_iters": int(it1[0]),
        "per_rhs_speedup_of_batching": 16 * t1 / t16, "setup_s": t_setup, "matrix_free": mf,
        "roofline": roofline}), flush=True)
    if args.copy_calibration:
        _copy_calibration(torch)


def bench_uneven8(args):
    """Eight independent 3D Q2 problems (16^3..48^3 cells, 35,937..912,673 DoFs) solved by PCG in one captured
    launch sequence (one graph branch per problem), compared with solving them one after another."""
    import torch
    import fixtures as F
    import paper_2607_28235_amd as P
    t0 = time.time()
    sizes = F.uneven_batch_sizes() if args.scale is None else [max(8, args.scale // 3 * k) for k in range(1, 9)]
    batch = F.uneven_batch(sizes)
    log(f"inputs: {[p.n for p, _ in batch]} ({time.time() - t0:.1f}s)")
    hs, bs, xs = [], [], []
    for prob, b in batch:
        o = P.Options(dim=3, coarse_degree=2, leaf_size=256, max_coarse_dofs=2000, vcycle_fp32=1,
                      skip_leaf_level=1)
        hs.append(P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o))
        bs.append(torch.from_numpy(b).to("cuda"))
        xs.append(torch.zeros(prob.n, dtype=torch.float64, device="cuda"))
    ntot = sum(p.n for p, _ in batch)

    def group():
        for x in xs:
            x.zero_()
        return P.solve_group(hs, bs, xs, rtol=1e-10, maxit=500)
    tg, (itg, rrg, okg) = _timed(group, args.steps, args.warmup)

    def seq():
        its = []
        for h, b, x in zip(hs, bs, xs):
            x.zero_()
            its.append(int(h.pcg(b, x, rtol=1e-10, maxit=500)[0][0]))
        return its
    ts, its = _timed(seq, args.steps, args.warmup)
    log(f"group {tg * 1e3:.1f} ms, sequential {ts * 1e3:.1f} ms")
    print(json.dumps({
        "metric": "DoF/s solved to rtol 1e-10, 8 uneven problems in one hipGraph launch sequence",
        "value": ntot / tg, "unit": "DoF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": tg * 1e3, "higher_is_better": True, "dtype": "f32 V-cycle / f64 CG",
        "config": {"workload": "3D Q2 Poisson cubes N^3, N in " + str(sizes), "n": [p.n for p, _ in batch]},
        "iters": [int(i) for i in itg], "all_converged": bool(okg), "sequential_ms": ts * 1e3,
        "sequential_iters": its, "speedup_over_sequential": ts / tg}), flush=True)


def bench_adjoint(args):
    """Forward and adjoint solves of -div(kappa grad u) = 1 on the 64^3 Q2 cube with lognormal per-cell kappa
    (262,144 cells): assembly, numeric re-set-up and PCG forward; adjoint PCG and per-cell gradient backward;
    the gradient is checked by central finite differences on seeded cells."""
    import torch
    import fixtures as F
    import paper_2607_28235_amd as P
    t0 = time.time()
    w = F.workload(5, scale=args.scale)
    prob = w.problem
    ut = torch.from_numpy(w.extra["target"]).to("cuda")
    log(f"inputs: n={prob.n} cells={prob.cells.shape[0]} ({time.time() - t0:.1f}s)")
    o = P.Options(dim=3, coarse_degree=2, leaf_size=256, max_coarse_dofs=2000, vcycle_fp32=1,
                  skip_leaf_level=w.skip_leaf_level)
    op = P.AdjointPoisson(prob.coords, prob.row_ptr, prob.col, prob.val, prob.cells, prob.Ke,
                          prob.mass_rhs_weights, o, rtol=1e-10)
    kappa = torch.from_numpy(prob.kappa).to("cuda")

    def fwd_bwd():
        k = kappa.clone().requires_grad_(True)
        u = op(k)
        L = 0.5 * torch.sum((u - ut) ** 2)
        L.backward()
        return k.grad, u, L
    # separate phase timings
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    for _ in range(args.warmup):
        fwd_bwd()
    tf, tb = [], []
    for _ in range(args.steps):
        k = (kappa * 1.0).requires_grad_(True)
        torch.cuda.synchronize()
        ev[0].record()
        u = op(k)
        ev[1].record()
        L = 0.5 * torch.sum((u - ut) ** 2)
        L.backward()
        ev[2].record()
        ev[2].synchronize()
        tf.append(ev[0].elapsed_time(ev[1]))
        tb.append(ev[1].elapsed_time(ev[2]))
    g = k.grad.cpu().numpy()
    uu = u.detach().cpu().numpy()
    kap = prob.kappa
    utn = w.extra["target"]
    euler = abs(kap @ g + (uu - utn) @ uu) / abs((uu - utn) @ uu)
    # central differences in the difference form: A(kappa +- h e_e) du = -+ h K_e u_e on the unconstrained rows,
    # L(kappa +- h) - L = (u - u_t).du + |du|^2 / 2 (no cancellation between two full solves)
    fd_err = []
    for e in w.extra["fd_cells"][:args.fd_cells]:
        hh = 1e-3 * kap[e]
        nodes = prob.cells[e]
        Ke = prob.Ke if prob.Ke.ndim == 2 else prob.Ke[e]
        Ku = Ke @ uu[nodes]
        dL = []
        for sgn in (1.0, -1.0):
            kp = kappa.clone()
            kp[e] += sgn * hh
            op.set_kappa(kp)
            rhs = np.zeros(prob.n)
            np.add.at(rhs, nodes, -sgn * hh * Ku)
            rhs[prob.boundary] = 0.0
            du, _ = op.solve_field(torch.from_numpy(rhs).to("cuda"))
            du = du.cpu().numpy()
            dL.append(float((uu - utn) @ du + 0.5 * du @ du))
        op.invalidate()
        fd = (dL[0] - dL[1]) / (2 * hh)
        fd_err.append(abs(fd - g[e]) / max(abs(g[e]), 1e-3 * np.abs(g).max()))
    log(f"forward {np.median(tf):.1f} ms, backward {np.median(tb):.1f} ms, FD max rel err {max(fd_err):.2e}")
    print(json.dumps({
        "metric": "forward+adjoint solve time (assembly, re-set-up, PCG; adjoint PCG, per-cell gradient)",
        "value": float(np.median(tf) + np.median(tb)), "unit": "ms", "higher_is_better": False, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "dtype": "f32 V-cycle / f64 CG",
        "config": {"workload": w.name, "n": prob.n, "ncells": int(prob.cells.shape[0])},
        "forward_ms": float(np.median(tf)), "backward_ms": float(np.median(tb)),
        "iters_forward_backward": list(op.last_iters), "euler_identity_rel": float(euler),
        "fd_cells": int(len(fd_err)), "fd_max_rel_err": float(max(fd_err)) if fd_err else None}), flush=True)


# Section 6.1 tables on the structured Q1 square (p' = 0 and 1), for context only -- the paper's R-tree (Boost's
# R*-tree, m = 2) differs from this library's bisection tree: per (agglomeration, table), rows of (refinements,
# levels, the paper's iterations and condition estimates for p' = 0, then for p' = 1).
# (ref, levels, paper iters / cond with the lower coarse degree, then with the higher one)
PAPER_Q1 = {
    ("point", "fixed_levels"): [(6, 2, 12, 3.84, 4, 1.04), (7, 2, 15, 4.30, 4, 1.04), (8, 2, 16, 4.48, 4, 1.04)],
    ("cell", "fixed_levels"): [(6, 2, 11, 3.63, 4, 1.03), (7, 2, 14, 3.98, 4, 1.02), (8, 2, 15, 4.08, 3, 1.01)],
    ("point", "growing_levels"): [(6, 3, 12, 5.11, 5, 1.07), (7, 4, 17, 9.70, 5, 1.19), (8, 5, 24, 18.52, 7, 1.54),
                                  (9, 6, 35, 36.37, 10, 2.16), (10, 7, 49, 71.66, 14, 3.73)],
    ("cell", "growing_levels"): [(6, 2, 11, 3.63, 4, 1.03), (7, 3, 15, 6.85, 4, 1.02), (8, 4, 22, 13.25, 4, 1.04),
                                 (9, 5, 30, 26.13, 6, 1.35), (10, 6, 42, 52.10, 8, 2.05)],
}
# Section 6, simplicial unit square with P1 elements, fixed levels (the paper's mesh starts from 942 triangles;
# refinement r has about 942 * 4^r triangles, matched here by N = 87 * 2^(r - 2) squares per side).  Two levels
# at a fixed H/h make the coarsest level grow with the mesh; refinements 5 and 6 would exceed the dense coarsest
# solve (R3MG_MAX_COARSEST_DOFS), where the paper uses a sparse direct solver.
PAPER_P1_SIMPLEX = {
    ("point", "fixed_levels"): [(2, 2, 16, 5.13, 5, 1.13), (3, 2, 19, 6.09, 5, 1.15), (4, 2, 21, 6.89, 5, 1.16)],
    ("cell", "fixed_levels"): [(2, 2, 17, 6.21, 5, 1.17), (3, 2, 21, 7.96, 7, 1.60), (4, 2, 22, 7.49, 6, 1.41)],
}


def bench_matfree(args):
    """Matrix-free fine operator against the CSR fine matrix on the 2D Q3 256^2 jittered square (591,361 DoFs,
    multilinear cells) and the 3D Q2 64^3 cube (2,146,689 DoFs, affine cells): solve time to rtol 1e-10 in both
    V-cycle precisions (median over the timed solves), the fused fine-level smoother step (both launches of the
    matrix-free form) and its algorithmic bytes."""
    import torch
    import fixtures as F
    import paper_2607_28235_amd as P
    rows = []
    for cfg in (2, 3):
        w = F.workload(cfg, scale=args.scale)
        prob = w.problem
        b = torch.from_numpy(w.rhs).cuda()
        for fp32 in (1, 0):
            o = P.Options(dim=prob.d, coarse_degree=w.coarse_degree, leaf_size=w.leaf_size, max_levels=w.max_levels,
                          max_coarse_dofs=w.max_coarse_dofs, pre_steps=w.pre_steps, post_steps=w.post_steps,
                          vcycle_fp32=fp32, skip_leaf_level=w.skip_leaf_level)
            h = P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o)
            row = {"workload": w.name, "n": prob.n, "vcycle": "fp32" if fp32 else "fp64"}
            xs = {}
            for mode in ("csr", "matrix_free"):
                if mode == "matrix_free":
                    ta = time.time()
                    h.set_matrix_free(prob.cells, prob.p)
                    row["matrix_free_setup_s"] = time.time() - ta
                x = torch.zeros_like(b)
                for _ in range(args.warmup):
                    x.zero_()
                    h.pcg(b, x, rtol=1e-10, maxit=500)
                # median of individually synchronised solves (robust to transient host-side noise)
                ts = []
                for _ in range(max(args.steps, 1)):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    x.zero_()
                    it, _, ok = h.pcg(b, x, rtol=1e-10, maxit=500)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                t = float(np.median(ts))
                kms, kby = h.time_smoother_kernel(0, 100)
                xs[mode] = x.cpu().numpy()
                row[mode] = {"ms_per_solve": t * 1e3, "DoF_per_s": prob.n / t, "iters": int(it[0]),
                             "converged": bool(ok), "fine_kernel": h.info()[0]["kernel"],
                             "fine_step_us": kms * 1e3, "fine_step_bytes": kby,
                             "fine_step_GBps": kby / (kms * 1e-3) / 1e9}
            row["solution_rel_diff"] = float(np.linalg.norm(xs["matrix_free"] - xs["csr"]) /
                                             np.linalg.norm(xs["csr"]))
            row["speedup"] = row["csr"]["ms_per_solve"] / row["matrix_free"]["ms_per_solve"]
            log(f"{w.name} {row['vcycle']}: CSR {row['csr']['ms_per_solve']:.2f} ms ({row['csr']['fine_step_us']:.1f} "
                f"us fine step), matrix-free {row['matrix_free']['ms_per_solve']:.2f} ms "
                f"({row['matrix_free']['fine_step_us']:.1f} us, {row['matrix_free']['fine_step_GBps']:.0f} GB/s), "
                f"iters {row['csr']['iters']}/{row['matrix_free']['iters']}, diff {row['solution_rel_diff']:.1e}")
            rows.append(row)
            h.close()
    print(json.dumps({"metric": "DoF/s solved to rtol 1e-10, matrix-free vs CSR fine operator", "unit": "DoF/s",
                      "n_gpus": 1, "data": "synthetic", "steps": args.steps, "warmup": args.warmup,
                      "rows": rows}), flush=True)
    if args.copy_calibration:
        _copy_calibration(torch)


def _copy_calibration(torch):
    """A plain elementwise copy of 256 MiB (the HBM-counter calibration kernel of the traffic profiles)."""
    src = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()


def _replicate_table(P, torch, family, tables, make, leaf, hmax_of):
    rows = []
    for (agg, table), spec in tables.items():
        for ref, lv, pit0, pcond0, pit1, pcond1 in spec:
            prob, b_np = make(ref)
            b = torch.from_numpy(b_np).cuda()
            row = {"family": family, "agglomeration": agg, "table": table, "ref": ref, "dofs": prob.n,
                   "levels": lv, "paper": {"iters_p0": pit0, "cond_p0": pcond0, "iters_p1": pit1, "cond_p1": pcond1}}
            for pc in (0, 1):
                o = P.Options(dim=2, coarse_degree=pc, leaf_size=leaf[agg], max_levels=lv,
                              max_coarse_dofs=1, skip_leaf_level=1, vcycle_fp32=0)
                h = P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o,
                                cells=prob.cells if agg == "cell" else None)
                info = h.info()
                x = torch.zeros_like(b)
                it, _, ok, cond = h.pcg(b, x, rtol=1e-6, atol=1e-9, maxit=500, return_cond=True)
                t = _timed(lambda: (x.zero_(), h.pcg(b, x, rtol=1e-6, atol=1e-9, maxit=500)), 3, 1)[0]
                row[f"p{pc}"] = {"iters": int(it[0]), "cond": float(cond[0]), "converged": bool(ok),
                                 "H_over_h": info[-1]["max_box_extent"] / hmax_of(prob, ref),
                                 "levels": len(info), "solve_ms": t * 1e3}
                h.close()
            log(f"{family} {agg} {table} ref {ref} n={prob.n} lvls {lv}: p'=0 {row['p0']['iters']} it (cond "
                f"{row['p0']['cond']:.2f}), p'=1 {row['p1']['iters']} it (cond {row['p1']['cond']:.2f}), H/h "
                f"{row['p1']['H_over_h']:.2f}; paper {pit0}/{pit1}")
            rows.append(row)
    return rows


def bench_replicate(args):
    """Paper-replication mode, PCG stopped at a 1e-6 reduction or 1e-9 absolute, V(2,2) Chebyshev-3, the leaf
    level skipped:
    - the structured Q1 square tables of Section 6.1 (fixed levels, then levels growing with the refinement),
      leaf size 8 points (point-based) or 4 cells (cell-based, the paper's m_cells = 2);
    - the simplicial P1 square table with fixed levels (Section 6), leaf size 4 points (m_points = 2) or
      16 cells (m_cells = 4), on a jittered structured triangulation standing in for the paper's unstructured
      one (H/h against the longest triangle edge)."""
    import torch
    import fixtures as F
    import paper_2607_28235_amd as P

    def q1(ref):
        prob = F.structured_qp(2, 2 ** ref, 1, cfg=1)
        return prob, F.nodal_rhs(prob, F.rng(1, F.PURPOSE_RHS, ref).uniform(-1, 1, prob.n), cfg=1)

    def p1_simplex(ref):
        prob = F.simplicial_pp(87 * 2 ** (ref - 2), 1, jitter=0.2, cfg=2)
        return prob, F.nodal_rhs(prob, F.rng(2, F.PURPOSE_RHS, ref).uniform(-1, 1, prob.n))

    rows = _replicate_table(P, torch, "structured_q1_square", PAPER_Q1, q1, {"point": 8, "cell": 4},
                            lambda prob, ref: np.sqrt(2.0) / 2 ** ref)   # cell diagonal of the uniform mesh
    rows += _replicate_table(P, torch, "simplicial_p1_square", PAPER_P1_SIMPLEX, p1_simplex,
                             {"point": 4, "cell": 16}, lambda prob, ref: prob.h)
    print(json.dumps({"metric": "paper replication: PCG iterations and condition estimates",
                      "unit": "iterations", "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": "Section 6.1 structured Q1 square (point leaf 8, cell leaf 4) and "
                                             "simplicial P1 square (point leaf 4, cell leaf 16), skip leaf level, "
                                             "V(2,2) Chebyshev-3, stop 1e-6 reduction or 1e-9 absolute"},
                      "rows": rows}), flush=True)


if __name__ == "__main__":
    main()
