"""Full-size parity of the 3D workloads on the GPU against the oracle, through the C ABI.

The oracle needs minutes at these sizes, so its outputs were computed once by tests/golden/make_full_size_oracle.py
(which calls only the oracle) and stored for 1024 seeded indices, with the norms and counts the checks need:

  3D Poisson Q2 64^3 (2,146,689 DoFs), p'=2, leaf 256, leaf level skipped, <= 2000 coarse DoFs, V(2,2), in the
  configuration the benchmark times: the level sizes; one float64 V-cycle (sampled entries to 1e-11 relative);
  PCG to rtol 1e-10 in both V-cycle precisions: iterations within one of the oracle's, the solution within 1e-9
  of the oracle's rtol-1e-13 solution, the true residual at the stop rule.
  -div(kappa grad u) = 1 on the same cube, lognormal kappa per cell (262,144 cells): the forward solution and
  the loss against the oracle, the adjoint gradient against the oracle's at the 32 seeded cells and at 1024
  sampled cells, central differences on the 32 cells, and the Euler identity sum_e kappa_e g_e = -(u - u_t)^T u.

The host analysis of the cube (partition, box bounds, fine transfer) is compared with the oracle's in full.

A relative 2-norm error is estimated from the samples: sqrt(n / m * sum over the m samples of the squared
difference) / (the reference's 2-norm).
"""
import json
import os
import sys

import numpy as np
import pytest

import fixtures as F

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _case(name):
    print(f"[gpu-case] {name}", flush=True)
    sys.stdout.flush()


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _gold(cfg):
    with open(os.path.join(GOLDEN, f"full_cfg{cfg}.json")) as f:
        return json.load(f)


def _sampled_rel(x, idx, ref, ref_norm, n):
    d = np.asarray(x)[idx] - np.asarray(ref)
    return float(np.sqrt(n / len(idx) * float(d @ d)) / ref_norm)


@pytest.fixture(scope="module")
def cube():
    _need_gpu()
    _case("full-size 3D Q2 64^3 inputs")
    w = F.workload(3)
    return w, _gold(3)


def test_full_size_3d_q2_partition(cube):
    """Host analysis of the same cube (no device work): constrained set, level sizes, every level's partition and
    box bounds and the fine transfer's sparsity bit-exact against the oracle, its values to 1e-15 (the oracle's
    Galerkin products are left out at this size; the V-cycle tests below compare the operators' action)."""
    import paper_2607_28235_amd as P
    from oracle import hierarchy as OH, rtree as ORT
    w, gold = cube
    prob = w.problem
    _case("full-size 3D Q2 64^3 partition against the oracle")
    h = P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val,
                    P.Options(dim=3, coarse_degree=w.coarse_degree, leaf_size=w.leaf_size,
                              max_coarse_dofs=w.max_coarse_dofs, skip_leaf_level=int(w.skip_leaf_level)),
                    factor=False)
    C = OH.constrained_set(prob.scipy())
    np.testing.assert_array_equal(C, prob.boundary)
    tree = ORT.bisection_rtree(prob.coords, w.leaf_size)
    B = (w.coarse_degree + 1) ** 3
    depths = ORT.select_levels(tree, 3, B, max_levels=w.max_levels, max_coarse_dofs=w.max_coarse_dofs,
                               skip_leaf_level=bool(w.skip_leaf_level))
    info = h.info()
    assert [lv["n"] for lv in info] == gold["levels"] and len(info) == len(depths) + 1
    for l, dep in enumerate(depths, start=1):
        own, lo, hi = h.export_partition(l)
        olo, ohi = tree.boxes(prob.coords, dep)
        np.testing.assert_array_equal(own, tree.owner(dep))
        np.testing.assert_array_equal(lo, olo)
        np.testing.assert_array_equal(hi, ohi)
        assert info[l]["n"] == olo.shape[0] * B
    olo, ohi = tree.boxes(prob.coords, depths[0])
    ip, ix, dt = OH.prolongation_fine(prob.coords, C, tree.owner(depths[0]), olo, ohi, w.coarse_degree)
    rp, cl, vl = h.export_P(0)
    np.testing.assert_array_equal(rp, ip)
    np.testing.assert_array_equal(cl, ix)
    np.testing.assert_allclose(vl, dt, rtol=0, atol=1e-15)
    h.close()


@pytest.mark.parametrize("fp32", [0, 1])
def test_full_size_3d_q2(cube, fp32):
    import paper_2607_28235_amd as P
    w, gold = cube
    prob = w.problem
    assert prob.n == gold["n"] and prob.nnz == gold["nnz"]
    _case(f"full-size 3D Q2 64^3 set-up fp32={fp32}")
    o = P.Options(dim=3, coarse_degree=w.coarse_degree, leaf_size=w.leaf_size, max_levels=w.max_levels,
                  max_coarse_dofs=w.max_coarse_dofs, pre_steps=w.pre_steps, post_steps=w.post_steps,
                  skip_leaf_level=int(w.skip_leaf_level), vcycle_fp32=fp32)
    h = P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o)
    info = h.info()
    assert [lv["n"] for lv in info] == gold["levels"]
    print("  kernels:", [lv["kernel"] for lv in info], flush=True)
    idx = np.asarray(gold["idx"])
    b = _t(w.rhs)
    if not fp32:
        _case("full-size 3D Q2 64^3 float64 V-cycle")
        z = torch.zeros_like(b)
        h.vcycle(b, z)
        torch.cuda.synchronize()
        zz = z.cpu().numpy()
        assert _sampled_rel(zz, idx, gold["vcycle_z"], gold["vcycle_z_norm"], prob.n) < 1e-11
        assert abs(np.linalg.norm(zz) - gold["vcycle_z_norm"]) <= 1e-11 * gold["vcycle_z_norm"]
    _case(f"full-size 3D Q2 64^3 PCG fp32={fp32}")
    x = torch.zeros_like(b)
    iters, relres, ok = h.pcg(b, x, rtol=1e-10, maxit=200)
    assert ok
    assert abs(int(iters[0]) - gold["iters_rtol_1e-10"]) <= 1, (iters, gold["iters_rtol_1e-10"])
    xx = x.cpu().numpy()
    err = _sampled_rel(xx, idx, gold["x_rtol_1e-13"], gold["x_norm"], prob.n)
    print(f"  iterations {int(iters[0])} (oracle {gold['iters_rtol_1e-10']}), sampled error {err:.2e}", flush=True)
    assert err < 1e-9
    r = w.rhs - prob.scipy() @ xx
    assert np.linalg.norm(r) <= 1.01e-10 * gold["b_norm"]
    if not fp32:
        # the recursion's residual history follows the oracle's (same recursion up to rounding)
        hist = h.history(0)
        ref = np.asarray(gold["residual_history_rtol_1e-10"])
        m = min(len(hist), len(ref))
        np.testing.assert_allclose(hist[:m], ref[:m], rtol=1e-3, atol=1e-12 * ref[0])
    h.close()


def test_full_size_kappa_gradient():
    """Forward and adjoint solves at rtol 1e-12 on the 262,144-cell lognormal-kappa cube."""
    _need_gpu()
    import paper_2607_28235_amd as P
    gold = _gold(5)
    _case("full-size kappa cube inputs")
    w = F.workload(5)
    prob = w.problem
    assert prob.n == gold["n"]
    kappa = np.exp(F.rng(5, F.PURPOSE_KAPPA).standard_normal(prob.cells.shape[0]))
    ut = w.extra["target"]
    fd_cells = np.asarray(w.extra["fd_cells"])
    assert list(fd_cells) == gold["fd_cells"]
    _case("full-size kappa cube set-up")
    o = P.Options(dim=3, coarse_degree=w.coarse_degree, leaf_size=w.leaf_size, max_levels=w.max_levels,
                  max_coarse_dofs=w.max_coarse_dofs, pre_steps=w.pre_steps, post_steps=w.post_steps,
                  skip_leaf_level=int(w.skip_leaf_level))
    op = P.AdjointPoisson(prob.coords, prob.row_ptr, prob.col, prob.val, prob.cells, prob.Ke,
                          prob.mass_rhs_weights, o, rtol=1e-12)
    assert [lv["n"] for lv in op.h.info()] == gold["levels"]
    _case("full-size kappa cube forward and adjoint")
    kt = _t(kappa).requires_grad_(True)
    u = op(kt)
    L = 0.5 * torch.sum((u - _t(ut)) ** 2)
    L.backward()
    g = kt.grad.cpu().numpy()
    un = u.detach().cpu().numpy()
    idx = np.asarray(gold["idx"])
    assert _sampled_rel(un, idx, gold["u_rtol_1e-13"], gold["u_norm"], prob.n) < 1e-9
    assert abs(float(L.detach()) - gold["loss"]) <= 1e-9 * gold["loss"]
    cidx = np.asarray(gold["cell_idx"])
    gerr = _sampled_rel(g, cidx, gold["grad_cells"], gold["grad_norm"], len(kappa))
    print(f"  gradient sampled error {gerr:.2e}", flush=True)
    assert gerr < 1e-9
    np.testing.assert_allclose(g[fd_cells], gold["grad_fd_cells"], rtol=1e-8,
                               atol=1e-9 * np.abs(gold["grad_fd_cells"]).max())
    # Euler identity (A is homogeneous of degree 1 in kappa on the unconstrained rows)
    lhs = float(kappa @ g)
    rhs = -float((un - ut) @ un)
    assert abs(lhs - rhs) <= 1e-9 * abs(rhs)
    # central differences in the difference form on the 32 seeded cells
    _case("full-size kappa cube central differences on 32 cells")
    worst = 0.0
    for e in fd_cells:
        hstep = 1e-3 * kappa[e]
        nodes = prob.cells[e]
        Ke = prob.Ke if prob.Ke.ndim == 2 else prob.Ke[e]
        Ku = Ke @ un[nodes]
        dL = []
        for sgn in (1.0, -1.0):
            kp = kappa.copy()
            kp[e] += sgn * hstep
            op.set_kappa(_t(kp))
            rhs_v = np.zeros(prob.n)
            np.add.at(rhs_v, nodes, -sgn * hstep * Ku)
            rhs_v[prob.boundary] = 0.0
            du, _ = op.solve_field(_t(rhs_v))
            du = du.cpu().numpy()
            dL.append((un - ut) @ du + 0.5 * du @ du)
        op.invalidate()
        fd = (dL[0] - dL[1]) / (2 * hstep)
        scale = max(abs(g[e]), 1e-3 * np.abs(g).max())
        worst = max(worst, abs(fd - g[e]) / scale)
        assert abs(fd - g[e]) <= 1e-6 * scale, (int(e), fd, g[e])
    print(f"  worst central-difference disagreement {worst:.2e}", flush=True)
