"""GPU checks of the batched (multi-RHS, autotuned SpMM, grouped hipGraph) and differentiated solves against
the FP64 oracle."""
import sys

import numpy as np
import pytest

import fixtures as F
import oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(name):
    print(f"[gpu-case] {name}", flush=True)
    sys.stdout.flush()


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def small3d_q3():
    _need_gpu()
    _case("small3d_q3 setup (3D Q3 8^3, 16 RHS, p'=2, leaf 256)")
    w = F.workload(4, scale=8)
    return w


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("kernel", [-1, 0, 1, 2, 3, 4])
def test_sixteen_rhs_block_pcg(small3d_q3, fp32, kernel):
    """16 right-hand sides in lockstep match the oracle per column, with the fine-level multi-RHS kernel chosen by
    timing (-1) or forced: lanes-per-row CSR (0), row blocks staged in LDS by a persistent pipelined workgroup per
    compute unit (1) or one workgroup per block (2), CSR with the columns split over lanes (3), the same with
    shared entry loads (4)."""
    import paper_2607_28235_amd as P
    w = small3d_q3
    prob = w.problem
    _case(f"16-rhs block pcg fp32={fp32} kernel={kernel} n={prob.n}")
    o = P.Options(dim=3, coarse_degree=2, leaf_size=256, max_coarse_dofs=600, vcycle_fp32=fp32,
                  multi_rhs_kernel=kernel)
    h = P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o)
    ho = O.build_hierarchy(prob.coords, prob.scipy(), coarse_degree=2, leaf_size=256, max_coarse_dofs=600)
    X = torch.zeros(16, prob.n, dtype=torch.float64, device="cuda")
    iters, relres, ok = h.pcg(_t(w.rhs), X, rtol=1e-10, maxit=200)
    assert ok
    Xh = X.cpu().numpy()
    for j in (0, 5, 15):
        xo, ko, _, _, _ = O.pcg(ho, w.rhs[j], rtol=1e-10)
        assert abs(int(iters[j]) - ko) <= 1, (j, iters[j], ko)
        assert _rel(Xh[j], xo) < 1e-9
    R = w.rhs - (prob.scipy() @ Xh.T).T
    assert np.all(np.linalg.norm(R, axis=1) <= 1.01e-10 * np.linalg.norm(w.rhs, axis=1))
    # a second call with the tuned tiles cached (and the graph captured) gives identical results
    X2 = torch.zeros_like(X)
    iters2, _, _ = h.pcg(_t(w.rhs), X2, rtol=1e-10, maxit=200)
    assert np.array_equal(iters, iters2) and torch.equal(X, X2)


@pytest.fixture(scope="module")
def q3_long_row():
    """The Q3 8^3 cube plus delta sum_j (e_i - e_j)(e_i - e_j)^T over 700 seeded free DoFs j (a graph Laplacian
    term: the matrix stays symmetric positive definite).  Row i then has more distinct columns than any staging
    class of the LDS-staged kernel holds (at most 640), so that kernel sums it from global memory."""
    _need_gpu()
    import scipy.sparse as sp
    w = F.workload(4, scale=8)
    prob = w.problem
    A = prob.scipy().tocsr()
    free = np.flatnonzero(~prob.boundary)
    g = np.random.default_rng(77)
    i = int(free[len(free) // 2])
    S = g.choice(free[free != i], size=700, replace=False)
    delta = 1e-2 * float(A[i, i])
    rows = np.concatenate([[i], S, np.full(len(S), i), S])
    cols = np.concatenate([[i], S, S, np.full(len(S), i)])
    vals = np.concatenate([[delta * len(S)], np.full(len(S), delta), np.full(2 * len(S), -delta)])
    A2 = (A + sp.csr_matrix((vals, (rows, cols)), shape=A.shape)).tocsr()
    A2.sort_indices()
    assert A2.indptr[i + 1] - A2.indptr[i] > 700
    ho = O.build_hierarchy(prob.coords, A2, coarse_degree=2, leaf_size=256, max_coarse_dofs=600)
    return prob, A2, ho


@pytest.mark.parametrize("kernel", [1, 2])
@pytest.mark.parametrize("nrhs,fp32", [(16, 1), (16, 0), (8, 0)])
def test_lds_staged_kernel_with_long_row(q3_long_row, kernel, nrhs, fp32):
    """The LDS-staged multi-RHS kernel in each staging class ((float, 16), (double, 16), (double, 8)), pipelined (1)
    or one workgroup per block (2), on a matrix with one row beyond every staging capacity: V-cycles per
    column against the oracle's, and a lockstep PCG solve (whose float64 operator also takes the kernel) against
    the oracle's solution."""
    import paper_2607_28235_amd as P
    prob, A2, ho = q3_long_row
    _case(f"LDS-staged kernel long row kernel={kernel} nrhs={nrhs} fp32={fp32} n={prob.n}")
    o = P.Options(dim=3, coarse_degree=2, leaf_size=256, max_coarse_dofs=600, vcycle_fp32=fp32,
                  multi_rhs_kernel=kernel)
    h = P.Hierarchy(prob.coords, A2.indptr.astype(np.int64), A2.indices.astype(np.int32), A2.data, o)
    g = np.random.default_rng(300 + nrhs)
    R = g.standard_normal((nrhs, prob.n))
    R[:, ho.constrained] = 0.0
    Z = torch.zeros(nrhs, prob.n, dtype=torch.float64, device="cuda")
    h.vcycle(_t(R), Z)
    torch.cuda.synchronize()
    Zh = Z.cpu().numpy()
    for j in range(nrhs):
        assert _rel(Zh[j], O.vcycle(ho, R[j])) < (2e-5 if fp32 else 1e-11), j
    X = torch.zeros(nrhs, prob.n, dtype=torch.float64, device="cuda")
    iters, relres, ok = h.pcg(_t(R), X, rtol=1e-10, maxit=200)
    assert ok
    Xh = X.cpu().numpy()
    for j in (0, nrhs - 1):
        xo, ko, _, _, _ = O.pcg(ho, R[j], rtol=1e-13)
        assert _rel(Xh[j], xo) < 1e-9, j
    res = R - (A2 @ Xh.T).T
    assert np.all(np.linalg.norm(res, axis=1) <= 1.01e-10 * np.linalg.norm(R, axis=1))
    h.close()


@pytest.mark.parametrize("kernel", [1, 2, 4])
def test_time_smoother_kernel_nrhs(small3d_q3, kernel):
    """Timing of the fine-level smoother kernel for 16 right-hand sides: the kernels are tuned on demand (no solve
    before), the bytes are those of the tuned kernel's format (LDS-staged kernels: values, 2-byte positions and the
    block's lists; CSR kernels: values and 4-byte columns) plus 7 vector streams of 16 columns, and other counts of
    right-hand sides are refused."""
    import paper_2607_28235_amd as P
    prob = small3d_q3.problem
    _case(f"time_smoother_kernel nrhs=16 kernel={kernel} n={prob.n}")
    o = P.Options(dim=3, coarse_degree=2, leaf_size=256, max_coarse_dofs=600, vcycle_fp32=1, multi_rhs_kernel=kernel)
    h = P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o)
    ms, by = h.time_smoother_kernel(0, 5, nrhs=16)
    ms_cold, _ = h.time_smoother_kernel(0, 2, flush_bytes=1 << 26, nrhs=16)
    assert ms > 0 and ms_cold > 0
    nnz, n = prob.nnz, prob.n
    vec = 7 * n * 4 * 16
    if kernel == 4:
        assert by == pytest.approx(nnz * 8 + 4 * (n + 1) + vec, rel=1e-12)
    else:
        assert nnz * 6 + vec < by < nnz * 8 + vec
    for bad in (3, 32):
        with pytest.raises(P.R3mgError):
            h.time_smoother_kernel(0, 1, nrhs=bad)
    h.close()


@pytest.fixture(scope="module")
def cfg4_24():
    """Config 4 at 24^3 cells (389,017 DoFs, 16 right-hand sides) with at most 500 coarse DoFs: levels 389,017 /
    6,912 / 864 / 108, the same level kinds as the 48^3 workload (CSR fine level, two block-row levels, dense
    coarsest); the oracle's solutions of columns 0 and 15."""
    _need_gpu()
    _case("config 4 at 24^3 inputs and oracle")
    w = F.workload(4, scale=24)
    prob = w.problem
    ho = O.build_hierarchy(prob.coords, prob.scipy(), coarse_degree=2, leaf_size=256, max_coarse_dofs=500,
                           skip_leaf_level=True)
    ref = {j: (O.pcg(ho, w.rhs[j], rtol=1e-10)[1], O.pcg(ho, w.rhs[j], rtol=1e-13)[0]) for j in (0, 15)}
    return w, ho, ref


@pytest.mark.slow
@pytest.mark.parametrize("fp32", [1, 0])
def test_config4_reduced_with_full_size_kernels(cfg4_24, fp32):
    """Config 4 at 24^3 with the kernels r3mg_info names for the 48^3 workload: the fine level's 2048-nonzero CSR
    row-block kernel (the shape the timing picks at 48^3, pinned here), the block-row workgroup kernel on both
    agglomerated levels, the dense coarsest inverse; the 16-column multi-RHS kernels as timed.  Lockstep PCG of
    the 16 columns: columns 0 and 15 against the oracle (iterations within one, solution within 1e-9 of the
    rtol-1e-13 solution), every column's true residual at the stop rule."""
    import paper_2607_28235_amd as P
    w, ho, ref = cfg4_24
    prob = w.problem
    _case(f"config 4 at 24^3 fp32={fp32}")
    o = P.Options(dim=3, coarse_degree=2, leaf_size=256, max_coarse_dofs=500, skip_leaf_level=1, fine_kernel=0,
                  vcycle_fp32=fp32)
    h = P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o)
    t = "float" if fp32 else "double"
    info = h.info()
    assert [lv["n"] for lv in info] == [lv.A.shape[0] for lv in ho.levels] == [389017, 6912, 864, 108]
    assert [lv["kernel"] for lv in info] == [f"k_level_stream<{t},2048,64,block>", f"k_level_blockrow_wg<{t}>",
                                             f"k_level_blockrow_wg<{t}>", "dense"]
    X = torch.zeros(16, prob.n, dtype=torch.float64, device="cuda")
    iters, relres, ok = h.pcg(_t(w.rhs), X, rtol=1e-10, maxit=200)
    assert ok
    Xh = X.cpu().numpy()
    for j, (ko, xt) in ref.items():
        assert abs(int(iters[j]) - ko) <= 1, (j, iters[j], ko)
        assert _rel(Xh[j], xt) < 1e-9, j
    R = w.rhs - (prob.scipy() @ Xh.T).T
    assert np.all(np.linalg.norm(R, axis=1) <= 1.01e-10 * np.linalg.norm(w.rhs, axis=1))
    h.close()


def test_uneven_group_in_one_graph():
    """Several independent problems of different sizes solved in one captured launch sequence.  A second group solve
    of the same handles replays the cached graph and gives bitwise the same solutions; after new values on one
    handle (its graphs dropped) the group is captured again and still solves."""
    _need_gpu()
    import paper_2607_28235_amd as P
    batch = F.uneven_batch([8, 10, 12, 14])
    _case("uneven group of 4 Q2 problems")
    hs, bs, xs, refs = [], [], [], []
    for prob, b in batch:
        o = P.Options(dim=3, coarse_degree=2, leaf_size=256, max_coarse_dofs=300, vcycle_fp32=1)
        hs.append(P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o))
        bs.append(_t(b))
        xs.append(torch.zeros(prob.n, dtype=torch.float64, device="cuda"))
        ho = O.build_hierarchy(prob.coords, prob.scipy(), coarse_degree=2, leaf_size=256, max_coarse_dofs=300)
        refs.append(O.pcg(ho, b, rtol=1e-10))
    iters, relres, ok = P.solve_group(hs, bs, xs, rtol=1e-10, maxit=200)
    assert ok
    for (prob, b), x, it, ref in zip(batch, xs, iters, refs):
        assert abs(int(it) - ref[1]) <= 1
        assert _rel(x.cpu().numpy(), ref[0]) < 1e-9
    xs2 = [torch.zeros_like(x) for x in xs]
    iters2, _, ok2 = P.solve_group(hs, bs, xs2, rtol=1e-10, maxit=200)
    assert ok2 and list(iters2) == list(iters)
    assert all(torch.equal(a, c) for a, c in zip(xs, xs2))
    prob0 = batch[0][0]
    hs[0].update_values(_t(prob0.val))
    torch.cuda.synchronize()
    xs3 = [torch.zeros_like(x) for x in xs]
    iters3, _, ok3 = P.solve_group(hs, bs, xs3, rtol=1e-10, maxit=200)
    assert ok3 and list(iters3) == list(iters)
    for x3, ref in zip(xs3, refs):
        assert _rel(x3.cpu().numpy(), ref[0]) < 1e-9


def _cfg5(N):
    ncells = N ** 3
    kappa = np.exp(F.rng(5, F.PURPOSE_KAPPA).standard_normal(ncells))
    prob = F.structured_qp(3, N, 2, cfg=5, kappa=kappa, keep_ke=True)
    ut = F.smooth_target(prob.coords, 5)
    return prob, kappa, ut


@pytest.fixture(scope="module")
def adjoint_small():
    _need_gpu()
    import paper_2607_28235_amd as P
    _case("adjoint setup (3D Q2 8^3, lognormal kappa)")
    prob, kappa, ut = _cfg5(8)
    o = P.Options(dim=3, coarse_degree=2, leaf_size=256, max_coarse_dofs=600)
    op = P.AdjointPoisson(prob.coords, prob.row_ptr, prob.col, prob.val, prob.cells, prob.Ke,
                          prob.mass_rhs_weights, o, rtol=1e-12)
    return prob, kappa, ut, op


def test_assembly_matches_oracle(adjoint_small):
    prob, kappa, ut, op = adjoint_small
    _case("kappa assembly")
    k2 = kappa * np.exp(0.3 * np.sin(np.arange(len(kappa))))
    op.asm.assemble(_t(k2), op.Ke, op.ke_stride, op.vals)
    torch.cuda.synchronize()
    A = O.assemble_kappa(prob.row_ptr, prob.col, prob.n, prob.cells, prob.Ke, k2, prob.boundary)
    np.testing.assert_allclose(op.vals.cpu().numpy(), A.data, rtol=1e-13, atol=1e-15)
    op.invalidate()


def test_adjoint_gradient_matches_oracle(adjoint_small):
    prob, kappa, ut, op = adjoint_small
    _case("adjoint gradient vs oracle")
    kt = _t(kappa).requires_grad_(True)
    u = op(kt)
    L = 0.5 * torch.sum((u - _t(ut)) ** 2)
    L.backward()
    g = kt.grad.cpu().numpy()

    def solve(k, rhs):
        A = O.assemble_kappa(prob.row_ptr, prob.col, prob.n, prob.cells, prob.Ke, k, prob.boundary)
        return np.linalg.solve(A.toarray(), rhs), A
    Lo, go, uo, lo = O.loss_and_gradient(solve, prob.cells, prob.Ke, kappa, prob.mass_rhs_weights, ut, prob.boundary)
    assert _rel(u.detach().cpu().numpy(), uo) < 1e-10
    assert abs(float(L.detach()) - Lo) <= 1e-9 * Lo
    assert _rel(g, go) < 1e-9
    # Euler identity: sum_e kappa_e g_e = -(u - u_t)^T u
    uu = u.detach().cpu().numpy()
    assert abs(kappa @ g + (uu - ut) @ uu) <= 1e-9 * abs((uu - ut) @ uu)


def test_adjoint_gradient_finite_differences(adjoint_small):
    """Central differences in the difference form (no cancellation between two full solves): with
    A(kappa +- h e_e) du = -+ h K_e u_e on the unconstrained rows, L(kappa +- h) - L = (u - u_t).du + |du|^2 / 2.
    Relative agreement 1e-6 on six seeded cells."""
    prob, kappa, ut, op = adjoint_small
    _case("adjoint gradient vs central differences")
    kt = _t(kappa).requires_grad_(True)
    u = op(kt)
    L = 0.5 * torch.sum((u - _t(ut)) ** 2)
    L.backward()
    g = kt.grad.cpu().numpy()
    un = u.detach().cpu().numpy()
    cells = F.rng(5, F.PURPOSE_FDCELLS).choice(len(kappa), size=6, replace=False)
    for e in cells:
        h = 1e-3 * kappa[e]
        nodes = prob.cells[e]
        Ke = prob.Ke if prob.Ke.ndim == 2 else prob.Ke[e]
        Ku = Ke @ un[nodes]
        dL = []
        for sgn in (1.0, -1.0):
            kp = kappa.copy()
            kp[e] += sgn * h
            op.set_kappa(_t(kp))
            rhs = np.zeros(prob.n)
            np.add.at(rhs, nodes, -sgn * h * Ku)
            rhs[prob.boundary] = 0.0
            du, _ = op.solve_field(_t(rhs))
            du = du.cpu().numpy()
            dL.append((un - ut) @ du + 0.5 * du @ du)
        op.invalidate()
        fd = (dL[0] - dL[1]) / (2 * h)
        assert abs(fd - g[e]) <= 1e-6 * max(abs(g[e]), 1e-3 * np.abs(g).max()), (e, fd, g[e])