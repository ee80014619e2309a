"""GPU parity of the matrix-free fine operator (Q_p stiffness action by sum factorisation) against the oracle.

Tolerances: the matrix-free float64 action is the assembled matrix's arithmetic in another order (Gauss points
summed per cell, cells summed per DoF), so it agrees with the oracle's action to 1e-13 of max |A x|; the V-cycle
and PCG bars are those of the CSR path (1e-11, iterations within one, solutions within 1e-9).
"""
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


def _P():
    import paper_2607_28235_amd as P
    return P


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _apply(h, x):
    y = torch.zeros_like(x)
    h.level_apply(0, x, y)
    torch.cuda.synchronize()
    return y.cpu().numpy()


# (name, d, N, p, jitter, p', leaf, kappa)
CASES = [
    ("2d_q3_multilinear", 2, 24, 3, 0.2, 2, 64, False),
    ("2d_q2_affine_kappa", 2, 32, 2, 0.0, 1, 64, True),
    ("2d_q1_multilinear", 2, 48, 1, 0.2, 1, 32, False),
    ("3d_q2_affine", 3, 8, 2, 0.0, 2, 128, False),
    ("3d_q2_multilinear_kappa", 3, 6, 2, 0.15, 1, 64, True),
    ("3d_q3_affine", 3, 5, 3, 0.0, 2, 128, False),
    ("3d_q1_multilinear", 3, 12, 1, 0.2, 1, 64, False),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_matrix_free_matches_oracle(case):
    _need_gpu()
    P = _P()
    name, d, N, p, jit, pc, leaf, kap = case
    _case(f"matrix-free {name}")
    kappa = np.exp(F.rng(6, F.PURPOSE_KAPPA).standard_normal(N ** d)) if kap else None
    prob = F.structured_qp(d, N, p, jitter=jit, cfg=6, kappa=kappa)
    b = F.nodal_rhs(prob, F.rng(6, F.PURPOSE_RHS).standard_normal(prob.n), jitter=jit, cfg=6)
    A = prob.scipy()
    ho = O.build_hierarchy(prob.coords, A, coarse_degree=pc, leaf_size=leaf, max_coarse_dofs=300)
    xo, ko, _, _, _ = O.pcg(ho, b, rtol=1e-10)
    for fp32 in (0, 1):
        o = P.Options(dim=d, coarse_degree=pc, leaf_size=leaf, max_coarse_dofs=300, vcycle_fp32=fp32)
        h = P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o)
        h.set_matrix_free(prob.cells, p, kappa)
        kname = h.info()[0]["kernel"]
        assert "k_mf_cell" in kname and ("affine" in kname) == (jit == 0.0), kname
        if not fp32:
            x = F.rng(6, F.PURPOSE_TARGET).standard_normal(prob.n)
            y = _apply(h, _t(x))
            yo = O.stiffness_apply(prob.coords, prob.cells, p, x, kappa=kappa, constrained=prob.boundary,
                                   cdiag=np.ones(prob.n))
            assert np.abs(y - yo).max() <= 1e-13 * np.abs(yo).max()
            r = np.random.default_rng(8).standard_normal(prob.n)
            r[ho.constrained] = 0.0
            z = torch.zeros(prob.n, dtype=torch.float64, device="cuda")
            h.vcycle(_t(r), z)
            torch.cuda.synchronize()
            assert _rel(z.cpu().numpy(), O.vcycle(ho, r)) < 1e-11
        xg = torch.zeros(prob.n, dtype=torch.float64, device="cuda")
        iters, relres, ok = h.pcg(_t(b), xg, rtol=1e-10, maxit=200)
        assert ok and abs(int(iters[0]) - ko) <= 1, (fp32, iters, ko)
        xs = xg.cpu().numpy()
        assert _rel(xs, xo) < 1e-9
        assert np.linalg.norm(b - A @ xs) <= 1.01e-10 * np.linalg.norm(b)
        h.close()


@pytest.fixture(scope="module")
def small2d():
    _need_gpu()
    P = _P()
    prob = F.structured_qp(2, 12, 2, jitter=0.2, cfg=6)
    b = F.nodal_rhs(prob, F.rng(6, F.PURPOSE_RHS).standard_normal(prob.n), jitter=0.2, cfg=6)
    o = P.Options(dim=2, coarse_degree=1, leaf_size=32, max_coarse_dofs=100)
    return prob, b, o


def test_matrix_free_rejects_inconsistent_cells(small2d):
    """Node order, degree, indices, coverage and kappa are checked; a rejected description leaves the CSR
    matrix in use."""
    P = _P()
    prob, b, o = small2d
    _case("matrix-free errors")
    h = P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o)
    csr_name = h.info()[0]["kernel"]
    # the node order reversed is the same cell seen from the opposite corner: accepted
    h.set_matrix_free(prob.cells[:, ::-1], 2)
    assert "k_mf_cell" in h.info()[0]["kernel"]
    h.set_matrix_free(None, 0)
    bad_cases = [
        (prob.cells[:, [1, 0, 2, 3, 4, 5, 6, 7, 8]], 2, None),      # two nodes swapped: another operator
        (prob.cells.reshape(-1, 3, 3).transpose(0, 2, 1).reshape(-1, 9), 2, None),  # axes swapped: inverted map
        (prob.cells[:, [0, 2, 6, 8]], 1, None),             # Q1 on the corner nodes: another operator
        (np.where(prob.cells == 5, prob.n, prob.cells), 2, None),  # index out of range
        (prob.cells[1:], 2, None),                          # the first cell's interior node is in no cell
        (prob.cells, 2, -np.ones(prob.cells.shape[0])),     # non-positive kappa
        (prob.cells, 4, None),                              # unsupported degree (binding checks the shape)
    ]
    for cells, deg, kap in bad_cases:
        if deg == 4:
            with pytest.raises(ValueError):
                h.set_matrix_free(cells, deg, kap)
            continue
        with pytest.raises(P.R3mgError) as e:
            h.set_matrix_free(cells, deg, kap)
        assert e.value.code == "INVALID"
        assert h.info()[0]["kernel"] == csr_name
    h.close()


def test_matrix_free_lifecycle_and_determinism(small2d):
    """Detaching returns to the CSR kernels; new values drop the operator; repeated solves are bitwise equal;
    multi-right-hand-side solves (CSR kernels) still agree with single solves."""
    P = _P()
    prob, b, o = small2d
    _case("matrix-free lifecycle")
    h = P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o)
    csr_name = h.info()[0]["kernel"]
    h.set_matrix_free(prob.cells, 2)
    assert "k_mf_cell" in h.info()[0]["kernel"]
    bt = _t(b)
    xs = []
    for _ in range(2):
        x = torch.zeros_like(bt)
        it, _, ok = h.pcg(bt, x, rtol=1e-10)
        assert ok
        xs.append(x.clone())
    assert torch.equal(xs[0], xs[1])
    B = torch.stack([bt, 2.0 * bt, -bt])
    X = torch.zeros_like(B)
    _, _, ok = h.pcg(B, X, rtol=1e-10)
    assert ok
    for j, s in enumerate((1.0, 2.0, -1.0)):
        assert _rel(X[j].cpu().numpy(), s * xs[0].cpu().numpy()) < 1e-9
    h.set_matrix_free(None, 0)
    assert h.info()[0]["kernel"] == csr_name
    h.set_matrix_free(prob.cells, 2)
    vals = _t(prob.val * 2.0)
    h.update_values(vals)
    assert h.info()[0]["kernel"] == csr_name
    x = torch.zeros_like(bt)
    h.pcg(bt, x, rtol=1e-10)
    assert _rel(x.cpu().numpy(), 0.5 * xs[0].cpu().numpy()) < 1e-9
    h.close()


@pytest.mark.parametrize("cfg", [2, 3])
def test_matrix_free_full_size(cfg):
    """The 2D Q3 256^2 jittered (591,361 DoFs, multilinear cells) and 3D Q2 64^3 (2,146,689 DoFs, affine cells)
    workloads: the action against the assembled matrix, sampled rows against the oracle cell by cell, and the
    FP32 V-cycle PCG solve against the CSR path's (iterations within one, solutions within 1e-9, true residual at
    the stop rule)."""
    _need_gpu()
    P = _P()
    _case(f"matrix-free full size cfg{cfg}")
    w = F.workload(cfg)
    prob = w.problem
    A = prob.scipy()
    o = P.Options(dim=prob.d, coarse_degree=w.coarse_degree, leaf_size=w.leaf_size, max_levels=w.max_levels,
                  max_coarse_dofs=w.max_coarse_dofs, pre_steps=w.pre_steps, post_steps=w.post_steps,
                  skip_leaf_level=int(w.skip_leaf_level), vcycle_fp32=1)
    h = P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o)
    bt = _t(w.rhs)
    x_csr = torch.zeros_like(bt)
    it_csr, _, ok = h.pcg(bt, x_csr, rtol=1e-10)
    assert ok
    h.set_matrix_free(prob.cells, prob.p)
    x = F.rng(cfg, F.PURPOSE_TARGET).standard_normal(prob.n)
    y = _apply(h, _t(x))
    ref = A @ x
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    # sampled rows from the oracle: y_i = sum over the cells holding i of (K_e x_e)_i
    g = np.random.default_rng(cfg)
    free = np.flatnonzero(~prob.boundary)
    xf = np.where(prob.boundary, 0.0, x)
    k = prob.p + 1
    corner_pos = [sum(((v >> ax) & 1) * prob.p * k ** ax for ax in range(prob.d)) for v in range(2 ** prob.d)]
    for i in g.choice(free, 24, replace=False):
        acc = 0.0
        for e in np.flatnonzero((prob.cells == i).any(axis=1)):
            c = prob.cells[e]
            Ke = O.element_stiffness(prob.coords[c[corner_pos]], prob.p)
            a = int(np.flatnonzero(c == i)[0])
            acc += float(Ke[a] @ xf[c])
        assert abs(y[i] - acc) <= 1e-13 * np.abs(ref).max(), i
    xg = torch.zeros_like(bt)
    it, _, ok = h.pcg(bt, xg, rtol=1e-10)
    assert ok and abs(int(it[0]) - int(it_csr[0])) <= 1, (it, it_csr)
    xs = xg.cpu().numpy()
    assert _rel(xs, x_csr.cpu().numpy()) < 1e-9
    assert np.linalg.norm(w.rhs - A @ xs) <= 1.01e-10 * np.linalg.norm(w.rhs)
    h.close()


@pytest.mark.parametrize("case,nr", [("2d_q3_multilinear", 4), ("3d_q2_affine", 16), ("3d_q3_affine", 2)])
def test_matrix_free_multi_rhs(case, nr):
    """Several right-hand sides through the matrix-free operator (cell kernel looping over the columns, per-DoF
    gather of 16-byte column groups): the float64 V-cycle of every column against the oracle (1e-11), and the
    block PCG in both V-cycle precisions against the oracle per column (iterations within one, solutions within
    1e-9)."""
    _need_gpu()
    P = _P()
    spec = {c[0]: c for c in CASES}[case]
    _, d, N, p, jit, pc, leaf, kap = spec
    _case(f"matrix-free multi-RHS {case} nr={nr}")
    prob = F.structured_qp(d, N, p, jitter=jit, cfg=6)
    g = F.rng(6, F.PURPOSE_RHS)
    Bm = np.stack([F.nodal_rhs(prob, g.standard_normal(prob.n), jitter=jit, cfg=6) for _ in range(nr)])
    ho = O.build_hierarchy(prob.coords, prob.scipy(), coarse_degree=pc, leaf_size=leaf, max_coarse_dofs=300)
    ref = [O.pcg(ho, Bm[j], rtol=1e-10)[:2] for j in range(nr)]
    for fp32 in (0, 1):
        o = P.Options(dim=d, coarse_degree=pc, leaf_size=leaf, max_coarse_dofs=300, vcycle_fp32=fp32)
        h = P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o)
        h.set_matrix_free(prob.cells, p)
        if not fp32:
            R = np.random.default_rng(9).standard_normal((nr, prob.n))
            R[:, ho.constrained] = 0.0
            Z = torch.zeros(nr, prob.n, dtype=torch.float64, device="cuda")
            h.vcycle(_t(R), Z)
            torch.cuda.synchronize()
            for j in range(nr):
                assert _rel(Z[j].cpu().numpy(), O.vcycle(ho, R[j])) < 1e-11, j
        X = torch.zeros(nr, prob.n, dtype=torch.float64, device="cuda")
        iters, relres, ok = h.pcg(_t(Bm), X, rtol=1e-10, maxit=200)
        assert ok
        for j in range(nr):
            xo, ko = ref[j]
            assert abs(int(iters[j]) - ko) <= 1, (fp32, j, iters[j], ko)
            assert _rel(X[j].cpu().numpy(), xo) < 1e-9, (fp32, j)
        h.close()
