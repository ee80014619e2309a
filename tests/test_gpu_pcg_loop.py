"""GPU checks of the PCG driver: convergence decided on the device, iterations enqueued in predicted chunks.

The solve enqueues the iterations it predicts (from the handle's last solve, or from the residual reduction of
the chunk just read) and reads the device state once per chunk.  Whatever the prediction, the iterates must be
those of the textbook recursion (Section 6 solver; the oracle's O11): the same stop test, the same iteration
counts within one, and a residual history that follows the oracle's.  These cases exercise a prediction that
is exact (a repeated solve), short (a tighter rtol) and long (a looser rtol: enqueued iterations that the
device skips), and a solve capped by maxit.
"""
import sys

import numpy as np
import pytest

import fixtures as F
import oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(name):
    print(f"[gpu-case] {name}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def prob2d():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _case("pcg-loop setup (2D Q3 48x48 jittered, p'=2, leaf 128, 4 levels)")
    prob = F.structured_qp(2, 48, 3, jitter=0.2, cfg=2)
    b = F.nodal_rhs(prob, F.rng(2, F.PURPOSE_RHS).standard_normal(prob.n), jitter=0.2, cfg=2)
    ho = O.build_hierarchy(prob.coords, prob.scipy(), coarse_degree=2, leaf_size=128, max_levels=4,
                           max_coarse_dofs=100)
    return prob, b, ho


def _hier(prob, fp32, use_graph=1):
    import paper_2607_28235_amd as P
    o = P.Options(dim=2, coarse_degree=2, leaf_size=128, max_levels=4, max_coarse_dofs=100, vcycle_fp32=fp32,
                  use_graph=use_graph)
    return P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("fp32", [0, 1])
def test_prediction_changes_nothing_but_the_schedule(prob2d, fp32):
    prob, b, ho = prob2d
    _case(f"pcg predicted chunks fp32={fp32}")
    h = _hier(prob, fp32)
    A = prob.scipy()
    bt = _t(b)
    xs = {}
    for run, rtol in enumerate([1e-10, 1e-10, 1e-12, 1e-6, 1e-10]):
        x = torch.zeros_like(bt)
        iters, relres, ok = h.pcg(bt, x, rtol=rtol, maxit=200)
        xo, ko, conv, hist_o, _ = O.pcg(ho, b, rtol=rtol)
        it = int(iters[0])
        assert ok and conv
        assert abs(it - ko) <= 1, (rtol, it, ko)
        hist = h.history(0)
        assert hist.shape == (it + 1,)
        np.testing.assert_allclose(hist[0], np.linalg.norm(b), rtol=1e-12)
        assert hist[-1] <= rtol * hist[0] and hist[-2] > rtol * hist[0]
        if not fp32:
            m = min(it, ko) + 1
            # the same recursion up to rounding, which is relative to ||r_0|| (late residuals are far smaller)
            ref = np.asarray(hist_o)[:m]
            np.testing.assert_allclose(hist[:m], ref, rtol=1e-3, atol=1e-12 * ref[0])
        xv = x.cpu().numpy()
        r = b - A @ xv
        assert np.linalg.norm(r) <= 1.01 * rtol * np.linalg.norm(b)
        xs.setdefault(rtol, []).append(xv)
    # identical inputs give bitwise identical results, whatever chunk the prediction enqueued
    for v in xs[1e-10][1:]:
        np.testing.assert_array_equal(v, xs[1e-10][0])


def test_maxit_caps_the_solve(prob2d):
    prob, b, ho = prob2d
    _case("pcg maxit 3")
    h = _hier(prob, 0)
    bt = _t(b)
    x = torch.zeros_like(bt)
    iters, relres, ok = h.pcg(bt, x, rtol=1e-14, maxit=3)
    assert not ok and int(iters[0]) == 3
    xo, ko, conv, hist_o, _ = O.pcg(ho, b, rtol=1e-14, maxit=3)
    assert not conv and ko == 3
    xv = x.cpu().numpy()
    assert np.linalg.norm(xv - xo) <= 1e-10 * np.linalg.norm(xo)   # the last iterate was written back
    np.testing.assert_allclose(relres[0], hist_o[-1] / hist_o[0], rtol=1e-8)
    # maxit = 0: x0 is returned untouched and the status says not converged
    x0 = _t(np.full(prob.n, 0.25))
    iters, relres, ok = h.pcg(bt, x0, rtol=1e-10, maxit=0)
    assert not ok and int(iters[0]) == 0
    assert torch.all(x0 == 0.25)


@pytest.mark.parametrize("fp32", [0, 1])
def test_graph_replay_equals_direct_launches(prob2d, fp32):
    prob, b, ho = prob2d
    _case(f"pcg graphs vs direct launches fp32={fp32}")
    bt = _t(b)
    out = []
    for g in (1, 0):
        h = _hier(prob, fp32, use_graph=g)
        x = torch.zeros_like(bt)
        iters, relres, ok = h.pcg(bt, x, rtol=1e-10, maxit=200)
        assert ok
        out.append((int(iters[0]), x.cpu().numpy()))
    assert out[0][0] == out[1][0]
    np.testing.assert_array_equal(out[0][1], out[1][1])


def test_zero_rhs_and_converged_start(prob2d):
    prob, b, ho = prob2d
    _case("pcg zero rhs and exact start")
    h = _hier(prob, 1)
    z = torch.zeros(prob.n, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(z)
    iters, relres, ok = h.pcg(z, x, rtol=1e-10)
    assert ok and int(iters[0]) == 0 and torch.all(x == 0)
    assert h.history(0).shape == (1,)
    # a start that already satisfies the stop rule (an absolute threshold above its residual)
    bt = _t(b)
    xs = torch.zeros_like(bt)
    h.pcg(bt, xs, rtol=1e-12)
    keep = xs.clone()
    iters, relres, ok = h.pcg(bt, xs, rtol=1e-6, atol=1e-6 * float(np.linalg.norm(b)))
    assert ok and int(iters[0]) == 0
    assert torch.equal(xs, keep)
