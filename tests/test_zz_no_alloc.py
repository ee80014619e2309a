"""r3mg_vcycle_noalloc (the V-cycle for callers that cannot allocate) against r3mg_vcycle, through the C ABI.

Two calls in a row, the second with a smaller input (another hierarchy with fewer DoFs and fewer columns), each
compared with r3mg_vcycle on the same handle: the same kernels run on work vectors carved from the static
scratch instead of the handle's buffers, so the results must agree bitwise, and with the oracle's V-cycle to the
V-cycle parity bar.  Also: work vectors larger than the scratch are rejected with nothing launched, and the call
can be captured into a HIP graph (it allocates and synchronises nothing) whose replays match the eager result.
"""
import ctypes as C
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


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _noalloc(h, r, z):
    import paper_2607_28235_amd as P
    nrhs = 1 if r.dim() == 1 else r.shape[0]
    st = P.lib().r3mg_vcycle_noalloc(h._h, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr()), nrhs,
                                     C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def _setup(prob, pc, leaf, max_levels, fp32, max_coarse=2000, pre=2, post=2):
    import paper_2607_28235_amd as P
    o = P.Options(dim=prob.d, coarse_degree=pc, leaf_size=leaf, max_levels=max_levels, max_coarse_dofs=max_coarse,
                  pre_steps=pre, post_steps=post, vcycle_fp32=fp32)
    return P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o)


@pytest.mark.parametrize("fp32", [0, 1])
def test_noalloc_matches_vcycle_on_two_calls(fp32):
    _need_gpu()
    _case(f"noalloc vcycle: larger then smaller input, fp32={fp32}")
    big = F.structured_qp(2, 40, 3, jitter=0.2, cfg=2)            # 14,641 DoFs, 4 columns
    small = F.workload(1).problem                                  # 1,089 DoFs, 1 column
    cases = [(big, _setup(big, 2, 128, 4, fp32, max_coarse=100), 4, 2, 128, 4, 100, 2, 2),
             (small, _setup(small, 1, 64, 2, fp32, pre=1, post=1), 1, 1, 64, 2, 2000, 1, 1)]
    g = np.random.default_rng(17)
    for prob, h, nrhs, pc, leaf, ml, mc, pre, post in cases:
        R = g.standard_normal((nrhs, prob.n))
        r = _t(R)
        z_ref = torch.zeros_like(r)
        z_na = torch.full_like(r, float("nan"))
        h.vcycle(r, z_ref)
        assert _noalloc(h, r, z_na) == 0
        torch.cuda.synchronize()
        a, b = z_na.cpu().numpy(), z_ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        np.testing.assert_array_equal(a, b)
        if not fp32:
            ho = O.build_hierarchy(prob.coords, prob.scipy(), coarse_degree=pc, leaf_size=leaf, max_levels=ml,
                                   max_coarse_dofs=mc, pre_steps=pre, post_steps=post)
            for j in range(nrhs):
                zo = O.vcycle(ho, R[j])
                assert np.linalg.norm(a[j] - zo) <= 1e-11 * np.linalg.norm(zo)
        h.close()


def test_noalloc_rejects_work_vectors_beyond_the_scratch():
    _need_gpu()
    _case("noalloc vcycle: size limit")
    import paper_2607_28235_amd as P
    prob = F.structured_qp(2, 120, 3, cfg=2)                       # 130,321 DoFs
    h = _setup(prob, 2, 128, 4, 0, max_coarse=2000)
    # 5 float64 vectors of n x 16 per level: more than 64 MiB; n x 4: less
    r16 = torch.ones(16, prob.n, dtype=torch.float64, device="cuda")
    z16 = torch.full_like(r16, 7.0)
    st = _noalloc(h, r16, z16)
    assert st == -1
    msg = P.lib().r3mg_last_error().decode()
    assert "scratch" in msg and str(P.NOALLOC_SCRATCH_BYTES) in msg
    torch.cuda.synchronize()
    assert torch.all(z16 == 7.0)                                    # nothing was launched
    assert _noalloc(h, r16[:3], z16[:3]) == -1                     # nrhs must be 1, 2, 4, 8 or 16
    r4, z4 = r16[:4].contiguous(), torch.zeros(4, prob.n, dtype=torch.float64, device="cuda")
    zr = torch.zeros_like(z4)
    h.vcycle(r4, zr)                      # times the 4-column kernels; the allocation-free call then uses them
    assert _noalloc(h, r4, z4) == 0
    torch.cuda.synchronize()
    np.testing.assert_array_equal(z4.cpu().numpy(), zr.cpu().numpy())
    h.close()


def test_noalloc_call_captured_in_a_graph():
    _need_gpu()
    _case("noalloc vcycle: graph capture and replays")
    prob = F.structured_qp(2, 24, 3, jitter=0.2, cfg=2)
    h = _setup(prob, 2, 128, 3, 1, max_coarse=2000)
    g = np.random.default_rng(5)
    r = _t(g.standard_normal(prob.n))
    z_eager = torch.zeros_like(r)
    assert _noalloc(h, r, z_eager) == 0
    torch.cuda.synchronize()
    z = torch.zeros_like(r)
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            st = _noalloc(h, r, z)
    torch.cuda.current_stream().wait_stream(s)
    assert st == 0
    for k in range(3):
        z.fill_(-1.0)
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(z.cpu().numpy(), z_eager.cpu().numpy())
        # eager work between the replays, on the same scratch
        w = torch.zeros_like(r)
        assert _noalloc(h, 2.0 * r, w) == 0
        torch.cuda.synchronize()
        np.testing.assert_allclose(w.cpu().numpy(), 2.0 * z_eager.cpu().numpy(), rtol=1e-6, atol=1e-12)
    h.close()
