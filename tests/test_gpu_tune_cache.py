"""The persisted tuning cache on the GPU: a handle records the kernel choices it timed (the fine level's row-block
shape at set-up, the multi-RHS kernels at the first 16-column solve); a later handle of the same structure takes
them from the cache without timing and gives identical results; tune_cache=0 ignores the cache; a cached code that
names no valid kernel is timed again."""
import sys

import numpy as np
import pytest

import fixtures as F

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(name):
    print(f"[gpu-case] {name}", flush=True)
    sys.stdout.flush()


def _lines(path):
    return path.read_text().splitlines() if path.exists() else []


def test_tuning_cache_reuses_choices(tmp_path, monkeypatch):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_28235_amd as P
    path = tmp_path / "tune-cache.txt"
    monkeypatch.setenv("R3MG_TUNE_CACHE", str(path))
    w = F.workload(4, scale=8)
    prob = w.problem
    _case(f"tuning cache n={prob.n}")

    def handle(**kw):
        o = P.Options(dim=3, coarse_degree=2, leaf_size=256, max_coarse_dofs=600, vcycle_fp32=1, **kw)
        return P.Hierarchy(prob.coords, prob.row_ptr, prob.col, prob.val, o)

    B = torch.from_numpy(np.ascontiguousarray(w.rhs)).to("cuda")

    def solve(h):
        X = torch.zeros_like(B)
        iters, _, ok = h.pcg(B, X, rtol=1e-10, maxit=200)
        assert ok
        return X, iters

    h1 = handle()
    after_factor = _lines(path)
    fine = [ln for ln in after_factor if "/fine1/f32 " in ln]
    assert len(fine) == 1
    X1, it1 = solve(h1)
    after_solve = _lines(path)
    mr = [ln for ln in after_solve if "/mr/" in ln]
    assert len(after_solve) > len(after_factor) and any("/mr/0/16/4 " in ln for ln in mr)
    assert any("/mr/-1/16/8 " in ln for ln in mr)
    info1 = [lv["kernel"] for lv in h1.info()]

    # same structure: every choice from the cache, nothing timed, same kernels and bitwise the same solution
    h2 = handle()
    X2, it2 = solve(h2)
    assert _lines(path) == after_solve
    assert [lv["kernel"] for lv in h2.info()] == info1
    assert np.array_equal(it1, it2) and torch.equal(X1, X2)

    # tune_cache = 0: timed again, the file untouched
    h3 = handle(tune_cache=0)
    X3, _ = solve(h3)
    assert _lines(path) == after_solve
    assert torch.allclose(X3, X1, rtol=0, atol=1e-9 * float(X1.abs().max()))

    # a cached shape that names no kernel: ignored and timed again (a valid line is appended for the key)
    key = fine[0].rsplit(" ", 1)[0]
    with open(path, "a") as f:
        f.write(f"{key} 9999\n")
    h4 = handle()
    tail = _lines(path)[-1]
    assert tail.startswith(key + " ") and int(tail.rsplit(" ", 1)[1]) != 9999
    X4, _ = solve(h4)
    assert torch.allclose(X4, X1, rtol=0, atol=1e-9 * float(X1.abs().max()))
    for h in (h1, h2, h3, h4):
        h.close()
