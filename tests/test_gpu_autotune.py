"""The autotuner picks a configuration the library accepts and caches it:
a second call returns the cached choice without timing again."""
import json

import pytest

from paper_2103_10116_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_tune_spmv_and_cache(tmp_path):
    import torch
    from paper_2103_10116_amd import autotune, mxs
    ctx = mxs.Context(0)
    A = I.stencil27(24)
    M = mxs.Matrix.from_host(ctx, A)
    cache = str(tmp_path / "tune.json")
    lines = []
    opts = autotune.tune_spmv(ctx, M, "f64", reps=3, cache=cache, log=lines.append)
    assert opts in autotune.CSR_CANDIDATES and len(lines) == len(autotune.CSR_CANDIDATES)
    B = M.convert("csr", "f64", **opts)
    x = torch.rand(A.n, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    mxs.spmv(ctx, B, x, y)
    torch.cuda.synchronize()
    lines.clear()
    assert autotune.tune_spmv(ctx, M, "f64", reps=3, cache=cache, log=lines.append) == opts
    assert not lines  # served from the cache
    assert any(k.startswith("spmv|") for k in json.load(open(cache)))
    ctx.close()


def test_tune_coo(tmp_path):
    """COO tuning: kernel, chunk size and work-group shape; cached apart from
    the CSR choice of the same matrix."""
    import torch
    from paper_2103_10116_amd import autotune, mxs
    ctx = mxs.Context(0)
    A = I.poisson3d(12)
    M = mxs.Matrix.from_host(ctx, A)
    cache = str(tmp_path / "tune.json")
    opts = autotune.tune_spmv(ctx, M, "f32", reps=2, cache=cache, fmt="coo")
    assert opts in autotune.COO_CANDIDATES
    B = M.convert("coo", "f32", **opts)
    assert B.info()["coo_kernel"] == mxs.COO_KERNELS[opts["coo_kernel"]]
    x = torch.rand(A.n, dtype=torch.float32, device="cuda")
    y = torch.zeros_like(x)
    mxs.spmv(ctx, B, x, y)
    torch.cuda.synchronize()
    keys = list(json.load(open(cache)))
    assert any(k.endswith("|coo") for k in keys)
    assert autotune.tune_spmv(ctx, M, "f32", reps=2, cache=cache) in autotune.CSR_CANDIDATES
    ctx.close()


def test_tune_batch_classes(tmp_path):
    from paper_2103_10116_amd import autotune, mxs
    ctx = mxs.Context(0)
    cache = str(tmp_path / "tune.json")
    classes = autotune.tune_batch_classes(ctx, bounds=(256, 1024), per_class=8, cache=cache)
    assert [c[0] for c in classes] == [256, 1024]
    assert all(c[1] in autotune.BLOCKS for c in classes)
    B = mxs.Batch(ctx, 64 << 20, 8, classes=classes)
    A = I.serving_system(20, 1)
    t = B.submit(A, I.serving_rhs(A.n, 1), 1e-10)
    while True:
        st = B.step()
        if st["active"] == 0 and st["pending"] == 0:
            break
    assert B.poll(t, A.n)[0] == mxs.OK
    B.close()
    ctx.close()


def test_tune_batch_classes_default_bounds(tmp_path):
    """The serving bench's call: every default size class (up to 10240 rows,
    whose other classes need 512 or 1024 threads to stay within 16 rows a
    thread) is timed and a valid shape is returned for each."""
    from paper_2103_10116_amd import autotune, mxs
    ctx = mxs.Context(0)
    classes = autotune.tune_batch_classes(ctx, per_class=4, cache=str(tmp_path / "t.json"))
    assert [c[0] for c in classes] == list(autotune.CLASS_BOUNDS)
    assert all(c[1] in autotune.BLOCKS and -(-c[0] // c[1]) <= 16 for c in classes)
    mxs.Batch(ctx, 64 << 20, 8, classes=classes).close()
    ctx.close()
