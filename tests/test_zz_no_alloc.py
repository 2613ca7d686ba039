"""The allocation-free product mxs_spmv_noalloc, through the C ABI: for every
kernel family (the chunked ones that need scratch -- merge-path CSR, also over
column panels, COO, the COO part of hybrid -- and the others) its result
equals mxs_spmv's bit for bit
and the oracle's within 1e-13 (FP64) or 1e-5 (FP32) of sum |a_ij||x_j| +
|beta||y_i|, on two inputs in a row (the second smaller), and it never calls
the context's allocator."""
import numpy as np
import pytest

from paper_2103_10116_amd import inputs as I

pytestmark = pytest.mark.gpu


def _mats(mxs, ctx, A):
    M = mxs.Matrix.from_host(ctx, A)
    return {"csr_auto": M,
            "csr_merge": M.convert("csr", "f64", csr_kernel="merge"),
            "csr_panels": M.convert("csr", "f64", csr_kernel="merge", col_panels=4),
            "csr_stream": M.convert("csr", "f64", csr_kernel="stream"),
            "coo": M.convert("coo", "f64", block_nnz=256),
            "coo_panels": M.convert("coo", "f64", block_nnz=256, col_panels=4),
            "coo_f32": M.convert("coo", "f32"),
            "hyb": M.convert("hyb", "f64"),
            "merge_f16": M.convert("csr", "f16", csr_kernel="merge"),
            "ell": M.convert("ell", "f64")}


def test_noalloc_equals_spmv(orc):
    import torch
    from paper_2103_10116_amd import mxs
    al = mxs.TorchAllocator(0)
    ctx_na = mxs.Context(0, allocator=al)   # its allocator counts every block
    ctx = mxs.Context(0)
    big = I.zipf_random(40000, 2.0, 3000, seed=51)
    small = I.zipf_random(1500, 1.8, 400, seed=52)
    runs = []
    for A in (big, small):              # the second call has a smaller input
        mats = _mats(mxs, ctx_na, A)
        assert mats["hyb"].info()["coo_nnz"] > 0
        assert mats["csr_panels"].info()["col_panels"] == 4
        x = I.uniform_vector(A.n, 53)
        y0 = I.uniform_vector(A.n, 54)
        runs.append((A, mats, x, y0))
    torch.cuda.synchronize()
    calls = al.calls
    for A, mats, x, y0 in runs:
        scale = 1.5 * orc.absrow(A, x) + 0.5 * np.abs(y0)
        ref64 = orc.spmv_csr(A, x, alpha=1.5, beta=-0.5, y=y0)
        for name, B in mats.items():
            low = B.dtype != mxs.F64
            dt = torch.float32 if low else torch.float64
            xd = torch.from_numpy(x).to(dt).cuda()
            ya = torch.from_numpy(y0).to(dt).cuda()
            yb = ya.clone()
            mxs.spmv(ctx_na, B, xd, ya, 1.5, -0.5, noalloc=True)
            mxs.spmv(ctx, B, xd, yb, 1.5, -0.5)
            torch.cuda.synchronize()
            a, b = ya.cpu().numpy(), yb.cpu().numpy()
            assert np.array_equal(a.view(np.uint32 if low else np.uint64),
                                  b.view(np.uint32 if low else np.uint64)), name
            if name == "coo_f32":
                _, v32 = orc.cast_f32(A.val)
                A32 = I.CSRMatrix(A.n, A.ncols, A.rowptr, A.col, v32.astype(np.float64))
                x32 = x.astype(np.float32).astype(np.float64)
                y32 = y0.astype(np.float32).astype(np.float64)
                ref = orc.spmv_csr(A32, x32, alpha=1.5, beta=-0.5, y=y32)
                bound = 1e-5 * (1.5 * orc.absrow(A32, x32) + 0.5 * np.abs(y32))
                assert np.all(np.abs(a - ref) <= bound + 1e-30), name
            elif not low:
                assert np.all(np.abs(a - ref64) <= 1e-13 * scale + 1e-300), name
    assert al.calls == calls, "mxs_spmv_noalloc called the allocator"
    ctx_na.close()
    ctx.close()


def test_noalloc_refuses_more_scratch_than_it_holds():
    """A product whose scratch exceeds the fixed 64 MiB (column panels of a
    2^21-row matrix: 8 partials of 8 bytes a row, 128 MiB) is refused with
    MXS_UNSUPPORTED before anything is launched (y untouched); mxs_spmv
    runs it."""
    import torch
    from paper_2103_10116_amd import mxs
    ctx = mxs.Context(0)
    n = 1 << 21
    d = I.uniform_vector(n, 55) + 2.0
    D = I.CSRMatrix(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    B = mxs.Matrix.from_host(ctx, D).convert("csr", "f64", csr_kernel="merge", col_panels=8)
    assert B.info()["col_panels"] == 8
    x = torch.from_numpy(I.uniform_vector(n, 56)).cuda()
    y = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(mxs.MxsError) as e:
        mxs.spmv(ctx, B, x, y, noalloc=True)
    assert e.value.status == mxs.UNSUPPORTED
    assert torch.all(y == 7.0)
    mxs.spmv(ctx, B, x, y)
    assert torch.equal(y, torch.from_numpy(d).cuda() * x)
    ctx.close()
