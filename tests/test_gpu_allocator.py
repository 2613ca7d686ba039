"""A context whose device memory comes from a caller's allocator (the C ABI's
mxs_allocator, here backed by torch's caching allocator): every format's
product, the solver paths and the batch engine run on it, every block is
handed back, and a block that is not 16-byte aligned is refused."""
import numpy as np
import pytest

from paper_2103_10116_amd import inputs as I

pytestmark = pytest.mark.gpu


def _dev(torch, a, dt):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()


def test_torch_allocator(orc):
    import torch
    from paper_2103_10116_amd import mxs
    al = mxs.TorchAllocator(0)
    ctx = mxs.Context(0, allocator=al)
    A = I.zipf_random(3000, 2.0, 1200, seed=3)
    M = mxs.Matrix.from_host(ctx, A)
    x = I.uniform_vector(A.n, 41)
    ref = orc.spmv_csr(A, x)
    scale = orc.absrow(A, x)
    for fmt in ("csr", "coo", "ell", "hyb"):
        B = M.convert(fmt, "f64")
        y = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        mxs.spmv(ctx, B, _dev(torch, x, torch.float64), y)
        err = np.abs(y.cpu().numpy() - ref)
        assert (err <= 1e-13 * scale + 1e-300).all(), fmt
        B.close()
    assert al.calls > 0 and al.live
    # CG: the one-work-group path (CSR) and the multi-kernel path (COO)
    P = I.poisson2d(32)
    Pm = mxs.Matrix.from_host(ctx, P)
    b = orc.spmv_csr(P, np.ones(P.n))
    for fmt in ("csr", "coo"):
        B = Pm if fmt == "csr" else Pm.convert("coo", "f64")
        xs = torch.zeros(P.n, dtype=torch.float64, device="cuda")
        r = mxs.solve(ctx, "cg", B, _dev(torch, b, torch.float64), xs, tol=1e-10)
        assert r.status == mxs.OK
        assert orc.true_relres(P, b, xs.cpu().numpy()) <= 1e-10 * (1 + 1e-6)
        if B is not Pm:
            B.close()
    Pm.close()
    M.close()
    # the batch engine: its arena, tables and class buffers
    B = mxs.Batch(ctx, 64 << 20, 8, iters_per_step=8)
    sys_ = [(I.serving_system(m, 90 + m), I.serving_rhs(m * m, 90 + m)) for m in (8, 20, 41)]
    tickets = [B.submit(S, bs, 1e-10) for S, bs in sys_]
    for _ in range(100000):
        st = B.step()
        if st["active"] == 0 and st["pending"] == 0:
            break
    for (S, bs), t in zip(sys_, tickets):
        s, xb, res = B.poll(t, S.n)
        assert s == mxs.OK and orc.true_relres(S, bs, xb) <= 1e-10 * (1 + 1e-6), res
    B.close()
    ctx.close()
    assert not al.live, f"{len(al.live)} blocks not handed back"


def test_misaligned_allocator_refused():
    from paper_2103_10116_amd import mxs
    al = mxs.TorchAllocator(0, offset=8)
    with pytest.raises(mxs.MxsError) as e:
        ctx = mxs.Context(0, allocator=al)
        try:
            mxs.Matrix.from_host(ctx, I.poisson2d(8))
        finally:
            ctx.close()
    assert e.value.status == mxs.OOM
    assert al.calls >= 1 and not al.live
