"""Complex CSR products (C128 and C64) through the C ABI against the
oracle's complex product, every CSR kernel, with complex alpha and beta;
exported values bit-exact; the complex paths that are not offered fail
with MXS_UNSUPPORTED."""
import numpy as np
import pytest

from paper_2103_10116_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2103_10116_amd import mxs
    ctx = mxs.Context(0)
    yield mxs, ctx, torch
    ctx.close()


def _zoo():
    out = {}
    for k, (name, A) in enumerate((("powerlaw", I.zipf_random(6000, 2.0, 4096, 80)),
                                   ("stencil27", I.stencil27(14)),
                                   ("poisson2d", I.poisson2d(40)))):
        g = I.rng(90 + k)
        out[name] = (A, A.val + 1j * g.uniform(-1, 1, A.nnz))
    # empty rows and an empty matrix row block
    A = I.dense_to_csr(np.array([[0, 1.0, 0, 0], [0, 0, 0, 0], [2.0, 0, 0, 3.0], [0, 0, 0, 0]]))
    out["empty_rows"] = (A, A.val * (1 - 0.5j))
    return out


ZOO = _zoo()
KERNELS = [dict(), dict(csr_kernel="stream", block_nnz=256), dict(csr_kernel="stream", block_nnz=1024),
           dict(csr_kernel="products", block_nnz=512), dict(csr_kernel="products", block_nnz=2048),
           dict(csr_kernel="rows_lds", block_nnz=1024), dict(csr_kernel="rows_lds", block_nnz=512, lanes_per_row=2),
           dict(csr_kernel="rows_lds", block_nnz=2048, lanes_per_row=4), dict(csr_kernel="vector", lanes_per_row=8),
           dict(csr_kernel="vector", lanes_per_row=1)]


@pytest.mark.parametrize("name", sorted(ZOO))
@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_complex_spmv(env, orc, name, dt):
    mxs, ctx, torch = env
    A, z = ZOO[name]
    M = mxs.Matrix.from_host_complex(ctx, A.n, A.ncols, A.rowptr, A.col, z)
    g = I.rng(81)
    x = g.uniform(-1, 1, A.ncols) + 1j * g.uniform(-1, 1, A.ncols)
    y0 = g.uniform(-1, 1, A.n) + 1j * g.uniform(-1, 1, A.n)
    tdt = torch.complex128 if dt == "c128" else torch.complex64
    if dt == "c64":  # the oracle on the rounded inputs
        zr, xr, yr = (np.asarray(v, np.complex64).astype(np.complex128) for v in (z, x, y0))
        tol = 1e-5
    else:
        zr, xr, yr = z, x, y0
        tol = 1e-13
    for alpha, beta in ((1.0, 0.0), (0.5 - 1.5j, 0.25 + 1j)):
        ab = (alpha, beta) if dt == "c128" else tuple(complex(np.complex64(v)) for v in (alpha, beta))
        ref = orc.spmv_csr_z(A.n, A.rowptr, A.col, zr, xr, ab[0], ab[1], yr)
        scale = abs(ab[0]) * orc.absrow_z(A.n, A.rowptr, A.col, zr, xr) + abs(ab[1]) * np.abs(yr)
        for opts in KERNELS:
            B = M.convert("csr", dt, **opts)
            y = torch.from_numpy(y0).to(tdt).cuda()
            if beta == 0.0:
                y.fill_(complex(np.nan, np.nan))
            mxs.spmv(ctx, B, torch.from_numpy(x).to(tdt).cuda(), y, alpha, beta)
            got = y.cpu().numpy().astype(np.complex128)
            assert np.all(np.abs(got - ref) <= tol * scale + 1e-300), (name, dt, opts)
            B.close()


@pytest.mark.slow
def test_complex_spmv_full_size(env, orc):
    """The 27-point 128^3 pattern with complex values (1.1 GB as C128, 0.67 GB
    as C64: both streamed with non-temporal loads) in AUTO's kernel and in
    rows-from-LDS at 1024-entry blocks, against the oracle's complex product
    per entry."""
    mxs, ctx, torch = env
    A = I.stencil27(128)
    g = I.rng(95)
    z = A.val + 1j * g.uniform(-1, 1, A.nnz)
    x = g.uniform(-1, 1, A.ncols) + 1j * g.uniform(-1, 1, A.ncols)
    M = mxs.Matrix.from_host_complex(ctx, A.n, A.ncols, A.rowptr, A.col, z)
    for dt, tol in (("c128", 1e-13), ("c64", 1e-5)):
        if dt == "c64":
            zr, xr = (np.asarray(v, np.complex64).astype(np.complex128) for v in (z, x))
        else:
            zr, xr = z, x
        ref = orc.spmv_csr_z(A.n, A.rowptr, A.col, zr, xr, 1.0, 0.0, np.zeros(A.n, complex))
        scale = orc.absrow_z(A.n, A.rowptr, A.col, zr, xr)
        tdt = torch.complex128 if dt == "c128" else torch.complex64
        for opts in (dict(), dict(csr_kernel="rows_lds", block_nnz=1024)):
            B = M.convert("csr", dt, **opts)
            y = torch.zeros(A.n, dtype=tdt, device="cuda")
            mxs.spmv(ctx, B, torch.from_numpy(x).to(tdt).cuda(), y)
            got = y.cpu().numpy().astype(np.complex128)
            assert np.all(np.abs(got - ref) <= tol * scale + 1e-300), (dt, opts)
            B.close()
    M.close()


def test_complex_export_and_limits(env, orc):
    mxs, ctx, torch = env
    A, z = ZOO["powerlaw"]
    M = mxs.Matrix.from_host_complex(ctx, A.n, A.ncols, A.rowptr, A.col, z)
    assert M.info()["dtype"] == mxs.C128
    assert np.array_equal(M.export(mxs.ARR_VAL).view(np.uint64), z.view(np.uint64))
    assert np.array_equal(M.export(mxs.ARR_COL), A.col)
    L = M.convert("csr", "c64")
    assert np.array_equal(L.export(mxs.ARR_VAL).view(np.uint32),
                          z.astype(np.complex64).view(np.uint32))
    for fmt, dt in (("coo", "c128"), ("ell", "c64"), ("csr", "f64")):
        with pytest.raises(mxs.MxsError) as e:
            M.convert(fmt, dt)
        assert e.value.status == mxs.UNSUPPORTED
    R = mxs.Matrix.from_host(ctx, A)
    with pytest.raises(mxs.MxsError) as e:
        R.convert("csr", "c128")
    assert e.value.status == mxs.UNSUPPORTED
    b = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    r = mxs.solve(ctx, "cg", M, b, b.clone(), raise_on_error=False)
    assert r.status == mxs.UNSUPPORTED
    big = z.copy()
    big[0] = 1e300 + 0j
    Mb = mxs.Matrix.from_host_complex(ctx, A.n, A.ncols, A.rowptr, A.col, big)
    with pytest.raises(mxs.MxsError) as e:
        Mb.convert("csr", "c64")
    assert e.value.status == mxs.UNSUPPORTED
    bad = A.col.copy()
    bad[1] = bad[0]
    with pytest.raises(mxs.MxsError) as e:
        mxs.Matrix.from_host_complex(ctx, A.n, A.ncols, A.rowptr, bad, z)
    assert e.value.status == mxs.INVALID_MATRIX
