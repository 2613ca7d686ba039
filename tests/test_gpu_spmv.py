"""GPU parity of ingest, conversions and SpMV against the CPU oracle, through
the C ABI.  Conversions must match bit for bit; FP64 products must agree per
entry within 1e-13 * (|alpha| sum_j |a_ij||x_j| + |beta||y_i|); FP32 and
FP16-row-scaled products within 1e-5 times the same scale, against the
oracle evaluated exactly on the rounded inputs."""
import numpy as np
import pytest

from conftest import load_golden
from paper_2103_10116_amd import inputs as I

pytestmark = pytest.mark.gpu

FORMATS = ["csr", "coo", "ell", "hyb"]


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2103_10116_amd import mxs
    ctx = mxs.Context(0)
    yield mxs, ctx, torch
    ctx.close()


def _dev(torch, a, dt=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dt is not None:
        t = t.to(dt)
    return t.cuda()


def golden_matrix():
    g = load_golden("formats_small.txt")
    return I.CSRMatrix(g["n"][0], g["ncols"][0], np.array(g["rowptr"], np.int32),
                       np.array(g["col"], np.int32), np.array(g["val"], float))


def matrix_zoo():
    """Small cases that span several work blocks and ragged tails."""
    zoo = {
        "golden": golden_matrix(),
        "one": I.dense_to_csr(np.array([[2.5]])),
        "poisson2d_64": I.poisson2d(64),
        "zipf_3000": I.zipf_random(3000, 2.0, 1200, seed=3),
        "zipf_rect": I.zipf_random(2500, 1.7, 700, seed=4, ncols=3001),
        "conv_13": I.convdiff3d(13),
        "st27_9": I.stencil27(9),
    }
    # every 7th row empty, row 101 longer than every block budget (1800
    # entries > 1024), 2113 rows (ragged against 64-row groups)
    g = I.rng(5)
    n = 2113
    M = I.zipf_random(n, 2.0, 40, seed=6)
    lens = M.row_lengths()
    rows = np.repeat(np.arange(n), lens)
    keep = (rows % 7 != 0) & (rows != 101)
    extra = np.sort(g.choice(n, 1800, replace=False))
    r = np.concatenate([rows[keep], np.full(len(extra), 101)])
    c = np.concatenate([M.col[keep], extra]).astype(np.int32)
    v = np.concatenate([M.val[keep], g.uniform(-1, 1, len(extra))])
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=rp[1:])
    zoo["empty_rows_longrow"] = I.CSRMatrix(n, n, rp.astype(np.int32), c, v)
    zoo["all_empty"] = I.CSRMatrix(70, 70, np.zeros(71, np.int32), np.zeros(0, np.int32),
                                   np.zeros(0))
    return zoo


ZOO = matrix_zoo()


# ---------------------------------------------------------------------------
# ingest
# ---------------------------------------------------------------------------
def test_create_rejects_invalid(env):
    mxs, ctx, torch = env
    A = golden_matrix()
    bad_cols = A.col.copy()
    bad_cols[1] = 0  # row 0 becomes (0, 0): duplicate
    for rp, ci, nc in [(A.rowptr, bad_cols, 6), (A.rowptr, A.col, 5),
                       (np.array([0, 2, 1, 5, 6, 10], np.int32), A.col, 6),
                       (np.array([0, 2, 2, 5, 6, 9], np.int32), A.col, 6)]:
        with pytest.raises(mxs.MxsError) as e:
            mxs.Matrix.from_csr(ctx, 5, nc, rp, ci, A.val)
        assert e.value.status == mxs.INVALID_MATRIX
    with pytest.raises(mxs.MxsError) as e:
        mxs.Matrix.from_csr(ctx, 5, 6, A.rowptr, A.col, A.val).convert("coo", "f16")
    assert e.value.status == mxs.UNSUPPORTED


def test_create_from_device_pointers(env, orc):
    mxs, ctx, torch = env
    A = ZOO["zipf_3000"]
    M = mxs.Matrix.from_csr(ctx, A.n, A.ncols, _dev(torch, A.rowptr), _dev(torch, A.col),
                            _dev(torch, A.val))
    assert np.array_equal(M.export(mxs.ARR_ROWPTR), A.rowptr)
    assert np.array_equal(M.export(mxs.ARR_COL), A.col)
    assert np.array_equal(M.export(mxs.ARR_VAL), A.val)


def _sort_sum_cases():
    g = load_golden("sort_and_sum_small.txt")
    cases = {"golden": (g["n"][0], g["ncols"][0], np.array(g["rowptr"], np.int32),
                        np.array(g["col"], np.int32), np.array(g["val"], float))}
    rp, col, val = I.unsorted_rows(3000, 4000, 60, 41, integer=False)
    cases["random_3000"] = (3000, 4000, rp, col, val)
    # rows at and around the in-LDS limit (2048 entries), and one of 5000
    # entries (sorted in global memory), with repeats; ragged row count
    gg = I.rng(42)
    lens = [0, 2048, 7, 2049, 1, 5000, 3, 64]
    cols = [gg.integers(0, 1800, L) for L in lens]
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    cases["long_rows"] = (len(lens), 1800, rp, np.concatenate(cols).astype(np.int32),
                          gg.uniform(-1, 1, int(rp[-1])))
    # every entry of a row repeats one column; rows already in order
    cases["all_repeats"] = (3, 5, np.array([0, 6, 6, 9], np.int32),
                            np.array([4, 4, 4, 4, 4, 4, 0, 1, 2], np.int32),
                            gg.uniform(-1, 1, 9))
    return cases


SORT_SUM = _sort_sum_cases()


@pytest.mark.parametrize("name", sorted(SORT_SUM))
@pytest.mark.parametrize("where", ["host", "device"])
def test_create_sort_and_sum(env, orc, name, where):
    """MXS_SORT_AND_SUM: the GPU's ordered, summed CSR equals the oracle's
    bit for bit (row pointers, columns, values), from host or device arrays;
    the product of the result agrees with the oracle's."""
    mxs, ctx, torch = env
    n, ncols, rp, col, val = SORT_SUM[name]
    st, (orp, oc, ov) = orc.csr_sort_and_sum(n, ncols, rp, col, val)
    assert st == orc.OK
    if where == "host":
        M = mxs.Matrix.from_csr(ctx, n, ncols, rp, col, val, sort_and_sum=True)
    else:
        M = mxs.Matrix.from_csr(ctx, n, ncols, _dev(torch, rp), _dev(torch, col),
                                _dev(torch, val), sort_and_sum=True)
    assert M.info()["nnz"] == len(oc)
    assert np.array_equal(M.export(mxs.ARR_ROWPTR), orp)
    assert np.array_equal(M.export(mxs.ARR_COL), oc)
    assert np.array_equal(M.export(mxs.ARR_VAL).view(np.uint64), ov.view(np.uint64))
    if name == "golden":
        g = load_golden("sort_and_sum_small.txt")
        assert np.array_equal(M.export(mxs.ARR_VAL), np.array(g["out_val"], float))
    A = I.CSRMatrix(n, ncols, orp, oc, ov)
    x = I.uniform_vector(ncols, 43)
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    for fmt in FORMATS:
        B = M if fmt == "csr" else M.convert(fmt, "f64")
        mxs.spmv(ctx, B, _dev(torch, x), y)
        _check(y.cpu().numpy(), orc.spmv_csr(A, x), orc.absrow(A, x), 1e-13)


def test_create_sort_and_sum_complex_and_rules(env, orc):
    """Complex values: parts summed separately in input order.  A valid CSR
    passes unchanged; without the flag unordered rows are rejected; with it
    a column out of range or bad row pointers still are."""
    mxs, ctx, torch = env
    rp, col, val = I.unsorted_rows(500, 300, 40, 44, integer=False)
    zv = val + 1j * I.uniform_vector(len(val), 45)
    st, (orp, oc, ov) = orc.csr_sort_and_sum(500, 300, rp, col, zv)
    Z = mxs.Matrix.from_host_complex(ctx, 500, 300, rp, col, zv, sort_and_sum=True)
    assert np.array_equal(Z.export(mxs.ARR_ROWPTR), orp)
    assert np.array_equal(Z.export(mxs.ARR_COL), oc)
    assert np.array_equal(Z.export(mxs.ARR_VAL).view(np.uint64),
                          ov.view(np.float64).view(np.uint64))
    A = ZOO["zipf_3000"]
    M = mxs.Matrix.from_csr(ctx, A.n, A.ncols, A.rowptr, A.col, A.val, sort_and_sum=True)
    assert np.array_equal(M.export(mxs.ARR_COL), A.col)
    assert np.array_equal(M.export(mxs.ARR_VAL).view(np.uint64), A.val.view(np.uint64))
    with pytest.raises(mxs.MxsError) as e:
        mxs.Matrix.from_csr(ctx, 500, 300, rp, col, val)
    assert e.value.status == mxs.INVALID_MATRIX
    bad = col.copy()
    bad[7] = 300
    with pytest.raises(mxs.MxsError) as e:
        mxs.Matrix.from_csr(ctx, 500, 300, rp, bad, val, sort_and_sum=True)
    assert e.value.status == mxs.INVALID_MATRIX
    rpb = rp.copy()
    rpb[250] = rp[-1] + 5        # past nnz, and the row pointers decrease after it
    with pytest.raises(mxs.MxsError) as e:
        mxs.Matrix.from_csr(ctx, 500, 300, rpb, col, val, sort_and_sum=True)
    assert e.value.status == mxs.INVALID_MATRIX


# ---------------------------------------------------------------------------
# conversions: bit-exact against the oracle's own conversions
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", sorted(ZOO))
def test_conversions_bit_exact(env, orc, name):
    mxs, ctx, torch = env
    A = ZOO[name]
    M = mxs.Matrix.from_host(ctx, A)
    coo_row = orc.csr_to_coo(A.n, A.rowptr)
    E = orc.csr_to_ell(A)
    for dt, vb in (("f64", 8), ("f32", 4)):
        st, v32 = orc.cast_f32(A.val)
        vals = A.val if dt == "f64" else v32
        cast = (lambda a: a) if dt == "f64" else (lambda a: orc.cast_f32(a)[1])
        C = M.convert("csr", dt)
        assert np.array_equal(C.export(mxs.ARR_ROWPTR), A.rowptr)
        assert np.array_equal(C.export(mxs.ARR_COL), A.col)
        assert np.array_equal(C.export(mxs.ARR_VAL).view(np.uint8), vals.view(np.uint8))
        C = M.convert("coo", dt)
        assert np.array_equal(C.export(mxs.ARR_ROW), coo_row)
        assert np.array_equal(C.export(mxs.ARR_COL), A.col)
        assert np.array_equal(C.export(mxs.ARR_VAL).view(np.uint8), vals.view(np.uint8))
        C = M.convert("ell", dt)
        assert (C.desc.ell_width, C.desc.ell_stride) == (E.K, E.stride)
        assert np.array_equal(C.export(mxs.ARR_ELL_COL), E.col)
        assert np.array_equal(C.export(mxs.ARR_ELL_VAL).view(np.uint8),
                              cast(E.val).view(np.uint8))
        H = orc.csr_to_hyb(A, vb)
        C = M.convert("hyb", dt)
        assert C.desc.ell_width == H.K and C.desc.coo_nnz == len(H.crow)
        assert np.array_equal(C.export(mxs.ARR_ELL_COL), H.ecol)
        assert np.array_equal(C.export(mxs.ARR_ELL_VAL).view(np.uint8),
                              cast(H.eval).view(np.uint8))
        assert np.array_equal(C.export(mxs.ARR_COO_ROW), H.crow)
        assert np.array_equal(C.export(mxs.ARR_COO_COL), H.ccol)
        assert np.array_equal(C.export(mxs.ARR_COO_VAL).view(np.uint8),
                              cast(H.cval).view(np.uint8))
    st, h, s = orc.rowscale_f16(A)
    C = M.convert("csr", "f16")
    assert np.array_equal(C.export(mxs.ARR_VAL), h)
    assert np.array_equal(C.export(mxs.ARR_SCALE), s)


def test_f32_range_rejected(env):
    mxs, ctx, torch = env
    A = I.dense_to_csr(np.array([[1.0, 4e38], [0.0, 2.0]]))
    M = mxs.Matrix.from_host(ctx, A)
    with pytest.raises(mxs.MxsError) as e:
        M.convert("csr", "f32")
    assert e.value.status == mxs.UNSUPPORTED


def test_forced_widths(env, orc):
    mxs, ctx, torch = env
    A = ZOO["zipf_3000"]
    M = mxs.Matrix.from_host(ctx, A)
    for K in (1, 3, 17):
        C = M.convert("hyb", "f64", ell_width=K)
        H = orc.csr_to_hyb(A, 8, K=K)
        assert np.array_equal(C.export(mxs.ARR_ELL_COL), H.ecol)
        assert np.array_equal(C.export(mxs.ARR_COO_COL), H.ccol)
    with pytest.raises(mxs.MxsError):
        M.convert("ell", "f64", ell_width=2)
    with pytest.raises(mxs.MxsError) as e:
        M.convert("ell", "f64", max_ell_bytes=1000)
    assert e.value.status == mxs.UNSUPPORTED


# ---------------------------------------------------------------------------
# SpMV parity
# ---------------------------------------------------------------------------
def _check(y, ref, scale, tol):
    err = np.abs(y - ref)
    bound = tol * scale + 1e-300
    bad = err > bound
    assert not bad.any(), f"{bad.sum()} entries out of bound; worst ratio {np.max(err / bound):.3g}"


# the work-unit shapes matter for CSR and COO (and for the COO part of HYB,
# which only the power-law matrix has); ELL and HYB run the default shape
_F64_CASES = [(name, fmt, bn, w) for name in sorted(ZOO) for fmt in FORMATS
              for bn, w in [(0, 0), (256, 1), (1024, 4), (512, 1)]
              if bn == 0 or fmt in ("csr", "coo") or name == "zipf_3000"]


@pytest.mark.parametrize("name,fmt,block_nnz,wpg", _F64_CASES)
def test_spmv_f64(env, orc, name, fmt, block_nnz, wpg):
    mxs, ctx, torch = env
    A = ZOO[name]
    M = mxs.Matrix.from_host(ctx, A)
    B = M.convert(fmt, "f64", block_nnz=block_nnz, waves_per_group=wpg)
    x = I.uniform_vector(A.ncols, 11)
    y0 = I.uniform_vector(A.n, 12)
    xd = _dev(torch, x)
    for alpha, beta in ((1.0, 0.0), (-2.5, 1.0), (0.5, -3.0)):
        y = _dev(torch, y0.copy()) if beta != 0 else torch.full((A.n,), float("nan"),
                                                                 dtype=torch.float64,
                                                                 device="cuda")
        mxs.spmv(ctx, B, xd, y, alpha, beta)
        ref = orc.spmv_csr(A, x, alpha, beta, y0 if beta != 0 else None)
        scale = abs(alpha) * orc.absrow(A, x) + abs(beta) * np.abs(y0)
        _check(y.cpu().numpy(), ref, scale, 1e-13)


CSR_VARIANTS = [dict(csr_kernel="stream", block_nnz=b, waves_per_group=w)
                for b in (256, 512, 1024) for w in (1, 4)] + [
    dict(csr_kernel="vector", lanes_per_row=g, rows_per_group=r)
    for g in (4, 8, 16, 32, 64) for r in (2, 4, 8)] + [
    dict(csr_kernel="vector", lanes_per_row=1)] + [
    dict(csr_kernel="rows_lds", block_nnz=b) for b in (0, 512, 1024, 2048)] + [
    dict(csr_kernel="rows_lds", block_nnz=b, lanes_per_row=g)
    for b in (512, 1024, 2048) for g in (1, 2, 4)] + [
    dict(csr_kernel="products", block_nnz=b, waves_per_group=w)
    for b in (0, 512, 1024, 2048) for w in (0, 1, 2, 4)] + [
    dict(csr_kernel="merge", block_nnz=b, waves_per_group=w)
    for b in (0, 256, 512, 1024) for w in (1, 4)] + [
    dict(csr_kernel="merge", block_nnz=b, waves_per_group=w, col_panels=p)
    for b in (256, 1024) for w in (1, 4) for p in (2, 4, 8)]


@pytest.mark.parametrize("name", sorted(ZOO))
@pytest.mark.parametrize("dt", ["f64", "f32", "f16"])
def test_spmv_csr_kernels(env, orc, name, dt):
    """Both CSR kernels with every work-unit shape, against the oracle."""
    mxs, ctx, torch = env
    A = ZOO[name]
    M = mxs.Matrix.from_host(ctx, A)
    x = I.uniform_vector(A.ncols, 18)
    y0 = I.uniform_vector(A.n, 19)
    if dt == "f64":
        Aref, xr, tol = A, x, 1e-13
    elif dt == "f32":
        _, v32 = orc.cast_f32(A.val)
        Aref = I.CSRMatrix(A.n, A.ncols, A.rowptr, A.col, v32.astype(np.float64))
        xr, tol = x.astype(np.float32).astype(np.float64), 1e-5
    else:
        _, h, sc = orc.rowscale_f16(A)
        dec = orc.f16_bits_to_f64(h) * np.repeat(sc.astype(np.float64), A.row_lengths())
        Aref = I.CSRMatrix(A.n, A.ncols, A.rowptr, A.col, dec)
        xr, tol = x.astype(np.float32).astype(np.float64), 1e-5
    y0r = y0.astype(np.float32).astype(np.float64) if dt != "f64" else y0
    ref = orc.spmv_csr(Aref, xr, 1.5, -0.5, y0r)
    scale = 1.5 * orc.absrow(Aref, xr) + 0.5 * np.abs(y0r)
    tdt = torch.float64 if dt == "f64" else torch.float32
    for opts in CSR_VARIANTS:
        B = M.convert("csr", dt, **opts)
        d = B.info()
        assert (d["lanes_per_row"] > 0) == (opts["csr_kernel"] in ("vector", "rows_lds"))
        if opts["csr_kernel"] == "rows_lds":
            g = d["lanes_per_row"]
            assert g == opts.get("lanes_per_row", g) and g in (1, 2, 4)
        assert d["csr_kernel"] == mxs.CSR_KERNELS[opts["csr_kernel"]]
        if opts["csr_kernel"] in ("rows_lds", "products", "merge") and opts["block_nnz"]:
            assert d["block_nnz"] == opts["block_nnz"]
        if "col_panels" in opts and A.nnz and A.ncols >= opts["col_panels"]:
            assert d["col_panels"] == opts["col_panels"]
        y = torch.from_numpy(y0r).to(tdt).cuda()
        mxs.spmv(ctx, B, torch.from_numpy(xr).to(tdt).cuda(), y, 1.5, -0.5)
        _check(y.cpu().numpy().astype(np.float64), ref, scale, tol)


@pytest.mark.parametrize("name", sorted(ZOO))
@pytest.mark.parametrize("kernel", ["lds", "runs"])
def test_spmv_coo_kernels(env, orc, name, kernel):
    """Both COO kernels (and the COO part of HYB, which the power-law matrices
    have at a forced width) at every chunk size and work-group shape, FP64
    and FP32, and both formats with their COO entries in 2 or 8 column
    panels; chunks of 256 entries leave ragged last chunks on every matrix."""
    mxs, ctx, torch = env
    A = ZOO[name]
    M = mxs.Matrix.from_host(ctx, A)
    x = I.uniform_vector(A.ncols, 21)
    y0 = I.uniform_vector(A.n, 22)
    _, v32 = orc.cast_f32(A.val)
    A32 = I.CSRMatrix(A.n, A.ncols, A.rowptr, A.col, v32.astype(np.float64))
    fmts = [("coo", 0)] + ([("hyb", 2)] if name.startswith("zipf") else [])
    for fmt, width in fmts:
        for dt, tdt, Ar, tol in (("f64", torch.float64, A, 1e-13),
                                 ("f32", torch.float32, A32, 1e-5)):
            xr = x.astype(np.float32).astype(np.float64) if dt == "f32" else x
            yr = y0.astype(np.float32).astype(np.float64) if dt == "f32" else y0
            ref = orc.spmv_csr(Ar, xr, 1.5, -0.5, yr)
            scale = 1.5 * orc.absrow(Ar, xr) + 0.5 * np.abs(yr)
            shapes = [(bn, wpg, 0) for bn in (256, 512, 1024) for wpg in (1, 4)]
            # entries (of COO, of the hybrid's COO part) in column-panel order
            shapes += [(bn, wpg, p) for bn in (256, 1024) for wpg in (1, 4) for p in (2, 8)]
            for bn, wpg, panels in shapes:
                extra = {"col_panels": panels} if panels else {}
                B = M.convert(fmt, dt, block_nnz=bn, waves_per_group=wpg,
                              coo_kernel=kernel, ell_width=width, **extra)
                d = B.info()
                assert d["block_nnz"] == bn and d["waves_per_group"] == wpg
                if d["coo_nnz"]:
                    assert d["coo_kernel"] == mxs.COO_KERNELS[kernel]
                if panels and d["coo_nnz"] and A.ncols >= panels:
                    assert d["col_panels"] == panels
                y = torch.from_numpy(yr).to(tdt).cuda()
                mxs.spmv(ctx, B, torch.from_numpy(xr).to(tdt).cuda(), y, 1.5, -0.5)
                _check(y.cpu().numpy().astype(np.float64), ref, scale, tol)
                B.close()


def test_coo_kernel_auto_choice(env):
    """AUTO keeps runs in registers for FP32 values when no row has more
    than 16 entries and stages products through LDS otherwise; an unknown
    kernel is rejected."""
    mxs, ctx, torch = env
    for name, want in (("poisson2d_64", mxs.COO_RUNS), ("conv_13", mxs.COO_RUNS),
                       ("zipf_3000", mxs.COO_LDS), ("st27_9", mxs.COO_LDS)):
        A = ZOO[name]
        assert (A.row_lengths().max() <= 16) == (want == mxs.COO_RUNS)
        M = mxs.Matrix.from_host(ctx, A)
        assert M.convert("coo", "f32").info()["coo_kernel"] == want
        assert M.convert("coo", "f64").info()["coo_kernel"] == mxs.COO_LDS
        assert M.convert("csr", "f64").info()["coo_kernel"] == 0
    with pytest.raises(mxs.MxsError):
        M.convert("coo", "f64", coo_kernel=3)


@pytest.mark.parametrize("name", sorted(ZOO))
@pytest.mark.parametrize("fmt", FORMATS)
def test_spmv_f32(env, orc, name, fmt):
    mxs, ctx, torch = env
    A = ZOO[name]
    M = mxs.Matrix.from_host(ctx, A)
    B = M.convert(fmt, "f32")
    _, v32 = orc.cast_f32(A.val)
    A32 = I.CSRMatrix(A.n, A.ncols, A.rowptr, A.col, v32.astype(np.float64))
    x = I.uniform_vector(A.ncols, 13).astype(np.float32)
    y0 = I.uniform_vector(A.n, 14).astype(np.float32)
    for alpha, beta in ((1.0, 0.0), (2.0, -1.0)):
        y = _dev(torch, y0.copy())
        mxs.spmv(ctx, B, _dev(torch, x), y, alpha, beta)
        ref = orc.spmv_csr(A32, x.astype(np.float64), alpha, beta, y0.astype(np.float64))
        scale = abs(alpha) * orc.absrow(A32, x.astype(np.float64)) + abs(beta) * np.abs(y0)
        _check(y.cpu().numpy().astype(np.float64), ref, scale, 1e-5)


@pytest.mark.parametrize("name", sorted(ZOO))
def test_spmv_f16_rowscaled(env, orc, name):
    mxs, ctx, torch = env
    A = ZOO[name]
    M = mxs.Matrix.from_host(ctx, A)
    B = M.convert("csr", "f16")
    st, h, s = orc.rowscale_f16(A)
    x = I.uniform_vector(A.ncols, 15).astype(np.float32)
    y = torch.zeros(A.n, dtype=torch.float32, device="cuda")
    mxs.spmv(ctx, B, _dev(torch, x), y, 1.0, 0.0)
    ref = orc.spmv_csr_f16(A, h, s, x.astype(np.float64))
    dec = orc.f16_bits_to_f64(h) * np.repeat(s.astype(np.float64), A.row_lengths())
    Ad = I.CSRMatrix(A.n, A.ncols, A.rowptr, A.col, dec)
    _check(y.cpu().numpy().astype(np.float64), ref, orc.absrow(Ad, x.astype(np.float64)), 1e-5)


def test_csr_merge_limits(env, orc):
    """The merge-path kernel refuses a chunk whose rows outgrow its LDS table
    (a long run of empty rows) and complex values; an all-empty matrix of
    many rows works (y = beta y)."""
    mxs, ctx, torch = env
    n = 2000
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = 1
    rp[n] = 2
    M = mxs.Matrix.from_csr(ctx, n, n, rp, np.array([0, n - 1], np.int32), np.array([2.0, 3.0]))
    with pytest.raises(mxs.MxsError) as e:
        M.convert("csr", "f64", csr_kernel="merge", block_nnz=256)
    assert e.value.status == mxs.UNSUPPORTED
    Z = mxs.Matrix.from_host_complex(ctx, 3, 3, np.array([0, 1, 2, 3], np.int32),
                                     np.array([0, 1, 2], np.int32), np.array([1 + 1j, 2, 3j]))
    with pytest.raises(mxs.MxsError):
        Z.convert("csr", "c128", csr_kernel="merge")
    # AUTO: a row over 64 entries asks for the merge path, but the one chunk
    # would span 3000 rows: the row-block stream kernel is used instead
    n2 = 3000
    rp2 = np.full(n2 + 1, 100, np.int32)
    rp2[0] = 0
    rp2[n2] = 101
    col2 = np.concatenate([np.arange(100) * 7, [5]]).astype(np.int32)
    val2 = I.uniform_vector(101, 61)
    A2 = I.CSRMatrix(n2, n2, rp2, col2, val2)
    M2 = mxs.Matrix.from_csr(ctx, n2, n2, rp2, col2, val2)
    assert M2.info()["csr_kernel"] == mxs.CSR_STREAM
    x2 = I.uniform_vector(n2, 62)
    y2 = torch.zeros(n2, dtype=torch.float64, device="cuda")
    mxs.spmv(ctx, M2, _dev(torch, x2), y2)
    ref2 = orc.spmv_csr(A2, x2)
    _check(y2.cpu().numpy(), ref2, orc.absrow(A2, x2), 1e-13)
    E = mxs.Matrix.from_csr(ctx, 300, 300, np.zeros(301, np.int32), np.zeros(0, np.int32),
                            np.zeros(0)).convert("csr", "f64", csr_kernel="merge")
    y = torch.ones(300, dtype=torch.float64, device="cuda")
    mxs.spmv(ctx, E, torch.ones(300, dtype=torch.float64, device="cuda"), y, 1.0, 2.0)
    assert torch.all(y == 2.0)


def test_spmv_empty_matrix(env):
    mxs, ctx, torch = env
    M = mxs.Matrix.from_csr(ctx, 0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32),
                            np.zeros(0))
    for fmt in FORMATS:
        B = M.convert(fmt, "f64")
        y = torch.zeros(0, dtype=torch.float64, device="cuda")
        mxs.spmv(ctx, B, torch.zeros(0, dtype=torch.float64, device="cuda"), y)
    ctx.synchronize()


def test_spmv_deterministic(env):
    mxs, ctx, torch = env
    A = ZOO["zipf_3000"]
    M = mxs.Matrix.from_host(ctx, A)
    x = _dev(torch, I.uniform_vector(A.n, 16))
    for fmt in FORMATS:
        B = M.convert(fmt, "f64")
        ys = []
        for _ in range(3):
            y = torch.zeros(A.n, dtype=torch.float64, device="cuda")
            mxs.spmv(ctx, B, x, y)
            ys.append(y.cpu().numpy())
        assert all(np.array_equal(ys[0].view(np.uint64), t.view(np.uint64)) for t in ys[1:])


def test_spmv_two_contexts_share_a_matrix(env, orc):
    """A matrix is read-only during a product: the chunked kernels (COO, the
    COO part of hybrid, merge-path CSR) keep their continuation partials in
    each context's own scratch, so two contexts on two streams may run
    products of the same matrix at the same time."""
    mxs, ctx, torch = env
    A = ZOO["zipf_3000"]
    M = mxs.Matrix.from_host(ctx, A)
    mats = {"csr_merge": M.convert("csr", "f64", csr_kernel="merge", block_nnz=256),
            "coo": M.convert("coo", "f64", block_nnz=256),
            "hyb": M.convert("hyb", "f64", block_nnz=256)}
    assert mats["hyb"].info()["coo_nnz"] > 0
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    c1, c2 = mxs.Context(0, stream=s1), mxs.Context(0, stream=s2)
    xs = [I.uniform_vector(A.n, 40 + k) for k in range(2)]
    xd = [_dev(torch, x) for x in xs]
    scale = [orc.absrow(A, x) for x in xs]
    refs = [orc.spmv_csr(A, x) for x in xs]
    reps = 12
    for name, B in mats.items():
        ys = [[torch.zeros(A.n, dtype=torch.float64, device="cuda") for _ in range(reps)]
              for _ in range(2)]
        torch.cuda.synchronize()
        for r in range(reps):   # interleaved launches on the two streams
            mxs.spmv(c1, B, xd[0], ys[0][r])
            mxs.spmv(c2, B, xd[1], ys[1][r])
        torch.cuda.synchronize()
        for k in range(2):
            for r in range(reps):
                _check(ys[k][r].cpu().numpy(), refs[k], scale[k], 1e-13)
    c1.close()
    c2.close()


@pytest.mark.slow
@pytest.mark.parametrize("which", ["stencil27_128", "zipf_2p20", "zipf_2p20_m16"])
def test_spmv_full_size(env, orc, which):
    """The benchmark's workloads at full size, every format, FP64 and FP32,
    all entries against the oracle."""
    mxs, ctx, torch = env
    if which == "stencil27_128":
        A = I.stencil27(128)
    elif which == "zipf_2p20":
        A = I.zipf_random(2 ** 20, 2.0, 4096)
    else:
        A = I.zipf_random(2 ** 20, 1.79, 4096)
    x = I.uniform_vector(A.n, 17)
    ref = orc.spmv_csr(A, x)
    scale = orc.absrow(A, x)
    _, v32 = orc.cast_f32(A.val)
    x32 = x.astype(np.float32)
    A32 = I.CSRMatrix(A.n, A.ncols, A.rowptr, A.col, v32.astype(np.float64))
    ref32 = orc.spmv_csr(A32, x32.astype(np.float64))
    scale32 = orc.absrow(A32, x32.astype(np.float64))
    M = mxs.Matrix.from_host(ctx, A)
    # COO in both kernels (AUTO picks one of them)
    cases = [("csr", {}), ("csr", {"csr_kernel": "merge", "col_panels": 1}),
             ("csr", {"csr_kernel": "merge", "col_panels": 8}), ("coo", {"coo_kernel": "lds"}),
             ("coo", {"coo_kernel": "runs"}), ("coo", {"col_panels": 1}), ("ell", {}),
             ("hyb", {})]
    if which == "stencil27_128":
        # the byte rule makes the hybrid all ELL here (K_h = 27): a forced
        # width of 20 sends 7 entries of every interior row to its COO part
        cases.append(("hyb", {"ell_width": 20}))
        # arrays above 256 MiB are streamed non-temporally: COO at the
        # 512-entry chunk (AUTO takes 256 there) and a hybrid whose COO part
        # (19 entries of every interior row, about 600 MB) is that large
        cases += [("coo", {"block_nnz": 512}), ("hyb", {"ell_width": 8})]
    for fmt, opts in cases:
        if fmt == "ell" and which == "zipf_2p20_m16":
            continue  # the same 4096-wide padded layout as zipf_2p20 (51.5 GB in FP64)
        B = M.convert(fmt, "f64", **opts)
        if fmt == "csr" and not opts and which != "stencil27_128":
            assert B.info()["col_panels"] == 4   # x of 8 MiB: slices of 2 MiB
        if fmt in ("coo", "hyb") and "col_panels" not in opts and B.info()["coo_nnz"]:
            # rows over 64 entries and an x of 8 MiB: panels; stencils: none
            assert B.info()["col_panels"] == (4 if which != "stencil27_128" else 1)
        if "ell_width" in opts:
            w = opts["ell_width"]
            assert B.info()["ell_width"] == w and B.info()["coo_nnz"] > (27 - w) * 120 ** 3
        if fmt == "coo" and which == "stencil27_128":
            assert B.info()["block_nnz"] == opts.get("block_nnz", 256)
        y = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        mxs.spmv(ctx, B, _dev(torch, x), y)
        _check(y.cpu().numpy(), ref, scale, 1e-13)
        del B
        B = M.convert(fmt, "f32", **opts)
        y = torch.zeros(A.n, dtype=torch.float32, device="cuda")
        mxs.spmv(ctx, B, _dev(torch, x32), y)
        _check(y.cpu().numpy().astype(np.float64), ref32, scale32, 1e-5)
        del B
