"""Pins for the CPU oracle (no GPU): every oracle routine is checked against
something other than itself -- hand-computed layouts, numpy's dense routines,
closed-form stencil eigenpairs, CG/GMRES finite termination, IEEE conversions
done by numpy -- chosen so that a dropped term, a wrong sign or index, or a
transposed operand fails at least one test."""
import numpy as np
import pytest

from conftest import load_golden
from paper_2103_10116_amd import inputs as I

U = 2.0 ** -53


def small_from_golden():
    g = load_golden("formats_small.txt")
    A = I.CSRMatrix(g["n"][0], g["ncols"][0], np.array(g["rowptr"], np.int32),
                    np.array(g["col"], np.int32), np.array(g["val"], float))
    return g, A


def random_pattern(n, m, density, seed, empty_rows=(), full_row=None):
    g = I.rng(seed)
    M = np.where(g.random((n, m)) < density, g.uniform(-1, 1, (n, m)), 0.0)
    for r in empty_rows:
        M[r, :] = 0.0
    if full_row is not None:
        M[full_row, :] = g.uniform(-1, 1, m)
    return M


# ---------------------------------------------------------------------------
# ingest
# ---------------------------------------------------------------------------
def test_validate_accepts_and_rejects(orc):
    g, A = small_from_golden()
    assert orc.validate(A.n, A.ncols, A.rowptr, A.col) == orc.OK
    bad = [
        (np.array([1, 2, 2, 5, 6, 10]), A.col),          # rowptr[0] != 0
        (np.array([0, 2, 1, 5, 6, 10]), A.col),          # not monotone
        (A.rowptr, np.array([0, 3, 1, 2, 5, 4, 0, 1, 2, 6])),   # col >= ncols
        (A.rowptr, np.array([3, 0, 1, 2, 5, 4, 0, 1, 2, 5])),   # unsorted row
        (A.rowptr, np.array([0, 0, 1, 2, 5, 4, 0, 1, 2, 5])),   # duplicate
        (A.rowptr, np.array([0, 3, -1, 2, 5, 4, 0, 1, 2, 5])),  # negative col
    ]
    for rp, ci in bad:
        assert orc.validate(A.n, A.ncols, rp, ci) == orc.INVALID_MATRIX


# ---------------------------------------------------------------------------
# conversions: hand-computed layouts and round trips
# ---------------------------------------------------------------------------
def test_sort_and_sum_golden(orc):
    """Hand-worked example: order within a row, ties in input order (the
    1e16 + 1 - 1e16 and 0.1 + 0.2 + 0.3 rows fix the summation order),
    empty and already-sorted rows, explicit zeros kept."""
    g = load_golden("sort_and_sum_small.txt")
    st, (rp, c, v) = orc.csr_sort_and_sum(g["n"][0], g["ncols"][0], np.array(g["rowptr"]),
                                          np.array(g["col"]), np.array(g["val"], float))
    assert st == orc.OK
    assert np.array_equal(rp, g["out_rowptr"]) and np.array_equal(c, g["out_col"])
    assert np.array_equal(v.view(np.uint64), np.array(g["out_val"], float).view(np.uint64))


@pytest.mark.parametrize("seed,max_len", [(1, 6), (2, 40), (3, 300)])
def test_sort_and_sum_vs_dense_accumulation(orc, seed, max_len):
    """Brute force: integer values make every sum exact whatever the order,
    so the result must equal a dense accumulation at exactly the (row, col)
    pairs the input lists, each row strictly ascending (a valid CSR)."""
    n, ncols = 60, 97
    rp, col, val = I.unsorted_rows(n, ncols, max_len, seed)
    st, (orp, oc, ov) = orc.csr_sort_and_sum(n, ncols, rp, col, val)
    assert st == orc.OK
    assert orc.validate(n, ncols, orp, oc) == orc.OK
    dense = np.zeros((n, ncols))
    present = np.zeros((n, ncols), bool)
    rows = np.repeat(np.arange(n), np.diff(rp))
    np.add.at(dense, (rows, col), val)
    present[rows, col] = True
    orows = np.repeat(np.arange(n), np.diff(orp))
    assert np.array_equal(present.nonzero()[0], orows)
    assert np.array_equal(present.nonzero()[1], oc)
    assert np.array_equal(dense[present], ov)
    # complex values: each part summed on its own
    cv = val + 1j * np.roll(val, 3)
    st, (_, oc2, ov2) = orc.csr_sort_and_sum(n, ncols, rp, col, cv)
    dz = np.zeros((n, ncols), complex)
    np.add.at(dz, (rows, col), cv)
    assert st == orc.OK and np.array_equal(oc2, oc) and np.array_equal(dz[present], ov2)


def test_sort_and_sum_identity_and_rejects(orc):
    """A valid CSR comes back unchanged, bit for bit; bad row pointers and
    columns out of range are still rejected."""
    A = I.zipf_random(800, 2.0, 120, seed=31)
    st, (rp, c, v) = orc.csr_sort_and_sum(A.n, A.ncols, A.rowptr, A.col, A.val)
    assert st == orc.OK and np.array_equal(rp, A.rowptr) and np.array_equal(c, A.col)
    assert np.array_equal(v.view(np.uint64), A.val.view(np.uint64))
    rp, col, val = I.unsorted_rows(10, 8, 5, 4)
    bad = col.copy()
    bad[3] = 8
    assert orc.csr_sort_and_sum(10, 8, rp, bad, val)[0] == orc.INVALID_MATRIX
    bad[3] = -1
    assert orc.csr_sort_and_sum(10, 8, rp, bad, val)[0] == orc.INVALID_MATRIX
    for k, d in ((0, 1), (10, -1), (5, 10 ** 6)):   # start, end, monotone
        rpb = rp.astype(np.int64).copy()
        rpb[k] += d
        assert orc.csr_sort_and_sum(10, 8, rpb.astype(np.int32), col, val)[0] == \
            orc.INVALID_MATRIX


def test_sort_and_sum_ties_keep_input_order(orc):
    """Three repeats whose sum depends on the order: only the input order
    gives (1e16 + 1) - 1e16 = 0; placed at random positions of long rows with
    random other columns, the sorted row still sums them in input order."""
    g = I.rng(77)
    n, ncols = 40, 500
    cols, vals, lens = [], [], []
    for i in range(n):
        other = g.choice(np.arange(1, ncols), size=30, replace=False)
        c = np.concatenate([other, [0, 0, 0]])
        v = np.concatenate([g.uniform(-1, 1, 30), [1e16, 1.0, -1e16]])
        perm = g.permutation(33)
        # keep the three repeats in their original relative order
        rep = np.sort(perm[30:])
        order = np.empty(33, np.int64)
        order[np.setdiff1d(np.arange(33), rep)] = g.permutation(30)
        order[rep] = [30, 31, 32]
        cols.append(c[order])
        vals.append(v[order])
        lens.append(33)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    st, (orp, oc, ov) = orc.csr_sort_and_sum(n, ncols, rp, np.concatenate(cols),
                                            np.concatenate(vals))
    assert st == orc.OK
    first = orp[:-1]
    assert np.array_equal(oc[first], np.zeros(n)) and np.array_equal(ov[first], np.zeros(n))


def test_formats_match_hand_layout(orc):
    g, A = small_from_golden()
    assert np.array_equal(orc.csr_to_coo(A.n, A.rowptr), g["coo_row"])
    E = orc.csr_to_ell(A)
    assert (E.K, E.stride) == (g["ell_K"][0], g["ell_stride"][0])
    exp_col = np.full(E.K * E.stride, -1, np.int32)
    exp_val = np.zeros(E.K * E.stride)
    for slot, c, v in g["ell_slot"]:
        exp_col[slot] = c
        exp_val[slot] = v
    assert np.array_equal(E.col, exp_col)
    assert np.array_equal(E.val, exp_val)
    assert not np.signbit(E.val[exp_col < 0]).any()  # padding is +0.0
    H = orc.csr_to_hyb(A, 8, K=1)
    assert np.array_equal(H.ecol, exp_col[:64]) and np.array_equal(H.eval, exp_val[:64])
    assert np.array_equal(H.crow, g["hyb1_coo_row"])
    assert np.array_equal(H.ccol, g["hyb1_coo_col"])
    assert np.array_equal(H.cval, g["hyb1_coo_val"])
    st, h, s = orc.rowscale_f16(A)
    assert st == orc.OK
    assert np.array_equal(s, np.array(g["f16_scale"], np.float32))
    assert np.array_equal(h, np.array(g["f16_bits"], np.uint16))


def test_spmv_all_formats_hand_example(orc):
    g, A = small_from_golden()
    x = np.array(g["x"], float)
    y = np.array(g["y"], float)
    assert np.array_equal(orc.spmv_csr(A, x), y)
    assert np.array_equal(orc.spmv_coo(A.n, orc.csr_to_coo(A.n, A.rowptr), A.col, A.val, x), y)
    assert np.array_equal(orc.spmv_ell(orc.csr_to_ell(A), x), y)
    for K in range(0, 5):
        assert np.array_equal(orc.spmv_hyb(orc.csr_to_hyb(A, 8, K=K), x), y)
    st, h, s = orc.rowscale_f16(A)
    assert np.array_equal(orc.spmv_csr_f16(A, h, s, x), y)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_round_trips(orc, seed):
    A = I.zipf_random(3000, 2.0, 200, seed=seed)
    row = orc.csr_to_coo(A.n, A.rowptr)
    assert np.array_equal(orc.coo_to_csr(A.n, row), A.rowptr)
    E = orc.csr_to_ell(A)
    # decode ELL column by column back to CSR arrays
    cols = E.col.reshape(E.K, E.stride)[:, :A.n].T
    vals = E.val.reshape(E.K, E.stride)[:, :A.n].T
    mask = cols >= 0
    assert np.array_equal(mask.sum(1), A.row_lengths())
    assert np.array_equal(cols[mask], A.col) and np.array_equal(vals[mask], A.val)
    assert (E.col.reshape(E.K, E.stride)[:, A.n:] == -1).all()
    for vb in (8, 4):
        H = orc.csr_to_hyb(A, vb)
        hc = H.ecol.reshape(H.K, H.stride)[:, :A.n].T
        lens = np.minimum(A.row_lengths(), H.K)
        assert np.array_equal((hc >= 0).sum(1), lens)
        assert len(H.crow) == int(np.maximum(A.row_lengths() - H.K, 0).sum())


def test_hyb_width_byte_rule(orc):
    # 64 rows (stride 64): an ELL column costs 64*(V+4) bytes and saves
    # count*(V+8) COO bytes; the column is kept only if it saves strictly more
    def width(nlong, vb):
        lens = np.zeros(64, np.int64)
        lens[:nlong] = 1
        rp = np.zeros(65, np.int32)
        rp[1:] = np.cumsum(lens)
        return orc.hyb_width(64, rp, vb)
    assert width(48, 8) == 0 and width(49, 8) == 1      # 48*16 == 64*12
    assert width(42, 4) == 0 and width(43, 4) == 1      # 43*12 > 64*8
    # a second column is kept only if it pays for itself too
    lens = np.array([3] * 60 + [1] * 4)
    rp = np.zeros(65, np.int32)
    rp[1:] = np.cumsum(lens)
    assert orc.hyb_width(64, rp, 8) == 3


def test_cast_f32_matches_ieee(orc):
    g = I.rng(5)
    v = np.concatenate([g.standard_normal(10000) * 10.0 ** g.integers(-45, 38, 10000) * 0.3,
                        [0.0, -0.0, np.inf, -np.inf, 3.4028234663852886e38, 1e-46, -1e-40]])
    st, out = orc.cast_f32(v)
    assert st == orc.OK
    with np.errstate(over="ignore"):
        ref = v.astype(np.float32)
    assert np.array_equal(out.view(np.uint32), ref.view(np.uint32))
    st, _ = orc.cast_f32(np.array([1.0, 3.5e38]))
    assert st == orc.UNSUPPORTED
    st, out = orc.cast_f32(np.array([np.nan]))
    assert st == orc.OK and np.isnan(out[0])


def test_f16_conversion_matches_ieee(orc):
    g = I.rng(6)
    v = np.concatenate([
        g.standard_normal(4000) * 2.0 ** g.integers(-30, 18, 4000),
        np.arange(-2048, 2049) * 2.0 ** -25,          # subnormal grid and its ties
        np.arange(0, 1025) * 2.0 ** -24 + 2.0 ** -25,  # exact ties between subnormals
        [65504.0, 65519.99, 65520.0, 1e6, -1e6, 2.0 ** -14, 2.0 ** -24, 2.0 ** -25,
         2.0 ** -25 * 1.0000001, 0.0, -0.0, np.inf, -np.inf],
        1.0 + np.arange(0, 64) * 2.0 ** -11,          # ties at 1.0 spacing
    ])
    bits = orc.f64_to_f16_bits(v)
    with np.errstate(over="ignore"):
        ref = v.astype(np.float16).view(np.uint16)
    assert np.array_equal(bits, ref)
    back = orc.f16_bits_to_f64(ref)
    with np.errstate(over="ignore"):
        assert np.array_equal(back, v.astype(np.float16).astype(np.float64))


# ---------------------------------------------------------------------------
# SpMV against dense products
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape,density,empty,full", [
    ((1, 1), 1.0, (), None), ((7, 7), 0.0, (), None), ((33, 40), 0.2, (0, 5, 32), 7),
    ((64, 64), 0.5, (3,), 63), ((50, 17), 0.3, (), 0)])
def test_spmv_vs_dense(orc, shape, density, empty, full):
    M = random_pattern(*shape, density, seed=sum(shape), empty_rows=empty, full_row=full)
    A = I.dense_to_csr(M)
    x = I.rng(9).uniform(-1, 1, shape[1])
    # naive sparse sum equals the naive dense loop exactly (same order,
    # zeros of the dense matrix add nothing)
    assert np.array_equal(orc.spmv_csr(A, x, mode="naive"), orc.dense_matvec(M, x))
    # accurate sums agree with numpy's dense product within its error bound
    bound = (shape[1] + 2) * U * (np.abs(M) @ np.abs(x)) + 1e-300
    y = orc.spmv_csr(A, x)
    assert (np.abs(y - M @ x) <= bound).all()
    # integer data and dyadic x: every product and partial sum is exact
    Mi = np.round(M * 8)
    Ai = I.dense_to_csr(Mi)
    xi = np.round(x * 1024) / 1024
    assert np.array_equal(orc.spmv_csr(Ai, xi), Mi @ xi)
    assert np.array_equal(orc.spmv_coo(Ai.n, orc.csr_to_coo(Ai.n, Ai.rowptr), Ai.col, Ai.val, xi), Mi @ xi)
    assert np.array_equal(orc.spmv_ell(orc.csr_to_ell(Ai), xi), Mi @ xi)
    assert np.array_equal(orc.spmv_hyb(orc.csr_to_hyb(Ai, 8), xi), Mi @ xi)


_DENSE_ZOO = [((1, 1), 1.0, (), None), ((7, 7), 0.0, (), None), ((33, 40), 0.2, (0, 5, 32), 7),
              ((64, 64), 0.5, (3,), 63), ((50, 17), 0.3, (), 0)]


@pytest.mark.parametrize("shape,density,empty,full", _DENSE_ZOO)
def test_absrow_vs_dense(orc, shape, density, empty, full):
    """The tolerance scale sum_j |a_ij| |x_j| of every parity check, against
    numpy's dense |M| |x| (a different summation order: within (L+1)u).
    The matrix is rectangular or nonsymmetric and x has no symmetry, so a
    row/column swap, a dropped modulus or a wrong index fails."""
    M = random_pattern(*shape, density, seed=sum(shape) + 1, empty_rows=empty, full_row=full)
    A = I.dense_to_csr(M)
    x = I.rng(19).uniform(-1, 1, shape[1])
    ref = np.abs(M) @ np.abs(x)
    got = orc.absrow(A, x)
    assert np.all(np.abs(got - ref) <= (shape[1] + 1) * U * ref)
    for r in empty:
        assert got[r] == 0.0
    # it bounds the product it scales: |y_i| <= sum_j |a_ij| |x_j|
    assert np.all(np.abs(orc.spmv_csr(A, x)) <= got * (1 + 4 * U))
    # x with one nonzero entry picks one column of |M|, exactly
    if shape[1] > 1 and density > 0:
        e = np.zeros(shape[1])
        e[shape[1] // 2] = -2.0
        assert np.array_equal(orc.absrow(A, e), 2.0 * np.abs(M[:, shape[1] // 2]))


@pytest.mark.parametrize("shape,density,empty,full", _DENSE_ZOO)
def test_absrow_z_vs_dense(orc, shape, density, empty, full):
    """Complex moduli: numpy's dense |M| |x| with |.| the complex modulus."""
    M = random_pattern(*shape, density, seed=sum(shape) + 2, empty_rows=empty, full_row=full)
    g = I.rng(23)
    Mz = M + 1j * np.where(M != 0, g.uniform(-1, 1, M.shape), 0.0)
    A = I.dense_to_csr(M)                       # the pattern of Mz (same nonzeros)
    zval = Mz[M != 0]                           # row-major, columns ascending
    x = g.uniform(-1, 1, shape[1]) + 1j * g.uniform(-1, 1, shape[1])
    ref = np.abs(Mz) @ np.abs(x)
    got = orc.absrow_z(A.n, A.rowptr, A.col, zval, x)
    assert np.all(np.abs(got - ref) <= (shape[1] + 2) * U * ref)
    # a purely imaginary matrix has the same scale as its real magnitudes
    zim = 1j * np.abs(A.val)
    assert np.array_equal(orc.absrow_z(A.n, A.rowptr, A.col, zim, np.abs(x) + 0j),
                          orc.absrow(I.CSRMatrix(A.n, A.ncols, A.rowptr, A.col, np.abs(A.val)),
                                     np.abs(x)))


def test_spmv_accurate_beats_naive(orc):
    # catastrophic cancellation: 1e16 + 1 - 1e16 is 1 exactly
    A = I.dense_to_csr(np.array([[1e16, 1.0, -1e16]]))
    x = np.ones(3)
    assert orc.spmv_csr(A, x)[0] == 1.0
    assert orc.spmv_csr(A, x, mode="naive")[0] == 0.0


def test_spmv_alpha_beta(orc):
    g, A = small_from_golden()
    x = np.array(g["x"], float)
    y = np.array(g["y"], float)
    y0 = np.array([1.0, -2.0, 0.5, 4.0, 8.0])
    assert np.array_equal(orc.spmv_csr(A, x, alpha=2.0, beta=-1.0, y=y0), 2.0 * y - y0)
    nan_y = np.full(5, np.nan)
    for f in (lambda yy: orc.spmv_csr(A, x, 1.5, 0.0, yy),
              lambda yy: orc.spmv_ell(orc.csr_to_ell(A), x, 1.5, 0.0, yy),
              lambda yy: orc.spmv_hyb(orc.csr_to_hyb(A, 8, K=1), x, 1.5, 0.0, yy),
              lambda yy: orc.spmv_coo(A.n, orc.csr_to_coo(A.n, A.rowptr), A.col, A.val, x, 1.5, 0.0, yy)):
        assert np.array_equal(f(nan_y), 1.5 * y)   # beta == 0 never reads y


def test_spmv_formats_agree_on_power_law(orc):
    A = I.zipf_random(5000, 2.0, 1000, seed=11)
    x = I.uniform_vector(A.n, 12)
    y = orc.spmv_csr(A, x)
    assert np.array_equal(orc.spmv_coo(A.n, orc.csr_to_coo(A.n, A.rowptr), A.col, A.val, x), y)
    assert np.array_equal(orc.spmv_ell(orc.csr_to_ell(A), x), y)
    assert np.array_equal(orc.spmv_hyb(orc.csr_to_hyb(A, 8), x), y)


# ---------------------------------------------------------------------------
# closed-form eigenpairs of the stencil matrices
# ---------------------------------------------------------------------------
def _modes(N, k, w=None):
    j = np.arange(1, N + 1)
    s = np.sin(j * k * np.pi / (N + 1))
    return s if w is None else s * w ** (j / 2.0)


def _check_eig(orc, A, v, lam):
    r = orc.spmv_csr(A, v) - lam * v
    scale = orc.absrow(A, v).max()
    assert np.abs(r).max() <= 1e-13 * scale, np.abs(r).max() / scale


@pytest.mark.parametrize("m,j,k", [(64, 1, 1), (64, 64, 64), (64, 3, 50), (9, 2, 7)])
def test_poisson2d_eigenpairs(orc, m, j, k):
    A = I.poisson2d(m)
    vx, vy = _modes(m, j), _modes(m, k)
    v = np.outer(vy, vx).ravel()  # index = x + m*y
    lam = 4 - 2 * np.cos(j * np.pi / (m + 1)) - 2 * np.cos(k * np.pi / (m + 1))
    _check_eig(orc, A, v, lam)


@pytest.mark.parametrize("N,ks", [(16, (1, 1, 1)), (16, (16, 2, 9)), (128, (1, 1, 1)), (128, (128, 64, 3))])
def test_poisson3d_eigenpairs(orc, N, ks):
    A = I.poisson3d(N)
    m = [_modes(N, k) for k in ks]
    v = np.einsum("z,y,x->zyx", m[2], m[1], m[0]).ravel()
    lam = 6 - sum(2 * np.cos(k * np.pi / (N + 1)) for k in ks)
    _check_eig(orc, A, v, lam)


@pytest.mark.parametrize("N,ks", [(12, (1, 1, 1)), (12, (12, 5, 2)), (40, (1, 40, 7))])
def test_stencil27_eigenpairs(orc, N, ks):
    A = I.stencil27(N)
    assert A.nnz == (3 * N - 2) ** 3
    m = [_modes(N, k) for k in ks]
    v = np.einsum("z,y,x->zyx", m[2], m[1], m[0]).ravel()
    lam = 27 - np.prod([1 + 2 * np.cos(k * np.pi / (N + 1)) for k in ks])
    _check_eig(orc, A, v, lam)


@pytest.mark.parametrize("N,ks", [(16, (1, 1, 1)), (16, (16, 3, 8)), (64, (2, 64, 31))])
def test_convdiff_eigenpairs(orc, N, ks):
    c = 10.0
    h = 1.0 / (N + 1)
    A = I.convdiff3d(N, c)
    w = 1 + c * h  # sub-diagonal (upwind) coefficient magnitude
    m = [_modes(N, k, w) for k in ks]
    v = np.einsum("z,y,x->zyx", m[2], m[1], m[0]).ravel()
    lam = sum((2 + c * h) - 2 * np.sqrt(w) * np.cos(k * np.pi / (N + 1)) for k in ks)
    _check_eig(orc, A, v, lam)


# ---------------------------------------------------------------------------
# dense LU
# ---------------------------------------------------------------------------
def test_lu_vs_numpy(orc):
    g = I.rng(21)
    for n in (1, 2, 5, 30):
        M = g.standard_normal((n, n)) + n * np.eye(n) * (g.random() > 0.5)
        b = g.standard_normal(n)
        st, x = orc.lu_solve(M, b)
        assert st == orc.OK
        xr = np.linalg.solve(M, b)
        assert np.linalg.norm(x - xr) <= 1e-12 * np.linalg.cond(M) * np.linalg.norm(xr)
    st, _ = orc.lu_solve(np.zeros((3, 3)), np.ones(3))
    assert st == orc.BREAKDOWN


def test_openmp_timing_build_matches(orc):
    """The OpenMP build of the same source (host-baseline timing only) gives
    the single-thread build's products bit for bit (rows are independent),
    and its CG, whose inner products are summed in another order, converges
    on the same system to the same tolerance."""
    A = I.stencil27(12)
    x = I.uniform_vector(A.n, 5)
    y1 = orc.spmv_csr(A, x)
    b = orc.spmv_csr(A, np.ones(A.n))
    r1 = orc.cg(A, b, tol=1e-10)
    prev = orc.use_threads(4)
    try:
        assert np.array_equal(orc.spmv_csr(A, x).view(np.uint64), y1.view(np.uint64))
        r4 = orc.cg(A, b, tol=1e-10)
        assert r4.status == orc.OK and r4.relres_true <= 1e-10 * (1 + 1e-6)
        assert abs(r4.iters - r1.iters) <= 2
    finally:
        orc.use_threads(prev)
    assert orc.lib() is orc._libs[orc._LIB]
