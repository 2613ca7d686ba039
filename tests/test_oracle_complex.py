"""Pins for the oracle's complex CSR product: it equals the real product of
the 2n x 2n real embedding [[Re A, -Im A], [Im A, Re A]] (computed by the
already-pinned real oracle), reduces to the real product for real data, and
matches numpy's dense complex arithmetic for complex alpha and beta."""
import numpy as np
import pytest

from paper_2103_10116_amd import inputs as I

U = 2.0 ** -53


def _complex_matrix(n, seed, density=0.05):
    g = I.rng(seed)
    A = I.zipf_random(n, 2.0, 64, seed)
    vi = g.uniform(-1, 1, A.nnz)
    return A, A.val + 1j * vi


def _embed(A, zval):
    """Real CSR of [[Re A, -Im A], [Im A, Re A]] (columns ascending)."""
    n = A.n
    rows, cols, vals = [], [], []
    for top in (True, False):
        for i in range(n):
            s, e = A.rowptr[i], A.rowptr[i + 1]
            c = A.col[s:e]
            re, im = zval[s:e].real, zval[s:e].imag
            left, right = (re, -im) if top else (im, re)
            rows.append(np.full(2 * (e - s), i if top else n + i))
            cols.append(np.concatenate([c, n + c]))
            vals.append(np.concatenate([left, right]))
    rows, cols, vals = map(np.concatenate, (rows, cols, vals))
    rp = np.zeros(2 * n + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    return I.CSRMatrix(2 * n, 2 * n, np.cumsum(rp).astype(np.int32), cols.astype(np.int32), vals)


def test_complex_equals_real_embedding(orc):
    A, z = _complex_matrix(3000, 70)
    g = I.rng(71)
    x = g.uniform(-1, 1, A.n) + 1j * g.uniform(-1, 1, A.n)
    y = orc.spmv_csr_z(A.n, A.rowptr, A.col, z, x)
    E = _embed(A, z)
    yr = orc.spmv_csr(E, np.concatenate([x.real, x.imag]))
    scale = orc.absrow_z(A.n, A.rowptr, A.col, z, x)
    assert np.all(np.abs(y.real - yr[:A.n]) <= 2 * U * scale)
    assert np.all(np.abs(y.imag - yr[A.n:]) <= 2 * U * scale)


def test_complex_reduces_to_real(orc):
    A = I.zipf_random(2000, 2.0, 64, 72)
    x = I.uniform_vector(A.n, 73)
    y = orc.spmv_csr_z(A.n, A.rowptr, A.col, A.val.astype(np.complex128), x.astype(np.complex128))
    assert np.array_equal(y.real, orc.spmv_csr(A, x)) and not y.imag.any()


@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (0.5 - 2j, 0.0), (1.5 + 0.25j, -0.5 + 1j)])
def test_complex_vs_numpy_dense(orc, alpha, beta):
    A, z = _complex_matrix(300, 74)
    D = np.zeros((A.n, A.n), np.complex128)
    for i in range(A.n):
        D[i, A.col[A.rowptr[i]:A.rowptr[i + 1]]] = z[A.rowptr[i]:A.rowptr[i + 1]]
    g = I.rng(75)
    x = g.uniform(-1, 1, A.n) + 1j * g.uniform(-1, 1, A.n)
    y0 = g.uniform(-1, 1, A.n) + 1j * g.uniform(-1, 1, A.n)
    y = orc.spmv_csr_z(A.n, A.rowptr, A.col, z, x, alpha, beta, y0)
    ref = alpha * (D @ x) + beta * y0
    L = np.diff(A.rowptr).max()
    scale = abs(alpha) * orc.absrow_z(A.n, A.rowptr, A.col, z, x) + abs(beta) * np.abs(y0)
    assert np.all(np.abs(y - ref) <= 4 * (2 * L + 8) * U * scale + 1e-300)
    if beta == 0.0:  # beta == 0 never reads y
        yn = orc.spmv_csr_z(A.n, A.rowptr, A.col, z, x, alpha, 0.0, np.full(A.n, np.nan + 0j))
        assert np.array_equal(yn, orc.spmv_csr_z(A.n, A.rowptr, A.col, z, x, alpha, 0.0))
