"""Pins for the oracle's Krylov solvers and iterative refinement (no GPU):
finite termination, eigenvector right-hand sides, Lanczos/Ritz values against
closed-form spectra, dense solves by numpy and by the oracle's LU, breakdown
and failure cases."""
import numpy as np
import pytest

from paper_2103_10116_amd import inputs as I


def _relerr(x, xr):
    return np.linalg.norm(x - xr) / np.linalg.norm(xr)


# ---------------------------------------------------------------------------
# CG
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,seed", [(4, 1), (10, 2), (16, 3)])
def test_cg_finite_termination(orc, n, seed):
    # exact arithmetic ends in <= n steps; with kappa = 10 rounding does not
    # delay it (larger kappa loses orthogonality and needs extra steps)
    M = I.random_spd_small(n, 10.0, seed)
    A = I.dense_to_csr(M)
    b = I.rng(seed + 50).standard_normal(n)
    r = orc.cg(A, b, tol=1e-12, maxit=n)
    assert r.status == orc.OK and r.iters <= n
    assert r.relres_true <= 1e-12
    xr = np.linalg.solve(M, b)
    assert _relerr(r.x, xr) <= 10.0 * 1e-10
    st, xl = orc.lu_solve(M, b)
    assert _relerr(r.x, xl) <= 10.0 * 1e-10


def test_cg_eigenvector_rhs_one_step(orc):
    m = 12
    A = I.poisson2d(m)
    j, k = 3, 5
    s = lambda kk: np.sin(np.arange(1, m + 1) * kk * np.pi / (m + 1))
    v = np.outer(s(k), s(j)).ravel()
    lam = 4 - 2 * np.cos(j * np.pi / (m + 1)) - 2 * np.cos(k * np.pi / (m + 1))
    r = orc.cg(A, v, tol=1e-12)
    assert r.status == orc.OK and r.iters == 1
    assert _relerr(r.x, v / lam) <= 1e-13


def test_cg_k_eigenvectors_k_steps(orc):
    m = 12
    A = I.poisson2d(m)
    s = lambda kk: np.sin(np.arange(1, m + 1) * kk * np.pi / (m + 1))
    pairs = [(1, 1), (2, 5), (7, 3), (12, 12)]  # four distinct eigenvalues
    b = sum(np.outer(s(k), s(j)).ravel() * (i + 1) for i, (j, k) in enumerate(pairs))
    r = orc.cg(A, b, tol=1e-11)
    assert r.status == orc.OK and r.iters <= len(pairs)


def test_cg_ritz_values_match_closed_form(orc):
    # the Lanczos tridiagonal built from CG's (alpha, beta) has extreme
    # eigenvalues converging to those of A (2D 5-point, 64 x 64)
    m = 64
    A = I.poisson2d(m)
    b = I.uniform_vector(A.n, 3)
    r = orc.cg(A, b, tol=1e-10, hist=True)
    assert r.status == orc.OK
    al, be = r.hist[:, 0], r.hist[:, 1]
    k = len(al)
    T = np.zeros((k, k))
    for i in range(k):
        T[i, i] = 1.0 / al[i] + (be[i - 1] / al[i - 1] if i > 0 else 0.0)
        if i + 1 < k:
            T[i, i + 1] = T[i + 1, i] = np.sqrt(be[i]) / al[i]
    ev = np.linalg.eigvalsh(T)
    lmin = 4 - 4 * np.cos(np.pi / (m + 1))
    lmax = 4 + 4 * np.cos(np.pi / (m + 1))
    assert abs(ev[0] - lmin) <= 1e-8 * lmin
    assert abs(ev[-1] - lmax) <= 1e-8 * lmax


def test_cg_poisson_64(orc):
    A = I.poisson2d(64)
    b = orc.spmv_csr(A, np.ones(A.n))
    r = orc.cg(A, b, tol=1e-10)
    assert r.status == orc.OK and r.relres_true <= 1e-10
    assert 100 <= r.iters <= 200
    assert _relerr(r.x, np.ones(A.n)) <= 1711.7 * 1e-10


def test_cg_special_cases(orc):
    A = I.poisson2d(8)
    r = orc.cg(A, np.zeros(A.n))
    assert r.status == orc.OK and r.iters == 0 and not r.x.any()
    b = np.ones(A.n)
    b[3] = np.nan
    assert orc.cg(A, b).status == orc.NONFINITE
    r = orc.cg(A, np.ones(A.n), maxit=3)
    assert r.status == orc.NOT_CONVERGED and r.iters == 3
    # indefinite matrix: p.Ap <= 0 somewhere
    M = np.diag([1.0, -1.0, 2.0, -3.0])
    r = orc.cg(I.dense_to_csr(M), np.ones(4))
    assert r.status == orc.BREAKDOWN
    # already converged initial guess: 0 iterations
    x0 = r_ = orc.cg(A, np.ones(A.n)).x
    r = orc.cg(A, np.ones(A.n), x0=x0)
    assert r.status == orc.OK and r.iters == 0


# ---------------------------------------------------------------------------
# BiCGSTAB
# ---------------------------------------------------------------------------
def test_bicgstab_scaled_identity(orc):
    n = 20
    A = I.dense_to_csr(3.0 * np.eye(n))
    b = I.uniform_vector(n, 4)
    r = orc.bicgstab(A, b, tol=1e-14)
    assert r.status == orc.OK and r.iters == 1
    assert np.allclose(r.x, b / 3.0, rtol=1e-15, atol=0)


@pytest.mark.parametrize("n,seed", [(6, 1), (25, 2)])
def test_bicgstab_nonsymmetric_vs_numpy(orc, n, seed):
    g = I.rng(seed)
    M = g.standard_normal((n, n)) * 0.3 + np.diag(np.full(n, 3.0))
    b = g.standard_normal(n)
    r = orc.bicgstab(I.dense_to_csr(M), b, tol=1e-12)
    assert r.status == orc.OK and r.relres_true <= 1e-12
    kappa = np.linalg.cond(M)
    assert _relerr(r.x, np.linalg.solve(M, b)) <= kappa * 1e-10


def test_bicgstab_breakdown(orc):
    M = np.array([[0.0, 1.0], [-1.0, 0.0]])  # skew-symmetric: r0 . A r0 = 0
    r = orc.bicgstab(I.dense_to_csr(M), np.array([1.0, 2.0]))
    assert r.status == orc.BREAKDOWN


def test_bicgstab_convdiff(orc):
    A = I.convdiff3d(12)
    xs = I.uniform_vector(A.n, 5)
    b = orc.spmv_csr(A, xs)
    r = orc.bicgstab(A, b, tol=1e-10)
    assert r.status == orc.OK and r.relres_true <= 1e-10
    assert orc.true_relres(A, b, r.x) <= 1e-10


# ---------------------------------------------------------------------------
# GMRES(m)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,seed", [(5, 1), (18, 2)])
def test_gmres_full_space_is_exact(orc, n, seed):
    g = I.rng(seed)
    M = g.standard_normal((n, n)) + np.diag(np.full(n, 2.0))
    b = g.standard_normal(n)
    r = orc.gmres(I.dense_to_csr(M), b, m=n, tol=1e-12, hist=True)
    assert r.status == orc.OK and r.iters <= n and r.restarts == 0
    assert _relerr(r.x, np.linalg.solve(M, b)) <= np.linalg.cond(M) * 1e-11
    # the residual estimate |g_{j+1}| never increases within a cycle
    assert (np.diff(r.hist) <= 1e-15 * r.hist[0]).all()


def test_gmres_eigenvector_happy_breakdown(orc):
    A = I.convdiff3d(6)
    N, c = 6, 10.0
    w = 1 + c / (N + 1)
    s = lambda k: np.sin(np.arange(1, N + 1) * k * np.pi / (N + 1)) * w ** (np.arange(1, N + 1) / 2)
    v = np.einsum("z,y,x->zyx", s(2), s(1), s(3)).ravel()
    r = orc.gmres(A, v, m=30, tol=1e-12)
    assert r.status == orc.OK and r.iters == 1


def test_gmres_restarted_convdiff(orc):
    A = I.convdiff3d(14)
    xs = I.uniform_vector(A.n, 6)
    b = orc.spmv_csr(A, xs)
    r = orc.gmres(A, b, m=30, tol=1e-10, hist=True)
    assert r.status == orc.OK and r.relres_true <= 1e-10
    assert r.restarts >= 1  # 2744 unknowns need more than one cycle of 30
    assert orc.true_relres(A, b, r.x) <= 1e-10


def test_gmres_not_converged(orc):
    A = I.convdiff3d(10)
    r = orc.gmres(A, np.ones(A.n), m=5, tol=1e-10, maxit=7)
    assert r.status == orc.NOT_CONVERGED and r.iters == 7


# ---------------------------------------------------------------------------
# iterative refinement
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("low", ["f32", "f16"])
def test_ir_poisson(orc, low):
    A = I.poisson3d(16)
    xs = I.uniform_vector(A.n, 7)
    b = orc.spmv_csr(A, xs)
    r = orc.ir(A, b, low=low, tol=1e-10)
    assert r.status == orc.OK and r.relres_true <= 1e-10
    assert orc.true_relres(A, b, r.x) <= 1e-10
    assert 2 <= r.outer_iters <= 5
    ref = orc.cg(A, b, tol=1e-12)
    assert _relerr(r.x, ref.x) <= 1e-8


def test_ir_f16_storage_exact_for_poisson(orc):
    A = I.poisson3d(8)
    st, h, s = orc.rowscale_f16(A)
    dec = orc.f16_bits_to_f64(h) * np.repeat(s.astype(float), A.row_lengths())
    assert np.array_equal(dec, A.val)


def test_ir_random_spd_small(orc):
    A = I.random_spd(4000, seed=8)
    xs = I.uniform_vector(A.n, 9)
    b = orc.spmv_csr(A, xs)
    for low in ("f32", "f16"):
        r = orc.ir(A, b, low=low, tol=1e-10, last_step_variant=True)
        assert r.status == orc.OK and r.relres_true <= 1e-10


@pytest.mark.parametrize("seed,cond,n", [(3, 30.0, 300), (5, 100.0, 400), (7, 10.0, 200)])
def test_ir_carried_direction_follows_cg(orc, seed, cond, n):
    """With the direction carried, refinement is one CG whose residual is
    replaced by the FP64 one at each step: in exact arithmetic it makes
    the iterates of plain CG.  After two steps x matches FP64 CG run for the
    same total number of iterations to FP32 rounding, while the restarted
    scheme stays about 3e-5 away (a wrong rescaling of the carried direction
    sends it thousands of steps off, or back to the restarted iterates)."""
    A = I.dense_to_csr(I.random_spd_small(n, cond, seed))
    b = I.uniform_vector(n, seed + 1)
    for carry in (False, True):
        r = orc.ir(A, b, tol=1e-14, outer_max=2, inner_tol=1e-2, carry_direction=carry)
        assert r.outer_iters == 2
        ref = orc.cg(A, b, tol=0.0, maxit=r.inner_iters_total)
        d = _relerr(r.x, ref.x)
        if carry:
            assert d <= 2e-6, d
        else:
            assert d >= 1e-5, d


@pytest.mark.parametrize("cap", [5, 10])
def test_ir_carried_direction_capped_inner(orc, cap):
    """Inner solves cut off after `cap` steps: carried, the refinement is CG
    with its residual replaced every `cap` steps and takes CG's own step
    count (98 here); restarted, it is CG restarted every `cap` steps and
    takes 2.4-4 times as many."""
    A = I.poisson3d(24)
    b = orc.spmv_csr(A, I.uniform_vector(A.n, 25))
    cg = orc.cg(A, b, tol=1e-10)
    carry = orc.ir(A, b, tol=1e-10, inner_max=cap, outer_max=200, carry_direction=True)
    restart = orc.ir(A, b, tol=1e-10, inner_max=cap, outer_max=200)
    assert carry.status == restart.status == orc.OK
    assert carry.relres_true <= 1e-10 and restart.relres_true <= 1e-10
    assert carry.inner_iters_total <= 1.05 * cg.iters + 2
    assert restart.inner_iters_total >= 2 * cg.iters


def test_ir_carried_direction_guard(orc):
    """Row-scaled FP16 values of the random SPD matrix are too far from A
    for the inner directions to serve the next step: the FP64 residual
    falls by about three times what the FP16 recurrence claimed, so the
    direction is never carried and the run is the restarted one exactly
    (carried regardless, this system takes 11 times the inner steps)."""
    A = I.random_spd(4000, seed=8)
    b = orc.spmv_csr(A, I.uniform_vector(A.n, 9))
    restart = orc.ir(A, b, low="f16", tol=1e-10)
    carry = orc.ir(A, b, low="f16", tol=1e-10, carry_direction=True)
    assert carry.status == orc.OK and carry.relres_true <= 1e-10
    assert carry.inner_iters_total == restart.inner_iters_total
    assert np.array_equal(carry.x, restart.x)


@pytest.mark.parametrize("low", ["f32", "f16"])
def test_ir_carried_direction_poisson(orc, low):
    A = I.poisson3d(24)
    b = orc.spmv_csr(A, I.uniform_vector(A.n, 7))
    restart = orc.ir(A, b, low=low, tol=1e-10)
    carry = orc.ir(A, b, low=low, tol=1e-10, carry_direction=True)
    assert carry.status == orc.OK and orc.true_relres(A, b, carry.x) <= 1e-10
    assert carry.outer_iters == restart.outer_iters
    # carrying the direction removes most of the restarts' extra steps:
    # within 20% of FP64 CG run to the same final residual (restarted: 139
    # against 118 here, carried 134)
    plain = orc.cg(A, b, tol=carry.relres_true)
    assert carry.inner_iters_total < restart.inner_iters_total
    assert carry.inner_iters_total <= 1.2 * plain.iters
    # with a Jacobi inner solve too
    st, M = orc.jacobi(A)
    pc = orc.ir(A, b, low=low, tol=1e-10, carry_direction=True, precond=M)
    assert pc.status == orc.OK and pc.relres_true <= 1e-10


# ---------------------------------------------------------------------------
# Jacobi / block-Jacobi preconditioned CG (Saad 2003, ch. 9-10)
# ---------------------------------------------------------------------------
def _scaled(A, s):
    return I.CSRMatrix(A.n, A.ncols, A.rowptr, A.col, A.val * s)


def test_pcg_unit_diagonal_is_cg(orc):
    # with a unit diagonal the Jacobi preconditioner is the identity (1/1 = 1
    # exactly), so PCG must reproduce the independently pinned CG bit for bit
    A = _scaled(I.poisson2d(24), 0.25)
    b = I.uniform_vector(A.n, 5)
    st, M = orc.jacobi(A)
    assert st == orc.OK and np.all(M.minv == 1.0)
    p = orc.pcg(A, b, M, tol=1e-10)
    c = orc.cg(A, b, tol=1e-10)
    assert p.status == c.status == orc.OK and p.iters == c.iters
    assert np.array_equal(p.x, c.x)


def test_pcg_exact_preconditioner_one_step(orc):
    # one block covering the matrix: M = A, z = A^{-1} r, one step is exact
    A = I.poisson2d(10)
    b = I.uniform_vector(A.n, 6)
    st, M = orc.block_jacobi(A, A.n)
    assert st == orc.OK
    r = orc.pcg(A, b, M, tol=1e-10)
    assert r.status == orc.OK and r.iters == 1 and r.relres_true <= 1e-12
    # a diagonal matrix with Jacobi: also one step
    D = I.dense_to_csr(np.diag(np.linspace(1.0, 50.0, 40)))
    st, MD = orc.jacobi(D)
    rd = orc.pcg(D, np.ones(40), MD, tol=1e-12)
    assert rd.status == orc.OK and rd.iters == 1


def test_block_jacobi_size_one_is_jacobi(orc):
    A = I.random_spd(2000, seed=7)
    b = I.uniform_vector(A.n, 7)
    s1, J = orc.jacobi(A)
    s2, B1 = orc.block_jacobi(A, 1)
    assert s1 == s2 == orc.OK and np.array_equal(J.minv, B1.minv)
    r = I.uniform_vector(A.n, 8)
    assert np.array_equal(orc.prec_apply(J, r), orc.prec_apply(B1, r))
    pj, pb = orc.pcg(A, b, J), orc.pcg(A, b, B1)
    assert pj.iters == pb.iters and np.array_equal(pj.x, pb.x)


@pytest.mark.parametrize("bs", [3, 8, 32])
def test_block_jacobi_inverse_vs_numpy(orc, bs):
    # every stored block is the inverse numpy computes for A[I, I]; the apply
    # is the block-diagonal product (ragged last block included)
    A = I.random_spd(1000 + bs // 2, seed=9)
    n = A.n
    Dn = np.zeros((n, n))
    for i in range(n):
        Dn[i, A.col[A.rowptr[i]:A.rowptr[i + 1]]] = A.val[A.rowptr[i]:A.rowptr[i + 1]]
    st, M = orc.block_jacobi(A, bs)
    assert st == orc.OK
    r = I.uniform_vector(n, 10)
    z = orc.prec_apply(M, r)
    for k in range(-(-n // bs)):
        r0, m = k * bs, min(bs, n - k * bs)
        inv = np.linalg.inv(Dn[r0:r0 + m, r0:r0 + m])
        slot = M.minv[k * bs * bs:(k + 1) * bs * bs].reshape(bs, bs).T  # column-major
        assert np.allclose(slot[:m, :m], inv, rtol=1e-12, atol=1e-14 * np.abs(inv).max())
        assert not slot[m:, :].any() and not slot[:, m:].any()
        zr = inv @ r[r0:r0 + m]
        assert np.abs(z[r0:r0 + m] - zr).max() <= 1e-12 * (np.abs(inv) @ np.abs(r[r0:r0 + m])).max()


def test_jacobi_pcg_error_bound(orc):
    # d_i = 1.1 sum_j |s_ij| puts spec(D^-1 A) in [1 - 1/1.1, 1 + 1/1.1]
    # (Gershgorin), kappa <= 21; PCG's A-norm error obeys
    # ||e_k||_A <= 2 ((sqrt(k)-1)/(sqrt(k)+1))^k ||e_0||_A at every k
    A = I.random_spd(1500, seed=11)
    n = A.n
    Dn = np.zeros((n, n))
    for i in range(n):
        Dn[i, A.col[A.rowptr[i]:A.rowptr[i + 1]]] = A.val[A.rowptr[i]:A.rowptr[i + 1]]
    b = I.uniform_vector(n, 12)
    xs = np.linalg.solve(Dn, b)
    anorm = lambda e: np.sqrt(e @ Dn @ e)
    st, M = orc.jacobi(A)
    kap = (1 + 1 / 1.1) / (1 - 1 / 1.1)
    rho = (np.sqrt(kap) - 1) / (np.sqrt(kap) + 1)
    e0 = anorm(xs)
    full = orc.pcg(A, b, M, tol=1e-10)
    assert full.status == orc.OK and full.relres_true <= 1e-10
    for k in (1, 3, 8, 15, full.iters):
        r = orc.pcg(A, b, M, tol=0.0, maxit=k)
        assert anorm(r.x - xs) <= 2 * rho ** k * e0 * (1 + 1e-6) + 1e-12 * e0, k
    plain = orc.cg(A, b, tol=1e-10)
    assert full.iters < plain.iters


def test_preconditioner_failures(orc):
    A = I.poisson2d(6)
    bad = I.CSRMatrix(A.n, A.ncols, A.rowptr, A.col, A.val.copy())
    k = [q for q in range(bad.rowptr[7], bad.rowptr[8]) if bad.col[q] == 7][0]
    bad.val[k] = 0.0
    assert orc.jacobi(bad)[0] == orc.BREAKDOWN
    # a singular 2x2 diagonal block [[1, 1], [1, 1]]
    S = I.dense_to_csr(np.array([[1.0, 1.0, 0, 0], [1.0, 1.0, 0, 0], [0, 0, 2.0, 0],
                                 [0, 0, 0, 3.0]]))
    assert orc.block_jacobi(S, 2)[0] == orc.BREAKDOWN
    assert orc.block_jacobi(S, 1)[0] == orc.OK
    # an indefinite preconditioner: (r, M^-1 r) < 0 stops PCG with a breakdown
    neg = I.dense_to_csr(np.diag([1.0, -1.0, 2.0]))
    st, M = orc.jacobi(neg)
    r = orc.pcg(neg, np.array([0.0, 1.0, 0.0]), M)
    assert r.status == orc.BREAKDOWN


def test_ir_with_jacobi_inner(orc):
    A = I.random_spd(3000, seed=13)
    b = I.uniform_vector(A.n, 14)
    st, M = orc.jacobi(A)
    plain = orc.ir(A, b, low="f32", tol=1e-10)
    pre = orc.ir(A, b, low="f32", tol=1e-10, precond=M)
    assert plain.status == pre.status == orc.OK
    assert pre.relres_true <= 1e-10
    assert pre.inner_iters_total * 5 < plain.inner_iters_total
    # block Jacobi on FP16 storage too
    st, MB = orc.block_jacobi(A, 16)
    r16 = orc.ir(A, b, low="f16", tol=1e-10, precond=MB)
    assert r16.status == orc.OK and r16.relres_true <= 1e-10


# ---------------------------------------------------------------------------
# CGS (Sonneveld 1989; Saad 2003, Algorithm 7.6)
# ---------------------------------------------------------------------------
def test_cgs_scaled_identity_one_step(orc):
    A = _scaled(I.dense_to_csr(np.eye(30)), 3.0)
    b = I.uniform_vector(30, 40)
    r = orc.cgs(A, b, tol=1e-14)
    assert r.status == orc.OK and r.iters == 1
    assert np.allclose(r.x, b / 3.0, rtol=0, atol=1e-15)


def test_cgs_is_squared_cg_on_symmetric(orc):
    # with r_hat = r0 on a symmetric matrix BiCG is CG, so the CGS residual
    # after k steps is phi_k(A)^2 r0 where phi_k(A) r0 is CG's residual:
    # in the eigenbasis c = Q^T r0, d = Q^T r_k(CG), CGS gives d^2 / c
    n = 12
    lam = np.linspace(1.0, 6.0, n)
    Q, _ = np.linalg.qr(I.rng(41).standard_normal((n, n)))
    Mx = Q @ np.diag(lam) @ Q.T
    Mx = (Mx + Mx.T) / 2
    A = I.dense_to_csr(Mx)
    b = Q @ (1.0 + I.rng(42).random(n))
    c = Q.T @ b
    for k in (1, 2, 3, 4):
        xcg = orc.cg(A, b, tol=0.0, maxit=k).x
        xcgs = orc.cgs(A, b, tol=0.0, maxit=k).x
        d = Q.T @ (b - Mx @ xcg)
        rcgs = Q.T @ (b - Mx @ xcgs)
        assert np.allclose(rcgs, d * d / c, rtol=1e-7, atol=1e-9 * np.abs(c).max()), k


@pytest.mark.parametrize("n,seed", [(6, 1), (20, 2)])
def test_cgs_nonsymmetric_vs_numpy(orc, n, seed):
    g = I.rng(seed + 60)
    Mx = np.eye(n) * 4 + 0.8 * g.standard_normal((n, n)) / np.sqrt(n)
    A = I.dense_to_csr(Mx)
    b = g.standard_normal(n)
    r = orc.cgs(A, b, tol=1e-12, maxit=200)
    assert r.status == orc.OK and r.relres_true <= 1e-12
    assert _relerr(r.x, np.linalg.solve(Mx, b)) <= 1e-10


def test_cgs_breakdown_and_convdiff(orc):
    # skew-symmetric: (r_hat, A p) = (r0, A r0) = 0 on the first step
    S = np.array([[0.0, 1.0, 0.0], [-1.0, 0.0, 2.0], [0.0, -2.0, 0.0]])
    r = orc.cgs(I.dense_to_csr(S), np.array([1.0, 2.0, 3.0]))
    assert r.status == orc.BREAKDOWN and r.iters == 0
    Cd = I.convdiff3d(12)
    b = orc.spmv_csr(Cd, I.uniform_vector(Cd.n, 43))
    r = orc.cgs(Cd, b, tol=1e-10)
    assert r.status == orc.OK and r.relres_true <= 1e-10
    nm = orc.cgs(Cd, b, tol=1e-10, maxit=3)
    assert nm.status == orc.NOT_CONVERGED and nm.iters == 3


# ---------------------------------------------------------------------------
# pipelined CG (Ghysels & Vanroose 2014)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,seed", [(8, 1), (16, 3)])
def test_pipecg_iterates_are_cg_iterates(orc, n, seed):
    # the same Krylov iterates as CG in exact arithmetic: after k steps the
    # two agree to rounding (CG is pinned independently above)
    Mx = I.random_spd_small(n, 10.0, seed)
    A = I.dense_to_csr(Mx)
    b = I.rng(seed + 70).standard_normal(n)
    for k in range(1, n):
        xc = orc.cg(A, b, tol=0.0, maxit=k).x
        xp = orc.pipecg(A, b, tol=0.0, maxit=k).x
        assert np.linalg.norm(xp - xc) <= 1e-11 * np.linalg.norm(xc), k
    r = orc.pipecg(A, b, tol=1e-12, maxit=n + 2)
    assert r.status == orc.OK and r.iters <= n + 1


def test_pipecg_poisson_and_eigenvector(orc):
    A = I.poisson2d(64)
    b = orc.spmv_csr(A, np.ones(A.n))
    r = orc.pipecg(A, b, tol=1e-10)
    c = orc.cg(A, b, tol=1e-10)
    assert r.status == orc.OK and r.relres_true <= 1e-10
    assert abs(r.iters - c.iters) <= 2
    m = 12
    P = I.poisson2d(m)
    s = lambda kk: np.sin(np.arange(1, m + 1) * kk * np.pi / (m + 1))
    v = np.outer(s(5), s(3)).ravel()
    r1 = orc.pipecg(P, v, tol=1e-12)
    assert r1.status == orc.OK and r1.iters == 1


def test_pipecg_failures(orc):
    # indefinite: (p, A p) <= 0 on the first step
    D = I.dense_to_csr(np.diag([1.0, -2.0, 3.0]))
    r = orc.pipecg(D, np.array([0.0, 1.0, 0.0]))
    assert r.status == orc.BREAKDOWN and r.iters == 0
    A = I.poisson2d(16)
    b = np.ones(A.n)
    r = orc.pipecg(A, b, tol=1e-10, maxit=5)
    assert r.status == orc.NOT_CONVERGED and r.iters == 5
    z = orc.pipecg(A, np.zeros(A.n))
    assert z.status == orc.OK and z.iters == 0 and not z.x.any()
