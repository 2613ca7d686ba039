"""GPU solvers through the C ABI, checked by the CPU oracle: the oracle
recomputes ||b - A x|| / ||b|| from the returned x with accurately summed
rows and it must meet the tolerance up to the residual-evaluation error
(|computed - exact| <= gamma * || |b| + |A||x| ||, gamma = 64 u); solutions
of tiny systems match dense LU; breakdown and failure statuses match the
oracle's."""
import numpy as np
import pytest

from paper_2103_10116_amd import inputs as I

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2103_10116_amd import mxs
    ctx = mxs.Context(0)
    yield mxs, ctx, torch
    ctx.close()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()


def _eval_slack(orc, A, b, x):
    """Residual-evaluation error bound relative to ||b||."""
    s = np.abs(b) + orc.absrow(A, x)
    return 64 * U * np.linalg.norm(s) / np.linalg.norm(b)


def _solve(env, A, b, kind, fmt="csr", tol=1e-10, x0=None, **kw):
    mxs, ctx, torch = env
    M = mxs.Matrix.from_host(ctx, A)
    B = M if fmt == "csr" else M.convert(fmt, "f64")
    x = _dev(torch, np.zeros(A.n) if x0 is None else x0)
    r = mxs.solve(ctx, kind, B, _dev(torch, b), x, tol=tol, raise_on_error=False, **kw)
    return r, x.cpu().numpy()


def _assert_converged(orc, A, b, x, r, tol):
    from paper_2103_10116_amd import mxs
    assert r.status == mxs.OK, r
    rel = orc.true_relres(A, b, x)
    assert rel <= tol + _eval_slack(orc, A, b, x), (rel, r)
    assert abs(rel - r.relres_true) <= 1e-3 * tol + _eval_slack(orc, A, b, x)


# ---------------------------------------------------------------------------
# CG
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("fmt", ["csr", "coo", "ell", "hyb"])
def test_cg_poisson64(env, orc, fmt):
    A = I.poisson2d(64)
    b = orc.spmv_csr(A, np.ones(A.n))
    r, x = _solve(env, A, b, "cg", fmt)
    _assert_converged(orc, A, b, x, r, 1e-10)
    ref = orc.cg(A, b, tol=1e-10)
    assert abs(r.iters - ref.iters) <= 3
    assert np.linalg.norm(x - np.ones(A.n)) / np.sqrt(A.n) <= 1711.7 * 1e-10


@pytest.mark.parametrize("n,seed", [(5, 1), (16, 2)])
def test_cg_tiny_vs_lu(env, orc, n, seed):
    M = I.random_spd_small(n, 10.0, seed)
    A = I.dense_to_csr(M)
    b = I.rng(seed + 9).standard_normal(n)
    r, x = _solve(env, A, b, "cg", tol=1e-12)
    _assert_converged(orc, A, b, x, r, 1e-12)
    assert r.iters <= n + 1
    st, xl = orc.lu_solve(M, b)
    assert np.linalg.norm(x - xl) <= 10 * 1e-10 * np.linalg.norm(xl)


def test_cg_statuses(env, orc):
    from paper_2103_10116_amd import mxs
    A = I.poisson2d(8)
    r, x = _solve(env, A, np.zeros(A.n), "cg")
    assert r.status == mxs.OK and r.iters == 0 and not x.any()
    b = np.ones(A.n)
    b[5] = np.nan
    r, _ = _solve(env, A, b, "cg")
    assert r.status == mxs.NONFINITE
    r, _ = _solve(env, A, np.ones(A.n), "cg", max_iters=3)
    assert r.status == mxs.NOT_CONVERGED and r.iters == 3
    r, _ = _solve(env, I.dense_to_csr(np.diag([1.0, -1.0, 2.0, -3.0])), np.ones(4), "cg")
    assert r.status == mxs.BREAKDOWN
    xs = orc.cg(A, np.ones(A.n), tol=1e-12).x
    r, _ = _solve(env, A, np.ones(A.n), "cg", x0=xs)
    assert r.status == mxs.OK and r.iters == 0


def test_cg_eigenvector_one_step(env, orc):
    m = 12
    A = I.poisson2d(m)
    s = lambda k: np.sin(np.arange(1, m + 1) * k * np.pi / (m + 1))
    v = np.outer(s(5), s(3)).ravel()
    r, x = _solve(env, A, v, "cg", tol=1e-12)
    assert r.iters == 1
    lam = 4 - 2 * np.cos(3 * np.pi / (m + 1)) - 2 * np.cos(5 * np.pi / (m + 1))
    assert np.linalg.norm(x - v / lam) <= 1e-13 * np.linalg.norm(v / lam)


# ---------------------------------------------------------------------------
# BiCGSTAB
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("fmt", ["csr", "coo", "hyb"])
def test_bicgstab_convdiff(env, orc, fmt):
    A = I.convdiff3d(16)
    b = orc.spmv_csr(A, I.uniform_vector(A.n, 21))
    r, x = _solve(env, A, b, "bicgstab", fmt)
    _assert_converged(orc, A, b, x, r, 1e-10)
    ref = orc.bicgstab(A, b)
    assert abs(r.iters - ref.iters) <= max(3, ref.iters // 10)


def test_bicgstab_identity_and_breakdown(env, orc):
    from paper_2103_10116_amd import mxs
    b = I.uniform_vector(20, 22)
    r, x = _solve(env, I.dense_to_csr(3.0 * np.eye(20)), b, "bicgstab", tol=1e-14)
    assert r.status == mxs.OK and r.iters == 1
    assert np.allclose(x, b / 3.0, rtol=1e-15, atol=0)
    r, _ = _solve(env, I.dense_to_csr(np.array([[0.0, 1.0], [-1.0, 0.0]])),
                  np.array([1.0, 2.0]), "bicgstab")
    assert r.status == mxs.BREAKDOWN


def test_bicgstab_nonsymmetric_vs_lu(env, orc):
    g = I.rng(23)
    n = 25
    M = g.standard_normal((n, n)) * 0.3 + np.diag(np.full(n, 3.0))
    b = g.standard_normal(n)
    r, x = _solve(env, I.dense_to_csr(M), b, "bicgstab", tol=1e-12)
    _assert_converged(orc, I.dense_to_csr(M), b, x, r, 1e-12)
    st, xl = orc.lu_solve(M, b)
    assert np.linalg.norm(x - xl) <= np.linalg.cond(M) * 1e-10 * np.linalg.norm(xl)


# ---------------------------------------------------------------------------
# GMRES
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("fmt", ["csr", "ell"])
def test_gmres_convdiff(env, orc, fmt):
    A = I.convdiff3d(16)
    b = orc.spmv_csr(A, I.uniform_vector(A.n, 24))
    r, x = _solve(env, A, b, "gmres", fmt, restart=30)
    _assert_converged(orc, A, b, x, r, 1e-10)
    assert r.restarts >= 1
    ref = orc.gmres(A, b, m=30)
    assert abs(r.iters - ref.iters) <= max(5, ref.iters // 10)


@pytest.mark.parametrize("n,seed", [(5, 1), (18, 2)])
def test_gmres_full_space_exact(env, orc, n, seed):
    g = I.rng(seed)
    M = g.standard_normal((n, n)) + np.diag(np.full(n, 2.0))
    b = g.standard_normal(n)
    r, x = _solve(env, I.dense_to_csr(M), b, "gmres", tol=1e-12, restart=n)
    assert r.iters <= n and r.restarts == 0
    st, xl = orc.lu_solve(M, b)
    assert np.linalg.norm(x - xl) <= np.linalg.cond(M) * 1e-11 * np.linalg.norm(xl)


def test_gmres_happy_breakdown_and_limits(env, orc):
    from paper_2103_10116_amd import mxs
    N, c = 6, 10.0
    A = I.convdiff3d(N)
    w = 1 + c / (N + 1)
    s = lambda k: np.sin(np.arange(1, N + 1) * k * np.pi / (N + 1)) * w ** (np.arange(1, N + 1) / 2)
    v = np.einsum("z,y,x->zyx", s(2), s(1), s(3)).ravel()
    r, x = _solve(env, A, v, "gmres", tol=1e-12)
    assert r.status == mxs.OK and r.iters == 1
    r, _ = _solve(env, I.convdiff3d(10), np.ones(1000), "gmres", tol=1e-10, restart=5,
                  max_iters=7)
    assert r.status == mxs.NOT_CONVERGED and r.iters == 7
    r, _ = _solve(env, A, v, "gmres", restart=40)
    assert r.status == mxs.UNSUPPORTED


# ---------------------------------------------------------------------------
# iterative refinement
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("low", ["f32", "f16"])
@pytest.mark.parametrize("variant", [False, True])
def test_ir_poisson3d(env, orc, low, variant):
    mxs, ctx, torch = env
    A = I.poisson3d(24)
    xs = I.uniform_vector(A.n, 25)
    b = orc.spmv_csr(A, xs)
    M = mxs.Matrix.from_host(ctx, A)
    L = M.convert("csr", low)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    r = mxs.solve_ir(ctx, M, L, _dev(torch, b), x, tol=1e-10, last_step_variant=variant)
    xh = x.cpu().numpy()
    assert r.status == mxs.OK
    rel = orc.true_relres(A, b, xh)
    assert rel <= 1e-10 + _eval_slack(orc, A, b, xh)
    ref = orc.ir(A, b, low=low, tol=1e-10, last_step_variant=variant)
    assert abs(r.outer_iters - ref.outer_iters) <= 1
    cg = orc.cg(A, b, tol=1e-12)
    assert np.linalg.norm(xh - cg.x) <= 1e-8 * np.linalg.norm(cg.x)


def test_ir_random_spd(env, orc):
    mxs, ctx, torch = env
    A = I.random_spd(20000, seed=26)
    b = orc.spmv_csr(A, I.uniform_vector(A.n, 27))
    M = mxs.Matrix.from_host(ctx, A)
    for low in ("f32", "f16"):
        L = M.convert("csr", low)
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        r = mxs.solve_ir(ctx, M, L, _dev(torch, b), x, tol=1e-10, last_step_variant=True)
        xh = x.cpu().numpy()
        assert r.status == mxs.OK
        assert orc.true_relres(A, b, xh) <= 1e-10 + _eval_slack(orc, A, b, xh)


@pytest.mark.slow
def test_full_size_krylov(env, orc):
    """The 128^3 solver workloads: CG on the 7-point Poisson matrix,
    BiCGSTAB and GMRES(30) on the upwind convection-diffusion matrix."""
    P = I.poisson3d(128)
    b = orc.spmv_csr(P, I.uniform_vector(P.n, 28))
    r, x = _solve(env, P, b, "cg")
    _assert_converged(orc, P, b, x, r, 1e-10)
    assert 300 <= r.iters <= 600
    Cd = I.convdiff3d(128)
    b = orc.spmv_csr(Cd, I.uniform_vector(Cd.n, 29))
    r, x = _solve(env, Cd, b, "bicgstab")
    _assert_converged(orc, Cd, b, x, r, 1e-10)
    r, x = _solve(env, Cd, b, "gmres", restart=30)
    _assert_converged(orc, Cd, b, x, r, 1e-10)
