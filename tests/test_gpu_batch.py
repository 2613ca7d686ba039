"""Batched persistent CG and the continuous-batching engine, through the C
ABI: every result meets the tolerance by the oracle's residual, each system's
result is bitwise the same alone and in a mix, admission respects the HBM
budget, and the serving loop completes every request."""
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


def _systems(ms, seed0=0):
    out = []
    for i, m in enumerate(ms):
        A = I.serving_system(int(m), seed0 + i)
        out.append((A, I.serving_rhs(A.n, seed0 + i)))
    return out


def _drain(B, limit=100000):
    for _ in range(limit):
        st = B.step()
        assert st["arena_used"] <= st["arena_size"]
        if st["active"] == 0 and st["pending"] == 0:
            return
    raise AssertionError("batch did not drain")


def _slack(orc, A, b, x):
    return 64 * U * np.linalg.norm(np.abs(b) + orc.absrow(A, x)) / np.linalg.norm(b)


def test_default_classes(env):
    mxs, ctx, torch = env
    B = mxs.Batch(ctx, 64 << 20, 64)
    cfg = [B.config(c) for c in range(5)]
    assert [c["max_n"] for c in cfg] == [1024, 2304, 4096, 8192, 10240]
    assert sum(c["slots"] for c in cfg) == 64
    assert all(c["block"] * c["rows_per_thread"] >= c["max_n"] for c in cfg)
    B.close()
    with pytest.raises(mxs.MxsError):
        mxs.Batch(ctx, 64 << 20, 8, classes=[(100, 256, 0), (50, 256, 0)])
    with pytest.raises(mxs.MxsError):
        mxs.Batch(ctx, 64 << 20, 8, classes=[(100, 300, 0)])
    with pytest.raises(mxs.MxsError) as e:  # 10240 / 512 = 20 rows per thread > 16
        mxs.Batch(ctx, 64 << 20, 8, classes=[(2304, 512, 0), (10240, 512, 0)])
    assert e.value.status == mxs.UNSUPPORTED


@pytest.mark.parametrize("classes", [None, [(1024, 128, 0), (4096, 256, 0), (10240, 1024, 0)],
                                     [(2304, 512, 0), (10240, 1024, 0)]])
def test_batch_matches_oracle(env, orc, classes):
    mxs, ctx, torch = env
    g = I.rng(41)
    ms = np.concatenate([[8, 9, 31, 32, 33, 48, 64, 95, 96], g.integers(8, 97, 23)])
    sys_ = _systems(ms, 100)
    B = mxs.Batch(ctx, 256 << 20, 16, iters_per_step=8, classes=classes)
    tickets = [B.submit(A, b, 1e-10) for A, b in sys_]
    _drain(B)
    done = set(B.completed())
    assert done == set(tickets)
    for (A, b), t in zip(sys_, tickets):
        s, x, res = B.poll(t, A.n)
        assert s == mxs.OK, res
        rel = orc.true_relres(A, b, x)
        assert rel <= 1e-10 + _slack(orc, A, b, x), (A.n, rel, res)
        ref = orc.cg(A, b, tol=1e-10)
        assert abs(res.iters - ref.iters) <= 2 + ref.iters // 20, (res.iters, ref.iters)
    B.close()


def test_alone_equals_mix_bitwise(env):
    mxs, ctx, torch = env
    probe = _systems([17, 64, 96], 200)
    others = _systems(I.rng(43).integers(8, 97, 40), 300)
    alone = []
    for A, b in probe:
        B = mxs.Batch(ctx, 64 << 20, 4, iters_per_step=5)
        t = B.submit(A, b, 1e-10)
        _drain(B)
        s, x, _ = B.poll(t, A.n)
        assert s == mxs.OK
        alone.append(x)
        B.close()
    # mixed: probes submitted among other systems, different slots and steps
    B = mxs.Batch(ctx, 512 << 20, 24, iters_per_step=7)
    order = others[:13] + [probe[0]] + others[13:30] + [probe[1]] + others[30:] + [probe[2]]
    tickets = [B.submit(A, b, 1e-10) for A, b in order]
    _drain(B)
    pos = [13, 31, len(order) - 1]
    for k, i in enumerate(pos):
        s, x, _ = B.poll(tickets[i], order[i][0].n)
        assert s == mxs.OK
        assert np.array_equal(x.view(np.uint64), alone[k].view(np.uint64)), k
    B.close()


def test_budget_and_queueing(env, orc):
    mxs, ctx, torch = env
    big = _systems([96], 400)[0]  # footprint about 0.88 MB
    B = mxs.Batch(ctx, 512 << 10, 8)
    with pytest.raises(mxs.MxsError) as e:
        B.submit(*big, 1e-10)
    assert e.value.status == mxs.BUDGET
    B.close()
    # 4 MiB budget, 30 systems of ~0.2-1 MB: most wait for space
    sys_ = _systems(I.rng(44).integers(40, 97, 30), 500)
    B = mxs.Batch(ctx, 4 << 20, 32, iters_per_step=8)
    tickets = [B.submit(A, b, 1e-10) for A, b in sys_]
    max_active = 0
    for _ in range(100000):
        st = B.step()
        assert st["arena_used"] <= st["arena_size"] == 4 << 20
        max_active = max(max_active, st["active"])
        if st["active"] == 0 and st["pending"] == 0:
            break
    assert max_active < len(sys_)
    for (A, b), t in zip(sys_, tickets):
        s, x, _ = B.poll(t, A.n)
        assert s == mxs.OK
        assert orc.true_relres(A, b, x) <= 1e-10 + _slack(orc, A, b, x)
    B.close()


def test_special_requests(env):
    mxs, ctx, torch = env
    A, b = _systems([12], 600)[0]
    B = mxs.Batch(ctx, 64 << 20, 8)
    t0 = B.submit(A, np.zeros(A.n), 1e-10)
    t1 = B.submit(A, b, 1e-10, max_iters=3)
    bad = I.CSRMatrix(A.n, A.n, A.rowptr, A.col.copy(), A.val)
    bad.col[1] = bad.col[0]
    with pytest.raises(mxs.MxsError) as e:
        B.submit(bad, b, 1e-10)
    assert e.value.status == mxs.INVALID_MATRIX
    with pytest.raises(mxs.MxsError) as e:
        B.submit(I.serving_system(110, 1), np.ones(110 * 110), 1e-10)
    assert e.value.status == mxs.UNSUPPORTED
    assert B.poll(t0, A.n)[0] == mxs.PENDING
    _drain(B)
    s, x, res = B.poll(t0, A.n)
    assert s == mxs.OK and not x.any() and res.iters == 0
    s, x, res = B.poll(t1, A.n)
    assert s == mxs.NOT_CONVERGED and res.iters == 3
    B.close()


def test_serving_loop(env, orc):
    mxs, ctx, torch = env
    from paper_2103_10116_amd import serve
    reqs = I.serving_stream(40, rate=2000.0, seed=7)
    systems = serve.build_systems(reqs)
    rb = serve.run_batched(ctx, reqs, systems, budget_bytes=64 << 20, max_slots=32,
                           keep_x=True)
    rp = serve.run_plain(ctx, reqs, systems, keep_x=True)
    assert rb.statuses == {mxs.OK: 40} and rp.statuses == {mxs.OK: 40}
    assert rb.max_active > 1  # requests overlapped on the device
    for r in reqs:
        A, b = systems[r.rid]
        for xs in (rb.x, rp.x):
            assert orc.true_relres(A, b, xs[r.rid]) <= 1e-10 + _slack(orc, A, b, xs[r.rid])
    assert rb.p99_ms > 0 and rp.p99_ms > 0


def test_submit_many(env):
    """Requests queued in one call (validated and packed on host threads)
    give the same tickets order and bitwise the same results as one at a
    time; malformed ones are rejected individually."""
    mxs, ctx, torch = env
    sys_ = _systems(I.rng(45).integers(8, 97, 60), 700)
    A0, b0 = sys_[5]
    bad = I.CSRMatrix(A0.n, A0.n, A0.rowptr, A0.col.copy(), A0.val)
    bad.col[2] = bad.col[1]  # duplicate column
    big = I.serving_system(110, 1)
    reqs = sys_[:20] + [(bad, b0)] + sys_[20:40] + [(big, np.ones(big.n))] + sys_[40:]
    B = mxs.Batch(ctx, 256 << 20, 32, iters_per_step=8)
    tickets, sts = B.submit_many(reqs, 1e-10)
    assert sts[20] == mxs.INVALID_MATRIX and tickets[20] == 0
    assert sts[41] == mxs.UNSUPPORTED and tickets[41] == 0
    ok = [i for i in range(len(reqs)) if i not in (20, 41)]
    assert (sts[ok] == mxs.OK).all()
    assert np.all(np.diff(tickets[ok].astype(np.int64)) > 0)
    _drain(B)
    many = {i: B.poll(int(tickets[i]), reqs[i][0].n) for i in ok}
    B.close()
    B = mxs.Batch(ctx, 256 << 20, 32, iters_per_step=8)
    one = {i: B.submit(*reqs[i], 1e-10) for i in ok}
    _drain(B)
    for i in ok:
        s1, x1, r1 = B.poll(one[i], reqs[i][0].n)
        sm, xm, rm = many[i]
        assert s1 == sm == mxs.OK and r1.iters == rm.iters
        assert np.array_equal(x1.view(np.uint64), xm.view(np.uint64)), i
    B.close()


def test_ir32_matches_oracle(env, orc):
    """Refinement mode (FP32 storage, FP64 residual and update): every
    result meets 1e-10 by the oracle's FP64 residual, with the oracle's
    refinement taking the same number of outer steps and about the same
    inner iterations."""
    mxs, ctx, torch = env
    ms = np.concatenate([[8, 9, 33, 64, 96], I.rng(46).integers(8, 97, 19)])
    sys_ = _systems(ms, 800)
    B = mxs.Batch(ctx, 256 << 20, 16, iters_per_step=8)
    tickets, sts = B.submit_many(sys_, 1e-10, mode="ir32")
    assert (sts == mxs.OK).all()
    _drain(B)
    for (A, b), t in zip(sys_, tickets.tolist()):
        s, x, res = B.poll(t, A.n)
        assert s == mxs.OK, (A.n, res)
        rel = orc.true_relres(A, b, x)
        assert rel <= 1e-10 + _slack(orc, A, b, x), (A.n, rel)
        ref = orc.ir(A, b, low="f32", tol=1e-10, outer_max=50, inner_tol=1e-4)
        assert ref.status == 0
        assert abs(res.restarts - ref.outer_iters) <= 1, (A.n, res.restarts, ref.outer_iters)
        assert abs(res.iters - ref.inner_iters_total) <= 3 + ref.inner_iters_total // 10, \
            (A.n, res.iters, ref.inner_iters_total)
    B.close()


def test_modes_mixed_and_alone_bitwise(env):
    """FP64 and refinement requests share one batch; each result is
    bitwise the one it gives alone."""
    mxs, ctx, torch = env
    sys_ = _systems(I.rng(47).integers(8, 97, 30), 900)
    modes = ["f64" if i % 3 else "ir32" for i in range(len(sys_))]
    B = mxs.Batch(ctx, 256 << 20, 24, iters_per_step=6)
    tk = []
    for (A, b), md in zip(sys_, modes):
        t, s = B.submit_many([(A, b)], 1e-10, mode=md)
        assert s[0] == mxs.OK
        tk.append(int(t[0]))
    _drain(B)
    mixed = [B.poll(t, A.n) for t, (A, b) in zip(tk, sys_)]
    B.close()
    for k in (0, 3, 4, 29):
        A, b = sys_[k]
        B = mxs.Batch(ctx, 64 << 20, 4, iters_per_step=6)
        t, _ = B.submit_many([(A, b)], 1e-10, mode=modes[k])
        _drain(B)
        s, x, res = B.poll(int(t[0]), A.n)
        B.close()
        assert s == mixed[k][0] == mxs.OK
        assert np.array_equal(x.view(np.uint64), mixed[k][1].view(np.uint64)), (k, modes[k])
        assert res.iters == mixed[k][2].iters and res.restarts == mixed[k][2].restarts


def test_ir32_limits(env):
    mxs, ctx, torch = env
    A, b = _systems([40], 950)[0]
    B = mxs.Batch(ctx, 64 << 20, 4)
    t, s = B.submit_many([(A, b), (A, np.zeros(A.n)), (A, b)], 1e-10, max_iters=5,
                         mode="ir32")
    t2, s2 = B.submit_many([(A, b)], 1e-10, mode="ir32", inner_tol=1.5)
    assert s2[0] == mxs.INVALID_ARG and t2[0] == 0
    _drain(B)
    s0, x0, r0 = B.poll(int(t[0]), A.n)
    assert s0 == mxs.NOT_CONVERGED and r0.iters <= 5
    s1, x1, r1 = B.poll(int(t[1]), A.n)
    assert s1 == mxs.OK and not x1.any() and r1.iters == 0
    B.close()


def test_step_halves_and_submit_in_flight(env, orc):
    """step_launch / step_finish: misuse is refused, and requests submitted
    while a step runs are solved bitwise as when submitted before it."""
    mxs, ctx, torch = env
    B = mxs.Batch(ctx, 256 << 20, 16, iters_per_step=6)
    with pytest.raises(mxs.MxsError):
        B.step_finish()
    B.step_launch()
    with pytest.raises(mxs.MxsError):
        B.step_launch()
    B.step_finish()
    first = _systems([12, 40, 90, 23], 500)
    later = _systems([64, 8, 77, 31, 50], 600)
    t1 = [B.submit(A, b, 1e-10) for A, b in first]
    B.step_launch()
    t2, sts = B.submit_many(later, 1e-10)           # packed while the step runs
    assert all(s == mxs.OK for s in sts.tolist())
    B.step_finish()
    for _ in range(10000):
        B.step_launch()
        st = B.step_finish()
        if st["active"] == 0 and st["pending"] == 0:
            break
    got = {}
    for t, (A, b) in zip(t1 + t2.tolist(), first + later):
        s, x, res = B.poll(t, A.n)
        assert s == mxs.OK
        r = b - orc.spmv_csr(A, x)
        assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10 + _slack(orc, A, b, x)
        got[id(A)] = x
    B.close()
    # the same systems through the synchronous step, all submitted first
    B = mxs.Batch(ctx, 256 << 20, 16, iters_per_step=6)
    tk = [B.submit(A, b, 1e-10) for A, b in first + later]
    _drain(B)
    for t, (A, b) in zip(tk, first + later):
        s, x, _ = B.poll(t, A.n)
        assert s == mxs.OK
        assert np.array_equal(x.view(np.uint64), got[id(A)].view(np.uint64))
    B.close()


def test_serving_concurrent_submission_bitwise(env):
    """The serving loop's submitter thread queues small chunks while the main
    thread steps; every result is bitwise the one of a plain submit-then-drain
    run of the same engine."""
    mxs, ctx, torch = env
    from paper_2103_10116_amd import serve
    reqs = I.serving_stream(60, rate=0.0, seed=11)
    systems = serve.build_systems(reqs)
    rb = serve.run_batched(ctx, reqs, systems, budget_bytes=128 << 20, max_slots=24,
                           iters_per_step=5, keep_x=True, chunk=5)
    assert rb.statuses == {mxs.OK: 60}
    B = mxs.Batch(ctx, 128 << 20, 24, iters_per_step=5)
    tk = {r.rid: B.submit(*systems[r.rid], 1e-10) for r in reqs}
    _drain(B)
    for r in reqs:
        s, x, _ = B.poll(tk[r.rid], systems[r.rid][0].n)
        assert s == mxs.OK
        assert np.array_equal(x.view(np.uint64), rb.x[r.rid].view(np.uint64)), r.rid
    B.close()


def test_starvation_guard(env, orc):
    """A request too large to fit beside the residents is passed over by the
    small ones behind it, but once it has been the oldest waiting request
    for 64 steps nothing behind it is admitted: the residents drain, it is
    admitted and finishes, although small requests keep arriving."""
    mxs, ctx, torch = env
    big = _systems([96], 700)[0]
    smalls = _systems([30] * 400, 800)
    # the footprints as the engine counts them
    B0 = mxs.Batch(ctx, 64 << 20, 8, iters_per_step=1)
    B0.submit(*big, 1e-10)
    fp_big = B0.step()["arena_used"]
    B0.close()
    B0 = mxs.Batch(ctx, 64 << 20, 8, iters_per_step=1)
    B0.submit(*smalls[0], 1e-10)
    fp_small = B0.step()["arena_used"]
    B0.close()
    assert fp_big > 8 * fp_small
    # room for the big one alone, or for several small ones, never for both
    B = mxs.Batch(ctx, fp_big + fp_small // 2, 32, iters_per_step=8)
    it = iter(smalls)
    tickets = [B.submit(*next(it), 1e-10) for _ in range(4)]
    B.step()
    tb = B.submit(*big, 1e-10)
    done_at = None
    for step in range(300):
        for _ in range(2):      # two new small requests every step
            nxt = next(it, None)
            if nxt is not None:
                tickets.append(B.submit(*nxt, 1e-10))
        B.step()
        s, x, _ = B.poll(tb, big[0].n)
        if s != mxs.PENDING:
            done_at = step
            break
    assert done_at is not None and done_at >= 64, done_at
    assert s == mxs.OK
    assert orc.true_relres(big[0], big[1], x) <= 1e-10 + _slack(orc, big[0], big[1], x)
    _drain(B)
    for t, (A, b) in zip(tickets, smalls):
        s, x, _ = B.poll(t, A.n)
        assert s == mxs.OK
    B.close()


def test_poll_many_equals_poll(env):
    """mxs_batch_poll_many hands back what mxs_batch_poll would, bit for bit,
    for several finished requests in one call; a request still waiting is
    reported PENDING and kept; an unknown ticket is refused."""
    mxs, ctx, torch = env
    sys_ = _systems([9, 40, 17, 64, 25, 33], 900)
    runs = []
    for use_many in (False, True):
        B = mxs.Batch(ctx, 64 << 20, 16, iters_per_step=8)
        tickets = [B.submit(A, b, 1e-10) for A, b in sys_]
        _drain(B)
        late = B.submit(*_systems([90], 901)[0], 1e-10)   # queued, not stepped
        if use_many:
            ns = [A.n for A, _ in sys_] + [8100]
            sts, x, off, info = B.poll_many(tickets + [late], ns)
            assert sts[-1] == mxs.PENDING
            s, _, _ = B.poll(late, 8100)
            assert s == mxs.PENDING   # still known: poll_many kept it
            out = [(int(sts[i]), x[off[i]:off[i] + ns[i]].copy(),
                    (int(info["iters"][i]), float(info["relres_true"][i]),
                     int(info["status"][i])))
                   for i in range(len(sys_))]
            with pytest.raises(mxs.MxsError):
                B.poll_many([10 ** 9], [1])   # never issued
        else:
            out = []
            for t, (A, _) in zip(tickets, sys_):
                s, xv, r = B.poll(t, A.n)
                out.append((s, xv, (r.iters, r.relres_true, s)))
        runs.append(out)
        B.close()
    for (s1, x1, r1), (s2, x2, r2) in zip(*runs):
        assert s1 == s2 == mxs.OK
        assert np.array_equal(x1.view(np.uint64), x2.view(np.uint64))
        assert r1 == r2
