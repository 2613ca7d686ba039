"""Measurement entry points: attainable HBM bandwidth and random-gather rate."""
import math

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    from paper_2103_10116_amd import mxs
    ctx = mxs.Context(0)
    yield mxs, ctx
    ctx.close()


def test_hbm_probe(env):
    """4 GiB arrays, 16 times the 256 MB Infinity Cache: every figure is an
    HBM rate, so none can pass the 8 TB/s peak, and a working probe reaches
    at least a third of it."""
    mxs, ctx = env
    r = mxs.hbm_probe(ctx, 4 << 30, 2)
    for k in ("read_gbs", "copy_gbs", "triad_gbs"):
        assert math.isfinite(r[k]) and 8000.0 / 3 < r[k] <= 8000.0, r
    assert r["best_gbs"] == max(r["read_gbs"], r["copy_gbs"], r["triad_gbs"])


@pytest.mark.parametrize("vb", [4, 8])
def test_gather_probe(env, vb):
    mxs, ctx = env
    small = mxs.gather_probe(ctx, 1 << 12, 1 << 22, vb, 2)   # x held in L2
    large = mxs.gather_probe(ctx, 1 << 24, 1 << 22, vb, 2)   # x spread past L2
    assert math.isfinite(small) and math.isfinite(large) and small > 0 and large > 0
    # a 16 KiB x cannot be slower to gather from than a 64-128 MiB one
    assert small > 0.8 * large
    # one gather per index: far below a load per clock per lane of 256 CUs
    assert large < 256 * 64 * 2.5e9


def test_probe_arguments(env):
    mxs, ctx = env
    with pytest.raises(mxs.MxsError):
        mxs.gather_probe(ctx, 1 << 10, 1 << 10, 2, 1)
    with pytest.raises(mxs.MxsError):
        mxs.gather_probe(ctx, 0, 1 << 10, 8, 1)
    with pytest.raises(mxs.MxsError):
        mxs.hbm_probe(ctx, 1 << 10, 1)
