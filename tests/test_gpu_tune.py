"""The autotuner through the C ABI: it times the fused path on the caller's
volume, keeps the fastest launch parameters, checks that no candidate
changes an output, and caches its choice; the tuned context still gives
the oracle's outputs bit for bit."""
import numpy as np
import pytest

import synth
from roixtest import compare_fused, criterion, default_caps, gpu_fused, log, oracle_fused

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2602_15917_amd import roix
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    roix.load()
    yield roix, torch


def candidates(roix, cus):
    mult = {"grid_stream": (4, 8, 16), "grid_read": (1, 2, 4), "grid_mask": (16, 32, 64), "grid_emit": (2, 4, 8),
            "seg_grid": (1, 2, 4), "stats_grid": (1, 2, 4)}
    c = {k: {m * cus for m in v} for k, v in mult.items()}
    c["seg_runs"] = {0, 1024, 2048, 4096}
    return c


def test_autotune_picks_and_caches(env, tmp_path):
    roix, torch = env
    w = synth.cylinder1024(n=256)
    crit = criterion(roix, w.criterion)
    ctx = roix.Context(0, 1 << 30)
    cus = ctx.get_param("compute_units")
    defaults = {k: ctx.get_param(k) for k in roix.TUNE_PARAMS}
    t = torch.from_numpy(w.volume).to("cuda:0")
    out = roix.Outputs("cuda:0", *default_caps(roix, w.volume, crit))
    cache = str(tmp_path / "tune.txt")
    log("[case] autotune 256^3 cylinder")
    res = ctx.autotune(t, w.eb_mode, w.eb_value, crit, out, reps=1, cache=cache)
    assert res.status == 0 and res.from_cache == 0 and res.n_timed > 7
    assert 0 < res.best_ms <= res.default_ms
    cand = candidates(roix, cus)
    for i, k in enumerate(roix.TUNE_PARAMS):
        v = res.params[i]
        assert v in cand[k] or v == defaults[k], (k, v)
        assert ctx.get_param(k) == v
    # the tuned context still gives the oracle's outputs
    g = gpu_fused(ctx, roix, torch, w.volume, w.eb_mode, w.eb_value, crit)
    compare_fused(g, oracle_fused(w.volume, w.eb_mode, w.eb_value, w.criterion))
    ctx.close()
    # a new context takes the cached values without timing
    ctx2 = roix.Context(0, 1 << 30)
    log("[case] autotune from the cache")
    res2 = ctx2.autotune(t, w.eb_mode, w.eb_value, crit, out, reps=1, cache=cache)
    assert res2.from_cache == 1 and res2.n_timed == 0
    assert list(res2.params) == list(res.params)
    assert [ctx2.get_param(k) for k in roix.TUNE_PARAMS] == list(res.params)
    ctx2.close()


def test_autotune_argument_errors(env):
    roix, torch = env
    ctx = roix.Context(0, 1 << 26)
    v = synth.ellipsoids128().volume
    crit = roix.Criterion("otsu", 0.0, 6, "min_size", 64)
    t = torch.from_numpy(v).to("cuda:0")
    out = roix.Outputs("cuda:0", *default_caps(roix, v, crit))
    for reps in (0, 101):
        with pytest.raises(roix.RoixError) as ei:
            ctx.autotune(t, "abs", 1e-3, crit, out, reps=reps)
        assert ei.value.status == roix.EINVAL
    # an output buffer too small: the extraction status comes back, nothing is tuned
    small = roix.Outputs("cuda:0", 16, 64, 16, 16)
    res = ctx.autotune(t, "abs", 1e-3, crit, small, reps=1)
    assert res.status == roix.ETRUNC and res.best_ms == 0.0
    ctx.close()
