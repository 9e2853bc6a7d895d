"""Batched form: many volumes of uneven size in one graph launch must give
exactly the outputs of separate plain calls -- on every replay of the
captured graph, with eager work in between, for every launch parameter."""
import numpy as np
import pytest

import synth
from roixtest import criterion, default_caps, log

pytestmark = pytest.mark.gpu


def _outputs_equal(a, b):
    for k in ("rows", "stream", "outliers", "comps"):
        assert a[k].tobytes() == b[k].tobytes(), k
    for k in ("qinfo", "sinfo", "einfo"):
        assert bytes(a[k]) == bytes(b[k]), k


@pytest.fixture(scope="module")
def batch_env():
    import torch

    from paper_2602_15917_amd import roix
    vols = [synth.batch_volume(j, side=(24, 96)) for j in range(12)]
    # a uint16 and a cylinder volume make the batch mixed in dtype and criterion
    vols.append(synth.rings2048(nxy=96, nz=9))
    vols.append(synth.cylinder1024(n=80))
    ctx = roix.Context(0, 1 << 30)
    items, plain = [], []
    for w in vols:
        crit = criterion(roix, w.criterion)
        t = torch.from_numpy(w.volume).to("cuda:0")
        caps = default_caps(roix, w.volume, crit)
        out = roix.Outputs("cuda:0", *caps)
        ref = roix.Outputs("cuda:0", *caps)
        ctx.fused(t, w.eb_mode, w.eb_value, crit, ref)
        items.append((t, w.eb_mode, w.eb_value, crit, out))
        plain.append(ref)
    torch.cuda.synchronize()
    plain = [r.collect() for r in plain]
    yield ctx, roix, torch, items, plain
    ctx.close()


def test_batch_graph_replays_equal_plain(batch_env):
    ctx, roix, torch, items, plain = batch_env
    for rep in range(4):
        log(f"[case] batch graph replay {rep}")
        for it in items:  # clear the outputs so that every replay must rewrite them
            it[4].stream.zero_()
            it[4].rows.zero_()
        ctx.fused_batch(items)
        torch.cuda.synchronize()
        for i, it in enumerate(items):
            _outputs_equal(it[4].collect(), plain[i])
        # eager work between replays
        t = items[0][0]
        ctx.fused(t, items[0][1], items[0][2], items[0][3], roix.Outputs("cuda:0", *default_caps(
            roix, t.cpu().numpy(), items[0][3])))
        torch.cuda.synchronize()


@pytest.mark.parametrize("streams,graph", [(1, 1), (2, 0), (3, 1), (8, 1), (8, 0)])
def test_batch_parameters_do_not_change_outputs(batch_env, streams, graph):
    ctx, roix, torch, items, plain = batch_env
    ctx.set_param("batch_streams", streams)
    ctx.set_param("batch_graph", graph)
    log(f"[case] batch streams={streams} graph={graph}")
    for it in items:
        it[4].stream.zero_()
    ctx.fused_batch(items)
    torch.cuda.synchronize()
    for i, it in enumerate(items):
        _outputs_equal(it[4].collect(), plain[i])
    ctx.set_param("batch_streams", 4)
    ctx.set_param("batch_graph", 1)


def test_batch_rejects_bad_descriptor(batch_env):
    ctx, roix, torch, items, plain = batch_env
    bad = list(items[:2]) + [(items[2][0], "abs", -1.0, items[2][3], items[2][4])]
    with pytest.raises(roix.RoixError) as ei:
        ctx.fused_batch(bad)
    assert ei.value.status == roix.EINVAL
