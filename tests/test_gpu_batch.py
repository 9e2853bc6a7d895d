"""Batched form: many volumes of uneven size in one call (one launch per
stage for all of them) must give exactly the outputs of separate plain calls
-- on every repeat, with eager work in between, for every launch parameter
and arena size, under both quantiser flows (the default
one, where volumes of at least 2^22 voxels with rows of a multiple of 4 take
the one-pass 16-bit-proxy flow, and the one-pass flow forced on every float32
volume with an absolute bound), and for the full 64-volume batch workload
(sides 64..512 per axis, eb from {1e-3, 1e-4, 1e-5})."""
import numpy as np
import pytest

import synth
from roixtest import assert_sections_equal, criterion, default_caps, device_sections, log

pytestmark = pytest.mark.gpu


def _outputs_equal(a, b):
    for k in ("rows", "stream", "outliers", "comps"):
        assert a[k].tobytes() == b[k].tobytes(), k
    for k in ("qinfo", "sinfo", "einfo"):
        assert bytes(a[k]) == bytes(b[k]), k


def _volumes():
    vols = [synth.batch_volume(j, side=(24, 96)) for j in range(12)]
    # a uint16 and a cylinder volume make the batch mixed in dtype and criterion
    vols.append(synth.rings2048(nxy=96, nz=9))
    vols.append(synth.cylinder1024(n=80))
    # volumes of at least 2^22 voxels with rows of a multiple of 4: plain
    # calls take the one-pass flow on them by default (16-bit proxy with K <=
    # 2^15, and its 1-byte fallback with K > 2^15), with outliers; the
    # "onepass" batches take it too
    big, _ = synth.ellipsoids(256, 96, 192, 2901, n_ell=5)
    vols.append(synth.Workload("256x96x192 f32 ellipsoids eb 1e-4", big, "abs", 1e-4,
                               synth.Criterion("otsu", 0.0, 6, "min_size", 64), None))
    wide, _ = synth.ellipsoids(192, 160, 144, 2902, n_ell=3)
    vols.append(synth.Workload("192x160x144 f32 ellipsoids eb 1e-5", wide, "abs", 1e-5,
                               synth.Criterion("otsu", 0.0, 26, "largest", 1), None))
    vols.append(synth.cylinder1024(n=176))
    return vols


@pytest.fixture(scope="module", params=["default", "onepass"])
def batch_env(request):
    import torch

    from paper_2602_15917_amd import roix
    vols = _volumes()
    ctx = roix.Context(0, 3 << 30)
    if request.param == "onepass":
        ctx.set_param("fused16_min_voxels", 0)
        ctx.set_param("batch_fused16_min_voxels", 0)
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
    # the batch covers what it is meant to: outliers in one-pass-sized volumes
    big = [i for i, w in enumerate(vols) if w.volume.size >= (1 << 22)]
    assert len(big) == 3 and all(vols[i].volume.shape[2] % 4 == 0 for i in big)
    assert sum(int(plain[i]["einfo"].n_outliers) for i in big) > 0
    yield ctx, roix, torch, items, plain
    ctx.close()


def test_batch_repeats_equal_plain(batch_env):
    ctx, roix, torch, items, plain = batch_env
    for rep in range(4):
        log(f"[case] batch repeat {rep}")
        for it in items:  # clear the outputs so that every repeat must rewrite them
            it[4].stream.zero_()
            it[4].rows.zero_()
        ctx.fused_batch(items)
        torch.cuda.synchronize()
        for i, it in enumerate(items):
            _outputs_equal(it[4].collect(), plain[i])
        # eager work between repeats
        t = items[0][0]
        ctx.fused(t, items[0][1], items[0][2], items[0][3], roix.Outputs("cuda:0", *default_caps(
            roix, t.cpu().numpy(), items[0][3])))
        torch.cuda.synchronize()


def test_batch_subsets_and_order(batch_env):
    # a batch of other volumes, in another order, then the first again
    ctx, roix, torch, items, plain = batch_env
    order = [len(items) - 1, 3, 0, len(items) - 3, 7]
    for sel in (order, list(range(len(items)))):
        log(f"[case] batch subset {sel}")
        for i in sel:
            items[i][4].stream.zero_()
        ctx.fused_batch([items[i] for i in sel])
        torch.cuda.synchronize()
        for i in sel:
            _outputs_equal(items[i][4].collect(), plain[i])


@pytest.mark.parametrize("group,graph,lanes", [(1, 1, 2), (2, 0, 1), (3, 1, 2), (5, 1, 2), (0, 0, 1), (0, 0, 2),
                                               (0, 0, 3), (2, 0, 4), (1, 0, 2)])
def test_batch_parameters_do_not_change_outputs(batch_env, group, graph, lanes):
    # volumes per launch group (1: every volume alone), graph capture or not,
    # concurrent lanes (each on its own stream and part of the arena)
    ctx, roix, torch, items, plain = batch_env
    ctx.set_param("batch_group", group)
    ctx.set_param("batch_graph", graph)
    ctx.set_param("batch_lanes", lanes)
    log(f"[case] batch group={group} graph={graph} lanes={lanes}")
    for it in items:
        it[4].stream.zero_()
    ctx.fused_batch(items)
    torch.cuda.synchronize()
    for i, it in enumerate(items):
        _outputs_equal(it[4].collect(), plain[i])
    ctx.set_param("batch_group", 0)
    ctx.set_param("batch_graph", 1)
    ctx.set_param("batch_lanes", 2)


def test_batch_small_arena_splits_into_groups(batch_env):
    # an arena that holds only a few volumes at a time: the batch runs in
    # groups, one after another, with the same outputs
    ctx, roix, torch, items, plain = batch_env
    need = max(roix.scratch_bytes(roix.dims_of(it[0]), roix.dtype_of(it[0]), it[3]) for it in items)
    small = roix.Context(0, int(need * 2.5))
    log("[case] batch in a small arena")
    for it in items:
        it[4].stream.zero_()
    small.fused_batch(items)
    torch.cuda.synchronize()
    for i, it in enumerate(items):
        _outputs_equal(it[4].collect(), plain[i])
    small.close()


def test_batch_rejects_bad_descriptor(batch_env):
    ctx, roix, torch, items, plain = batch_env
    bad = list(items[:2]) + [(items[2][0], "abs", -1.0, items[2][3], items[2][4])]
    with pytest.raises(roix.RoixError) as ei:
        ctx.fused_batch(bad)
    assert ei.value.status == roix.EINVAL


def test_full_batch_workload_equals_plain():
    """The 64-volume batch workload (5.7 GB of float32 volumes) against 64
    plain calls, every output section compared on the device."""
    import torch

    from paper_2602_15917_amd import roix
    items, need = [], 0
    for j in range(64):
        w = synth.batch_volume(j)
        crit = criterion(roix, w.criterion)
        t = torch.from_numpy(w.volume).to("cuda:0")
        dims = roix.dims_of(t)
        b = roix.bounds(dims, roix.F32, crit)
        caps = (b["rows"], b["stream_bytes"], min(b["outliers"], 1 << 24), min(b["components"], 1 << 20))
        items.append((t, w.eb_mode, w.eb_value, crit, roix.Outputs("cuda:0", *caps), roix.Outputs("cuda:0", *caps)))
        need += roix.scratch_bytes(dims, roix.F32, crit)
    ctx = roix.Context(0, need + (64 << 20))  # every volume's layout at once: one launch group
    log(f"[case] 64-volume batch, {sum(it[0].numel() for it in items) * 4 / 1e9:.2f} GB")
    for (t, ebm, ebv, crit, _, ref) in items:
        ctx.fused(t, ebm, ebv, crit, ref)
    ctx.fused_batch([it[:5] for it in items])
    torch.cuda.synchronize()
    n_out = 0
    for j, it in enumerate(items):
        a, b = device_sections(it[4]), device_sections(it[5])
        assert a["status"] == (0, 0), (j, a["status"])
        assert_sections_equal(a, b, f"volume {j}")
        n_out += int(roix.ExtractInfo.from_buffer_copy(b["einfo"]).n_outliers)
    assert n_out > 0
    ctx.close()
