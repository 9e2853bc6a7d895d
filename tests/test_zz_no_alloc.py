"""roix_fused_noalloc (the fused path on the library's fixed scratch array,
for callers that cannot allocate) gives exactly roix_fused's outputs: two
calls in a row, the second on a smaller volume, each compared byte for byte
with a context's roix_fused on the same input; a volume whose worst-case
scratch exceeds the array is refused before anything is enqueued."""
import numpy as np
import pytest

import synth
from roixtest import criterion, default_caps, log

pytestmark = pytest.mark.gpu


def _equal(a, b):
    for k in ("rows", "stream", "outliers", "comps"):
        assert a[k].tobytes() == b[k].tobytes(), k
    for k in ("qinfo", "sinfo", "einfo"):
        assert bytes(a[k]) == bytes(b[k]), k


def _run_both(roix, torch, ctx, w):
    crit = criterion(roix, w.criterion)
    t = torch.from_numpy(np.ascontiguousarray(w.volume)).to("cuda:0")
    caps = default_caps(roix, w.volume, crit)
    ref = roix.Outputs("cuda:0", *caps)
    got = roix.Outputs("cuda:0", *caps)
    ctx.fused(t, w.eb_mode, w.eb_value, crit, ref)
    roix.fused_noalloc(t, w.eb_mode, w.eb_value, crit, got)
    torch.cuda.synchronize()
    return got.collect(), ref.collect()


def test_noalloc_equals_fused_two_calls_second_smaller():
    import torch

    from paper_2602_15917_amd import roix
    ctx = roix.Context(0, 1 << 30)
    big = synth.ellipsoids128()
    small = synth.batch_volume(5, side=(40, 72))
    assert small.volume.size < big.volume.size
    for name, w in (("128^3 ellipsoids", big), ("small ellipsoids", small)):
        dims = roix.Dims(*w.volume.shape[::-1])
        assert roix.scratch_bytes(dims, roix.F32) <= roix.NOALLOC_SCRATCH_BYTES
        log(f"[case] noalloc vs fused: {name} {w.volume.shape}")
        got, ref = _run_both(roix, torch, ctx, w)
        assert got["einfo"].status == 0 and got["einfo"].n_codes > 0
        _equal(got, ref)
    ctx.close()


def test_noalloc_refuses_volumes_beyond_the_array():
    import torch

    from paper_2602_15917_amd import roix
    shape = (200, 200, 200)
    dims = roix.Dims(*shape)
    assert roix.scratch_bytes(dims, roix.F32) > roix.NOALLOC_SCRATCH_BYTES
    vol = torch.zeros(shape, dtype=torch.float32, device="cuda:0")
    crit = roix.Criterion()
    out = roix.Outputs("cuda:0", 16, 16, 16, 16)
    log("[case] noalloc refuses 200^3")
    with pytest.raises(roix.RoixError) as ei:
        roix.fused_noalloc(vol, "abs", 1e-3, crit, out)
    assert ei.value.status == roix.ENOMEM
