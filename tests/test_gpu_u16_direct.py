"""GPU parity of uint16 volumes whose rows are whole 64-voxel words (the
mask pass reads the values themselves and compares them with the smallest
value whose code reaches the threshold code; no proxy is written): every
output against the oracle, bit for bit, for row widths of 1, 2, 3, 64 and 65
words (the last one on the long-row path), Otsu, fixed and multi-level
thresholds, absolute and relative bounds, both connectivities, thresholds that
take every voxel or none, and the same volume at offsets that do and do not
keep its rows 16-byte aligned."""
import numpy as np
import pytest

import oracle  # noqa: F401  (the oracle behind oracle_fused)
import synth
from roixtest import compare_fused, criterion, default_caps, gpu_fused, log, oracle_fused

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2602_15917_amd import roix
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    roix.load()
    ctx = roix.Context(0, 1 << 30)
    yield ctx, roix, torch
    ctx.close()


def u16_volume(shape, seed):
    """Ellipsoids over a noisy background, scaled to the uint16 range."""
    nz, ny, nx = shape
    vol, _ = synth.ellipsoids(nx, ny, nz, seed, n_ell=3, ax=(0.5, 6.0))
    return np.clip(np.rint(vol.astype(np.float64) * 60000.0), 0, 65535).astype(np.uint16)


def run(env, name, vol, ebm, ebv, c):
    ctx, roix, torch = env
    log(f"[case] {name} shape={vol.shape} eb={ebm}:{ebv} crit={c}")
    crit = criterion(roix, c)
    g = gpu_fused(ctx, roix, torch, vol, ebm, ebv, crit)
    o = oracle_fused(vol, ebm, ebv, c)
    compare_fused(g, o)
    return g, o


SHAPES = [(3, 17, 64), (5, 9, 128), (4, 11, 192), (2, 6, 4096), (2, 3, 4160)]


@pytest.mark.parametrize("k", range(len(SHAPES)))
@pytest.mark.parametrize("conn", [6, 26])
def test_u16_whole_word_rows(env, k, conn):
    vol = u16_volume(SHAPES[k], 7100 + k)
    for ebm, ebv in (("abs", 2.0), ("abs", 150.0), ("rel", 1e-4)):
        run(env, f"u16 rows {SHAPES[k]} otsu", vol, ebm, ebv, synth.Criterion("otsu", 0.0, conn, "largest", 1))
    run(env, f"u16 rows {SHAPES[k]} fixed", vol, "abs", 2.0,
        synth.Criterion("fixed", 30000.0, conn, "min_size", 2))
    run(env, f"u16 rows {SHAPES[k]} multi3", vol, "rel", 1e-4, synth.Criterion("multi3", 0.0, conn, "largest", 1))
    run(env, f"u16 rows {SHAPES[k]} multi4", vol, "abs", 4.0, synth.Criterion("multi4", 0.0, conn, "min_size", 1))


def test_u16_every_voxel_or_none(env):
    vol = u16_volume((3, 8, 128), 7200)
    vol[1, 2, 5] = 0  # the smallest value, 0, is present
    # a fixed threshold below every code: every voxel is object (the smallest value is 0)
    g, o = run(env, "u16 all object", vol, "abs", 3.0, synth.Criterion("fixed", -10.0, 6, "largest", 1))
    assert int(o["info"].n_mask) == vol.size
    # above every code: no object voxel
    g, o = run(env, "u16 no object", vol, "abs", 3.0, synth.Criterion("fixed", 70000.0, 6, "largest", 1))
    assert int(o["info"].n_mask) == 0
    # the full value range with the largest value present
    v2 = vol.copy()
    v2[2, 7, 127] = 65535
    run(env, "u16 65535", v2, "abs", 0.5, synth.Criterion("fixed", 65535.0, 26, "largest", 1))


def test_u16_alignment(env):
    # the same volume 16-byte aligned (values compared directly) and 8-byte
    # aligned (through the 1-byte proxy): both equal the oracle
    ctx, roix, torch = env
    vol = u16_volume((4, 10, 128), 7300)
    c = synth.Criterion("otsu", 0.0, 26, "largest", 1)
    crit = criterion(roix, c)
    o = oracle_fused(vol, "rel", 1e-4, c)
    n = vol.size
    flat = torch.from_numpy(np.ascontiguousarray(vol).ravel()).to("cuda:0")
    base = torch.zeros(n + 16, dtype=flat.dtype, device="cuda:0")
    for off in (0, 8, 4):
        log(f"[case] u16 offset {off} elements")
        base[off: off + n] = flat
        t = base[off: off + n].view(vol.shape)
        out = roix.Outputs("cuda:0", *default_caps(roix, vol, crit))
        ctx.fused(t, "rel", 1e-4, crit, out)
        torch.cuda.synchronize()
        compare_fused(out.collect(), o)
