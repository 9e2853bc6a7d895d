"""GPU parity of the mask pass when each wave walks many steps: the grid is
cut to one workgroup (grid_mask = 1, four waves), so the two register sets of
the pipelined 16-bit path take turns over several steps, a wave runs out of
whole steps on either set, and the volume's last, partial step goes through
the general loads.  Rows of 4 and 16 words (steps of 16 and 4 rows), uint16
volumes read directly and float32 volumes through the 16-bit proxy (the
one-pass flow, forced on small volumes), both connectivities; every output
against the oracle, bit for bit."""
import numpy as np
import pytest

import oracle  # noqa: F401  (the oracle behind oracle_fused)
import synth
from roixtest import compare_fused, criterion, gpu_fused, log, oracle_fused

pytestmark = pytest.mark.gpu

# (nz, ny, nx): 185 rows of 4 words = 11 whole steps of 16 rows + 9 rows;
# 123 rows of 16 words = 30 whole steps of 4 rows + 3 rows
SHAPES = [(5, 37, 256), (3, 41, 1024)]


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2602_15917_amd import roix
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    roix.load()
    ctx = roix.Context(0, 1 << 30)
    ctx.set_param("grid_mask", 1)
    ctx.set_param("fused16_min_voxels", 0)
    yield ctx, roix, torch
    ctx.close()


def volume(shape, seed, u16):
    nz, ny, nx = shape
    vol, _ = synth.ellipsoids(nx, ny, nz, seed, n_ell=3, ax=(0.5, 6.0))
    if u16:
        return np.clip(np.rint(vol.astype(np.float64) * 60000.0), 0, 65535).astype(np.uint16)
    return vol.astype(np.float32)


@pytest.mark.parametrize("k", range(len(SHAPES)))
@pytest.mark.parametrize("conn", [6, 26])
@pytest.mark.parametrize("u16", [True, False])
def test_mask_many_steps_per_wave(env, k, conn, u16):
    ctx, roix, torch = env
    vol = volume(SHAPES[k], 7400 + k, u16)
    ebm, ebv = ("abs", 2.0) if u16 else ("abs", 1e-3)
    c = synth.Criterion("otsu", 0.0, conn, "largest", 1)
    log(f"[case] mask steps shape={vol.shape} u16={u16} conn={conn}")
    ctx.set_timing(True)
    g = gpu_fused(ctx, roix, torch, vol, ebm, ebv, criterion(roix, c))
    torch.cuda.synchronize()
    stages = ctx.read_timing()
    ctx.set_timing(False)
    o = oracle_fused(vol, ebm, ebv, c)
    if not u16:
        # the one-pass flow wrote the 16-bit proxy
        assert stages["quant_range16"][1] > 0
    assert stages["mask_runs"][1] > 0
    assert 0 < int(o["info"].n_mask) < vol.size
    compare_fused(g, o)
