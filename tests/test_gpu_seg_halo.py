"""GPU parity of the cross-segment unions when segments are much shorter than
a slice (seg_runs = 256).  In a noisy volume whose mask percolates, a segment
spans a few rows of one slice; its head then reaches two row windows of
earlier runs (the previous slice under its rows, and the rows just before its
first run) with a gap between them that is not staged.  In a sparse volume a
segment spans several slices and the two windows merge.  Both connectivities
and keep rules; every output against the oracle, bit for bit."""
import numpy as np
import pytest

import oracle  # noqa: F401  (the oracle behind oracle_fused)
import synth
from roixtest import compare_fused, criterion, gpu_fused, log, oracle_fused

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2602_15917_amd import roix
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    roix.load()
    ctx = roix.Context(0, 1 << 30)
    ctx.set_param("seg_runs", 256)
    yield ctx, roix, torch
    ctx.close()


def noise_volume(shape, seed):
    """Independent uniform values: Otsu splits the noise itself, the mask
    breaks into many short runs per row and percolates."""
    return np.random.default_rng(seed).random(shape, dtype=np.float32)


def sparse_volume(shape, seed):
    nz, ny, nx = shape
    vol, _ = synth.ellipsoids(nx, ny, nz, seed, n_ell=3, ax=(0.5, 6.0))
    return vol.astype(np.float32)


CASES = [("noise", (4, 60, 128), noise_volume), ("noise-wide", (3, 40, 320), noise_volume),
         ("sparse", (6, 24, 64), sparse_volume)]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("conn", [6, 26])
@pytest.mark.parametrize("keep", ["largest", "min_size"])
def test_short_segments(env, case, conn, keep):
    ctx, roix, torch = env
    name, shape, make = CASES[case]
    vol = make(shape, 7500 + case)
    c = synth.Criterion("otsu", 0.0, conn, keep, 1 if keep == "largest" else 3)
    log(f"[case] short segments {name} shape={shape} conn={conn} keep={keep}")
    g = gpu_fused(ctx, roix, torch, vol, "abs", 1e-3, criterion(roix, c))
    o = oracle_fused(vol, "abs", 1e-3, c)
    n_comp = int(o["info"].n_components)
    log(f"  runs/components: {n_comp} components")
    if name.startswith("noise") and conn == 6:
        assert n_comp > 100  # 26-connected, the noise mask is one component
    compare_fused(g, o)
