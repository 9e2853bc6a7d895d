"""GPU parity of the paper's absolute error-bounded quantisation (Sec. 4.2.3)
through the C ABI: roix_abs_quantize against the oracle's sequential scan,
byte for byte with the same group count, on seeded sequences of every kind
the scan meets (uniform noise, random walks, X-CT-like pixel sections,
repeated values, exact ramps whose group chains never meet), at sizes from
empty to several tiles with ragged tails, and at the full size of
the benchmark's pixel section."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from roixtest import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2602_15917_amd import roix
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    roix.load()
    ctx = roix.Context(0, max(1 << 26, roix.abs_quantize_scratch_bytes(1 << 22)))
    yield ctx, roix, torch
    ctx.close()


def sequence(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        d = rng.integers(0, 256, n)
    elif kind == "walk":
        d = np.clip(np.round(128 + np.cumsum(rng.normal(0, 1.5, n))), 0, 255)
    elif kind == "section":
        return synth.pixel_section_u8(n, seed) if n > 0 else np.zeros(0, np.uint8)
    elif kind == "repeats":
        d = np.repeat(rng.integers(0, 256, max(n // 37 + 1, 1)), 37)[:n]
    elif kind == "ramp":  # a value every 3 pixels, wrapping: chains meet at each wrap
        d = (np.arange(n) // 3) % 256
    elif kind == "slow":  # one ramp over the whole sequence: chains from different starts stay out of phase
        d = (np.arange(n, dtype=np.int64) * 256) // max(n, 1)
    else:
        raise ValueError(kind)
    return np.asarray(d, dtype=np.uint8)


def run(env, d, e, inplace=False):
    ctx, roix, torch = env
    t = torch.from_numpy(d).to("cuda:0")
    q, info = ctx.abs_quantize(t, e, t if inplace else None)
    torch.cuda.synchronize()
    return q.cpu().numpy(), roix.absq_info(info)


SIZES = [0, 1, 15, 16, 17, 255, 256, 257, 1000, 16383, 16384, 16385, 100_003, 1 << 20]
KINDS = ["uniform", "walk", "section", "repeats", "ramp", "slow"]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", SIZES)
def test_abs_quantize_equals_oracle(env, kind, n):
    d = sequence(kind, n, 5000 + n % 977)
    for e in (0.0, 1.0, 2.5, 7.0):
        log(f"[case] abs_quantize kind={kind} n={n} E={e}")
        st, oq, og = oracle.abs_quantize(d, e)
        q, info = run(env, d, e)
        assert info.status == 0 and st == 0
        assert info.n_groups == og, (info.n_groups, og)
        assert q.tobytes() == oq.tobytes()


def test_abs_quantize_wide_tolerance_and_overlap(env):
    d = sequence("section", 300_001, 71)
    for e in (127.0, 128.0, 500.0):  # one group over the whole sequence
        log(f"[case] abs_quantize wide E={e}")
        q, info = run(env, d, e)
        st, oq, og = oracle.abs_quantize(d, e)
        assert og == 1 and info.n_groups == 1 and q.tobytes() == oq.tobytes()
    # the output may not overlap the pixels, not even exactly
    ctx, roix, torch = env
    t = torch.from_numpy(d).to("cuda:0")
    with pytest.raises(roix.RoixError) as ei:
        ctx.abs_quantize(t, 2.0, t)
    assert ei.value.status == roix.EINVAL


def test_abs_quantize_long_ramp_uses_the_finisher(env):
    # group chains of an exact ramp never meet: the rounds cannot settle the
    # chunks and the sequential pass does; the result is still the scan's
    d = sequence("slow", 3 << 20, 0)
    log("[case] abs_quantize long ramp")
    q, info = run(env, d, 1.0)
    st, oq, og = oracle.abs_quantize(d, 1.0)
    assert q.tobytes() == oq.tobytes() and info.n_groups == og
    assert info.finisher_chunks > 0


def test_abs_quantize_argument_errors(env):
    ctx, roix, torch = env
    lib = roix.load()
    d = torch.zeros(64, dtype=torch.uint8, device="cuda:0")
    q = torch.zeros(64, dtype=torch.uint8, device="cuda:0")
    info = torch.zeros(ctypes.sizeof(roix.AbsqInfo), dtype=torch.uint8, device="cuda:0")
    null = ctypes.c_void_p(0)
    ok = (ctx.h, d.data_ptr(), 32, 1.0, q.data_ptr(), info.data_ptr(), null)
    assert lib.roix_abs_quantize(*ok) == 0
    torch.cuda.synchronize()
    assert roix.absq_info(info).status == 0

    def bad(i, v):
        a = list(ok)
        a[i] = v
        return lib.roix_abs_quantize(*a)

    assert bad(3, -1.0) == roix.EINVAL
    assert bad(3, float("nan")) == roix.EINVAL
    assert bad(2, -5) == roix.EINVAL
    assert bad(1, d.data_ptr() + 1) == roix.EINVAL       # misaligned pixels
    assert bad(4, d.data_ptr() + 16) == roix.EINVAL      # partial overlap
    assert bad(5, None) == roix.EINVAL
    # an arena too small for the chunk state: rejected before any launch
    # (buffers of the full length, so that nothing could read past them)
    n = 1 << 22
    dd = torch.zeros(n, dtype=torch.uint8, device="cuda:0")
    qq = torch.zeros(n, dtype=torch.uint8, device="cuda:0")
    tiny = roix.Context(0, 1024)
    assert roix.abs_quantize_scratch_bytes(n) > 1024
    assert lib.roix_abs_quantize(tiny.h, dd.data_ptr(), n, 1.0, qq.data_ptr(), info.data_ptr(), null) == roix.ENOMEM
    tiny.close()


def test_abs_quantize_full_size(env):
    # the benchmark's pixel section (514 688 000 pixels), against the oracle
    ctx, roix, torch = env
    m = synth.PIXEL_SECTION_FULL
    d = synth.pixel_section_u8(m)
    big = roix.Context(0, roix.abs_quantize_scratch_bytes(m))
    t = torch.from_numpy(d).to("cuda:0")
    for e in (2.0, 5.0):
        log(f"[case] abs_quantize full size E={e}")
        q, info = big.abs_quantize(t, e)
        torch.cuda.synchronize()
        st, oq, og = oracle.abs_quantize(d, e)
        i = roix.absq_info(info)
        assert i.status == 0 and i.n_groups == og
        assert torch.equal(q, torch.from_numpy(oq).to("cuda:0"))
        del q
    big.close()
