"""GPU parity of the lossless Huffman stage through the C ABI: code lengths,
block offsets and payload words identical to the oracle's on seeded byte
sequences (uniform, peaked, constant, two-valued, heavy-tailed, the code
stream of an extraction, the paper quantiser's output) at sizes across the
4096-byte block edges; the sub-block index (code bits of every 256-byte
sub-block) identical to the oracle's; the GPU decoder returning the input,
from the block starts alone and from every sub-block's start, from the
GPU's encoding and from the oracle's; lengths beyond 32 bits, a payload too
small, corrupted offsets, tables and sub-block indexes; and at the full size
of the benchmark stream, properties that hold at any size."""
import numpy as np
import pytest

import oracle
import synth
from roixtest import criterion, default_caps, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2602_15917_amd import roix
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    roix.load()
    ctx = roix.Context(0, 1 << 24)
    yield ctx, roix, torch
    ctx.close()


def data(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.integers(0, 256, n).astype(np.uint8)
    if kind == "peaked":
        return np.clip(np.round(rng.normal(120, 4, n)), 0, 255).astype(np.uint8)
    if kind == "constant":
        return np.full(n, 42, np.uint8)
    if kind == "two":
        return np.where(rng.random(n) < 0.9, 7, 200).astype(np.uint8)
    if kind == "pareto":
        return np.minimum(rng.pareto(0.8, n) * 3, 255).astype(np.uint8)
    if kind == "section":
        return synth.pixel_section_u8(n, seed) if n > 0 else np.zeros(0, np.uint8)
    raise ValueError(kind)


def gpu_encode(env, d, cap=None):
    ctx, roix, torch = env
    t = torch.from_numpy(d).to("cuda:0") if d.size else torch.zeros(16, dtype=torch.uint8, device="cuda:0")[:0]
    ln, off, pay, info = ctx.huff_encode(t, cap)
    torch.cuda.synchronize()
    i = roix.huff_info(info)
    return ln.cpu().numpy(), off.cpu().numpy().astype(np.uint64), pay, i


SIZES = [0, 1, 15, 16, 17, 2048, 4095, 4096, 4097, 7096, 100_003, (1 << 20) + 5]
KINDS = ["uniform", "peaked", "constant", "two", "pareto", "section"]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", SIZES)
def test_huffman_equals_oracle(env, kind, n):
    ctx, roix, torch = env
    d = data(kind, n, 6000 + n % 1009)
    log(f"[case] huffman kind={kind} n={n}")
    st, oln, ooff, opay = oracle.huff_encode(d)
    ln, off, pay, info = gpu_encode(env, d)
    assert st == 0 and info.status == 0
    assert np.array_equal(ln, oln)
    assert np.array_equal(off, ooff)
    words = int(ooff[-1])
    assert info.payload_words == words and info.n_blocks == len(ooff) - 1
    assert info.compressed_bytes == 256 + 8 * len(ooff) + 4 * words
    assert pay[:words].cpu().numpy().view(np.uint32).tobytes() == opay.tobytes()
    # the GPU decoder, from the GPU's encoding and from the oracle's
    lt = torch.from_numpy(oln).to("cuda:0")
    ot = torch.from_numpy(ooff.astype(np.int64)).to("cuda:0")
    pt = torch.from_numpy(opay.view(np.int32) if opay.size else np.zeros(1, np.int32)).to("cuda:0")
    for src in ((ln, off, pay), (lt, ot, pt)):
        l_, o_, p_ = src
        l_ = torch.as_tensor(l_).to("cuda:0")
        o_ = torch.as_tensor(o_.astype(np.int64) if isinstance(o_, np.ndarray) else o_).to("cuda:0")
        back, dinfo = ctx.huff_decode(l_, o_, p_, words, n)
        torch.cuda.synchronize()
        assert roix.huff_info(dinfo).status == 0
        assert back.cpu().numpy().tobytes() == d.tobytes()


SUB_SIZES = [0, 1, 255, 256, 257, 4095, 4096, 4097, 7096, 100_003, (1 << 20) + 5]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", SUB_SIZES)
def test_huffman_sub_block_index(env, kind, n):
    # the index equals the oracle's and the payload is unchanged by it; the
    # sub-block decoder returns the input from the GPU's encoding and from
    # the oracle's
    ctx, roix, torch = env
    d = data(kind, n, 8100 + n % 1013)
    log(f"[case] huffman sub-block index kind={kind} n={n}")
    st, oln, ooff, opay, osub = oracle.huff_encode(d, with_sub=True)
    t = torch.from_numpy(d).to("cuda:0") if d.size else torch.zeros(16, dtype=torch.uint8, device="cuda:0")[:0]
    ln, off, pay, info, sub = ctx.huff_encode(t, with_sub=True)
    torch.cuda.synchronize()
    i = roix.huff_info(info)
    nb = len(ooff) - 1
    assert st == 0 and i.status == 0
    assert np.array_equal(ln.cpu().numpy(), oln) and np.array_equal(off.cpu().numpy().astype(np.uint64), ooff)
    words = int(ooff[-1])
    assert pay[:words].cpu().numpy().view(np.uint32).tobytes() == opay.tobytes()
    assert np.array_equal(sub[: 16 * nb].cpu().numpy().view(np.uint16), osub)
    assert i.compressed_bytes == 256 + 8 * len(ooff) + 4 * words + 32 * nb
    ot = torch.from_numpy(ooff.astype(np.int64)).to("cuda:0")
    pt = torch.from_numpy(opay.view(np.int32) if opay.size else np.zeros(1, np.int32)).to("cuda:0")
    st_ = torch.from_numpy(osub.view(np.int16) if osub.size else np.zeros(1, np.int16)).to("cuda:0")
    for l_, o_, p_, s_ in ((ln, off, pay, sub), (torch.from_numpy(oln).to("cuda:0"), ot, pt, st_)):
        back, dinfo = ctx.huff_decode(l_, o_, p_, words, n, sub=s_)
        torch.cuda.synchronize()
        assert roix.huff_info(dinfo).status == 0
        assert back.cpu().numpy().tobytes() == d.tobytes()


@pytest.mark.parametrize("where", ["first", "middle", "last"])
@pytest.mark.parametrize("delta", [1, -1])
def test_huffman_sub_block_index_corrupted(env, where, delta):
    # a sub-block length one bit off: the oracle and the GPU both refuse it
    ctx, roix, torch = env
    d = data("section", 50_000, 23)
    st, oln, ooff, opay, osub = oracle.huff_encode(d, with_sub=True)
    j = {"first": 0, "middle": 16 * 5 + 7, "last": (d.size - 1) // 256}[where]
    bad = osub.astype(np.int64)
    bad[j] += delta
    bad = bad.astype(np.uint16)
    assert oracle.huff_decode(oln, ooff, opay, d.size, bad)[0] == oracle.EINVAL
    log(f"[case] huffman sub-block index {where} {delta:+d}")
    back, dinfo = ctx.huff_decode(torch.from_numpy(oln).to("cuda:0"),
                                  torch.from_numpy(ooff.astype(np.int64)).to("cuda:0"),
                                  torch.from_numpy(opay.view(np.int32)).to("cuda:0"), int(ooff[-1]), d.size,
                                  sub=torch.from_numpy(bad.view(np.int16)).to("cuda:0"))
    torch.cuda.synchronize()
    assert roix.huff_info(dinfo).status == roix.EINVAL


@pytest.mark.parametrize("kind", ["section", "uniform", "two"])
@pytest.mark.parametrize("n", [17, 4097, 100_003, (1 << 20) + 5])
def test_huffman_decode_unaligned_payload(env, kind, n):
    # a payload that is 4-byte but not 16-byte aligned: the decoder reads it
    # word by word instead of in 16-byte loads
    ctx, roix, torch = env
    d = data(kind, n, 7700 + n % 101)
    st, oln, ooff, opay = oracle.huff_encode(d)
    words = int(ooff[-1])
    log(f"[case] huffman decode, unaligned payload kind={kind} n={n}")
    buf = torch.zeros(words + 4, dtype=torch.int32, device="cuda:0")
    buf[1:1 + words] = torch.from_numpy(opay.view(np.int32)).to("cuda:0")
    p = buf[1:1 + words]
    assert st == 0 and p.data_ptr() % 16 == 4
    back, dinfo = ctx.huff_decode(torch.from_numpy(oln).to("cuda:0"),
                                  torch.from_numpy(ooff.astype(np.int64)).to("cuda:0"), p, words, n)
    torch.cuda.synchronize()
    assert roix.huff_info(dinfo).status == 0
    assert back.cpu().numpy().tobytes() == d.tobytes()


def test_huffman_decode_truncated_payload(env):
    # the last block's offset cut short: its codes run past its words
    ctx, roix, torch = env
    d = data("section", 50_000, 19)
    st, oln, ooff, opay = oracle.huff_encode(d)
    o = ooff.astype(np.int64).copy()
    o[-1] -= 1
    words = int(o[-1])
    log("[case] huffman decode, last block one word short")
    back, dinfo = ctx.huff_decode(torch.from_numpy(oln).to("cuda:0"), torch.from_numpy(o).to("cuda:0"),
                                  torch.from_numpy(opay.view(np.int32)).to("cuda:0"), words, d.size)
    torch.cuda.synchronize()
    assert roix.huff_info(dinfo).status == roix.EINVAL


def test_huffman_of_an_extraction_stream(env):
    # the packed code stream of an extraction (16-bit codes) and the paper
    # quantiser's 8-bit output
    ctx, roix, torch = env
    w = synth.cylinder1024(n=128)
    crit = criterion(roix, w.criterion)
    out = roix.Outputs("cuda:0", *default_caps(roix, w.volume, crit))
    ctx.fused(torch.from_numpy(w.volume).to("cuda:0"), w.eb_mode, w.eb_value, crit, out)
    torch.cuda.synchronize()
    g = out.collect()
    stream = g["stream"]
    log(f"[case] huffman of an extraction stream ({stream.size} bytes)")
    for d in (stream, oracle.abs_quantize(synth.pixel_section_u8(300_000, 5), 2.0)[1]):
        st, oln, ooff, opay = oracle.huff_encode(d)
        ln, off, pay, info = gpu_encode(env, np.ascontiguousarray(d))
        assert st == 0 and info.status == 0 and np.array_equal(ln, oln) and np.array_equal(off, ooff)
        assert pay[: int(ooff[-1])].cpu().numpy().view(np.uint32).tobytes() == opay.tobytes()
        assert info.compressed_bytes < d.size  # these sequences compress


def test_huffman_lengths_beyond_32_bits(env):
    # Fibonacci counts over 34 bytes need a 33-bit code: ERANGE, as the oracle
    fib = [1, 1]
    while len(fib) < 34:
        fib.append(fib[-1] + fib[-2])
    d = np.repeat(np.arange(34, dtype=np.uint8), fib)
    np.random.default_rng(3).shuffle(d)
    log(f"[case] huffman Fibonacci counts ({d.size} bytes)")
    st, *_ = oracle.huff_encode(d)
    ln, off, pay, info = gpu_encode(env, d)
    assert st == oracle.ERANGE and info.status == roix_status(env, "ERANGE") and info.max_len == 33


@pytest.mark.parametrize("nsym", [26, 29, 31])
def test_huffman_long_codes_and_wide_blocks(env, nsym):
    # Fibonacci counts over nsym bytes give codes of up to nsym - 1 bits
    # (25: code and length share one table entry; 28 and 30: they do not);
    # the rarest bytes come first, so the first block needs 1491 to 2131
    # payload words and the encoder goes through it in several LDS windows
    ctx, roix, torch = env
    fib = [1, 1]
    while len(fib) < nsym:
        fib.append(fib[-1] + fib[-2])
    d = np.repeat(np.arange(nsym, dtype=np.uint8), fib)
    np.random.default_rng(nsym).shuffle(d[4096:])
    log(f"[case] huffman long codes nsym={nsym} ({d.size} bytes)")
    st, oln, ooff, opay = oracle.huff_encode(d)
    ln, off, pay, info = gpu_encode(env, d)
    assert st == 0 and info.status == 0 and info.max_len == nsym - 1
    assert int(ooff[1]) > 1024
    assert np.array_equal(ln, oln) and np.array_equal(off, ooff)
    words = int(ooff[-1])
    assert pay[:words].cpu().numpy().view(np.uint32).tobytes() == opay.tobytes()
    back, dinfo = ctx.huff_decode(torch.as_tensor(ln).to("cuda:0"), torch.from_numpy(off.astype(np.int64)).to("cuda:0"),
                                  pay, words, d.size)
    torch.cuda.synchronize()
    assert roix.huff_info(dinfo).status == 0
    assert back.cpu().numpy().tobytes() == d.tobytes()
    # and from every sub-block's start (sub-blocks of up to 256 * 30 bits)
    st, _, _, _, osub = oracle.huff_encode(d, with_sub=True)
    back, dinfo = ctx.huff_decode(torch.as_tensor(ln).to("cuda:0"), torch.from_numpy(off.astype(np.int64)).to("cuda:0"),
                                  pay, words, d.size, sub=torch.from_numpy(osub.view(np.int16)).to("cuda:0"))
    torch.cuda.synchronize()
    assert roix.huff_info(dinfo).status == 0
    assert back.cpu().numpy().tobytes() == d.tobytes()


def roix_status(env, name):
    return getattr(env[1], name)


def test_huffman_payload_too_small_and_bad_inputs(env):
    ctx, roix, torch = env
    d = data("uniform", 50_000, 11)
    st, oln, ooff, opay = oracle.huff_encode(d)
    log("[case] huffman payload too small")
    ln, off, pay, info = gpu_encode(env, d, cap=100)
    assert info.status == roix.ETRUNC and info.payload_words == int(ooff[-1]) and np.array_equal(off, ooff)
    lt = torch.from_numpy(oln).to("cuda:0")
    pt = torch.from_numpy(opay.view(np.int32)).to("cuda:0")
    words = int(ooff[-1])
    # offsets past the payload, decreasing offsets, a first offset not 0
    for name, edit in (("past", lambda o: o.__setitem__(-1, o[-1] + 3)),
                       ("decreasing", lambda o: o.__setitem__(3, o[2] - 1)),
                       ("first", lambda o: o.__setitem__(0, 1))):
        o = ooff.astype(np.int64).copy()
        edit(o)
        log(f"[case] huffman decode, offsets {name}")
        back, dinfo = ctx.huff_decode(lt, torch.from_numpy(o).to("cuda:0"), pt, words, d.size)
        torch.cuda.synchronize()
        assert roix.huff_info(dinfo).status == roix.EINVAL, name
    # lengths that are no prefix code (every used byte one bit)
    bad = oln.copy()
    bad[bad > 0] = 1
    log("[case] huffman decode, bad lengths")
    back, dinfo = ctx.huff_decode(torch.from_numpy(bad).to("cuda:0"), torch.from_numpy(ooff.astype(np.int64)).to(
        "cuda:0"), pt, words, d.size)
    torch.cuda.synchronize()
    assert roix.huff_info(dinfo).status == roix.EINVAL


def test_huffman_full_size_stream(env):
    # the benchmark volume's code stream: the lengths are the oracle's for
    # the GPU histogram, the payload is the optimal size the lengths give, and
    # the decoder returns the stream
    ctx, roix, torch = env
    w = synth.cylinder1024()
    crit = criterion(roix, w.criterion)
    x = torch.from_numpy(w.volume).to("cuda:0")
    del w.volume
    dims = roix.dims_of(x)
    big = roix.Context(0, roix.scratch_bytes(dims, roix.F32, crit))
    b = roix.bounds(dims, roix.F32, crit)
    out = roix.Outputs("cuda:0", b["rows"], b["stream_bytes"], 1 << 22, 1 << 22)
    big.fused(x, w.eb_mode, w.eb_value, crit, out)
    torch.cuda.synchronize()
    del x
    e = out.collect()["einfo"]
    q = out.collect()["qinfo"]
    n = int(e.n_codes) * (int(q.width_bits) // 8)
    s = out.stream[:n]
    log(f"[case] huffman full-size stream ({n} bytes)")
    ln, off, pay, info = big.huff_encode(s)
    torch.cuda.synchronize()
    i = roix.huff_info(info)
    hist = torch.bincount(s.to(torch.int64), minlength=256).cpu().numpy().astype(np.uint64)
    st, oln = oracle.huff_lengths(hist)
    assert i.status == 0 and st == 0 and np.array_equal(ln.cpu().numpy(), oln)
    bits = int((hist.astype(object) * oln.astype(object)).sum())
    assert bits <= i.payload_words * 32 < bits + 32 * i.n_blocks
    back, dinfo = big.huff_decode(ln, off, pay, i.payload_words, n)
    torch.cuda.synchronize()
    assert roix.huff_info(dinfo).status == 0 and torch.equal(back, s)
    # with the sub-block index: the same payload; every 256-byte sub-block's
    # bits are the sum of its bytes' code lengths; the decoder returns the
    # stream from every sub-block's start
    log("[case] huffman full-size stream, sub-block index")
    ln2, off2, pay2, info2, sub = big.huff_encode(s, with_sub=True)
    torch.cuda.synchronize()
    i2 = roix.huff_info(info2)
    assert i2.status == 0 and i2.payload_words == i.payload_words
    assert torch.equal(pay2[: i.payload_words], pay[: i.payload_words]) and torch.equal(off2, off)
    lens = torch.from_numpy(oln.astype(np.int32)).to("cuda:0")
    pad = torch.zeros(16 * int(i.n_blocks) * 256, dtype=torch.int32, device="cuda:0")
    pad[:n] = lens[s.to(torch.int64)]
    want = pad.view(-1, 256).sum(dim=1)
    assert torch.equal(sub[: 16 * int(i.n_blocks)].to(torch.int32) & 0xFFFF, want)
    back.zero_()
    back, dinfo = big.huff_decode(ln2, off2, pay2, i2.payload_words, n, back, sub=sub)
    torch.cuda.synchronize()
    assert roix.huff_info(dinfo).status == 0 and torch.equal(back, s)
    big.close()
