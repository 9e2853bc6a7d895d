"""GPU parity of the decoder (the reverse process of Sec. 4.3) through the C
ABI: the library's extraction of each case, decoded on the GPU, against the
oracle's decode of the oracle's extraction, bit for bit, for several
background values; inconsistent tables against the oracle's verdict; and at
full size, properties that hold at any size (every span voxel within the
bound of its input value or equal to it, every other voxel the background,
as many decoded voxels as codes)."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from roixtest import criterion, default_caps, log, oracle_fused

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


def extract_and_decode(env, vol, eb_mode, eb_value, crit_o, backgrounds):
    ctx, roix, torch = env
    crit = criterion(roix, crit_o)
    t = torch.from_numpy(np.ascontiguousarray(vol)).to("cuda:0")
    out = roix.Outputs("cuda:0", *default_caps(roix, vol, crit))
    ctx.fused(t, eb_mode, eb_value, crit, out)
    res = []
    for bg in backgrounds:
        d, di = ctx.decode(out, roix.dims_of(t), bg)
        torch.cuda.synchronize()
        res.append((d.cpu().numpy(), roix.decode_info(di)))
    return out.collect(), res


CASES = [
    ("ellipsoids128", lambda: synth.ellipsoids128().volume, "abs", 1e-3, synth.Criterion("otsu", 0.0, 6, "min_size", 64)),
    ("cylinder 96", lambda: synth.cylinder1024(n=96).volume, "abs", 1e-4, synth.Criterion("otsu", 0.0, 26, "largest", 1)),
    ("rings u16", lambda: synth.rings2048(nxy=128, nz=6).volume, "rel", 1e-4,
     synth.Criterion("otsu", 0.0, 26, "largest", 1)),
    ("noise 8-bit", lambda: synth.normal((7, 33, 101), 5, 0.5, 0.2), "abs", 5e-3,
     synth.Criterion("fixed", 0.45, 6, "min_size", 1)),
    ("noise 32-bit escapes", lambda: synth.normal((6, 20, 97), 77, 0.5, 0.2), "abs", 3.3e-6,
     synth.Criterion("fixed", 0.5, 26, "min_size", 1)),
    ("large values, 16-bit escapes", lambda: (1000.0 + 1000.0 * np.random.default_rng(7).random((4, 16, 256)))
     .astype(np.float32), "abs", 0.03, synth.Criterion("otsu", 0.0, 26, "largest", 1)),
    ("large values, 8-bit escapes", lambda: (1.0e6 + 2000.0 * np.random.default_rng(8).random((3, 9, 192)))
     .astype(np.float32), "abs", 7.3, synth.Criterion("fixed", 1.0008e6, 6, "min_size", 1)),
    ("ragged rows", lambda: synth.normal((3, 5, 67), 9, 0.0, 1.0), "abs", 1e-3,
     synth.Criterion("otsu", 0.0, 6, "min_size", 1)),
    # rows of several 512-voxel units and a ragged last unit
    ("long rows, 16-bit", lambda: synth.normal((2, 6, 1100), 13, 0.5, 0.2), "abs", 1e-4,
     synth.Criterion("fixed", 0.45, 26, "min_size", 1)),
    ("long rows, 32-bit escapes", lambda: synth.normal((2, 5, 1300), 14, 0.5, 0.2), "abs", 3.3e-6,
     synth.Criterion("fixed", 0.5, 6, "min_size", 1)),
]


@pytest.mark.parametrize("k", range(len(CASES)))
def test_decode_equals_oracle(env, k):
    name, make, ebm, ebv, c = CASES[k]
    vol = make()
    log(f"[case] decode {name} shape={vol.shape} dtype={vol.dtype}")
    bgs = (0.0, -7.25, float("nan"))
    g, res = extract_and_decode(env, vol, ebm, ebv, c, bgs)
    o = oracle_fused(vol, ebm, ebv, c)
    assert g["einfo"].status == 0 and o["info"].ext_status == 0
    assert g["stream"].tobytes() == o["stream"].tobytes()
    for bg, (dec, di) in zip(bgs, res):
        st, ref = oracle.decode(o["rows"], o["stream"], o["outliers"], o["params"], vol.shape, background=bg)
        assert st == 0 and di.status == 0, (st, di.status)
        assert (di.n_rows, di.n_outliers) == (o["info"].n_rows, o["info"].n_outliers)
        assert dec.view(np.uint32).tobytes() == ref.view(np.uint32).tobytes(), f"decode differs (background {bg})"


def test_decode_empty_roi(env):
    # nothing is object: no rows, every voxel is the background
    v = synth.normal((3, 9, 70), 5, 1.0, 0.1)
    g, res = extract_and_decode(env, v, "abs", 1e-3, synth.Criterion("fixed", 100.0, 26, "largest", 1), (2.5,))
    dec, di = res[0]
    assert g["einfo"].n_rows == 0 and di.status == 0
    assert np.all(dec == np.float32(2.5))


def corrupt_and_decode(env, out, dims, edit):
    """Apply edit(rows) to a host copy of the row table, upload it into the
    outputs' table, decode, and return the decoder's status."""
    ctx, roix, torch = env
    e = out.collect()
    rows = e["rows"].view(oracle.ROW_DTYPE).copy()
    edit(rows)
    out.rows[: rows.nbytes].copy_(torch.from_numpy(rows.view(np.uint8)).to(out.rows.device))
    d, di = ctx.decode(out, dims, 0.0)
    torch.cuda.synchronize()
    return roix.decode_info(di).status, rows


def test_decode_inconsistent_tables(env):
    ctx, roix, torch = env
    w = synth.cylinder1024(n=64)
    vol = w.volume
    crit = criterion(roix, w.criterion)
    t = torch.from_numpy(vol).to("cuda:0")
    dims = roix.dims_of(t)
    o = oracle_fused(vol, "abs", 3.3e-6, w.criterion)  # tiny bound: escapes in many rows
    assert o["info"].n_outliers > 10

    def fresh():
        out = roix.Outputs("cuda:0", *default_caps(roix, vol, crit))
        ctx.fused(t, "abs", 3.3e-6, crit, out)
        torch.cuda.synchronize()
        return out

    def shift_outliers(r):
        r["outlier_off"][len(r) // 2:] += 1

    def empty_span(r):
        r["xe"][3] = r["xs"][3]

    def outside(r):
        r["z"][-1] = vol.shape[0]

    # cases both the oracle and the decoder reject
    for name, edit in (("outlier offsets", shift_outliers), ("empty span", empty_span), ("row outside", outside)):
        log(f"[case] decode inconsistent: {name}")
        st, rows = corrupt_and_decode(env, fresh(), dims, edit)
        ost, _ = oracle.decode(rows, o["stream"], o["outliers"], o["params"], vol.shape)
        assert ost == oracle.EINVAL and st == roix.EINVAL, (name, ost, st)

    # rows out of raster order: the decoder insists on the order the extraction writes
    def swap(r):
        r[[1, 2]] = r[[2, 1]]
    log("[case] decode inconsistent: order")
    st, _ = corrupt_and_decode(env, fresh(), dims, swap)
    assert st == roix.EINVAL

    # an extraction that reported truncation is not decoded
    log("[case] decode after truncation")
    caps = list(default_caps(roix, vol, crit))
    caps[1] = 64
    out = roix.Outputs("cuda:0", *caps)
    ctx.fused(t, "abs", 3.3e-6, crit, out)
    d, di = ctx.decode(out, dims, 0.0)
    torch.cuda.synchronize()
    assert out.collect()["einfo"].status == roix.ETRUNC and roix.decode_info(di).status == roix.EINVAL


def test_decode_argument_errors(env):
    ctx, roix, torch = env
    lib = roix.load()
    dims = roix.Dims(8, 4, 2)
    d = torch.empty(64, dtype=torch.float32, device="cuda:0")
    q = torch.zeros(ctypes.sizeof(roix.QuantInfo), dtype=torch.uint8, device="cuda:0")
    e = torch.zeros(ctypes.sizeof(roix.ExtractInfo), dtype=torch.uint8, device="cuda:0")
    di = torch.zeros(ctypes.sizeof(roix.DecodeInfo), dtype=torch.uint8, device="cuda:0")
    ok = (ctx.h, None, 0, None, 0, None, 0, q.data_ptr(), e.data_ptr(), dims, 0.0, d.data_ptr(), di.data_ptr(),
          None)
    assert lib.roix_decode(*ok) == 0
    torch.cuda.synchronize()
    assert roix.decode_info(di).status == roix.EINVAL  # the zeroed quant info has no valid width
    bad = list(ok)
    bad[2] = 5  # a row capacity without a table
    assert lib.roix_decode(*bad) == roix.EINVAL
    bad = list(ok)
    bad[11] = d.data_ptr() + 2  # misaligned output
    assert lib.roix_decode(*bad) == roix.EINVAL
    bad = list(ok)
    bad[9] = roix.Dims(0, 4, 2)
    assert lib.roix_decode(*bad) == roix.EINVAL


def test_decode_fullsize_properties(env):
    ctx, roix, torch = env
    w = synth.cylinder1024()
    log("[case] decode full size: fused + decode")
    crit = criterion(roix, w.criterion)
    x = torch.from_numpy(w.volume).to("cuda:0")
    del w.volume
    dims = roix.dims_of(x)
    big = roix.Context(0, roix.scratch_bytes(dims, roix.F32, crit))
    b = roix.bounds(dims, roix.F32, crit)
    out = roix.Outputs("cuda:0", b["rows"], b["stream_bytes"], 1 << 20, 1 << 20)
    big.fused(x, w.eb_mode, w.eb_value, crit, out)
    dec, di = big.decode(out, dims, float("nan"))
    torch.cuda.synchronize()
    info = roix.decode_info(di)
    e = out.collect()["einfo"]
    q = out.collect()["qinfo"]
    big.close()
    assert e.status == 0 and info.status == 0
    inside = ~torch.isnan(dec)
    assert int(inside.sum()) == e.n_codes
    err = (dec - x).abs()
    assert bool((err[inside] <= q.eb32).all())
    exact = int((err[inside] == 0).sum())
    assert exact >= e.n_outliers
