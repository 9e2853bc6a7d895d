"""GPU parity of background subtraction (Sec. 4.1.1) and its inverse through
the C ABI: roix_background against the oracle bit for bit (float32 and
uint16 input, one calibration plane or a reference volume, vector and
single-voxel paths, in place); the whole path on the subtracted volume
against the oracle's path on the oracle's subtraction; decode plus the
reference added back against the oracle's; argument errors."""
import ctypes

import numpy as np
import pytest

import oracle
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


def volume(shape, dtype, seed):
    rng = np.random.default_rng(seed)
    if dtype == np.uint16:
        return rng.integers(0, 65536, shape).astype(np.uint16)
    v = rng.normal(0.3, 2.0, shape).astype(np.float32)
    flat = v.reshape(-1)
    flat[:: 97] = rng.uniform(-1e-38, 1e-38, flat[:: 97].shape).astype(np.float32)  # subnormal results
    flat[1:: 89] = (rng.uniform(-1, 1, flat[1:: 89].shape) * 3e38).astype(np.float32)
    return v


def reference(shape, planes, seed):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    b = rng.normal(0.0, 1.5, (planes, ny, nx)).astype(np.float32)
    b.reshape(-1)[:: 53] = rng.uniform(-1e-38, 1e-38, b.reshape(-1)[:: 53].shape).astype(np.float32)
    return b


SHAPES = [(1, 1, 1), (3, 5, 7), (4, 16, 64), (2, 33, 100), (5, 1, 4096), (3, 64, 65), (17, 3, 12)]


@pytest.mark.parametrize("k", range(len(SHAPES)))
@pytest.mark.parametrize("dt", [np.float32, np.uint16])
def test_background_equals_oracle(env, k, dt):
    ctx, roix, torch = env
    shape = SHAPES[k]
    vol = volume(shape, dt, 700 + k)
    for planes in sorted({1, shape[0]}):
        bg = reference(shape, planes, 800 + k)
        ops = ("subtract", "add") if dt == np.float32 else ("subtract",)
        for op in ops:
            for misalign in (False, True):
                log(f"[case] background {op} shape={shape} dtype={np.dtype(dt)} planes={planes} misalign={misalign}")
                st, ref = oracle.background(vol, bg, op)
                assert st == oracle.OK
                t = torch.from_numpy(vol).to("cuda:0")
                b = torch.from_numpy(bg).to("cuda:0")
                if misalign:  # 4 bytes past a 16-byte boundary: the single-voxel path
                    n = vol.size
                    buf = torch.empty(n + 4, dtype=torch.float32, device="cuda:0")
                    dst = buf[1: n + 1].view(shape)
                else:
                    dst = None
                out = ctx.background(t, b, op, dst)
                torch.cuda.synchronize()
                got = out.cpu().numpy()
                assert got.view(np.uint32).tobytes() == ref.view(np.uint32).tobytes()


def test_background_in_place(env):
    ctx, roix, torch = env
    shape = (6, 40, 128)
    vol = volume(shape, np.float32, 901)
    bg = reference(shape, 1, 902)
    st, ref = oracle.background(vol, bg)
    t = torch.from_numpy(vol).to("cuda:0")
    out = ctx.background(t, torch.from_numpy(bg).to("cuda:0"), "subtract", t)
    torch.cuda.synchronize()
    assert out.data_ptr() == t.data_ptr()
    assert t.cpu().numpy().view(np.uint32).tobytes() == ref.view(np.uint32).tobytes()


def background_field(shape, seed):
    """A smooth background: an offset, a tilt across x and a radial falloff
    (a flat-field-like calibration plane)."""
    nz, ny, nx = shape
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    rr = ((x - nx / 2) ** 2 + (y - ny / 2) ** 2) / (nx * nx / 4)
    rng = np.random.default_rng(seed)
    return (0.3 + 0.4 * x / nx - 0.2 * rr + rng.normal(0, 0.005, (ny, nx)))[None].astype(np.float32)


@pytest.mark.parametrize("conn", [6, 26])
def test_path_after_subtraction(env, conn):
    # subtraction then the fused path equals the oracle's path on the
    # oracle's subtraction, every output bit for bit
    ctx, roix, torch = env
    w = synth.ellipsoids128()
    bg = background_field(w.volume.shape, 903)
    img = (w.volume + bg).astype(np.float32)
    st, m = oracle.background(img, bg)
    c = synth.Criterion("otsu", 0.0, conn, "min_size", 64)
    crit = criterion(roix, c)
    log(f"[case] path after subtraction conn={conn}")
    t = torch.from_numpy(img).to("cuda:0")
    mt = ctx.background(t, torch.from_numpy(bg).to("cuda:0"), "subtract")
    torch.cuda.synchronize()
    assert mt.cpu().numpy().view(np.uint32).tobytes() == m.view(np.uint32).tobytes()
    g = gpu_fused(ctx, roix, torch, mt.cpu().numpy(), "abs", 1e-3, crit)
    o = oracle_fused(m, "abs", 1e-3, c)
    compare_fused(g, o)
    assert o["info"].n_components >= 3


def test_decode_and_add_back(env):
    # reverse process: decode the extraction of M and put the reference back
    ctx, roix, torch = env
    w = synth.ellipsoids128()
    bg = background_field(w.volume.shape, 904)
    img = (w.volume + bg).astype(np.float32)
    c = synth.Criterion("otsu", 0.0, 26, "min_size", 64)
    crit = criterion(roix, c)
    log("[case] decode and add back")
    t = torch.from_numpy(img).to("cuda:0")
    b = torch.from_numpy(bg).to("cuda:0")
    m = ctx.background(t, b, "subtract")
    out = roix.Outputs("cuda:0", *default_caps(roix, img, crit))
    ctx.fused(m, "abs", 1e-3, crit, out)
    dec, di = ctx.decode(out, roix.dims_of(m), 0.0)
    back = ctx.background(dec, b, "add")
    torch.cuda.synchronize()
    _, om = oracle.background(img, bg)
    o = oracle_fused(om, "abs", 1e-3, c)
    st, odec = oracle.decode(o["rows"], o["stream"], o["outliers"], o["params"], img.shape)
    _, oback = oracle.background(odec, bg, "add")
    assert st == 0 and roix.decode_info(di).status == 0
    assert back.cpu().numpy().view(np.uint32).tobytes() == oback.view(np.uint32).tobytes()
    # inside the kept spans the image comes back within the bound plus the two roundings
    inside = odec != 0
    q = o["params"]
    err = np.abs(oback.astype(np.float64) - img.astype(np.float64))[inside]
    slack = 2 * np.spacing(np.abs(img[inside]) + np.abs(bg.repeat(img.shape[0], 0)[inside]) + 1.0)
    assert np.all(err <= q.eb32 + slack)


def test_background_argument_errors(env):
    ctx, roix, torch = env
    lib = roix.load()
    d = roix.Dims(8, 4, 3)
    # 96 voxels; every buffer has room for 128 float32 values, so that no
    # rejected call could reach past one even if it were launched
    v = torch.zeros(128, dtype=torch.float32, device="cuda:0")
    u = torch.zeros(256, dtype=torch.int16, device="cuda:0")
    b = torch.zeros(128, dtype=torch.float32, device="cuda:0")
    o = torch.zeros(128, dtype=torch.float32, device="cuda:0")
    null = ctypes.c_void_p(0)

    def call(src, dt, bg, planes, op, dst):
        return lib.roix_background(ctx.h, src, dt, d, bg, planes, op, dst, null)

    assert call(v.data_ptr(), roix.F32, b.data_ptr(), 1, 0, o.data_ptr()) == 0
    assert call(v.data_ptr(), roix.F32, b.data_ptr(), 3, 1, o.data_ptr()) == 0
    assert call(v.data_ptr(), roix.F32, b.data_ptr(), 1, 0, v.data_ptr()) == 0       # in place
    torch.cuda.synchronize()
    assert call(v.data_ptr(), roix.F32, b.data_ptr(), 2, 0, o.data_ptr()) == roix.EINVAL  # planes not 1 or nz
    assert call(u.data_ptr(), roix.U16, b.data_ptr(), 1, 1, o.data_ptr()) == roix.EINVAL  # ADD on uint16
    assert call(v.data_ptr(), roix.F32, b.data_ptr(), 1, 2, o.data_ptr()) == roix.EINVAL  # unknown op
    assert call(v.data_ptr(), roix.F32, None, 1, 0, o.data_ptr()) == roix.EINVAL
    assert call(v.data_ptr() + 2, roix.F32, b.data_ptr(), 1, 0, o.data_ptr()) == roix.EINVAL  # misaligned
    assert call(v.data_ptr(), roix.F32, b.data_ptr(), 1, 0, v.data_ptr() + 4) == roix.EINVAL  # partial overlap
    assert call(v.data_ptr(), roix.F32, o.data_ptr(), 1, 0, o.data_ptr()) == roix.EINVAL  # output over reference
    assert call(u.data_ptr(), roix.U16, b.data_ptr(), 1, 0, u.data_ptr()) == roix.EINVAL  # uint16 in place


def fused_bg_case(ctx, roix, torch, img, bg, ebm, ebv, c, name):
    log(f"[case] fused background {name} shape={img.shape} planes={bg.shape[0]} eb={ebm}:{ebv} crit={c}")
    crit = criterion(roix, c)
    t = torch.from_numpy(img).to("cuda:0")
    b = torch.from_numpy(bg).to("cuda:0")
    out = roix.Outputs("cuda:0", *default_caps(roix, img, crit),
                       nz_slices=img.shape[0] if c.thr == "otsu_slice" else 0)
    ctx.fused_background(t, b, ebm, ebv, crit, out)
    torch.cuda.synchronize()
    st, m = oracle.background(img, bg)
    o = oracle_fused(m, ebm, ebv, c)
    g = out.collect()
    compare_fused(g, o)
    assert g["rows"].tobytes() == o["rows"].tobytes()
    assert g["stream"].tobytes() == o["stream"].tobytes()
    assert g["outliers"].view(np.uint32).tobytes() == o["outliers"].view(np.uint32).tobytes()
    return g, o


@pytest.mark.parametrize("small_fused", [False, True])
def test_fused_background_equals_subtract_then_path(env, small_fused):
    # the subtraction folded into the path gives the outputs of subtracting
    # first; small_fused lets volumes below the default size take the
    # one-pass flow, where the folding happens
    ctx, roix, torch = env
    c2 = roix.Context(0, 1 << 30)
    if small_fused:
        c2.set_param("fused16_min_voxels", 0)
    w = synth.ellipsoids128()
    plane = background_field(w.volume.shape, 910)
    img = (w.volume + plane).astype(np.float32)
    crit = synth.Criterion("otsu", 0.0, 26, "min_size", 64)
    fused_bg_case(c2, roix, torch, img, plane, "abs", 1e-3, crit, "plane")
    vref = np.concatenate([plane * (1.0 + 0.01 * z) for z in range(img.shape[0])]).astype(np.float32)
    img_v = (w.volume + vref).astype(np.float32)
    fused_bg_case(c2, roix, torch, img_v, vref, "abs", 1e-3, crit, "volume reference")
    # escapes: a bound so small that fp32 rounding misses it on many voxels
    g, o = fused_bg_case(c2, roix, torch, img, plane, "abs", 3.3e-6, crit, "escapes")
    assert o["info"].n_outliers > 0
    # more than 2^15 codes: the range pass falls back to the 1-byte proxy and M is written on the device
    big = (1000.0 + 1000.0 * np.random.default_rng(9).random((4, 16, 256))).astype(np.float32)
    bplane = background_field(big.shape, 911) * 100.0
    g, o = fused_bg_case(c2, roix, torch, (big + bplane).astype(np.float32), bplane, "abs", 0.01,
                         synth.Criterion("otsu", 0.0, 26, "largest", 1), "wide code range")
    assert o["params"].K > (1 << 15)
    # outliers on the one-pass flow: K <= 2^15 keeps the 16-bit proxy, whose
    # flag bits find the outliers, whose values are gathered as I - B; rows of
    # whole 64-voxel words, and 4096-voxel rows so that a span needs several
    # rounds of loads
    for shape, seed in (((4, 16, 256), 916), ((2, 5, 4096), 917)):
        m = (1000.0 + 50.0 * np.random.default_rng(seed).random(shape)).astype(np.float32)
        oplane = background_field(shape, seed + 10) * 100.0
        img_o = (m + oplane).astype(np.float32)
        st_o, m_o = oracle.background(img_o, oplane)
        o_chk = oracle_fused(m_o, "abs", 0.03, synth.Criterion("otsu", 0.0, 26, "largest", 1))
        assert o_chk["params"].K <= (1 << 15) and o_chk["info"].n_outliers > 0, (o_chk["params"].K,
                                                                                  o_chk["info"].n_outliers)
        fused_bg_case(c2, roix, torch, img_o, oplane, "abs", 0.03, synth.Criterion("otsu", 0.0, 26, "largest", 1),
                      f"outliers on the one-pass flow {shape}")
    # many short spans: the proxy emit queues chunks for the general kernel, which reads M
    noise = synth.normal((11, 200, 64), 912, 0.5, 0.1)
    nplane = background_field(noise.shape, 913)
    g, o = fused_bg_case(c2, roix, torch, (noise + nplane).astype(np.float32), nplane, "abs", 1e-3,
                         synth.Criterion("fixed", 0.75, 6, "min_size", 1), "short spans")
    assert o["info"].n_rows > 500 and o["info"].n_codes < 64 * o["info"].n_rows
    # long rows (the range pass loads each plane row once for 8 slices; 19
    # slices leave a partial block) and 768-voxel rows
    for shape in ((19, 12, 1024), (10, 7, 768)):
        nz, ny, nx = shape
        vol, _ = synth.ellipsoids(nx, ny, nz, 914, n_ell=3, ax=(3.0, 40.0))
        lp = background_field(shape, 915)
        fused_bg_case(c2, roix, torch, (vol + lp).astype(np.float32), lp, "abs", 1e-3,
                      synth.Criterion("otsu", 0.0, 26, "min_size", 8), f"long rows {shape}")
    # rows that are no whole 64-voxel words, a relative bound, per-slice thresholds: subtract first
    odd = (w.volume[:, :, :100] + plane[:, :, :100]).astype(np.float32)
    fused_bg_case(c2, roix, torch, np.ascontiguousarray(odd), np.ascontiguousarray(plane[:, :, :100]), "abs", 1e-3,
                  crit, "ragged rows")
    fused_bg_case(c2, roix, torch, img, plane, "rel", 1e-4, crit, "relative bound")
    fused_bg_case(c2, roix, torch, img, plane, "abs", 1e-3, synth.Criterion("otsu_slice", 0.0, 26, "largest", 1),
                  "per-slice")
    c2.close()


def test_fused_background_argument_errors(env):
    ctx, roix, torch = env
    img = np.zeros((2, 4, 64), np.float32)
    crit = roix.Criterion("otsu", 0.0, 26, "largest", 1)
    t = torch.from_numpy(img).to("cuda:0")
    b = torch.zeros((1, 4, 64), dtype=torch.float32, device="cuda:0")
    out = roix.Outputs("cuda:0", *default_caps(roix, img, crit))
    with pytest.raises(roix.RoixError) as ei:  # workspace over the image
        ctx.fused_background(t, b, "abs", 1e-3, crit, out, work=t)
    assert ei.value.status == roix.EINVAL
    with pytest.raises(roix.RoixError) as ei:  # a reference of neither 1 nor nz planes
        ctx.fused_background(t, torch.zeros((3, 4, 64), dtype=torch.float32, device="cuda:0"), "abs", 1e-3, crit,
                             out)
    assert ei.value.status == roix.EINVAL
