"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bit-exact on every output: quantiser fields, histogram, threshold, component
table, row table, code stream and outlier values.  Inputs are the seeded
synthetic volumes of ``synth`` plus hand-made edge cases.  Every case runs
twice: with the default launch parameters, and with the one-pass 16-bit proxy
flow of float32 volumes forced down to the smallest volumes
(fused16_min_voxels = 0), so that both quantiser flows meet every case.
"""
import numpy as np
import pytest

import oracle
import synth
from roixtest import (compare_fused, criterion, default_caps, gpu_fused, log, oracle_fused)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["default", "fused16"])
def env(request):
    import torch

    from paper_2602_15917_amd import roix
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    roix.load()
    ctx = roix.Context(0, 1 << 30)
    if request.param == "fused16":
        ctx.set_param("fused16_min_voxels", 0)
    log(f"[env] {request.param}")
    yield ctx, roix, torch
    ctx.close()


def run_case(env, name, vol, eb_mode, eb_value, crit_o, caps=None):
    ctx, roix, torch = env
    log(f"[case] {name} shape={vol.shape} dtype={vol.dtype} eb={eb_mode}:{eb_value} crit={crit_o}")
    crit = criterion(roix, crit_o)
    g = gpu_fused(ctx, roix, torch, vol, eb_mode, eb_value, crit, caps)
    o = oracle_fused(vol, eb_mode, eb_value, crit_o, caps)
    compare_fused(g, o)
    return g, o


def test_ellipsoids128_full(env):
    w = synth.ellipsoids128()
    g, o = run_case(env, "ellipsoids128", w.volume, w.eb_mode, w.eb_value, w.criterion)
    assert o["info"].n_components == 3 and g["einfo"].n_codes > 0


SHAPES = [(1, 1, 1), (1, 1, 7), (1, 5, 3), (3, 1, 1), (2, 3, 64), (4, 9, 65), (5, 7, 130), (3, 4, 200),
          (17, 13, 33), (9, 40, 64), (6, 6, 127), (2, 2, 1000), (40, 3, 5), (2, 3, 2052), (2, 2, 4160),
          (1, 1, 4)]


@pytest.mark.parametrize("k", range(len(SHAPES)))
@pytest.mark.parametrize("conn", [6, 26])
def test_small_ellipsoid_volumes(env, k, conn):
    nz, ny, nx = SHAPES[k]
    vol, _ = synth.ellipsoids(nx, ny, nz, 4000 + k, n_ell=3, ax=(0.5, 6.0))
    for keep, ms in (("largest", 1), ("min_size", 3)):
        c = synth.Criterion("otsu", 0.0, conn, keep, ms)
        run_case(env, f"ellipsoids{SHAPES[k]}", vol, "abs", 1e-3, c)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("conn", [6, 26])
def test_noise_many_components(env, seed, conn):
    # threshold inside the noise: thousands of small components and long union chains
    vol = synth.normal((11, 37, 70 + seed), 5000 + seed, 0.5, 0.1)
    for keep, ms in (("min_size", 1), ("min_size", 5), ("largest", 1)):
        c = synth.Criterion("fixed", 0.55, conn, keep, ms)
        run_case(env, f"noise seed={seed}", vol, "abs", 1e-3, c)
    c = synth.Criterion("otsu", 0.0, conn, "min_size", 2)
    run_case(env, f"noise-otsu seed={seed}", vol, "abs", 1e-4, c)


@pytest.mark.parametrize("conn", [6, 26])
def test_dense_planes_fallback(env, conn):
    # z-planes of ~45k runs: many segments per plane, and more distinct root pairs
    # across segment boundaries than the pair table holds (direct global unions)
    vol = synth.normal((4, 300, 301), 6000 + conn, 0.5, 0.1)
    for keep, ms in (("min_size", 1), ("largest", 1)):
        run_case(env, f"dense planes conn={conn}", vol, "abs", 1e-3, synth.Criterion("fixed", 0.5, conn, keep, ms))


@pytest.mark.parametrize("seg_runs,seg_grid", [(256, 3), (2048, 1), (16384, 512), (0, 7), (768, 64)])
def test_segment_parameters(env, seg_runs, seg_grid):
    # segments of any size cut rows and planes anywhere; the labels must not change
    ctx, roix, torch = env
    ctx.set_param("seg_runs", seg_runs)
    ctx.set_param("seg_grid", seg_grid)
    try:
        vol = synth.normal((9, 41, 133), 6100, 0.5, 0.1)
        for conn in (6, 26):
            run_case(env, f"segments T={seg_runs} G={seg_grid} noise", vol, "abs", 1e-3,
                     synth.Criterion("fixed", 0.55, conn, "min_size", 2))
        w = synth.cylinder1024(n=96)
        run_case(env, f"segments T={seg_runs} G={seg_grid} cylinder", w.volume, w.eb_mode, w.eb_value, w.criterion)
    finally:
        ctx.set_param("seg_runs", 0)
        ctx.set_param("seg_grid", ctx.get_param("compute_units") * 2)


def short_span_volume(shape, seed, max_len, dtype):
    """One object run per row at a random place, 1..max_len voxels long (row
    spans of a few codes, many span starts inside one 4-code quad), and a
    kept voxel at the volume's very last position."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    lo, hi = (0.0, 1.0) if dtype == np.float32 else (100, 40000)
    vol = np.full(shape, lo, dtype=np.float64)
    vol += rng.random(shape) * (hi - lo) * 0.2
    ln = rng.integers(1, max_len + 1, size=(nz, ny))
    x0 = rng.integers(0, nx, size=(nz, ny))
    for z in range(nz):
        for y in range(ny):
            if rng.random() < 0.9:
                a = min(x0[z, y], nx - ln[z, y])
                vol[z, y, a:a + ln[z, y]] = hi * (0.8 + 0.2 * rng.random())
    vol[-1, -1, -1] = hi
    return vol.astype(dtype)


@pytest.mark.parametrize("max_len", [1, 3, 9, 40])
@pytest.mark.parametrize("dt", ["f32", "u16"])
def test_short_spans(env, max_len, dt):
    dtype = np.float32 if dt == "f32" else np.uint16
    thr = 0.5 if dt == "f32" else 20000.0
    # f32: 16-bit codes, 16-bit codes with escapes, 32-bit codes with escapes;
    # u16: 16- and 8-bit codes
    ebs = (1e-3, 1e-5, 1e-6) if dt == "f32" else (2.0, 200.0)
    for shape in ((20, 300, 257), (3, 101, 64)):
        vol = short_span_volume(shape, 6200 + max_len, max_len, dtype)
        for eb in ebs:
            run_case(env, f"short spans {dt} len<={max_len} {shape} eb={eb}", vol, "abs", eb,
                     synth.Criterion("fixed", thr, 6, "min_size", 1))


@pytest.mark.parametrize("shape", [(4, 16, 256), (3, 9, 192), (2, 5, 4096)])
def test_large_values_with_outliers(env, shape):
    # values far above the step, so that fp32 rounding puts many voxels just
    # outside the bound: escapes in 16-bit (K ~ 1.7e4) and 8-bit (K ~ 125)
    # code streams, on rows of whole 64-voxel words
    rng = np.random.default_rng(sum(shape))
    base = rng.random(shape)
    v16 = (1000.0 + 1000.0 * base).astype(np.float32)
    g, o = run_case(env, f"outliers16 {shape}", v16, "abs", 0.03, synth.Criterion("otsu", 0.0, 26, "largest", 1))
    assert o["info"].n_outliers > 0
    v8 = (1.0e6 + 2000.0 * base).astype(np.float32)
    v8[:, : shape[1] // 2, :] += np.float32(1000.0)
    g, o = run_case(env, f"outliers8 {shape}", v8, "abs", 7.3, synth.Criterion("fixed", 1.0008e6, 6, "min_size", 3))
    assert o["params"].width_bits == 8 and o["info"].n_outliers > 0


def test_uint16_rings_small(env):
    w = synth.rings2048(nxy=256, nz=12)
    run_case(env, "rings u16 small", w.volume, w.eb_mode, w.eb_value, w.criterion)


def test_cylinder_medium(env):
    w = synth.cylinder1024(n=192)
    run_case(env, "cylinder 192^3", w.volume, w.eb_mode, w.eb_value, w.criterion)


@pytest.mark.parametrize("eb", [1e-2, 1e-3, 1e-4, 1e-5, 3.3e-6])
def test_code_widths_and_outliers(env, eb):
    # K spans the 8/16/32-bit widths; small bounds give fp32 escapes
    vol = synth.normal((6, 20, 97), 77, 0.5, 0.2)
    c = synth.Criterion("fixed", 0.5, 26, "min_size", 1)
    g, o = run_case(env, f"widths eb={eb}", vol, "abs", eb, c)


def test_edge_cases(env):
    c6 = synth.Criterion("otsu", 0.0, 6, "min_size", 1)
    # constant volume: degenerate histogram, empty ROI, no rows
    run_case(env, "constant", np.full((4, 5, 66), 0.25, np.float32), "abs", 1e-3, c6)
    run_case(env, "constant x4", np.full((3, 7, 256), -3.5, np.float32), "abs", 1e-3, c6)
    # flat regions beside noise; K just below 2^15 with codes on both sides
    # of zero, then of 2^15, then K above 2^15 (the 1-byte proxy flow)
    v = synth.normal((4, 16, 128), 11, 0.0, 1.0)
    v[:, :8, :] = np.float32(-1.0)
    v[1:3, 4:12, 32:96] = np.float32(2.0)
    c26 = synth.Criterion("otsu", 0.0, 26, "largest", 1)
    run_case(env, "flat and noise", v, "abs", 1.2e-4, c26)
    run_case(env, "flat and noise shifted", (v + np.float32(8.5)).astype(np.float32), "abs", 1.2e-4, c26)
    run_case(env, "flat and noise fixed", v, "abs", 1.2e-4, synth.Criterion("fixed", 0.3, 6, "min_size", 2))
    run_case(env, "flat and noise wide", v, "abs", 2e-5, c26)
    # relative bound on a constant volume: invalid bound
    run_case(env, "constant rel", np.full((2, 3, 4), 7.0, np.float32), "rel", 1e-4, c6)
    # everything is object
    v = synth.normal((3, 9, 70), 5, 1.0, 0.1)
    run_case(env, "all object", v, "abs", 1e-3, synth.Criterion("fixed", -100.0, 26, "largest", 1))
    # nothing is object
    run_case(env, "no object", v, "abs", 1e-3, synth.Criterion("fixed", 100.0, 26, "largest", 1))
    # negative values and signed zeros
    v = synth.normal((3, 8, 40), 6, -0.2, 0.3)
    v[0, 0, 0], v[1, 1, 1] = -0.0, 0.0
    run_case(env, "negative", v, "abs", 1e-3, c6)
    # denormal inputs
    v = (synth.normal((2, 4, 64), 8, 0.0, 1.0) * np.float32(1e-38)).astype(np.float32)
    assert (np.abs(v) < np.finfo(np.float32).tiny).any()
    run_case(env, "denormals", v, "abs", 1e-37, c6)
    run_case(env, "denormal bound", v, "abs", 1e-39, c6)
    # non-finite input
    for bad in (np.nan, np.inf, -np.inf):
        v = synth.normal((2, 3, 50), 9, 0.0, 1.0)
        v[1, 2, 33] = bad
        run_case(env, f"non-finite {bad}", v, "abs", 1e-3, c6)
    # codes beyond 2^24
    run_case(env, "erange", synth.normal((2, 3, 10), 10, 0.0, 1e4), "abs", 1e-6, c6)
    # uint16 extremes
    u = np.zeros((3, 4, 70), np.uint16)
    u[1, 1:3, 5:60] = 65535
    run_case(env, "u16 extremes", u, "abs", 0.5, synth.Criterion("otsu", 0.0, 26, "largest", 1))
    run_case(env, "u16 rel", u, "rel", 1e-4, synth.Criterion("otsu", 0.0, 6, "largest", 1))


def test_misaligned_input(env):
    # volumes that do not start on a 16-byte boundary: element-wise head/tail paths
    ctx, roix, torch = env
    for w, offs in ((synth.ellipsoids128(), (1, 2, 3)), (synth.rings2048(nxy=64, nz=5), (1, 3, 5, 7))):
        n = w.volume.size
        flat = torch.from_numpy(np.ascontiguousarray(w.volume).ravel()).to("cuda:0")
        base = torch.zeros(n + 8, dtype=flat.dtype, device="cuda:0")
        crit = criterion(roix, w.criterion)
        o = oracle_fused(w.volume, w.eb_mode, w.eb_value, w.criterion)
        for off in offs:
            log(f"[case] misaligned {w.name} offset={off}")
            base[off: off + n] = flat
            t = base[off: off + n].view(w.volume.shape)
            out = roix.Outputs("cuda:0", *default_caps(roix, w.volume, crit))
            ctx.fused(t, w.eb_mode, w.eb_value, crit, out)
            torch.cuda.synchronize()
            compare_fused(out.collect(), o)


def test_truncation_reports_full_counts(env):
    w = synth.ellipsoids128()
    c = w.criterion
    caps = (10, 100, 0, 3)
    run_case(env, "etrunc rows/stream", w.volume, w.eb_mode, w.eb_value, c, caps)
    run_case(env, "etrunc comps", w.volume, w.eb_mode, w.eb_value, c, (16384, 1 << 24, 1 << 20, 2))


def test_scratch_too_small_for_runs(env):
    _, roix, torch = env
    vol = synth.normal((8, 32, 128), 11, 0.5, 0.1)
    nz, ny, nx = vol.shape
    dims = roix.Dims(nx, ny, nz)
    crit = roix.Criterion("fixed", 0.5, 6, "min_size", 1)
    need = roix.scratch_bytes(dims, roix.F32, crit)
    worst_run_bytes = 17 * ny * nz * (nx // 2)
    small = roix.Context(0, need - worst_run_bytes + 17 * 100)  # room for 100 runs only
    log("[case] enomem")
    g = gpu_fused(small, roix, torch, vol, "abs", 1e-3, crit)
    small.close()
    assert g["sinfo"].status == roix.ENOMEM and g["einfo"].status == roix.ENOMEM
    tiny = roix.Context(0, 4096)
    with pytest.raises(roix.RoixError) as ei:
        gpu_fused(tiny, roix, torch, vol, "abs", 1e-3, crit)
    assert ei.value.status == roix.ENOMEM
    tiny.close()


def test_staged_equals_fused_and_oracle(env):
    ctx, roix, torch = env
    for name, w in (("ellipsoids128", synth.ellipsoids128()), ("rings", synth.rings2048(nxy=128, nz=6)),
                    ("cyl", synth.cylinder1024(n=96))):
        for conn in (6, 26):
            c = synth.Criterion(w.criterion.thr, 0.0, conn, w.criterion.keep, w.criterion.min_size)
            crit = criterion(roix, c)
            log(f"[case] staged {name} conn={conn}")
            t = torch.from_numpy(w.volume).to("cuda:0")
            codes, bits, qinfo = ctx.quantize(t, w.eb_mode, w.eb_value)
            caps = default_caps(roix, w.volume, crit)
            keep, labels, comps, sinfo = ctx.segment(codes, qinfo, crit, caps[3], want_labels=True)
            out = roix.Outputs("cuda:0", *caps)
            ctx.extract(t, keep, qinfo, out)
            torch.cuda.synchronize()
            # quantiser
            st, lo, hi = oracle.value_range(w.volume)
            p = oracle.resolve(lo, hi, w.eb_mode, w.eb_value)
            _, oc, ob, on = oracle.quantize(w.volume, p)
            q = roix.parse_info(qinfo, roix.QuantInfo)
            assert q.status == 0 and q.n_outliers == on
            assert np.array_equal(codes.cpu().numpy(), oc)
            assert np.array_equal(bits.cpu().numpy().view(np.uint32), ob)
            # segmentation: per-voxel keep and labels against the oracle's labelling of its own mask
            f = oracle_fused(w.volume, w.eb_mode, w.eb_value, c)
            mask = (oc >= f["info"].q_thr).astype(np.uint8)
            _, olab, okeep, ocomps = oracle.label(mask, conn, c.keep, c.min_size)
            assert np.array_equal(labels.cpu().numpy(), olab)
            assert np.array_equal(keep.cpu().numpy(), okeep)
            s = roix.parse_info(sinfo, roix.SegInfo)
            assert s.n_components == len(ocomps)
            assert comps[: len(ocomps) * 48].cpu().numpy().tobytes() == ocomps.tobytes()
            # extraction: identical to the fused oracle outputs
            g = out.collect()
            e = g["einfo"]
            oi = f["info"]
            assert (e.status, e.n_rows, e.n_codes, e.n_outliers) == (0, oi.n_rows, oi.n_codes, oi.n_outliers)
            assert g["rows"].tobytes() == f["rows"].tobytes()
            assert g["stream"].tobytes() == f["stream"].tobytes()
            assert g["outliers"].tobytes() == f["outliers"].tobytes()


def test_repeat_determinism(env):
    ctx, roix, torch = env
    w = synth.cylinder1024(n=128)
    crit = criterion(roix, w.criterion)
    ref = None
    for i in range(5):
        log(f"[case] repeat {i}")
        g = gpu_fused(ctx, roix, torch, w.volume, w.eb_mode, w.eb_value, crit)
        cur = (g["rows"].tobytes(), g["stream"].tobytes(), g["comps"].tobytes(), g["outliers"].tobytes())
        if ref is None:
            ref = cur
        assert cur == ref


def three_materials(shape, seed):
    """Background, a matrix block and an inclusion of distinct intensities."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    vol = 0.1 + rng.normal(0, 0.01, shape)
    vol[nz // 6: nz - nz // 6, ny // 6: ny - ny // 6, nx // 5: nx - nx // 5] = 0.5
    vol[nz // 3: nz - nz // 3, ny // 3: ny - ny // 3, nx // 3: nx - nx // 3] = 0.9
    vol += rng.normal(0, 0.01, shape)
    return vol.astype(np.float32)


@pytest.mark.parametrize("thr", ["multi3", "multi4"])
@pytest.mark.parametrize("conn", [6, 26])
def test_multi_otsu(env, thr, conn):
    # multi-level Otsu: thresholds, class count and every output against the oracle
    cases = [
        ("three materials", three_materials((12, 24, 96), 31), "abs", 1e-3),
        ("three materials ragged", three_materials((7, 19, 133), 32), "abs", 1e-4),
        ("ellipsoids", synth.ellipsoids(130, 40, 9, 4100, n_ell=4, ax=(2.0, 20.0))[0], "abs", 1e-3),
        ("noise", synth.normal((9, 31, 70), 4200, 0.5, 0.1), "abs", 1e-3),
        ("rings u16", synth.rings2048(nxy=96, nz=5).volume, "rel", 1e-4),
        ("constant", np.full((3, 8, 64), 2.5, np.float32), "abs", 1e-3),
        ("two values", np.where(np.arange(3 * 8 * 64).reshape(3, 8, 64) % 3 == 0, 1.0, 0.0).astype(np.float32),
         "abs", 1e-3),
        ("single voxel", np.full((1, 1, 1), 0.25, np.float32), "abs", 1e-3),
    ]
    for name, vol, ebm, ebv in cases:
        for keep, ms in (("largest", 1), ("min_size", 4)):
            c = synth.Criterion(thr, 0.0, conn, keep, ms)
            g, o = run_case(env, f"{thr} {name}", vol, ebm, ebv, c)
            assert g["sinfo"].n_classes == (3 if thr == "multi3" else 4)


@pytest.mark.parametrize("thr", ["multi3", "multi4"])
def test_multi_otsu_staged(env, thr):
    # the staged segmentation takes the same thresholds from the codes' histogram
    ctx, roix, torch = env
    vol = three_materials((10, 30, 128), 33)
    c = synth.Criterion(thr, 0.0, 26, "min_size", 1)
    crit = criterion(roix, c)
    log(f"[case] staged {thr}")
    t = torch.from_numpy(vol).to("cuda:0")
    codes, bits, qinfo = ctx.quantize(t, "abs", 1e-3)
    caps = default_caps(roix, vol, crit)
    keep, labels, comps, sinfo = ctx.segment(codes, qinfo, crit, caps[3], want_labels=True)
    torch.cuda.synchronize()
    s = roix.parse_info(sinfo, roix.SegInfo)
    f = oracle_fused(vol, "abs", 1e-3, c)
    oi = f["info"]
    assert s.status == 0 and list(s.thresholds) == list(oi.thresholds) and s.n_classes == oi.n_classes
    assert (s.otsu_bin, s.q_thr, s.n_mask, s.n_components) == (oi.otsu_bin, oi.q_thr, oi.n_mask, oi.n_components)


def drifting(shape, seed, span=0.6):
    """A block object whose brightness, and the background's, rises along z."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    obj = np.zeros(shape, bool)
    obj[:, ny // 4: ny - ny // 4, nx // 4: nx - nx // 4] = True
    drift = np.linspace(0.0, span, nz)[:, None, None]
    return (np.where(obj, 0.35, 0.05) + drift + rng.normal(0, 0.01, shape)).astype(np.float32)


@pytest.mark.parametrize("conn", [6, 26])
def test_per_slice_otsu(env, conn):
    # each z-slice thresholded on its own: the splits and every output
    cases = [
        ("drift", drifting((8, 24, 96), 41), "abs", 1e-3),
        ("drift ragged rows", drifting((5, 19, 133), 42), "abs", 1e-4),
        ("drift narrow rows", drifting((6, 9, 13), 43), "abs", 1e-3),
        ("one slice", drifting((1, 40, 64), 44), "abs", 1e-3),
        ("drift long rows", drifting((3, 5, 4160), 46), "abs", 1e-3),  # 65 mask words a row
        ("ellipsoids", synth.ellipsoids(130, 40, 9, 4300, n_ell=4, ax=(2.0, 20.0))[0], "abs", 1e-3),
        ("rings u16", synth.rings2048(nxy=96, nz=5).volume, "rel", 1e-4),
        ("cylinder", synth.cylinder1024(n=96).volume, "abs", 1e-4),
    ]
    vol = drifting((6, 20, 64), 45)
    vol[3] = 0.5  # a constant slice: no split there
    cases.append(("constant slice", vol, "abs", 1e-3))
    for name, vol, ebm, ebv in cases:
        for keep, ms in (("largest", 1), ("min_size", 4)):
            c = synth.Criterion("otsu_slice", 0.0, conn, keep, ms)
            g, o = run_case(env, f"per-slice {name}", vol, ebm, ebv, c)
            assert g["sinfo"].flags & 8 and g["slice_thr"] is not None
            assert np.array_equal(g["slice_thr"], o["slice_thr"])


def test_per_slice_batched_and_rejected_forms(env):
    ctx, roix, torch = env
    # the batched form takes the per-slice criterion like the plain call
    vols = [drifting((4 + k, 16, 48 + 16 * k), 50 + k) for k in range(3)]
    crit = roix.Criterion("otsu_slice", 0.0, 26, "largest", 1)
    items, outs = [], []
    for v in vols:
        out = roix.Outputs("cuda:0", *default_caps(roix, v, crit), nz_slices=v.shape[0])
        items.append((torch.from_numpy(v).to("cuda:0"), "abs", 1e-3, crit, out))
        outs.append(out)
    log("[case] per-slice batched")
    ctx.fused_batch(items)
    torch.cuda.synchronize()
    for v, out in zip(vols, outs):
        o = oracle_fused(v, "abs", 1e-3, synth.Criterion("otsu_slice", 0.0, 26, "largest", 1))
        compare_fused(out.collect(), o)
    # the staged segmentation and the served form refuse it
    t = torch.from_numpy(vols[0]).to("cuda:0")
    codes, bits, qinfo = ctx.quantize(t, "abs", 1e-3)
    with pytest.raises(roix.RoixError) as ei:
        ctx.segment(codes, qinfo, crit, 1024)
    assert ei.value.status == roix.EINVAL
