"""GPU parity of the normalised 8-bit pixel section (Sec. 4.1.2, Eq. 1)
through the C ABI: roix_section on the outputs of a roix_fused call against
the oracle's section of the same extraction, byte for byte, for code widths
of 8, 16 and 32 bits, float32 and uint16 volumes, escaped codes, more codes
than one sweep of the grid covers, ragged tails, an empty region of
interest, a short output buffer, an extraction that failed and an escape
list larger than the arena holds; and the paper's quantiser on the section
against the oracle's."""
import numpy as np
import pytest

import oracle
import synth
from roixtest import compare_fused, criterion, default_caps, log, oracle_fused

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


CASES = ["ellipsoids128 f32 w16", "rings 96x96x9 u16", "cylinder 80^3", "ellipsoids w8", "offset w8 escapes",
         "normal w32 ragged rows", "normal 64x256x1024 all kept", "batch volume 5"]
# cases whose extraction has escaped codes (outliers) of 8, 16 and 32 bits
WITH_ESCAPES = {"rings 96x96x9 u16", "cylinder 80^3", "offset w8 escapes", "normal w32 ragged rows",
                "normal 64x256x1024 all kept"}


def make_case(name):
    """(volume, eb mode, eb value, criterion) of a named case."""
    if name.startswith("ellipsoids"):
        w = synth.ellipsoids128()
        if name == "ellipsoids w8":
            return w.volume, "abs", 1e-2, synth.Criterion("otsu", 0.0, 6, "largest", 1)
    elif name.startswith("rings"):
        w = synth.rings2048(nxy=96, nz=9)
    elif name.startswith("cylinder"):
        w = synth.cylinder1024(n=80)
    elif name == "offset w8 escapes":
        # values near 2e4 with eb 1e-2: 8-bit codes, and float rounding of x r
        # and q w leaves about 1% of the voxels outside the bound
        return synth.normal((10, 30, 201), 91, 20000.0, 0.5), "abs", 1e-2, synth.Criterion("fixed", 19990.0, 6,
                                                                                          "largest", 1)
    elif name == "normal w32 ragged rows":
        # |x| < 5 with eb 1e-6: K ~ 5e6 codes, 32-bit codes
        return synth.normal((12, 40, 333), 77, 0.0, 1.0), "abs", 1e-6, synth.Criterion("fixed", 0.5, 26, "min_size", 1)
    elif name == "normal 64x256x1024 all kept":
        # every voxel kept: 16.7M codes, more than one sweep of the default grid
        return (synth.normal((64, 256, 1024), 78, 0.5, 0.1), "abs", 1e-3,
                synth.Criterion("fixed", -1.0, 6, "largest", 1))
    else:
        w = synth.batch_volume(5, side=(24, 96))
    return w.volume, w.eb_mode, w.eb_value, w.criterion


@pytest.mark.parametrize("name", CASES)
def test_section_equals_oracle(env, name):
    ctx, roix, torch = env
    vol, ebm, ebv, c = make_case(name)
    log(f"[case] section {name}")
    crit = criterion(roix, c)
    caps = default_caps(roix, vol, crit)
    t = torch.from_numpy(np.ascontiguousarray(vol)).to("cuda:0")
    out = roix.Outputs("cuda:0", *caps)
    ctx.fused(t, ebm, ebv, crit, out)
    sec, info = ctx.section(t, out)
    torch.cuda.synchronize()
    g = out.collect()
    o = oracle_fused(vol, ebm, ebv, crit, caps)
    compare_fused(g, o)
    si = roix.section_info(info)
    n = int(o["info"].n_codes)
    assert (si.status, si.n_codes) == (0, n)
    st, want = oracle.section(vol, o["params"], o["rows"], n)
    assert st == 0
    got = sec[:n].cpu().numpy()
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, f"{bad.size} levels differ, first at {bad[0]}: gpu {got[bad[0]]} oracle {want[bad[0]]}"
    if name in WITH_ESCAPES:
        assert int(o["info"].n_outliers) > 0  # escaped codes went through the row search


def test_section_escape_list_overflow(env):
    # an arena with room for one listed escape per workgroup of the
    # streaming pass: most of this extraction's 2556 escapes (in few
    # workgroups: 157 645 codes) are resolved in the streaming pass, with the
    # same levels
    ctx, roix, torch = env
    vol, ebm, ebv, c = make_case("normal w32 ragged rows")
    crit = criterion(roix, c)
    caps = default_caps(roix, vol, crit)
    t = torch.from_numpy(vol).to("cuda:0")
    out = roix.Outputs("cuda:0", *caps)
    ctx.fused(t, ebm, ebv, crit, out)
    small = roix.Context(0, 2 * 8 * 4096)
    log("[case] section with one listed escape per workgroup")
    sec, info = small.section(t, out)
    torch.cuda.synchronize()
    small.close()
    o = oracle_fused(vol, ebm, ebv, crit, caps)
    n = int(o["info"].n_codes)
    assert int(o["info"].n_outliers) > 2000
    assert roix.section_info(info).status == 0
    st, want = oracle.section(vol, o["params"], o["rows"], n)
    assert np.array_equal(sec[:n].cpu().numpy(), want)


def test_section_empty_roi(env):
    ctx, roix, torch = env
    vol = synth.normal((3, 20, 70), 5, 0.5, 0.1)
    crit = roix.Criterion("fixed", 10.0, 6, "largest", 1)
    t = torch.from_numpy(vol).to("cuda:0")
    out = roix.Outputs("cuda:0", *default_caps(roix, vol, crit))
    log("[case] section of an empty region of interest")
    ctx.fused(t, "abs", 1e-3, crit, out)
    sec, info = ctx.section(t, out)
    torch.cuda.synchronize()
    si = roix.section_info(info)
    assert (si.status, si.n_codes) == (0, 0)
    assert int(out.collect()["einfo"].n_rows) == 0


def test_section_short_buffer_and_failed_extraction(env):
    ctx, roix, torch = env
    w = synth.ellipsoids128()
    crit = criterion(roix, w.criterion)
    t = torch.from_numpy(w.volume).to("cuda:0")
    caps = default_caps(roix, w.volume, crit)
    out = roix.Outputs("cuda:0", *caps)
    ctx.fused(t, w.eb_mode, w.eb_value, crit, out)
    torch.cuda.synchronize()
    n = int(out.collect()["einfo"].n_codes)
    log("[case] section into a buffer of n - 1 bytes")
    small = torch.full((n - 1,), 7, dtype=torch.uint8, device="cuda:0")
    _, info2 = ctx.section(t, out, small)
    torch.cuda.synchronize()
    assert roix.section_info(info2).status == roix.ETRUNC and bool((small == 7).all())
    # an extraction whose stream did not fit: its error, nothing written
    log("[case] section of a truncated extraction")
    short = roix.Outputs("cuda:0", caps[0], 4096, caps[2], caps[3])
    ctx.fused(t, w.eb_mode, w.eb_value, crit, short)
    dst3 = torch.full((n + 16,), 7, dtype=torch.uint8, device="cuda:0")
    sec3, info3 = ctx.section(t, short, dst3)
    torch.cuda.synchronize()
    assert int(short.collect()["einfo"].status) == roix.ETRUNC
    assert roix.section_info(info3).status == roix.ETRUNC and bool((dst3 == 7).all())


@pytest.mark.parametrize("e", [2.0, 1.0, 5.0])
def test_abs_quantize_on_the_section(env, e):
    # the section as the paper's quantiser's input: byte for byte and the
    # same group count as the oracle's sequential scan of the oracle's section
    ctx, roix, torch = env
    w = synth.ellipsoids128()
    crit = criterion(roix, w.criterion)
    t = torch.from_numpy(w.volume).to("cuda:0")
    out = roix.Outputs("cuda:0", *default_caps(roix, w.volume, crit))
    log(f"[case] abs_quantize on the ellipsoids128 section, E = {e}")
    ctx.fused(t, w.eb_mode, w.eb_value, crit, out)
    sec, info = ctx.section(t, out)
    torch.cuda.synchronize()
    n = int(roix.section_info(info).n_codes)
    px = sec[:n].clone()
    ac = roix.Context(0, roix.abs_quantize_scratch_bytes(n))
    q, qi = ac.abs_quantize(px, e)
    torch.cuda.synchronize()
    ac.close()
    o = oracle_fused(w.volume, w.eb_mode, w.eb_value, crit)
    st, osec = oracle.section(w.volume, o["params"], o["rows"], int(o["info"].n_codes))
    st, oq, ng = oracle.abs_quantize(osec, e)
    assert np.array_equal(q.cpu().numpy(), oq)
    assert int(roix.absq_info(qi).n_groups) == ng
