"""Full-size parity: the benchmark workload (1024^3 float32) and the 8 GB
uint16 stack (2048 x 2048 x 1024) through the fused C-ABI call, in the launch
configuration the benchmark times, compared bit-exactly with the CPU oracle
through SHA-256 digests of every output section; then the Eq. 1 normalised
8-bit pixel section of the same extraction and the paper's quantiser on it.  The digests are written by
tests/golden/make_digests.py, which runs only the oracle."""
import hashlib
import json
import os

import numpy as np
import pytest

import synth
from roixtest import criterion, log

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "digests.json")


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.mark.parametrize("name", ["ellipsoids128", "cylinder1024", "rings2048"])
def test_fullsize_digests(name):
    import torch

    from paper_2602_15917_amd import roix
    gold = json.load(open(GOLDEN)).get(name)
    if gold is None:
        pytest.skip(f"no oracle digest for {name}")
    log(f"[case] full-size {name}: generating")
    w = getattr(synth, name)()
    assert w.sha256() == gold["input_sha256"], "generator output differs from the digested input"
    crit = criterion(roix, w.criterion)
    x = torch.from_numpy(w.volume).to("cuda:0")
    del w.volume
    dims = roix.dims_of(x)
    dt = roix.F32 if x.dtype == torch.float32 else roix.U16
    ctx = roix.Context(0, roix.scratch_bytes(dims, dt, crit))
    b = roix.bounds(dims, dt, crit)
    out = roix.Outputs("cuda:0", b["rows"], b["stream_bytes"], int(gold["extract"]["n_outliers"]) + 1024, 1 << 20)
    log(f"[case] full-size {name}: fused")
    ctx.fused(x, w.eb_mode, w.eb_value, crit, out)
    torch.cuda.synchronize()
    g = out.collect()
    gsec = gold.get("section")
    if gsec is not None:
        # the Eq. 1 normalised section of the same extraction, and the
        # paper's quantiser on it
        log(f"[case] full-size {name}: section")
        n = int(g["einfo"].n_codes)
        sec, sinfo = ctx.section(x, out, torch.empty(n + 16, dtype=torch.uint8, device="cuda:0"))
        torch.cuda.synchronize()
        si = roix.section_info(sinfo)
        assert (si.status, si.n_codes) == (gsec["status"], gsec["n"])
        px = sec[:n]
        assert sha(px.cpu().numpy()) == gsec["sha256"], "section"
        ac = roix.Context(0, roix.abs_quantize_scratch_bytes(n))
        for e, ga in gold["absq_on_section"].items():
            log(f"[case] full-size {name}: abs_quantize on the section, E = {e}")
            q, qi = ac.abs_quantize(px, float(e))
            torch.cuda.synchronize()
            a = roix.absq_info(qi)
            assert (a.status, a.n_groups) == (ga["status"], ga["n_groups"]), e
            assert sha(q.cpu().numpy()) == ga["sha256"], e
        ac.close()
        del sec, px
    ctx.close()
    q, s, e = g["qinfo"], g["sinfo"], g["einfo"]
    assert (q.status, s.status, e.status) == (0, 0, 0)
    gq = gold["quant"]
    for f in ("qmin", "qmax", "K", "width_bits", "esc"):
        assert getattr(q, f) == gq[f], f
    for f in ("xmin", "xmax", "eb32", "w", "r"):
        assert np.float32(getattr(q, f)) == np.float32(gq[f]), f
    gs = gold["seg"]
    for f in ("otsu_bin", "q_thr", "flags", "n_mask", "n_components", "n_kept", "n_kept_voxels"):
        assert getattr(s, f) == gs[f], f
    assert list(s.bbox) == gs["bbox"]
    assert sha(np.frombuffer(bytes(s.hist), np.uint64)) == gs["hist_sha256"]
    ge = gold["extract"]
    for f in ("n_rows", "n_codes", "n_outliers", "stream_bytes"):
        assert getattr(e, f) == ge[f], f
    hs = gold["sha256"]
    assert sha(g["rows"]) == hs["rows"]
    assert sha(g["stream"]) == hs["stream"]
    assert sha(g["outliers"]) == hs["outliers"]
    assert sha(g["comps"]) == hs["comps"]
