"""Helpers shared by the GPU parity tests: run the library through the C ABI
and compare its outputs with the CPU oracle, field by field and byte by byte."""
from __future__ import annotations

import hashlib
import sys

import numpy as np

import oracle


def log(msg):
    """Name the case before each GPU step (flushed, so it survives a crash)."""
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


def criterion(roix, c):
    return roix.Criterion(c.thr, c.fixed_value, c.connectivity, c.keep, c.min_size)


def default_caps(roix, vol, crit, comps_cap=None):
    nz, ny, nx = vol.shape
    b = roix.bounds(roix.Dims(nx, ny, nz), roix.F32 if vol.dtype == np.float32 else roix.U16, crit)
    cc = b["components"] if comps_cap is None else comps_cap
    return b["rows"], b["stream_bytes"], b["outliers"], min(cc, 1 << 22)


def gpu_fused(ctx, roix, torch, vol, eb_mode, eb_value, crit, caps=None, device="cuda:0"):
    t = torch.from_numpy(np.ascontiguousarray(vol)).to(device)
    caps = caps or default_caps(roix, vol, crit)
    out = roix.Outputs(device, *caps, nz_slices=vol.shape[0] if crit.thr == "otsu_slice" else 0)
    ctx.fused(t, eb_mode, eb_value, crit, out)
    torch.cuda.synchronize()
    return out.collect()


def oracle_fused(vol, eb_mode, eb_value, crit, caps=None):
    kw = {}
    if caps is not None:
        kw = dict(rows_cap=caps[0], stream_cap_bytes=caps[1], outliers_cap=caps[2], comps_cap=caps[3])
    return oracle.fused(vol, eb_mode, eb_value, crit.thr, crit.fixed_value, crit.connectivity, crit.keep,
                        crit.min_size, **kw)


def f32_bits(x):
    return np.float32(x).view(np.uint32)


def compare_fused(g, o, check_outputs=True):
    """Assert GPU fused outputs == oracle outputs (bit-exact)."""
    q, p = g["qinfo"], o["params"]
    oi = o["info"]
    assert q.status == p.status, ("qinfo.status", q.status, p.status)
    if p.status == 0:
        for f in ("xmin", "xmax", "eb32", "w", "r"):
            assert f32_bits(getattr(q, f)) == f32_bits(getattr(p, f)), (f, getattr(q, f), getattr(p, f))
        for f in ("qmin", "qmax", "K", "width_bits", "esc"):
            assert getattr(q, f) == getattr(p, f), (f, getattr(q, f), getattr(p, f))
    s = g["sinfo"]
    assert s.status == oi.seg_status, ("sinfo.status", s.status, oi.seg_status)
    if p.status == 0:
        gh = np.frombuffer(bytes(s.hist), np.uint64)
        assert np.array_equal(gh, o["hist"]), "histogram"
        for f, of in (("otsu_bin", "otsu_bin"), ("q_thr", "q_thr"), ("flags", "flags"), ("n_mask", "n_mask"),
                      ("n_components", "n_components")):
            assert getattr(s, f) == getattr(oi, of), (f, getattr(s, f), getattr(oi, of))
    if oi.seg_status == 0:
        for f in ("n_kept", "n_kept_voxels"):
            assert getattr(s, f) == getattr(oi, f), (f, getattr(s, f), getattr(oi, f))
        assert list(s.bbox) == list(oi.bbox), ("bbox", list(s.bbox), list(oi.bbox))
    if p.status == 0 and s.status == 0:
        assert list(s.thresholds) == list(oi.thresholds), ("thresholds", list(s.thresholds), list(oi.thresholds))
        assert s.n_classes == oi.n_classes, ("n_classes", s.n_classes, oi.n_classes)
        if g.get("slice_thr") is not None:
            assert np.array_equal(g["slice_thr"], o["slice_thr"]), "per-slice splits"
    e = g["einfo"]
    assert e.status == oi.ext_status, ("einfo.status", e.status, oi.ext_status)
    for f in ("n_rows", "n_codes", "n_outliers", "stream_bytes"):
        assert getattr(e, f) == getattr(oi, f), (f, getattr(e, f), getattr(oi, f))
    if not check_outputs:
        return
    if oi.seg_status == 0:
        gc = np.frombuffer(g["comps"].tobytes(), oracle.COMP_DTYPE)
        assert gc.tobytes() == o["comps"].tobytes(), first_diff(gc, o["comps"], "comps")
    if oi.ext_status in (0, oracle.ETRUNC):
        gr = np.frombuffer(g["rows"].tobytes(), oracle.ROW_DTYPE)
        assert gr.tobytes() == o["rows"].tobytes(), first_diff(gr, o["rows"], "rows")
        assert g["stream"].tobytes() == o["stream"].tobytes(), first_diff(g["stream"], o["stream"], "stream")
        assert g["outliers"].view(np.uint32).tobytes() == o["outliers"].view(np.uint32).tobytes(), "outliers"


def first_diff(a, b, what):
    n = min(len(a), len(b))
    for i in range(n):
        if a[i].tobytes() != b[i].tobytes():
            return f"{what}: first difference at {i}: gpu {a[i]} oracle {b[i]} (len {len(a)} vs {len(b)})"
    return f"{what}: lengths {len(a)} vs {len(b)}"


def digest(g):
    """SHA-256 of every output section (for full-size comparisons)."""
    h = {}
    for k in ("rows", "stream", "outliers", "comps"):
        h[k] = hashlib.sha256(np.ascontiguousarray(g[k]).tobytes()).hexdigest()
    return h


def device_sections(out):
    """The info structs (host bytes) and the output sections trimmed to their
    counts, left on the device (for large comparisons without host copies)."""
    import torch

    from paper_2602_15917_amd import roix
    q = bytes(out.qinfo.cpu().numpy().tobytes())
    s = bytes(out.sinfo.cpu().numpy().tobytes())
    e = bytes(out.einfo.cpu().numpy().tobytes())
    ei = roix.ExtractInfo.from_buffer_copy(e)
    si = roix.SegInfo.from_buffer_copy(s)
    rows_cap, stream_cap, outl_cap, comps_cap = out.caps
    nr = min(int(ei.n_rows), rows_cap)
    nb = min(int(ei.stream_bytes), stream_cap)
    no = min(int(ei.n_outliers), outl_cap)
    nc = min(int(si.n_components), comps_cap)
    return {"qinfo": q, "sinfo": s, "einfo": e, "status": (int(ei.status), int(si.status)),
            "rows": out.rows[: nr * roix.ROW_BYTES], "stream": out.stream[:nb],
            "outliers": out.outliers[:no].view(torch.int32), "comps": out.comps[: nc * roix.COMP_BYTES]}


def assert_sections_equal(a, b, what=""):
    """Byte equality of two device_sections() results."""
    import torch
    for k in ("qinfo", "sinfo", "einfo"):
        assert a[k] == b[k], (what, k)
    for k in ("rows", "stream", "outliers", "comps"):
        assert a[k].numel() == b[k].numel() and torch.equal(a[k], b[k]), (what, k)
