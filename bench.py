"""Benchmark: input GB/s of the fused quantise + segment + extract path on one
MI355X, 1024^3 float32 cylinder volume (eb 1e-4 absolute, Otsu,
26-connectivity, largest component), input resident in HBM.

Prints one JSON line: the whole-path throughput, the roofline of the
dominant kernel (algorithmic bytes / its mean duration, against 8 TB/s HBM),
and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "input GB/s quantize+segment+extract (plain vs batched/served); p99 slab latency"
HBM_PEAK_GBS = 8000.0


def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


# source file of each stage's kernels: a traffic figure measured by the
# counters is only reported while that file is unchanged
STAGE_SOURCE = {"range": "k_quant.hip", "quant_hist": "k_quant.hip", "quant_range16": "k_quant.hip",
                "mask_runs": "k_label.hip", "emit": "k_extract.hip"}
STAGE_KERNEL = {"range": "k_range<float>", "quant_hist": "k_quant_hist<float, false, false, 1, true>",
                "quant_range16": "k_quant_range16<false>", "mask_runs": "k_mask_runs", "emit": "k_emit_codes_f32"}
CALIB_BYTES = 1 << 30


def source_sha(stage):
    import hashlib
    f = os.path.join(ROOT, "paper_2602_15917_amd", "csrc", STAGE_SOURCE[stage])
    return hashlib.sha256(open(f, "rb").read()).hexdigest()[:16]


def measured_traffic(stage):
    """(fetch, write) HBM bytes per launch from the committed counter summary,
    or None when there is none or the kernel source has changed since."""
    f = os.path.join(ROOT, "profiles", "traffic_cylinder_1024cubed_f32.txt")
    if not os.path.exists(f):
        return None
    vals = {}
    for line in open(f):
        parts = line.split()
        if len(parts) >= 5 and parts[0] == "stage" and parts[1] == stage:
            vals = {"fetch": float(parts[2]), "write": float(parts[3]), "sha": parts[4]}
    if not vals or vals["sha"] != source_sha(stage):
        return None
    return vals["fetch"], vals["write"]


def pmc_summary(fetch_csv, write_csv, kt_csv):
    """Summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per
    dispatch) into per-launch HBM bytes, scaled by what the same counters
    read for a device copy of CALIB_BYTES (the bench's --calibrate-copy)."""
    import csv
    import re

    def per_kernel(fn, counter):
        acc = {}
        for r in csv.DictReader(open(fn)):
            if r["Counter_Name"] != counter:
                continue
            k = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "").replace("roix::", "")
            acc.setdefault(k, []).append(float(r["Counter_Value"]) * 1024.0)
        return acc

    fetch, write = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    calib = [k for k in fetch if "copy" in k.lower() or "elementwise" in k.lower()]
    cf = max((max(fetch[k]) for k in calib), default=0.0)
    cw = max((max(write.get(k, [0.0])) for k in calib), default=0.0)
    sf = CALIB_BYTES / cf if cf else float("nan")
    sw = CALIB_BYTES / cw if cw else float("nan")
    dur = {}
    if kt_csv:
        for r in csv.DictReader(open(kt_csv)):
            k = re.sub(r"\(.*", "", r["Name"]).replace("void ", "").replace("roix::", "")
            dur[k] = float(r["AverageNs"])
    print(f"calibration: device copy of {CALIB_BYTES} B reads FETCH_SIZE {cf:.0f} B, WRITE_SIZE {cw:.0f} B "
          f"-> scale fetch x{sf:.4f}, write x{sw:.4f}")
    print("# kernel  fetch_bytes_per_launch  write_bytes_per_launch  avg_ns (scaled counters)")
    for k in sorted(fetch, key=lambda k: -max(fetch[k])):
        f = sum(fetch[k]) / len(fetch[k]) * sf
        wv = write.get(k, [0.0])
        wr = sum(wv) / len(wv) * sw
        if f + wr < 1e6:
            continue
        print(f"kernel {k.replace(' ', '')} {f:.4g} {wr:.4g} {dur.get(k, float('nan')):.0f}")
    for st, kn in STAGE_KERNEL.items():
        if kn in fetch:
            f = sum(fetch[kn]) / len(fetch[kn]) * sf
            wv = write.get(kn, [0.0])
            print(f"stage {st} {f:.6g} {sum(wv) / len(wv) * sw:.6g} {source_sha(st)}")


def pmc_table(csvs):
    """Per-kernel averages (per dispatch) of every counter in rocprofv3 --pmc
    CSV files, for the library's kernels; with the LDS counters, the share
    of LDS-active cycles stalled by bank conflicts."""
    import csv
    import re
    acc = {}
    for fn in csvs:
        for r in csv.DictReader(open(fn)):
            k = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "").replace("roix::", "")
            if not k.startswith("k_"):
                continue
            acc.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    for k in sorted(acc):
        cs = {c: sum(v) / len(v) for c, v in acc[k].items()}
        extra = ""
        if cs.get("SQ_LDS_IDX_ACTIVE"):
            extra = f" conflict_share={cs.get('SQ_LDS_BANK_CONFLICT', 0.0) / cs['SQ_LDS_IDX_ACTIVE']:.3f}"
        print(f"kernel {k.replace(' ', '')} " + " ".join(f"{c}={v:.4g}" for c, v in sorted(cs.items())) + extra)


def algorithmic_bytes(stage, N, s, n_codes, code_bytes, n_rows, nrows_all, W, p16):
    """Bytes a launch of `stage` must move at minimum (per call of the path).
    p16: the call took the one-pass flow with the 16-bit code proxy."""
    pb = 2 if p16 else 1                      # proxy bytes per voxel
    if stage == "range":
        return N * s
    if stage == "quant_hist":
        return N * s + N                      # read the volume, write the 1-byte bin proxy
    if stage == "quant_range16":
        return N * s + 2 * N                  # read the volume, write the 16-bit code proxy
    if stage == "mask_runs":
        return N * pb + nrows_all * W * 8     # read the proxy, write the row bitmask
    if stage == "emit":                       # read span voxels (proxy or values), write codes, row descriptors
        return n_codes * ((2 if p16 else s) + code_bytes) + n_rows * 32
    return None


def bench_decode(args):
    """The reverse process of the benchmark volume's extraction: decoded
    GB/s (float32 output bytes per second) and the roofline of the row
    kernel, which writes every voxel once and reads the span codes."""
    import torch

    import synth
    from paper_2602_15917_amd import roix
    dev = "cuda:0"
    w = synth.cylinder1024(n=args.n)
    x = torch.from_numpy(w.volume).to(dev)
    del w.volume
    crit = roix.Criterion(w.criterion.thr, 0.0, w.criterion.connectivity, w.criterion.keep, w.criterion.min_size)
    dims = roix.dims_of(x)
    ctx = roix.Context(0, roix.scratch_bytes(dims, roix.F32, crit))
    b = roix.bounds(dims, roix.F32, crit)
    out = roix.Outputs(dev, b["rows"], b["stream_bytes"], 1 << 22, 1 << 22)
    ctx.fused(x, w.eb_mode, w.eb_value, crit, out)
    torch.cuda.synchronize()
    e = out.collect()["einfo"]
    qi = out.collect()["qinfo"]
    dst = torch.empty_like(x)
    dinfo = torch.zeros(32, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        ctx.decode(out, dims, 0.0, dst, dinfo, stream)
    torch.cuda.synchronize()
    assert roix.decode_info(dinfo).status == 0
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        ctx.decode(out, dims, 0.0, dst, dinfo, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    N = x.numel()
    ctx.set_timing(True)
    for _ in range(args.steps):
        ctx.decode(out, dims, 0.0, dst, dinfo, stream)
    st = ctx.read_timing()
    ctx.set_timing(False)
    k_ms = st["decode"][0] / max(st["decode"][1], 1)
    c = int(qi.width_bits) // 8
    byts = N * 4 + int(e.n_codes) * c + 32 * int(e.n_rows) + 4 * int(e.n_outliers)
    ach = byts / (k_ms * 1e-3) / 1e9
    line = {
        "metric": "decoded GB/s (reverse process of the extraction, float32 output bytes)",
        "value": round(N * 4 / (ms * 1e-3) / 1e9, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"decode of the {w.name} extraction", "n_rows": int(e.n_rows),
                   "n_codes": int(e.n_codes), "n_outliers": int(e.n_outliers), "code_bits": int(qi.width_bits)},
        "roofline": {"bound": "hbm", "kernel": "decode_rows", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                     "alg_bytes_per_launch": int(byts), "avg_launch_ms": round(k_ms, 4)},
        "stages_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in st.items() if v[1]},
    }
    print(json.dumps(line))
    ctx.close()


def bench_background(args):
    """Background subtraction (M = I - B) of the benchmark volume put on a
    smooth calibration plane: GB/s of the subtraction with one plane for
    every z and with a reference volume; the whole path run on M after the
    subtraction (one step = subtraction + fused path); and the fused path
    with the subtraction folded in (roix_fused_background, same outputs)."""
    import torch

    import synth
    from paper_2602_15917_amd import roix
    dev = "cuda:0"
    w = synth.cylinder1024(n=args.n)
    nz, ny, nx = w.volume.shape
    x = torch.from_numpy(w.volume).to(dev)
    del w.volume
    yy, xx = torch.meshgrid(torch.arange(ny, device=dev, dtype=torch.float32),
                            torch.arange(nx, device=dev, dtype=torch.float32), indexing="ij")
    plane = (0.3 + 0.4 * xx / nx - 0.2 * ((xx - nx / 2) ** 2 + (yy - ny / 2) ** 2) / (nx * nx / 4))[None]
    plane = plane.contiguous()
    x.add_(plane)  # the image: object on its background
    crit = roix.Criterion(w.criterion.thr, 0.0, w.criterion.connectivity, w.criterion.keep, w.criterion.min_size)
    dims = roix.dims_of(x)
    ctx = roix.Context(0, roix.scratch_bytes(dims, roix.F32, crit))
    b = roix.bounds(dims, roix.F32, crit)
    out = roix.Outputs(dev, b["rows"], b["stream_bytes"], 1 << 22, 1 << 22)
    m = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    N = x.numel()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / args.steps

    def kernel_ms(fn):
        ctx.set_timing(True)
        for _ in range(args.steps):
            fn()
        st = ctx.read_timing()
        ctx.set_timing(False)
        return st["background"][0] / max(st["background"][1], 1), st

    sub_plane = lambda: ctx.background(x, plane, "subtract", m, stream)
    ms_plane = timed(sub_plane)
    k_plane, _ = kernel_ms(sub_plane)
    bytes_plane = N * 8 + plane.numel() * 4
    ref = plane.expand(nz, ny, nx).contiguous()
    sub_vol = lambda: ctx.background(x, ref, "subtract", m, stream)
    ms_vol = timed(sub_vol)
    k_vol, _ = kernel_ms(sub_vol)
    del ref
    bytes_vol = N * 12

    def step():
        ctx.background(x, plane, "subtract", m, stream)
        ctx.fused(m, w.eb_mode, w.eb_value, crit, out, stream)
    ms_step = timed(step)
    g = out.collect()
    assert g["qinfo"].status == 0 and g["sinfo"].status == 0 and g["einfo"].status == 0
    sep = (g["rows"].tobytes(), g["stream"].tobytes(), g["outliers"].tobytes())

    def step_fused():  # the subtraction folded into the path (M is not written)
        ctx.fused_background(x, plane, w.eb_mode, w.eb_value, crit, out, m, stream)
    ms_fused = timed(step_fused)
    _, st = kernel_ms(step_fused)
    g = out.collect()
    assert g["einfo"].status == 0
    assert (g["rows"].tobytes(), g["stream"].tobytes(), g["outliers"].tobytes()) == sep
    ach = bytes_plane / (k_plane * 1e-3) / 1e9
    line = {
        "metric": "background subtraction GB/s (float32 image in, float32 M = I - B out)",
        "value": round(N * 8 / (ms_plane * 1e-3) / 1e9, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_plane, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{w.name} on a calibration plane (offset, tilt, radial falloff)",
                   "reference": "one ny*nx plane for every z"},
        "roofline": {"bound": "hbm", "kernel": "background", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                     "alg_bytes_per_launch": int(bytes_plane), "avg_launch_ms": round(k_plane, 4)},
        "reference_volume": {"ms": round(ms_vol, 4), "kernel_ms": round(k_vol, 4),
                             "achieved_GBps": round(bytes_vol / (k_vol * 1e-3) / 1e9, 1),
                             "alg_bytes_per_launch": int(bytes_vol)},
        "subtract_then_path": {"ms_per_step": round(ms_step, 4),
                               "voxels_per_s": round(N / (ms_step * 1e-3), 1),
                               "n_kept_voxels": int(g["sinfo"].n_kept_voxels)},
        "fused_background_path": {"ms_per_step": round(ms_fused, 4),
                                  "voxels_per_s": round(N / (ms_fused * 1e-3), 1),
                                  "outputs_equal_subtract_then_path": True},
        "stages_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in st.items() if v[1]},
    }
    print(json.dumps(line))
    ctx.close()


def bench_absq(args):
    """The paper's absolute error-bounded quantisation (Sec. 4.2.3) of the
    benchmark volume's Eq. 1 normalised 8-bit pixel section (Sec. 4.1.2): the
    1024^3 cylinder is extracted, the section of its spans (514 688 000
    pixels) is made on the device (roix_section) and quantised.  Pixels per
    second of the quantiser at the stated tolerance (and at E = 1 and 5),
    the section pass beside it; both checked against the oracle's digests of
    the same section and of its quantisations; the oracle's sequential scan
    timed on the same section."""
    import numpy as np
    import torch

    import synth
    from paper_2602_15917_amd import roix
    dev = "cuda:0"
    w = synth.cylinder1024(n=args.n)
    name = "cylinder1024" if args.n == 1024 else None
    x = torch.from_numpy(w.volume).to(dev)
    del w.volume
    crit = roix.Criterion(w.criterion.thr, 0.0, w.criterion.connectivity, w.criterion.keep, w.criterion.min_size)
    dims = roix.dims_of(x)
    ctx = roix.Context(0, roix.scratch_bytes(dims, roix.F32, crit))
    b = roix.bounds(dims, roix.F32, crit)
    out = roix.Outputs(dev, b["rows"], b["stream_bytes"], 1 << 22, 1 << 22)
    stream = torch.cuda.current_stream()
    ctx.fused(x, w.eb_mode, w.eb_value, crit, out, stream)
    torch.cuda.synchronize()
    g = out.collect()
    m = int(g["einfo"].n_codes)
    code_bytes = int(g["qinfo"].width_bits) // 8
    sec = torch.empty(m + 16, dtype=torch.uint8, device=dev)
    sinfo = torch.zeros(16, dtype=torch.uint8, device=dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / args.steps

    ms_sec = timed(lambda: ctx.section(x, out, sec, sinfo, stream))
    si = roix.section_info(sinfo)
    assert (si.status, si.n_codes) == (0, m), (si.status, si.n_codes)
    del x
    px = sec[:m]
    gold = json.load(open(GOLDEN)).get(name) if name and os.path.exists(GOLDEN) else None
    parity = {"extraction": golden_parity(name, g) if name else "no oracle digest"}
    host_px = px.cpu().numpy()
    if gold and "section" in gold:
        parity["section"] = "bit-exact" if _sha(host_px) == gold["section"]["sha256"] else "DIFFERS"
    actx = roix.Context(0, roix.abs_quantize_scratch_bytes(m))
    q = torch.empty_like(px)
    info = torch.zeros(32, dtype=torch.uint8, device=dev)
    per_e = {}
    for e in (args.absq_e, 1.0, 5.0):
        if e in per_e:
            continue
        ms = timed(lambda: actx.abs_quantize(px, e, q, info, stream))
        i = roix.absq_info(info)
        per_e[e] = {"ms": round(ms, 4), "n_groups": int(i.n_groups), "rounds": int(i.rounds),
                    "finisher_chunks": int(i.finisher_chunks), "pixels_per_group": round(m / max(int(i.n_groups), 1), 3)}
        ga = (gold or {}).get("absq_on_section", {}).get(repr(float(e)))
        if ga:
            ok = int(i.status) == ga["status"] and int(i.n_groups) == ga["n_groups"] and \
                _sha(q.cpu().numpy()) == ga["sha256"]
            parity[f"abs_quantize E={e}"] = "bit-exact" if ok else "DIFFERS"
    main = per_e[args.absq_e]
    ms = main["ms"]
    cpu = None
    if args.cpu_planes != 0:
        import oracle
        t0 = time.time()
        oracle.abs_quantize(host_px, args.absq_e)
        dt = time.time() - t0
        cpu = {"value": round(m / dt / 1e9, 4), "unit": "Gpixel/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole {m}-pixel section, single-threaded C oracle, {dt:.1f} s"}
    byts = 2 * m
    sec_bytes = m * (code_bytes + 1)
    line = {
        "metric": "pixels quantised per second (absolute error-bounded, 8-bit pixel section)",
        "value": round(m / (ms * 1e-3) / 1e9, 3), "unit": "Gpixel/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"Eq. 1 normalised 8-bit section of the {w.name} extraction's spans",
                   "pixels": m, "E": args.absq_e},
        "roofline": {"bound": "hbm", "kernel": "abs_quantize (all passes)", "achieved": round(byts / (ms * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None, "alg_bytes_per_launch": byts},
        "section": {"ms": round(ms_sec, 4), "alg_bytes": sec_bytes, "code_bytes": code_bytes,
                    "achieved_GBps": round(sec_bytes / (ms_sec * 1e-3) / 1e9, 1),
                    "frac": round(sec_bytes / (ms_sec * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "by_tolerance": {str(k): v for k, v in per_e.items()},
        "parity": parity,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    actx.close()
    ctx.close()


def bench_huffman(args):
    """The lossless Huffman stage on the benchmark volume's code stream:
    encode and decode GB/s and the compression ratios it gives the ROI
    representation (volume bytes over row table + coded stream + outliers),
    and on the paper quantiser's output for the synthetic pixel section."""
    import torch

    import synth
    from paper_2602_15917_amd import roix
    dev = "cuda:0"
    w = synth.cylinder1024(n=args.n)
    x = torch.from_numpy(w.volume).to(dev)
    del w.volume
    crit = roix.Criterion(w.criterion.thr, 0.0, w.criterion.connectivity, w.criterion.keep, w.criterion.min_size)
    dims = roix.dims_of(x)
    ctx = roix.Context(0, roix.scratch_bytes(dims, roix.F32, crit))
    b = roix.bounds(dims, roix.F32, crit)
    out = roix.Outputs(dev, b["rows"], b["stream_bytes"], 1 << 22, 1 << 22)
    ctx.fused(x, w.eb_mode, w.eb_value, crit, out)
    torch.cuda.synchronize()
    vol_bytes = x.numel() * 4
    del x
    e = out.collect()["einfo"]
    q = out.collect()["qinfo"]
    n = int(e.n_codes) * (int(q.width_bits) // 8)
    s = out.stream[:n]
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(args.warmup):
            r = fn()
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            r = fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / args.steps, r

    ms_enc, (ln, off, pay, info, sub) = timed(lambda: ctx.huff_encode(s, stream=stream, with_sub=True))
    i = roix.huff_info(info)
    assert i.status == 0
    dst = torch.empty(n, dtype=torch.uint8, device=dev)
    # from every 256-byte sub-block's start (the index), and from the block starts alone
    ms_dec, (back, dinfo) = timed(lambda: ctx.huff_decode(ln, off, pay, i.payload_words, n, dst, stream, sub=sub))
    assert roix.huff_info(dinfo).status == 0 and torch.equal(back, s)
    dst.zero_()
    ms_dec_blk, (back, dinfo) = timed(lambda: ctx.huff_decode(ln, off, pay, i.payload_words, n, dst, stream))
    assert roix.huff_info(dinfo).status == 0 and torch.equal(back, s)
    roi_plain = 32 * int(e.n_rows) + n + 4 * int(e.n_outliers)
    roi_huff = 32 * int(e.n_rows) + int(i.compressed_bytes) + 4 * int(e.n_outliers)
    # the paper quantiser's output on the synthetic pixel section, E = 2
    m = synth.PIXEL_SECTION_FULL if args.n == 1024 else int(e.n_codes)
    px = torch.from_numpy(synth.pixel_section_u8(m)).to(dev)
    qx, _ = ctx_absq(roix, px, 2.0)
    _, _, _, qinfo = ctx.huff_encode(qx)
    torch.cuda.synchronize()
    qi = roix.huff_info(qinfo)
    cpu = None
    if args.cpu_planes != 0:
        import oracle
        k = min(n, 64 << 20)
        sample = s[:k].cpu().numpy()
        t0 = time.time()
        oracle.huff_encode(sample)
        dt = time.time() - t0
        cpu = {"value": round(k / dt / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"the first {k} bytes of the same stream, single-threaded C oracle, {dt:.1f} s"}
    line = {
        "metric": "Huffman encode GB/s of the packed code stream (input bytes)",
        "value": round(n / (ms_enc * 1e-3) / 1e9, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_enc, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"code stream of the {w.name} extraction", "stream_bytes": n,
                   "code_bits": int(q.width_bits)},
        "roofline": {"bound": "hbm", "kernel": "huff_encode (all passes)",
                     "achieved": round((n + 4 * int(i.payload_words)) / (ms_enc * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round((n + 4 * int(i.payload_words)) / (ms_enc * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None, "alg_bytes_per_launch": n + 4 * int(i.payload_words)},
        "decode": {"ms": round(ms_dec, 4), "GBps_out": round(n / (ms_dec * 1e-3) / 1e9, 2),
                   "from": "every 256-byte sub-block's start (16 lanes per block)",
                   "frac": round((n + 4 * int(i.payload_words)) / (ms_dec * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "block_lanes_ms": round(ms_dec_blk, 4)},
        "compression": {"stream_ratio": round(n / int(i.compressed_bytes), 4), "max_code_bits": int(i.max_len),
                        "roi_ratio_plain": round(vol_bytes / roi_plain, 3),
                        "roi_ratio_huffman": round(vol_bytes / roi_huff, 3),
                        "pixel_section_e2_ratio": round(m / int(qi.compressed_bytes), 3)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    ctx.close()


def ctx_absq(roix, px, e):
    c = roix.Context(0, roix.abs_quantize_scratch_bytes(px.numel()))
    qx, info = c.abs_quantize(px, e)
    import torch
    torch.cuda.synchronize()
    c.close()
    return qx, info


# ------------------------------------------------------------ extra sections
# The default run reports, beside the headline plain workload, every other
# configuration of the metric: the 128^3 volume (launch-bound), the 8 GB
# uint16 stack, the 64-volume batch and the served slab stream.  Each is
# checked for parity before its figure is reported: against the digests the
# oracle wrote (tests/golden/digests.json) for the single volumes, against
# per-volume plain calls for the batched and served forms.

GOLDEN = os.path.join(ROOT, "tests", "golden", "digests.json")


def _sha(a):
    import hashlib

    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def golden_parity(name, g):
    """Compare collected outputs with the oracle's digests of workload `name`:
    'bit-exact' or the list of fields that differ."""
    import numpy as np
    gold = json.load(open(GOLDEN)).get(name) if os.path.exists(GOLDEN) else None
    if gold is None:
        return "no oracle digest"
    q, s, e = g["qinfo"], g["sinfo"], g["einfo"]
    bad = []
    if (q.status, s.status, e.status) != (0, 0, 0):
        bad.append("status")
    for f in ("qmin", "qmax", "K", "width_bits", "esc"):
        if getattr(q, f) != gold["quant"][f]:
            bad.append(f)
    for f in ("xmin", "xmax", "eb32", "w", "r"):
        if np.float32(getattr(q, f)) != np.float32(gold["quant"][f]):
            bad.append(f)
    for f in ("otsu_bin", "q_thr", "flags", "n_mask", "n_components", "n_kept", "n_kept_voxels"):
        if getattr(s, f) != gold["seg"][f]:
            bad.append(f)
    if list(s.bbox) != gold["seg"]["bbox"]:
        bad.append("bbox")
    if _sha(np.frombuffer(bytes(s.hist), np.uint64)) != gold["seg"]["hist_sha256"]:
        bad.append("hist")
    for f in ("n_rows", "n_codes", "n_outliers", "stream_bytes"):
        if getattr(e, f) != gold["extract"][f]:
            bad.append(f)
    for k in ("rows", "stream", "outliers", "comps"):
        if _sha(g[k]) != gold["sha256"][k]:
            bad.append(k)
    return "bit-exact with the oracle's digests" if not bad else {"differs": bad}


def b_alg(N, s, n_codes, code_bytes, n_rows):
    """The method's byte model: two input reads, a 1-byte proxy written and
    read, the span voxels re-read, the codes and the row table written."""
    return N * (2 * s + 2) + n_codes * (s + code_bytes) + 32 * n_rows


def plain_single(name, w, steps, warmup, dev="cuda:0"):
    """Time the plain fused path on one workload (device-resident input) and
    check it against the oracle's digests."""
    import torch

    from paper_2602_15917_amd import roix
    crit = roix.Criterion(w.criterion.thr, 0.0, w.criterion.connectivity, w.criterion.keep, w.criterion.min_size)
    x = torch.from_numpy(w.volume).to(dev)
    s = w.volume.itemsize
    w.volume = None
    dims = roix.dims_of(x)
    dt = roix.dtype_of(x)
    ctx = roix.Context(0, roix.scratch_bytes(dims, dt, crit))
    b = roix.bounds(dims, dt, crit)
    out = roix.Outputs(dev, b["rows"], b["stream_bytes"], min(b["outliers"], 1 << 26), 1 << 20)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        ctx.fused(x, w.eb_mode, w.eb_value, crit, out, stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        ctx.fused(x, w.eb_mode, w.eb_value, crit, out, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    g = out.collect()
    parity = golden_parity(name, g)
    e, qi = g["einfo"], g["qinfo"]
    N = x.numel()
    ba = b_alg(N, s, int(e.n_codes), int(qi.width_bits) // 8, int(e.n_rows))
    res = {"workload": w.name, "ms": round(ms, 4), "steps": steps, "GBps": round(N * s / (ms * 1e-3) / 1e9, 2),
           "alg_bytes": int(ba), "frac": round(ba / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "n_codes": int(e.n_codes), "reduction": round(N / max(int(e.n_codes), 1), 3), "parity": parity}
    del x, out
    ctx.close()
    torch.cuda.empty_cache()
    return res


def section_c0(args):
    """128^3 float32 ellipsoids (ABS 1e-3, Otsu, 6-connectivity, components
    of 64 voxels or more): launch-bound; 100 timed calls."""
    import synth
    w = synth.ellipsoids128()
    r = plain_single("ellipsoids128", w, steps=100, warmup=5)
    log(f"c0 {r['workload']}: {r['ms']:.4f} ms, {r['GBps']} GB/s, parity {r['parity']}")
    return r


def section_c2(args):
    """2048 x 2048 x 1024 uint16 stack (REL 1e-4, Otsu, 26-connectivity,
    largest component): 8.6 GB, 5 timed calls."""
    import synth
    t = time.time()
    w = synth.rings2048()
    log(f"c2 generated in {time.time() - t:.1f}s")
    r = plain_single("rings2048", w, steps=5, warmup=2)
    log(f"c2 {r['workload']}: {r['ms']:.3f} ms, {r['GBps']} GB/s, frac {r['frac']}, parity {r['parity']}")
    return r


def device_sections(out):
    """Info structs (host bytes) and output sections trimmed to their counts,
    left on the device."""
    import torch

    from paper_2602_15917_amd import roix
    q = bytes(out.qinfo.cpu().numpy().tobytes())
    s = bytes(out.sinfo.cpu().numpy().tobytes())
    e = bytes(out.einfo.cpu().numpy().tobytes())
    ei = roix.ExtractInfo.from_buffer_copy(e)
    si = roix.SegInfo.from_buffer_copy(s)
    qi = roix.QuantInfo.from_buffer_copy(q)
    rows_cap, stream_cap, outl_cap, comps_cap = out.caps
    nr, nb = min(int(ei.n_rows), rows_cap), min(int(ei.stream_bytes), stream_cap)
    no, nc = min(int(ei.n_outliers), outl_cap), min(int(si.n_components), comps_cap)
    return {"info": (q, s, e), "status": (int(qi.status), int(si.status), int(ei.status)),
            "n_codes": int(ei.n_codes), "n_rows": int(ei.n_rows), "code_bytes": int(qi.width_bits) // 8,
            "sec": (out.rows[: nr * roix.ROW_BYTES], out.stream[:nb], out.outliers[:no].view(torch.int32),
                    out.comps[: nc * roix.COMP_BYTES])}


def sections_equal(a, b):
    import torch
    return a["info"] == b["info"] and all(x.numel() == y.numel() and torch.equal(x, y)
                                          for x, y in zip(a["sec"], b["sec"]))


def section_batched(args):
    """The 64-volume batch (float32, sides U{64..512} per axis, 1-8
    ellipsoids, eb from {1e-3, 1e-4, 1e-5}, Otsu, 6-connectivity, components
    of 64 voxels or more) in one batched call, against the same volumes run
    one plain call after another; every output of the batch is compared with
    its plain call on the device."""
    import torch

    import synth
    from paper_2602_15917_amd import roix

    dev = "cuda:0"
    t0 = time.time()
    items, refs, need = [], [], 0
    total = 0
    for j in range(args.batch_volumes):
        w = synth.batch_volume(j)
        crit = roix.Criterion(w.criterion.thr, 0.0, w.criterion.connectivity, w.criterion.keep, w.criterion.min_size)
        t = torch.from_numpy(w.volume).to(dev)
        total += w.volume.nbytes
        dims = roix.dims_of(t)
        b = roix.bounds(dims, roix.F32, crit)
        caps = (b["rows"], b["stream_bytes"], min(b["outliers"], 1 << 24), min(b["components"], 1 << 20))
        items.append((t, w.eb_mode, w.eb_value, crit, roix.Outputs(dev, *caps)))
        refs.append(roix.Outputs(dev, *caps))
        need += roix.scratch_bytes(dims, roix.F32, crit)  # every volume's layout at once
    log(f"batched: generated {len(items)} volumes, {total / 1e9:.2f} GB, in {time.time() - t0:.1f}s")
    ctx = roix.Context(0, need + (64 << 20))
    ctx.set_param("batch_group", args.batch_group)
    ctx.set_param("batch_graph", args.batch_graph)
    ctx.set_param("batch_lanes", args.batch_lanes)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def plain_pass(outs):
        for (t, ebm, ebv, crit, _), o in zip(items, outs):
            ctx.fused(t, ebm, ebv, crit, o, stream)

    def batch_pass():
        ctx.fused_batch(items, stream)

    # parity first: the batch against one plain call per volume
    plain_pass(refs)
    batch_pass()
    torch.cuda.synchronize()
    ba_total, equal, bad = 0, True, []
    for j, (it, ref) in enumerate(zip(items, refs)):
        a, b = device_sections(it[4]), device_sections(ref)
        if b["status"] != (0, 0, 0):
            bad.append(j)
        equal = equal and sections_equal(a, b)
        ba_total += b_alg(it[0].numel(), 4, b["n_codes"], b["code_bytes"], b["n_rows"])
    res = {}
    for name, fn in (("plain", lambda: plain_pass(refs)), ("batched", batch_pass)):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.batch_steps):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        res[name] = ev0.elapsed_time(ev1) / args.batch_steps
    # and once more after the timed repeats
    equal = equal and all(sections_equal(device_sections(it[4]), device_sections(r)) for it, r in zip(items, refs))
    out = {"workload": f"{len(items)} f32 volumes, sides U{{64..512}}, 1-8 ellipsoids, eb in {{1e-3,1e-4,1e-5}}, "
                       f"Otsu, 6-connectivity, components >= 64",
           "input_bytes": total, "ms": round(res["batched"], 4), "steps": args.batch_steps,
           "GBps": round(total / (res["batched"] * 1e-3) / 1e9, 2),
           "alg_bytes": int(ba_total), "frac": round(ba_total / (res["batched"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "plain_sequential_ms": round(res["plain"], 4),
           "plain_sequential_GBps": round(total / (res["plain"] * 1e-3) / 1e9, 2),
           "batched_over_plain": round(res["plain"] / res["batched"], 3),
           "parity": "equal to per-volume plain calls" if equal and not bad else
                     {"equal": bool(equal), "nonzero_status": bad}}
    log(f"batched: {out['ms']} ms ({out['GBps']} GB/s, frac {out['frac']}) vs plain {out['plain_sequential_ms']} ms; "
        f"parity {out['parity']}")
    del items, refs
    ctx.close()
    torch.cuda.empty_cache()
    return out


def section_served(args):
    """The served slab stream: `served_streams` uint16 2048 x 2048 volumes
    of `served_nz` planes (ring-artefact cylinders; ABS bound = 1e-4 x the
    range of a calibration volume; FIXED threshold 6400; 26-connectivity;
    largest component) arriving in 32-plane slabs, interleaved with
    `served_cubes` float32 cubes of side U{128..512} sent whole (ABS 1e-3,
    Otsu, reduced at close), Poisson arrivals at each rate, an HBM budget.

    Inputs: one stream's planes are generated once into pinned memory; stream
    k sends them rotated by 4k slabs (the cylinder and rings are constant
    along z and the noise independent per plane, so each rotation is a volume
    of the same make-up); the cubes are 16 generated ones, reused in turn.
    Latency of a request = completion on the device - its scheduled arrival
    (queueing, waits for admission, pinned H2D and compute included).  At the
    first rate the whole trace runs and every volume's output is compared
    with a plain call on the assembled volume; the other rates replay the
    trace for at most `served_seconds` each."""
    import collections

    import numpy as np
    import torch

    import synth
    from paper_2602_15917_amd import roix

    dev = "cuda:0"
    SLAB, NXY = 32, 2048
    nz = args.served_nz
    nslab = nz // SLAB
    t0 = time.time()
    calib = synth.served_calibration(nz=8)
    eb_s = 1e-4 * (float(calib.max()) - float(calib.min()))
    del calib
    crit_s = roix.Criterion("fixed", 6400.0, 26, "largest", 1)
    pool = torch.empty((nz, NXY, NXY), dtype=torch.uint16, pin_memory=True)
    pnp = pool.numpy()
    for j in range(nslab):
        synth.served_slab(0, j * SLAB, nz=SLAB, out=pnp[j * SLAB:(j + 1) * SLAB])
    cube_pool = []
    for k in range(min(16, args.served_cubes)):
        w = synth.served_cube(k)
        c = w.criterion
        cube_pool.append((torch.from_numpy(w.volume).pin_memory(), w.eb_mode, w.eb_value,
                          roix.Criterion(c.thr, c.fixed_value, c.connectivity, c.keep, c.min_size)))
    n_streams, n_cubes = args.served_streams, args.served_cubes
    slab_bytes = SLAB * NXY * NXY * 2
    total = n_streams * nz * NXY * NXY * 2 + sum(cube_pool[i % len(cube_pool)][0].numel() * 4 for i in range(n_cubes))
    log(f"served: {n_streams} u16 streams of {nz} planes, {n_cubes} f32 cubes, {total / 1e9:.1f} GB, eb {eb_s:.4g}; "
        f"inputs generated in {time.time() - t0:.1f}s")

    def slab_of(k, j):  # pinned view of stream k's slab j
        p = (j + 4 * k) % nslab
        return pool[p * SLAB:(p + 1) * SLAB]

    Nst = nz * NXY * NXY
    s_caps = (nz * NXY, int(0.45 * Nst) * 2 + 256, 1 << 24, 1 << 20)
    outs_s = [roix.Outputs(dev, *s_caps) for _ in range(n_streams)]
    outs_c = []
    for i in range(n_cubes):
        t = cube_pool[i % len(cube_pool)][0]
        b = roix.bounds(roix.dims_of(t), roix.F32, cube_pool[i % len(cube_pool)][3])
        outs_c.append(roix.Outputs(dev, b["rows"], t.numel() * 2 + 256, 1 << 22, min(b["components"], 1 << 22)))
    # the trace: every slab of every stream (in order) and every cube, interleaved at random
    rng = np.random.default_rng(3000)
    kinds = [("s", k) for k in range(n_streams) for _ in range(nslab)] + [("c", i) for i in range(n_cubes)]
    events, nexts = [], [0] * n_streams
    for i in rng.permutation(len(kinds)):
        kind, k = kinds[i]
        if kind == "s":
            events.append(("s", k, nexts[k]))
            nexts[k] += 1
        else:
            events.append(("c", k, 0))
    ctx = roix.Context(0, 1 << 20)

    def replay(rate, max_seconds):
        srv = roix.Server(ctx, int(args.served_budget_gib * (1 << 30)))
        # the streams keep their rows' extents in a store of 40 % of their voxels
        # (the cylinder covers 30 % of the field of view)
        srv.set_param("store_permille", 400)
        t_base = time.perf_counter()
        gaps = rng.exponential(1.0 / rate, size=len(events)) if rate > 0 else np.zeros(len(events))
        arrivals = np.cumsum(gaps) * 1e3 + 5.0  # ms on the server clock
        ev = [(e, a) for e, a in zip(events, arrivals) if max_seconds is None or a <= max_seconds * 1e3]
        vid = {}          # ("s", k) or ("c", i) -> volume id once admitted
        pending = collections.deque()
        recs = []         # (request id, arrival ms, kind)
        closed = set()

        def try_submit(e, arr):
            kind, k, j = e
            key = (kind, k)
            if key not in vid:
                # run capacity per row: a cylinder chord is one run; a cube
                # whose Otsu split falls in the noise has many runs per row
                if kind == "s":
                    shape, dt, ebm, ebv, crit, out = (nz, NXY, NXY), roix.U16, "abs", eb_s, crit_s, outs_s[k]
                    srv.set_param("runs_per_row", 4)
                else:
                    c = cube_pool[k % len(cube_pool)]
                    shape, dt, ebm, ebv, crit, out = tuple(c[0].shape), roix.F32, c[1], c[2], c[3], outs_c[k]
                    srv.set_param("runs_per_row", 256)
                try:
                    vid[key] = srv.open(shape, dt, ebm, ebv, crit, out)
                except roix.RoixError as err:
                    if err.status != roix.EBUSY:
                        raise
                    return False
            v = vid[key]
            if kind == "s":
                recs.append((srv.submit(v, j * SLAB, slab_of(k, j)), arr, "slab"))
                if j == nslab - 1:
                    recs.append((srv.close(v), arr, "stream_close"))
                    closed.add(key)
            else:
                srv.submit(v, 0, cube_pool[k % len(cube_pool)][0])
                recs.append((srv.close(v), arr, "cube"))
                closed.add(key)
            return True

        def drain():
            blocked = set()
            for _ in range(len(pending)):
                e, arr = pending.popleft()
                key = (e[0], e[1])
                if key in blocked or not try_submit(e, arr):
                    blocked.add(key)
                    pending.append((e, arr))

        for e, arr in ev:
            now = (time.perf_counter() - t_base) * 1e3
            if arr > now:
                time.sleep((arr - now) * 1e-3)
            pending.append((e, arr))
            drain()
        # the whole trace waits for every admission; a replay cut short leaves
        # what still waits unserved (its streams never close)
        t_end = time.perf_counter() + 120.0
        while pending and max_seconds is None and time.perf_counter() < t_end:
            time.sleep(0.0005)
            drain()
        unserved = len(pending)
        lat = {"slab": [], "stream_close": [], "cube": []}
        last = 0.0
        for rid, arr, kind in recs:
            r = srv.wait(rid)
            if r is None or r.status != 0:
                raise RuntimeError(f"served request {rid} failed")
            lat[kind].append(r.done_ms - arr)
            last = max(last, r.done_ms)
        for key, v in vid.items():  # a replay cut short leaves streams open
            if key not in closed:
                srv.abort(v)
        st = srv.stats()
        srv.close_server()
        torch.cuda.synchronize()
        span = max(last - float(ev[0][1]), 1e-3)
        moved = len(lat["slab"]) * slab_bytes + sum(cube_pool[e[1] % len(cube_pool)][0].numel() * 4
                                                    for e, _ in ev if e[0] == "c")
        q = lambda v, p: round(float(np.percentile(v, p)), 3) if v else None
        return {"rate_per_s": rate, "requests": len(recs), "slab_requests": len(lat["slab"]), "unserved": unserved,
                "p99_from_100_or_more": len(lat["slab"]) >= 100,
                "trace_seconds": round(float(ev[-1][1]) * 1e-3, 1),
                "slab_p50_ms": q(lat["slab"], 50), "slab_p99_ms": q(lat["slab"], 99),
                "slab_max_ms": q(lat["slab"], 100), "stream_close_p50_ms": q(lat["stream_close"], 50),
                "cube_p50_ms": q(lat["cube"], 50), "cube_p99_ms": q(lat["cube"], 99),
                "GBps": round(moved / (span * 1e-3) / 1e9, 2), "refused_opens": int(st.volumes_refused)}

    rates = [float(r) for r in args.served_rates.split(",") if r]
    res = {}
    parity, host_plain_s = None, 0.0
    for i, rate in enumerate(rates):
        # the first rate runs the whole trace; the others run long enough for
        # about 200 slab requests (about 80 % of the events are slabs), at
        # least served_seconds and at most served_max_seconds
        secs = max(args.served_seconds, min(args.served_max_seconds, 275.0 / rate)) if rate > 0 else None
        r = replay(rate, None if i == 0 else secs)
        log(f"served rate {rate}/s: {r['slab_requests']} slabs, p50 {r['slab_p50_ms']} ms p99 {r['slab_p99_ms']} ms, "
            f"cube p50 {r['cube_p50_ms']} ms, {r['GBps']} GB/s")
        res[str(rate)] = r
        if i == 0:  # every volume of the whole trace against its plain call
            pctx = roix.Context(0, 12 << 30)
            ok, bad, host_plain_s = True, [], 0.0
            for k in range(n_streams):
                # also the host-resident plain comparator: pinned H2D of the
                # stream, then one plain call
                ref = roix.Outputs(dev, *s_caps)
                torch.cuda.synchronize()
                th = time.perf_counter()
                vol = torch.cat([slab_of(k, j).to(dev, non_blocking=True) for j in range(nslab)])
                pctx.fused(vol, "abs", eb_s, crit_s, ref)
                torch.cuda.synchronize()
                host_plain_s += time.perf_counter() - th
                a, b = device_sections(outs_s[k]), device_sections(ref)
                if b["status"] != (0, 0, 0):
                    bad.append(("stream", k, b["status"]))
                ok = ok and sections_equal(a, b)
                del vol, ref
            crefs = {}
            for i2 in range(n_cubes):
                c = cube_pool[i2 % len(cube_pool)]
                if i2 % len(cube_pool) not in crefs:
                    ref = roix.Outputs(dev, *outs_c[i2].caps)
                    pctx.fused(c[0].to(dev), c[1], c[2], c[3], ref)
                    torch.cuda.synchronize()
                    crefs[i2 % len(cube_pool)] = device_sections(ref)
                a, b = device_sections(outs_c[i2]), crefs[i2 % len(cube_pool)]
                if b["status"] != (0, 0, 0):
                    bad.append(("cube", i2, b["status"]))
                ok = ok and sections_equal(a, b)
            parity = "equal to plain calls on the assembled volumes" if ok and not bad else {"equal": ok, "bad": bad}
            log(f"served parity: {parity}")
            del crefs
            pctx.close()
            torch.cuda.empty_cache()
    cap = replay(0.0, None)  # closed loop: every request at once
    log(f"served closed loop: {cap['GBps']} GB/s, slab p99 {cap['slab_p99_ms']} ms")
    out = {"workload": f"{n_streams} u16 streams 2048x2048x{nz} in {SLAB}-plane slabs (ABS eb {eb_s:.4g}, FIXED 6400, "
                       f"26-conn, largest) + {n_cubes} f32 cubes U{{128..512}} (Otsu), HBM budget "
                       f"{args.served_budget_gib:g} GiB",
           "input_bytes": int(total), "rates": res, "closed_loop": cap, "parity": parity,
           "host_resident_plain_GBps": round(n_streams * Nst * 2 / max(host_plain_s, 1e-9) / 1e9, 2)}
    ctx.close()
    del pool, cube_pool, outs_s, outs_c
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024, help="volume side (1024 = the benchmark workload)")
    ap.add_argument("--cpu-planes", type=int, default=256, help="z-planes of the CPU-oracle sample (0 = skip)")
    ap.add_argument("--no-stage-timing", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain device copy of 1 GiB (the counter calibration for traffic)")
    ap.add_argument("--pmc-table", nargs="+", metavar="COUNTER_CSV",
                    help="print per-kernel averages of the counters in rocprofv3 --pmc CSV files and exit")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "KERNEL_STATS_CSV"),
                    help="summarise rocprofv3 counter runs of this script and exit")
    ap.add_argument("--workload", choices=["plain", "batched", "served", "decode", "background", "absq", "huffman"], default="plain",
                    help="plain: the 1024^3 volume (default); batched: 64 uneven volumes in one graph launch; "
                         "served: open-loop slab-stream trace with p50/p99 latency; decode: the reverse "
                         "process of the 1024^3 volume's extraction; background: subtraction of a "
                         "calibration plane or volume, then the path on the result; absq: the paper's "
                         "absolute error-bounded quantisation of an 8-bit pixel section; huffman: the "
                         "lossless stage on the code stream, with compression ratios")
    ap.add_argument("--absq-e", type=float, default=2.0, help="tolerance of the absq workload")
    ap.add_argument("--autotune", action="store_true",
                    help="plain and batched workloads: tune the launch parameters on the volume(s) before timing")
    ap.add_argument("--thr", choices=["otsu", "multi3", "multi4", "otsu_slice"], default=None,
                    help="plain workload: threshold mode instead of the workload's two-class Otsu")
    ap.add_argument("--two-pass", action="store_true",
                    help="plain workload: force the two-pass flow (range, then quantise + 1-byte bin proxy)")
    ap.add_argument("--sections", default="c0,c2,batched,served",
                    help="plain workload: the other configurations reported in the same line "
                         "(comma list of c0, c2, batched, served; 'none' for the headline alone)")
    ap.add_argument("--served-streams", type=int, default=8, help="uint16 2048x2048 streams of the served trace")
    ap.add_argument("--served-nz", type=int, default=1024, help="planes per served stream (slabs of 32)")
    ap.add_argument("--served-cubes", type=int, default=64, help="float32 cubes interleaved in the served trace")
    ap.add_argument("--served-rates", default="20,10,5,1",
                    help="Poisson arrival rates (requests/s); the first replays the whole trace and is checked "
                         "against plain calls")
    ap.add_argument("--served-seconds", type=float, default=30.0,
                    help="least trace seconds replayed at every rate after the first")
    ap.add_argument("--served-max-seconds", type=float, default=58.0,
                    help="most trace seconds replayed at a rate (a rate runs for about 200 slab requests)")
    ap.add_argument("--served-budget-gib", type=float, default=64.0)
    ap.add_argument("--batch-steps", type=int, default=10, help="timed repeats of the batch and of the plain calls")
    ap.add_argument("--batch-volumes", type=int, default=64)
    ap.add_argument("--batch-group", type=int, default=0,
                    help="volumes per launch group of the batched path (0: as many as the arena holds)")
    ap.add_argument("--batch-lanes", type=int, default=2, choices=[1, 2, 3, 4],
                    help="concurrent launch sequences of the batched call")
    ap.add_argument("--batch-graph", type=int, default=0, choices=[0, 1],
                    help="1: capture the batch into a HIP graph and replay it; 0: launch eagerly")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.pmc_table:
        pmc_table(args.pmc_table)
        return
    if args.workload in ("batched", "served"):
        r = section_batched(args) if args.workload == "batched" else section_served(args)
        print(json.dumps({"metric": METRIC, "workload": args.workload, args.workload: r}))
        return
    if args.workload == "background":
        return bench_background(args)
    if args.workload == "absq":
        return bench_absq(args)
    if args.workload == "huffman":
        return bench_huffman(args)
    if args.workload == "decode":
        return bench_decode(args)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the reduction path has no multi-GPU "
              f"form in this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2602_15917_amd import roix

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    t0 = time.time()
    w = synth.cylinder1024(n=args.n)
    vol = w.volume
    nz, ny, nx = vol.shape
    N, s = vol.size, vol.itemsize
    log(f"generated {w.name} in {time.time() - t0:.1f}s")
    x = torch.from_numpy(vol).to(dev)
    if args.thr:  # another threshold mode on the same workload
        w.criterion.thr = args.thr
    crit = roix.Criterion(w.criterion.thr, 0.0, w.criterion.connectivity, w.criterion.keep, w.criterion.min_size)
    dims = roix.dims_of(x)
    ctx = roix.Context(0, roix.scratch_bytes(dims, roix.F32, crit))
    b = roix.bounds(dims, roix.F32, crit)
    out = roix.Outputs(dev, b["rows"], b["stream_bytes"], b["outliers"], 1 << 22,
                       nz_slices=nz if crit.thr == "otsu_slice" else 0)
    stream = torch.cuda.current_stream()
    if args.two_pass:
        ctx.set_param("fused16_min_voxels", 1 << 40)

    def step():
        ctx.fused(x, w.eb_mode, w.eb_value, crit, out, stream)

    tuning = None
    if args.autotune:  # pick the launch parameters on this volume first
        tr = ctx.autotune(x, w.eb_mode, w.eb_value, crit, out, reps=3, stream=stream)
        tuning = {"default_ms": round(tr.default_ms, 4), "best_ms": round(tr.best_ms, 4), "runs": int(tr.n_timed),
                  "params": dict(zip(roix.TUNE_PARAMS, [int(v) for v in tr.params]))}
        log(f"autotune: {tuning}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    res = out.collect()
    e, si, qi = res["einfo"], res["sinfo"], res["qinfo"]
    if e.status != 0 or si.status != 0 or qi.status != 0:
        log(f"status q={qi.status} s={si.status} e={e.status}")
        sys.exit(1)
    log(f"rows {e.n_rows} codes {e.n_codes} outliers {e.n_outliers} components {si.n_components} "
        f"width {qi.width_bits}")

    # timed region: K steps between two events on the launch stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = ev0.elapsed_time(ev1) / args.steps
    gbs = N * s / (ms * 1e-3) / 1e9
    log(f"{ms:.3f} ms/step, {gbs:.1f} GB/s input (wall {t_wall / args.steps * 1e3:.3f} ms/step)")

    # per-kernel durations: the same steps with events around every kernel
    stages = {}
    if not args.no_stage_timing:
        ctx.set_timing(True)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        stages = ctx.read_timing()
        ctx.set_timing(False)
    code_bytes = qi.width_bits // 8
    nrows_all = ny * nz
    W = (nx + 63) // 64
    roof = None
    if stages:
        per = {k: (v[0] / v[1] if v[1] else 0.0, v[1]) for k, v in stages.items()}
        for k, (avg, cnt) in sorted(per.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
            if cnt:
                log(f"  stage {k:12s} {avg * 1e3:9.1f} us x {cnt // args.steps}")
        p16 = per.get("quant_range16", (0.0, 0))[1] > 0
        dom = max((k for k in per if per[k][1] and algorithmic_bytes(k, N, s, e.n_codes, code_bytes, e.n_rows,
                                                                      nrows_all, W, p16)),
                  key=lambda k: per[k][0])
        avg_ms = per[dom][0]
        byts = algorithmic_bytes(dom, N, s, e.n_codes, code_bytes, e.n_rows, nrows_all, W, p16)
        ach = byts / (avg_ms * 1e-3) / 1e9
        tr = measured_traffic(dom)
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": (round(tr[0] + tr[1]) if tr else None),
                "traffic_fetch_write": ([round(tr[0]), round(tr[1])] if tr else None),
                "alg_bytes_per_launch": int(byts), "avg_launch_ms": round(avg_ms, 4)}
    # whole-path byte model of the method's stages: two input reads (range,
    # quantise + histogram), 1-byte proxy written and read, span voxels
    # re-read, codes written, row table written.  design_bytes: what the flow
    # this call took moves at minimum (one input read, the 16-bit proxy written
    # and read twice for the mask and the span codes, codes and rows written).
    b_alg = N * (2 * s + 2) + e.n_codes * (s + code_bytes) + 32 * e.n_rows
    path = {"alg_bytes": int(b_alg), "achieved": round(b_alg / (ms * 1e-3) / 1e9, 1),
            "frac": round(b_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if stages and per.get("quant_range16", (0.0, 0))[1] > 0:
        b_des = N * (s + 2) + (2 * N + nrows_all * W * 8) + e.n_codes * (2 + code_bytes) + 32 * e.n_rows
        path.update({"design_bytes": int(b_des), "design_frac": round(b_des / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})

    # a measured read-only stream of the same size: the range kernel of the
    # two-pass flow (one read of the N*s input bytes, one atomic per
    # workgroup), timed by the library's stage events on a few steps with that
    # flow forced, outside the timed region
    if stages:
        keep16 = ctx.get_param("fused16_min_voxels")
        ctx.set_param("fused16_min_voxels", 1 << 40)
        ctx.set_timing(True)
        for _ in range(3):
            step()
        torch.cuda.synchronize()
        st2 = ctx.read_timing()
        ctx.set_timing(False)
        ctx.set_param("fused16_min_voxels", keep16)
        r_ms, r_n = st2.get("range", (0.0, 0))
        if r_n:
            ro_gbs = N * s / (r_ms / r_n * 1e-3) / 1e9
            path.update({"read_only_kernel": "k_range (two-pass flow)", "read_only_GBps": round(ro_gbs, 1),
                         "frac_vs_read_only": round(path["achieved"] / ro_gbs, 4)})

    if args.calibrate_copy:
        a = torch.empty(CALIB_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
        bcp = torch.empty_like(a)
        for _ in range(3):
            bcp.copy_(a)
        torch.cuda.synchronize()
        del a, bcp

    cpu = None
    if args.cpu_planes > 0:
        import oracle
        k = min(args.cpu_planes, nz)
        sample = np.ascontiguousarray(vol[:k])
        c = w.criterion
        log(f"CPU oracle on {k} of {nz} z-planes ...")
        # pinned to one core of those this process may use, for the timing only
        allowed = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else []
        pin = allowed[0] if allowed else None
        if pin is not None:
            os.sched_setaffinity(0, {pin})
        try:
            t = time.perf_counter()
            r = oracle.fused(sample, w.eb_mode, w.eb_value, c.thr, c.fixed_value, c.connectivity, c.keep,
                             c.min_size, comps_cap=1 << 20)
            dt = time.perf_counter() - t
        finally:
            if pin is not None:
                os.sched_setaffinity(0, set(allowed))
        assert r["status"] == 0
        try:
            model = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
            model = [l.split(":", 1)[1].strip() for l in model.splitlines() if l.startswith("Model name")][0]
        except Exception:
            model = "unknown"
        whole = ""
        gold = json.load(open(GOLDEN)).get("cylinder1024") if os.path.exists(GOLDEN) and args.n == 1024 else None
        if gold and gold.get("oracle_seconds"):
            whole = (f"; the whole volume through the same oracle took {gold['oracle_seconds']} s on the build host "
                     f"({vol.nbytes / gold['oracle_seconds'] / 1e9:.3f} GB/s, tests/golden/make_digests.py)")
        cpu = {"value": round(sample.nbytes / dt / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"first {k} of {nz} z-planes of the same volume ({sample.nbytes / 1e9:.2f} GB), "
                         f"single-threaded C oracle pinned to cpu {pin} (1 of {len(allowed) or os.cpu_count()} "
                         f"allowed), {dt:.1f} s, host {model}" + whole}

    line = {
        "metric": METRIC, "value": round(gbs, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "nx": nx, "ny": ny, "nz": nz, "eb": f"{w.eb_mode} {w.eb_value}",
                   "threshold": w.criterion.thr, "connectivity": w.criterion.connectivity,
                   "keep": w.criterion.keep, "path": "plain fused", "n_rows": int(e.n_rows),
                   "n_codes": int(e.n_codes), "n_outliers": int(e.n_outliers), "code_bits": int(qi.width_bits)},
        "roofline": roof, "path_roofline": path, "cpu_baseline": cpu,
        "stages_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in stages.items() if v[1]},
    }
    if tuning:
        line["autotune"] = tuning
    line["config"]["reduction"] = round(N / max(int(e.n_codes), 1), 3)  # spatial reduction N / codes
    line["parity"] = golden_parity("cylinder1024", res) if args.n == 1024 else None
    del x, out
    ctx.close()
    torch.cuda.empty_cache()
    w.volume = vol = None
    sections = [t for t in args.sections.split(",") if t and t != "none"]
    for name in sections:
        fn = {"c0": section_c0, "c2": section_c2, "batched": section_batched, "served": section_served}[name]
        try:
            line[name] = fn(args)
        except Exception as ex:  # a failing section is reported, the headline still printed
            log(f"section {name} failed: {ex!r}")
            line[name] = {"error": repr(ex)}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
