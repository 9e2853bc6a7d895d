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


def algorithmic_bytes(stage, N, s, n_codes, code_bytes, n_rows, nrows_all, W):
    """Bytes a launch of `stage` must move at minimum (per call of the path)."""
    if stage == "range":
        return N * s
    if stage == "quant_hist":
        return N * s + N                      # read the volume, write the 1-byte bin proxy
    if stage == "mask_runs":
        return N + nrows_all * W * 8          # read the proxy, write the row bitmask
    if stage == "emit":
        return n_codes * (s + code_bytes) + n_rows * 32
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024, help="volume side (1024 = the benchmark workload)")
    ap.add_argument("--cpu-planes", type=int, default=256, help="z-planes of the CPU-oracle sample (0 = skip)")
    ap.add_argument("--no-stage-timing", action="store_true")
    args = ap.parse_args()
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
    w = synth.config1(n=args.n)
    vol = w.volume
    nz, ny, nx = vol.shape
    N, s = vol.size, vol.itemsize
    log(f"generated {w.name} in {time.time() - t0:.1f}s")
    x = torch.from_numpy(vol).to(dev)
    crit = roix.Criterion(w.criterion.thr, 0.0, w.criterion.connectivity, w.criterion.keep, w.criterion.min_size)
    dims = roix.dims_of(x)
    ctx = roix.Context(0, roix.scratch_bytes(dims, roix.F32, crit))
    b = roix.bounds(dims, roix.F32, crit)
    out = roix.Outputs(dev, b["rows"], b["stream_bytes"], b["outliers"], 1 << 22)
    stream = torch.cuda.current_stream()

    def step():
        ctx.fused(x, w.eb_mode, w.eb_value, crit, out, stream)

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
        dom = max((k for k in per if algorithmic_bytes(k, N, s, e.n_codes, code_bytes, e.n_rows, nrows_all, W)),
                  key=lambda k: per[k][0])
        avg_ms = per[dom][0]
        byts = algorithmic_bytes(dom, N, s, e.n_codes, code_bytes, e.n_rows, nrows_all, W)
        ach = byts / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "alg_bytes_per_launch": int(byts),
                "avg_launch_ms": round(avg_ms, 4)}
    # whole-path byte model: two input reads, 1-byte proxy written and read,
    # span voxels re-read, codes written, row table written
    b_alg = N * (2 * s + 2) + e.n_codes * (s + code_bytes) + 32 * e.n_rows
    path = {"alg_bytes": int(b_alg), "achieved": round(b_alg / (ms * 1e-3) / 1e9, 1),
            "frac": round(b_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    cpu = None
    if args.cpu_planes > 0:
        import oracle
        k = min(args.cpu_planes, nz)
        sample = np.ascontiguousarray(vol[:k])
        c = w.criterion
        log(f"CPU oracle on {k} of {nz} z-planes ...")
        t = time.perf_counter()
        r = oracle.fused(sample, w.eb_mode, w.eb_value, c.thr, c.fixed_value, c.connectivity, c.keep, c.min_size,
                         comps_cap=1 << 20)
        dt = time.perf_counter() - t
        assert r["status"] == 0
        try:
            model = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
            model = [l.split(":", 1)[1].strip() for l in model.splitlines() if l.startswith("Model name")][0]
        except Exception:
            model = "unknown"
        cpu = {"value": round(sample.nbytes / dt / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"first {k} of {nz} z-planes of the same volume ({sample.nbytes / 1e9:.2f} GB), "
                         f"single-threaded C oracle, {dt:.1f} s, host {model}, {os.cpu_count()} cpus visible"}

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
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
