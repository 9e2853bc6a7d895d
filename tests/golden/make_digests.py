"""Write the expected outputs of the full-size workloads (SHA-256 digests and
info fields) by running the CPU oracle.  Calls only ``synth`` (inputs) and
``oracle``; nothing here touches the GPU library.

    python tests/golden/make_digests.py [ellipsoids128] [cylinder1024] [rings2048]

ellipsoids128 (128^3 f32) takes a second; cylinder1024 (1024^3 f32) about two
minutes and 10 GB of host memory; rings2048 (2048 x 2048 x 1024 u16) about ten
minutes and 30 GB.
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

ABSQ_E = (2.0, 1.0, 5.0)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "digests.json")


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def digest(name, w):
    c = w.criterion
    t = time.time()
    r = oracle.fused(w.volume, w.eb_mode, w.eb_value, c.thr, c.fixed_value, c.connectivity, c.keep, c.min_size,
                     comps_cap=1 << 20)
    dt = time.time() - t
    i, p = r["info"], r["params"]
    # the Eq. 1 normalised 8-bit section of the extracted spans, and the
    # paper's quantiser (Sec. 4.2.3) on it at the benchmark's tolerances
    sst, sec = oracle.section(w.volume, p, r["rows"], i.n_codes)
    absq = {}
    for e in ABSQ_E:
        ast, q, ng = oracle.abs_quantize(sec, e)
        absq[repr(e)] = {"status": ast, "n_groups": int(ng), "sha256": sha(q)}
    return {
        "workload": w.name,
        "input_sha256": w.sha256(),
        "oracle_seconds": round(dt, 1),
        "status": r["status"],
        "quant": {"xmin": float(p.xmin), "xmax": float(p.xmax), "eb32": float(p.eb32), "w": float(p.w),
                  "r": float(p.r), "qmin": p.qmin, "qmax": p.qmax, "K": p.K, "width_bits": p.width_bits,
                  "esc": p.esc},
        "seg": {"otsu_bin": i.otsu_bin, "q_thr": i.q_thr, "flags": i.flags, "n_mask": i.n_mask,
                "n_components": i.n_components, "n_kept": i.n_kept, "n_kept_voxels": i.n_kept_voxels,
                "bbox": list(i.bbox), "hist_sha256": sha(r["hist"])},
        "extract": {"n_rows": i.n_rows, "n_codes": i.n_codes, "n_outliers": i.n_outliers,
                    "stream_bytes": i.stream_bytes},
        "sha256": {"rows": sha(r["rows"]), "stream": sha(r["stream"]), "outliers": sha(r["outliers"]),
                   "comps": sha(r["comps"])},
        "section": {"status": sst, "n": int(len(sec)), "sha256": sha(sec),
                    "level_counts_sha256": sha(np.bincount(sec, minlength=256).astype(np.uint64))},
        "absq_on_section": absq,
    }


def main():
    which = sys.argv[1:] or ["ellipsoids128", "cylinder1024", "rings2048"]
    out = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in which:
        w = getattr(synth, name)()
        out[name] = digest(name, w)
        del w
        json.dump(out, open(OUT, "w"), indent=1, sort_keys=True)
        print(name, "done", out[name]["oracle_seconds"], "s", flush=True)


if __name__ == "__main__":
    main()
