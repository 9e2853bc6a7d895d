"""CPU oracle for the ROI reduction path -- TEST INFRASTRUCTURE ONLY.

Plain single-threaded C (``roix_oracle.c``) behind ctypes.  Only the test
suite, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg
may import this package.  The GPU library never uses it and shares no code
with it.

Each wrapper names the passage of ROIX-Comp (arXiv 2602.15917) it follows;
the C file states the readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "roix_oracle.c")
_LIB = os.path.join(_HERE, "libroix_oracle.so")
_lib = None

OK, EINVAL, ERANGE, ENOMEM, ETRUNC = 0, 1, 2, 3, 4
FLAG_DEGENERATE, FLAG_EMPTY_ROI, FLAG_FIXED = 1, 2, 4
DTYPES = {np.dtype(np.float32): 0, np.dtype(np.uint16): 1}


class Params(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("xmin", ctypes.c_float), ("xmax", ctypes.c_float),
                ("eb32", ctypes.c_float), ("w", ctypes.c_float), ("r", ctypes.c_float),
                ("qmin", ctypes.c_int32), ("qmax", ctypes.c_int32), ("K", ctypes.c_int64),
                ("width_bits", ctypes.c_int32), ("esc", ctypes.c_uint32)]


class FusedInfo(ctypes.Structure):
    _fields_ = [("q", Params), ("seg_status", ctypes.c_int32), ("otsu_bin", ctypes.c_int32),
                ("q_thr", ctypes.c_int32), ("flags", ctypes.c_uint32), ("hist", ctypes.c_uint64 * 256),
                ("n_mask", ctypes.c_uint64), ("n_components", ctypes.c_uint64), ("n_kept", ctypes.c_uint64),
                ("n_kept_voxels", ctypes.c_uint64), ("bbox", ctypes.c_uint32 * 6),
                ("ext_status", ctypes.c_int32), ("pad", ctypes.c_int32), ("n_rows", ctypes.c_uint64),
                ("n_codes", ctypes.c_uint64), ("n_outliers", ctypes.c_uint64), ("stream_bytes", ctypes.c_uint64),
                ("stage_seconds", ctypes.c_double * 8), ("thresholds", ctypes.c_int32 * 3),
                ("n_classes", ctypes.c_int32)]


COMP_DTYPE = np.dtype([("label", "<u8"), ("size", "<u8"), ("x0", "<u4"), ("x1", "<u4"), ("y0", "<u4"),
                       ("y1", "<u4"), ("z0", "<u4"), ("z1", "<u4"), ("kept", "<u4"), ("pad", "<u4")])
ROW_DTYPE = np.dtype([("z", "<u4"), ("y", "<u4"), ("xs", "<u4"), ("xe", "<u4"), ("code_off", "<u8"),
                      ("outlier_off", "<u8")])


def build(force: bool = True) -> str:
    """Compile the oracle (plain C, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        vp, i64, u64, ci, dbl, f32 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_float)
        lib.oracle_range.argtypes = [vp, ci, u64, vp, vp]
        lib.oracle_range.restype = ci
        lib.oracle_resolve.argtypes = [f32, f32, ci, dbl, ctypes.POINTER(Params)]
        lib.oracle_resolve.restype = ci
        lib.oracle_quantize.argtypes = [vp, ci, u64, ctypes.POINTER(Params), vp, vp, vp]
        lib.oracle_quantize.restype = ci
        lib.oracle_histogram_codes.argtypes = [vp, u64, ctypes.POINTER(Params), vp]
        lib.oracle_histogram_codes.restype = None
        lib.oracle_otsu.argtypes = [vp, vp]
        lib.oracle_otsu.restype = ctypes.c_uint32
        lib.oracle_multi_otsu.argtypes = [vp, ci, vp]
        lib.oracle_multi_otsu.restype = ctypes.c_uint32
        lib.oracle_q_thr_otsu.argtypes = [ctypes.c_int32, ctypes.POINTER(Params)]
        lib.oracle_q_thr_otsu.restype = ctypes.c_int32
        lib.oracle_q_thr_fixed.argtypes = [dbl, ctypes.POINTER(Params)]
        lib.oracle_q_thr_fixed.restype = ctypes.c_int32
        lib.oracle_label.argtypes = [vp, i64, i64, i64, ci, ci, i64, vp, vp, vp, i64, vp]
        lib.oracle_label.restype = ci
        lib.oracle_rows.argtypes = [vp, i64, i64, i64, vp, i64]
        lib.oracle_rows.restype = u64
        lib.oracle_stream.argtypes = [vp, ci, i64, i64, ctypes.POINTER(Params), vp, u64, vp, u64, vp, u64, vp, vp]
        lib.oracle_stream.restype = ci
        lib.oracle_decode.argtypes = [vp, u64, vp, vp, u64, ctypes.POINTER(Params), i64, i64, i64, f32, vp]
        lib.oracle_decode.restype = ci
        lib.oracle_background.argtypes = [vp, ci, vp, i64, i64, i64, i64, ci, vp]
        lib.oracle_background.restype = ci
        lib.oracle_abs_quantize.argtypes = [vp, u64, dbl, vp, vp]
        lib.oracle_section.argtypes = [vp, ci, i64, i64, i64, ctypes.POINTER(Params), vp, u64, vp]
        lib.oracle_section.restype = ci
        lib.oracle_abs_quantize.restype = ci
        lib.oracle_huff_lengths.argtypes = [vp, vp]
        lib.oracle_huff_lengths.restype = ci
        lib.oracle_huff_encode.argtypes = [vp, u64, vp, vp, vp, u64, vp, vp]
        lib.oracle_huff_encode.restype = ci
        lib.oracle_huff_decode.argtypes = [vp, vp, vp, u64, u64, vp, vp]
        lib.oracle_huff_decode.restype = ci
        lib.oracle_fused.argtypes = [vp, ci, i64, i64, i64, ci, dbl, ci, dbl, ci, ci, i64, vp, i64, vp, i64, vp,
                                     i64, vp, i64, ctypes.POINTER(FusedInfo), vp]
        lib.oracle_fused.restype = ci
        lib.oracle_sizes.argtypes = [vp]
        lib.oracle_sizes.restype = None
        _lib = lib
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _dt(vol):
    try:
        return DTYPES[vol.dtype]
    except KeyError:
        raise TypeError(f"unsupported dtype {vol.dtype}") from None


def struct_sizes():
    out = np.zeros(4, dtype=np.int64)
    _load().oracle_sizes(_p(out))
    return {"params": int(out[0]), "comp": int(out[1]), "row": int(out[2]), "fused_info": int(out[3])}


def value_range(vol):
    """xmin, xmax (I_max of Eq. 1); raises on non-finite input."""
    vol = np.ascontiguousarray(vol)
    lo, hi = np.zeros(1, np.float32), np.zeros(1, np.float32)
    st = _load().oracle_range(_p(vol), _dt(vol), vol.size, _p(lo), _p(hi))
    return st, float(lo[0]), float(hi[0])


def resolve(xmin, xmax, eb_mode, eb_value):
    """Error bound resolution (Sec. 4.2.3: E_abs > 0). eb_mode 'abs'|'rel'."""
    p = Params()
    _load().oracle_resolve(xmin, xmax, 0 if eb_mode == "abs" else 1, eb_value, ctypes.byref(p))
    return p


def quantize(vol, p):
    """Per-voxel codes and the outlier bitmap (bit v%32 of word v//32)."""
    vol = np.ascontiguousarray(vol)
    codes = np.empty(vol.shape, np.int32)
    bits = np.empty((vol.size + 31) // 32, np.uint32)
    n = np.zeros(1, np.uint64)
    st = _load().oracle_quantize(_p(vol), _dt(vol), vol.size, ctypes.byref(p), _p(codes), _p(bits), _p(n))
    return st, codes, bits, int(n[0])


def histogram(codes, p):
    """256-bin histogram of floor(256 (q - qmin) / K) (Eq. 1 on codes)."""
    codes = np.ascontiguousarray(codes, dtype=np.int32)
    h = np.zeros(256, np.uint64)
    _load().oracle_histogram_codes(_p(codes), codes.size, ctypes.byref(p), _p(h))
    return h


def otsu(hist):
    """Two-class Otsu split t* (Sec. 4.1.3) and flags."""
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    t = np.zeros(1, np.int32)
    flags = _load().oracle_otsu(_p(h), _p(t))
    return int(t[0]), int(flags)


def multi_otsu(hist, classes):
    """Multi-level Otsu thresholds (3 or 4 classes; Liao et al. 2001, the
    method Sec. 4.1.3 names) and flags."""
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    t = np.zeros(3, np.int32)
    flags = _load().oracle_multi_otsu(_p(h), int(classes), _p(t))
    return tuple(int(v) for v in t[: classes - 1]), int(flags)


THR_MODES = {"otsu": 0, "fixed": 1, "multi3": 2, "multi4": 3, "otsu_slice": 4}
FLAG_SLICE = 8


def q_thr_otsu(t_star, p):
    return int(_load().oracle_q_thr_otsu(t_star, ctypes.byref(p)))


def q_thr_fixed(T, p):
    return int(_load().oracle_q_thr_fixed(T, ctypes.byref(p)))


def label(mask, connectivity, keep="largest", min_size=1, comps_cap=None):
    """3-D connected components of a mask (Sec. 4.2.1 in 3-D), labels = min
    linear index, -1 for background; keep flags per voxel."""
    mask = np.ascontiguousarray(mask).astype(np.uint8, copy=False)
    nz, ny, nx = mask.shape
    labels = np.empty(mask.shape, np.int64)
    keepm = np.empty(mask.shape, np.uint8)
    cap = mask.size if comps_cap is None else comps_cap
    comps = np.zeros(max(cap, 1), COMP_DTYPE)
    n = np.zeros(1, np.uint64)
    st = _load().oracle_label(_p(mask), nx, ny, nz, connectivity, 1 if keep == "largest" else 0, min_size,
                              _p(labels), _p(keepm), _p(comps), cap, _p(n))
    nc = int(n[0])
    return st, labels, keepm, comps[:min(nc, cap)].copy()


def rows(keep):
    """Geometry section (Eq. 3) from a per-voxel keep mask."""
    keep = np.ascontiguousarray(keep).astype(np.uint8, copy=False)
    nz, ny, nx = keep.shape
    cap = nz * ny
    r = np.zeros(max(cap, 1), ROW_DTYPE)
    n = int(_load().oracle_rows(_p(keep), nx, ny, nz, _p(r), cap))
    return r[:n].copy()


def stream(vol, p, row_table):
    """Pixel section (Eq. 4): packed codes + outlier values; fills offsets."""
    vol = np.ascontiguousarray(vol)
    nz, ny, nx = vol.shape
    rt = np.ascontiguousarray(row_table.copy())
    total = int((rt["xe"].astype(np.int64) - rt["xs"].astype(np.int64)).sum()) if len(rt) else 0
    nbytes = total * (p.width_bits // 8)
    s = np.zeros(max(nbytes, 1), np.uint8)
    o = np.zeros(max(total, 1), np.float32)
    nc, no = np.zeros(1, np.uint64), np.zeros(1, np.uint64)
    st = _load().oracle_stream(_p(vol), _dt(vol), nx, ny, ctypes.byref(p), _p(rt), len(rt), _p(s), nbytes,
                               _p(o), total, _p(nc), _p(no))
    return st, rt, s[:nbytes].copy(), o[:int(no[0])].copy()


def decode(row_table, stream_bytes, outliers, p, shape, background=0.0):
    """Reverse process of Sec. 4.3: rebuild the volume from rows + stream."""
    nz, ny, nx = shape
    out = np.empty(shape, np.float32)
    rt = np.ascontiguousarray(row_table)
    sb = np.ascontiguousarray(stream_bytes, dtype=np.uint8)
    ol = np.ascontiguousarray(outliers, dtype=np.float32)
    st = _load().oracle_decode(_p(rt), len(rt), _p(sb) if sb.size else None, _p(ol) if ol.size else None,
                               ol.size, ctypes.byref(p), nx, ny, nz, background, _p(out))
    return st, out


def background(vol, bg, op="subtract"):
    """Background subtraction of Sec. 4.1.1, M = I - B voxel by voxel
    (op "subtract"), or I + B (op "add": the decoded object back on its
    background, Sec. 4.3).  bg: float32 of shape (1, ny, nx) -- one
    calibration plane for every z -- or (nz, ny, nx).  Returns (status,
    float32 volume)."""
    vol = np.ascontiguousarray(vol)
    bg = np.ascontiguousarray(bg, dtype=np.float32)
    nz, ny, nx = vol.shape
    if bg.ndim != 3 or bg.shape[1:] != (ny, nx):
        return EINVAL, None
    out = np.empty(vol.shape, np.float32)
    st = _load().oracle_background(_p(vol), _dt(vol), _p(bg), bg.shape[0], nx, ny, nz,
                                   {"subtract": 0, "add": 1}[op], _p(out))
    return st, out


def section(vol, p, row_table, n_codes):
    """The normalised 8-bit pixel section of an extraction (Sec. 4.1.2, Eq. 1):
    bin(q) of every span voxel in stream order.  Returns (status, uint8[n_codes])."""
    vol = np.ascontiguousarray(vol)
    nz, ny, nx = vol.shape
    rt = np.ascontiguousarray(row_table, dtype=ROW_DTYPE)
    out = np.zeros(max(int(n_codes), 1), np.uint8)
    st = _load().oracle_section(_p(vol), _dt(vol), nx, ny, nz, ctypes.byref(p), _p(rt) if rt.size else None,
                                len(rt), _p(out))
    return st, out[:int(n_codes)]


def abs_quantize(pixels, e_abs):
    """The paper's absolute error-bounded quantisation of an 8-bit pixel
    sequence (Sec. 4.2.3; tolerance floor(e_abs) on integer pixels).  Returns (status, Q uint8, number of groups)."""
    d = np.ascontiguousarray(pixels, dtype=np.uint8).reshape(-1)
    q = np.empty(max(d.size, 1), np.uint8)
    n = np.zeros(1, np.uint64)
    st = _load().oracle_abs_quantize(_p(d) if d.size else None, d.size, float(e_abs), _p(q), _p(n))
    return st, q[: d.size].copy(), int(n[0])


HUFF_BLOCK = 4096
HUFF_SUB = 256  # bytes per sub-block of the optional sub-block index
HUFF_SUBS = HUFF_BLOCK // HUFF_SUB


def huff_lengths(hist):
    """Huffman code lengths (bits) for 256 byte counts; (status, uint8[256])."""
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    ln = np.zeros(256, np.uint8)
    st = _load().oracle_huff_lengths(_p(h), _p(ln))
    return st, ln


def huff_encode(data, cap_words=None, with_sub=False):
    """Canonical Huffman coding of a byte sequence in blocks of 4096 bytes.
    Returns (status, lengths uint8[256], block offsets uint64[nblocks + 1]
    in 32-bit words, payload uint32[words]), and with with_sub the sub-block
    index as a fifth item (uint16[16 nblocks]: code bits of each 256-byte
    sub-block)."""
    d = np.ascontiguousarray(data, dtype=np.uint8).reshape(-1)
    nb = (d.size + HUFF_BLOCK - 1) // HUFF_BLOCK
    cap = nb * HUFF_BLOCK if cap_words is None else cap_words  # 32 bits per byte at most
    ln = np.zeros(256, np.uint8)
    off = np.zeros(nb + 1, np.uint64)
    pay = np.zeros(max(cap, 1), np.uint32)
    tot = np.zeros(1, np.uint64)
    sub = np.zeros(max(HUFF_SUBS * nb, 1), np.uint16)
    st = _load().oracle_huff_encode(_p(d) if d.size else None, d.size, _p(ln), _p(off), _p(pay), cap, _p(tot),
                                    _p(sub) if with_sub else None)
    r = (st, ln, off, pay[: min(int(tot[0]), cap)].copy())
    return r + (sub[: HUFF_SUBS * nb].copy(),) if with_sub else r


def huff_decode(lengths, block_off, payload, n, sub_bits=None):
    """Inverse of huff_encode, from the block starts alone or, with the
    sub-block index, from every sub-block's start; (status, bytes)."""
    ln = np.ascontiguousarray(lengths, dtype=np.uint8)
    off = np.ascontiguousarray(block_off, dtype=np.uint64)
    pay = np.ascontiguousarray(payload, dtype=np.uint32)
    out = np.zeros(max(n, 1), np.uint8)
    sub = None if sub_bits is None else np.ascontiguousarray(sub_bits, dtype=np.uint16)
    st = _load().oracle_huff_decode(_p(ln), _p(off), _p(pay) if pay.size else None, pay.size, n, _p(out),
                                    _p(sub) if sub is not None and sub.size else None)
    return st, out[:n].copy()


def fused(vol, eb_mode, eb_value, thr="otsu", fixed_value=0.0, connectivity=26, keep="largest", min_size=1,
          comps_cap=None, rows_cap=None, stream_cap_bytes=None, outliers_cap=None):
    """The whole path (range, bound, codes, histogram, threshold, mask,
    components, keep, rows, stream).  Returns a dict of numpy outputs,
    trimmed to the reported counts."""
    vol = np.ascontiguousarray(vol)
    nz, ny, nx = vol.shape
    N = vol.size
    comps_cap = N if comps_cap is None else comps_cap
    rows_cap = nz * ny if rows_cap is None else rows_cap
    stream_cap_bytes = 4 * N if stream_cap_bytes is None else stream_cap_bytes
    outliers_cap = N if outliers_cap is None else outliers_cap
    # the component table is sized lazily: most volumes have few components
    comps = np.zeros(max(min(comps_cap, 1 << 20), 1), COMP_DTYPE)
    rows_a = np.zeros(max(rows_cap, 1), ROW_DTYPE)
    s = np.zeros(max(stream_cap_bytes, 1), np.uint8)
    o = np.zeros(max(min(outliers_cap, N), 1), np.float32)
    info = FusedInfo()
    lib = _load()
    sthr = np.full(nz, -1, np.int32)
    args = (_p(vol), _dt(vol), nx, ny, nz, 0 if eb_mode == "abs" else 1, eb_value, THR_MODES[thr],
            fixed_value, connectivity, 1 if keep == "largest" else 0, min_size)
    st = lib.oracle_fused(*args, _p(comps), min(comps_cap, len(comps)), _p(rows_a), rows_cap, _p(s),
                          stream_cap_bytes, _p(o), len(o), ctypes.byref(info), _p(sthr))
    if info.n_components > len(comps) and comps_cap >= info.n_components:
        comps = np.zeros(int(info.n_components), COMP_DTYPE)
        info = FusedInfo()
        st = lib.oracle_fused(*args, _p(comps), len(comps), _p(rows_a), rows_cap, _p(s), stream_cap_bytes,
                              _p(o), len(o), ctypes.byref(info), _p(sthr))
    nb = min(int(info.stream_bytes), stream_cap_bytes)
    return {
        "status": st,
        "info": info,
        "params": info.q,
        "comps": comps[:min(int(info.n_components), len(comps))].copy(),
        "rows": rows_a[:min(int(info.n_rows), rows_cap)].copy(),
        "stream": s[:nb].copy(),
        "outliers": o[:min(int(info.n_outliers), len(o))].copy(),
        "hist": np.frombuffer(bytes(info.hist), dtype=np.uint64).copy(),
        "slice_thr": sthr,
    }
