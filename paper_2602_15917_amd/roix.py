"""Python binding of libroix.so (ctypes).

Argument marshalling only: torch tensors provide device memory and the HIP
stream; every step of the reduction runs in the library's HIP kernels.  If
the library is not built, every call raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libroix.so")

OK, EINVAL, ERANGE, ENOMEM, ETRUNC, EDEVICE, EBUSY, ESEQ = range(8)
F32, U16 = 0, 1
EB_ABS, EB_REL = 0, 1
THR_OTSU, THR_FIXED, THR_MULTI_OTSU, THR_OTSU_SLICE = 0, 1, 2, 3
FLAG_PER_SLICE = 8
BG_OPS = {"subtract": 0, "add": 1}
KEEP_MIN_SIZE, KEEP_LARGEST = 0, 1
FLAG_DEGENERATE_HISTOGRAM, FLAG_EMPTY_ROI, FLAG_FIXED_THRESHOLD = 1, 2, 4
NOT_COMPUTED = (1 << 64) - 1


class RoixError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: status {status}")
        self.status = status


class Dims(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64)]


class Eb(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("pad", ctypes.c_int32), ("value", ctypes.c_double)]


class CCriterion(ctypes.Structure):
    _fields_ = [("thr", ctypes.c_int32), ("connectivity", ctypes.c_int32), ("fixed_value", ctypes.c_double),
                ("keep", ctypes.c_int32), ("classes", ctypes.c_int32), ("min_size", ctypes.c_int64)]


class QuantInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("xmin", ctypes.c_float), ("xmax", ctypes.c_float),
                ("eb32", ctypes.c_float), ("w", ctypes.c_float), ("r", ctypes.c_float), ("qmin", ctypes.c_int32),
                ("qmax", ctypes.c_int32), ("K", ctypes.c_int64), ("width_bits", ctypes.c_int32),
                ("esc", ctypes.c_uint32), ("n_outliers", ctypes.c_uint64)]


class SegInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("otsu_bin", ctypes.c_int32), ("q_thr", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("hist", ctypes.c_uint64 * 256), ("n_mask", ctypes.c_uint64),
                ("n_components", ctypes.c_uint64), ("n_kept", ctypes.c_uint64), ("n_kept_voxels", ctypes.c_uint64),
                ("bbox", ctypes.c_uint32 * 6), ("thresholds", ctypes.c_int32 * 3), ("n_classes", ctypes.c_int32)]


class ExtractInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("pad", ctypes.c_int32), ("n_rows", ctypes.c_uint64),
                ("n_codes", ctypes.c_uint64), ("n_outliers", ctypes.c_uint64), ("stream_bytes", ctypes.c_uint64)]


class FusedOut(ctypes.Structure):
    _fields_ = [("d_rows", ctypes.c_void_p), ("rows_cap", ctypes.c_int64), ("d_stream", ctypes.c_void_p),
                ("stream_cap_bytes", ctypes.c_int64), ("d_outliers", ctypes.c_void_p),
                ("outliers_cap", ctypes.c_int64), ("d_comps", ctypes.c_void_p), ("comps_cap", ctypes.c_int64),
                ("d_qinfo", ctypes.c_void_p), ("d_sinfo", ctypes.c_void_p), ("d_einfo", ctypes.c_void_p),
                ("d_slice_thr", ctypes.c_void_p)]


class VolumeDesc(ctypes.Structure):
    _fields_ = [("d_in", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("pad", ctypes.c_int32), ("dims", Dims),
                ("eb", Eb), ("crit", CCriterion), ("out", FusedOut)]


class ReqResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("kind", ctypes.c_int32), ("vol_id", ctypes.c_int64),
                ("submit_ms", ctypes.c_double), ("done_ms", ctypes.c_double), ("latency_ms", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("volumes_admitted", ctypes.c_int64), ("volumes_refused", ctypes.c_int64),
                ("volumes_open", ctypes.c_int64), ("slabs_done", ctypes.c_int64), ("closes_done", ctypes.c_int64),
                ("bytes_in", ctypes.c_int64), ("budget_bytes", ctypes.c_uint64), ("bytes_in_use", ctypes.c_uint64),
                ("slab_p50_ms", ctypes.c_double), ("slab_p99_ms", ctypes.c_double), ("slab_max_ms", ctypes.c_double),
                ("close_p50_ms", ctypes.c_double), ("close_p99_ms", ctypes.c_double)]


REQ_SLAB, REQ_CLOSE = 0, 1
COMP_BYTES, ROW_BYTES = 48, 32
STAGE_MAX = 64

_lib = None


def load():
    """Load libroix.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, ci, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
    P = ctypes.POINTER
    lib.roix_ctx_create.argtypes = [ci, sz, P(vp)]
    lib.roix_ctx_destroy.argtypes = [vp]
    lib.roix_scratch_bytes.argtypes = [Dims, ci, P(CCriterion)]
    lib.roix_scratch_bytes.restype = sz
    lib.roix_bounds.argtypes = [Dims, ci, P(CCriterion), P(i64), P(i64), P(i64), P(i64)]
    lib.roix_quantize.argtypes = [vp, vp, ci, Dims, Eb, vp, vp, vp, vp]
    lib.roix_segment.argtypes = [vp, vp, Dims, vp, P(CCriterion), vp, vp, vp, i64, vp, vp]
    lib.roix_extract.argtypes = [vp, vp, ci, vp, Dims, vp, P(FusedOut), vp]
    lib.roix_fused.argtypes = [vp, vp, ci, Dims, Eb, P(CCriterion), P(FusedOut), vp]
    lib.roix_fused_noalloc.argtypes = [vp, ci, Dims, Eb, P(CCriterion), P(FusedOut), vp]
    lib.roix_stage_count.restype = ci
    lib.roix_stage_name.argtypes = [ci]
    lib.roix_stage_name.restype = ctypes.c_char_p
    lib.roix_ctx_set_timing.argtypes = [vp, ci]
    lib.roix_ctx_read_timing.argtypes = [vp, P(ctypes.c_double), P(i64)]
    lib.roix_fused_batch.argtypes = [vp, ctypes.c_int32, vp, vp]
    lib.roix_ctx_set_param.argtypes = [vp, ctypes.c_char_p, i64]
    lib.roix_ctx_get_param.argtypes = [vp, ctypes.c_char_p, P(i64)]
    lib.roix_status_string.argtypes = [ci]
    lib.roix_status_string.restype = ctypes.c_char_p
    lib.roix_server_create.argtypes = [vp, sz, P(vp)]
    lib.roix_server_destroy.argtypes = [vp]
    lib.roix_server_volume_bytes.argtypes = [vp, Dims, ci, Eb, P(CCriterion)]
    lib.roix_server_set_param.argtypes = [vp, ctypes.c_char_p, i64]
    lib.roix_server_set_param.restype = ci
    lib.roix_server_volume_bytes.restype = sz
    lib.roix_volume_open.argtypes = [vp, Dims, ci, Eb, P(CCriterion), P(FusedOut), P(i64)]
    lib.roix_slab_submit.argtypes = [vp, i64, i64, i64, vp, ci, P(i64)]
    lib.roix_volume_close.argtypes = [vp, i64, P(i64)]
    lib.roix_volume_abort.argtypes = [vp, i64]
    lib.roix_wait.argtypes = [vp, i64, i64, P(ReqResult)]
    lib.roix_server_stats.argtypes = [vp, P(ServerStats)]
    lib.roix_decode.argtypes = [vp, vp, i64, vp, i64, vp, i64, vp, vp, Dims, ctypes.c_float, vp, vp, vp]
    lib.roix_background.argtypes = [vp, vp, ci, Dims, vp, i64, ci, vp, vp]
    lib.roix_fused_background.argtypes = [vp, vp, Dims, vp, i64, Eb, P(CCriterion), P(FusedOut), vp, vp]
    lib.roix_abs_quantize.argtypes = [vp, vp, i64, ctypes.c_double, vp, vp, vp]
    lib.roix_huff_encode.argtypes = [vp, vp, i64, vp, vp, vp, vp, i64, vp, vp]
    lib.roix_autotune.argtypes = [vp, vp, ci, Dims, Eb, P(CCriterion), P(FusedOut), ctypes.c_int32, ctypes.c_char_p,
                                  P(TuneResult), vp]
    lib.roix_huff_decode.argtypes = [vp, vp, vp, vp, vp, i64, i64, vp, vp, vp]
    lib.roix_abs_quantize_scratch_bytes.argtypes = [i64]
    lib.roix_section.argtypes = [vp, vp, ci, Dims, P(FusedOut), vp, i64, vp, vp]
    lib.roix_abs_quantize_scratch_bytes.restype = sz
    for f in ("roix_ctx_create", "roix_ctx_destroy", "roix_bounds", "roix_quantize", "roix_segment",
              "roix_extract", "roix_fused", "roix_fused_noalloc", "roix_ctx_set_timing", "roix_ctx_read_timing", "roix_fused_batch",
              "roix_ctx_set_param", "roix_ctx_get_param", "roix_server_create", "roix_server_destroy",
              "roix_volume_open", "roix_slab_submit", "roix_volume_close", "roix_volume_abort", "roix_wait",
              "roix_server_stats", "roix_decode", "roix_background", "roix_fused_background", "roix_abs_quantize",
              "roix_huff_encode", "roix_huff_decode", "roix_autotune", "roix_section"):
        getattr(lib, f).restype = ci
    _lib = lib
    return lib


@dataclass
class Criterion:
    """ROI criterion (mirrors roix_criterion)."""
    thr: str = "otsu"          # "otsu" | "fixed" | "multi3" | "multi4" (multi-level Otsu) | "otsu_slice"
    fixed_value: float = 0.0
    connectivity: int = 26     # 6 | 26
    keep: str = "largest"      # "largest" | "min_size"
    min_size: int = 1

    def c(self) -> CCriterion:
        thr, classes = _THR_CODES[self.thr]
        return CCriterion(thr, int(self.connectivity), float(self.fixed_value),
                          KEEP_LARGEST if self.keep == "largest" else KEEP_MIN_SIZE, classes, int(self.min_size))


_THR_CODES = {"otsu": (THR_OTSU, 0), "fixed": (THR_FIXED, 0), "multi3": (THR_MULTI_OTSU, 3),
              "multi4": (THR_MULTI_OTSU, 4), "otsu_slice": (THR_OTSU_SLICE, 0)}


def dims_of(vol: torch.Tensor) -> Dims:
    nz, ny, nx = vol.shape
    return Dims(nx, ny, nz)


def dtype_of(vol: torch.Tensor) -> int:
    if vol.dtype == torch.float32:
        return F32
    if vol.dtype == torch.uint16:
        return U16
    raise TypeError(f"unsupported dtype {vol.dtype}")


def eb_of(mode: str, value: float) -> Eb:
    return Eb(EB_ABS if mode == "abs" else EB_REL, 0, float(value))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check(st, what):
    if st != OK:
        raise RoixError(st, what)


NOALLOC_SCRATCH_BYTES = 64 << 20  # ROIX_NOALLOC_SCRATCH_BYTES


def fused_noalloc(vol: torch.Tensor, eb_mode: str, eb_value: float, crit: Criterion, out: "Outputs",
                  stream=None):
    """roix_fused_noalloc: the fused path on the library's fixed scratch array
    (no context, no device allocation; volumes whose worst-case scratch fits
    NOALLOC_SCRATCH_BYTES).  Runs on the current device."""
    c = crit.c()
    st = load().roix_fused_noalloc(_ptr(vol), dtype_of(vol), dims_of(vol), eb_of(eb_mode, eb_value),
                                   ctypes.byref(c), ctypes.byref(out.c), _stream(stream))
    _check(st, "roix_fused_noalloc")


def scratch_bytes(dims: Dims, dtype: int, crit: Criterion | None = None) -> int:
    c = crit.c() if crit is not None else CCriterion()
    return int(load().roix_scratch_bytes(dims, dtype, ctypes.byref(c)))


def bounds(dims: Dims, dtype: int, crit: Criterion | None = None):
    c = crit.c() if crit is not None else CCriterion()
    r, s, o, k = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load().roix_bounds(dims, dtype, ctypes.byref(c), ctypes.byref(r), ctypes.byref(s), ctypes.byref(o),
                              ctypes.byref(k)), "roix_bounds")
    return {"rows": r.value, "stream_bytes": s.value, "outliers": o.value, "components": k.value}


def decode_info(dinfo: torch.Tensor) -> "DecodeInfo":
    return _info(dinfo, DecodeInfo)


def absq_info(info: torch.Tensor) -> "AbsqInfo":
    return _info(info, AbsqInfo)


def section_info(info: torch.Tensor) -> "SectionInfo":
    return _info(info, SectionInfo)


def huff_info(info: torch.Tensor) -> "HuffInfo":
    return _info(info, HuffInfo)


def abs_quantize_scratch_bytes(m: int) -> int:
    return int(load().roix_abs_quantize_scratch_bytes(int(m)))


def stage_names():
    lib = load()
    return [lib.roix_stage_name(i).decode() for i in range(lib.roix_stage_count())]


def _info(buf: torch.Tensor, cls):
    return cls.from_buffer_copy(bytes(buf.cpu().numpy().tobytes()))


class Outputs:
    """Caller-owned output buffers of extract/fused (device tensors)."""

    def __init__(self, device, rows_cap, stream_cap_bytes, outliers_cap, comps_cap, nz_slices=0):
        self.rows = torch.empty(max(rows_cap, 1) * ROW_BYTES, dtype=torch.uint8, device=device)
        self.stream = torch.empty(max(stream_cap_bytes, 4), dtype=torch.uint8, device=device)
        self.outliers = torch.empty(max(outliers_cap, 1), dtype=torch.float32, device=device)
        self.comps = torch.empty(max(comps_cap, 1) * COMP_BYTES, dtype=torch.uint8, device=device)
        self.qinfo = torch.zeros(ctypes.sizeof(QuantInfo), dtype=torch.uint8, device=device)
        self.sinfo = torch.zeros(ctypes.sizeof(SegInfo), dtype=torch.uint8, device=device)
        self.einfo = torch.zeros(ctypes.sizeof(ExtractInfo), dtype=torch.uint8, device=device)
        # per-slice thresholds (criterion "otsu_slice"): one int32 per z-slice
        self.slice_thr = torch.full((nz_slices,), -1, dtype=torch.int32, device=device) if nz_slices else None
        self.caps = (rows_cap, stream_cap_bytes, outliers_cap, comps_cap)
        self.c = FusedOut(self.rows.data_ptr(), rows_cap, self.stream.data_ptr(), stream_cap_bytes,
                          self.outliers.data_ptr(), outliers_cap, self.comps.data_ptr(), comps_cap,
                          self.qinfo.data_ptr(), self.sinfo.data_ptr(), self.einfo.data_ptr(),
                          self.slice_thr.data_ptr() if nz_slices else None)

    def collect(self):
        """Host copies of the infos and the outputs trimmed to the counts
        (call after the stream has been synchronised)."""
        q, s, e = _info(self.qinfo, QuantInfo), _info(self.sinfo, SegInfo), _info(self.einfo, ExtractInfo)
        rows_cap, stream_cap, outl_cap, comps_cap = self.caps
        nr = min(int(e.n_rows), rows_cap)
        nb = min(int(e.stream_bytes), stream_cap)
        no = min(int(e.n_outliers), outl_cap)
        nc = min(int(s.n_components), comps_cap)
        return {
            "qinfo": q, "sinfo": s, "einfo": e,
            "rows": self.rows[: nr * ROW_BYTES].cpu().numpy(),
            "stream": self.stream[:nb].cpu().numpy(),
            "outliers": self.outliers[:no].cpu().numpy(),
            "comps": self.comps[: nc * COMP_BYTES].cpu().numpy(),
            "slice_thr": self.slice_thr.cpu().numpy() if self.slice_thr is not None else None,
        }


class DecodeInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("pad", ctypes.c_int32), ("n_rows", ctypes.c_uint64),
                ("n_codes", ctypes.c_uint64), ("n_outliers", ctypes.c_uint64)]


class HuffInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("max_len", ctypes.c_int32), ("n", ctypes.c_uint64),
                ("n_blocks", ctypes.c_uint64), ("payload_words", ctypes.c_uint64),
                ("compressed_bytes", ctypes.c_uint64), ("pad", ctypes.c_uint64 * 3)]


HUFF_BLOCK = 4096
HUFF_SUBS = 16  # 256-byte sub-blocks per block in the sub-block index


class TuneResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_timed", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("default_ms", ctypes.c_double), ("best_ms", ctypes.c_double),
                ("params", ctypes.c_int64 * 7)]


TUNE_PARAMS = ("grid_stream", "grid_read", "grid_mask", "grid_emit", "seg_grid", "stats_grid", "seg_runs")


class SectionInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("pad", ctypes.c_int32), ("n_codes", ctypes.c_uint64)]


class AbsqInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("rounds", ctypes.c_int32), ("n_groups", ctypes.c_uint64),
                ("finisher_chunks", ctypes.c_uint64), ("pad", ctypes.c_uint64)]


class Context:
    """A library context (scratch arena) on one device."""

    def __init__(self, device: int = 0, scratch_bytes: int = 0):
        lib = load()
        self.device = device
        h = ctypes.c_void_p()
        _check(lib.roix_ctx_create(device, scratch_bytes, ctypes.byref(h)), "roix_ctx_create")
        self.h = h

    def close(self):
        if self.h:
            load().roix_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------- timing
    def set_timing(self, on: bool):
        _check(load().roix_ctx_set_timing(self.h, 1 if on else 0), "roix_ctx_set_timing")

    def read_timing(self):
        lib = load()
        n = lib.roix_stage_count()
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(lib.roix_ctx_read_timing(self.h, ms, cnt), "roix_ctx_read_timing")
        names = stage_names()
        return {names[i]: (ms[i], cnt[i]) for i in range(n)}

    # ------------------------------------------------------- parameters
    def set_param(self, name: str, value: int):
        _check(load().roix_ctx_set_param(self.h, name.encode(), int(value)), f"roix_ctx_set_param({name})")

    def get_param(self, name: str) -> int:
        v = ctypes.c_int64()
        _check(load().roix_ctx_get_param(self.h, name.encode(), ctypes.byref(v)), f"roix_ctx_get_param({name})")
        return v.value

    # ----------------------------------------------------------- calls
    def decode(self, out: Outputs, dims: Dims, background: float = 0.0, dst: torch.Tensor | None = None,
               dinfo: torch.Tensor | None = None, stream=None):
        """Enqueue the reverse process of the extraction held in `out` (its
        device row table, stream, outliers and infos).  Returns (volume, dinfo)
        device tensors; read dinfo with decode_info() after a sync."""
        dev = out.rows.device
        if dst is None:
            dst = torch.empty((dims.nz, dims.ny, dims.nx), dtype=torch.float32, device=dev)
        if dinfo is None:
            dinfo = torch.zeros(ctypes.sizeof(DecodeInfo), dtype=torch.uint8, device=dev)
        rows_cap, stream_cap, outl_cap, _ = out.caps
        st = load().roix_decode(self.h, out.rows.data_ptr(), rows_cap, out.stream.data_ptr(), stream_cap,
                                out.outliers.data_ptr(), outl_cap, out.qinfo.data_ptr(), out.einfo.data_ptr(),
                                dims, float(background), dst.data_ptr(), dinfo.data_ptr(), _stream(stream))
        _check(st, "roix_decode")
        return dst, dinfo

    def background(self, vol: torch.Tensor, bg: torch.Tensor, op: str = "subtract",
                   dst: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Enqueue M = vol - bg (op "subtract") or vol + bg (op "add") on the
        device; bg is float32 of shape (1, ny, nx) or (nz, ny, nx).  dst
        (float32, the volume's shape) may be vol itself for a float32 volume.
        Returns dst."""
        if not (vol.is_contiguous() and bg.is_contiguous()):
            raise ValueError("background: volume and reference must be contiguous")
        if dst is None:
            dst = torch.empty(vol.shape, dtype=torch.float32, device=vol.device)
        planes = bg.shape[0] if bg.dim() == 3 else -1
        st = load().roix_background(self.h, _ptr(vol), dtype_of(vol), dims_of(vol), _ptr(bg), planes,
                                    BG_OPS[op], _ptr(dst), _stream(stream))
        _check(st, "roix_background")
        return dst

    def fused_background(self, vol: torch.Tensor, bg: torch.Tensor, eb_mode: str, eb_value: float, crit: Criterion,
                         out: Outputs, work: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Enqueue the fused path on M = vol - bg (float32 volume; bg of shape
        (1, ny, nx) or (nz, ny, nx)).  work: float32 workspace of the volume's
        size (allocated when None).  Returns the workspace."""
        if vol.dtype != torch.float32 or not (vol.is_contiguous() and bg.is_contiguous()):
            raise ValueError("fused_background: contiguous float32 volume and reference")
        if work is None:
            work = torch.empty_like(vol)
        c = crit.c()
        planes = bg.shape[0] if bg.dim() == 3 else -1
        st = load().roix_fused_background(self.h, _ptr(vol), dims_of(vol), _ptr(bg), planes, eb_of(eb_mode, eb_value),
                                          ctypes.byref(c), ctypes.byref(out.c), _ptr(work), _stream(stream))
        _check(st, "roix_fused_background")
        return work

    def section(self, vol: torch.Tensor, out: Outputs, dst: torch.Tensor | None = None,
                info: torch.Tensor | None = None, stream=None):
        """Enqueue the normalised 8-bit pixel section of the extraction in
        `out`, made from `vol`.  Returns (section, info); the section holds
        info.n_codes levels (dst defaults to the stream's capacity)."""
        if dst is None:
            dst = torch.empty(max(out.caps[1], 16), dtype=torch.uint8, device=vol.device)
        if info is None:
            info = torch.zeros(ctypes.sizeof(SectionInfo), dtype=torch.uint8, device=vol.device)
        st = load().roix_section(self.h, _ptr(vol), dtype_of(vol), dims_of(vol), ctypes.byref(out.c), _ptr(dst),
                                 dst.numel(), _ptr(info), _stream(stream))
        _check(st, "roix_section")
        return dst, info

    def abs_quantize(self, pixels: torch.Tensor, e_abs: float, dst: torch.Tensor | None = None,
                     info: torch.Tensor | None = None, stream=None):
        """Enqueue the absolute error-bounded quantisation of a uint8 pixel
        sequence (any contiguous shape, taken flat).  Returns (Q, info)."""
        if pixels.dtype != torch.uint8 or not pixels.is_contiguous():
            raise ValueError("abs_quantize: a contiguous uint8 tensor")
        if dst is None:
            dst = torch.empty_like(pixels)
        if info is None:
            info = torch.zeros(ctypes.sizeof(AbsqInfo), dtype=torch.uint8, device=pixels.device)
        st = load().roix_abs_quantize(self.h, _ptr(pixels), pixels.numel(), float(e_abs), _ptr(dst), _ptr(info),
                                      _stream(stream))
        _check(st, "roix_abs_quantize")
        return dst, info

    def autotune(self, vol: torch.Tensor, eb_mode: str, eb_value: float, crit: Criterion, out: Outputs, reps: int = 3,
                 cache: str | None = None, stream=None) -> "TuneResult":
        """Tune the context's launch parameters on this volume (synchronous;
        see roix_autotune).  Returns the TuneResult."""
        c = crit.c()
        res = TuneResult()
        st = load().roix_autotune(self.h, _ptr(vol), dtype_of(vol), dims_of(vol), eb_of(eb_mode, eb_value),
                                  ctypes.byref(c), ctypes.byref(out.c), int(reps),
                                  cache.encode() if cache else None, ctypes.byref(res), _stream(stream))
        _check(st, "roix_autotune")
        return res

    def huff_encode(self, data: torch.Tensor, payload_cap_words: int | None = None, stream=None,
                    with_sub: bool = False):
        """Enqueue the Huffman stage over a contiguous uint8 tensor (taken
        flat).  Returns (lengths, block_off, payload, info); the payload holds
        payload_cap_words words (default: enough for any input).  with_sub:
        also the sub-block index, returned as a fifth item (int16 view of the
        16 nblocks bit counts)."""
        if data.dtype != torch.uint8 or not data.is_contiguous():
            raise ValueError("huff_encode: a contiguous uint8 tensor")
        n = data.numel()
        nb = (n + HUFF_BLOCK - 1) // HUFF_BLOCK
        cap = nb * HUFF_BLOCK if payload_cap_words is None else int(payload_cap_words)
        dev = data.device
        lengths = torch.zeros(256, dtype=torch.uint8, device=dev)
        off = torch.zeros(nb + 1, dtype=torch.int64, device=dev)
        payload = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        info = torch.zeros(ctypes.sizeof(HuffInfo), dtype=torch.uint8, device=dev)
        sub = torch.zeros(max(HUFF_SUBS * nb, 1), dtype=torch.int16, device=dev) if with_sub else None
        st = load().roix_huff_encode(self.h, _ptr(data), n, _ptr(lengths), _ptr(off),
                                     _ptr(sub) if with_sub else None, _ptr(payload), cap, _ptr(info),
                                     _stream(stream))
        _check(st, "roix_huff_encode")
        return (lengths, off, payload, info, sub) if with_sub else (lengths, off, payload, info)

    def huff_decode(self, lengths: torch.Tensor, off: torch.Tensor, payload: torch.Tensor, payload_words: int,
                    n: int, dst: torch.Tensor | None = None, stream=None, sub: torch.Tensor | None = None):
        """Enqueue the decoder (from every sub-block's start when the
        sub-block index `sub` is given); returns (bytes, info)."""
        if dst is None:
            dst = torch.empty(max(n, 1), dtype=torch.uint8, device=lengths.device)
        info = torch.zeros(ctypes.sizeof(HuffInfo), dtype=torch.uint8, device=lengths.device)
        st = load().roix_huff_decode(self.h, _ptr(lengths), _ptr(off), _ptr(sub) if sub is not None else None,
                                     _ptr(payload), int(payload_words), int(n), _ptr(dst), _ptr(info),
                                     _stream(stream))
        _check(st, "roix_huff_decode")
        return dst[:n], info

    def fused(self, vol: torch.Tensor, eb_mode: str, eb_value: float, crit: Criterion, out: Outputs,
              stream=None):
        """Enqueue the fused path; returns after launching (sync, then out.collect())."""
        c = crit.c()
        st = load().roix_fused(self.h, _ptr(vol), dtype_of(vol), dims_of(vol), eb_of(eb_mode, eb_value),
                               ctypes.byref(c), ctypes.byref(out.c), _stream(stream))
        _check(st, "roix_fused")

    def fused_batch(self, items, stream=None):
        """items: list of (volume tensor, eb_mode, eb_value, Criterion, Outputs).
        Enqueues the batched path (one graph launch when capture is on)."""
        arr = (VolumeDesc * len(items))()
        for i, (vol, ebm, ebv, crit, out) in enumerate(items):
            arr[i] = VolumeDesc(vol.data_ptr(), dtype_of(vol), 0, dims_of(vol), eb_of(ebm, ebv), crit.c(), out.c)
        st = load().roix_fused_batch(self.h, len(items), ctypes.cast(arr, ctypes.c_void_p), _stream(stream))
        _check(st, "roix_fused_batch")

    def quantize(self, vol: torch.Tensor, eb_mode: str, eb_value: float, with_bits: bool = True, stream=None):
        n = vol.numel()
        codes = torch.empty(vol.shape, dtype=torch.int32, device=vol.device)
        bits = torch.empty(((n + 31) // 32,), dtype=torch.int32, device=vol.device) if with_bits else None
        qinfo = torch.zeros(ctypes.sizeof(QuantInfo), dtype=torch.uint8, device=vol.device)
        st = load().roix_quantize(self.h, _ptr(vol), dtype_of(vol), dims_of(vol), eb_of(eb_mode, eb_value),
                                  _ptr(codes), _ptr(bits), _ptr(qinfo), _stream(stream))
        _check(st, "roix_quantize")
        return codes, bits, qinfo

    def segment(self, codes: torch.Tensor, qinfo: torch.Tensor, crit: Criterion, comps_cap: int,
                want_labels: bool = False, stream=None):
        keep = torch.empty(codes.shape, dtype=torch.uint8, device=codes.device)
        labels = torch.empty(codes.shape, dtype=torch.int64, device=codes.device) if want_labels else None
        comps = torch.empty(max(comps_cap, 1) * COMP_BYTES, dtype=torch.uint8, device=codes.device)
        sinfo = torch.zeros(ctypes.sizeof(SegInfo), dtype=torch.uint8, device=codes.device)
        c = crit.c()
        st = load().roix_segment(self.h, _ptr(codes), dims_of(codes), _ptr(qinfo), ctypes.byref(c), _ptr(keep),
                                 _ptr(labels), _ptr(comps), comps_cap, _ptr(sinfo), _stream(stream))
        _check(st, "roix_segment")
        return keep, labels, comps, sinfo

    def extract(self, vol: torch.Tensor, keep: torch.Tensor, qinfo: torch.Tensor, out: Outputs, stream=None):
        st = load().roix_extract(self.h, _ptr(vol), dtype_of(vol), _ptr(keep), dims_of(vol), _ptr(qinfo),
                                 ctypes.byref(out.c), _stream(stream))
        _check(st, "roix_extract")


def parse_info(buf: torch.Tensor, cls):
    return _info(buf, cls)


class Server:
    """Served form: volumes streamed slab by slab into an HBM pool of
    `budget_bytes` on the context's device (see roix_server_create)."""

    def __init__(self, ctx: Context, budget_bytes: int):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.roix_server_create(ctx.h, int(budget_bytes), ctypes.byref(h)), "roix_server_create")
        self.h = h
        self.ctx = ctx  # the context must outlive the server
        self._outs = {}

    def close_server(self):
        if self.h:
            load().roix_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close_server()
        except Exception:
            pass

    def volume_bytes(self, shape, dtype: int, eb_mode: str, eb_value: float, crit: Criterion) -> int:
        nz, ny, nx = shape
        c = crit.c()
        return int(load().roix_server_volume_bytes(self.h, Dims(nx, ny, nz), dtype, eb_of(eb_mode, eb_value),
                                                   ctypes.byref(c)))

    def set_param(self, name: str, value: int):
        _check(load().roix_server_set_param(self.h, name.encode(), int(value)), f"roix_server_set_param({name})")

    def open(self, shape, dtype: int, eb_mode: str, eb_value: float, crit: Criterion, out: Outputs) -> int:
        """Admit a volume of shape (nz, ny, nx); returns its id.  Raises
        RoixError with status EBUSY when the pool has no room now."""
        nz, ny, nx = shape
        c = crit.c()
        vid = ctypes.c_int64()
        _check(load().roix_volume_open(self.h, Dims(nx, ny, nz), dtype, eb_of(eb_mode, eb_value), ctypes.byref(c),
                                       ctypes.byref(out.c), ctypes.byref(vid)), "roix_volume_open")
        self._outs[vid.value] = out  # keep the output buffers alive until close
        return vid.value

    def submit(self, vol_id: int, z0: int, slab: torch.Tensor) -> int:
        """Planes [z0, z0 + slab.shape[0]) from a host (ideally pinned) or
        device tensor; the tensor must stay alive and unchanged until the
        request completes."""
        assert slab.is_contiguous()
        rid = ctypes.c_int64()
        _check(load().roix_slab_submit(self.h, vol_id, z0, slab.shape[0], ctypes.c_void_p(slab.data_ptr()),
                                       1 if slab.is_cuda else 0, ctypes.byref(rid)), "roix_slab_submit")
        return rid.value

    def close(self, vol_id: int) -> int:
        rid = ctypes.c_int64()
        _check(load().roix_volume_close(self.h, vol_id, ctypes.byref(rid)), "roix_volume_close")
        return rid.value

    def abort(self, vol_id: int):
        _check(load().roix_volume_abort(self.h, vol_id), "roix_volume_abort")
        self._outs.pop(vol_id, None)

    def wait(self, req_id: int, timeout_ms: int = -1):
        """ReqResult once the request has completed; None on timeout."""
        res = ReqResult()
        st = load().roix_wait(self.h, req_id, int(timeout_ms), ctypes.byref(res))
        if st == EBUSY:
            return None
        _check(st, "roix_wait")
        if res.kind == REQ_CLOSE:
            self._outs.pop(res.vol_id, None)
        return res

    def stats(self) -> ServerStats:
        s = ServerStats()
        _check(load().roix_server_stats(self.h, ctypes.byref(s)), "roix_server_stats")
        return s
