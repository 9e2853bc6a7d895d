"""The C-ABI library loads, exports every function include/roix.h declares,
its struct layouts match the Python binding, and argument errors come back
synchronously (no GPU needed: nothing here launches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "roix.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2602_15917_amd import roix
    return roix, roix.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(roix_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_path_calls():
    names = declared_functions()
    for n in ("roix_quantize", "roix_segment", "roix_extract", "roix_fused", "roix_ctx_create",
              "roix_ctx_destroy", "roix_scratch_bytes", "roix_bounds", "roix_decode", "roix_background", "roix_fused_background",
              "roix_abs_quantize", "roix_huff_encode", "roix_huff_decode",
              "roix_autotune"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    _, L = lib
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_struct_sizes_match_binding(lib):
    roix, L = lib
    L.roix_sizeof.argtypes = [ctypes.c_char_p]
    L.roix_sizeof.restype = ctypes.c_size_t
    for name, cls in (("roix_quant_info", roix.QuantInfo), ("roix_seg_info", roix.SegInfo),
                      ("roix_extract_info", roix.ExtractInfo), ("roix_fused_out", roix.FusedOut),
                      ("roix_criterion", roix.CCriterion), ("roix_eb", roix.Eb), ("roix_dims", roix.Dims),
                      ("roix_volume_desc", roix.VolumeDesc), ("roix_req_result", roix.ReqResult),
                      ("roix_server_stats_t", roix.ServerStats), ("roix_decode_info", roix.DecodeInfo),
                      ("roix_absq_info", roix.AbsqInfo), ("roix_huff_info", roix.HuffInfo),
                      ("roix_tune_result", roix.TuneResult)):
        assert L.roix_sizeof(name.encode()) == ctypes.sizeof(cls), name
    assert L.roix_sizeof(b"roix_component") == roix.COMP_BYTES == 48
    assert L.roix_sizeof(b"roix_row") == roix.ROW_BYTES == 32
    assert L.roix_sizeof(b"nope") == 0


def test_oracle_struct_layouts_match_library(lib):
    import oracle
    roix, L = lib
    L.roix_sizeof.argtypes = [ctypes.c_char_p]
    L.roix_sizeof.restype = ctypes.c_size_t
    assert oracle.COMP_DTYPE.itemsize == L.roix_sizeof(b"roix_component")
    assert oracle.ROW_DTYPE.itemsize == L.roix_sizeof(b"roix_row")


def test_sync_argument_errors(lib):
    roix, L = lib
    d = roix.Dims(8, 8, 8)
    eb = roix.Eb(roix.EB_ABS, 0, 1e-3)
    c = roix.Criterion().c()
    out = roix.FusedOut()
    null = ctypes.c_void_p(0)
    # null context / input
    assert L.roix_fused(null, null, roix.F32, d, eb, ctypes.byref(c), ctypes.byref(out), null) == roix.EINVAL
    assert L.roix_fused_noalloc(null, roix.F32, d, eb, ctypes.byref(c), ctypes.byref(out), null) == roix.EINVAL
    # beyond the fixed scratch array: refused before any device call
    big = roix.Dims(200, 200, 200)
    assert roix.scratch_bytes(big, roix.F32) > roix.NOALLOC_SCRATCH_BYTES
    fake = ctypes.c_void_p(1 << 20)
    assert L.roix_fused_noalloc(fake, roix.F32, big, eb, ctypes.byref(c), ctypes.byref(out), null) == roix.ENOMEM
    assert L.roix_quantize(null, null, roix.F32, d, eb, null, null, null, null) == roix.EINVAL
    assert L.roix_segment(null, null, d, null, ctypes.byref(c), null, null, null, 0, null, null) == roix.EINVAL
    assert L.roix_extract(null, null, roix.F32, null, d, null, ctypes.byref(out), null) == roix.EINVAL
    assert L.roix_ctx_destroy(null) == roix.EINVAL
    assert L.roix_ctx_set_timing(null, 1) == roix.EINVAL
    # served form
    h = ctypes.c_void_p()
    i = ctypes.c_int64()
    assert L.roix_server_create(null, 1 << 20, ctypes.byref(h)) == roix.EINVAL
    assert L.roix_server_destroy(null) == roix.EINVAL
    assert L.roix_volume_open(null, d, roix.F32, eb, ctypes.byref(c), ctypes.byref(out), ctypes.byref(i)) == roix.EINVAL
    assert L.roix_slab_submit(null, 1, 0, 1, null, 0, ctypes.byref(i)) == roix.EINVAL
    assert L.roix_volume_close(null, 1, ctypes.byref(i)) == roix.EINVAL
    assert L.roix_volume_abort(null, 1) == roix.EINVAL
    assert L.roix_wait(null, 1, 0, ctypes.byref(roix.ReqResult())) == roix.EINVAL
    assert L.roix_server_stats(null, ctypes.byref(roix.ServerStats())) == roix.EINVAL
    assert L.roix_decode(null, null, 0, null, 0, null, 0, null, null, d, 0.0, null, null, null) == roix.EINVAL
    assert L.roix_background(null, null, roix.F32, d, null, 1, 0, null, null) == roix.EINVAL
    assert L.roix_abs_quantize(null, null, 0, 1.0, null, null, null) == roix.EINVAL
    # section: checked before any device call (a non-null stand-in context)
    assert L.roix_section(null, fake, roix.F32, d, ctypes.byref(out), fake, 16, fake, null) == roix.EINVAL
    so = roix.FusedOut(0, 0, 0, 64, 0, 0, 0, 0, 1 << 20, 0, 1 << 21, None)
    assert L.roix_section(fake, fake, roix.F32, d, ctypes.byref(so), fake, 16, fake, null) == roix.EINVAL  # stream
    so = roix.FusedOut(0, 0, 1 << 20, 64, 0, 0, 0, 0, 0, 0, 1 << 21, None)
    assert L.roix_section(fake, fake, roix.F32, d, ctypes.byref(so), fake, 16, fake, null) == roix.EINVAL  # qinfo
    so = roix.FusedOut(0, 0, (1 << 20) + 4, 64, 0, 0, 0, 0, 1 << 20, 0, 1 << 21, None)
    assert L.roix_section(fake, fake, roix.F32, d, ctypes.byref(so), fake, 16, fake, null) == roix.EINVAL  # align
    so = roix.FusedOut(0, 0, 1 << 20, 64, 0, 0, 0, 0, 1 << 20, 0, 1 << 21, None)
    assert L.roix_section(fake, fake, roix.F32, d, ctypes.byref(so), (1 << 20) + 8, 16, fake, null) == roix.EINVAL
    assert L.roix_section(fake, fake, roix.F32, d, ctypes.byref(so), fake, -1, fake, null) == roix.EINVAL
    assert L.roix_section(fake, fake, 7, d, ctypes.byref(so), fake, 16, fake, null) == roix.EINVAL
    assert L.roix_huff_encode(null, null, 0, null, null, null, null, 0, null, null) == roix.EINVAL
    assert L.roix_huff_decode(null, null, null, null, null, 0, 0, null, null, null) == roix.EINVAL
    assert L.roix_autotune(null, null, roix.F32, d, eb, ctypes.byref(c), ctypes.byref(out), 1, None,
                           ctypes.byref(roix.TuneResult()), null) == roix.EINVAL


def test_served_calls_without_server(lib):
    roix, L = lib
    null = ctypes.c_void_p(0)
    c = roix.Criterion(thr="fixed", fixed_value=0.5).c()
    eb = roix.Eb(roix.EB_ABS, 0, 1e-3)
    assert L.roix_server_volume_bytes(null, roix.Dims(8, 8, 8), roix.F32, eb, ctypes.byref(c)) == 0
    assert L.roix_server_set_param(null, b"runs_per_row", 8) == roix.EINVAL


def test_sizes_and_bounds(lib):
    roix, L = lib
    d = roix.Dims(1024, 1024, 1024)
    c26 = roix.Criterion(connectivity=26)
    n = roix.scratch_bytes(d, roix.F32, c26)
    N = 1024 ** 3
    assert n > N + N // 8 and n < 20 * N
    assert roix.scratch_bytes(roix.Dims(0, 4, 4), roix.F32, c26) == 0
    assert roix.scratch_bytes(roix.Dims(1 << 12, 1 << 11, 1 << 11), roix.F32, c26) == 0  # > 2^33 voxels
    b = roix.bounds(d, roix.F32, c26)
    assert b == {"rows": 1024 * 1024, "stream_bytes": 4 * N, "outliers": N, "components": 512 ** 3}
    assert roix.bounds(roix.Dims(3, 3, 3), roix.U16, roix.Criterion(connectivity=6))["components"] == 27
    with pytest.raises(roix.RoixError):
        roix.bounds(roix.Dims(-1, 3, 3), roix.F32, c26)


def test_status_strings_and_stages(lib):
    roix, L = lib
    for s in range(8):
        assert L.roix_status_string(s)
    names = roix.stage_names()
    assert "quant_hist" in names and "emit" in names and len(names) == L.roix_stage_count()


def test_bin_division_forms_exact(tmp_path):
    # the kernels' multiply-high forms of floor(256 u / K), checked for every
    # K <= 65536 and u < K by a small C program
    import subprocess
    src = os.path.join(os.path.dirname(__file__), "bin_division_check.c")
    exe = str(tmp_path / "bin_division_check")
    subprocess.run(["gcc", "-O2", "-o", exe, src], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout
    assert r.stdout.split()[:2] == ["max_k24", "46340"], r.stdout
