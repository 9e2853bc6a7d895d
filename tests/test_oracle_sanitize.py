"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a
driver (oracle/sanitize_driver.c) runs every oracle entry point on small
inputs -- fused path with every threshold and keep mode, truncated outputs,
non-finite and overflowing inputs, decode with a corrupted table, background
subtraction, the pixel-sequence quantiser and the Huffman stage -- and any
out-of-bounds access, leak or undefined arithmetic fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", ORACLE,
           os.path.join(ORACLE, "sanitize_driver.c"), "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "libasan" in (r.stderr + r.stdout):
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    # a preloaded library of the environment may come before the sanitizer
    # runtime: let ASan accept that order rather than refuse to start
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stderr[-4000:]
    assert "oracle sanitizer run: ok" in run.stdout
