"""The host geometry tables of the engine (csrc/geometry.cpp: validation of
the solid mask and cut links, the link sort, the per-node and per-wave
tables) built with g++ under the address and undefined-behaviour sanitizers
and driven by tests/host/geometry_sanitize.cpp on seeded random geometries,
valid and invalid (no GPU: the unit has no HIP code)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1712_08288_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_geometry_tables_under_sanitizers(tmp_path):
    exe = str(tmp_path / "geometry_sanitize")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(CSRC, "geometry.cpp"),
           os.path.join(ROOT, "tests", "host", "geometry_sanitize.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ)
    # a preloaded library ahead of the sanitizer runtime is tolerated
    env["ASAN_OPTIONS"] = "verify_asan_link_order=0:detect_leaks=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert out.startswith("ok:"), out[-2000:]
