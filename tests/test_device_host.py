"""Device code of the line engine run on the CPU from the same source:

* the tile element walk (tests/walk_check.hip includes the engine header and
  calls the walk with explicit thread indices): exact coverage of every
  tile's elements, offsets that follow the row-major and 8x4-blocked storage
  formulas and stay inside the patch's storage, and termination, for both
  layouts, both line directions, workgroups of 64..1024 threads and ragged
  tiles;
* the in-register DFT butterflies of every radix the FFT plans use
  (tests/radix_check.hip), prime, prime-factor and Cooley-Tukey, against a
  direct double-precision DFT."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _build_and_run(tmp_path, name):
    exe = tmp_path / name
    cmd = [HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", name + ".hip"),
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:]
    return r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_tile_walk_covers_every_element_in_bounds(tmp_path):
    assert "cases ok" in _build_and_run(tmp_path, "walk_check")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_dft_butterflies_match_direct_dft(tmp_path):
    out = _build_and_run(tmp_path, "radix_check")
    assert out.count(" ok") >= 15 and "FAIL" not in out
