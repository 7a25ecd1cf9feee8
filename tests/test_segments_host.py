"""Host logic of the segment layout (the cut of the sorted surfels into
segments of at most 5 nodes, their pair masks, the block entries and the
packs), built with AddressSanitizer and UBSan from the library's own source
and checked property by property on constructed and random node sets."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1904_13073_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_segment_layout_properties(tmp_path):
    exe = str(tmp_path / "segments_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I" + CSRC, os.path.join(CSRC, "segments.cpp"),
           os.path.join(ROOT, "tests", "host", "segments_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.strip().endswith("ok")
