"""The host's octree and interaction-list code (csrc/tree.cpp) built with
the address and undefined-behaviour sanitizers and run on seeded point sets
(tests/host/tree_check.cpp): the panel permutation, box ranges and spheres,
and that each target group's P2P leaves and accepted M2P boxes cover every
source panel exactly once, every accepted box passing the acceptance test
for every target of the group.  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_tree_and_lists_under_sanitizers(tmp_path):
    exe = str(tmp_path / "tree_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", os.path.join(ROOT, "tests", "host", "tree_check.cpp"),
           os.path.join(ROOT, "paper_1506_03745_amd", "csrc", "tree.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
    assert "0 failures" in r.stdout
