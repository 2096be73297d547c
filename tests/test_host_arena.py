"""The serving loop's arena allocator (paper_1101_0265_amd/csrc/arena.h), checked on the CPU
against a brute-force model of the range (tests/host/arena_check.cpp: first fit, 256-byte
alignment, no overlap, coalesced free list, success exactly when a free run fits), built with
AddressSanitizer and UndefinedBehaviorSanitizer."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "arena_check.cpp")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("arena") / "arena_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


@pytest.mark.parametrize("seed", [1, 2, 3, 17, 1234])
def test_arena_matches_model(checker, seed):
    r = subprocess.run([checker, str(seed), "20000"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    ok, n_alloc, n_fail = r.stdout.split()
    assert ok == "ok" and int(n_alloc) > 1000 and int(n_fail) > 0   # both paths exercised
