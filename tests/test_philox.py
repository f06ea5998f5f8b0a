"""Pins the oracle's Philox4x32-10 (Salmon et al., SC'11).

Two independent pins: the published known-answer block for the all-zero
counter and key, and rocRAND's Philox4x32-10 engine (a library
implementation of the same generator) run as a host program on random
counters and keys.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import core

HERE = os.path.dirname(os.path.abspath(__file__))


def test_zero_counter_known_answer():
    assert core.philox(0, [0, 0, 0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]


@pytest.fixture(scope="module")
def rocrand_helper(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND host helper")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_philox")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-I/opt/rocm/include", "-o", exe,
                    os.path.join(HERE, "helpers", "rocrand_philox.cpp")], check=True, capture_output=True)
    return exe


def test_matches_rocrand(rocrand_helper):
    rng = np.random.default_rng(11)
    n = 2000
    keys = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64)
    ctrs = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64)
    ctrs[:, 1] %= 2 ** 30          # the engine reaches counter word 1 only below 2^30 via its offset
    ctrs[:10] = 0
    ctrs[10:20, 0] = 2 ** 32 - 1   # carries are not part of the block function: spot the extremes
    lines = "\n".join(" ".join(str(int(x)) for x in list(k) + list(c)) for k, c in zip(keys, ctrs))
    res = subprocess.run([rocrand_helper], input=lines, capture_output=True, text=True, check=True)
    ref = np.array([[int(x) for x in l.split()] for l in res.stdout.strip().splitlines()], dtype=np.uint64)
    for i in range(n):
        key = int(keys[i, 0]) | (int(keys[i, 1]) << 32)
        assert core.philox(key, [int(x) for x in ctrs[i]]) == ref[i].tolist()
