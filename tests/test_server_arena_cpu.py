"""The request server's device-memory arena (ffp_arena.h), compiled for the
host and checked against a byte-map model: first-fit placement, no overlap,
coalesced free ranges, used and peak byte counts.  No GPU involved."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def arena_check(tmp_path_factory):
    exe = tmp_path_factory.mktemp("arena") / "arena_check"
    subprocess.run(["g++", "-O2", "-std=c++17",
                    "-I", os.path.join(ROOT, "paper_2101_11408_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host_logic", "arena_check.cpp"),
                    "-o", str(exe)], check=True, capture_output=True)
    return str(exe)


@pytest.mark.parametrize("size,steps,seed", [(4096, 100_000, 1), (300, 100_000, 2),
                                             (1 << 14, 20_000, 3), (1, 1000, 4)])
def test_arena_matches_model(arena_check, size, steps, seed):
    res = subprocess.run([arena_check, str(size), str(steps), str(seed)],
                         capture_output=True, text=True)
    assert res.returncode == 0 and res.stdout.startswith("ok"), res.stdout
