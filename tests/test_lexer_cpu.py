"""The parse kernel's bitmap lexers (ffp_lexer.h: fast_lex and long_lex),
compiled for the host and compared token by token with the byte-by-byte
lexer, which test_device_logic_cpu.py checks against the oracle.  Tokens sit
at random offsets of a tile of random neighbouring bytes; wave-wide votes
are taken alone and with random other lanes (both sides of every uniform
branch)."""

import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

from gen import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2101_11408_amd")


@pytest.fixture(scope="module")
def lexer_check(tmp_path_factory):
    d = tmp_path_factory.mktemp("lexer_check")
    exe = d / "lexer_check"
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(PKG, "csrc"), os.path.join(ROOT, "tests", "host_logic",
                                                         "lexer_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    return str(exe)


def run(exe, toks, flags=0, seed=1):
    with tempfile.NamedTemporaryFile("wb", suffix=".txt", delete=False) as f:
        f.write("\n".join(toks).encode() + b"\n")
        path = f.name
    try:
        res = subprocess.run([exe, path, str(flags), str(seed)], check=True, capture_output=True,
                             text=True)
    finally:
        os.unlink(path)
    lines = res.stdout.strip().splitlines()
    n, bad = map(int, lines[-1].split())
    assert bad == 0, "\n".join(lines[:-1])
    return n


def _tokens(seed):
    rng = np.random.default_rng(seed)
    toks = W.mixed_tokens(rng, 20_000) + W.hard_tokens(rng, 1500)
    toks += W.uniform_shortest(rng, 5000) + W.coordinates(rng, 5000) + W.random_bits_e17(rng, 5000)
    toks += [t for t in W.INVALID_EXAMPLES if t and "\n" not in t]
    # leading zeros of fractions, short and long integers, exponent forms
    toks += ["0." + "0" * int(z) + str(int(v)) for z, v in
             zip(rng.integers(0, 12, 3000), rng.integers(1, 10 ** 17, 3000, dtype=np.int64))]
    toks += [str(int(v)) for v in rng.integers(0, 2 ** 63, 2000, dtype=np.int64)]
    toks += ["%de%d" % (int(v), int(e)) for v, e in
             zip(rng.integers(0, 10 ** 9, 2000), rng.integers(-400, 400, 2000))]
    toks += ["1.045526078145", "0", "-0", ".5", "5.", "+7", "1e5", "1E-05", "00012.50",
             "9999999999999999999", "12345678901234567890", "1.e5", ".e5", "-.5e-3", "0e0"]
    return toks


@pytest.mark.parametrize("flags", [0, 1])
def test_bitmap_lexers_match_byte_lexer(lexer_check, flags):
    n = run(lexer_check, _tokens(61), flags=flags, seed=7 + flags)
    assert n > 80_000
