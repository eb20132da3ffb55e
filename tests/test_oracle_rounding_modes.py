"""Pins for the oracle's directed rounding modes (toward zero, toward
+infinity, toward -infinity).  The paper treats round-to-nearest, ties to
even, and notes that the approach extends to the other modes (the footnote
of Section 6); each mode here is checked against something other than the
oracle:

* brute force from the definition over every representable value of tiny
  formats, binary16 and bfloat16: toward -infinity is the largest
  representable value not above v, toward +infinity the smallest not below
  it, toward zero whichever of the two lies between v and zero;
* glibc's strtod / strtof, which honour the rounding mode set by fesetround,
  on decimal and hexadecimal tokens in binary64 and binary32;
* invariants: the nearest value is one of the two directed ones, the two
  coincide exactly when v is representable, and otherwise are neighbours.
"""

import bisect
import ctypes
import ctypes.util
import math
import platform
import struct
from fractions import Fraction

import numpy as np
import pytest

from gen import workloads as W
from oracle import (
    BFLOAT16,
    BINARY16,
    BINARY32,
    BINARY64,
    FLAG_HEX,
    FLAG_ROUND_DOWN,
    FLAG_ROUND_TOWARD_ZERO,
    FLAG_ROUND_UP,
    ROUND_DOWN,
    ROUND_NEAREST,
    ROUND_TOWARD_ZERO,
    ROUND_UP,
    STATUS_INVALID,
    STATUS_OK,
    STATUS_OUT_OF_RANGE,
    parse_token,
    round_decimal,
)
from test_oracle_pins import MINI_FORMATS, _corpus, _representables, _small_format_cases, decode_value

DIRECTED = (ROUND_TOWARD_ZERO, ROUND_UP, ROUND_DOWN)
FLAG_OF = {ROUND_NEAREST: 0, ROUND_TOWARD_ZERO: FLAG_ROUND_TOWARD_ZERO, ROUND_UP: FLAG_ROUND_UP,
           ROUND_DOWN: FLAG_ROUND_DOWN}


# ---------------------------------------------------------------------------
# brute force from the definition
# ---------------------------------------------------------------------------

class _Directed:
    def __init__(self, fmt):
        table = _representables(fmt)
        self.finite = [t[0] for t in table[:-1]]  # non-negative finite values, sorted
        self.two_emax1 = table[-1][0]             # 2^(emax+1)
        self.fmt = fmt

    def _bounds(self, a):
        f = self.finite
        i = bisect.bisect_right(f, a)
        lo = f[i - 1]
        j = bisect.bisect_left(f, a)
        hi = f[j] if j < len(f) else None
        return lo, hi

    def expect(self, v: Fraction, mode: str):
        """(value, status) of rounding v (nonzero) in the mode: value is a
        Fraction or +-inf; status per the IEEE overflow condition and the
        total-underflow rule."""
        neg = v < 0
        a = -v if neg else v
        lo, hi = self._bounds(a)
        # magnitudes of the two neighbours of v on the number line
        if mode == ROUND_TOWARD_ZERO:
            mag_down = True
        elif mode == ROUND_UP:
            mag_down = neg          # toward +inf lowers the magnitude of negatives
        else:
            mag_down = not neg
        if mag_down:
            r, overflow = lo, a >= self.two_emax1
        else:
            r, overflow = hi, hi is None
        val = math.inf if r is None else r
        st = STATUS_OUT_OF_RANGE if overflow or val == 0 else STATUS_OK
        return (-val if neg else val), st


def _check(fmt, D, E, mode, brute):
    v = Fraction(D) * Fraction(10) ** E
    for neg in (False, True):
        bits, st = round_decimal(neg, D, E, fmt, mode)
        got = decode_value(bits, fmt)
        assert bool(bits & fmt.sign_bit) == neg, (D, E, mode)
        if D == 0:
            assert got == 0 and st == STATUS_OK
            continue
        want, wst = brute.expect(-v if neg else v, mode)
        assert got == want, (fmt.name, mode, neg, D, E, got, want)
        assert st == wst, (fmt.name, mode, neg, D, E, st, wst)


@pytest.mark.parametrize("fmt", MINI_FORMATS, ids=lambda f: f.name)
@pytest.mark.parametrize("mode", DIRECTED)
def test_bruteforce_mini_formats(fmt, mode):
    brute = _Directed(fmt)
    rng = np.random.default_rng(4321)
    cases = [(D, E) for D in range(0, 700) for E in range(-7, 3)]
    cases += [(int(d), int(e)) for d, e in zip(rng.integers(0, 10 ** 7, 2000),
                                               rng.integers(-14, 3, 2000))]
    # every representable value in decimal, and one unit of a far digit on
    # either side of it
    for x in brute.finite[1:]:
        k = x.denominator.bit_length() - 1
        D, E = x.numerator * 5 ** k, -k
        cases += [(D, E), (D * 1000 + 1, E - 3), (D * 1000 - 1, E - 3)]
    for D, E in cases:
        _check(fmt, D, E, mode, brute)


@pytest.mark.parametrize("fmt,stride", [(BINARY16, 2), (BFLOAT16, 5)],
                         ids=["binary16", "bfloat16"])
@pytest.mark.parametrize("mode", DIRECTED)
def test_bruteforce_half_formats(fmt, stride, mode):
    _, _, cases = _small_format_cases(fmt, 98, stride)
    brute = _Directed(fmt)
    for D, E in cases:
        _check(fmt, D, E, mode, brute)


# ---------------------------------------------------------------------------
# glibc strtod / strtof under fesetround
# ---------------------------------------------------------------------------

# <fenv.h> rounding-mode constants of x86-64 (the x87 / SSE rounding-control
# encodings)
_FE = {ROUND_NEAREST: 0x000, ROUND_DOWN: 0x400, ROUND_UP: 0x800, ROUND_TOWARD_ZERO: 0xC00}


@pytest.fixture(scope="module")
def glibc():
    if platform.machine() != "x86_64":
        pytest.skip("rounding-mode constants are those of x86-64")
    libc = ctypes.CDLL(ctypes.util.find_library("c"))
    libm = ctypes.CDLL(ctypes.util.find_library("m"))
    libc.strtod.restype = ctypes.c_double
    libc.strtod.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_char_p)]
    libc.strtof.restype = ctypes.c_float
    libc.strtof.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_char_p)]
    libm.fesetround.argtypes = [ctypes.c_int]
    libm.fegetround.restype = ctypes.c_int

    def parse(tok: bytes, mode: str, single: bool):
        end = ctypes.c_char_p()
        assert libm.fesetround(_FE[mode]) == 0
        try:
            assert libm.fegetround() == _FE[mode]
            v = (libc.strtof if single else libc.strtod)(tok, ctypes.byref(end))
        finally:
            libm.fesetround(0)
        if single:
            return struct.unpack("<I", struct.pack("<f", v))[0]
        return struct.unpack("<Q", struct.pack("<d", v))[0]

    return parse


def _overflow_underflow_tokens(rng, n):
    toks = []
    for _ in range(n):
        k = int(rng.integers(0, 4))
        d = "".join(str(int(x)) for x in rng.integers(0, 10, int(rng.integers(1, 30))))
        d = d.lstrip("0") or "1"
        if k == 0:
            toks.append("%s.%se%d" % (d[0], d[1:] or "0", int(rng.integers(300, 320))))
        elif k == 1:
            toks.append("%s.%se%d" % (d[0], d[1:] or "0", int(rng.integers(-345, -300))))
        elif k == 2:
            toks.append("%s.%se%d" % (d[0], d[1:] or "0", int(rng.integers(36, 41))))
        else:
            toks.append("%s.%se%d" % (d[0], d[1:] or "0", int(rng.integers(-50, -35))))
        if rng.integers(0, 2):
            toks[-1] = "-" + toks[-1]
    return toks


def _glibc_corpus(seed):
    rng = np.random.default_rng(seed)
    toks = _corpus(n_each=800, seed=seed)
    toks += [t.encode() for t in _overflow_underflow_tokens(rng, 1500)]
    toks += [b"1.7976931348623157e308", b"1.7976931348623158e308", b"1.797693134862315807e308",
             b"1.7976931348623159e308", b"3.4028234663852886e38", b"3.4028235677973366e38",
             b"4.9e-324", b"2.4703282292062327e-324", b"2.4703282292062328e-324",
             b"1.4e-45", b"7.006492321624085e-46", b"0.1", b"-0.1", b"1", b"-1"]
    return toks


@pytest.mark.parametrize("mode", DIRECTED)
def test_binary64_matches_glibc_strtod(glibc, mode):
    n = 0
    for tok in _glibc_corpus(31):
        bits, st = parse_token(tok, BINARY64, FLAG_OF[mode])
        assert st != STATUS_INVALID, tok
        assert bits == glibc(tok, mode, False), (mode, tok, hex(bits))
        n += 1
    assert n > 4000


@pytest.mark.parametrize("mode", DIRECTED)
def test_binary32_matches_glibc_strtof(glibc, mode):
    for tok in _glibc_corpus(32):
        bits, st = parse_token(tok, BINARY32, FLAG_OF[mode])
        assert bits == glibc(tok, mode, True), (mode, tok, hex(bits))


@pytest.mark.parametrize("mode", DIRECTED)
def test_hex_tokens_match_glibc(glibc, mode):
    """strtod / strtof read hexadecimal floating-point tokens too."""
    rng = np.random.default_rng(33)
    for tok in W.hex_tokens(rng, 4000):
        t = tok.encode()
        b64, _ = parse_token(t, BINARY64, FLAG_HEX | FLAG_OF[mode])
        b32, _ = parse_token(t, BINARY32, FLAG_HEX | FLAG_OF[mode])
        assert b64 == glibc(t, mode, False), (mode, tok, hex(b64))
        assert b32 == glibc(t, mode, True), (mode, tok, hex(b32))


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------

def test_directed_bracket_nearest():
    """RD(v) <= v <= RU(v) as neighbouring encodings (equal iff exact), the
    nearest result is one of them, toward zero picks the one nearer zero,
    and toward +inf of -v is minus toward -inf of v."""
    for tok in _corpus(n_each=600, seed=34):
        for fmt in (BINARY64, BINARY32):
            bn, sn = parse_token(tok, fmt, 0)
            bz, _ = parse_token(tok, fmt, FLAG_ROUND_TOWARD_ZERO)
            bu, _ = parse_token(tok, fmt, FLAG_ROUND_UP)
            bd, _ = parse_token(tok, fmt, FLAG_ROUND_DOWN)
            neg = tok.startswith(b"-")
            # magnitude order of encodings: for a sign, a larger encoding is a
            # larger magnitude
            lo, hi = (bu, bd) if neg else (bd, bu)
            assert hi - lo in (0, 1), (tok, fmt.name)
            assert bn in (lo, hi)
            assert bz == lo
            mtok = tok[1:] if neg else b"-" + tok.lstrip(b"+")
            mu, _ = parse_token(mtok, fmt, FLAG_ROUND_UP)
            assert mu == bd ^ fmt.sign_bit, (tok, fmt.name)
