"""Pins of the oracle's exact sum (oracle/reduce.py) against CPython's
math.fsum (a correctly rounded sum of binary64 values), IEEE special cases
and numpy's decoding of each format."""

import math
import struct
from fractions import Fraction

import numpy as np
import pytest

from oracle import reduce as R

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def f64_bits(x: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def random_doubles(rng, n):
    """Values over the whole exponent range, both signs, subnormals,
    near-cancelling pairs and exact halves."""
    out = []
    for _ in range(n):
        k = rng.integers(0, 6)
        if k == 0:
            out.append(float(rng.standard_normal()))
        elif k == 1:
            out.append(float(rng.standard_normal()) * 10.0 ** int(rng.integers(-300, 300)))
        elif k == 2:  # subnormals
            out.append(float(rng.integers(-(1 << 52), 1 << 52)) * 5e-324)
        elif k == 3:
            x = float(rng.uniform(0, 1))
            out += [x, -x * (1 + 2.0 ** -52)]
        elif k == 4:
            out.append(math.ldexp(float(rng.integers(1, 1 << 53)), int(rng.integers(-1074, 970))))
        else:
            out.append(float(rng.uniform(-1, 1)))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_sum_matches_fsum(seed):
    rng = np.random.default_rng(seed)
    n = [1, 2, 3, 40, 500, 3000][seed]
    xs = random_doubles(rng, n)
    bits = [f64_bits(x) for x in xs]
    got, exact = R.exact_sum(bits, [0] * len(bits), "f64")
    want = math.fsum(xs)
    assert got == f64_bits(want) or (want == 0 and got in (0, 1 << 63)), (seed, hex(got), want)
    assert exact == (sum(Fraction(x) for x in xs) == Fraction(want))


def test_sum_ties_round_to_even():
    # 1 + 2^-53 is a tie between 1 and 1 + 2^-52: even (1); 1 + 2^-52 + 2^-53
    # ties to 1 + 2^-51; a sticky bit beyond the tie rounds up
    one = f64_bits(1.0)
    u = f64_bits(2.0 ** -53)
    assert R.exact_sum([one, u], [0, 0]) == (one, False)
    assert R.exact_sum([f64_bits(1 + 2.0 ** -52), u], [0, 0]) == (f64_bits(1 + 2.0 ** -51), False)
    assert R.exact_sum([one, u, f64_bits(2.0 ** -1074)], [0, 0, 0]) == (
        f64_bits(1 + 2.0 ** -52), False)


def test_sum_special_cases():
    inf, ninf = R.INF64, R.INF64 | R.SIGN64
    one = f64_bits(1.0)
    big = f64_bits(1.7976931348623157e308)
    assert R.exact_sum([big, big], [0, 0]) == (inf, False)  # overflow
    assert R.exact_sum([big, big, f64_bits(-1.7976931348623157e308)], [0, 0, 0]) == (big, True)
    assert R.exact_sum([one, inf], [0, 0]) == (inf, True)
    assert R.exact_sum([ninf, one], [0, 0]) == (ninf, True)
    assert R.exact_sum([inf, ninf], [0, 0])[0] == R.QNAN64
    assert R.exact_sum([R.QNAN64, one], [0, 0]) == (one, True)  # NaN encodings skipped
    assert R.exact_sum([one, one], [0, 1]) == (one, True)  # status other than OK skipped
    assert R.exact_sum([], []) == (0, True)
    assert R.exact_sum([R.SIGN64, R.SIGN64], [0, 0]) == (R.SIGN64, True)  # -0 + -0
    assert R.exact_sum([R.SIGN64, 0], [0, 0]) == (0, True)
    assert R.exact_sum([one, f64_bits(-1.0)], [0, 0]) == (0, True)
    # subnormals add exactly
    assert R.exact_sum([1, 1], [0, 0]) == (2, True)
    assert R.exact_sum([f64_bits(1e308), f64_bits(-1e308), f64_bits(1e-300)], [0] * 3) == (
        f64_bits(1e-300), True)


@pytest.mark.parametrize("fmt,npdt,width", [("f32", np.float32, 32), ("f16", np.float16, 16)])
def test_decode_matches_numpy(fmt, npdt, width):
    rng = np.random.default_rng(width)
    raw = rng.integers(0, 1 << width, 4000, dtype=np.uint64)
    raw = np.concatenate([raw, np.array([0, 1, (1 << (width - 1)), (1 << (width - 1)) + 1],
                                        dtype=np.uint64)])
    vals = raw.astype({32: np.uint32, 16: np.uint16}[width]).view(npdt).astype(np.float64)
    for b, v in zip(raw.tolist(), vals.tolist()):
        kind, neg, x = R.decode(int(b), fmt)
        if v != v:
            assert kind == "nan"
        elif math.isinf(v):
            assert kind == "inf" and neg == (v < 0)
        else:
            assert kind == "finite" and x == Fraction(v) and neg == (math.copysign(1, v) < 0)


def test_decode_bfloat16_is_the_top_half_of_binary32():
    rng = np.random.default_rng(7)
    for b in rng.integers(0, 1 << 16, 3000).tolist():
        v = float(np.array([b << 16], dtype=np.uint32).view(np.float32)[0])
        kind, neg, x = R.decode(int(b), "bf16")
        if v != v:
            assert kind == "nan"
        elif math.isinf(v):
            assert kind == "inf"
        else:
            assert x == Fraction(v)


def test_sum_of_narrow_formats_is_rounded_to_binary64():
    # binary32 values convert exactly to binary64: fsum over them is the pin
    rng = np.random.default_rng(9)
    xs = (rng.standard_normal(2000) * 10.0 ** rng.integers(-30, 30, 2000)).astype(np.float32)
    bits = xs.view(np.uint32).astype(np.uint64).tolist()
    got, _ = R.exact_sum(bits, [0] * len(bits), "f32")
    assert got == f64_bits(math.fsum(xs.astype(np.float64).tolist()))
    h = rng.standard_normal(500).astype(np.float16)
    hb = h.view(np.uint16).astype(np.uint64).tolist()
    got, exact = R.exact_sum(hb, [0] * len(hb), "f16")
    assert got == f64_bits(math.fsum(h.astype(np.float64).tolist())) and exact
