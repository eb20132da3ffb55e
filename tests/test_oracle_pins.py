"""Pins for the CPU oracle: every check here compares the oracle with something
other than itself -- values the paper prints, brute force over tiny formats,
CPython's correctly rounded float(), glibc strtof, closed forms and
invariants.  None of these tests touch the GPU path."""

import bisect
import ctypes
import math
import os
import struct
from fractions import Fraction

import numpy as np
import pytest

from oracle import (
    BFLOAT16,
    BINARY16,
    BINARY32,
    BINARY64,
    FLAG_REJECT_PLUS,
    Format,
    STATUS_INVALID,
    STATUS_OK,
    STATUS_OUT_OF_RANGE,
    decompose,
    parse_buffer,
    parse_token,
    round_decimal,
    split_tokens,
)
from gen import workloads as W


# ---------------------------------------------------------------------------
# independent helpers (decoding only; no rounding)
# ---------------------------------------------------------------------------

def decode_value(bits: int, fmt: Format):
    """Exact value of an encoding as a Fraction, or +-inf as a float."""
    sign = -1 if bits & fmt.sign_bit else 1
    field = (bits >> (fmt.p - 1)) & ((1 << fmt.ebits) - 1)
    frac = bits & ((1 << (fmt.p - 1)) - 1)
    if field == (1 << fmt.ebits) - 1:
        assert frac == 0
        return sign * math.inf
    if field == 0:
        m, e = frac, fmt.emin - fmt.p + 1
    else:
        m, e = frac | (1 << (fmt.p - 1)), field - fmt.bias - fmt.p + 1
    return sign * Fraction(m) * (Fraction(2) ** e)


def f64_bits(x: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def f32_bits_from_strtof(s: bytes):
    libc = ctypes.CDLL("libc.so.6")
    libc.strtof.restype = ctypes.c_float
    libc.strtof.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_char_p)]
    end = ctypes.c_char_p()
    v = libc.strtof(s, ctypes.byref(end))
    return struct.unpack("<I", struct.pack("<f", v))[0]


def load_tsv(path):
    rows = []
    with open(path, encoding="utf-8") as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            rows.append(line.rstrip("\n").split("\t"))
    return rows


# ---------------------------------------------------------------------------
# values the paper prints
# ---------------------------------------------------------------------------

def test_paper_worked_examples(golden_dir):
    rows = load_tsv(os.path.join(golden_dir, "paper_examples.tsv"))
    assert len(rows) >= 20
    for tok, fmtname, kind, expected, cite in rows:
        fmt = BINARY64 if fmtname == "f64" else BINARY32
        bits, st = parse_token(tok.encode(), fmt)
        assert st == STATUS_OK, (tok, cite)
        val = decode_value(bits, fmt)
        neg, D, E = decompose(tok.encode())
        exact = Fraction(D) * Fraction(10) ** E
        if kind == "m_p":
            m, p = map(int, expected.split())
            assert val == Fraction(m) * Fraction(2) ** p, (tok, cite)
        elif kind == "hex":
            assert val == Fraction(float.fromhex(expected)), (tok, cite)
        elif kind == "int":
            assert val == int(expected), (tok, cite)
        elif kind == "sig":
            m = int(expected)
            assert m.bit_length() == fmt.p
            # the value must be m times a power of two
            ratio = val / m
            assert ratio.numerator == 1 or ratio.denominator == 1
            r = ratio.numerator if ratio.denominator == 1 else ratio.denominator
            assert r & (r - 1) == 0, (tok, cite)
        elif kind == "exact":
            assert val == exact, (tok, cite)
        elif kind == "inexact":
            assert val != exact, (tok, cite)
        else:
            raise AssertionError(kind)


def _exact_decimal_string(num: int, e2: int) -> bytes:
    """num * 2^e2 written exactly in decimal (e2 < 0): num*5^-e2 e e2."""
    assert e2 < 0
    return b"%de%d" % (num * 5 ** (-e2), e2)


def test_paper_subnormal_examples():
    # Section 9.3: (2^53-1) * 2^(-1022-54) becomes 2^51 * 2^(-1022-52)
    tok = _exact_decimal_string(2 ** 53 - 1, -1022 - 54)
    bits, st = parse_token(tok, BINARY64)
    assert st == STATUS_OK
    assert decode_value(bits, BINARY64) == Fraction(2) ** 51 * Fraction(2) ** (-1074)
    assert bits == 2 ** 51
    # Section 9.3: (2^53-1) * 2^(-1022-53) rounds up to the smallest normal
    tok = _exact_decimal_string(2 ** 53 - 1, -1022 - 53)
    bits, st = parse_token(tok, BINARY64)
    assert st == STATUS_OK
    assert decode_value(bits, BINARY64) == Fraction(2) ** (-1022)


def test_paper_768_digit_midpoint():
    # Section 11: the midpoint 2^-1022 + 2^-1074 + 2^-1075 needs 768
    # significant digits and rounds to the even neighbour, the larger value.
    num = 2 ** 53 + 2 + 1  # (2^-1022 + 2^-1074 + 2^-1075) * 2^1075
    digits = str(num * 5 ** 1075).rstrip("0")
    assert len(digits) == 768
    tok = _exact_decimal_string(num, -1075)
    bits, st = parse_token(tok, BINARY64)
    assert st == STATUS_OK
    assert decode_value(bits, BINARY64) == Fraction(2) ** -1022 + Fraction(2) ** -1073
    assert float.fromhex("0x1.0000000000002p-1022") == struct.unpack(
        "<d", struct.pack("<Q", bits))[0]
    # every truncation of those digits is closer to the lower neighbour
    for keep in (17, 19, 100, 400, 767):
        t = (digits[:keep] + "e%d" % (len(str(num * 5 ** 1075)) - keep - 1075)).encode()
        b2, _ = parse_token(t, BINARY64)
        assert decode_value(b2, BINARY64) == Fraction(2) ** -1022 + Fraction(2) ** -1074


def test_exact_numbers_section6():
    # Section 6: w*10^q can be exact only for q in [-27, 22] (binary64).
    for q in range(0, 23):
        bits, _ = parse_token(b"1e%d" % q, BINARY64)
        assert decode_value(bits, BINARY64) == 10 ** q
    bits, _ = parse_token(b"1e23", BINARY64)
    assert decode_value(bits, BINARY64) != 10 ** 23
    for q in range(1, 28):
        w = 5 ** q  # w * 10^-q = 2^-q exactly
        bits, _ = parse_token(b"%de-%d" % (w, q), BINARY64)
        assert decode_value(bits, BINARY64) == Fraction(1, 2 ** q)


def test_exponent_of_ten_formula_section10():
    # Section 10: the binary exponent of 10^q is q + floor(log2 5^q); the
    # oracle's result for 10^q must have that leading exponent.
    for q in range(-300, 300, 7):
        bits, _ = parse_token(b"1e%d" % q, BINARY64)
        field = (bits >> 52) & 0x7FF
        if q >= 0:
            expect = q + (5 ** q).bit_length() - 1
        else:
            p5 = 5 ** (-q)
            expect = q - (p5.bit_length() - (1 if p5 & (p5 - 1) == 0 else 0))
        assert field - 1023 == expect


# ---------------------------------------------------------------------------
# brute force over tiny formats
# ---------------------------------------------------------------------------

MINI_FORMATS = [
    Format("mini3", 3, -2, 3, 3),
    Format("mini4", 4, -6, 7, 4),
    Format("mini5", 5, -14, 15, 5),
]


def _representables(fmt: Format):
    """Sorted list of (value, significand) for every finite non-negative
    number of the format, plus infinity as the even virtual value 2^(emax+1)."""
    out = [(Fraction(0), 0)]
    q0 = fmt.emin - fmt.p + 1
    for m in range(1, 1 << (fmt.p - 1)):
        out.append((Fraction(m) * Fraction(2) ** q0, m))
    for e in range(fmt.emin, fmt.emax + 1):
        for m in range(1 << (fmt.p - 1), 1 << fmt.p):
            out.append((Fraction(m) * Fraction(2) ** (e - fmt.p + 1), m))
    out.append((Fraction(2) ** (fmt.emax + 1), 0))  # infinity, even
    out.sort()
    return out


def _brute_nearest(v: Fraction, table, keys):
    i = bisect.bisect_left(keys, v)
    if i < len(keys) and keys[i] == v:
        return keys[i]
    if i >= len(keys):
        return keys[-1]
    lo, hi = table[i - 1], table[i]
    dl, dh = v - lo[0], hi[0] - v
    if dl < dh:
        return lo[0]
    if dh < dl:
        return hi[0]
    return lo[0] if lo[1] % 2 == 0 else hi[0]


@pytest.mark.parametrize("fmt", MINI_FORMATS, ids=lambda f: f.name)
def test_bruteforce_mini_format(fmt):
    table = _representables(fmt)
    keys = [t[0] for t in table]
    inf_value = keys[-1]
    rng = np.random.default_rng(1234)
    cases = [(D, E) for D in range(0, 1200) for E in range(-7, 3)]
    cases += [(int(d), int(e)) for d, e in zip(rng.integers(0, 10 ** 7, 3000),
                                               rng.integers(-14, 3, 3000))]
    # exact midpoints of neighbouring representables, written in decimal
    for (a, _), (b, _) in zip(table[:-1], table[1:]):
        mid = (a + b) / 2
        den = mid.denominator
        k = den.bit_length() - 1  # den is a power of two
        D = mid.numerator * 5 ** k
        cases.append((D, -k))
    for D, E in cases:
        v = Fraction(D) * Fraction(10) ** E
        want = _brute_nearest(v, table, keys)
        for neg in (False, True):
            bits, st = round_decimal(neg, D, E, fmt)
            got = decode_value(bits, fmt)
            if want == inf_value:
                assert got == (-math.inf if neg else math.inf), (D, E)
                assert st == STATUS_OUT_OF_RANGE
            else:
                assert got == (-want if neg else want), (D, E, fmt.name)
                assert bool(bits & fmt.sign_bit) == neg
                if want == 0 and D != 0:
                    assert st == STATUS_OUT_OF_RANGE
                else:
                    assert st == STATUS_OK


# ---------------------------------------------------------------------------
# binary16 and bfloat16: brute force over every representable value, and the
# library conversions of exactly representable midpoints
# ---------------------------------------------------------------------------

def _exact_decimal(v: Fraction):
    """(D, E) with D * 10^E == v for a dyadic rational v >= 0."""
    k = v.denominator.bit_length() - 1  # denominator is a power of two
    return v.numerator * 5 ** k, -k


def _small_format_cases(fmt, seed, stride):
    """Every representable value, every midpoint of neighbours (and the
    midpoint nudged up and down by one unit of a digit far below it), random
    decimals across the format's range."""
    table = _representables(fmt)
    keys = [t[0] for t in table]
    cases = []
    for i in range(0, len(table) - 1, stride):
        a, b = keys[i], keys[i + 1]
        D, E = _exact_decimal(a)
        cases.append((D, E))
        D, E = _exact_decimal((a + b) / 2)
        cases += [(D, E), (D * 1000 + 1, E - 3), (D * 1000 - 1, E - 3)]
    rng = np.random.default_rng(seed)
    lo = int(math.floor(math.log10(float(keys[1])))) - 2
    hi = int(math.ceil(math.log10(float(keys[-1])))) + 1
    for d, e in zip(rng.integers(1, 10 ** 9, 6000), rng.integers(lo - 9, hi - 8, 6000)):
        cases.append((int(d), int(e)))
    return table, keys, cases


@pytest.mark.parametrize("fmt,stride", [(BINARY16, 1), (BFLOAT16, 3)],
                         ids=["binary16", "bfloat16"])
def test_bruteforce_half_formats(fmt, stride):
    table, keys, cases = _small_format_cases(fmt, 99, stride)
    inf_value = keys[-1]
    for D, E in cases:
        v = Fraction(D) * Fraction(10) ** E
        want = _brute_nearest(v, table, keys)
        bits, st = round_decimal(False, D, E, fmt)
        got = decode_value(bits, fmt)
        if want == inf_value:
            assert got == math.inf and st == STATUS_OUT_OF_RANGE, (D, E)
        else:
            assert got == want, (D, E, fmt.name)
            assert st == (STATUS_OUT_OF_RANGE if want == 0 and D else STATUS_OK)


def test_binary16_matches_numpy_on_midpoints():
    """numpy rounds binary64 -> binary16 to nearest, ties to even; every
    binary16 value and midpoint is exact in binary64."""
    table = _representables(BINARY16)
    vals = []
    for (a, _), (b, _) in zip(table[:-1], table[1:]):
        vals += [a, (a + b) / 2]
    for v in vals:
        D, E = _exact_decimal(v)
        bits, _ = round_decimal(False, D, E, BINARY16)
        with np.errstate(over="ignore"):  # 65520 rounds to infinity
            want = int(np.array([float(v)], dtype=np.float64).astype(np.float16).view(np.uint16)[0])
        assert bits == want, (float(v), hex(bits), hex(want))


def test_bfloat16_matches_torch_on_midpoints():
    """torch rounds binary32 -> bfloat16 to nearest, ties to even; bfloat16
    values and midpoints are exact in binary32 (below its overflow)."""
    torch = pytest.importorskip("torch")
    table = _representables(BFLOAT16)
    vals = []
    for (a, _), (b, _) in zip(table[:-1], table[1:]):
        if b < Fraction(2) ** 127 * 2:
            vals += [a, (a + b) / 2]
    vals = vals[::5]
    x = torch.tensor([float(v) for v in vals], dtype=torch.float32)
    want = x.to(torch.bfloat16).view(torch.int16).numpy().astype(np.uint16)
    for v, w in zip(vals, want.tolist()):
        D, E = _exact_decimal(v)
        bits, _ = round_decimal(False, D, E, BFLOAT16)
        assert bits == w, (float(v), hex(bits), hex(w))


def test_half_format_specials():
    cases = [
        ("65504", BINARY16, 0x7BFF, STATUS_OK),
        ("65519.99", BINARY16, 0x7BFF, STATUS_OK),
        ("65520", BINARY16, 0x7C00, STATUS_OUT_OF_RANGE),  # tie with 2^16: even = infinity
        ("5.9604644775390625e-8", BINARY16, 0x0001, STATUS_OK),  # 2^-24
        ("2.98023223876953125e-8", BINARY16, 0x0000, STATUS_OUT_OF_RANGE),  # 2^-25, tie to 0
        ("2.9802322387695313e-8", BINARY16, 0x0001, STATUS_OK),
        ("6.103515625e-5", BINARY16, 0x0400, STATUS_OK),  # 2^-14, smallest normal
        ("1", BINARY16, 0x3C00, STATUS_OK),
        ("-2", BINARY16, 0xC000, STATUS_OK),
        ("1", BFLOAT16, 0x3F80, STATUS_OK),
        ("3.3895313892515355e38", BFLOAT16, 0x7F7F, STATUS_OK),
        ("3.40e38", BFLOAT16, 0x7F80, STATUS_OUT_OF_RANGE),
        ("1.00390625", BFLOAT16, 0x3F80, STATUS_OK),  # 1 + 2^-8: tie, even is 1
        ("1.01171875", BFLOAT16, 0x3F82, STATUS_OK),  # 1 + 3*2^-8: tie, even is up
    ]
    for tok, fmt, bits, st in cases:
        got = parse_token(tok.encode(), fmt)
        assert got == (bits, st), (tok, fmt.name, hex(got[0]), got[1])


# ---------------------------------------------------------------------------
# correctly rounded library parsers on the real formats
# ---------------------------------------------------------------------------

def _corpus(n_each=4000, seed=77):
    rng = np.random.default_rng(seed)
    toks = []
    toks += W.uniform_shortest(rng, n_each)
    toks += W.coordinates(rng, n_each)
    toks += W.random_bits_e17(rng, n_each)
    toks += W.hard_tokens(rng, n_each)
    toks += [str(int(v)) for v in rng.integers(0, 2 ** 64, 500, dtype=np.uint64)]
    toks += ["%.*e" % (int(k), float(x)) for k, x in
             zip(rng.integers(0, 30, 2000), rng.standard_normal(2000) * 10.0 ** rng.integers(-300, 300, 2000))]
    return [t.encode() for t in toks]


def test_binary64_matches_cpython_float():
    n = 0
    for tok in _corpus():
        bits, st = parse_token(tok, BINARY64)
        assert st != STATUS_INVALID, tok
        assert bits == f64_bits(float(tok)), tok
        n += 1
    assert n > 18000


def test_binary32_matches_glibc_strtof():
    n = 0
    for tok in _corpus(n_each=2500, seed=78):
        bits, st = parse_token(tok, BINARY32)
        assert st != STATUS_INVALID, tok
        assert bits == f32_bits_from_strtof(tok), tok
        n += 1
    assert n > 10000


def test_binary32_double_rounding_traps():
    # rounding through binary64 first would give a different answer
    cases = {
        b"1.0000000596046447753906250001": 0x3F800001,
        b"3.4028235677973366e38": 0x7F7FFFFF,
        b"1.4e-45": 0x00000001,
        b"1.17549435e-38": 0x00800000,
    }
    for tok, want in cases.items():
        bits, st = parse_token(tok, BINARY32)
        assert bits == want, tok
        assert bits == f32_bits_from_strtof(tok)


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------

def test_roundtrip_binary64():
    # Section 1: 17 significant digits always parse back to the same double.
    rng = np.random.default_rng(5)
    u = rng.integers(0, 2 ** 64, 20000, dtype=np.uint64)
    u = u[((u >> np.uint64(52)) & np.uint64(0x7FF)) != np.uint64(0x7FF)]
    for x in u.view(np.float64).tolist():
        for s in (repr(x), "%.17e" % x):
            bits, st = parse_token(s.encode(), BINARY64)
            assert bits == f64_bits(x), s


def test_roundtrip_binary32():
    # Section 2: 9 significant digits always parse back to the same float.
    rng = np.random.default_rng(6)
    u = rng.integers(0, 2 ** 32, 20000, dtype=np.uint64).astype(np.uint32)
    u = u[((u >> np.uint32(23)) & np.uint32(0xFF)) != np.uint32(0xFF)]
    for b, x in zip(u.tolist(), u.view(np.float32).tolist()):
        s = "%.8e" % x  # 9 significant digits
        bits, st = parse_token(s.encode(), BINARY32)
        assert bits == b, s


def test_sign_symmetry_and_monotonicity():
    rng = np.random.default_rng(7)
    toks = W.hard_tokens(rng, 3000) + W.uniform_shortest(rng, 1000)
    vals = []
    for t in toks:
        t = t.lstrip("+-")
        b, _ = parse_token(t.encode(), BINARY64)
        bn, _ = parse_token(("-" + t).encode(), BINARY64)
        assert bn == b | BINARY64.sign_bit
        neg, D, E = decompose(t.encode())
        vals.append((Fraction(D) * Fraction(10) ** E if abs(E) < 2000 else None, b))
    vals = [v for v in vals if v[0] is not None]
    vals.sort(key=lambda t: t[0])
    prev = None
    for _, b in vals:
        x = decode_value(b, BINARY64)
        if prev is not None:
            assert x >= prev
        prev = x


def test_scale_invariance():
    rng = np.random.default_rng(8)
    for D, E in zip(rng.integers(1, 10 ** 18, 2000).tolist(), rng.integers(-340, 300, 2000).tolist()):
        a = round_decimal(False, D, E, BINARY64)
        b = round_decimal(False, D * 10, E - 1, BINARY64)
        c = round_decimal(False, D * 1000, E - 3, BINARY64)
        assert a == b == c


# ---------------------------------------------------------------------------
# grammar, status codes and tokenisation (library contract)
# ---------------------------------------------------------------------------

def test_grammar_golden(golden_dir):
    rows = load_tsv(os.path.join(golden_dir, "grammar.tsv"))
    for tok, flags, st, hexbits in rows:
        bits, status = parse_token(tok.encode(), BINARY64, int(flags))
        assert status == int(st), tok
        assert bits == int(hexbits, 16), tok


def test_grammar_agrees_with_cpython_on_acceptance():
    # CPython float() also accepts '_', surrounding blanks and inf/nan; on
    # tokens without those it must agree with the oracle on acceptance.
    rng = np.random.default_rng(9)
    alphabet = list("0123456789.eE+-") + ["x", "_", "1"]
    for _ in range(20000):
        n = int(rng.integers(1, 8))
        tok = "".join(alphabet[int(i)] for i in rng.integers(0, len(alphabet), n))
        if "_" in tok or "x" in tok:
            continue
        try:
            float(tok)
            ok_py = True
        except ValueError:
            ok_py = False
        _, st = parse_token(tok.encode(), BINARY64)
        assert (st != STATUS_INVALID) == ok_py, tok


def test_invalid_examples_rejected():
    for tok in W.INVALID_EXAMPLES:
        bits, st = parse_token(tok.encode(), BINARY64)
        assert st == STATUS_INVALID, tok
        assert bits == 0x7FF8000000000000
        bits, st = parse_token(tok.encode(), BINARY32)
        assert bits == 0x7FC00000


def test_reject_plus_flag():
    assert parse_token(b"+1", BINARY64, FLAG_REJECT_PLUS)[1] == STATUS_INVALID
    assert parse_token(b"1e+1", BINARY64, FLAG_REJECT_PLUS)[1] == STATUS_OK
    assert parse_token(b"-1", BINARY64, FLAG_REJECT_PLUS)[1] == STATUS_OK


def test_split_tokens():
    assert split_tokens(b"") == []
    assert split_tokens(b"\n\n\n") == []
    assert split_tokens(b"1") == [(0, 1)]
    assert split_tokens(b"1\n") == [(0, 1)]
    assert split_tokens(b"\n12\n\n3") == [(1, 3), (5, 6)]
    assert split_tokens(b"1,2 3\t4", b", \t") == [(0, 1), (2, 3), (4, 5), (6, 7)]
    bits, st = parse_buffer(b"1\n\nx\n2.5", "f64")
    assert st == [STATUS_OK, STATUS_INVALID, STATUS_OK]
    assert bits[2] == f64_bits(2.5)


# ---------------------------------------------------------------------------
# JSON grammar and inf/nan tokens (library contract)
# ---------------------------------------------------------------------------

def test_json_and_infnan_golden(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "grammar_json_infnan.tsv")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tok, flags, st, bits = line.rstrip("\n").split("\t")
            rows.append((tok, int(flags), int(st), int(bits, 16)))
    assert len(rows) > 30
    for tok, flags, st, bits in rows:
        assert parse_token(tok.encode(), BINARY64, flags) == (bits, st), (tok, flags)


def _mutated_numbers(rng, n):
    """Number-like strings from the alphabet of the grammar, biased toward
    the edge cases of the JSON rules."""
    parts = ["", "-", "+", "0", "00", "1", "01", "9", "12", ".", ".5", "5.", "e", "E",
             "e+", "e-", "3", "0.", ".0"]
    out = []
    for _ in range(n):
        k = int(rng.integers(1, 5))
        out.append("".join(parts[int(i)] for i in rng.integers(0, len(parts), k)))
    return [t for t in out if t]


def test_json_acceptance_matches_json_module():
    """A token is a JSON number exactly when Python's json module reads it as
    a number (json also reads NaN/Infinity literals: none are generated)."""
    import json
    rng = np.random.default_rng(5)
    for tok in set(_mutated_numbers(rng, 20_000)):
        try:
            v = json.loads(tok)
            ok = isinstance(v, (int, float)) and not isinstance(v, bool)
        except ValueError:
            ok = False
        _, st = parse_token(tok.encode(), BINARY64, 2)
        assert (st != 1) == ok, tok


def test_infnan_acceptance_matches_float():
    """Letter tokens: accepted with the inf/nan flag exactly when float()
    reads them (float also accepts blanks and digit separators: none are
    generated), and then to the same infinity or NaN."""
    rng = np.random.default_rng(6)
    pieces = ["", "-", "+", "i", "I", "n", "N", "f", "F", "a", "A", "in", "nan", "inf",
              "ity", "ini", "t", "y"]
    toks = set()
    for _ in range(20_000):
        k = int(rng.integers(1, 5))
        toks.add("".join(pieces[int(i)] for i in rng.integers(0, len(pieces), k)))
    for tok in toks:
        if not tok:
            continue
        try:
            v = float(tok)
            ok = True
        except ValueError:
            ok = False
        bits, st = parse_token(tok.encode(), BINARY64, 4)
        assert (st == 0) == ok, tok
        if ok:
            want = struct.unpack("<Q", struct.pack("<d", v))[0]
            if math.isnan(v):
                assert bits & 0x7FFFFFFFFFFFFFFF == 0x7FF8000000000000, tok
                assert bool(bits >> 63) == tok.startswith("-"), tok
            else:
                assert bits == want, tok


# ---------------------------------------------------------------------------
# hexadecimal floating-point tokens (Appendix C)
# ---------------------------------------------------------------------------

def test_hexfloat_golden(golden_dir):
    n = 0
    with open(os.path.join(golden_dir, "hexfloat.tsv")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tok, st, bits, _ = line.rstrip("\n").split("\t")
            assert parse_token(tok.encode(), BINARY64, 8) == (int(bits, 16), int(st)), tok
            n += 1
    assert n >= 20


def test_hexfloat_matches_fromhex():
    """float.fromhex rounds to nearest, ties to even (binary64)."""
    rng = np.random.default_rng(8)
    for tok in W.hex_tokens(rng, 20_000):
        mant = tok.lower().lstrip("+-")[2:].split("p")[0].replace(".", "")
        nonzero = int(mant or "0", 16) != 0
        try:
            v = float.fromhex(tok)
            want = struct.unpack("<Q", struct.pack("<d", v))[0]
            want_st = 2 if math.isinf(v) or (v == 0 and nonzero) else 0
        except OverflowError:
            want = 0x7FF0000000000000 | (1 << 63 if tok.startswith("-") else 0)
            want_st = 2
        bits, st = parse_token(tok.encode(), BINARY64, 8)
        assert bits == want, (tok, hex(bits), hex(want))
        assert st == want_st, (tok, st, want_st)


def test_hexfloat_narrow_formats_match_numpy():
    """Hex values exact in binary64, rounded once to binary32 / binary16."""
    rng = np.random.default_rng(9)
    for _ in range(20_000):
        m = int(rng.integers(1, 2 ** 40))
        e = int(rng.integers(-180, 140))
        tok = "0x%xp%d" % (m, e)
        v = float.fromhex(tok)  # exact: 40 bits, in range
        with np.errstate(over="ignore", under="ignore"):
            w32 = int(np.array([v]).astype(np.float32).view(np.uint32)[0])
            w16 = int(np.array([v]).astype(np.float16).view(np.uint16)[0])
        assert parse_token(tok.encode(), BINARY32, 8)[0] == w32, tok
        assert parse_token(tok.encode(), BINARY16, 8)[0] == w16, tok
