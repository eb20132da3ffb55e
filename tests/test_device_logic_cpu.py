"""The library's per-token logic (ffp_device.h: lexer, Algorithm 1 and the
w / w+1 test), compiled for the host and compared bit for bit with the
oracle on every token it decides.  Tokens it sends to the exact fallback (a
wavefront-cooperative GPU kernel) carry status 255 and are counted; they,
the tile scan and the kernels themselves are covered by the GPU tests."""

import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

from gen import workloads as W
from oracle import parse_buffer

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2101_11408_amd")


@pytest.fixture(scope="module")
def host_check(tmp_path_factory):
    d = tmp_path_factory.mktemp("host_check")
    sys.path.insert(0, os.path.join(PKG, "csrc"))
    try:
        import gen_table
    finally:
        sys.path.pop(0)
    inc = d / "ffp_table.inc"
    inc.write_text(gen_table.render())
    exe = d / "host_check"
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"), "-I", str(d),
           os.path.join(ROOT, "tests", "host_logic", "host_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    return str(exe)


def run_host(exe, buf: bytes, fmt: str, flags=0, delims=b"\n"):
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "in.txt")
        out = os.path.join(td, "out.bin")
        with open(src, "wb") as f:
            f.write(buf)
        res = subprocess.run([exe, src, fmt, str(flags), out, delims.decode()],
                             check=True, capture_output=True, text=True)
        ntok, nfb = map(int, res.stdout.split())
        raw = np.fromfile(out, dtype=np.dtype([("bits", "<u8"), ("st", "u1")]))
    assert len(raw) == ntok
    return raw["bits"], raw["st"], nfb


def check(exe, buf, fmt, label, **kw):
    bits, st, nfb = run_host(exe, buf, fmt, **kw)
    wb, ws = parse_buffer(buf, fmt, **kw)
    assert len(bits) == len(wb), label
    wb = np.array(wb, dtype=np.uint64)
    ws = np.array(ws, dtype=np.uint8)
    decided = st != 255
    assert int((~decided).sum()) == nfb, label
    bad = np.flatnonzero(decided & ((bits != wb) | (st != ws)))
    if bad.size:
        toks = [t for t in buf.split(b"\n") if t] if kw.get("delims", b"\n") == b"\n" else None
        i = int(bad[0])
        tok = toks[i][:100] if toks else "?"
        raise AssertionError("%s %s: %d mismatches, first #%d %r host=%x/%d oracle=%x/%d" % (
            label, fmt, bad.size, i, tok, int(bits[i]), int(st[i]), int(wb[i]), int(ws[i])))
    return nfb


def test_uniform_and_mixed(host_check):
    buf = W.config2(seed=44, n=60_000)
    for fmt in ("f64", "f32"):
        check(host_check, buf, fmt, "mixed")


def test_hard_cases_exercise_fallback(host_check):
    buf = W.config3(seed=45, n=20_000)
    nfb64 = check(host_check, buf, "f64", "hard")
    nfb32 = check(host_check, buf, "f32", "hard")
    assert nfb64 > 1000 and nfb32 > 1000


def test_grammar_and_specials(host_check):
    toks = [t for t in W.INVALID_EXAMPLES if t and "\n" not in t and " " not in t]
    toks += ["1", "-1", "+1", "-0", ".5", "5.", "1e309", "1e-400", "4.9e-324",
             "2.4703282292062327e-324", "2.4703282292062328e-324", "9007199254740993",
             "9000000000000000.5", "9000000000000001.5", "1e+100000000000000000000",
             "0e99999999999", "1" * 40 + "e-40", "0." + "0" * 400 + "1"]
    buf = W.join_tokens(toks)
    for fmt in ("f64", "f32"):
        check(host_check, buf, fmt, "grammar")
    check(host_check, b"+1\n1\n-1\n", "f64", "reject-plus", flags=1)


def test_random_bit_patterns_e17_and_integers(host_check):
    rng = np.random.default_rng(46)
    toks = W.random_bits_e17(rng, 30_000)
    toks += [str(int(v)) for v in rng.integers(0, 2 ** 64, 5000, dtype=np.uint64)]
    toks += ["%.*e" % (int(k), float(x)) for k, x in
             zip(rng.integers(0, 25, 5000), rng.standard_normal(5000) * 10.0 ** rng.integers(-320, 300, 5000))]
    buf = W.join_tokens(toks)
    for fmt in ("f64", "f32"):
        check(host_check, buf, fmt, "bits")


def test_exact_ties_near_one(host_check):
    """Exact midpoints written with few digits: the tie windows of Section 6
    (q in [-4, 23] for binary64, [-17, 10] for binary32)."""
    rng = np.random.default_rng(47)
    toks = []
    for _ in range(20_000):
        m = int(rng.integers(2 ** 52, 2 ** 53))
        e = int(rng.integers(-20, 40))
        num = 2 * m + 1  # midpoint (2m+1) * 2^(e-1)
        if e - 1 >= 0:
            toks.append(str(num << (e - 1)))
        else:
            toks.append("%de%d" % (num * 5 ** (1 - e), e - 1))
    for _ in range(10_000):
        m = int(rng.integers(2 ** 23, 2 ** 24))
        e = int(rng.integers(-30, 40))
        num = 2 * m + 1
        toks.append(str(num << (e - 1)) if e >= 1 else "%de%d" % (num * 5 ** (1 - e), e - 1))
    buf = W.join_tokens(toks)
    for fmt in ("f64", "f32"):
        check(host_check, buf, fmt, "ties")


def test_half_formats(host_check):
    """binary16 and bfloat16 through the same logic; long tokens just above
    or below a midpoint (w and w + 1 round differently) go to the fallback."""
    rng = np.random.default_rng(48)
    toks = W.mixed_tokens(rng, 20_000) + W.hard_tokens(rng, 1000)
    toks += ["65504", "65519.99", "65520", "5.9604644775390625e-8", "2.98023223876953125e-8",
             "6.103515625e-5", "1.00390625", "1.01171875", "3.3895313892515355e38", "1e-40",
             "9.18354961579912115600575419704879435795832466228193376178712270530013483949005e-41"]
    # small integers and short decimals, the range binary16 represents
    toks += [str(int(v)) for v in rng.integers(0, 70_000, 5000)]
    toks += ["%.*f" % (int(k), float(x)) for k, x in zip(rng.integers(0, 8, 5000),
                                                         rng.random(5000) * 1000)]
    toks += ["%d.%s1" % (v, "0" * int(z)) for v, z in zip(range(2049, 2200, 2), rng.integers(18, 30, 76))]
    toks += ["%d.%s1" % (v, "0" * int(z)) for v, z in zip(range(257, 400, 2), rng.integers(18, 30, 72))]
    buf = W.join_tokens(toks)
    for fmt in ("f16", "bf16"):
        nfb = check(host_check, buf, fmt, "half")
        assert nfb > 0


def _half_ties(rng, mant, emin, n):
    """Exact midpoints between neighbouring values of a format with `mant`
    stored significand bits and smallest normal exponent `emin`, written
    with at most 19 significant digits: integers, w * 10^q with 5^-q
    dividing w, and subnormal midpoints."""
    toks = []
    while len(toks) < n:
        if rng.random() < 0.15:  # between subnormals: (2k + 1) * 2^(emin - mant - 1)
            num, e = 2 * int(rng.integers(0, 2 ** mant)) + 1, emin - mant - 1
        else:
            num = 2 * int(rng.integers(2 ** mant, 2 ** (mant + 1))) + 1
            e = int(rng.integers(emin - mant, 16)) - 1
        if e >= 0:
            toks.append(str(num << e))
        else:
            w = num * 5 ** -e
            if w < 10 ** 19:
                toks.append("%de%d" % (w, e))
    return toks


def test_half_format_short_ties_inline(host_check):
    """binary16 / bfloat16 midpoints of up to 19 significant digits are
    decided without the exact fallback (q in [0, 27]: exact product; q in
    [-27, -1]: 5^-q divides w), and rounded to even like the oracle."""
    rng = np.random.default_rng(53)
    for fmt, mant, emin in (("f16", 10, -14), ("bf16", 7, -126)):
        toks = _half_ties(rng, mant, emin, 20_000)
        toks += [str(v) for v in range(2 ** (mant + 1) + 1, 2 ** (mant + 2), 2)]
        buf = W.join_tokens(toks)
        nfb = check(host_check, buf, fmt, "half-ties")
        assert nfb == 0, (fmt, nfb)


def _flag_tokens(seed):
    rng = np.random.default_rng(seed)
    parts = ["", "-", "+", "0", "00", "1", "01", "9", "12", ".", ".5", "5.", "e", "E",
             "e+", "e-", "3", "0.", ".0", "inf", "Inf", "nan", "NaN", "infinity", "INFINITY",
             "in", "na"]
    toks = set()
    for _ in range(6000):
        k = int(rng.integers(1, 5))
        toks.add("".join(parts[int(i)] for i in rng.integers(0, len(parts), k)))
    return sorted(t for t in toks if t)


@pytest.mark.parametrize("flags", [2, 4, 6, 5])
def test_json_and_infnan_flags(host_check, flags):
    """The byte-by-byte lexer under the JSON and inf/nan flags."""
    buf = W.join_tokens(_flag_tokens(49))
    for fmt in ("f64", "f32"):
        check(host_check, buf, fmt, "flags-%d" % flags, flags=flags)


def _hex_buffer(seed):
    rng = np.random.default_rng(seed)
    toks = W.hex_tokens(rng, 8000)
    with open(os.path.join(ROOT, "tests", "golden", "hexfloat.tsv")) as f:
        toks += [ln.split("\t")[0] for ln in f if ln.strip() and not ln.startswith("#")]
    # decimal tokens and near-misses of the hexadecimal form in the same text
    toks += W.mixed_tokens(rng, 2000) + ["0", "0x", "x1", "00x1", "0x1p+", "0x1.p-", "+0x1",
                                         "0x1e", "0xg", "0x.", "0x1.2.3", "0x1p1p1"]
    rng.shuffle(toks)
    return W.join_tokens(toks)


@pytest.mark.parametrize("flags", [8, 12, 9, 10])
def test_hex_flag(host_check, flags):
    """Hexadecimal tokens (Appendix C) through the byte-by-byte lexer and
    their rounding, in every format."""
    buf = _hex_buffer(50)
    for fmt in ("f64", "f32", "f16", "bf16"):
        check(host_check, buf, fmt, "hex-%d" % flags, flags=flags)


def _directed_tokens(seed):
    """Tokens for the directed rounding modes: the usual mixes, decimals that
    are exactly representable (dyadic fractions written out, integers), their
    neighbours one unit of a far digit away, and the ends of every format's
    range."""
    rng = np.random.default_rng(seed)
    toks = W.mixed_tokens(rng, 6000) + W.hard_tokens(rng, 800)
    for _ in range(3000):
        j = int(rng.integers(1, 28))
        num = int(rng.integers(1, 2 ** 20))
        digits, e10 = W._exact_decimal(num, -j)  # num * 2^-j = digits * 10^e10 exactly
        d = int(digits)
        toks += ["%de%d" % (d, e10), "%de%d" % (d * 10 ** 7 + 1, e10 - 7),
                 "%de%d" % (d * 10 ** 7 - 1, e10 - 7)]
    for _ in range(1000):
        toks.append(str(int(rng.integers(1, 2 ** 62)) << int(rng.integers(0, 40))))
    toks += ["7450580596923828125e-27", "0.5", "0.25", "1.5", "0.1", "-0.1", "1e23", "9007199254740993",
             "18446744073709551616", "1e309", "-1e309", "1.7976931348623157e308",
             "1.7976931348623158e308", "1.7976931348623159e308", "4.9e-324", "2e-324", "1e-400",
             "-1e-400", "3.4028235e38", "3.4028236e38", "1.4e-45", "1e-46", "-1e-46", "65504",
             "65519", "65520", "6e-8", "5.96e-8", "2.9e-8", "3.3895313892515355e38", "1e39", "9.2e-41"]
    return toks


@pytest.mark.parametrize("flags", [16, 32, 48, 56])
def test_directed_rounding_modes(host_check, flags):
    """Directed rounding (toward zero, +inf, -inf; 56 = -inf with hex tokens)
    through the byte-by-byte lexer and Algorithm 1's directed form."""
    toks = _directed_tokens(51)
    if flags & 8:
        toks += W.hex_tokens(np.random.default_rng(52), 2000)
    buf = W.join_tokens(toks)

    def significant(tok):
        s = tok.lstrip("+-")
        if s[:2].lower() == "0x":
            return 0  # hexadecimal: always exact in-line
        mant = s.split("e")[0].split("E")[0].replace(".", "")
        return len(mant.strip("0"))

    short = np.array([significant(tk) <= 19 for tk in toks])
    for fmt in ("f64", "f32", "f16", "bf16"):
        check(host_check, buf, fmt, "round-%d" % flags, flags=flags)
        _, st, _ = run_host(host_check, buf, fmt, flags=flags)
        # up to 19 significant digits Algorithm 1's directed form decides
        # in-line; longer tokens whose value is within their dropped digits
        # of a representable value need the exact fallback
        assert not (short & (st == 255)).any(), [toks[i] for i in np.flatnonzero(short & (st == 255))[:5]]
