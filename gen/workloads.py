"""Seeded synthetic workloads for the decimal parser.

This module only *prints* numbers (binary -> decimal, via CPython's correctly
rounded ``repr`` / ``%`` formatting and exact integer expansions); it holds none
of the parsing method's arithmetic.  Both the tests (against the oracle) and
the benchmark (against the GPU path) draw their inputs from here.

The workloads stand in for the paper's datasets (Section 12): "uniform" is
random doubles in the unit interval printed with the fewest digits; the
"canada" geographic-coordinate file is not available, so coordinates uniform in
[-180, 180] printed with 6-15 fraction digits stand in for it.

Every function is deterministic in its seed.
"""

import numpy as np

_MAX_FINITE_F64_BITS = 0x7FEFFFFFFFFFFFFF
_MAX_FINITE_F32_BITS = 0x7F7FFFFF


# ---------------------------------------------------------------------------
# individual token formats
# ---------------------------------------------------------------------------

def _positional_from_repr(s: str) -> str:
    """Rewrite CPython's shortest repr in plain positional notation."""
    if "e" not in s:
        return s
    mant, exp = s.split("e")
    exp = int(exp)
    neg = mant.startswith("-")
    if neg:
        mant = mant[1:]
    if "." in mant:
        ip, fp = mant.split(".")
    else:
        ip, fp = mant, ""
    digits = ip + fp
    point = len(ip) + exp  # position of the decimal point within digits
    if point <= 0:
        out = "0." + "0" * (-point) + digits
    elif point >= len(digits):
        out = digits + "0" * (point - len(digits)) + ".0"
    else:
        out = digits[:point] + "." + digits[point:]
    return ("-" if neg else "") + out


def uniform_shortest(rng, n: int):
    """Doubles uniform in [0,1), shortest round-trip digits, positional."""
    xs = rng.random(n).tolist()
    return [_positional_from_repr(repr(x)) for x in xs]


def coordinates(rng, n: int):
    """Values uniform in [-180,180] printed with 6..15 fraction digits."""
    xs = rng.uniform(-180.0, 180.0, n).tolist()
    ks = rng.integers(6, 16, size=n).tolist()
    return ["%.*f" % (k, x) for k, x in zip(ks, xs)]


def random_bits_e17(rng, n: int):
    """Random finite binary64 bit patterns (both signs, subnormals included)
    printed as '%.17e'."""
    out = []
    need = n
    while need > 0:
        u = rng.integers(0, 2 ** 64, size=need + need // 512 + 16, dtype=np.uint64)
        ok = ((u >> np.uint64(52)) & np.uint64(0x7FF)) != np.uint64(0x7FF)
        u = u[ok][:need]
        xs = u.view(np.float64).tolist()
        out.extend("%.17e" % x for x in xs)
        need = n - len(out)
    return out


# ---------------------------------------------------------------------------
# buffers
# ---------------------------------------------------------------------------

def join_tokens(tokens, delim: str = "\n", trailing: bool = True) -> bytes:
    body = delim.join(tokens)
    if trailing and tokens:
        body += delim
    return body.encode("utf-8")


def config1(seed: int = 1, n: int = 100_000) -> bytes:
    """100k uniform [0,1) doubles, shortest digits, positional, one per line."""
    rng = np.random.default_rng(seed)
    return join_tokens(uniform_shortest(rng, n))


def mixed_tokens(rng, n: int):
    """The 50/25/25 interleaved mix: uniform shortest, coordinates, %.17e."""
    kind = rng.choice(3, size=n, p=[0.5, 0.25, 0.25])
    counts = [int((kind == k).sum()) for k in range(3)]
    pools = [
        iter(uniform_shortest(rng, counts[0])),
        iter(coordinates(rng, counts[1])),
        iter(random_bits_e17(rng, counts[2])),
    ]
    return [next(pools[k]) for k in kind.tolist()]


def config2(seed: int = 2, n: int = 10_000_000) -> bytes:
    """10M numbers in one buffer: 50% uniform shortest, 25% coordinates,
    25% random finite bit patterns as %.17e; newline separated."""
    rng = np.random.default_rng(seed)
    return join_tokens(mixed_tokens(rng, n))


# ---------------------------------------------------------------------------
# hard cases (config 3)
# ---------------------------------------------------------------------------

def _decode(bits: int, pbits: int, ebits: int):
    """(m, e) with value m * 2^e for a positive finite encoding."""
    frac_mask = (1 << (pbits - 1)) - 1
    field = bits >> (pbits - 1)
    bias = (1 << (ebits - 1)) - 1
    if field == 0:
        return bits & frac_mask, 1 - bias - (pbits - 1)
    return (bits & frac_mask) | (1 << (pbits - 1)), field - bias - (pbits - 1)


def _exact_decimal(num: int, e2: int):
    """Exact decimal expansion of num * 2^e2 as (digit string, exp10) with no
    trailing zeros: value = int(digits) * 10^exp10."""
    if e2 >= 0:
        digits, exp10 = str(num << e2), 0
    else:
        digits, exp10 = str(num * 5 ** (-e2)), e2
    stripped = digits.rstrip("0")
    exp10 += len(digits) - len(stripped)
    return stripped or "0", exp10


def _render(rng, neg: bool, digits: str, exp10: int, allow_positional=True) -> str:
    """Render int(digits)*10^exp10 either positionally or in e-notation."""
    sign = "-" if neg else ""
    ndig = len(digits)
    lead_exp = exp10 + ndig - 1
    style = int(rng.integers(0, 3)) if allow_positional else 2
    if style < 2 and -400 < lead_exp < 400:
        point = ndig + exp10
        if point <= 0:
            body = "0." + "0" * (-point) + digits
        elif point >= ndig:
            body = digits + "0" * (point - ndig)
            if style == 1:
                body += ".0"
        else:
            body = digits[:point] + "." + digits[point:]
        return sign + body
    e_char = "e" if rng.integers(0, 2) else "E"
    mant = digits[0] + ("." + digits[1:] if ndig > 1 else "")
    return "%s%s%s%d" % (sign, mant, e_char, lead_exp)


def _midpoint_token(rng, pbits: int, ebits: int, max_bits: int) -> str:
    bits = int(rng.integers(0, max_bits))  # [0, max) so bits+1 stays finite
    m, e = _decode(bits, pbits, ebits)
    # midpoint of bits and bits+1 is (2m+1) * 2^(e-1)
    digits, exp10 = _exact_decimal(2 * m + 1, e - 1)
    n = int(rng.integers(20, 801))
    if n < len(digits):
        exp10 += len(digits) - n
        digits = digits[:n]
    else:
        exp10 -= n - len(digits)
        digits = digits + "0" * (n - len(digits))
    delta = int(rng.integers(-1, 2))
    v = int(digits) + delta
    if v <= 0:
        v = 1
    digits = str(v)
    return _render(rng, bool(rng.integers(0, 2)), digits, exp10)


_SPECIAL_SUBNORMAL = [
    "4.9e-324", "5e-324", "2.4703282292062327e-324", "2.4703282292062328e-324",
    "4.9406564584124654e-324", "2.2250738585072011e-308",
    "2.2250738585072014e-308", "2.2250738585072009e-308",
    "1.4e-45", "1.401298464324817e-45", "7.006492321624085e-46",
    "7.006492321624086e-46", "1.17549435e-38", "1.1754942e-38",
    "1e-323", "1e-324", "1e-325", "3e-324", "2e-45", "7e-46",
]

_SPECIAL_BIG = [
    "1.7976931348623157e308", "1.7976931348623158e308",
    "1.7976931348623159e308", "1.7976931348623157e+308", "1e308", "1e309",
    "-1e309", "1.8e308", "3.4028234663852886e38", "3.4028235677973366e38",
    "3.4028236e38", "3.4028235e38", "1e39", "1e38", "9.999999e307",
    "1e+100000000000000000000", "1e-100000000000000000000",
    "0e999999999999", "0.0e-99999999999999", "-0e100000000000000000000",
    "1e-400", "1e-342", "1e-343", "9e-343", "1e308", "1e-307",
]


def _subnormal_token(rng) -> str:
    r = int(rng.integers(0, 6))
    if r == 0:
        return _SPECIAL_SUBNORMAL[int(rng.integers(0, len(_SPECIAL_SUBNORMAL)))]
    if r == 1:  # random binary64 subnormal, printed with k digits
        bits = int(rng.integers(1, 1 << 52))
        x = np.array([bits], dtype=np.uint64).view(np.float64)[0]
        return "%.*e" % (int(rng.integers(0, 26)), float(x))
    if r == 2:  # random binary32 subnormal
        bits = int(rng.integers(1, 1 << 23))
        m, e = _decode(bits, 24, 8)
        digits, exp10 = _exact_decimal(m, e)
        k = int(rng.integers(1, 30))
        if k < len(digits):
            exp10 += len(digits) - k
            digits = digits[:k]
        return _render(rng, False, digits, exp10, allow_positional=False)
    if r == 3:  # exact 2^-1075 (binary64) or 2^-150 (binary32), nudged
        e = -1075 if rng.integers(0, 2) else -150
        digits, exp10 = _exact_decimal(1, e)
        v = int(digits) + int(rng.integers(-1, 2))
        return _render(rng, False, str(v), exp10, allow_positional=False)
    if r == 4:  # subnormal midpoints, binary64
        bits = int(rng.integers(0, 1 << 52))
        m, e = _decode(bits, 53, 11)
        digits, exp10 = _exact_decimal(2 * m + 1, e - 1)
        v = int(digits) + int(rng.integers(-1, 2))
        return _render(rng, bool(rng.integers(0, 2)), str(max(v, 1)), exp10,
                       allow_positional=False)
    # subnormal midpoints, binary32
    bits = int(rng.integers(0, 1 << 23))
    m, e = _decode(bits, 24, 8)
    digits, exp10 = _exact_decimal(2 * m + 1, e - 1)
    v = int(digits) + int(rng.integers(-1, 2))
    return _render(rng, bool(rng.integers(0, 2)), str(max(v, 1)), exp10,
                   allow_positional=False)


def _big_token(rng) -> str:
    r = int(rng.integers(0, 5))
    if r == 0:
        return _SPECIAL_BIG[int(rng.integers(0, len(_SPECIAL_BIG)))]
    if r == 1:  # random mantissa, exponent near +-308 / +-38
        nd = int(rng.integers(1, 25))
        digits = "".join(str(int(d)) for d in rng.integers(0, 10, size=nd))
        digits = str(int(rng.integers(1, 10))) + digits
        ex = int(rng.choice([int(rng.integers(295, 315)), int(rng.integers(-330, -300)),
                             int(rng.integers(30, 45)), int(rng.integers(-50, -35))]))
        sign = "-" if rng.integers(0, 2) else ""
        return "%s%s.%se%d" % (sign, digits[0], digits[1:], ex)
    if r == 2:  # exact overflow threshold 2^1024 - 2^970 (binary64), nudged
        if rng.integers(0, 2):
            digits, exp10 = _exact_decimal((1 << 54) - 1, 970 - 1)
        else:
            digits, exp10 = _exact_decimal((1 << 25) - 1, 104 - 1)
        v = int(digits) + int(rng.integers(-1, 2))
        return _render(rng, bool(rng.integers(0, 2)), str(v), exp10)
    if r == 3:  # huge exponent strings
        nd = int(rng.integers(1, 21))
        ex = "".join(str(int(d)) for d in rng.integers(0, 10, size=nd))
        mant = rng.choice(["1", "0", "0.000", "123.456", "9" * 30, "0." + "0" * 50 + "1"])
        esign = rng.choice(["", "+", "-"])
        return "%se%s%s" % (mant, esign, ex)
    # near the largest finite values with many digits
    bits = int(rng.integers(_MAX_FINITE_F64_BITS - 1000, _MAX_FINITE_F64_BITS))
    m, e = _decode(bits, 53, 11)
    digits, exp10 = _exact_decimal(2 * m + 1, e - 1)
    n = int(rng.integers(17, 320))
    if n < len(digits):
        exp10 += len(digits) - n
        digits = digits[:n]
    v = int(digits) + int(rng.integers(-1, 2))
    return _render(rng, False, str(v), exp10)


def _integer_token(rng) -> str:
    r = int(rng.integers(0, 4))
    specials = [2 ** 53 - 1, 2 ** 53, 2 ** 53 + 1, 2 ** 53 + 2, 2 ** 53 + 3,
                2 ** 64 - 1, 2 ** 64, 2 ** 63, 2 ** 63 - 1, 2 ** 24 + 1,
                2 ** 24, 2 ** 25 + 1, 10 ** 19, 10 ** 19 - 1, 0, 1]
    if r == 0:
        return str(specials[int(rng.integers(0, len(specials)))])
    if r == 1:
        return str(int(rng.integers(0, 2 ** 64, dtype=np.uint64)))
    if r == 2:
        return str(int(rng.integers(0, 2 ** 32)))
    return str(int(rng.integers(0, 2 ** 63)) + 2 ** 63 * int(rng.integers(0, 2)))


def _variant_token(rng) -> str:
    r = int(rng.integers(0, 8))
    x = float(rng.random() * 10 ** int(rng.integers(-5, 6)))
    s = repr(x)
    if r == 0:
        return "+" + s
    if r == 1:
        return rng.choice(["-0", "-0.0", "+0", "0", "0.", ".0", "-.0", "-0e-999",
                           "0.000000", "-0.0e-999", "00000", "+0e+0"])
    if r == 2:
        return "." + str(int(rng.integers(0, 10 ** 9)))
    if r == 3:
        return str(int(rng.integers(0, 10 ** 9))) + "."
    if r == 4:  # leading zeros, up to 400
        z = int(rng.integers(1, 401))
        return "0" * z + s
    if r == 5:
        z = int(rng.integers(1, 401))
        return "0." + "0" * z + str(int(rng.integers(1, 10 ** 17)))
    if r == 6:
        return "-" + s.replace("e", "E")
    return "%se%+d" % (s.replace("e", "x").split("x")[0], int(rng.integers(-30, 30)))


def _long_token(rng) -> str:
    r = int(rng.integers(0, 3))
    if r == 0:  # three random u64 concatenated
        return "".join(str(int(v)) for v in rng.integers(0, 2 ** 64, size=3, dtype=np.uint64))
    n = int(rng.integers(20, 801))
    digits = "".join(map(str, rng.integers(0, 10, size=n).tolist()))
    digits = str(int(rng.integers(1, 10))) + digits[1:]
    if r == 1:
        point = int(rng.integers(1, n))
        return digits[:point] + "." + digits[point:]
    ex = int(rng.integers(-340, 300))
    return digits[0] + "." + digits[1:] + "e" + str(ex)


def hard_tokens(rng, n: int):
    """The hard-case mix: 35% binary64 midpoints +-1 in the last of 20-800
    digits, 10% binary32 midpoints, 15% subnormal region, 10% near overflow /
    huge exponents, 10% integers up to 2^64, 10% sign / leading-zero /
    format variants, 10% long non-midpoint strings."""
    kind = rng.choice(7, size=n, p=[0.35, 0.10, 0.15, 0.10, 0.10, 0.10, 0.10])
    out = []
    for k in kind.tolist():
        if k == 0:
            out.append(_midpoint_token(rng, 53, 11, _MAX_FINITE_F64_BITS))
        elif k == 1:
            out.append(_midpoint_token(rng, 24, 8, _MAX_FINITE_F32_BITS))
        elif k == 2:
            out.append(_subnormal_token(rng))
        elif k == 3:
            out.append(_big_token(rng))
        elif k == 4:
            out.append(_integer_token(rng))
        elif k == 5:
            out.append(_variant_token(rng))
        else:
            out.append(_long_token(rng))
    return out


def config3(seed: int = 3, n: int = 2_000_000) -> bytes:
    """Hard cases, newline separated (parsed to both binary64 and binary32)."""
    rng = np.random.default_rng(seed)
    return join_tokens(hard_tokens(rng, n))


# ---------------------------------------------------------------------------
# invalid tokens (grammar rejections)
# ---------------------------------------------------------------------------

INVALID_EXAMPLES = [
    "", ".", "+", "-", "+-1", "--1", "e5", "E5", ".e5", "1e", "1e+", "1e-",
    "1.2.3", "1..2", "1e5.0", "1e5e5", "0x1p3", "inf", "nan", "-inf", "NaN",
    "1_000", "1 2", " 1", "1 ", "1,5", "١", "1f", "1d", "++1", "1e++5",
    "1-", "1+", "e", ".-1", "-.", "+.", "1.e", "abc", "0x10",
]


# ---------------------------------------------------------------------------
# batched and served workloads (configs 4 and 5)
# ---------------------------------------------------------------------------

def lognormal_sizes(rng, count: int, median: float, sigma: float, lo: int, hi: int):
    s = np.exp(rng.normal(np.log(median), sigma, size=count))
    return np.clip(s, lo, hi).astype(np.int64)


def config4_sizes(seed: int = 4, nbuf: int = 4096):
    """4096 buffer sizes, lognormal with median 256 KiB, clipped to
    [1 KiB, 16 MiB] (sigma 1.5)."""
    rng = np.random.default_rng(seed)
    return lognormal_sizes(rng, nbuf, 256 * 1024, 1.5, 1024, 16 * 1024 * 1024)


def slice_plan(rng, pool: bytes, sizes):
    """Cut buffers of the given sizes out of a token pool: each buffer starts
    at the beginning of a token chosen at random; the last token of a buffer
    may be cut short.  Returns a list of (start, length) into ``pool``,
    wrapping is avoided by drawing starts within the pool."""
    starts = np.flatnonzero(np.frombuffer(pool, dtype=np.uint8) == 10) + 1
    starts = np.concatenate([[0], starts[:-1]])
    out = []
    n = len(pool)
    for sz in np.asarray(sizes).tolist():
        sz = min(int(sz), n)
        hi = np.searchsorted(starts, n - sz, side="right")
        st = int(starts[int(rng.integers(0, max(hi, 1)))])
        out.append((st, sz))
    return out


def token_pool(seed: int, n: int, kind: str = "mixed") -> bytes:
    rng = np.random.default_rng(seed)
    if kind == "mixed":
        return join_tokens(mixed_tokens(rng, n))
    if kind == "uniform":
        return join_tokens(uniform_shortest(rng, n))
    if kind == "hard":
        return join_tokens(hard_tokens(rng, n))
    raise ValueError(kind)


def config5_requests(seed: int, rate: float, count: int):
    """Open-loop Poisson arrivals for the serving workload.

    Returns arrays (t_arrive seconds, size bytes, is_f32, is_hard).  Sizes are
    lognormal with median 64 KiB, sigma 1.5, clipped to [512 B, 8 MiB]; 10% of
    requests ask for binary32; 1% carry hard cases."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    sizes = lognormal_sizes(rng, count, 64 * 1024, 1.5, 512, 8 * 1024 * 1024)
    is_f32 = rng.random(count) < 0.10
    is_hard = rng.random(count) < 0.01
    return t, sizes, is_f32, is_hard


def geojson_document(seed: int, nfeat: int, npts: int) -> bytes:
    """A GeoJSON-like document (the shape of the canada test file): nfeat
    polygon features of npts [longitude, latitude] pairs printed with 6-15
    fraction digits, keys and strings around them."""
    rng = np.random.default_rng(seed)
    out = ['{"type":"FeatureCollection","features":[']
    for f in range(nfeat):
        xs = rng.uniform(-180, 180, npts)
        ys = rng.uniform(-90, 90, npts)
        kx = rng.integers(6, 16, npts)
        ky = rng.integers(6, 16, npts)
        ring = ",".join("[%.*f,%.*f]" % (int(a), float(x), int(b), float(y))
                        for a, x, b, y in zip(kx, xs, ky, ys))
        out.append('{"type":"Feature","properties":{"name":"n%d"},"geometry":'
                   '{"type":"Polygon","coordinates":[[%s]]}}%s'
                   % (f, ring, "," if f + 1 < nfeat else ""))
    out.append("]}\n")
    return "".join(out).encode()


# Delimiters that make the numbers of such a document its tokens.
JSON_DELIMS = b'[]{},:" \n'


def hex_tokens(rng, n: int):
    """Hexadecimal floating-point tokens: random doubles in their own hex
    form, long significands across the whole exponent range, exact ties of
    53-, 24-, 11- and 8-bit significands (and their neighbours), upper-case
    and fraction-only forms."""
    toks = []
    hexd = list("0123456789abcdef")
    for _ in range(n):
        k = int(rng.integers(0, 5))
        if k == 0:
            x = float(rng.standard_normal() * 10.0 ** rng.integers(-300, 300))
            toks.append(x.hex())
        elif k == 1:
            digits = "".join(rng.choice(hexd, int(rng.integers(1, 40))))
            toks.append("0x%s.%sp%d" % (digits[:3] or "0", digits[3:],
                                       int(rng.integers(-1200, 1100))))
        elif k == 2:
            p = int(rng.choice([53, 24, 11, 8]))
            m = int(rng.integers(2 ** (p - 1), 2 ** p)) * 2 + 1 + int(rng.integers(-1, 2))
            m <<= int(rng.integers(0, 12))
            lo, hi = {53: (-1130, 1000), 24: (-180, 110), 11: (-40, 10), 8: (-150, 110)}[p]
            toks.append("%s0x%xp%d" % ("-" if rng.integers(0, 2) else "", m,
                                       int(rng.integers(lo, hi))))
        elif k == 3:
            digits = "".join(rng.choice(list("0123456789ABCDEF"), int(rng.integers(1, 20))))
            toks.append("%s0X.%sP%+d" % ("-" if rng.integers(0, 2) else "", digits,
                                         int(rng.integers(-60, 60))))
        else:
            toks.append("0x%x.%xp%d" % (int(rng.integers(0, 2 ** 16)), int(rng.integers(0, 2 ** 20)),
                                        int(rng.integers(-30, 30))))
    return toks


def json_tricky_document(seed: int, nitems: int, indent=None, long_strings=False) -> bytes:
    """A JSON document whose strings and keys hold digits, commas, colons,
    brackets, escaped quotes, backslash runs and unicode escapes, next to
    numbers of every JSON form (integers, fractions, exponents, signs),
    true/false/null and nested containers.  With long_strings some strings
    run for thousands of bytes (across tiles and blocks) and end in long
    backslash runs."""
    import json

    rng = np.random.default_rng(seed)
    pieces = ["12", "3,4", "5.6e7", '"', '\\', '\\"', "-0", ":", "[", "]", "{", "}", " ",
              "é", "☃", "true", "1e5", "x", "\t", "\n"]

    def rstring():
        k = int(rng.integers(0, 8))
        s = "".join(pieces[int(i)] for i in rng.integers(0, len(pieces), k))
        if long_strings and rng.random() < 0.05:
            s += "".join(pieces[int(i)] for i in rng.integers(0, len(pieces), 2000))
            s += "\\" * int(rng.integers(1, 40))
        return s

    def rnumber():
        r = rng.random()
        if r < 0.3:
            return int(rng.integers(-10 ** 12, 10 ** 12))
        if r < 0.6:
            return float(rng.standard_normal() * 10.0 ** int(rng.integers(-30, 30)))
        if r < 0.7:
            return int(rng.integers(0, 10))
        if r < 0.8:
            return float(rng.uniform(-180, 180))
        return float(rng.random())

    def value(depth):
        r = rng.random()
        if depth < 3 and r < 0.15:
            return [value(depth + 1) for _ in range(int(rng.integers(0, 6)))]
        if depth < 3 and r < 0.3:
            return {rstring(): value(depth + 1) for _ in range(int(rng.integers(0, 5)))}
        if r < 0.55:
            return rnumber()
        if r < 0.8:
            return rstring()
        return [True, False, None][int(rng.integers(0, 3))]

    doc = [value(0) for _ in range(nitems)]
    ensure_ascii = bool(rng.random() < 0.5)
    return (json.dumps(doc, indent=indent, ensure_ascii=ensure_ascii) + "\n").encode()


def csv_table(rng, rows: int, max_cols: int = 80, extra_space: bool = False, crlf: bool = False,
              trailing_newline: bool = True, long_field_every: int = 0) -> str:
    """A CSV table (no quoting) of `rows` rows of 1..max_cols fields: empty
    fields, words, decimals of all magnitudes, integers, exponents and
    out-of-range values; with extra_space, spaces around some fields; with
    crlf, rows end in CR LF; long_field_every > 0 puts a 3-9 KB word field in
    every such row (rows longer than a 4 KiB window)."""
    lines = []
    for r in range(rows):
        ncol = int(rng.integers(1, max_cols))
        fields = []
        for _ in range(ncol):
            k = rng.integers(0, 6)
            if k == 0:
                f = ""
            elif k == 1:
                f = "abc%d" % rng.integers(0, 100)
            elif k == 2:
                f = "%.17g" % (rng.standard_normal() * 10.0 ** rng.integers(-30, 30))
            elif k == 3:
                f = str(int(rng.integers(-10 ** 6, 10 ** 6)))
            elif k == 4:
                f = "-%d.%de%d" % (rng.integers(0, 99), rng.integers(0, 99), rng.integers(-20, 20))
            else:
                f = "1e999"
            if extra_space and f and rng.integers(0, 2):
                f = " " * int(rng.integers(1, 3)) + f + " " * int(rng.integers(0, 2))
            fields.append(f)
        if long_field_every and r % long_field_every == 0:
            fields.insert(int(rng.integers(0, len(fields) + 1)), "w" * int(rng.integers(3000, 9000)))
        lines.append(",".join(fields))
    sep = "\r\n" if crlf else "\n"
    return sep.join(lines) + (sep if trailing_newline else "")


# Columns of the CSV benchmark table: id, name, lon, lat, value, big, flag,
# price, qty, note; the numeric columns selected are lon, lat, value, big
# and price.
CSV_BENCH_COLUMNS = (1 << 2) | (1 << 3) | (1 << 4) | (1 << 5) | (1 << 7)


def csv_benchmark_table(seed: int, rows: int) -> bytes:
    """A ten-column CSV table (no quoting, '\\n' rows): an integer id, a
    word, two coordinates with 6-15 fraction digits, a uniform [0,1) double
    in shortest digits, a random double as %.17e, a flag word, a price with
    two decimals, an integer quantity and a word; see CSV_BENCH_COLUMNS."""
    rng = np.random.default_rng(seed)
    lon = coordinates(rng, rows)
    lat = coordinates(rng, rows)
    val = uniform_shortest(rng, rows)
    big = random_bits_e17(rng, rows)
    price = rng.integers(0, 10 ** 7, rows).tolist()
    qty = rng.integers(0, 1000, rows).tolist()
    flags = rng.integers(0, 3, rows).tolist()
    words = ["alpha", "beta", "gamma", "delta", "eps", "zeta12", "eta", "theta"]
    wi = rng.integers(0, len(words), (rows, 2)).tolist()
    out = []
    for i in range(rows):
        out.append("%d,%s,%s,%s,%s,%s,%s,%d.%02d,%d,%s\n" % (
            i, words[wi[i][0]], lon[i], lat[i], val[i], big[i], ("yes", "no", "")[flags[i]],
            price[i] // 100, price[i] % 100, qty[i], words[wi[i][1]]))
    return "".join(out).encode()
