"""Reductions over parsed values, written out plainly.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's benchmark keeps a running minimum of the parsed values
(Section 12); the library can also keep their exact sum.  The contract
restated here, from first principles:

* the values summed are those of the tokens with status OK whose encoding is
  not a NaN (the same set the minimum, maximum and count cover);
* every such value is a dyadic rational m * 2^e, so their sum is an exact
  rational; the result is that sum rounded once, to nearest with ties to
  even, to binary64 (whatever the output format of the tokens), with
  overflow to an infinity of the sum's sign;
* infinities follow IEEE addition: +inf if some value is +inf and none is
  -inf, -inf in the mirror case, the canonical quiet NaN if both occur;
* an exact zero sum is +0, except that a set of values that are all -0 (or
  an empty set) sums to -0 and +0 respectively, as IEEE addition from +0
  gives: -0 + -0 = -0 and the empty sum is +0.  (Any nonzero or +0 value in
  the set makes an exact zero sum +0.)

``exact_sum`` also reports whether the rounding was exact.
"""

from fractions import Fraction

from .exact import BINARY64, STATUS_OK
from .grammar import round_binary

# (precision p, bias, exponent width) of the encodings the parser writes
_FIELDS = {
    "f64": (53, 1023, 11),
    "f32": (24, 127, 8),
    "f16": (11, 15, 5),
    "bf16": (8, 127, 8),
}

QNAN64 = 0x7FF8000000000000
INF64 = 0x7FF0000000000000
SIGN64 = 1 << 63


def decode(bits: int, fmt: str):
    """(kind, neg, value) of an encoding: kind is 'nan', 'inf' or 'finite';
    value is the exact Fraction of a finite encoding (IEEE 754 binary
    interchange layout: sign, biased exponent, trailing significand)."""
    p, bias, ew = _FIELDS[fmt]
    t = p - 1  # trailing significand bits
    width = 1 + ew + t
    neg = (bits >> (width - 1)) & 1 == 1
    field = (bits >> t) & ((1 << ew) - 1)
    frac = bits & ((1 << t) - 1)
    if field == (1 << ew) - 1:
        return ("nan" if frac else "inf"), neg, None
    if field == 0:  # subnormal or zero: frac * 2^(1 - bias - t)
        mag = Fraction(frac) * Fraction(2) ** (1 - bias - t)
    else:
        mag = Fraction(frac + (1 << t)) * Fraction(2) ** (field - bias - t)
    return "finite", neg, (-mag if neg else mag)


def exact_sum(bits, status, fmt: str = "f64"):
    """(binary64 encoding of the rounded sum, exact flag) over the tokens
    with status OK and a non-NaN value (module docstring)."""
    total = Fraction(0)
    pos_inf = neg_inf = False
    all_neg_zero = True  # every summed value so far is -0 (vacuously at start)
    count = 0
    for b, s in zip(bits, status):
        if s != STATUS_OK:
            continue
        kind, neg, v = decode(int(b), fmt)
        if kind == "nan":
            continue
        count += 1
        if kind == "inf":
            pos_inf |= not neg
            neg_inf |= neg
            all_neg_zero = False
            continue
        if not (v == 0 and neg):
            all_neg_zero = False
        total += v
    if pos_inf and neg_inf:
        return QNAN64, False
    if pos_inf or neg_inf:
        return (INF64 | (SIGN64 if neg_inf else 0)), True
    if total == 0:
        return (SIGN64 if (count and all_neg_zero) else 0), True
    neg = total < 0
    mag = -total if neg else total
    # mag = M * 2^B with M odd or B = 0... any exact M * 2^B form will do
    den = mag.denominator  # a power of two
    B = -(den.bit_length() - 1)
    M = mag.numerator
    enc, _status = round_binary(neg, M, B, BINARY64)
    kind, _neg, back = decode(enc, "f64")
    exact = kind == "finite" and back == total
    return enc, exact
