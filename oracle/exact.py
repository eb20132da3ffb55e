"""Exact CPU oracle: decimal ASCII -> nearest IEEE-754 binary64 / binary32.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports this module:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code, table or constant generator with
the HIP path.

What it computes is the plain definition of the problem, not the paper's fast
algorithm:

* the result is the binary floating-point number nearest to the exact value of
  the decimal string, ties broken toward the even significand (Section 1,
  the ``round`` entry of Table 1, and Section 6);
* normal numbers have a p-bit significand in [2^(p-1), 2^p) and exponent in
  [emin, emax]; below 2^emin the subnormal quantum 2^(emin-p+1) applies
  (Section 2, Table 2, Section 9.3);
* a value that rounds past the largest finite number becomes infinity, a
  nonzero value that rounds to nothing becomes zero (Sections 4 and 8);
* the sign is applied last, by symmetry (Sections 5 and 6);
* the biased exponent field is p + bias with bias 1023 / 127, field 0 holds
  subnormals and the all-ones field holds infinities (Section 10).

All arithmetic uses Python's unbounded integers.  No floating point, no library
parser.  Every rounding is an integer division with remainder followed by
round-half-to-even, so the reader can check each step by eye.

The status codes and the quiet-NaN payload for rejected strings are the
library contract (the paper leaves them open); they are pinned by golden
files, not by the paper.
"""

import sys
from dataclasses import dataclass

# Tokens may carry tens of thousands of digits; CPython limits int <-> str
# conversions to 4300 digits by default.
if hasattr(sys, "set_int_max_str_digits"):
    sys.set_int_max_str_digits(0)

STATUS_OK = 0
STATUS_INVALID = 1
STATUS_OUT_OF_RANGE = 2

# Rounding-direction attributes of IEEE 754.  The paper works with
# round-to-nearest, ties to even, and notes (the footnote of Section 6) that
# the approach extends to the other modes; these are the three directed
# ones.
ROUND_NEAREST = "nearest"
ROUND_TOWARD_ZERO = "zero"
ROUND_UP = "up"        # toward +infinity
ROUND_DOWN = "down"    # toward -infinity
ROUNDING_MODES = (ROUND_NEAREST, ROUND_TOWARD_ZERO, ROUND_UP, ROUND_DOWN)


def _away_from_zero(mode: str, neg: bool) -> bool:
    """For a directed mode: does the magnitude round up (away from zero)?

    Toward zero truncates the magnitude for either sign; toward +infinity
    raises the magnitude of positive values and truncates negative ones;
    toward -infinity the reverse.
    """
    if mode == ROUND_TOWARD_ZERO:
        return False
    if mode == ROUND_UP:
        return not neg
    if mode == ROUND_DOWN:
        return neg
    raise ValueError("not a directed rounding mode: %r" % (mode,))


@dataclass(frozen=True)
class Format:
    """A binary interchange-style format.

    p     -- significand precision in bits, hidden bit included
    emin  -- smallest normal unbiased exponent
    emax  -- largest unbiased exponent
    ebits -- width of the biased exponent field
    """

    name: str
    p: int
    emin: int
    emax: int
    ebits: int

    @property
    def nbits(self) -> int:
        return 1 + self.ebits + (self.p - 1)

    @property
    def bias(self) -> int:
        return self.emax

    @property
    def sign_bit(self) -> int:
        return 1 << (self.nbits - 1)

    @property
    def inf_bits(self) -> int:
        return ((1 << self.ebits) - 1) << (self.p - 1)

    @property
    def qnan_bits(self) -> int:
        # canonical quiet NaN: all-ones exponent, top fraction bit set
        return self.inf_bits | (1 << (self.p - 2))


# Section 2, Table 2: binary64 has 53 significand bits and exponents
# -1022..+1023; binary32 has 24 bits and -126..+127.
BINARY64 = Format("binary64", 53, -1022, 1023, 11)
BINARY32 = Format("binary32", 24, -126, 127, 8)
# The paper names binary16 among the standard formats (Section 2); bfloat16
# keeps binary32's exponent range with an 8-bit significand.  Both follow
# the same definition of rounding.
BINARY16 = Format("binary16", 11, -14, 15, 5)
BFLOAT16 = Format("bfloat16", 8, -126, 127, 8)
FORMATS = {"f64": BINARY64, "f32": BINARY32, "f16": BINARY16, "bf16": BFLOAT16}


def _decimal_digits(n: int) -> int:
    """Number of decimal digits of a positive integer."""
    return len(str(n))


def _overflow_decade(fmt: Format) -> int:
    """Smallest k with 10^k >= 2^(emax+1).

    Any value >= 10^k is at least 2^(emax+1), which is beyond the largest
    finite value plus half an ulp, so it rounds to infinity.
    """
    k = 0
    limit = 1 << (fmt.emax + 1)
    while 10 ** k < limit:
        k += 1
    return k


def _underflow_decade(fmt: Format) -> int:
    """Largest k (k <= 0) with 10^k <= 2^(emin-p), i.e. half the smallest subnormal.

    Any value < 10^k is strictly below half of the smallest subnormal and
    rounds to zero.
    """
    j = 0
    limit = 1 << (fmt.p - fmt.emin)  # 2^(p-emin) = 1 / 2^(emin-p)
    while 10 ** j < limit:
        j += 1
    return -j


_DECADE_CACHE = {}


def _decades(fmt: Format):
    key = fmt
    if key not in _DECADE_CACHE:
        _DECADE_CACHE[key] = (_overflow_decade(fmt), _underflow_decade(fmt))
    return _DECADE_CACHE[key]


def round_decimal(neg: bool, D: int, E: int, fmt: Format, mode: str = ROUND_NEAREST):
    """Round the exact value (-1)^neg * D * 10^E to ``fmt``.

    D >= 0 and E are arbitrary integers.  Returns (bits, status) where bits is
    the IEEE encoding as an unsigned integer.

    ``mode`` is the rounding direction.  Directed modes follow IEEE 754: the
    result is the representable value next to v on the mode's side (v itself
    when it is representable); past the largest finite value a mode that
    truncates the magnitude delivers that largest value and the others
    infinity, both with status OUT_OF_RANGE (the IEEE overflow condition);
    a nonzero value below the smallest subnormal becomes zero (status
    OUT_OF_RANGE) or, rounding away from zero, the smallest subnormal.
    """
    sign = fmt.sign_bit if neg else 0
    if D == 0:
        # zero significand: signed zero, exact
        return sign, STATUS_OK
    nearest = mode == ROUND_NEAREST
    away = False if nearest else _away_from_zero(mode, neg)
    largest = fmt.inf_bits - 1  # largest finite encoding
    overflow = (sign | (fmt.inf_bits if nearest or away else largest), STATUS_OUT_OF_RANGE)

    # Magnitude pre-checks keep 10^|E| finite for absurd exponents.  The value
    # lies in [10^(n-1+E), 10^(n+E)).
    n = _decimal_digits(D)
    over_k, under_k = _decades(fmt)
    if n - 1 + E >= over_k:
        return overflow
    if n + E <= under_k:
        # strictly between 0 and half the smallest subnormal
        if away:
            return sign | 1, STATUS_OK
        return sign, STATUS_OUT_OF_RANGE

    # v = N / Dn exactly, both positive integers.
    if E >= 0:
        N, Dn = D * 10 ** E, 1
    else:
        N, Dn = D, 10 ** (-E)

    # e = floor(log2(v)).  From bit lengths v is in [2^(e0-1), 2^(e0+1)).
    e0 = N.bit_length() - Dn.bit_length()
    if e0 >= 0:
        ge = N >= (Dn << e0)
    else:
        ge = (N << (-e0)) >= Dn
    e = e0 if ge else e0 - 1

    # Quantum of the result: 2^(e-p+1) for normal values, the fixed subnormal
    # quantum 2^(emin-p+1) below 2^emin.
    k = max(e, fmt.emin) - (fmt.p - 1)

    # Integer significand at that quantum: v / 2^k = num / den.
    if k >= 0:
        num, den = N, Dn << k
    else:
        num, den = N << (-k), Dn
    m, r = divmod(num, den)

    if nearest:
        # Round half to even.
        twice_r = 2 * r
        if twice_r > den or (twice_r == den and (m & 1)):
            m += 1
    elif away and r != 0:
        # Directed: the magnitude is m (exact or truncated) or the next one up.
        m += 1

    # Rounding may carry into a new binade.
    if m == (1 << fmt.p):
        m >>= 1
        k += 1

    if m == 0:
        # nonzero decimal that rounds to zero: total underflow
        return sign, STATUS_OUT_OF_RANGE

    hidden = 1 << (fmt.p - 1)
    if m < hidden:
        # subnormal: exponent field 0, fraction holds m (quantum 2^(emin-p+1))
        return sign | m, STATUS_OK

    unbiased = k + fmt.p - 1
    if unbiased > fmt.emax:
        return overflow
    field = unbiased + fmt.bias
    return sign | (field << (fmt.p - 1)) | (m - hidden), STATUS_OK
