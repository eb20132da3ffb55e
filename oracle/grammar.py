"""Token splitting and decimal grammar for the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/exact.py``).

Section 4 of the paper lists the steps of reading a decimal string: the string
is explicitly delimited and nothing outside it is read; an optional leading
sign ('+' may be disallowed by some formats); a significand of digits with an
optional '.', holding at least one digit; an optional 'e'/'E' exponent with its
own sign, which must carry digits (the paper lets a parser either fail or
truncate there; this library fails).  The exact value is then the integer of
all significand digits times ten to the explicit exponent minus the number of
fraction digits.

Buffers hold many such strings separated by delimiter bytes: the tokens are
the maximal non-empty runs of non-delimiter bytes, in buffer order.  That
convention, the status codes and the NaN payload for rejected tokens are the
library contract; the paper does not fix them.
"""

import re

from .exact import (BINARY32, BINARY64, FORMATS, ROUND_DOWN, ROUND_NEAREST,
                    ROUND_TOWARD_ZERO, ROUND_UP, STATUS_INVALID, STATUS_OK, round_decimal)

# [+-]? ( D+ ('.' D*)? | '.' D+ ) ( [eE] [+-]? D+ )?   -- whole token
_TOKEN_RE = re.compile(
    rb"([+-]?)(?:([0-9]+)(?:\.([0-9]*))?|\.([0-9]+))(?:[eE]([+-]?[0-9]+))?"
)

FLAG_REJECT_PLUS = 1
# JSON numbers: the number grammar of the JSON specification (RFC 8259,
# section 6): no '+' (the JSON rule the paper mentions in Section 4), no
# leading zeros, at least one digit on each side of a '.'.
FLAG_JSON = 2
# inf, infinity and nan in any letter case, with an optional sign: +-infinity
# and the quiet NaN (the sign bit follows the sign).
FLAG_INFNAN = 4
# Hexadecimal floating-point tokens (Appendix C): 0x, hexadecimal digits with
# an optional point, an optional binary exponent p[+-]digits; the value is
# the hexadecimal significand times 16^-(fraction nibbles) times 2^exponent.
FLAG_HEX = 8
# Rounding direction, a two-bit field: 0 nearest (ties to even), then toward
# zero, toward +infinity and toward -infinity.
FLAG_ROUND_MASK = 0x30
FLAG_ROUND_TOWARD_ZERO = 0x10
FLAG_ROUND_UP = 0x20
FLAG_ROUND_DOWN = 0x30
_MODE_OF_FLAGS = {0: ROUND_NEAREST, FLAG_ROUND_TOWARD_ZERO: ROUND_TOWARD_ZERO,
                  FLAG_ROUND_UP: ROUND_UP, FLAG_ROUND_DOWN: ROUND_DOWN}


def rounding_mode(flags: int) -> str:
    return _MODE_OF_FLAGS[flags & FLAG_ROUND_MASK]

_HEX_RE = re.compile(
    rb"([+-]?)0[xX](?:([0-9a-fA-F]+)(?:\.([0-9a-fA-F]*))?|\.([0-9a-fA-F]+))(?:[pP]([+-]?[0-9]+))?"
)

_JSON_RE = re.compile(rb"-?(?:0|[1-9][0-9]*)(?:\.[0-9]+)?(?:[eE][+-]?[0-9]+)?")
_INFNAN_RE = re.compile(rb"([+-]?)(?:inf|infinity|nan)", re.IGNORECASE)


def decompose(tok: bytes, flags: int = 0):
    """Return (neg, D, E) with value (-1)^neg * D * 10^E, or None if invalid."""
    m = _TOKEN_RE.fullmatch(tok)
    if m is None:
        return None
    if (flags & FLAG_JSON) and _JSON_RE.fullmatch(tok) is None:
        return None
    sign, int_digits, frac_digits, only_frac, exp = m.groups()
    if sign == b"+" and (flags & FLAG_REJECT_PLUS):
        return None
    if only_frac is not None:
        int_digits, frac_digits = b"", only_frac
    if frac_digits is None:
        frac_digits = b""
    digits = int_digits + frac_digits
    D = int(digits)
    E = (int(exp) if exp is not None else 0) - len(frac_digits)
    return sign == b"-", D, E


def decompose_hex(tok: bytes, flags: int = 0):
    """(neg, M, B) with value (-1)^neg * M * 2^B for a hexadecimal token, or
    None."""
    m = _HEX_RE.fullmatch(tok)
    if m is None:
        return None
    sign, int_digits, frac_digits, only_frac, exp = m.groups()
    if sign == b"+" and (flags & (FLAG_REJECT_PLUS | FLAG_JSON)):
        return None
    if only_frac is not None:
        int_digits, frac_digits = b"", only_frac
    if frac_digits is None:
        frac_digits = b""
    M = int(int_digits + frac_digits, 16)
    B = (int(exp) if exp is not None else 0) - 4 * len(frac_digits)
    return sign == b"-", M, B


def round_binary(neg: bool, M: int, B: int, fmt, mode: str = ROUND_NEAREST):
    """Round (-1)^neg * M * 2^B to ``fmt`` (through the decimal rounding, as
    M * 2^B = M * 5^-B * 10^B exactly)."""
    if M == 0:
        return round_decimal(neg, 0, 0, fmt, mode)
    top = M.bit_length() + B  # value in [2^(top-1), 2^top)
    if top - 1 > fmt.emax + 1:  # at least 2^(emax+2): overflows in every mode
        return round_decimal(neg, 1, 400, fmt, mode)
    if top < fmt.emin - fmt.p - 1:  # below 2^(emin-p-1): as any such tiny value
        return round_decimal(neg, 1, -400, fmt, mode)
    if B >= 0:
        return round_decimal(neg, M << B, 0, fmt, mode)
    return round_decimal(neg, M * 5 ** (-B), B, fmt, mode)


def parse_token(tok: bytes, fmt=BINARY64, flags: int = 0):
    """(bits, status) for one token."""
    if isinstance(fmt, str):
        fmt = FORMATS[fmt]
    mode = rounding_mode(flags)
    if flags & FLAG_HEX:
        parts = decompose_hex(tok, flags)
        if parts is not None:
            return round_binary(*parts, fmt, mode)
    if flags & FLAG_INFNAN:
        m = _INFNAN_RE.fullmatch(tok)
        if m is not None and not (m.group(1) == b"+" and flags & (FLAG_REJECT_PLUS | FLAG_JSON)):
            sign = fmt.sign_bit if m.group(1) == b"-" else 0
            special = fmt.qnan_bits if tok[-1:] in (b"n", b"N") else fmt.inf_bits
            return sign | special, STATUS_OK
    parts = decompose(tok, flags)
    if parts is None:
        return fmt.qnan_bits, STATUS_INVALID
    neg, D, E = parts
    return round_decimal(neg, D, E, fmt, mode)


def _delim_class(delims: bytes) -> bytes:
    if len(delims) == 0:
        raise ValueError("the delimiter set must not be empty")
    body = b"".join(b"\\x%02x" % c for c in sorted(set(delims)))
    return b"[^" + body + b"]+"


def split_tokens(buf: bytes, delims: bytes = b"\n"):
    """List of (start, end) byte ranges of the tokens of ``buf``."""
    pat = re.compile(_delim_class(delims))
    return [(mt.start(), mt.end()) for mt in pat.finditer(buf)]


def parse_buffer(buf: bytes, fmt="f64", delims: bytes = b"\n", flags: int = 0):
    """Parse every token of ``buf``.  Returns (bits list, status list)."""
    if isinstance(fmt, str):
        fmt = FORMATS[fmt]
    pat = re.compile(_delim_class(delims))
    bits, status = [], []
    for mt in pat.finditer(buf):
        b, s = parse_token(mt.group(0), fmt, flags)
        bits.append(b)
        status.append(s)
    return bits, status


__all__ = [
    "BINARY32",
    "BINARY64",
    "FLAG_HEX",
    "FLAG_INFNAN",
    "FLAG_JSON",
    "FLAG_REJECT_PLUS",
    "decompose",
    "decompose_hex",
    "parse_buffer",
    "parse_token",
    "split_tokens",
]


# ---------------------------------------------------------------------------
# JSON documents (structural index).  Number tokens of a JSON text are the
# runs of bytes outside strings that are neither structural characters,
# whitespace nor quotes, and that start with '-' or a digit (true, false and
# null start with a letter).  A quote preceded by an odd number of
# consecutive backslashes is escaped: it neither opens nor closes a string
# (inside a string that is JSON's escape rule).  Each number token is read
# with the JSON number grammar.  The library contract for documents; the
# paper's benchmark reads such a file (Section 12).
# ---------------------------------------------------------------------------
FLAG_JSON_DOCUMENT = 0x40
JSON_STRUCTURE = b"[]{},:"
JSON_WHITESPACE = b" \t\n\r"


def json_number_spans(buf: bytes):
    """(start, end) of every number token of a JSON text, in order."""
    spans = []
    in_string = False
    backslashes = 0  # consecutive backslashes just before the current byte
    start = -1       # start of the run being read, -1 outside a run
    for i, c in enumerate(buf):
        quote = c == 0x22 and backslashes % 2 == 0
        token_byte = not in_string and not quote and c not in JSON_STRUCTURE \
            and c not in JSON_WHITESPACE
        if quote:
            in_string = not in_string
        backslashes = backslashes + 1 if c == 0x5C else 0
        if token_byte and start < 0:
            start = i
        elif not token_byte and start >= 0:
            spans.append((start, i))
            start = -1
    if start >= 0:
        spans.append((start, len(buf)))
    return [(a, b) for a, b in spans if buf[a] == 0x2D or 0x30 <= buf[a] <= 0x39]


def parse_json_document(buf: bytes, fmt="f64", flags: int = 0):
    """(bits list, status list) of the number tokens of a JSON text, each
    read with the JSON number grammar."""
    bits, status = [], []
    for a, b in json_number_spans(buf):
        v, s = parse_token(buf[a:b], fmt, flags | FLAG_JSON)
        bits.append(v)
        status.append(s)
    return bits, status


# ---------------------------------------------------------------------------
# CSV number columns: the text is a table whose rows end at '\n' and whose
# fields are separated by ','; a field's column is the number of ',' bytes
# before it in its row (0-based).  Tokens are the maximal runs of bytes that
# are not delimiters (',' and '\n' always are; the caller's delimiter set can
# add others, such as spaces or '\r'), and a token belongs to the column of
# the field holding it.  Only tokens of the selected columns (a 64-bit mask
# over columns 0..63) are parsed and numbered, in text order, with the
# context's grammar flags.  Fields are not quoted.  The library contract for
# CSV input; the paper names such structural parsing as future work
# (Section 13).
# ---------------------------------------------------------------------------
FLAG_CSV = 0x80


def csv_number_spans(buf: bytes, columns: int, delims: bytes = b",\n"):
    """(start, end) of every token of the selected columns, in order."""
    seps = set(delims) | {0x2C, 0x0A}
    spans = []
    col = 0
    i, n = 0, len(buf)
    while i < n:
        c = buf[i]
        if c == 0x0A:
            col = 0
        elif c == 0x2C:
            col += 1
        if c in seps:
            i += 1
            continue
        j = i
        while j < n and buf[j] not in seps:
            j += 1
        if col < 64 and (columns >> col) & 1:
            spans.append((i, j))
        i = j
    return spans


def parse_csv(buf: bytes, columns: int, fmt="f64", delims: bytes = b",\n", flags: int = 0):
    """(bits list, status list) of the tokens of the selected columns."""
    bits, status = [], []
    for a, b in csv_number_spans(buf, columns, delims):
        v, s = parse_token(buf[a:b], fmt, flags)
        bits.append(v)
        status.append(s)
    return bits, status
