"""CPU oracle for exact decimal -> binary64/binary32 parsing.

TEST INFRASTRUCTURE ONLY: importable from ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; never from the product path.
It shares no code with the HIP implementation.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against the paper's worked examples, brute force over tiny formats, CPython's
correctly rounded ``float()`` and glibc ``strtof``, and round-trip invariants.
The status codes and NaN payload are the library contract (the paper leaves
them open) and are pinned by golden files only.
"""

from .exact import (
    BFLOAT16,
    BINARY16,
    BINARY32,
    BINARY64,
    FORMATS,
    STATUS_INVALID,
    STATUS_OK,
    STATUS_OUT_OF_RANGE,
    ROUND_DOWN,
    ROUND_NEAREST,
    ROUND_TOWARD_ZERO,
    ROUND_UP,
    ROUNDING_MODES,
    Format,
    round_decimal,
)
from .grammar import (
    FLAG_CSV,
    FLAG_HEX,
    FLAG_INFNAN,
    FLAG_JSON,
    FLAG_JSON_DOCUMENT,
    FLAG_REJECT_PLUS,
    FLAG_ROUND_DOWN,
    FLAG_ROUND_MASK,
    FLAG_ROUND_TOWARD_ZERO,
    FLAG_ROUND_UP,
    csv_number_spans,
    decompose,
    json_number_spans,
    parse_buffer,
    parse_csv,
    parse_json_document,
    parse_token,
    rounding_mode,
    split_tokens,
)

__all__ = [
    "BFLOAT16",
    "BINARY16",
    "BINARY32",
    "BINARY64",
    "FLAG_CSV",
    "FLAG_HEX",
    "FLAG_INFNAN",
    "FLAG_JSON",
    "FLAG_JSON_DOCUMENT",
    "FLAG_REJECT_PLUS",
    "FLAG_ROUND_DOWN",
    "FLAG_ROUND_MASK",
    "FLAG_ROUND_TOWARD_ZERO",
    "FLAG_ROUND_UP",
    "ROUND_DOWN",
    "ROUND_NEAREST",
    "ROUND_TOWARD_ZERO",
    "ROUND_UP",
    "ROUNDING_MODES",
    "rounding_mode",
    "FORMATS",
    "Format",
    "STATUS_INVALID",
    "STATUS_OK",
    "STATUS_OUT_OF_RANGE",
    "csv_number_spans",
    "decompose",
    "json_number_spans",
    "parse_buffer",
    "parse_csv",
    "parse_json_document",
    "parse_token",
    "round_decimal",
    "split_tokens",
]
