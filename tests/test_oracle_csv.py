"""Pins of the oracle's CSV column selection (csv_number_spans) against
Python's csv module on generated tables, and its special cases."""

import csv
import io

import numpy as np
import pytest

from gen.workloads import csv_table as random_table
from oracle import csv_number_spans, parse_csv, parse_token, split_tokens


def csv_module_tokens(text, columns, split_spaces):
    out = []
    for row in csv.reader(io.StringIO(text, newline=""), delimiter=",", quoting=csv.QUOTE_NONE):
        for col, field in enumerate(row):
            if col < 64 and (columns >> col) & 1:
                out += field.split() if split_spaces else ([field] if field else [])
    return out


@pytest.mark.parametrize("seed", range(8))
def test_spans_match_csv_module(seed):
    rng = np.random.default_rng(400 + seed)
    extra_space = seed % 2 == 1
    crlf = seed % 4 == 3
    text = random_table(rng, 60, extra_space=extra_space, crlf=crlf,
                        trailing_newline=seed % 3 != 0, long_field_every=seed % 5)
    buf = text.encode()
    delims = b",\n" + (b" " if extra_space else b"") + (b"\r" if crlf else b"")
    for columns in [1, 0b101, 1 << 63, (1 << 64) - 1, int(rng.integers(0, 1 << 62)), 0]:
        got = [buf[a:b].decode() for a, b in csv_number_spans(buf, columns, delims)]
        want = csv_module_tokens(text, columns, extra_space or crlf)
        assert got == want, (seed, hex(columns))


def test_all_columns_is_plain_splitting():
    rng = np.random.default_rng(9)
    buf = random_table(rng, 40).encode()
    spans = csv_number_spans(buf, (1 << 64) - 1, b",\n")
    # rows are short enough here that every column is below 64
    if max(len(line.split(b",")) for line in buf.split(b"\n")) <= 64:
        assert [buf[a:b] for a, b in spans] == split_tokens(buf, b",\n")


def test_special_cases():
    assert csv_number_spans(b"", 1) == []
    assert csv_number_spans(b"5", 1) == [(0, 1)]
    assert csv_number_spans(b"5", 2) == []
    # a token runs to the next delimiter; the row resets the column
    assert csv_number_spans(b"1,2\n3,4", 0b10) == [(2, 3), (6, 7)]
    # empty fields still count as columns
    assert csv_number_spans(b",,7,\n", 0b100) == [(2, 3)]
    # columns from 64 on are never selected
    row = b",".join(b"%d" % i for i in range(70)) + b"\n"
    assert [row[a:b] for a, b in csv_number_spans(row, (1 << 64) - 1)] == \
        [b"%d" % i for i in range(64)]
    bits, status = parse_csv(b"x,1.5\ny,-2e3\n", 0b10)
    assert (bits, status) == ([parse_token(b"1.5")[0], parse_token(b"-2e3")[0]], [0, 0])
