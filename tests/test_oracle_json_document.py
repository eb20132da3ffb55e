"""The oracle's JSON structural index (oracle.json_number_spans,
parse_json_document) pinned against Python's json module: on documents whose
strings and keys hold digits, commas, escaped quotes and backslash runs, the
number tokens found are exactly the number literals json.loads reads, in
document order; plus hand-written edge cases."""

import json

import pytest

from gen import workloads as W
from oracle import (FLAG_JSON, json_number_spans, parse_json_document, parse_token)


def _literals(doc: bytes):
    """Number literals of a JSON text, in document order, as json.loads reads
    them."""
    out = []
    marker = object()

    def collect(v):
        if isinstance(v, tuple) and v and v[0] is marker:
            out.append(v[1].encode())
        elif isinstance(v, list):
            for x in v:
                collect(x)
        elif isinstance(v, dict):
            for x in v.values():
                collect(x)

    collect(json.loads(doc.decode(), parse_float=lambda s: (marker, s),
                       parse_int=lambda s: (marker, s)))
    return out


@pytest.mark.parametrize("seed,indent,long_strings", [(1, None, False), (2, 2, False),
                                                      (3, None, True), (4, 1, True)])
def test_spans_equal_json_module(seed, indent, long_strings):
    doc = W.json_tricky_document(seed, 400, indent=indent, long_strings=long_strings)
    got = [doc[a:b] for a, b in json_number_spans(doc)]
    want = _literals(doc)
    assert len(want) > 100
    assert got == want


def test_edge_documents():
    cases = {
        b'{"a\\\\":1}': [b"1"],                       # key a\ ends at its quote
        b'["a\\"b", 2]': [b"2"],                      # escaped quote inside a string
        b'["\\\\\\"x", 3, "y"]': [b"3"],              # \\ then \" inside one string
        b'[1,"2",3]': [b"1", b"3"],                   # digits inside a string
        b'[true,false,null,-0.5e-3]': [b"-0.5e-3"],   # literals are not numbers
        b'{"k":[{"12":12,"3,4":-7}]}': [b"12", b"-7"],
        b'  42  ': [b"42"],
        b'"unterminated 5': [],
        b'': [],
    }
    for doc, want in cases.items():
        got = [doc[a:b] for a, b in json_number_spans(doc)]
        assert got == want, (doc, got)
        if want:
            assert _literals(doc) == want


def test_values_are_json_grammar_parses():
    doc = W.json_tricky_document(5, 300)
    bits, status = parse_json_document(doc, "f64")
    toks = [doc[a:b] for a, b in json_number_spans(doc)]
    assert len(bits) == len(toks) > 50
    for t, b, s in zip(toks, bits, status):
        assert (b, s) == parse_token(t, "f64", FLAG_JSON)
        if s == 0:
            assert json.loads(t) == json.loads(t)  # a valid JSON number
