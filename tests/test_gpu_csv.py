"""FFP_CSV (tokens of selected columns of a CSV table) on the GPU against
the oracle's parse_csv, element by element: column masks, delimiter sets,
tile and block sizes, rows longer than the backward column scan's 4 KiB
window, CR LF rows, texts that start mid-granule and the JSON grammar."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gen import workloads as W
from oracle import parse_csv

pytestmark = pytest.mark.gpu

NP_DT = {"f64": np.uint64, "f32": np.uint32}
TORCH = {"f64": (torch.float64, torch.int64), "f32": (torch.float32, torch.int32)}


def _log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ffpmod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_11408_amd import ffp
    ffp.load()
    return ffp


def run_csv(ctx, buf, fmt, offset=0):
    dev = torch.device("cuda", 0)
    text = torch.frombuffer(bytearray(b"\n" * offset + buf), dtype=torch.uint8).to(dev)[offset:]
    cap = len(buf) // 2 + 1
    vdt, idt = TORCH[fmt]
    values = torch.empty(cap, dtype=vdt, device=dev)
    status = torch.full((cap,), 255, dtype=torch.uint8, device=dev)
    count = torch.full((1,), -1, dtype=torch.int64, device=dev)
    rc = ctx.parse_into(text, values, status, count, sync=True)
    n = int(count.item())
    bits = values.view(idt).cpu().numpy().view(NP_DT[fmt])
    return rc, n, bits, status.cpu().numpy()


def check(ctx, buf, columns, delims, flags, fmt, label, offset=0):
    _log("case csv", label, fmt, hex(columns), len(buf), "bytes, offset", offset)
    rc, n, bits, status = run_csv(ctx, buf, fmt, offset)
    wb, ws = parse_csv(buf, columns, fmt, delims, flags)
    assert rc == len(wb) and n == len(wb), (label, rc, n, len(wb))
    bad = np.flatnonzero((bits[:n] != np.array(wb, dtype=NP_DT[fmt])) |
                         (status[:n] != np.array(ws, dtype=np.uint8)))
    assert bad.size == 0, (label, fmt, hex(columns), bad[:5])


def make_ctx(ffpmod, delims, flags):
    return ffpmod.Context(0, delims=delims, flags=ffpmod.FFP_CSV | flags)


@pytest.mark.parametrize("tile_k,block_kib", [(0, 0), (1, 4), (2, 16), (4, 64)])
def test_csv_columns_match_oracle(ffpmod, tile_k, block_kib):
    rng = np.random.default_rng(500 + tile_k)
    buf = W.csv_table(rng, 3000).encode()                       # ~0.5 MB, many blocks
    c = make_ctx(ffpmod, b",\n", 0)
    try:
        if tile_k:
            c.set_tuning(tile_k, 0, block_kib)
        for columns in [1, 0b101, (1 << 64) - 1, 1 << 63, int(rng.integers(0, 1 << 62)), 0]:
            c.set_csv_columns(columns)
            for fmt in ("f64", "f32"):
                check(c, buf, columns, b",\n", 0, fmt, "table tile %d" % tile_k,
                      offset=int(rng.integers(0, 16)))
    finally:
        c.close()


@pytest.mark.parametrize("variant", ["spaces", "crlf", "long_rows", "no_newline", "json"])
def test_csv_variants(ffpmod, variant):
    rng = np.random.default_rng({"spaces": 510, "crlf": 511, "long_rows": 512,
                                 "no_newline": 513, "json": 514}[variant])
    delims, flags = b",\n", 0
    kw = {}
    if variant == "spaces":
        delims, kw = b",\n ", dict(extra_space=True)
    elif variant == "crlf":
        delims, kw = b",\n\r", dict(crlf=True)
    elif variant == "long_rows":
        kw = dict(long_field_every=2)      # rows of 3-9 KB: the column scan reads back past 4 KiB
    elif variant == "no_newline":
        kw = dict(trailing_newline=False)
    elif variant == "json":
        flags = ffpmod.FFP_JSON | ffpmod.FFP_INFNAN
    buf = W.csv_table(rng, 1500, **kw).encode()
    if variant == "json":
        buf += b"inf,-nan,01,1.,+1,-0\n"
    c = make_ctx(ffpmod, delims, flags)
    try:
        for tk in (0, 1, 4):
            if tk:
                c.set_tuning(tk, 0, {1: 4, 4: 64}[tk])
            for columns in [0b1011, (1 << 64) - 1]:
                c.set_csv_columns(columns)
                check(c, buf, columns, delims, flags, "f64", "%s tile %d" % (variant, tk))
    finally:
        c.close()


def test_csv_one_giant_row(ffpmod):
    """A single row of 40,000 fields (no '\\n' before the end): every block's
    column comes from a backward scan over the whole text before it, and only
    columns below 64 can be selected."""
    row = ",".join("%d.%d" % (i, i % 7) for i in range(40000)) + "\n"
    buf = (row + "1,2,3\n").encode()
    c = make_ctx(ffpmod, b",\n", 0)
    try:
        c.set_tuning(1, 0, 4)
        for columns in [1, (1 << 64) - 1, 1 << 63, 0b110]:
            c.set_csv_columns(columns)
            check(c, buf, columns, b",\n", 0, "f64", "giant row")
    finally:
        c.close()


def test_csv_context_rules(ffpmod):
    with pytest.raises(Exception):  # ',' and '\n' must be delimiters
        ffpmod.Context(0, delims=b"\n", flags=ffpmod.FFP_CSV)
    with pytest.raises(Exception):  # no hexadecimal tokens with FFP_CSV
        ffpmod.Context(0, delims=b",\n", flags=ffpmod.FFP_CSV | ffpmod.FFP_HEX)
