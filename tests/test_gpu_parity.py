"""Parity of the HIP path with the CPU oracle, bit for bit, on values, status
codes and the token count.  Every call goes through the C-ABI (libffp.so)."""

import math
import os

import numpy as np
import pytest

from gen import workloads as W
from oracle import parse_buffer, parse_token, split_tokens

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ffpmod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_11408_amd import ffp
    ffp.load()
    return ffp


@pytest.fixture(scope="module")
def ctx(ffpmod):
    c = ffpmod.Context(0)
    yield c
    c.close()


TORCH_DT = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16,
            "bf16": torch.bfloat16}
INT_DT = {"f64": torch.int64, "f32": torch.int32, "f16": torch.int16, "bf16": torch.int16}
NP_DT = {"f64": np.uint64, "f32": np.uint32, "f16": np.uint16, "bf16": np.uint16}


def run_gpu(ctx, buf: bytes, fmt: str, capacity=None, offset=0):
    """Parses buf on the GPU; with offset > 0 the device text starts that many
    bytes past an allocation boundary."""
    dev = torch.device("cuda", 0)
    text = torch.frombuffer(bytearray(b"\n" * offset + buf), dtype=torch.uint8).to(dev)[offset:] \
        if buf else torch.empty(0, dtype=torch.uint8, device=dev)
    dt = TORCH_DT[fmt]
    if capacity is None:
        capacity = len(buf) // 2 + 1
    values = torch.empty(max(capacity, 1), dtype=dt, device=dev)
    status = torch.full((max(capacity, 1),), 255, dtype=torch.uint8, device=dev)
    count = torch.full((1,), -1, dtype=torch.int64, device=dev)
    rc = ctx.parse_into(text, values, status, count, sync=True) if len(buf) else \
        ctx.parse_into(text, values, status, count, nbytes=0, sync=True)
    n = int(count.item())
    bits = values.view(INT_DT[fmt]).cpu().numpy().view(NP_DT[fmt])
    return rc, n, bits, status.cpu().numpy()


def compare_full(ctx, buf: bytes, fmt: str, label: str):
    _log("case", label, fmt, len(buf), "bytes")
    rc, n, bits, status = run_gpu(ctx, buf, fmt)
    want_bits, want_st = parse_buffer(buf, fmt)
    assert rc == len(want_bits), (label, rc)
    assert n == len(want_bits)
    wb = np.array(want_bits, dtype=NP_DT[fmt])
    ws = np.array(want_st, dtype=np.uint8)
    bad = np.flatnonzero((bits[:n] != wb) | (status[:n] != ws))
    if bad.size:
        toks = split_tokens(buf)
        msgs = []
        for i in bad[:10].tolist():
            s, e = toks[i]
            msgs.append("%d %r gpu=%x/%d oracle=%x/%d" % (i, buf[s:e][:80], int(bits[i]),
                                                           int(status[i]), int(wb[i]), int(ws[i])))
        raise AssertionError("%s %s: %d mismatches\n%s" % (label, fmt, bad.size, "\n".join(msgs)))
    return n


def compare_sampled(ctx, buf: bytes, fmt: str, label: str, nsample: int, seed: int):
    _log("case", label, fmt, len(buf), "bytes (sampled)")
    rc, n, bits, status = run_gpu(ctx, buf, fmt)
    toks = split_tokens(buf)
    assert rc == len(toks) and n == len(toks), (rc, n, len(toks))
    rng = np.random.default_rng(seed)
    idx = np.unique(np.concatenate([rng.integers(0, n, nsample), [0, n - 1]]))
    for i in idx.tolist():
        s, e = toks[i]
        b, st = parse_token(buf[s:e], fmt)
        assert int(bits[i]) == b and int(status[i]) == st, (label, i, buf[s:e][:80])
    # every status is a public code: nothing left pending
    assert status[:n].max() <= 2
    return n


# ---------------------------------------------------------------------------
# configs at sizes the oracle finishes in seconds
# ---------------------------------------------------------------------------

def test_config1_full(ctx):
    buf = W.config1()
    assert compare_full(ctx, buf, "f64", "config1") == 100_000
    assert compare_full(ctx, buf, "f32", "config1") == 100_000


def test_config2_mix_300k(ctx):
    buf = W.config2(seed=22, n=300_000)
    assert compare_full(ctx, buf, "f64", "config2-300k") == 300_000
    compare_full(ctx, buf, "f32", "config2-300k")


def test_config3_hard_40k(ctx):
    buf = W.config3(seed=33, n=40_000)
    compare_full(ctx, buf, "f64", "config3-40k")
    compare_full(ctx, buf, "f32", "config3-40k")


def test_ragged_random_layout(ctx):
    """Tokens of random lengths separated by runs of 1-3 delimiters, so that
    tokens start, end and straddle at every offset of the tiles."""
    rng = np.random.default_rng(11)
    toks = W.mixed_tokens(rng, 60_000) + W.hard_tokens(rng, 3000)
    rng.shuffle(toks)
    seps = rng.integers(1, 4, size=len(toks))
    buf = b"".join(t.encode() + b"\n" * int(k) for t, k in zip(toks, seps))
    for cut in (0, 1, 7):  # also without trailing delimiters
        b = buf[: len(buf) - cut] if cut else buf
        compare_full(ctx, b.rstrip(b"\n") if cut == 7 else b, "f64", "ragged-%d" % cut)


@pytest.mark.parametrize("tile_k", [1, 2, 4])
def test_tile_sizes(ffpmod, tile_k):
    os.environ["FFP_TILE_K"] = str(tile_k)
    try:
        c = ffpmod.Context(0)
    finally:
        del os.environ["FFP_TILE_K"]
    try:
        rng = np.random.default_rng(100 + tile_k)
        toks = W.mixed_tokens(rng, 20_000) + W.hard_tokens(rng, 500)
        rng.shuffle(toks)
        buf = W.join_tokens(toks)
        compare_full(c, buf, "f64", "tile-k%d" % tile_k)
        compare_full(c, buf, "f32", "tile-k%d" % tile_k)
    finally:
        c.close()


@pytest.fixture(scope="module")
def ragged_blocks_case():
    """About 1.4 MB of mixed and hard tokens behind runs of 1-3 delimiters,
    starting 3 bytes into the buffer, with the oracle's answer."""
    rng = np.random.default_rng(12)
    toks = W.mixed_tokens(rng, 50_000) + W.hard_tokens(rng, 1500)
    rng.shuffle(toks)
    seps = rng.integers(1, 4, size=len(toks))
    buf = b"7\n\n" + b"".join(t.encode() + b"\n" * int(k) for t, k in zip(toks, seps))
    buf = buf[3:]
    return buf, {fmt: parse_buffer(buf, fmt) for fmt in ("f64", "f32")}


@pytest.mark.parametrize("block_kib,tile_k", [(4, 1), (16, 1), (16, 2), (16, 4), (64, 1),
                                              (64, 2), (64, 4)])
def test_block_sizes(ffpmod, ragged_blocks_case, block_kib, tile_k):
    """Every block size with every tile size that fits it, forced through the
    tuning call; parse and batched calls."""
    buf, want = ragged_blocks_case
    c = ffpmod.Context(0)
    try:
        c.set_tuning(tile_k, 0, block_kib)
        for fmt in ("f64", "f32"):
            _log("case blocks", block_kib, "tile_k", tile_k, fmt)
            rc, n, bits, status = run_gpu(c, buf, fmt, offset=5)
            wb, ws = want[fmt]
            assert rc == len(wb) and n == len(wb)
            assert np.array_equal(bits[:n], np.array(wb, dtype=NP_DT[fmt])), (block_kib, tile_k,
                                                                              fmt)
            assert np.array_equal(status[:n], np.array(ws, dtype=np.uint8))
        # the same text as three jobs of one batched call (cut inside tokens)
        dev = torch.frombuffer(bytearray(buf), dtype=torch.uint8).to("cuda:0")
        cuts = [0, len(buf) // 3, 2 * len(buf) // 3 + 7, len(buf)]
        texts = [dev[a:b] for a, b in zip(cuts, cuts[1:])]
        fmts = ["f64", "f32", "f64"]
        vals = [torch.empty(t.numel() // 2 + 1, dtype=TORCH_DT[f], device="cuda:0")
                for t, f in zip(texts, fmts)]
        sts = [torch.full((t.numel() // 2 + 1,), 255, dtype=torch.uint8, device="cuda:0")
               for t in texts]
        table = ffpmod.JobTable(texts, vals, sts, "cuda:0")
        c.parse_batch(table.dev, table.n, len(buf))
        torch.cuda.synchronize()
        for j, ((count, err), (a, b), f) in enumerate(zip(table.download(), zip(cuts, cuts[1:]),
                                                          fmts)):
            wb, ws = parse_buffer(buf[a:b], f)
            assert err == 0 and count == len(wb), (block_kib, tile_k, j, count, err)
            got = vals[j][:count].view(INT_DT[f]).cpu().numpy().view(NP_DT[f])
            assert np.array_equal(got, np.array(wb, dtype=NP_DT[f])), (block_kib, tile_k, j)
            assert np.array_equal(sts[j][:count].cpu().numpy(), np.array(ws, dtype=np.uint8))
    finally:
        c.close()


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------

def test_empty_and_tiny_buffers(ctx):
    for buf in [b"", b"\n", b"\n\n\n", b"1", b"7\n", b"\n5", b"-", b".", b"0"]:
        for fmt in ("f64", "f32"):
            rc, n, bits, status = run_gpu(ctx, buf, fmt, capacity=4)
            want_bits, want_st = parse_buffer(buf, fmt)
            assert n == len(want_bits) and rc == n, buf
            assert list(map(int, bits[:n])) == want_bits, buf
            assert list(map(int, status[:n])) == want_st, buf


def test_grammar_edge_tokens(ctx):
    toks = W.INVALID_EXAMPLES[1:] + [
        "1", "-1", "+1", "-0", "0", ".5", "5.", "1.e1", "1e+1", "1E-1", "1e0001",
        "0e999999999999", "-0.0e-999", "1e309", "1e-400", "4.9e-324",
        "2.4703282292062327e-324", "2.4703282292062328e-324", "18446744073709551615",
        "18446744073709551616", "9007199254740993", "9000000000000000.5",
        "1e+100000000000000000000", "1e-100000000000000000000",
        "00000000000000000000000000000000000000001", "0." + "0" * 500 + "1e500",
        "1" * 40 + "e-40", "9" * 19, "9" * 20, "1" + "0" * 19, "1" + "0" * 30 + "1",
    ]
    toks = [t.replace(" ", "").replace("\n", "") or "x" for t in toks if "\n" not in t]
    buf = W.join_tokens(toks)
    compare_full(ctx, buf, "f64", "grammar")
    compare_full(ctx, buf, "f32", "grammar")


def test_capacity_smaller_than_count(ctx, ffpmod):
    buf = W.config1(seed=5, n=5000)
    rc, n, bits, status = run_gpu(ctx, buf, "f64", capacity=1234)
    assert rc == ffpmod.FFP_E_CAPACITY
    assert n == 5000
    wb, ws = parse_buffer(buf, "f64")
    assert list(map(int, bits[:1234])) == wb[:1234]
    assert list(map(int, status[:1234])) == ws[:1234]


def test_many_tiny_tokens(ctx):
    # the densest layout: one digit per token, half the bytes are delimiters
    buf = b"7\n" * 300_000 + b"8"
    compare_full(ctx, buf, "f64", "dense")


@pytest.mark.parametrize("tile_k,block_kib", [(1, 64), (2, 64), (1, 16), (2, 16)])
def test_dense_blocks_with_small_tiles(ffpmod, tile_k, block_kib):
    """Dense text (one-digit tokens, 8192 starts per 16 KiB) with a fixed
    schedule of 4 or 8 KiB tiles in 16 and 64 KiB blocks: calls of at most
    1024 blocks run without the scan kernel and read the count kernel's
    block counts as they are (no dense-tile flag in them), larger ones
    through the scan; plain and batched calls against the oracle."""
    rng = np.random.default_rng(180 + tile_k + block_kib)
    dense = b"7\n" * 150_000 + b"8"
    sparse = W.join_tokens(W.mixed_tokens(rng, 20_000))
    mixed = sparse[:300_000] + b"\n" + b"1\n" * 40_000 + sparse[300_000:]
    c = ffpmod.Context(0)
    try:
        c.set_tuning(tile_k, 0, block_kib)
        for label, buf in (("dense", dense), ("mixed", mixed)):
            _log("case dense blocks small tiles", tile_k, block_kib, label)
            rc, n, bits, status = run_gpu(c, buf, "f64", offset=5)
            wb, ws = parse_buffer(buf, "f64")
            assert rc == n == len(wb), (label, rc, n, len(wb))
            assert np.array_equal(bits[:n], np.array(wb, dtype=NP_DT["f64"])), label
            assert np.array_equal(status[:n], np.array(ws, dtype=np.uint8)), label
        dev = torch.device("cuda", 0)
        texts = [torch.frombuffer(bytearray(b), dtype=torch.uint8).to(dev)
                 for b in (dense, mixed, sparse[:5000])]
        want = [parse_buffer(b, "f64") for b in (dense, mixed, sparse[:5000])]
        vals = [torch.empty(len(w[0]) + 1, dtype=torch.float64, device=dev) for w in want]
        sts = [torch.empty(len(w[0]) + 1, dtype=torch.uint8, device=dev) for w in want]
        table = ffpmod.JobTable(texts, vals, sts, dev)
        c.parse_batch(table.dev, table.n, sum(t.numel() for t in texts))
        res = table.download()
        for i, (wb, ws) in enumerate(want):
            assert res[i] == (len(wb), 0), (i, res[i])
            got = vals[i].view(torch.int64).cpu().numpy().view(np.uint64)[:len(wb)]
            assert np.array_equal(got, np.array(wb, dtype=np.uint64)), i
    finally:
        c.close()


@pytest.mark.parametrize("block_kib", [16, 64])
def test_dense_tiles_at_16k(ffpmod, block_kib):
    """16 KiB tiles: the plain instance keeps at most 4096 starts per tile and
    runs when no tile of the call has more (16 KiB blocks: their counts; 64
    KiB blocks: a per-tile flag of the count kernel); otherwise its
    full-list twin runs.  Dense text (one-digit tokens: 8192 per tile),
    sparse text, a text dense in one block only, tiles with exactly 4097 and
    4096 starts at each tile position of a block, short tokens (dense per
    block, not per tile), in plain calls and in one batched call mixing
    them; every output against the oracle."""
    rng = np.random.default_rng(170 + block_kib)
    dense = b"7\n" * 150_000 + b"8"
    sparse = W.join_tokens(W.mixed_tokens(rng, 20_000))
    mixed = sparse[:300_000] + b"\n" + b"1\n" * 40_000 + sparse[300_000:]
    c = ffpmod.Context(0)
    try:
        c.set_tuning(4, 0, block_kib)
        for label, buf in (("dense", dense), ("sparse", sparse), ("mixed", mixed)):
            for fmt in ("f64", "f32"):
                _log("case dense tiles", block_kib, label, fmt)
                rc, n, bits, status = run_gpu(c, buf, fmt, offset=9)
                wb, ws = parse_buffer(buf, fmt)
                assert rc == n == len(wb), (label, rc, n, len(wb))
                bad = np.flatnonzero((bits[:n] != np.array(wb, dtype=NP_DT[fmt])) |
                                     (status[:n] != np.array(ws, dtype=np.uint8)))
                assert bad.size == 0, (label, fmt, bad[:5])
        # tiles at the limit: a text placed 9 bytes past a 16-byte boundary
        # has its 16 KiB tiles at text offsets 16384 t - 9; one tile with
        # exactly 4097 (dense) or 4096 (not) starts at each of a 64 KiB
        # block's four tile positions, the rest sparse
        filler = W.join_tokens(W.mixed_tokens(rng, 8000))
        for t in (1, 2, 3, 4):
            at = 16384 * t - 9
            head = filler[:at]
            head = head[: head.rfind(b"\n") + 1]
            head += b"\n" * (at - len(head))
            for k, rest in ((4097, b""), (4096, b"\n" * (16384 - 8192))):
                buf = head + b"1\n" * k + rest + filler[at:at + 40000]
                buf = buf[: buf.rfind(b"\n") + 1]
                _log("case dense tile limit", block_kib, t, k)
                rc, n, bits, status = run_gpu(c, buf, "f64", offset=9)
                wb, ws = parse_buffer(buf, "f64")
                assert rc == n == len(wb), (t, k, rc, n, len(wb))
                bad = np.flatnonzero((bits[:n] != np.array(wb, dtype=NP_DT["f64"])) |
                                     (status[:n] != np.array(ws, dtype=np.uint8)))
                assert bad.size == 0, (t, k, bad[:5])
        # short tokens: more than 4096 starts per 64 KiB block, at most 4096
        # per 16 KiB tile (the per-tile flag keeps the short start list)
        short = W.join_tokens(["%d.%d" % (int(a), int(b)) for a, b in
                               zip(rng.integers(0, 10, 60000), rng.integers(0, 100, 60000))])
        _log("case dense tiles short tokens", block_kib)
        rc, n, bits, status = run_gpu(c, short, "f64", offset=9)
        wb, ws = parse_buffer(short, "f64")
        assert rc == n == len(wb)
        assert np.array_equal(bits[:n], np.array(wb, dtype=NP_DT["f64"]))
        assert np.array_equal(status[:n], np.array(ws, dtype=np.uint8))
        # one batched call: the flag covers the whole call
        dev = torch.device("cuda", 0)
        texts = [torch.frombuffer(bytearray(b), dtype=torch.uint8).to(dev)
                 for b in (sparse, dense, mixed, sparse[:5000])]
        want = [parse_buffer(b, "f64") for b in (sparse, dense, mixed, sparse[:5000])]
        vals = [torch.empty(len(w[0]) + 1, dtype=torch.float64, device=dev) for w in want]
        sts = [torch.empty(len(w[0]) + 1, dtype=torch.uint8, device=dev) for w in want]
        table = ffpmod.JobTable(texts, vals, sts, dev)
        c.parse_batch(table.dev, table.n, sum(t.numel() for t in texts))
        res = table.download()
        for i, (wb, ws) in enumerate(want):
            assert res[i] == (len(wb), 0), (i, res[i])
            got = vals[i].view(torch.int64).cpu().numpy().view(np.uint64)[:len(wb)]
            assert np.array_equal(got, np.array(wb, dtype=np.uint64)), i
            assert np.array_equal(sts[i].cpu().numpy()[:len(wb)], np.array(ws, dtype=np.uint8)), i
    finally:
        c.close()


def test_long_tokens(ctx):
    rng = np.random.default_rng(12)
    long_digits = "".join(map(str, rng.integers(0, 10, 100_000).tolist()))
    toks = ["1" + long_digits, "0." + long_digits, long_digits[:5000] + "e-5200",
            "0" * 70_000 + "3.25", "1" + "0" * 50_000 + "e-50000"]
    buf = W.join_tokens(toks)
    compare_full(ctx, buf, "f64", "long")
    compare_full(ctx, buf, "f32", "long")


@pytest.fixture(scope="module")
def straddle_case():
    """Tokens that start just before a 4 KiB boundary and run past it by
    1..2000 bytes (around the 16-byte chunk, the 32-byte bitmap window and the
    1 KiB of text the parse kernel keeps after each tile), short filler in
    between, and a last token that reaches the end of the text."""
    rng = np.random.default_rng(67)
    overhangs = [1, 2, 15, 16, 17, 31, 32, 33, 100, 1007, 1008, 1023, 1024, 1025, 1040, 2000]
    digits = "".join(map(str, rng.integers(0, 10, 4000).tolist()))
    out, toks = bytearray(), []
    for i in range(48):
        # the next 4 KiB boundary at least 200 bytes ahead (sometimes one more)
        boundary = ((len(out) + 200) // 4096 + 1 + (i % 3 == 2)) * 4096
        while len(out) < boundary - 40:  # filler up to just before the boundary
            tok = W.mixed_tokens(rng, 1)[0]
            if len(out) + len(tok) + 1 > boundary - 40:
                tok = "7" * max(1, boundary - 41 - len(out))
            out += tok.encode() + b"\n"
            toks.append(tok)
        start = boundary - int(rng.integers(1, 40))
        while len(out) < start:
            out += b"\n"
        start = len(out)
        over = overhangs[i % len(overhangs)]
        n = boundary + over - start
        kind = i % 4
        if kind == 0:
            tok = "1" + digits[: max(0, n - 1)]
        elif kind == 1:
            tok = ("0." + digits)[:n]
        elif kind == 2:
            tok = (digits[: max(1, n - 5)] + "e-" + "123")[:n] if n > 6 else "5" * n
        else:
            tok = ("-" + "0" * (n - 3) + "25")[:n] if n > 3 else "9" * n
        out += tok.encode() + b"\n"
        toks.append(tok)
    tail = "3." + digits[:1500]  # ends exactly at the end of the text (no delimiter)
    out += tail.encode()
    toks.append(tail)
    buf = bytes(out)
    return toks, buf, {fmt: parse_buffer(buf, fmt) for fmt in ("f64", "f32")}


@pytest.mark.parametrize("tile_k,block_kib", [(4, 16), (4, 64), (2, 16), (1, 16), (1, 4)])
def test_tokens_across_tile_ends(ffpmod, straddle_case, tile_k, block_kib):
    """A token running past its tile is lexed from the text kept after the
    tile (the next tile's chunks inside a block, loaded ones at a block's
    end) or, beyond that, from global memory; all must match the oracle."""
    toks, buf, want = straddle_case
    c = ffpmod.Context(0)
    try:
        c.set_tuning(tile_k, 0, block_kib)
        for fmt in ("f64", "f32"):
            _log("case straddle", tile_k, block_kib, fmt, len(buf))
            rc, n, bits, status = run_gpu(c, buf, fmt)
            wb, ws = want[fmt]
            assert rc == len(wb) and n == len(wb)
            bad = np.flatnonzero((bits[:n] != np.array(wb, dtype=NP_DT[fmt])) |
                                 (status[:n] != np.array(ws, dtype=np.uint8)))
            assert bad.size == 0, (tile_k, block_kib, fmt, [toks[i][:60] for i in bad[:3]])
    finally:
        c.close()


def _long_grammar_tokens(seed, n=3000):
    """Tokens of 20-600 characters: digit strings with a dot anywhere (or
    none), leading and trailing zeros, signs, exponents with leading zeros or
    more than 17 significant digits, all-zero mantissas, and broken forms."""
    rng = np.random.default_rng(seed)
    toks = []
    for _ in range(n):
        nd = int(rng.integers(20, 500))
        d = "".join(map(str, rng.integers(0, 10, nd).tolist()))
        k = int(rng.integers(0, 8))
        if k == 1:
            d = "0" * int(rng.integers(1, 300)) + d
        elif k == 2:
            d = d + "0" * int(rng.integers(1, 300))
        elif k == 3:
            d = "0" * nd
        dot = int(rng.integers(-1, len(d) + 1))
        m = d if dot < 0 else d[:dot] + "." + d[dot:]
        sign = ["", "-", "+"][int(rng.integers(0, 3))]
        ek = int(rng.integers(0, 6))
        if ek == 0:
            ex = ""
        elif ek == 1:
            ex = "e%+d" % int(rng.integers(-400, 400))
        elif ek == 2:
            ex = "E" + "0" * int(rng.integers(1, 40)) + str(int(rng.integers(0, 400)))
        elif ek == 3:
            ex = "e-" + "".join(map(str, rng.integers(0, 10, int(rng.integers(17, 30))).tolist()))
        elif ek == 4:
            ex = "e" + str(int(rng.integers(0, 10))) * int(rng.integers(15, 19))
        else:
            ex = ["e", "e+", "e-", "ee5", "e5.", "x"][int(rng.integers(0, 6))]
        tok = sign + m + ex
        if rng.integers(0, 20) == 0:  # a stray byte somewhere
            i = int(rng.integers(0, len(tok)))
            tok = tok[:i] + "ab.-+"[int(rng.integers(0, 5))] + tok[i:]
        toks.append(tok)
    return toks


@pytest.mark.parametrize("flags", [0, 1])
def test_long_token_grammar(ffpmod, flags):
    """The long-token lexer against the oracle on long valid and invalid
    tokens, with and without FFP_REJECT_PLUS, mixed with short tokens."""
    rng = np.random.default_rng(68 + flags)
    toks = _long_grammar_tokens(69 + flags) + W.mixed_tokens(rng, 5000)
    rng.shuffle(toks)
    buf = W.join_tokens(toks)
    c = ffpmod.Context(0, flags=flags)
    try:
        for fmt in ("f64", "f32"):
            _log("case long grammar", flags, fmt, len(buf))
            rc, n, bits, status = run_gpu(c, buf, fmt, offset=7)
            wb, ws = parse_buffer(buf, fmt, flags=flags)
            assert rc == len(wb) and n == len(wb)
            bad = np.flatnonzero((bits[:n] != np.array(wb, dtype=NP_DT[fmt])) |
                                 (status[:n] != np.array(ws, dtype=np.uint8)))
            assert bad.size == 0, (flags, fmt, [toks[i][:80] for i in bad[:3]])
    finally:
        c.close()


def _leading_zero_fraction_tokens(seed, n=6000):
    """Short tokens (under 32 bytes) whose fraction starts with zeros and
    whose digit count exceeds 19 while the significant digits may not: an
    integer part that is empty, '0', '-0', '+0' or '00', 0-12 leading zeros,
    then 1-20 digits, with or without an exponent."""
    rng = np.random.default_rng(seed)
    toks = []
    while len(toks) < n:
        ip = ["", "0", "-0", "+0", "00", "-", "1"][int(rng.integers(0, 7))]
        z = int(rng.integers(0, 13))
        d = "".join(map(str, rng.integers(0, 10, int(rng.integers(1, 21))).tolist()))
        ex = ["", "e%d" % int(rng.integers(-30, 30)), "E+5", "e-300"][int(rng.integers(0, 4))]
        tok = ip + "." + "0" * z + d + ex
        if len(tok) < 32 and (ip not in ("", "-") or rng.integers(0, 4) == 0):
            toks.append(tok)
    return toks


@pytest.mark.parametrize("flags", [0, 2])
def test_leading_zero_fractions(ffpmod, flags):
    """Fractions with leading zeros beyond 19 digits stay on the bitmap
    lexer when their significant digits fit; parity with the oracle either
    way, with and without FFP_JSON."""
    rng = np.random.default_rng(90 + flags)
    toks = _leading_zero_fraction_tokens(91 + flags) + W.mixed_tokens(rng, 4000)
    rng.shuffle(toks)
    buf = W.join_tokens(toks)
    c = ffpmod.Context(0, flags=flags)
    try:
        for fmt in ("f64", "f32", "f16"):
            _log("case leading zeros", flags, fmt, len(buf))
            rc, n, bits, status = run_gpu(c, buf, fmt, offset=3)
            wb, ws = parse_buffer(buf, fmt, flags=flags)
            assert rc == len(wb) and n == len(wb)
            bad = np.flatnonzero((bits[:n] != np.array(wb, dtype=NP_DT[fmt])) |
                                 (status[:n] != np.array(ws, dtype=np.uint8)))
            assert bad.size == 0, (flags, fmt, [toks[i] for i in bad[:3]])
    finally:
        c.close()


def test_delimiter_set_and_flags(ffpmod):
    c = ffpmod.Context(0, delims=b",; \t\r\n", flags=ffpmod.FFP_REJECT_PLUS)
    try:
        rng = np.random.default_rng(13)
        toks = W.mixed_tokens(rng, 20_000)
        seps = [b",", b";", b" ", b"\t", b"\r\n", b", "]
        parts = []
        for i, t in enumerate(toks):
            parts.append(("+" + t if i % 97 == 0 else t).encode())
            parts.append(seps[int(rng.integers(0, len(seps)))])
        buf = b"".join(parts)
        rc, n, bits, status = run_gpu(c, buf, "f64")
        wb, ws = parse_buffer(buf, "f64", delims=b",; \t\r\n", flags=1)
        assert rc == n == len(wb)
        assert np.array_equal(bits[:n], np.array(wb, dtype=np.uint64))
        assert np.array_equal(status[:n], np.array(ws, dtype=np.uint8))
        assert (status[:n] == 1).sum() >= 20000 // 97
    finally:
        c.close()


@pytest.mark.parametrize("delims", [b",\n", b"\x00\x7f", b" \t\n", b",;\r\n", b"\n\x80",
                                    b",; \t\r\n"])
def test_small_delimiter_sets(ffpmod, delims):
    """Sets of 2 to 4 bytes below 0x80 are classified by byte comparisons,
    other sets (a member at or above 0x80, more members) by the table:
    parity either way, with the neighbours of each member (0x7f next to
    0x80, NUL) inside tokens, every tile size and a ragged start."""
    rng = np.random.default_rng(150 + len(delims) + delims[0])
    toks = [t.encode() for t in W.mixed_tokens(rng, 12_000)]
    near = bytes(sorted({(d + k) & 0xFF for d in delims for k in (-1, 1)} - set(delims)))
    parts = []
    for i, t in enumerate(toks):
        if i % 53 == 0 and near:  # a token holding a byte next to a delimiter: invalid
            t = t[:2] + near[i % len(near):i % len(near) + 1] + t[2:]
        parts.append(t)
        parts.append(delims[i % len(delims):i % len(delims) + 1] *
                     int(rng.integers(1, 3)))
    buf = b"".join(parts)
    wb, ws = parse_buffer(buf, "f64", delims=delims)
    c = ffpmod.Context(0, delims=delims)
    try:
        for tk, kib in ((0, 0), (1, 4), (4, 16)):
            if tk:
                c.set_tuning(tk, 0, kib)
            _log("case small delimiter set", delims, tk)
            rc, n, bits, status = run_gpu(c, buf, "f64", offset=7)
            assert rc == n == len(wb)
            bad = np.flatnonzero((bits[:n] != np.array(wb, dtype=np.uint64)) |
                                 (status[:n] != np.array(ws, dtype=np.uint8)))
            assert bad.size == 0, (delims, tk, bad[:5])
    finally:
        c.close()


def test_grammar_bytes_rejected_as_delimiters(ffpmod):
    """A delimiter may not be a byte that a token of the selected grammar can
    contain: hexadecimal letters, x and p under FFP_HEX, the letters of inf,
    infinity and nan under FFP_INFNAN."""
    bad = [(b"p", ffpmod.FFP_HEX), (b"x", ffpmod.FFP_HEX), (b"\nA", ffpmod.FFP_HEX),
           (b"n", ffpmod.FFP_INFNAN), (b"Y", ffpmod.FFP_INFNAN), (b"\na", ffpmod.FFP_INFNAN),
           (b"e", 0), (b"-", 0)]
    for delims, flags in bad:
        with pytest.raises(ffpmod.FFPError) as e:
            ffpmod.Context(0, delims=delims, flags=flags)
        assert e.value.code == ffpmod.FFP_E_ARG, (delims, flags)
    for delims, flags in [(b"p", 0), (b"n", ffpmod.FFP_HEX), (b"x", ffpmod.FFP_INFNAN),
                          (b"g", ffpmod.FFP_HEX | ffpmod.FFP_INFNAN)]:
        c = ffpmod.Context(0, delims=delims, flags=flags)
        try:
            buf = delims[:1].join([b"1.5", b"-2", b"7e3"])
            rc, n, bits, status = run_gpu(c, buf, "f64")
            wb, ws = parse_buffer(buf, "f64", delims=delims, flags=flags)
            assert n == len(wb) == 3 and list(map(int, bits[:n])) == wb, (delims, flags)
        finally:
            c.close()


def test_half_format_short_ties(ctx, ffpmod):
    """More than 200k exact binary16 / bfloat16 midpoints of few digits in one
    call: decided in-line (no fallback), rounded to even like the oracle."""
    rng = np.random.default_rng(57)
    for fmt, mant, emin in (("f16", 10, -14), ("bf16", 7, -126)):
        toks = [str(v) for v in range(2 ** (mant + 1) + 1, 2 ** (mant + 2), 2)]
        # between subnormals: (2k + 1) * 2^(emin - mant - 1)
        sub = 5 ** (mant + 1 - emin)
        toks += ["%de%d" % ((2 * k + 1) * sub, emin - mant - 1) for k in range(40)
                 if (2 * k + 1) * sub < 10 ** 19]
        while len(toks) < 220_000:
            num = 2 * int(rng.integers(2 ** mant, 2 ** (mant + 1))) + 1
            e = int(rng.integers(max(emin - mant, -24), 12)) - 1
            if e >= 0:
                toks.append(str(num << e))
            elif num * 5 ** -e < 10 ** 19:
                toks.append("%de%d" % (num * 5 ** -e, e))
        buf = W.join_tokens(toks)
        ctx.counters(True)
        ctx.counters_read()
        n = compare_full(ctx, buf, fmt, "short-ties")
        cnt = ctx.counters_read()
        ctx.counters(False)
        assert n == len(toks) and cnt["fallback"] == 0, (fmt, cnt)


def test_path_counters(ctx, ffpmod):
    buf = W.config3(seed=34, n=5000)
    ctx.counters(True)
    ctx.counters_read()
    run_gpu(ctx, buf, "f64")
    cnt = ctx.counters_read()
    ctx.counters(False)
    assert cnt["tokens"] == 5000
    assert cnt["invalid"] + cnt["early"] + cnt["one"] + cnt["two"] + cnt["fallback"] == 5000
    assert cnt["fallback"] > 0


# ---------------------------------------------------------------------------
# full sizes, sampled against the oracle
# ---------------------------------------------------------------------------

def test_config2_full_size_sampled(ctx):
    buf = W.config2()
    assert compare_sampled(ctx, buf, "f64", "config2-full", 100_000, 21) == 10_000_000


def test_config3_full_size_sampled(ctx):
    buf = W.config3()
    compare_sampled(ctx, buf, "f64", "config3-full", 20_000, 31)
    compare_sampled(ctx, buf, "f32", "config3-full", 20_000, 32)


# ---------------------------------------------------------------------------
# binary16 and bfloat16 results
# ---------------------------------------------------------------------------

def test_half_formats_mixed_and_hard(ctx):
    rng = np.random.default_rng(61)
    toks = W.mixed_tokens(rng, 40_000) + W.hard_tokens(rng, 2000)
    toks += [str(int(v)) for v in rng.integers(0, 70_000, 10_000)]
    toks += ["%.*f" % (int(k), float(x)) for k, x in zip(rng.integers(0, 8, 10_000),
                                                         rng.random(10_000) * 1000)]
    rng.shuffle(toks)
    buf = W.join_tokens(toks)
    for fmt in ("f16", "bf16"):
        compare_full(ctx, buf, fmt, "half-mixed")


def _dyadic_decimal(num: int, den_log2: int) -> str:
    """num / 2^den_log2 written exactly: (num * 5^k)e-k."""
    return "%de-%d" % (num * 5 ** den_log2, den_log2) if den_log2 > 0 else str(num << -den_log2)


def _value_and_midpoint_tokens(p, emin, emax, stride):
    """Every stride-th finite non-negative value of a format as an exact
    decimal, the exact midpoints of neighbours and the midpoints nudged by a
    digit far below them, both signs."""
    q0 = emin - p + 1
    vals = [(m, -q0) for m in range(0, 1 << (p - 1))]  # subnormals and zero: m * 2^q0
    for e in range(emin, emax + 1):
        vals += [(m, -(e - p + 1)) for m in range(1 << (p - 1), 1 << p)]
    vals.append((1, -(emax + 1)))  # 2^(emax+1): the midpoint above the largest is needed
    toks = []
    for i in range(0, len(vals) - 1, stride):
        (ma, ka), (mb, kb) = vals[i], vals[i + 1]
        k = max(ka, kb) + 1  # both neighbours as integers over 2^k
        a = ma * 2 ** (k - ka)
        b = mb * 2 ** (k - kb)
        mid = a + b  # midpoint = (a + b) / 2^(k+1)
        toks.append(_dyadic_decimal(a, k))
        m_str = _dyadic_decimal(mid, k + 1)
        toks.append(m_str)
        if "e" in m_str:
            d, e = m_str.split("e")
            toks.append("%s1e%d" % (d, int(e) - 1))      # nudged up
            toks.append("%se%d" % (str(int(d) * 10 - 1), int(e) - 1))  # nudged down
    return toks + ["-" + t for t in toks[::7]]


def test_binary16_every_value_and_midpoint(ctx):
    toks = _value_and_midpoint_tokens(11, -14, 15, 1)
    # shortest round-trip digits of every finite binary16 value
    allh = np.arange(0, 0x7C00, dtype=np.uint16).view(np.float16)
    toks += [repr(float(x)) for x in allh[::3]]
    buf = W.join_tokens(toks)
    _log("binary16 tokens", len(toks))
    compare_full(ctx, buf, "f16", "binary16-exhaustive")


def test_bfloat16_values_and_midpoints(ctx):
    toks = _value_and_midpoint_tokens(8, -126, 127, 5)
    buf = W.join_tokens(toks)
    _log("bfloat16 tokens", len(toks))
    compare_full(ctx, buf, "bf16", "bfloat16-sampled")


# ---------------------------------------------------------------------------
# JSON grammar, inf/nan, JSON documents
# ---------------------------------------------------------------------------

def _flag_tokens(seed, n=8000):
    rng = np.random.default_rng(seed)
    parts = ["", "-", "+", "0", "00", "1", "01", "9", "12", ".", ".5", "5.", "e", "E",
             "e+", "e-", "3", "0.", ".0", "inf", "Inf", "nan", "NaN", "infinity", "INFINITY",
             "in", "na", "0.1234567890123456789", "123456789012345678901234"]
    toks = []
    for _ in range(n):
        k = int(rng.integers(1, 5))
        t = "".join(parts[int(i)] for i in rng.integers(0, len(parts), k))
        if t:
            toks.append(t)
    return toks


@pytest.mark.parametrize("flags", [2, 4, 6])
def test_json_and_infnan_flags(ffpmod, flags):
    rng = np.random.default_rng(62 + flags)
    toks = _flag_tokens(70 + flags) + W.mixed_tokens(rng, 20_000)
    rng.shuffle(toks)
    buf = W.join_tokens(toks)
    c = ffpmod.Context(0, flags=flags)
    try:
        for fmt in ("f64", "f32", "f16"):
            _log("case flags", flags, fmt)
            rc, n, bits, status = run_gpu(c, buf, fmt)
            wb, ws = parse_buffer(buf, fmt, flags=flags)
            assert rc == len(wb) and n == len(wb)
            bad = np.flatnonzero((bits[:n] != np.array(wb, dtype=NP_DT[fmt])) |
                                 (status[:n] != np.array(ws, dtype=np.uint8)))
            assert bad.size == 0, (flags, fmt, [toks[i] for i in bad[:5]])
    finally:
        c.close()


def test_json_document_numbers(ffpmod):
    """Numbers of a JSON document with its structure bytes as delimiters:
    every coordinate parses, keys and string values come back invalid."""
    doc = W.geojson_document(63, 400, 40)
    delims = W.JSON_DELIMS
    c = ffpmod.Context(0, delims=delims, flags=ffpmod.FFP_JSON)
    try:
        rc, n, bits, status = run_gpu(c, doc, "f64")
        wb, ws = parse_buffer(doc, "f64", delims=delims, flags=2)
        assert rc == len(wb) == n
        assert np.array_equal(bits[:n], np.array(wb, dtype=np.uint64))
        assert np.array_equal(status[:n], np.array(ws, dtype=np.uint8))
        assert int((status[:n] == 0).sum()) == 400 * 40 * 2
    finally:
        c.close()


@pytest.fixture(scope="module")
def hex_case():
    rng = np.random.default_rng(65)
    toks = W.hex_tokens(rng, 30_000) + W.mixed_tokens(rng, 30_000) + W.hard_tokens(rng, 500)
    toks += ["0x", "0x.p1", "0x1p", "+0x1", "-0x0p0", "0X1P-1074", "0x1.fffffffffffff8p1023",
             "inf", "-nan", "0x1.8e3", "0x1p99999999999999999999"]
    rng.shuffle(toks)
    return toks, W.join_tokens(toks)


@pytest.mark.parametrize("flags", [8, 12])
@pytest.mark.parametrize("tile_k", [1, 2, 4])
def test_hex_tokens(ffpmod, hex_case, flags, tile_k):
    """Hexadecimal tokens (Appendix C) beside decimal ones, every tile size,
    every output type."""
    toks, buf = hex_case
    c = ffpmod.Context(0, flags=flags)
    try:
        c.set_tuning(tile_k, 0, 16)
        for fmt in ("f64", "f32", "f16", "bf16"):
            _log("case hex flags", flags, "tile_k", tile_k, fmt)
            rc, n, bits, status = run_gpu(c, buf, fmt, offset=3)
            wb, ws = parse_buffer(buf, fmt, flags=flags)
            assert rc == len(wb) and n == len(wb)
            bad = np.flatnonzero((bits[:n] != np.array(wb, dtype=NP_DT[fmt])) |
                                 (status[:n] != np.array(ws, dtype=np.uint8)))
            assert bad.size == 0, (flags, tile_k, fmt, [toks[i] for i in bad[:5]])
    finally:
        c.close()


def test_hex_tokens_with_reduction(ffpmod, hex_case):
    toks, buf = hex_case
    c = ffpmod.Context(0, flags=ffpmod.FFP_HEX | ffpmod.FFP_INFNAN)
    out = torch.full((3,), -1, dtype=torch.int64, device="cuda:0")
    try:
        c.set_reduce(out)
        for fmt in ("f64", "f32"):
            _log("case hex reduce", fmt)
            rc, n, bits, status = run_gpu(c, buf, fmt)
            wb, ws = parse_buffer(buf, fmt, flags=12)
            assert np.array_equal(bits[:n], np.array(wb, dtype=NP_DT[fmt]))
            got = [int(x) & 0xFFFFFFFFFFFFFFFF for x in out.cpu().tolist()]
            want = _expected_minmax(wb, ws, fmt)
            assert tuple(got) == want, (fmt, [hex(x) for x in got], [hex(x) for x in want])
        c.set_reduce(None)
    finally:
        c.close()


@pytest.fixture(scope="module")
def directed_case():
    """Mixed and hard tokens, exactly representable decimals (dyadic
    fractions written out, large integers) with neighbours one unit of a far
    digit away, hexadecimal tokens, and the ends of every format's range."""
    rng = np.random.default_rng(66)
    toks = W.mixed_tokens(rng, 20_000) + W.hard_tokens(rng, 1500) + W.hex_tokens(rng, 3000)
    for _ in range(4000):
        digits, e10 = W._exact_decimal(int(rng.integers(1, 2 ** 20)), -int(rng.integers(1, 28)))
        d = int(digits)
        toks += ["%de%d" % (d, e10), "%de%d" % (d * 10 ** 7 + 1, e10 - 7),
                 "%de%d" % (d * 10 ** 7 - 1, e10 - 7)]
    toks += [str(int(rng.integers(1, 2 ** 62)) << int(rng.integers(0, 40))) for _ in range(1000)]
    toks += ["1e309", "-1e309", "1.7976931348623158e308", "1.7976931348623159e308", "4.9e-324",
             "2e-324", "1e-400", "-1e-400", "3.4028235e38", "3.4028236e38", "1e-46", "-1e-46",
             "65504", "65520", "6e-8", "2.9e-8", "1e39", "-0", "0", "inf", "-nan", "x"]
    rng.shuffle(toks)
    return toks, W.join_tokens(toks)


@pytest.mark.parametrize("mode", [0x10, 0x20, 0x30])
@pytest.mark.parametrize("tile_k", [1, 4])
def test_directed_rounding(ffpmod, directed_case, mode, tile_k):
    """Rounding toward zero, +inf and -inf (with hexadecimal and inf/nan
    tokens), every output type; long tokens near representable values go
    through the exact fallback."""
    toks, buf = directed_case
    flags = mode | ffpmod.FFP_HEX | ffpmod.FFP_INFNAN
    c = ffpmod.Context(0, flags=flags)
    try:
        c.set_tuning(tile_k, 0, 16)
        for fmt in ("f64", "f32", "f16", "bf16"):
            _log("case directed", hex(mode), "tile_k", tile_k, fmt)
            rc, n, bits, status = run_gpu(c, buf, fmt, offset=1)
            wb, ws = parse_buffer(buf, fmt, flags=flags)
            assert rc == len(wb) and n == len(wb)
            bad = np.flatnonzero((bits[:n] != np.array(wb, dtype=NP_DT[fmt])) |
                                 (status[:n] != np.array(ws, dtype=np.uint8)))
            assert bad.size == 0, (hex(mode), tile_k, fmt, [toks[i] for i in bad[:5]])
    finally:
        c.close()


# ---------------------------------------------------------------------------
# in-kernel reduction
# ---------------------------------------------------------------------------

def _expected_minmax(bits, status, fmt):
    """(min bits, max bits, count) over OK, non-NaN values: numeric order,
    -0 before +0; NaN encodings for an empty set."""
    npdt = {"f64": np.float64, "f32": np.float32, "f16": np.float16}
    vals = []
    for b, s in zip(bits, status):
        if s != 0:
            continue
        if fmt == "bf16":
            v = float(np.array([b << 16], dtype=np.uint32).view(np.float32)[0])
        else:
            v = float(np.array([b], dtype=NP_DT[fmt]).view(npdt[fmt])[0])
        if v != v:
            continue
        vals.append(((v, 1 if (v != 0 or not math.copysign(1, v) < 0) else 0), b))
    if not vals:
        qnan = {"f64": 0x7FF8000000000000, "f32": 0x7FC00000, "f16": 0x7E00, "bf16": 0x7FC0}
        return qnan[fmt], qnan[fmt], 0
    return min(vals)[1], max(vals)[1], len(vals)


@pytest.mark.parametrize("fmt", ["f64", "f32", "f16", "bf16"])
def test_min_max_reduction(ffpmod, fmt):
    rng = np.random.default_rng(64)
    toks = W.mixed_tokens(rng, 50_000) + W.hard_tokens(rng, 2000)
    toks += ["-0", "0", "nan", "-nan", "inf", "-inf", "x1", "1e999", "-1e999", "1e-999"]
    rng.shuffle(toks)
    buf = W.join_tokens(toks)
    c = ffpmod.Context(0, flags=ffpmod.FFP_INFNAN)
    out = torch.full((3,), -1, dtype=torch.int64, device="cuda:0")
    try:
        c.set_reduce(out)
        for rep in range(2):  # the second call starts from a clean state
            rc, n, bits, status = run_gpu(c, buf, fmt)
            got = [int(x) & 0xFFFFFFFFFFFFFFFF for x in out.cpu().tolist()]
            wb, ws = parse_buffer(buf, fmt, flags=4)
            want = _expected_minmax(wb, ws, fmt)
            assert tuple(got) == want, (fmt, rep, [hex(x) for x in got], [hex(x) for x in want])
        # nothing to reduce: NaN encodings and a zero count
        rc, n, bits, status = run_gpu(c, b"x\ny\n-\n", fmt)
        got = [int(x) & 0xFFFFFFFFFFFFFFFF for x in out.cpu().tolist()]
        assert tuple(got) == _expected_minmax([], [], fmt)
        c.set_reduce(None)
    finally:
        c.close()


@pytest.mark.parametrize("flags", [0, 2 | 4, 8 | 0x20])
@pytest.mark.parametrize("reduce", [False, True])
def test_instances_at_8k_tiles(ffpmod, flags, reduce):
    """Every instance family (plain; JSON and inf / nan; hex and a directed
    mode), with and without the reduction, on 8 KiB tiles set explicitly
    (by default only the plain instance without a reduction runs there):
    parity with the oracle, and the reduction's minimum, maximum and
    count."""
    rng = np.random.default_rng(120 + flags + reduce)
    toks = W.mixed_tokens(rng, 30_000) + W.hard_tokens(rng, 600)
    toks += ["inf", "-nan", "0x1.8p3", "-0x1p-1074", "1.", "01", "-0"]
    rng.shuffle(toks)
    buf = W.join_tokens(toks)
    c = ffpmod.Context(0, flags=flags)
    out = torch.full((3,), -1, dtype=torch.int64, device="cuda:0")
    try:
        c.set_tuning(2, 0, 0)
        if reduce:
            c.set_reduce(out)
        for fmt in ("f64", "f32"):
            _log("case 8k tiles", hex(flags), reduce, fmt)
            rc, n, bits, status = run_gpu(c, buf, fmt, offset=5)
            wb, ws = parse_buffer(buf, fmt, flags=flags)
            assert rc == len(wb) and n == len(wb)
            bad = np.flatnonzero((bits[:n] != np.array(wb, dtype=NP_DT[fmt])) |
                                 (status[:n] != np.array(ws, dtype=np.uint8)))
            assert bad.size == 0, (hex(flags), reduce, fmt, [toks[i] for i in bad[:3]])
            if reduce:
                got = [int(x) & 0xFFFFFFFFFFFFFFFF for x in out.cpu().tolist()]
                assert tuple(got) == _expected_minmax(wb, ws, fmt), (hex(flags), fmt)
        if reduce:
            c.set_reduce(None)
    finally:
        c.close()


@pytest.mark.parametrize("delim", [b"\n", b"\x80", b"\xff"])
def test_high_bytes_and_high_delimiters(ffpmod, delim):
    """Bytes at or above 0x80 inside tokens (invalid tokens) and as the one
    delimiter byte: the single-delimiter classification covers bytes below
    0x80, a lone high delimiter takes the table path; parity either way."""
    rng = np.random.default_rng(130 + delim[0])
    toks = [t.encode() for t in W.mixed_tokens(rng, 20_000)]
    high = [b"\x80", b"\xa0", b"\xb0", b"\xb9", b"\xc3\xa9", b"\xff", b"\x8a", b"\xaa"]
    for i in rng.integers(0, len(toks), 800).tolist():
        t = toks[i]
        k = int(rng.integers(0, len(t) + 1))
        toks[i] = t[:k] + high[int(rng.integers(0, len(high)))] + t[k:]
    buf = delim.join(toks) + delim
    c = ffpmod.Context(0, delims=delim)
    try:
        for fmt in ("f64", "f32"):
            _log("case high bytes", delim, fmt)
            rc, n, bits, status = run_gpu(c, buf, fmt)
            wb, ws = parse_buffer(buf, fmt, delims=delim)
            assert rc == len(wb) and n == len(wb)
            assert np.array_equal(bits[:n], np.array(wb, dtype=NP_DT[fmt])), (delim, fmt)
            assert np.array_equal(status[:n], np.array(ws, dtype=np.uint8)), (delim, fmt)
            assert (status[:n] == 1).sum() >= 500
    finally:
        c.close()


# ---------------------------------------------------------------------------
# JSON documents: the structural index (FFP_JSON_DOCUMENT)
# ---------------------------------------------------------------------------

def _json_noise(seed, n):
    """Bytes from JSON's alphabet in random order (mostly not valid JSON):
    quotes, backslash runs, digits, signs, structure, letters."""
    rng = np.random.default_rng(seed)
    alphabet = np.frombuffer(b'0123456789012345-.eE+"""\\\\\\,,[]{}:  \n\tabtrue', dtype=np.uint8)
    return bytes(alphabet[rng.integers(0, len(alphabet), n)])


@pytest.fixture(scope="module")
def json_docs():
    docs = [W.json_tricky_document(91, 3000), W.json_tricky_document(92, 2000, indent=2),
            W.json_tricky_document(93, 1500, long_strings=True),
            W.geojson_document(94, 40, 200), _json_noise(95, 300_000)]
    from oracle import parse_json_document
    want = [{fmt: parse_json_document(d, fmt) for fmt in ("f64", "f32")} for d in docs]
    return docs, want


@pytest.mark.parametrize("block_kib,tile_k", [(0, 0), (4, 1), (16, 2), (16, 4), (64, 4), (64, 1)])
def test_json_document_numbers_outside_strings(ffpmod, json_docs, block_kib, tile_k):
    """Numbers of JSON texts whose strings hold digits, commas, escaped quotes
    and backslash runs (across chunks, tiles and blocks), and of random
    JSON-alphabet noise: count, values and status equal the oracle's."""
    docs, want = json_docs
    c = ffpmod.Context(0, flags=ffpmod.FFP_JSON_DOCUMENT)
    try:
        if tile_k:
            c.set_tuning(tile_k, 0, block_kib)
        for i, (doc, w) in enumerate(zip(docs, want)):
            for fmt in ("f64", "f32"):
                _log("case json-doc", i, fmt, block_kib, tile_k, len(doc))
                rc, n, bits, status = run_gpu(c, doc, fmt, offset=i % 16)
                wb, ws = w[fmt]
                assert rc == n == len(wb), (i, fmt, rc, n, len(wb))
                bad = np.flatnonzero((bits[:n] != np.array(wb, dtype=NP_DT[fmt])) |
                                     (status[:n] != np.array(ws, dtype=np.uint8)))
                assert bad.size == 0, (i, fmt, int(bad[0]))
    finally:
        c.close()


def test_json_document_plain_calls_only(ffpmod):
    c = ffpmod.Context(0, flags=ffpmod.FFP_JSON_DOCUMENT)
    try:
        t = torch.frombuffer(bytearray(b'[1, "2", 3]'), dtype=torch.uint8).to("cuda:0")
        v = torch.empty(4, dtype=torch.float64, device="cuda:0")
        s = torch.empty(4, dtype=torch.uint8, device="cuda:0")
        table = ffpmod.JobTable([t], [v], [s], "cuda:0")
        with pytest.raises(ffpmod.FFPError) as e:
            c.parse_batch(table.dev, 1, t.numel())
        assert e.value.code == ffpmod.FFP_E_ARG
        with pytest.raises(ffpmod.FFPError) as e:
            ffpmod.Server(c, hbm_budget_bytes=64 << 20)
        assert e.value.code == ffpmod.FFP_E_ARG
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
        assert c.parse_into(t, v, s, cnt, sync=True) == 2
        assert v[:2].cpu().tolist() == [1.0, 3.0]
    finally:
        c.close()


def test_small_calls_alternate_device_states(ffpmod):
    """Plain calls of at most 8 blocks of 4 KiB run without the count kernel,
    on two spare device states used in turn; larger calls use the main state
    and clean both spares.  A mixed sequence on one context (fallback tokens
    queued in some calls, a capacity error in one, texts that start
    mid-granule): each call matches the oracle and reports its own count and
    error code."""
    rng = np.random.default_rng(300)
    easy = W.join_tokens(W.mixed_tokens(rng, 1200))                     # ~24 KB
    hard = W.join_tokens(W.hard_tokens(rng, 90))                        # ~29 KB, queued
    big = W.join_tokens(W.mixed_tokens(rng, 20000) + W.hard_tokens(rng, 200))  # ~450 KB
    one_block = b"1.5\n-2e3\n" + b"0.1\n" * 900                        # below 4 KiB
    seq = [("hard", hard, None, 0), ("easy", easy, None, 0), ("big", big, None, 0),
           ("hard", hard, None, 7), ("hard", hard, None, 0), ("easy-cap", easy, 100, 0),
           ("one-block", one_block, None, 3), ("easy", easy, None, 5), ("big", big, None, 1),
           ("one-block", one_block, None, 0)]
    c = ffpmod.Context(0)
    try:
        for label, buf, cap, off in seq:
            _log("case alternate states", label, len(buf), "bytes, offset", off)
            for fmt in ("f64", "f32"):
                rc, n, bits, status = run_gpu(c, buf, fmt, capacity=cap, offset=off)
                wb, ws = parse_buffer(buf, fmt)
                assert n == len(wb), (label, fmt, n, len(wb))
                k = len(wb) if cap is None else min(cap, len(wb))
                if cap is not None and cap < len(wb):
                    assert rc == ffpmod.FFP_E_CAPACITY, (label, rc)
                else:
                    assert rc == len(wb), (label, rc)
                bad = np.flatnonzero((bits[:k] != np.array(wb[:k], dtype=NP_DT[fmt])) |
                                     (status[:k] != np.array(ws[:k], dtype=np.uint8)))
                assert bad.size == 0, (label, fmt, bad[:5])
                assert c.last_device_error() == 0, label
    finally:
        c.close()


@pytest.mark.parametrize("flags", [0, 0x06, 0x30 | 0x08])
def test_small_calls_decide_queued_tokens_in_parse(ffpmod, flags):
    """Plain calls of at most 32 blocks of 4 KiB decide their queued tokens in
    the parse kernel (each workgroup those of its own block, from the block's
    queue segment); larger calls keep the fallback kernel.  Texts of nothing
    but queued tokens (every block's segment busy), of mixed tokens, and of
    sizes around the 128 KiB limit, in every output type, with the plain,
    the JSON / inf-nan and the directed-rounding lexers."""
    rng = np.random.default_rng(310)
    hard = W.join_tokens(W.hard_tokens(rng, 3000))
    mixed = W.join_tokens(W.mixed_tokens(rng, 4000) + W.hard_tokens(rng, 300))
    # the first 20 digits of binary64 midpoints (2w + 1) 2^(e-1): their
    # truncations to 19 digits fall on either side of the midpoint, so every
    # token is queued (about 178 in each 4 KiB block)
    mids = []
    for _ in range(7000):
        w = int(rng.integers(2 ** 52, 2 ** 53))
        x = str((2 * w + 1) << int(rng.integers(20, 70)))
        mids.append("%se%d" % (x[:20], len(x) - 20))
    dense = W.join_tokens(mids)
    cases = []
    for name, pool in (("hard", hard), ("mixed", mixed), ("dense", dense)):
        for kib in (4, 60, 128, 132):
            buf = pool[: kib * 1024 - 37]
            cases.append((name, kib, buf[: buf.rfind(b"\n") + 1]))
    c = ffpmod.Context(0, flags=flags)
    try:
        for name, kib, buf in cases:
            for fmt in ("f64", "f32", "f16", "bf16"):
                _log("case local fallback", hex(flags), name, kib, "KiB", fmt)
                rc, n, bits, status = run_gpu(c, buf, fmt, offset=kib % 7)
                wb, ws = parse_buffer(buf, fmt, flags=flags)
                assert rc == len(wb) and n == len(wb), (name, kib, fmt, rc, len(wb))
                bad = np.flatnonzero((bits[:n] != np.array(wb, dtype=NP_DT[fmt])) |
                                     (status[:n] != np.array(ws, dtype=np.uint8)))
                assert bad.size == 0, (name, kib, fmt, bad[:5])
                assert c.last_device_error() == 0
    finally:
        c.close()
