"""The exact in-kernel sum (ffp_set_reduce_sum) against the oracle's exact
sum of the oracle's own values, for every output format, tile size and
block size, with the minimum / maximum reduction on and off."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gen import workloads as W
from oracle import parse_buffer
from oracle.reduce import exact_sum

pytestmark = pytest.mark.gpu

TORCH_DT = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16,
            "bf16": torch.bfloat16}


def _log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ffpmod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_11408_amd import ffp
    ffp.load()
    return ffp


def parse_with_sum(ctx, buf: bytes, fmt: str, out, minmax=None):
    dev = torch.device("cuda", 0)
    text = torch.frombuffer(bytearray(buf), dtype=torch.uint8).to(dev) if buf else \
        torch.empty(0, dtype=torch.uint8, device=dev)
    cap = len(buf) // 2 + 1
    values = torch.empty(cap, dtype=TORCH_DT[fmt], device=dev)
    status = torch.empty(cap, dtype=torch.uint8, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    out.fill_(-1)
    if minmax is not None:
        minmax.fill_(-1)
    if buf:
        ctx.parse_into(text, values, status, count, sync=True)
    else:
        ctx.parse_into(text, values, status, count, nbytes=0, sync=True)
    got = [int(x) & 0xFFFFFFFFFFFFFFFF for x in out.cpu().tolist()]
    return got[0], bool(got[1])


def tokens(seed, n):
    rng = np.random.default_rng(seed)
    toks = W.mixed_tokens(rng, n) + W.hard_tokens(rng, max(1, n // 40))
    # exact cancellations, subnormals, all scales
    toks += ["1e308", "1e308", "-1e308", "-1e308", "4.9e-324", "-4.9e-324", "2.5e-320",
             "1.7976931348623157e308", "-1.7976931348623157e308", "-0", "0", "x", "1e999",
             "-1e-999", "123456789012345678901234567890", "-0.000000000000000000001"]
    rng.shuffle(toks)
    return toks


@pytest.mark.parametrize("fmt", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("tile_k,block_kib", [(0, 0), (1, 4), (2, 16), (4, 64)])
def test_sum_matches_oracle(ffpmod, fmt, tile_k, block_kib):
    toks = tokens(200 + tile_k, 30_000)
    buf = W.join_tokens(toks)
    wb, ws = parse_buffer(buf, fmt)
    want = exact_sum(wb, ws, fmt)
    c = ffpmod.Context(0)
    out = torch.zeros(2, dtype=torch.int64, device="cuda:0")
    mm = torch.zeros(3, dtype=torch.int64, device="cuda:0")
    try:
        if tile_k:
            c.set_tuning(tile_k, 0, block_kib)
        c.set_reduce_sum(out)
        for rep, with_minmax in enumerate([False, True, False]):
            c.set_reduce(mm if with_minmax else None)
            _log("case sum", fmt, tile_k, block_kib, "rep", rep)
            got = parse_with_sum(c, buf, fmt, out, mm if with_minmax else None)
            assert got == want, (fmt, tile_k, rep, hex(got[0]), hex(want[0]), got[1], want[1])
    finally:
        c.close()


def test_sum_special_cases(ffpmod):
    c = ffpmod.Context(0, flags=ffpmod.FFP_INFNAN)
    out = torch.zeros(2, dtype=torch.int64, device="cuda:0")
    cases = [
        [],                                   # empty sum: +0, exact
        ["-0", "-0.0", "-0e5"],               # every value -0: -0
        ["-0", "0"],                          # +0
        ["1", "-1"],                          # exact cancellation: +0
        ["inf", "1"],                         # +inf
        ["-inf", "1e300"],                    # -inf
        ["inf", "-inf"],                      # NaN
        ["nan", "2"],                         # NaN tokens are not summed
        ["1.7976931348623157e308", "1.7976931348623157e308"],  # overflow: +inf, inexact
        ["1", "1.1102230246251565e-16"],      # a tie (1 + 2^-53): rounds to even, 1
        ["4.9e-324", "4.9e-324", "4.9e-324"],  # subnormals add exactly
        ["1e-320", "1e300", "-1e300"],        # a tiny value survives cancellation
    ]
    try:
        c.set_reduce_sum(out)
        for toks in cases:
            buf = W.join_tokens(toks) if toks else b""
            wb, ws = parse_buffer(buf, "f64", flags=4) if toks else ([], [])
            want = exact_sum(wb, ws, "f64")
            _log("case sum special", toks)
            got = parse_with_sum(c, buf, "f64", out)
            assert got == want, (toks, hex(got[0]), hex(want[0]), got, want)
    finally:
        c.close()


def test_sum_large_input_many_blocks(ffpmod):
    """600,000 tokens in 4 KiB blocks over one workgroup per CU (every
    workgroup flushes a dozen blocks into the call's accumulators), then in
    16 KiB blocks; each call starts from zeroed accumulators."""
    rng = np.random.default_rng(210)
    vals = rng.standard_normal(600_000) * 10.0 ** rng.integers(-20, 20, 600_000)
    buf = b"\n".join(repr(float(v)).encode() for v in vals) + b"\n"
    wb, ws = parse_buffer(buf, "f64")
    want = exact_sum(wb, ws, "f64")
    c = ffpmod.Context(0)
    out = torch.zeros(2, dtype=torch.int64, device="cuda:0")
    try:
        c.set_reduce_sum(out)
        for rep in range(2):
            c.set_tuning(*[(1, 1, 4), (2, 0, 16)][rep])
            _log("case sum large rep", rep)
            got = parse_with_sum(c, buf, "f64", out)
            assert got == want, (rep, hex(got[0]), hex(want[0]))
    finally:
        c.close()
