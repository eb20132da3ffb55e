"""Batched parsing on the GPU (ffp_parse_batch, captured graphs, autotuner):
every job must equal the oracle's parse of its own text, bit for bit."""

import os

import numpy as np
import pytest

from gen import workloads as W
from oracle import parse_buffer

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


@pytest.fixture(scope="module")
def pool():
    rng = np.random.default_rng(71)
    toks = W.mixed_tokens(rng, 120_000) + W.hard_tokens(rng, 4000)
    rng.shuffle(toks)
    host = W.join_tokens(toks)
    dev = torch.frombuffer(bytearray(host), dtype=torch.uint8).to("cuda:0")
    return host, dev


FMT_OF = {torch.float64: "f64", torch.float32: "f32", torch.float16: "f16",
          torch.bfloat16: "bf16"}
INT_OF = {"f64": (torch.int64, np.uint64), "f32": (torch.int32, np.uint32),
          "f16": (torch.int16, np.uint16), "bf16": (torch.int16, np.uint16)}


def build_jobs(ffpmod, pool, sizes, f32_mask, seed, dtypes=None):
    host, dev = pool
    rng = np.random.default_rng(seed)
    plan = W.slice_plan(rng, host, sizes)
    # also start some jobs at odd offsets inside a token
    texts, values, statuses, spans = [], [], [], []
    for i, (st, ln) in enumerate(plan):
        if i % 7 == 3 and ln > 2:
            st, ln = st + 1, ln - 1
        texts.append(dev[st:st + ln])
        cap = ln // 2 + 1
        dt = dtypes[i] if dtypes is not None else (torch.float32 if f32_mask[i] else torch.float64)
        values.append(torch.empty(cap, dtype=dt, device="cuda:0"))
        statuses.append(torch.full((cap,), 255, dtype=torch.uint8, device="cuda:0"))
        spans.append((st, ln))
    table = ffpmod.JobTable(texts, values, statuses, "cuda:0")
    return table, values, statuses, spans


def check_jobs(pool, table, values, statuses, spans, label, flags=0):
    host, _ = pool
    res = table.download()
    for i, ((st, ln), (count, err)) in enumerate(zip(spans, res)):
        buf = host[st:st + ln]
        fmt = FMT_OF[values[i].dtype]
        wb, ws = parse_buffer(buf, fmt, flags=flags)
        assert count == len(wb), (label, i, count, len(wb))
        assert err == 0, (label, i, err)
        n = len(wb)
        if n == 0:
            continue
        ib, npb = INT_OF[fmt]
        got = values[i][:n].view(ib).cpu().numpy().view(npb)
        gs = statuses[i][:n].cpu().numpy()
        bad = np.flatnonzero((got != np.array(wb, dtype=npb)) | (gs != np.array(ws, dtype=np.uint8)))
        assert bad.size == 0, (label, i, fmt, int(bad[0]))


def test_batch_matches_oracle(ctx, ffpmod, pool):
    rng = np.random.default_rng(5)
    sizes = W.lognormal_sizes(rng, 300, 6000, 1.5, 1, 200_000)
    sizes[:5] = [0, 1, 2, 15, 16]
    f32 = rng.random(300) < 0.15
    table, values, statuses, spans = build_jobs(ffpmod, pool, sizes, f32, 6)
    _log("batch jobs", table.n, "bytes", table.total_bytes)
    ctx.parse_batch(table.dev, table.n, table.total_bytes)
    torch.cuda.synchronize()
    assert ctx.last_device_error() == 0
    check_jobs(pool, table, values, statuses, spans, "batch")


def test_single_job_batch_equals_plain(ctx, ffpmod, pool):
    host, dev = pool
    text = dev[3:700_003]
    values = torch.empty(400_000, dtype=torch.float64, device="cuda:0")
    status = torch.empty(400_000, dtype=torch.uint8, device="cuda:0")
    table = ffpmod.JobTable([text], [values], [status], "cuda:0")
    ctx.parse_batch(table.dev, 1, text.numel())
    torch.cuda.synchronize()
    (count, err), = table.download()
    v2 = torch.empty_like(values)
    s2 = torch.empty_like(status)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    n = ctx.parse_into(text, v2, s2, cnt, sync=True)
    assert err == 0 and count == n
    assert torch.equal(values[:n].view(torch.int64), v2[:n].view(torch.int64))
    assert torch.equal(status[:n], s2[:n])


def test_batch_graph_replays(ctx, ffpmod, pool):
    rng = np.random.default_rng(8)
    n = 64
    sizes_a = W.lognormal_sizes(rng, n, 20_000, 1.0, 100, 150_000)
    f32 = rng.random(n) < 0.2
    table, values, statuses, spans = build_jobs(ffpmod, pool, sizes_a, f32, 9)
    budget = 64 * 150_000
    graph = ffpmod.BatchGraph(ctx, table, budget)
    try:
        host, dev = pool
        for rep in range(4):
            if rep:
                # rewrite the records on the device: new text slices for the
                # same output buffers
                plan = W.slice_plan(np.random.default_rng(100 + rep), host,
                                    [min(int(s), 150_000) for s in
                                     W.lognormal_sizes(np.random.default_rng(200 + rep), n,
                                                       20_000, 1.0, 100, 150_000)])
                spans = []
                for i, (st, ln) in enumerate(plan):
                    ln = min(ln, 2 * (values[i].numel() - 1))
                    table.host[i].text = dev[st:st + ln].data_ptr()
                    table.host[i].nbytes = ln
                    table.host[i].count = 0
                    table.host[i].err = 0
                    spans.append((st, ln))
                table.upload()
            # the program's own eager work between replays
            scratch = torch.arange(1 << 20, device="cuda:0").sum()
            _ = scratch.item()
            graph.launch()
            torch.cuda.synchronize()
            _log("graph replay", rep)
            check_jobs(pool, table, values, statuses, spans, "graph-%d" % rep)
    finally:
        graph.close()


def test_batch_job_errors(ctx, ffpmod, pool):
    host, dev = pool
    t1 = dev[0:50_000]
    t2 = dev[50_000:60_000]
    v1 = torch.empty(100, dtype=torch.float64, device="cuda:0")  # far too small
    s1 = torch.empty(100, dtype=torch.uint8, device="cuda:0")
    v2 = torch.empty(10_000, dtype=torch.float64, device="cuda:0")
    s2 = torch.empty(10_000, dtype=torch.uint8, device="cuda:0")
    table = ffpmod.JobTable([t1, t2], [v1, v2], [s1, s2], "cuda:0")
    table.host[1].dtype = 7  # unknown output type
    table.upload()
    ctx.parse_batch(table.dev, 2, 60_000)
    torch.cuda.synchronize()
    (c1, e1), (c2, e2) = table.download()
    wb, ws = parse_buffer(host[0:50_000], "f64")
    assert c1 == len(wb) and e1 == ffpmod.FFP_E_CAPACITY
    got = v1.view(torch.int64).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, np.array(wb[:100], dtype=np.uint64))
    assert c2 == 0 and e2 == ffpmod.FFP_E_ARG
    # the byte bound of the call is exceeded: every job reports it
    table.host[1].dtype = 0
    table.upload()
    ctx.parse_batch(table.dev, 2, 1000)
    torch.cuda.synchronize()
    res = table.download()
    assert all(c == 0 and e == ffpmod.FFP_E_CAPACITY for c, e in res)


def test_autotune_and_cache(ffpmod, pool, tmp_path):
    rng = np.random.default_rng(10)
    sizes = W.lognormal_sizes(rng, 200, 30_000, 1.5, 100, 300_000)
    table, values, statuses, spans = build_jobs(ffpmod, pool, sizes, np.zeros(200, bool), 11)
    cache = tmp_path / "tune.json"
    os.environ["FFP_TUNE_CACHE"] = str(cache)
    try:
        c = ffpmod.Context(0)
        k, b = c.autotune_batch(table.dev, table.n, table.total_bytes)
        assert k in (1, 2, 4) and b >= 1
        assert c.get_tuning() == (k, b)
        assert cache.exists() and "cus=" in cache.read_text()
        c.close()
        c2 = ffpmod.Context(0)
        assert c2.autotune_batch(table.dev, table.n, table.total_bytes) == (k, b)
        c2.parse_batch(table.dev, table.n, table.total_bytes)
        torch.cuda.synchronize()
        check_jobs(pool, table, values, statuses, spans, "tuned")
        c2.close()
    finally:
        del os.environ["FFP_TUNE_CACHE"]


def test_batch_all_output_types(ctx, ffpmod, pool):
    """Jobs of the four output types in one batch."""
    rng = np.random.default_rng(15)
    n = 160
    sizes = W.lognormal_sizes(rng, n, 8000, 1.5, 1, 120_000)
    kinds = [torch.float64, torch.float32, torch.float16, torch.bfloat16]
    dtypes = [kinds[int(k)] for k in rng.integers(0, 4, n)]
    table, values, statuses, spans = build_jobs(ffpmod, pool, sizes, None, 16, dtypes)
    ctx.parse_batch(table.dev, table.n, table.total_bytes)
    torch.cuda.synchronize()
    check_jobs(pool, table, values, statuses, spans, "four-types")


def test_batch_hex_tokens(ffpmod):
    """Hexadecimal and decimal tokens (flag FFP_HEX) in jobs of the four
    output types."""
    rng = np.random.default_rng(17)
    toks = W.hex_tokens(rng, 40_000) + W.mixed_tokens(rng, 40_000) + W.hard_tokens(rng, 1000)
    rng.shuffle(toks)
    host = W.join_tokens(toks)
    hp = (host, torch.frombuffer(bytearray(host), dtype=torch.uint8).to("cuda:0"))
    n = 120
    sizes = W.lognormal_sizes(rng, n, 8000, 1.5, 1, 100_000)
    kinds = [torch.float64, torch.float32, torch.float16, torch.bfloat16]
    dtypes = [kinds[int(k)] for k in rng.integers(0, 4, n)]
    c = ffpmod.Context(0, flags=ffpmod.FFP_HEX)
    try:
        table, values, statuses, spans = build_jobs(ffpmod, hp, sizes, None, 18, dtypes)
        c.parse_batch(table.dev, table.n, table.total_bytes)
        torch.cuda.synchronize()
        assert c.last_device_error() == 0
        check_jobs(hp, table, values, statuses, spans, "hex", flags=8)
    finally:
        c.close()


def test_batch_directed_rounding(ffpmod, pool):
    """Rounding toward -infinity in a batch of the four output types."""
    rng = np.random.default_rng(19)
    n = 100
    sizes = W.lognormal_sizes(rng, n, 8000, 1.5, 1, 100_000)
    kinds = [torch.float64, torch.float32, torch.float16, torch.bfloat16]
    dtypes = [kinds[int(k)] for k in rng.integers(0, 4, n)]
    c = ffpmod.Context(0, flags=ffpmod.FFP_ROUND_DOWN)
    try:
        table, values, statuses, spans = build_jobs(ffpmod, pool, sizes, None, 20, dtypes)
        c.parse_batch(table.dev, table.n, table.total_bytes)
        torch.cuda.synchronize()
        assert c.last_device_error() == 0
        check_jobs(pool, table, values, statuses, spans, "round-down", flags=0x30)
    finally:
        c.close()


def _check_against(pool, table, values, statuses, spans, want, label):
    """Every job's count, error, value bits and status against precomputed
    oracle results."""
    host, _ = pool
    res = table.download()
    for i, ((st, ln), (count, err), (wb, ws)) in enumerate(zip(spans, res, want)):
        assert err == 0, (label, i, err)
        assert count == len(wb), (label, i, count, len(wb))
        n = len(wb)
        if n == 0:
            continue
        fmt = FMT_OF[values[i].dtype]
        ib, npb = INT_OF[fmt]
        got = values[i][:n].view(ib).cpu().numpy().view(npb)
        gs = statuses[i][:n].cpu().numpy()
        bad = np.flatnonzero((got != np.array(wb, dtype=npb)) | (gs != np.array(ws, dtype=np.uint8)))
        assert bad.size == 0, (label, i, fmt, ln, int(bad[0]))


@pytest.mark.parametrize("block_kib,tile_k", [(64, 4), (64, 2), (16, 4)])
def test_batch_4096_jobs_large_blocks(ffpmod, block_kib, tile_k):
    """The shape of the 4096-buffer workloads: 4096 jobs, blocks of 64 KiB
    walked in several tiles (and 16 KiB blocks of one 16 KiB tile), jobs
    from empty to several blocks long, some starting inside a token; the
    batched call and replays of its captured graph, every job against the
    oracle."""
    from oracle_par import parse_many
    rng = np.random.default_rng(81)
    toks = W.mixed_tokens(rng, 200_000) + W.hard_tokens(rng, 1500)
    rng.shuffle(toks)
    host = W.join_tokens(toks)
    pool = (host, torch.frombuffer(bytearray(host), dtype=torch.uint8).to("cuda:0"))
    n = 4096
    sizes = W.lognormal_sizes(rng, n, 6000, 1.5, 1, 400_000)
    sizes[:6] = [0, 1, 17, 65536, 65536 + 16, 3 * 65536 - 5]
    kinds = [torch.float64, torch.float32, torch.float16, torch.bfloat16]
    dtypes = [kinds[int(k)] for k in rng.choice(4, n, p=[0.7, 0.2, 0.05, 0.05])]
    table, values, statuses, spans = build_jobs(ffpmod, pool, sizes, None, 82, dtypes)
    want = parse_many([host[st:st + ln] for st, ln in spans],
                      [FMT_OF[v.dtype] for v in values])
    _log("4096 jobs", table.total_bytes, "bytes, blocks", block_kib, "KiB, tile_k", tile_k)
    c = ffpmod.Context(0)
    graph = None
    try:
        c.set_tuning(tile_k, 0, block_kib)
        c.parse_batch(table.dev, table.n, table.total_bytes)
        torch.cuda.synchronize()
        assert c.last_device_error() == 0
        _check_against(pool, table, values, statuses, spans, want, "batch")
        graph = ffpmod.BatchGraph(c, table, table.total_bytes)
        for rep in range(3):
            for s in statuses:
                s.fill_(255)
            table.upload()  # counts and errors back to zero
            _ = torch.arange(1 << 20, device="cuda:0").sum().item()  # eager work between
            graph.launch()
            torch.cuda.synchronize()
            _log("graph replay", rep)
            _check_against(pool, table, values, statuses, spans, want, "graph-%d" % rep)
    finally:
        if graph is not None:
            graph.close()
        c.close()
