"""Benchmark: exact decimal -> binary64/binary32 parsing on one MI355X.

Default workload (config2): 10M numbers in one ~198 MB buffer (50% uniform
[0,1) shortest digits, 25% coordinates with 6-15 fraction digits, 25% random
finite bit patterns as %.17e) parsed to binary64 by the plain single-buffer
entry point.  One step = one ffp_parse_f64 call (count, scan, parse and
fallback kernels) over the whole buffer, text already resident in HBM.

Other workloads (--workload):
  config1   100k uniform [0,1) shortest digits, one 1.93 MB buffer (latency)
  config3   2M hard cases (long midpoints, subnormals, overflow ...), binary64
  config4   4096 buffers, lognormal sizes (median 256 KiB, 1 KiB - 16 MiB),
            mixed formats; plain (one call per buffer) vs batched vs graph
  config4u  the same buffer sizes filled with config-1-format text (about
            3 GB, far above the 256 MB Infinity Cache): the HBM target run
  config5   served requests: Poisson open-loop arrivals at several rates,
            sizes lognormal (median 64 KiB, 512 B - 8 MiB), 90% binary64 /
            10% binary32, 1% hard cases, under a 32 GiB HBM budget; the
            continuous-batching server vs the plain one-launch-per-request
            server on the same arrivals, text on the device and in pinned
            host memory (H2D copy counted); p50/p99/p99.9 latency and GB/s

Prints one JSON line.  `roofline` reports the parse kernel's algorithmic
bytes (text read once + value + 1-byte status per token) over its average
duration measured with HIP events on the launch stream; `cpu_baseline` times
the CPU oracle on a bounded sample of the same text (config2 only).
"""

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GB/s input text + Mfloats/s parsed (bit-exact), batched/served vs plain; p50/p99"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2101_11408_amd/csrc/ffp_kernels.hip",
                  "paper_2101_11408_amd/csrc/ffp_device.h",
                  "paper_2101_11408_amd/csrc/ffp_internal.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str):
    """HBM traffic per launch from committed rocprofv3 counter runs, valid only
    for the kernel sources they were taken on."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    ent = data.get(workload)
    if not ent or ent.get("kernel_hash") != kernel_hash():
        return None
    return ent.get("bytes_per_launch")


# ---------------------------------------------------------------------------
# CPU oracle baseline
# ---------------------------------------------------------------------------
_SAMPLE = None


def _oracle_slice(bounds):
    from oracle import parse_buffer
    a, b = bounds
    bits, st = parse_buffer(_SAMPLE[a:b], "f64")
    return len(bits)


def cpu_baseline(buf: bytes, sample_tokens: int):
    global _SAMPLE
    end = 0
    for _ in range(sample_tokens):
        nxt = buf.find(b"\n", end)
        if nxt < 0:
            end = len(buf)
            break
        end = nxt + 1
    _SAMPLE = buf[:end]
    cores = max(1, min(16, os.cpu_count() or 1))
    step = max(1, end // (cores * 4))
    bounds, a = [], 0
    while a < end:
        b = min(end, a + step)
        nl = _SAMPLE.find(b"\n", b)
        b = end if nl < 0 else nl + 1
        bounds.append((a, b))
        a = b
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        n = sum(pool.map(_oracle_slice, bounds))
    dt = time.perf_counter() - t0
    return {
        "value": round(end / dt / 1e9, 6),
        "unit": "GB/s",
        "cores": cores,
        "kind": "oracle",
        "sample": "first %d tokens (%.1f MB) of the same buffer, %d worker processes; "
                  "%.3f Mfloats/s, %.2f s wall" % (n, end / 1e6, cores, n / dt / 1e6, dt),
    }


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def roofline(alg_bytes, kern_ms, workload):
    achieved = alg_bytes / (kern_ms / 1e3) / 1e9
    return {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": load_traffic(workload),
        "kernel": "k_parse",
        "kernel_avg_ms": round(kern_ms, 4),
        "algorithmic_bytes_per_launch": alg_bytes,
    }


def base_record(args, value, ms, workload, config, dtype="u64"):
    return {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": dict(workload=workload, **config),
    }


def timed_steps(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps if steps else 0.0


# ---------------------------------------------------------------------------
# single-buffer workloads
# ---------------------------------------------------------------------------

def run_plain(args, buf, ntok, workload, desc, out_dtype="f64", cpu=False):
    import torch
    from paper_2101_11408_amd import ffp
    dev = torch.device("cuda", 0)
    text = torch.frombuffer(bytearray(buf), dtype=torch.uint8).to(dev)
    dt = torch.float64 if out_dtype == "f64" else torch.float32
    values = torch.empty(ntok, dtype=dt, device=dev)
    status = torch.empty(ntok, dtype=torch.uint8, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    ctx = ffp.Context(0)
    ctx.reserve(len(buf))
    stream = torch.cuda.current_stream()
    n = ctx.parse_into(text, values, status, count, stream=stream, sync=True)
    assert n == ntok, n
    ms = timed_steps(torch, lambda: ctx.parse_into(text, values, status, count, stream=stream),
                     0, args.warmup)
    ctx.timing(True)
    ctx.timing_read()
    ms = timed_steps(torch, lambda: ctx.parse_into(text, values, status, count, stream=stream),
                     args.steps, 0)
    kern_ms, launches = ctx.timing_read()
    ctx.timing(False)
    assert launches == args.steps
    assert ctx.last_device_error() == 0
    assert int(count.item()) == ntok
    kavg = kern_ms / launches
    vbytes = 8 if out_dtype == "f64" else 4
    alg = len(buf) + (vbytes + 1) * ntok
    log("steps done: %.3f ms/step, parse kernel %.3f ms" % (ms, kavg))
    rec = base_record(args, len(buf) / (ms / 1e3) / 1e9, ms, workload, {
        "description": desc, "tokens": ntok, "bytes": len(buf),
        "output": "binary64" if out_dtype == "f64" else "binary32",
        "parallelism": "single GPU"})
    rec["mfloats_per_s"] = round(ntok / (ms / 1e3) / 1e6, 1)
    rec["roofline"] = roofline(alg, kavg, workload)
    rec["cpu_baseline"] = cpu_baseline(buf, min(args.cpu_sample, ntok)) if cpu else None
    ctx.close()
    return rec


# ---------------------------------------------------------------------------
# batched workloads (config 4)
# ---------------------------------------------------------------------------

def run_batched(args, kind, workload):
    import numpy as np
    import torch
    from gen import workloads as W
    from paper_2101_11408_amd import ffp
    dev = torch.device("cuda", 0)
    t0 = time.time()
    sizes = W.config4_sizes(4, args.nbuf)
    pool = W.token_pool(44, 2_000_000, "mixed" if kind == "mixed" else "uniform")
    plan = W.slice_plan(np.random.default_rng(4), pool, sizes)
    pool_dev = torch.frombuffer(bytearray(pool), dtype=torch.uint8).to(dev)
    texts, values, statuses, counts = [], [], [], []
    ntok_total = 0
    for st, ln in plan:
        t = torch.empty(ln, dtype=torch.uint8, device=dev)
        t.copy_(pool_dev[st:st + ln])
        cap = pool.count(b"\n", st, st + ln) + 1
        ntok_total += cap
        texts.append(t)
        values.append(torch.empty(cap, dtype=torch.float64, device=dev))
        statuses.append(torch.empty(cap, dtype=torch.uint8, device=dev))
        counts.append(torch.zeros(1, dtype=torch.int64, device=dev))
    del pool_dev
    torch.cuda.synchronize()
    total = int(sum(sizes))
    log("%d buffers, %.1f MB, built in %.1f s" % (len(texts), total / 1e6, time.time() - t0))

    ctx = ffp.Context(0)
    table = ffp.JobTable(texts, values, statuses, dev)
    stream = torch.cuda.current_stream()
    tune = ctx.autotune_batch(table.dev, table.n, total)
    log("autotuned schedule (tile_k, workgroups/CU):", tune)

    # plain: one call per buffer, back to back on one stream
    ctx.reserve(int(max(sizes)))

    def plain_all():
        for t, v, s, c in zip(texts, values, statuses, counts):
            ctx.parse_into(t, v, s, c, stream=stream)
    ms_plain = timed_steps(torch, plain_all, max(1, args.steps // 5), 1)

    # batched (one call) with the parse kernel timed
    ms_batch = timed_steps(torch, lambda: ctx.parse_batch(table.dev, table.n, total, stream),
                           0, args.warmup)
    ctx.timing(True)
    ctx.timing_read()
    ms_batch = timed_steps(torch, lambda: ctx.parse_batch(table.dev, table.n, total, stream),
                           args.steps, 0)
    kern_ms, launches = ctx.timing_read()
    ctx.timing(False)
    kavg = kern_ms / launches
    res = table.download()
    ntok = sum(c for c, e in res)
    assert all(e == 0 for c, e in res), "job errors"

    # captured graph replay
    graph = ffp.BatchGraph(ctx, table, total)
    ms_graph = timed_steps(torch, lambda: graph.launch(stream), args.steps, args.warmup)
    res2 = table.download()
    assert [c for c, e in res2] == [c for c, e in res] and all(e == 0 for c, e in res2)
    graph.close()
    assert ctx.last_device_error() == 0

    alg = total + 9 * ntok
    gbs = lambda ms: total / (ms / 1e3) / 1e9
    log("plain %.3f ms, batched %.3f ms, graph %.3f ms, parse kernel %.3f ms"
        % (ms_plain, ms_batch, ms_graph, kavg))
    rec = base_record(args, gbs(ms_graph), ms_graph, workload, {
        "description": "%d independent buffers, lognormal sizes (median 256 KiB, sigma 1.5, "
                       "1 KiB - 16 MiB), %s text, binary64; value = one replay of the "
                       "captured batched graph" % (len(texts),
                                                   "mixed-format" if kind == "mixed"
                                                   else "uniform [0,1) shortest-digit"),
        "buffers": len(texts), "tokens": ntok, "bytes": total, "output": "binary64",
        "parallelism": "single GPU", "schedule": {"tile_k": tune[0], "workgroups_per_cu": tune[1]}})
    rec["mfloats_per_s"] = round(ntok / (ms_graph / 1e3) / 1e6, 1)
    rec["compare"] = {
        "plain_one_call_per_buffer": {"ms": round(ms_plain, 3), "GB/s": round(gbs(ms_plain), 1)},
        "batched_call": {"ms": round(ms_batch, 3), "GB/s": round(gbs(ms_batch), 1)},
        "batched_graph": {"ms": round(ms_graph, 3), "GB/s": round(gbs(ms_graph), 1)},
    }
    rec["roofline"] = roofline(alg, kavg, workload)
    rec["cpu_baseline"] = None
    ctx.close()
    return rec


# ---------------------------------------------------------------------------
# served workload (config 5)
# ---------------------------------------------------------------------------

def serve_once(ffp, ctx, reqs, on_device, opts):
    """Replays one arrival schedule against a fresh server; returns per-request
    (latency ns, count, batch size) and the wall span."""
    import ctypes
    import queue
    import threading
    import numpy as np
    ptrs, sizes, dtypes, arrive = reqs
    n = len(ptrs)
    srv = ffp.Server(ctx, **opts)
    lat = np.zeros(n, dtype=np.int64)
    t_arr = np.zeros(n, dtype=np.int64)
    t_done = np.zeros(n, dtype=np.int64)
    counts = np.zeros(n, dtype=np.int64)
    batch = np.zeros(n, dtype=np.int64)
    errs = []
    tq = queue.SimpleQueue()

    def collector():
        for i in range(n):
            tk = tq.get()
            if tk is None:
                return
            r = srv.wait(tk)
            t_arr[i], t_done[i] = r.t_arrive_ns, r.t_done_ns
            counts[i], batch[i] = r.count, r.batch_jobs
            if r.err:
                errs.append((i, r.err))
            srv.release(tk)

    th = threading.Thread(target=collector)
    th.start()
    lib = ffp.load()
    submit = lib.ffp_server_submit
    h = srv.handle
    tkt = ctypes.c_uint64()
    ref = ctypes.byref(tkt)
    clock = time.monotonic_ns  # CLOCK_MONOTONIC, the server's clock
    assert abs(ffp.clock_ns() - clock()) < 50_000_000
    base = clock() + 20_000_000
    ondev = 1 if on_device else 0
    try:
        for i in range(n):
            target = base + int(arrive[i])
            d = target - clock()
            if d > 400_000:
                time.sleep((d - 250_000) / 1e9)
            while clock() < target:
                pass
            rc = submit(h, ptrs[i], int(sizes[i]), ondev, int(dtypes[i]), target, ref)
            if rc != 0:
                raise ffp.FFPError(rc, "ffp_server_submit")
            tq.put(tkt.value)
    except BaseException:
        tq.put(None)  # the collector stops after the tickets already queued
        th.join()
        srv.close()
        raise
    th.join()
    st = srv.stats()
    srv.close()
    assert not errs, errs[:5]
    lat[:] = t_done - t_arr
    span = (t_done.max() - t_arr.min()) / 1e9
    return lat, counts, batch, span, st


def summarize(lat, counts, sizes, batch, span, st):
    import numpy as np
    q = np.percentile(lat / 1e3, [50, 99, 99.9])
    return {
        "p50_us": round(float(q[0]), 1), "p99_us": round(float(q[1]), 1),
        "p999_us": round(float(q[2]), 1), "mean_us": round(float(lat.mean() / 1e3), 1),
        "GB/s": round(float(sizes.sum()) / span / 1e9, 3),
        "Mfloats/s": round(float(counts.sum()) / span / 1e6, 2),
        "span_s": round(span, 3), "batches": int(st["batches"]),
        "mean_batch": round(float(len(lat)) / max(1, st["batches"]), 2),
        "max_batch": int(st["max_batch_seen"]),
        "arena_peak_MB": round(st["arena_peak_bytes"] / 1e6, 1),
    }


def run_served(args, workload):
    import numpy as np
    import torch
    from gen import workloads as W
    from paper_2101_11408_amd import ffp
    sys.setswitchinterval(1e-4)
    dev = torch.device("cuda", 0)
    t0 = time.time()
    mixed = W.token_pool(55, 1_000_000, "mixed")
    hard = W.token_pool(56, 40_000, "hard")
    log("pools: mixed %.1f MB, hard %.1f MB, built in %.1f s"
        % (len(mixed) / 1e6, len(hard) / 1e6, time.time() - t0))
    pools = []
    for host in (mixed, hard):
        d = torch.frombuffer(bytearray(host), dtype=torch.uint8).to(dev)
        p = torch.empty(len(host), dtype=torch.uint8, pin_memory=True)
        p.copy_(torch.frombuffer(bytearray(host), dtype=torch.uint8))
        pools.append((d, p, len(host)))
    torch.cuda.synchronize()
    ctx = ffp.Context(0)
    budget = 32 << 30
    batched = dict(hbm_budget_bytes=budget, max_batch_bytes=256 << 20,
                   streams=args.serve_streams, max_batch_jobs=1024,
                   use_graph=args.serve_graph)
    plain = dict(hbm_budget_bytes=budget, max_batch_bytes=256 << 20,
                 mode=ffp.FFP_SERVE_PLAIN, streams=1)
    rows = []
    for ri, rate in enumerate(int(r) for r in args.rates.split(",")):
        t, sizes, is_f32, is_hard = W.config5_requests(5 + ri, rate, args.requests)
        rng = np.random.default_rng(500 + ri)
        which = is_hard.astype(np.int64)
        lim = np.array([pools[k][2] for k in which])
        sizes = np.minimum(sizes, lim)
        starts = (rng.random(len(sizes)) * (lim - sizes + 1)).astype(np.int64)
        dtypes = is_f32.astype(np.int64)
        arrive = (t * 1e9).astype(np.int64)
        row = {"rate_req_s": rate, "requests": len(sizes),
               "offered_GB/s": round(float(sizes.sum()) / float(t[-1]) / 1e9, 3),
               "binary32_share": round(float(is_f32.mean()), 3),
               "hard_share": round(float(is_hard.mean()), 4)}
        for name, opts, on_device in (("batched", batched, True), ("plain", plain, True),
                                      ("batched_host_text", batched, False)):
            ptrs = [(pools[k][0] if on_device else pools[k][1]).data_ptr() + int(s)
                    for k, s in zip(which, starts)]
            lat, counts, batch, span, st = serve_once(ffp, ctx, (ptrs, sizes, dtypes, arrive),
                                                      on_device, opts)
            row[name] = summarize(lat, counts, sizes, batch, span, st)
            log("rate %d %s: %s" % (rate, name, json.dumps(row[name])))
        rows.append(row)
    ctx.close()
    top = rows[-1]
    rec = base_record(args, top["batched"]["GB/s"], top["batched"]["p50_us"] / 1e3, workload, {
        "description": "served parse requests, Poisson open-loop arrivals at %s req/s, %d "
                       "requests per rate, sizes lognormal (median 64 KiB, sigma 1.5, 512 B - "
                       "8 MiB), 90%% binary64 / 10%% binary32, 1%% hard cases, 32 GiB HBM "
                       "budget; value = GB/s served by the continuous-batching server at the "
                       "highest rate (device-resident text); ms_per_step = its p50 latency"
                       % (args.rates, args.requests),
        "streams": args.serve_streams, "graph": bool(args.serve_graph),
        "parallelism": "single GPU"})
    rec["steps"] = args.requests
    rec["p50_us"] = top["batched"]["p50_us"]
    rec["p99_us"] = top["batched"]["p99_us"]
    rec["serve"] = rows
    rec["roofline"] = None
    rec["roofline_note"] = ("served batches are small and latency-bound; the parse kernel's "
                            "HBM roofline is measured on config4u")
    rec["cpu_baseline"] = None
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="config2",
                    choices=["config1", "config2", "config3", "config4", "config4u",
                             "config5"])
    ap.add_argument("--tokens", type=int, default=None)
    ap.add_argument("--nbuf", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=4_000_000)
    ap.add_argument("--rates", default="2000,5000,10000,20000")
    ap.add_argument("--requests", type=int, default=60_000)
    ap.add_argument("--serve-streams", type=int, default=2)
    ap.add_argument("--serve-graph", type=int, default=0)
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the parser's multi-GPU split is a design "
              "note (one prefix sum of per-shard token counts), not built; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    from gen import workloads as W

    wl = args.workload
    if wl == "config2":
        n = args.tokens or 10_000_000
        t0 = time.time()
        buf = W.config2(n=n)
        log("generated %d bytes in %.1f s" % (len(buf), time.time() - t0))
        rec = run_plain(args, buf, n, "config2-10M-mixed-binary64-plain",
                        "10M numbers in one %.1f MB buffer: 50%% uniform [0,1) shortest "
                        "digits, 25%% coordinates (6-15 fraction digits), 25%% random finite "
                        "bit patterns as %%.17e; binary64 output; one ffp_parse_f64 call per "
                        "step" % (len(buf) / 1e6), cpu=not args.no_cpu_baseline)
    elif wl == "config1":
        n = args.tokens or 100_000
        buf = W.config1(n=n)
        rec = run_plain(args, buf, n, "config1-100k-uniform-binary64-plain",
                        "100k uniform [0,1) doubles, shortest digits, positional, one "
                        "%.2f MB buffer; binary64" % (len(buf) / 1e6))
    elif wl == "config3":
        n = args.tokens or 2_000_000
        t0 = time.time()
        buf = W.config3(n=n)
        log("generated %d bytes in %.1f s" % (len(buf), time.time() - t0))
        rec = run_plain(args, buf, n, "config3-2M-hard-binary64-plain",
                        "2M hard cases (midpoints +-1 in the last of 20-800 digits, "
                        "subnormals, overflow, integers to 2^64, sign/zero variants) in one "
                        "%.1f MB buffer; binary64" % (len(buf) / 1e6))
    elif wl == "config4":
        rec = run_batched(args, "mixed", "config4-4096-buffers-mixed-batched")
    elif wl == "config5":
        rec = run_served(args, "config5-served-poisson")
    else:
        rec = run_batched(args, "uniform", "config4u-4096-buffers-uniform-batched")
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
