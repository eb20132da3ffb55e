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
import re
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD_NAMES = {
    "config1": "config1-100k-uniform-binary64-plain",
    "config2": "config2-10M-mixed-binary64-plain",
    "config3": "config3-2M-hard-binary64-plain",
    "config4": "config4-4096-buffers-mixed-batched",
    "config4u": "config4u-4096-buffers-uniform-batched",
    "config5": "config5-served-poisson",
    "copycal": "copy-calibration",
    "jsondoc": "jsondoc-10M-coordinates-binary64-plain",
    "hexfloat": "hexfloat-10M-binary64-plain",
}
ROUND_FLAGS = {"nearest": 0x00, "zero": 0x10, "up": 0x20, "down": 0x30}
OUT_NAMES = {"f64": "binary64", "f32": "binary32", "f16": "binary16", "bf16": "bfloat16"}
METRIC = "GB/s input text + Mfloats/s parsed (bit-exact), batched/served vs plain; p50/p99"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2101_11408_amd/csrc/ffp_kernels.hip",
                  "paper_2101_11408_amd/csrc/ffp_device.h",
                  "paper_2101_11408_amd/csrc/ffp_internal.h"]


def out_name(wl, out, rnd="nearest"):
    """Workload name with the output format (and a directed rounding mode) of
    a plain run."""
    name = WORKLOAD_NAMES[wl].replace("binary64", OUT_NAMES[out])
    return name if rnd == "nearest" else name + "-round-" + rnd


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
        "spinup_ms": args.spinup_ms,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": dict(workload=workload, **config),
    }


def spin_up(torch, fn, ms):
    """Untimed calls for at least `ms` milliseconds of wall time, so that the
    timed steps run at the GPU's steady clocks rather than during the clock
    ramp after a process starts (a few warmup steps of this size take only
    a millisecond or two)."""
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()


def timed_steps(torch, fn, steps, warmup, spinup_ms=0.0):
    if spinup_ms > 0:
        spin_up(torch, fn, spinup_ms)
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

def run_plain(args, buf, ntok, workload, desc, out_dtype="f64", cpu=False, delims=b"\n",
              flags=0, expect_ok=None):
    import torch
    from paper_2101_11408_amd import ffp
    dev = torch.device("cuda", 0)
    text = torch.frombuffer(bytearray(buf), dtype=torch.uint8).to(dev)
    dt = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16,
          "bf16": torch.bfloat16}[out_dtype]
    values = torch.empty(ntok, dtype=dt, device=dev)
    status = torch.empty(ntok, dtype=torch.uint8, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    ctx = ffp.Context(0, delims=delims, flags=flags)
    ctx.reserve(len(buf))
    red = None
    if args.reduce:
        red = torch.zeros(3, dtype=torch.int64, device=dev)
        ctx.set_reduce(red)
    stream = torch.cuda.current_stream()
    n = ctx.parse_into(text, values, status, count, stream=stream, sync=True)
    assert n == ntok, n
    if expect_ok is not None:
        assert int((status[:n] == 0).sum()) == expect_ok
    ms = timed_steps(torch, lambda: ctx.parse_into(text, values, status, count, stream=stream),
                     0, args.warmup, args.spinup_ms)
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
    vbytes = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[out_dtype]
    alg = len(buf) + (vbytes + 1) * ntok
    log("steps done: %.3f ms/step, parse kernel %.3f ms" % (ms, kavg))
    rec = base_record(args, len(buf) / (ms / 1e3) / 1e9, ms, workload, {
        "description": desc, "tokens": ntok, "bytes": len(buf),
        "output": OUT_NAMES[out_dtype], "parallelism": "single GPU"})
    rec["mfloats_per_s"] = round(ntok / (ms / 1e3) / 1e6, 1)
    rec["roofline"] = roofline(alg, kavg, workload)
    rec["cpu_baseline"] = cpu_baseline(buf, min(args.cpu_sample, ntok)) if cpu else None
    if red is not None:
        mn, mx, cnt = [int(x) & 0xFFFFFFFFFFFFFFFF for x in red.cpu().tolist()]
        rec["reduce"] = {"min_bits": hex(mn), "max_bits": hex(mx), "count": cnt}
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
    if args.schedule:
        ctx.set_tuning(*[int(x) for x in args.schedule.split(",")])
        tune = ctx.get_tuning()
        log("fixed schedule (tile_k, workgroups/CU):", tune)
    else:
        tune = ctx.autotune_batch(table.dev, table.n, total)
        log("autotuned schedule (tile_k, workgroups/CU):", tune)

    # plain: one call per buffer, back to back on one stream
    ctx.reserve(int(max(sizes)))

    def plain_all():
        for t, v, s, c in zip(texts, values, statuses, counts):
            ctx.parse_into(t, v, s, c, stream=stream)
    ms_plain = None if args.profile else timed_steps(torch, plain_all,
                                                     max(1, args.steps // 5), 1)

    # batched (one call) with the parse kernel timed
    ms_batch = timed_steps(torch, lambda: ctx.parse_batch(table.dev, table.n, total, stream),
                           0, args.warmup, args.spinup_ms)
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
    if args.profile:
        ms_plain = ms_graph = ms_batch
    else:
        graph = ffp.BatchGraph(ctx, table, total)
        ms_graph = timed_steps(torch, lambda: graph.launch(stream), args.steps, args.warmup,
                               args.spinup_ms)
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
    """Replays one arrival schedule against a fresh server (ffp_server_replay:
    submission at each arrival time and in-order collection run in native
    threads); returns per-request latency (ns), counts, batch sizes, the wall
    span and the server's statistics."""
    import numpy as np
    ptrs, sizes, dtypes, arrive = reqs
    srv = ffp.Server(ctx, **opts)
    try:
        base = ffp.clock_ns() + 20_000_000
        out = srv.replay(ptrs, sizes, 1 if on_device else 0, dtypes, base + arrive)
        st = srv.stats()
    finally:
        srv.close()
    bad = np.flatnonzero(out["err"] != 0)
    assert bad.size == 0, ("request errors", bad[:5], out["err"][bad[:5]])
    ta = out["t_arrive_ns"].astype(np.int64)
    td = out["t_done_ns"].astype(np.int64)
    lat = td - ta
    exp = (base + arrive).astype(np.int64)
    off = np.flatnonzero(ta != exp)
    if off.size:
        raise AssertionError(
            "arrival mismatch at %d requests, first %s: got %d want %d (done %d launch %d "
            "count %d err %d)" % (off.size, off[:5].tolist(), int(ta[off[0]]), int(exp[off[0]]),
                                  int(td[off[0]]), int(out["t_launch_ns"][off[0]]),
                                  int(out["count"][off[0]]), int(out["err"][off[0]])))
    log("  arrivals %d..%d done %d..%d max latency %.1f us at %d"
        % (int(ta.min()) - int(base), int(ta.max()) - int(base), int(td.min()) - int(base),
           int(td.max()) - int(base), lat.max() / 1e3, int(lat.argmax())))
    span = (int(td.max()) - int(ta.min())) / 1e9
    return lat, out["count"].astype(np.int64), out["batch_jobs"], span, st


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
    config_rates = [int(r) for r in args.rates.split(",")]
    extra_rates = [int(r) for r in args.extra_rates.split(",") if r]
    for ri, rate in enumerate(config_rates + extra_rates):
        t, sizes, is_f32, is_hard = W.config5_requests(5 + ri, rate, args.requests)
        rng = np.random.default_rng(500 + ri)
        which = is_hard.astype(np.int64)
        lim = np.array([pools[k][2] for k in which])
        sizes = np.minimum(sizes, lim)
        starts = (rng.random(len(sizes)) * (lim - sizes + 1)).astype(np.int64)
        dtypes = is_f32.astype(np.int64)
        arrive = (t * 1e9).astype(np.int64)
        row = {"rate_req_s": rate, "requests": len(sizes),
               "beyond_config": rate not in config_rates,
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
    top = [r for r in rows if not r["beyond_config"]][-1]
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


# ---------------------------------------------------------------------------
# HBM traffic from rocprofv3 counters
# ---------------------------------------------------------------------------
CAL_BYTES = 1 << 30


def run_copycal(args):
    """A plain streaming kernel of known size (read 1 GiB, write 1 GiB), the
    calibration point of the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.ones(CAL_BYTES // 8, dtype=torch.int64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(max(1, args.steps)):
        torch.bitwise_not(src, out=dst)
    torch.cuda.synchronize()
    return {"calibration": "bitwise_not int64", "read_bytes": CAL_BYTES,
            "write_bytes": CAL_BYTES, "launches": max(1, args.steps)}


def _counter_rows(csv_path, counter, match):
    import csv
    vals = []
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] == counter and match(row["Kernel_Name"]):
                vals.append(float(row["Counter_Value"]))
    if not vals:
        raise SystemExit("no %s rows for the kernel in %s" % (counter, csv_path))
    return vals


def reduce_traffic(workload, fetch_csv, write_csv, cal_fetch_csv, cal_write_csv, command):
    """profiles/traffic.json[workload] = HBM bytes per parse-kernel launch:
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch, averaged over dispatches),
    each scaled by bytes / counter of the calibration kernel."""
    is_parse = lambda n: "k_parse" in n
    is_cal = lambda n: "bitwise_not" in n or "BitwiseNot" in n
    mean = lambda v: sum(v) / len(v)
    f_k = mean(_counter_rows(fetch_csv, "FETCH_SIZE", is_parse))
    w_k = mean(_counter_rows(write_csv, "WRITE_SIZE", is_parse))
    f_c = mean(_counter_rows(cal_fetch_csv, "FETCH_SIZE", is_cal))
    w_c = mean(_counter_rows(cal_write_csv, "WRITE_SIZE", is_cal))
    ff = CAL_BYTES / (f_c * 1024.0)
    fw = CAL_BYTES / (w_c * 1024.0)
    ent = {
        "kernel_hash": kernel_hash(),
        "bytes_per_launch": round(f_k * 1024.0 * ff + w_k * 1024.0 * fw),
        "fetch_bytes": round(f_k * 1024.0 * ff),
        "write_bytes": round(w_k * 1024.0 * fw),
        "fetch_kib_raw": f_k, "write_kib_raw": w_k,
        "calibration_fetch_factor": round(ff, 4), "calibration_write_factor": round(fw, 4),
        "command": command,
    }
    path = os.path.join(ROOT, "profiles", "traffic.json")
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data[workload] = ent
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")
    md = ["# HBM traffic of the parse kernel: %s" % workload, "",
          "Commands (from the repository root, on one MI355X):", "", "    " + command, "",
          "| quantity | value |", "|---|---|",
          "| FETCH_SIZE per dispatch (raw, KiB) | %.1f |" % f_k,
          "| WRITE_SIZE per dispatch (raw, KiB) | %.1f |" % w_k,
          "| calibration kernel (bitwise NOT of 1 GiB int64) FETCH_SIZE, WRITE_SIZE (KiB) | "
          "%.1f, %.1f |" % (f_c, w_c),
          "| factors (true bytes / counter bytes) fetch, write | %.4f, %.4f |" % (ff, fw),
          "| HBM bytes fetched per launch | %d |" % ent["fetch_bytes"],
          "| HBM bytes written per launch | %d |" % ent["write_bytes"],
          "| total (bench.py roofline.traffic) | %d |" % ent["bytes_per_launch"],
          "| kernel source hash | %s |" % ent["kernel_hash"], ""]
    with open(os.path.join(ROOT, "profiles", "k_parse_%s_traffic.md" % workload), "w") as f:
        f.write("\n".join(md))
    return ent


def summarize_trace(workload, trace_dir, command, bench_json=None):
    """profiles/<kernel>_<workload>.md from a rocprofv3 --kernel-trace --stats
    run: the per-kernel table, the parse kernel's dispatches grouped by grid
    size, and the bench's own HIP-event average for comparison."""
    import csv
    import glob
    stats = glob.glob(os.path.join(trace_dir, "*kernel_stats.csv"))[0]
    trace = glob.glob(os.path.join(trace_dir, "*kernel_trace.csv"))[0]
    lines = ["# rocprofv3 kernel trace: %s" % workload, "",
             "Command (from the repository root, on one MI355X):", "",
             "    " + command, "",
             "## Per-kernel statistics (`--stats`)", "",
             "| kernel | calls | avg us | min us | max us | share % |",
             "|---|---|---|---|---|---|"]
    with open(stats) as f:
        rows = list(csv.DictReader(f))
    for r in rows[:10]:
        lines.append("| `%s` | %s | %.1f | %.1f | %.1f | %s |" % (
            r["Name"][:70], r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, r["Percentage"]))
    groups = {}
    with open(trace) as f:
        for r in csv.DictReader(f):
            if "k_parse" not in r["Kernel_Name"]:
                continue
            key = (r["Kernel_Name"], int(r["Grid_Size_X"]))
            groups.setdefault(key, []).append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines += ["", "## Parse kernel dispatches by grid size (`kernel_trace.csv`)", "",
              "| kernel | grid (threads) | dispatches | avg us | min us | max us |",
              "|---|---|---|---|---|---|"]
    ranked = sorted(groups.items(), key=lambda kv: -sum(kv[1]))
    for (name, grid), d in ranked[:8]:
        lines.append("| `%s` | %d | %d | %.1f | %.1f | %.1f |" % (
            name[:40], grid, len(d), sum(d) / len(d), min(d), max(d)))
    rest = [x for _, d in ranked[8:] for x in d]
    if rest:
        lines.append("| %d other grid sizes | | %d | %.1f | %.1f | %.1f |" % (
            len(ranked) - 8, len(rest), sum(rest) / len(rest), min(rest), max(rest)))
    if bench_json:
        with open(bench_json) as f:
            rec = json.loads(f.read().strip().splitlines()[-1])
        rf = rec.get("roofline") or {}
        lines += ["", "## The same run's bench line", "",
                  "HIP-event average of the parse kernel over the timed steps: %.1f us; "
                  "value %s %s; ms_per_step %s." % (
                      rf.get("kernel_avg_ms", float("nan")) * 1e3, rec["value"], rec["unit"],
                      rec["ms_per_step"])]
        if rec.get("config", {}).get("schedule"):
            lines.append("Schedule chosen by the autotuner: %s." % rec["config"]["schedule"])
    name = "k_parse_%s.md" % workload
    with open(os.path.join(ROOT, "profiles", name), "w") as f:
        f.write("\n".join(lines) + "\n")
    return name


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--spinup-ms", type=float, default=200.0,
                    help="untimed calls for this long before the warmup steps (GPU clock ramp)")
    ap.add_argument("--workload", default="config2",
                    choices=["config1", "config2", "config3", "config4", "config4u",
                             "config5", "copycal", "jsondoc", "hexfloat"])
    ap.add_argument("--round", default="nearest", choices=sorted(ROUND_FLAGS),
                    help="plain workloads: rounding direction (FFP_ROUND_*)")
    ap.add_argument("--tokens", type=int, default=None)
    ap.add_argument("--nbuf", type=int, default=4096)
    ap.add_argument("--reduce", action="store_true",
                    help="plain workloads: also keep the min, max and count of the values")
    ap.add_argument("--out", default="f64", choices=["f64", "f32", "f16", "bf16"],
                    help="plain workloads: output format")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=4_000_000)
    ap.add_argument("--rates", default="2000,5000,10000,20000")
    ap.add_argument("--extra-rates", default="50000,100000",
                    help="served workload: rates beyond the configuration's range, "
                         "reported separately (saturation)")
    ap.add_argument("--requests", type=int, default=60_000)
    ap.add_argument("--serve-streams", type=int, default=2)
    ap.add_argument("--serve-graph", type=int, default=0)
    ap.add_argument("--schedule", default="",
                    help="batched workloads: tile_k,workgroups_per_cu instead of the autotuner")
    ap.add_argument("--profile", action="store_true",
                    help="batched workloads: only the timed batched calls (for counter runs)")
    ap.add_argument("--reduce-traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV",
                                                          "CAL_FETCH_CSV", "CAL_WRITE_CSV"),
                    help="write profiles/traffic.json for --workload from rocprofv3 "
                         "counter CSVs (no GPU needed)")
    ap.add_argument("--traffic-command", default="")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_DIR", "BENCH_JSON"),
                    help="write profiles/k_parse_<workload>.md from a rocprofv3 kernel "
                         "trace of the bench command given by --traffic-command")
    args = ap.parse_args()

    if args.summarize_trace:
        print(summarize_trace(WORKLOAD_NAMES[args.workload], args.summarize_trace[0],
                              args.traffic_command, args.summarize_trace[1]))
        return

    if args.reduce_traffic:
        ent = reduce_traffic(WORKLOAD_NAMES[args.workload], *args.reduce_traffic,
                             args.traffic_command)
        print(json.dumps(ent), flush=True)
        return

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
        rec = run_plain(args, buf, n, out_name(wl, args.out, args.round),
                        "10M numbers in one %.1f MB buffer: 50%% uniform [0,1) shortest "
                        "digits, 25%% coordinates (6-15 fraction digits), 25%% random finite "
                        "bit patterns as %%.17e; %s output; one parse call per step"
                        % (len(buf) / 1e6, OUT_NAMES[args.out]), out_dtype=args.out,
                        cpu=not args.no_cpu_baseline and args.out == "f64" and args.round == "nearest",
                        flags=ROUND_FLAGS[args.round])
    elif wl == "config1":
        n = args.tokens or 100_000
        buf = W.config1(n=n)
        rec = run_plain(args, buf, n, out_name(wl, args.out, args.round),
                        "100k uniform [0,1) doubles, shortest digits, positional, one "
                        "%.2f MB buffer; %s" % (len(buf) / 1e6, OUT_NAMES[args.out]),
                        out_dtype=args.out, flags=ROUND_FLAGS[args.round])
    elif wl == "config3":
        n = args.tokens or 2_000_000
        t0 = time.time()
        buf = W.config3(n=n)
        log("generated %d bytes in %.1f s" % (len(buf), time.time() - t0))
        rec = run_plain(args, buf, n, out_name(wl, args.out, args.round),
                        "2M hard cases (midpoints +-1 in the last of 20-800 digits, "
                        "subnormals, overflow, integers to 2^64, sign/zero variants) in one "
                        "%.1f MB buffer; %s" % (len(buf) / 1e6, OUT_NAMES[args.out]),
                        out_dtype=args.out, flags=ROUND_FLAGS[args.round])
    elif wl == "config4":
        rec = run_batched(args, "mixed", WORKLOAD_NAMES[wl])
    elif wl == "jsondoc":
        t0 = time.time()
        nfeat = (args.tokens or 10_000_000) // 2000
        doc = W.geojson_document(7, nfeat, 1000)
        ntok = len(re.findall(b"[^" + re.escape(W.JSON_DELIMS) + b"]+", doc))
        log("generated %d bytes, %d tokens in %.1f s" % (len(doc), ntok, time.time() - t0))
        rec = run_plain(args, doc, ntok, out_name(wl, args.out),
                        "GeoJSON-like document (%.1f MB): %d features of 1000 coordinate pairs "
                        "with 6-15 fraction digits; JSON number grammar, the document's "
                        "structure bytes as delimiters (keys and strings come back invalid); "
                        "%s" % (len(doc) / 1e6, nfeat, OUT_NAMES[args.out]),
                        out_dtype=args.out, delims=W.JSON_DELIMS, flags=2,
                        expect_ok=nfeat * 2000)
    elif wl == "hexfloat":
        import numpy as np
        n = args.tokens or 10_000_000
        t0 = time.time()
        rng = np.random.default_rng(9)
        x = rng.standard_normal(n) * np.power(10.0, rng.integers(-300, 300, n).astype(np.float64))
        buf = ("\n".join(float(v).hex() for v in x.tolist()) + "\n").encode()
        log("generated %d bytes in %.1f s" % (len(buf), time.time() - t0))
        rec = run_plain(args, buf, n, out_name(wl, args.out, args.round),
                        "10M random doubles (normal * 10^U[-300,300)) in their own hexadecimal "
                        "form (Appendix C), one %.1f MB buffer; FFP_HEX; %s"
                        % (len(buf) / 1e6, OUT_NAMES[args.out]), out_dtype=args.out,
                        flags=8 | ROUND_FLAGS[args.round], expect_ok=n)
    elif wl == "config5":
        rec = run_served(args, WORKLOAD_NAMES[wl])
    elif wl == "copycal":
        rec = run_copycal(args)
    else:
        rec = run_batched(args, "uniform", WORKLOAD_NAMES[wl])
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
