"""Benchmark: exact decimal -> binary64/binary32 parsing on one MI355X.

Default workload (config4u, the HBM target run): 4096 independent buffers with
lognormal sizes (median 256 KiB, sigma 1.5, 1 KiB - 16 MiB; about 3.06 GB,
far above the 256 MB Infinity Cache), filled with config-1-format text
(uniform [0,1) doubles, shortest round-trip digits, newline-separated),
parsed to binary64.  One step = one replay of the captured batched graph
(job-table, count, scan, parse and fallback kernels over all 4096 buffers),
text already resident in HBM.  The same buffers are also parsed with one
batched call per step and with one plain call per buffer (the comparison
point), and every output of the three forms is compared.  A short served
run (config 5's arrivals at 2k-20k requests/s, fewer requests per rate)
adds p50/p99/p99.9 latency of the continuous-batching server against one
launch per request.

Other workloads (--workload):
  config1   100k uniform [0,1) shortest digits, one 1.93 MB buffer (latency)
  config2   10M numbers, one 198 MB buffer: 50% uniform shortest digits, 25%
            coordinates with 6-15 fraction digits, 25% %.17e of random bits
  config3   2M hard cases (long midpoints, subnormals, overflow ...)
  config4   4096 buffers as config4u, filled with config-2's mix of formats
  config5   served requests: Poisson open-loop arrivals at several rates,
            sizes lognormal (median 64 KiB, 512 B - 8 MiB), 90% binary64 /
            10% binary32, 1% hard cases, under a 32 GiB HBM budget; the
            continuous-batching server vs one launch per request, text on
            the device and in pinned host memory (H2D copy counted)
  jsondoc, hexfloat   widened rows (JSON document, hexadecimal tokens)
  copycal   a plain streaming kernel of known size (counter calibration)

Prints one JSON line.  `roofline`: the parse kernel's algorithmic bytes
(text read once + value + 1-byte status per token) over its average
duration measured with HIP events on the launch stream, against 8 TB/s and
against a streaming copy measured in the same run.  `cpu_baseline`: the CPU
oracle timed over the workload's distinct text on the machine's CPU share; the
same oracle results are compared with every GPU output (`parity`).
"""

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import re
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
    "csv": "csv-1M-rows-5-of-10-columns-binary64-plain",
    "hexfloat": "hexfloat-10M-binary64-plain",
}
ROUND_FLAGS = {"nearest": 0x00, "zero": 0x10, "up": 0x20, "down": 0x30}
OUT_NAMES = {"f64": "binary64", "f32": "binary32", "f16": "binary16", "bf16": "bfloat16"}
VALUE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}
METRIC = "GB/s input text + Mfloats/s parsed (bit-exact), batched/served vs plain; p50/p99"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2101_11408_amd/csrc/ffp_kernels.hip",
                  "paper_2101_11408_amd/csrc/ffp_device.h",
                  "paper_2101_11408_amd/csrc/ffp_lexer.h",
                  "paper_2101_11408_amd/csrc/ffp_fallback.h",
                  "paper_2101_11408_amd/csrc/ffp_internal.h"]
# worker processes for host-side work: the CPU share of one GPU on the
# measurement boxes
MAX_WORKERS = 16


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


def workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(MAX_WORKERS, n))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------------------
# Tokens of a text (numpy; no parsing): spans of the runs of non-delimiters
# ---------------------------------------------------------------------------

def token_spans(text: bytes, delims: bytes = b"\n"):
    import numpy as np
    arr = np.frombuffer(text, dtype=np.uint8)
    lut = np.zeros(256, dtype=bool)
    lut[list(delims)] = True
    nd = ~lut[arr]
    if nd.size == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    prev = np.concatenate([[False], nd[:-1]])
    nxt = np.concatenate([nd[1:], [False]])
    return np.flatnonzero(nd & ~prev), np.flatnonzero(nd & ~nxt) + 1


class PoolIndex:
    """Token spans of a pool of text from which buffers or requests are cut.
    A slice [a, b) of the pool holds the pool's tokens that lie wholly inside
    it, plus at most one cut token at each end (bytes of a pool token that
    the slice starts or ends inside of)."""

    def __init__(self, pool: bytes):
        self.pool = pool
        self.starts, self.ends = token_spans(pool)

    def slice(self, a: int, b: int):
        """(k0, k1, head, tail): pool tokens k0..k1-1 lie inside [a, b);
        head / tail are the cut tokens before / after them (bytes or None)."""
        import numpy as np
        s, e = self.starts, self.ends
        k0 = int(np.searchsorted(s, a, side="left"))   # first token starting at or after a
        k1 = int(np.searchsorted(e, b, side="right"))  # tokens ending at or before b
        head = tail = None
        if k0 > 0 and e[k0 - 1] > a:  # a token that starts before a and ends after it
            head = self.pool[a:min(int(e[k0 - 1]), b)] or None
        if k1 < len(s) and a <= s[k1] < b:  # a token that starts inside and ends after b
            tail = self.pool[int(s[k1]):b]
        if k1 < k0:  # the slice lies inside one token: it is the head
            k1 = k0
        return k0, k1, head, tail


# ---------------------------------------------------------------------------
# The cpu_baseline leg: the CPU oracle over the workload's distinct text,
# timed, on worker processes; its results are what the GPU outputs are
# compared with (parity).  The only part of this file that runs the oracle.
# ---------------------------------------------------------------------------
_SHARED = {}


def _oracle_chunk(args):
    from oracle import parse_buffer, parse_csv, parse_json_document
    import numpy as np
    a, b, fmt = args
    if _SHARED.get("csv") is not None:
        bits, st = parse_csv(_SHARED["text"][a:b], _SHARED["csv"], fmt, _SHARED["delims"],
                             _SHARED["flags"] & ~0x80)
    elif _SHARED.get("doc"):
        bits, st = parse_json_document(_SHARED["text"][a:b], fmt, flags=_SHARED["flags"])
    else:
        bits, st = parse_buffer(_SHARED["text"][a:b], fmt, delims=_SHARED["delims"],
                                flags=_SHARED["flags"])
    return np.array(bits, dtype=np.uint64), np.array(st, dtype=np.uint8)


def _oracle_tokens(args):
    from oracle import parse_token
    import numpy as np
    toks, fmt = args
    out = [parse_token(t, fmt, _SHARED["flags"]) for t in toks]
    return (np.array([b for b, _ in out], dtype=np.uint64),
            np.array([s for _, s in out], dtype=np.uint8))


def cpu_baseline_leg(text: bytes, fmts, extra_tokens=(), delims=b"\n", flags=0, what="",
                     doc_split=None, csv_columns=None):
    """Times the oracle over every token of `text` (for each output format
    in `fmts`) and over `extra_tokens` (cut tokens of slices), on the box's
    CPU share.  With doc_split the text is a JSON document read as one
    (numbers outside strings), cut for the workers just after occurrences of
    doc_split, which must lie outside strings and between tokens.  Returns
    (cpu_baseline record, {fmt: (bits, status)} for the text's tokens,
    {fmt: (bits, status)} for the extra tokens)."""
    import numpy as np
    _SHARED.update(text=text, delims=delims, flags=flags, doc=doc_split is not None,
                   csv=csv_columns)
    if csv_columns is not None:  # a CSV table is cut after row ends only
        doc_split = b"\n"
    nw = workers()
    # chunks cut at delimiters (or after doc_split), several per worker
    nchunk = max(1, min(64 * nw, len(text) // 4096 or 1))
    bounds, a = [], 0
    lut = set(delims)
    for k in range(1, nchunk + 1):
        b = len(text) if k == nchunk else max(a, len(text) * k // nchunk)
        if doc_split is not None:
            j = text.find(doc_split, b)
            b = len(text) if j < 0 else j + len(doc_split)
        else:
            while b < len(text) and text[b] not in lut:
                b += 1
        if b > a:
            bounds.append((a, b))
        a = b
    extra = list(extra_tokens)
    ctx = mp.get_context("fork")
    res_text, res_extra, secs = {}, {}, {}
    with ctx.Pool(nw) as pool:
        for fmt in fmts:
            t0 = time.perf_counter()
            parts = pool.map(_oracle_chunk, [(a, b, fmt) for a, b in bounds], chunksize=1)
            secs[fmt] = time.perf_counter() - t0
            res_text[fmt] = (np.concatenate([p[0] for p in parts]) if parts else
                             np.zeros(0, np.uint64),
                             np.concatenate([p[1] for p in parts]) if parts else
                             np.zeros(0, np.uint8))
            step = max(1, len(extra) // (4 * nw) + 1)
            eparts = pool.map(_oracle_tokens, [(extra[i:i + step], fmt)
                                               for i in range(0, len(extra), step)])
            res_extra[fmt] = (np.concatenate([p[0] for p in eparts]) if eparts else
                              np.zeros(0, np.uint64),
                              np.concatenate([p[1] for p in eparts]) if eparts else
                              np.zeros(0, np.uint8))
    f0 = fmts[0]
    ntok = len(res_text[f0][0])
    dt = secs[f0]
    rec = {
        "value": round(len(text) / dt / 1e9, 6),
        "unit": "GB/s",
        "cores": nw,
        "kind": "oracle",
        "sample": "%s: %d tokens (%.1f MB), %s output, %d worker processes (the CPU share of "
                  "one GPU; %d CPUs visible); %.3f Mfloats/s, %.2f s wall"
                  % (what, ntok, len(text) / 1e6, OUT_NAMES.get(f0, f0), nw,
                     os.cpu_count() or 0, ntok / dt / 1e6, dt),
        "mfloats_per_s": round(ntok / dt / 1e6, 3),
        "cpu_model": cpu_model(),
    }
    return rec, res_text, res_extra


def strtod_context(text: bytes, threads=(1, None)):
    """The C library's strtod over the same text (context, not a target)."""
    import ctypes
    from paper_2101_11408_amd.build import STRTOD_LIB
    if not os.path.exists(STRTOD_LIB):
        return None
    lib = ctypes.CDLL(STRTOD_LIB)
    fn = lib.ffp_ctx_strtod_seconds
    fn.restype = ctypes.c_double
    fn.argtypes = [ctypes.c_char_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                   ctypes.POINTER(ctypes.c_uint64)]
    out = {}
    for th in threads:
        th = th or workers()
        n = ctypes.c_uint64()
        s = fn(text, len(text), 0, th, 3, ctypes.byref(n))
        if s > 0:
            out["threads_%d" % th] = {"GB/s": round(len(text) / s / 1e9, 4),
                                      "Mfloats/s": round(n.value / s / 1e6, 2)}
    return {"what": "glibc strtod over the same text (best of 3), binary64",
            "cpu_model": cpu_model(), **out}


def count_mismatches(got_bits, got_st, want_bits, want_st):
    import numpy as np
    if len(got_bits) != len(want_bits):
        return max(len(got_bits), len(want_bits))
    return int(np.count_nonzero((got_bits != want_bits) | (got_st != want_st)))


def slice_parity(slices, pool_ids, fmts, pool_res, extra_res, got):
    """Mismatches between GPU outputs of slices of token pools and the
    oracle.  slices: PoolIndex.slice results; pool_res[pool][fmt]: the
    oracle's (bits, status) of every token of a pool; extra_res[fmt]: the
    same for the cut tokens of all slices, in slice order (head, then tail);
    got(i) -> (bits, status) the GPU produced for slice i."""
    import numpy as np
    bad, e = 0, 0
    for i, ((k0, k1, h, t), pid, f) in enumerate(zip(slices, pool_ids, fmts)):
        pb, ps = pool_res[pid][f]
        eb, es = extra_res[f]
        wb, ws = [pb[k0:k1]], [ps[k0:k1]]
        if h is not None:
            wb.insert(0, eb[e:e + 1])
            ws.insert(0, es[e:e + 1])
            e += 1
        if t is not None:
            wb.append(eb[e:e + 1])
            ws.append(es[e:e + 1])
            e += 1
        gb, gs = got(i)
        bad += count_mismatches(gb, gs, np.concatenate(wb), np.concatenate(ws))
    return bad


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def copy_peak(torch, reps=10):
    """A streaming copy (bitwise NOT of 1 GiB of int64, read once and written
    once) timed with events on torch's stream: the bandwidth a plain
    streaming kernel reaches on this GPU, the second roofline denominator."""
    n = (1 << 30) // 8
    src = torch.ones(n, dtype=torch.int64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.bitwise_not(src, out=dst)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        torch.bitwise_not(src, out=dst)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    del src, dst
    return 2 * (1 << 30) / (times[len(times) // 2] / 1e3) / 1e9


def roofline(alg_bytes, kern_ms, workload, copy_gbs=None):
    achieved = alg_bytes / (kern_ms / 1e3) / 1e9
    rec = {
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
    if copy_gbs:
        rec["copy_peak_measured"] = round(copy_gbs, 1)
        rec["frac_of_copy_peak"] = round(achieved / copy_gbs, 4)
    return rec


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
    ramp after a process starts."""
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


def repeat_stats(torch, fn, reps):
    """Min and median of `reps` calls, each bracketed by HIP events on the
    current stream (the paper reports the minimum and the median over
    repetitions, Section 12); run after the timed steps, apart from them."""
    if reps <= 0:
        return None
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in evs)
    return {"reps": reps, "min_ms": round(ts[0], 4), "median_ms": round(ts[len(ts) // 2], 4),
            "how": "HIP events around each call on the launch stream, after the timed steps"}


# ---------------------------------------------------------------------------
# single-buffer workloads
# ---------------------------------------------------------------------------

def run_plain(args, buf, ntok, workload, desc, out_dtype="f64", cpu=True, delims=b"\n",
              flags=0, expect_ok=None, doc_split=None, csv_columns=None):
    import numpy as np
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
    if csv_columns is not None:
        ctx.set_csv_columns(csv_columns)
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
    rep = None if args.profile else repeat_stats(
        torch, lambda: ctx.parse_into(text, values, status, count, stream=stream), args.reps)
    assert ctx.last_device_error() == 0
    assert int(count.item()) == ntok
    kavg = kern_ms / launches
    alg = len(buf) + (VALUE_BYTES[out_dtype] + 1) * ntok
    log("steps done: %.3f ms/step, parse kernel %.3f ms" % (ms, kavg))
    rec = base_record(args, len(buf) / (ms / 1e3) / 1e9, ms, workload, {
        "description": desc, "tokens": ntok, "bytes": len(buf),
        "output": OUT_NAMES[out_dtype], "parallelism": "single GPU"})
    rec["mfloats_per_s"] = round(ntok / (ms / 1e3) / 1e6, 1)
    rec["repeat"] = rep
    rec["roofline"] = roofline(alg, kavg, workload, None if args.profile else copy_peak(torch))
    if red is not None:
        mn, mx, cnt = [int(x) & 0xFFFFFFFFFFFFFFFF for x in red.cpu().tolist()]
        rec["reduce"] = {"min_bits": hex(mn), "max_bits": hex(mx), "count": cnt}
    got_bits = values.view({8: torch.int64, 4: torch.int32, 2: torch.int16}[
        VALUE_BYTES[out_dtype]]).cpu().numpy().astype(np.uint64)
    got_bits &= np.uint64((1 << (8 * VALUE_BYTES[out_dtype])) - 1)
    got_st = status.cpu().numpy()
    ctx.close()
    rec["cpu_baseline"] = None
    if cpu and not args.profile:
        cb, res, _ = cpu_baseline_leg(buf, [out_dtype], delims=delims, flags=flags,
                                      what="the whole buffer", doc_split=doc_split,
                                      csv_columns=csv_columns)
        wb, ws = res[out_dtype]
        rec["cpu_baseline"] = cb
        rec["parity"] = {"vs": "oracle", "tokens_checked": int(len(wb)),
                         "tokens": ntok, "full": True,
                         "mismatches": count_mismatches(got_bits, got_st, wb, ws)}
        if red is not None:  # the minimum, maximum and count of the oracle's values
            want = expected_minmax(wb, ws, out_dtype)
            rec["reduce"]["oracle"] = {"min_bits": hex(want[0]), "max_bits": hex(want[1]),
                                       "count": want[2]}
            rec["parity"]["reduce_matches"] = want == (mn, mx, cnt)
        rec["context"] = {"glibc_strtod": strtod_context(buf)} if out_dtype == "f64" and \
            delims == b"\n" and flags == 0 else {}
    return rec


def expected_minmax(bits, status, out_dtype):
    """(minimum bits, maximum bits, count) of the values with status OK, NaN
    left out, -0 ordered before +0; the format's quiet NaN twice and 0 for
    an empty set (the reduction's contract)."""
    import numpy as np
    qnan = {"f64": 0x7FF8000000000000, "f32": 0x7FC00000, "f16": 0x7E00, "bf16": 0x7FC0}
    width = VALUE_BYTES[out_dtype] * 8
    b = np.asarray(bits, dtype=np.uint64)[np.asarray(status, dtype=np.uint8) == 0]
    if out_dtype == "f64":
        v = b.view(np.float64)
    elif out_dtype == "f32":
        v = b.astype(np.uint32).view(np.float32).astype(np.float64)
    elif out_dtype == "f16":
        v = b.astype(np.uint16).view(np.float16).astype(np.float64)
    else:
        v = (b.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)
    keep = ~np.isnan(v)
    b, v = b[keep], v[keep]
    if b.size == 0:
        return qnan[out_dtype], qnan[out_dtype], 0
    sign = np.uint64(1 << (width - 1))
    neg_zero = (v == 0) & ((b & sign) != 0)
    lo, hi = v.min(), v.max()
    if lo == 0:
        mn = int(sign) if neg_zero.any() else 0
    else:
        mn = int(b[np.argmin(v)])
    if hi == 0:
        mx = 0 if (~neg_zero & (v == 0)).any() else int(sign)
    else:
        mx = int(b[np.argmax(v)])
    return mn, mx, int(b.size)


# ---------------------------------------------------------------------------
# 4096 buffers (configs 4 and 4u): plain per buffer vs batched vs graph
# ---------------------------------------------------------------------------

def run_buffers(args, kind, workload):
    import numpy as np
    import torch
    from gen import workloads as W
    from paper_2101_11408_amd import ffp
    dev = torch.device("cuda", 0)
    t0 = time.time()
    sizes = W.config4_sizes(4, args.nbuf)
    pool = W.token_pool(44, 2_000_000, "mixed" if kind == "mixed" else "uniform")
    plan = W.slice_plan(np.random.default_rng(4), pool, sizes)
    pidx = PoolIndex(pool)
    slices = [pidx.slice(st, st + ln) for st, ln in plan]
    caps = np.array([(k1 - k0) + (h is not None) + (t is not None)
                     for k0, k1, h, t in slices], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(caps)])
    ntok_total = int(offs[-1])
    pool_dev = torch.frombuffer(bytearray(pool), dtype=torch.uint8).to(dev)
    texts = []
    for st, ln in plan:
        t = torch.empty(ln, dtype=torch.uint8, device=dev)  # separate allocations
        t.copy_(pool_dev[st:st + ln])
        texts.append(t)
    del pool_dev
    # flat outputs; job i writes values[offs[i] : offs[i] + caps[i]]
    vals = {k: torch.zeros(ntok_total, dtype=torch.float64, device=dev) for k in ("plain", "batch")}
    stat = {k: torch.full((ntok_total,), 255, dtype=torch.uint8, device=dev)
            for k in ("plain", "batch")}
    counts = torch.zeros(len(texts), dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    total = int(sum(sizes))
    log("%d buffers, %.1f MB, %d tokens, built in %.1f s"
        % (len(texts), total / 1e6, ntok_total, time.time() - t0))

    def views(k, i):
        a, b = int(offs[i]), int(offs[i + 1])
        return vals[k][a:b], stat[k][a:b]

    ctx = ffp.Context(0)
    table = ffp.JobTable(texts, *zip(*[views("batch", i) for i in range(len(texts))]), dev)
    stream = torch.cuda.current_stream()
    if args.schedule:
        ctx.set_tuning(*[int(x) for x in args.schedule.split(",")])
        tune = ctx.get_tuning()
        log("fixed schedule (tile_k, workgroups/CU):", tune)
    else:
        tune = ctx.autotune_batch(table.dev, table.n, total)
        log("autotuned schedule (tile_k, workgroups/CU):", tune)

    # plain: one call per buffer, back to back on one stream
    pctx = ffp.Context(0)
    pctx.reserve(int(max(sizes)))
    pviews = [views("plain", i) for i in range(len(texts))]

    def plain_all():
        for i, (t, (v, s)) in enumerate(zip(texts, pviews)):
            pctx.parse_into(t, v, s, counts[i:i + 1], stream=stream)
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
    assert all(e == 0 for c, e in res), "job errors"
    job_counts = np.array([c for c, e in res], dtype=np.int64)
    assert np.array_equal(job_counts, caps), "token counts"
    ntok = int(job_counts.sum())
    check = {}
    if not args.profile:
        assert np.array_equal(counts.cpu().numpy(), caps), "plain token counts"
        check["batched_vs_plain_mismatches"] = int(
            ((vals["plain"].view(torch.int64) != vals["batch"].view(torch.int64)) |
             (stat["plain"] != stat["batch"])).sum().item())

    # captured graph replay, into outputs cleared first
    rep = None
    if args.profile:
        ms_plain = ms_graph = ms_batch
    else:
        vals["batch"].fill_(-1.0)
        stat["batch"].fill_(254)
        table.upload()
        graph = ffp.BatchGraph(ctx, table, total)
        ms_graph = timed_steps(torch, lambda: graph.launch(stream), args.steps, args.warmup,
                               args.spinup_ms)
        rep = repeat_stats(torch, lambda: graph.launch(stream), args.reps)
        res2 = table.download()
        assert [c for c, e in res2] == [c for c, e in res] and all(e == 0 for c, e in res2)
        graph.close()
        check["graph_vs_plain_mismatches"] = int(
            ((vals["plain"].view(torch.int64) != vals["batch"].view(torch.int64)) |
             (stat["plain"] != stat["batch"])).sum().item())
    assert ctx.last_device_error() == 0 and pctx.last_device_error() == 0

    alg = total + 9 * ntok
    gbs = lambda ms: total / (ms / 1e3) / 1e9
    log("plain %.3f ms, batched %.3f ms, graph %.3f ms, parse kernel %.3f ms"
        % (ms_plain, ms_batch, ms_graph, kavg))
    rec = base_record(args, gbs(ms_graph), ms_graph, workload, {
        "description": "%d independent buffers (separate allocations), lognormal sizes "
                       "(median 256 KiB, sigma 1.5, 1 KiB - 16 MiB), %s text, binary64; "
                       "value = one replay of the captured batched graph"
                       % (len(texts), "config-2 mix of formats" if kind == "mixed"
                          else "config-1 format (uniform [0,1) shortest digits)"),
        "buffers": len(texts), "tokens": ntok, "bytes": total, "output": "binary64",
        "parallelism": "single GPU", "schedule": {"tile_k": tune[0], "workgroups_per_cu": tune[1]}})
    rec["mfloats_per_s"] = round(ntok / (ms_graph / 1e3) / 1e6, 1)
    rec["compare"] = {
        "plain_one_call_per_buffer": {"ms": round(ms_plain, 3), "GB/s": round(gbs(ms_plain), 1)},
        "batched_call": {"ms": round(ms_batch, 3), "GB/s": round(gbs(ms_batch), 1)},
        "batched_graph": {"ms": round(ms_graph, 3), "GB/s": round(gbs(ms_graph), 1)},
    }
    rec["repeat"] = rep  # graph replays one by one
    rec["roofline"] = roofline(alg, kavg, workload, None if args.profile else copy_peak(torch))
    rec["cpu_baseline"] = None
    if not args.profile:
        # the oracle over the pool (every distinct token of the workload) and
        # the cut tokens at buffer ends; compared with every plain output
        extra = [x for k0, k1, h, t in slices for x in (h, t) if x is not None]
        cb, res_pool, res_extra = cpu_baseline_leg(
            pool, ["f64"], extra, what="the token pool all 4096 buffers are cut from, plus "
                                       "the tokens cut at buffer ends")
        got_b = vals["plain"].view(torch.int64).cpu().numpy().view(np.uint64)
        got_s = stat["plain"].cpu().numpy()
        bad = slice_parity(slices, [0] * len(slices), ["f64"] * len(slices), [res_pool],
                           res_extra, lambda i: (got_b[offs[i]:offs[i + 1]],
                                                 got_s[offs[i]:offs[i + 1]]))
        rec["cpu_baseline"] = cb
        check.update({"vs": "oracle (plain outputs), batched and graph outputs vs plain",
                      "tokens_checked": ntok, "tokens": ntok, "full": True,
                      "mismatches": bad})
        rec["parity"] = check
        rec["context"] = {"glibc_strtod": strtod_context(pool)}
    ctx.close()
    pctx.close()
    return rec


# ---------------------------------------------------------------------------
# served workload (config 5)
# ---------------------------------------------------------------------------

def serve_once(ffp, ctx, reqs, on_device, opts, dst=None):
    """Replays one arrival schedule against a fresh server (ffp_server_replay:
    submission at each arrival time and in-order collection run in native
    threads); returns per-request latency (ns), counts, batch sizes, the wall
    span and the server's statistics."""
    import numpy as np
    ptrs, sizes, dtypes, arrive = reqs
    srv = ffp.Server(ctx, **opts)
    try:
        base = ffp.clock_ns() + 20_000_000
        kw = {} if dst is None else dict(dst_values=dst[0], dst_status=dst[1],
                                         dst_capacity=dst[2])
        out = srv.replay(ptrs, sizes, 1 if on_device else 0, dtypes, base + arrive, **kw)
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
        raise AssertionError("arrival mismatch at %d requests, first %s"
                             % (off.size, off[:5].tolist()))
    span = (int(td.max()) - int(ta.min())) / 1e9
    # the two parts of a latency: waiting for a launch, and launch to done
    tl = out["t_launch_ns"].astype(np.int64)
    lat = (lat, tl - ta, td - tl)
    return lat, out["count"].astype(np.int64), out["batch_jobs"], span, st


def summarize(lat, counts, sizes, batch, span, st):
    import numpy as np
    lat, wait, run = lat
    q = np.percentile(lat / 1e3, [50, 99, 99.9])
    qw = np.percentile(wait / 1e3, [50, 99])
    qr = np.percentile(run / 1e3, [50, 99])
    return {
        "p50_us": round(float(q[0]), 1), "p99_us": round(float(q[1]), 1),
        "p999_us": round(float(q[2]), 1), "mean_us": round(float(lat.mean() / 1e3), 1),
        "GB/s": round(float(sizes.sum()) / span / 1e9, 3),
        "Mfloats/s": round(float(counts.sum()) / span / 1e6, 2),
        "span_s": round(span, 3), "batches": int(st["batches"]),
        "mean_batch": round(float(len(lat)) / max(1, st["batches"]), 2),
        "max_batch": int(st["max_batch_seen"]),
        "arena_peak_MB": round(st["arena_peak_bytes"] / 1e6, 1),
        "wait_p50_p99_us": [round(float(x), 1) for x in qw],
        "run_p50_p99_us": [round(float(x), 1) for x in qr],
    }


def served_rows(args, rates, extra_rates, requests, modes, parity_rate=None):
    """Config 5's arrivals at each rate against the servers in `modes`
    (batched, plain, batched_host_text); with parity_rate, the batched
    server's results at that rate are copied out by the replay and compared
    with the oracle.  Returns (rows, parity record or None, cpu_baseline)."""
    import numpy as np
    import torch
    from gen import workloads as W
    from paper_2101_11408_amd import ffp
    dev = torch.device("cuda", 0)
    t0 = time.time()
    hosts = [W.token_pool(55, 1_000_000, "mixed"), W.token_pool(56, 40_000, "hard")]
    log("pools: mixed %.1f MB, hard %.1f MB, built in %.1f s"
        % (len(hosts[0]) / 1e6, len(hosts[1]) / 1e6, time.time() - t0))
    pools = []
    for host in hosts:
        d = torch.frombuffer(bytearray(host), dtype=torch.uint8).to(dev)
        p = torch.empty(len(host), dtype=torch.uint8, pin_memory=True)
        p.copy_(torch.frombuffer(bytearray(host), dtype=torch.uint8))
        pools.append((d, p, len(host)))
    torch.cuda.synchronize()
    ctx = ffp.Context(0)
    budget = 32 << 30
    opts = {"batched": dict(hbm_budget_bytes=budget, max_batch_bytes=256 << 20,
                            streams=args.serve_streams, max_batch_jobs=1024,
                            use_graph=args.serve_graph, spin_us=args.serve_spin_us),
            "plain": dict(hbm_budget_bytes=budget, max_batch_bytes=256 << 20,
                          mode=ffp.FFP_SERVE_PLAIN, streams=1, spin_us=args.serve_spin_us)}
    rows, parity, cpu = [], None, None
    for ri, rate in enumerate(rates + extra_rates):
        t, sizes, is_f32, is_hard = W.config5_requests(5 + ri, rate, requests)
        rng = np.random.default_rng(500 + ri)
        which = is_hard.astype(np.int64)
        lim = np.array([pools[k][2] for k in which])
        sizes = np.minimum(sizes, lim)
        starts = (rng.random(len(sizes)) * (lim - sizes + 1)).astype(np.int64)
        dtypes = is_f32.astype(np.int64)
        arrive = (t * 1e9).astype(np.int64)
        row = {"rate_req_s": rate, "requests": len(sizes),
               "beyond_config": rate not in rates,
               "offered_GB/s": round(float(sizes.sum()) / float(t[-1]) / 1e9, 3),
               "binary32_share": round(float(is_f32.mean()), 3),
               "hard_share": round(float(is_hard.mean()), 4)}
        for name in modes:
            on_device = name != "batched_host_text"
            ptrs = [(pools[k][0] if on_device else pools[k][1]).data_ptr() + int(s)
                    for k, s in zip(which, starts)]
            dst = None
            if name == "batched" and rate == parity_rate:
                # outputs for every request, sized by its token count
                idx = [PoolIndex(h) for h in hosts]
                sl = [idx[k].slice(int(s), int(s) + int(n)) for k, s, n in zip(which, starts, sizes)]
                caps = np.array([(k1 - k0) + (h is not None) + (tt is not None)
                                 for k0, k1, h, tt in sl], dtype=np.int64)
                offs = np.concatenate([[0], np.cumsum(caps)])
                dv = torch.zeros(int(offs[-1]) + 1, dtype=torch.int64, device=dev)
                ds = torch.full((int(offs[-1]) + 1,), 255, dtype=torch.uint8, device=dev)
                # 8-byte slots; binary32 results are packed 4 bytes apart
                dst = ([dv.data_ptr() + 8 * int(o) for o in offs[:-1]],
                       [ds.data_ptr() + int(o) for o in offs[:-1]], caps)
            lat, counts, batch, span, st = serve_once(
                ffp, ctx, (ptrs, sizes, dtypes, arrive), on_device,
                opts["plain" if name == "plain" else "batched"], dst)
            row[name] = summarize(lat, counts, sizes, batch, span, st)
            log("rate %d %s: %s" % (rate, name, json.dumps(row[name])))
            if dst is not None:
                assert np.array_equal(counts, caps), "served token counts"
                got_v = dv.cpu().numpy().view(np.uint64)
                got_s = ds.cpu().numpy()
                fmts = ["f32" if d == 1 else "f64" for d in dtypes]
                # the oracle over both pools (every distinct token) and the
                # tokens cut at request ends, in both output formats
                extra = [x for k0, k1, h, tt in sl for x in (h, tt) if x is not None]
                pool_res = []
                for k, host in enumerate(hosts):
                    cb, rt, rx = cpu_baseline_leg(host, ["f64", "f32"], [] if k else extra,
                                                  what="the mixed request pool" if k == 0
                                                  else "the hard-case pool")
                    pool_res.append(rt)
                    if k == 0:
                        cpu, extra_res = cb, rx

                def got(i):
                    a, c = int(offs[i]), int(caps[i])
                    if fmts[i] == "f64":
                        return got_v[a:a + c], got_s[a:a + c]
                    # binary32 results sit 4 bytes apart from the slot's start
                    return got_v[a:a + (c + 1) // 2].view(np.uint32)[:c].astype(np.uint64), \
                        got_s[a:a + c]
                bad = slice_parity(sl, which.tolist(), fmts, pool_res, extra_res, got)
                parity = {"vs": "oracle", "rate_req_s": rate, "server": "batched",
                          "requests": len(sizes), "tokens_checked": int(caps.sum()),
                          "full": True, "mismatches": bad}
                del dv, ds
        rows.append(row)
    ctx.close()
    return rows, parity, cpu


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
    """Counter values of the matching kernels' dispatches, by kernel name."""
    import csv
    vals = {}
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] == counter and match(row["Kernel_Name"]):
                vals.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    if not vals:
        raise SystemExit("no %s rows for the kernel in %s" % (counter, csv_path))
    return vals


def _per_launch(vals):
    """Mean per dispatch of each kernel, summed over the kernels: a parse
    launch of 16 KiB tiles dispatches two instances (the one not needed for
    the call returns at once), and both count towards the launch."""
    return sum(sum(v) / len(v) for v in vals.values())


def reduce_traffic(workload, fetch_csv, write_csv, cal_fetch_csv, cal_write_csv, command):
    """profiles/traffic.json[workload] = HBM bytes per parse-kernel launch:
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch, averaged over dispatches,
    summed over the instances a launch dispatches), each scaled by bytes /
    counter of the calibration kernel."""
    is_parse = lambda n: "k_parse" in n
    is_cal = lambda n: "bitwise_not" in n or "BitwiseNot" in n
    f_k = _per_launch(_counter_rows(fetch_csv, "FETCH_SIZE", is_parse))
    w_k = _per_launch(_counter_rows(write_csv, "WRITE_SIZE", is_parse))
    f_c = _per_launch(_counter_rows(cal_fetch_csv, "FETCH_SIZE", is_cal))
    w_c = _per_launch(_counter_rows(cal_write_csv, "WRITE_SIZE", is_cal))
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
            lines.append("Schedule (the autotuner's choice, or --schedule): %s."
                         % rec["config"]["schedule"])
    name = "k_parse_%s.md" % workload
    with open(os.path.join(ROOT, "profiles", name), "w") as f:
        f.write("\n".join(lines) + "\n")
    return name




def run_served(args, workload):
    """Config 5 on its own: every rate, the three servers, parity at the
    highest configured rate."""
    rates = [int(r) for r in args.rates.split(",")]
    extra = [int(r) for r in args.extra_rates.split(",") if r]
    rows, parity, cpu = served_rows(args, rates, extra, args.requests,
                                    ["batched", "plain", "batched_host_text"],
                                    parity_rate=None if args.no_cpu_baseline else rates[-1])
    top = [r for r in rows if not r["beyond_config"]][-1]
    rec = base_record(args, top["batched"]["GB/s"], top["batched"]["p50_us"] / 1e3, workload, {
        "description": "served parse requests, Poisson open-loop arrivals at %s req/s, %d "
                       "requests per rate, sizes lognormal (median 64 KiB, sigma 1.5, 512 B - "
                       "8 MiB), 90%% binary64 / 10%% binary32, 1%% hard cases, 32 GiB HBM "
                       "budget; value = GB/s served by the continuous-batching server at the "
                       "highest rate (device-resident text); ms_per_step = its p50 latency"
                       % (args.rates, args.requests),
        "streams": args.serve_streams, "graph": bool(args.serve_graph),
        "dispatcher_spin_us": args.serve_spin_us,
        "parallelism": "single GPU"})
    rec["steps"] = args.requests
    rec["p50_us"] = top["batched"]["p50_us"]
    rec["p99_us"] = top["batched"]["p99_us"]
    rec["p999_us"] = top["batched"]["p999_us"]
    rec["serve"] = rows
    rec["roofline"] = None
    rec["roofline_note"] = ("served batches are small and latency-bound; the parse kernel's "
                            "HBM roofline is measured on config4u")
    rec["cpu_baseline"] = cpu
    if parity:
        rec["parity"] = parity
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--reps", type=int, default=100,
                    help="after the timed steps: calls timed one by one (min and median)")
    ap.add_argument("--spinup-ms", type=float, default=200.0,
                    help="untimed calls for this long before the warmup steps (GPU clock ramp)")
    ap.add_argument("--workload", default="config4u",
                    choices=["config1", "config2", "config3", "config4", "config4u",
                             "config5", "copycal", "jsondoc", "hexfloat", "csv"])
    ap.add_argument("--round", default="nearest", choices=sorted(ROUND_FLAGS),
                    help="plain workloads: rounding direction (FFP_ROUND_*)")
    ap.add_argument("--tokens", type=int, default=None)
    ap.add_argument("--nbuf", type=int, default=4096)
    ap.add_argument("--reduce", action="store_true",
                    help="plain workloads: also keep the min, max and count of the values")
    ap.add_argument("--out", default="f64", choices=["f64", "f32", "f16", "bf16"],
                    help="plain workloads: output format")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (cpu_baseline and parity)")
    ap.add_argument("--rates", default="2000,5000,10000,20000")
    ap.add_argument("--extra-rates", default="50000,100000",
                    help="served workload: rates beyond the configuration's range, "
                         "reported separately (saturation)")
    ap.add_argument("--requests", type=int, default=60_000,
                    help="served workload: requests per rate")
    ap.add_argument("--serve-requests", type=int, default=10_000,
                    help="default workload: requests per rate of its short served run "
                         "(0: none)")
    ap.add_argument("--serve-streams", type=int, default=2)
    ap.add_argument("--serve-graph", type=int, default=0)
    ap.add_argument("--serve-spin-us", type=int, default=200,
                    help="served workloads: the idle dispatcher polls this long before "
                         "sleeping (ffp_server_options.spin_us)")
    ap.add_argument("--schedule", default="",
                    help="batched workloads: tile_k,workgroups_per_cu instead of the autotuner")
    ap.add_argument("--profile", action="store_true",
                    help="only the timed batched or plain calls (for profiler runs)")
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
    if args.profile:
        args.no_cpu_baseline = True

    from gen import workloads as W

    wl = args.workload
    cpu = not args.no_cpu_baseline
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
                        cpu=cpu, flags=ROUND_FLAGS[args.round])
    elif wl == "config1":
        n = args.tokens or 100_000
        buf = W.config1(n=n)
        rec = run_plain(args, buf, n, out_name(wl, args.out, args.round),
                        "100k uniform [0,1) doubles, shortest digits, positional, one "
                        "%.2f MB buffer; %s" % (len(buf) / 1e6, OUT_NAMES[args.out]),
                        out_dtype=args.out, cpu=cpu, flags=ROUND_FLAGS[args.round])
    elif wl == "config3":
        n = args.tokens or 2_000_000
        t0 = time.time()
        buf = W.config3(n=n)
        log("generated %d bytes in %.1f s" % (len(buf), time.time() - t0))
        rec = run_plain(args, buf, n, out_name(wl, args.out, args.round),
                        "2M hard cases (midpoints +-1 in the last of 20-800 digits, "
                        "subnormals, overflow, integers to 2^64, sign/zero variants) in one "
                        "%.1f MB buffer; %s" % (len(buf) / 1e6, OUT_NAMES[args.out]),
                        out_dtype=args.out, cpu=cpu, flags=ROUND_FLAGS[args.round])
    elif wl == "config4":
        rec = run_buffers(args, "mixed", WORKLOAD_NAMES[wl])
    elif wl == "jsondoc":
        t0 = time.time()
        nfeat = (args.tokens or 10_000_000) // 2000
        doc = W.geojson_document(7, nfeat, 1000)
        ntok = nfeat * 2000  # every number of the document is a coordinate
        log("generated %d bytes in %.1f s" % (len(doc), time.time() - t0))
        rec = run_plain(args, doc, ntok, out_name(wl, args.out),
                        "GeoJSON-like document (%.1f MB): %d features of 1000 coordinate pairs "
                        "with 6-15 fraction digits, keys and strings around them; "
                        "FFP_JSON_DOCUMENT (numbers outside strings, JSON number grammar); %s"
                        % (len(doc) / 1e6, nfeat, OUT_NAMES[args.out]),
                        out_dtype=args.out, cpu=cpu, flags=0x40, expect_ok=ntok,
                        doc_split=b"]]}},")
    elif wl == "csv":
        t0 = time.time()
        rows = (args.tokens or 5_000_000) // 5
        table = W.csv_benchmark_table(8, rows)
        ntok = rows * 5  # five selected numeric columns, one token each
        log("generated %d bytes in %.1f s" % (len(table), time.time() - t0))
        rec = run_plain(args, table, ntok, out_name(wl, args.out),
                        "CSV table (%.1f MB): %d rows of 10 columns (id, word, two coordinates, "
                        "a uniform double, a %%.17e double, a flag word, a price, a quantity, a "
                        "word); FFP_CSV selecting the five decimal columns; %s"
                        % (len(table) / 1e6, rows, OUT_NAMES[args.out]),
                        out_dtype=args.out, cpu=cpu, delims=b",\n", flags=0x80,
                        expect_ok=ntok, csv_columns=W.CSV_BENCH_COLUMNS)
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
                        % (len(buf) / 1e6, OUT_NAMES[args.out]), out_dtype=args.out, cpu=cpu,
                        flags=8 | ROUND_FLAGS[args.round], expect_ok=n)
    elif wl == "config5":
        rec = run_served(args, WORKLOAD_NAMES[wl])
    elif wl == "copycal":
        rec = run_copycal(args)
    else:  # config4u: the HBM target run, with a short served run beside it
        rec = run_buffers(args, "uniform", WORKLOAD_NAMES[wl])
        if args.serve_requests and not args.profile:
            rates = [int(r) for r in args.rates.split(",")]
            rows, parity, _ = served_rows(args, rates, [], args.serve_requests,
                                          ["batched", "plain"],
                                          parity_rate=rates[-1] if cpu else None)
            top = rows[-1]
            rec["latency_us"] = {
                "what": "config 5 arrivals (%d requests per rate, text on the device): "
                        "continuous-batching server vs one launch per request"
                        % args.serve_requests,
                "rate_req_s": top["rate_req_s"],
                "batched": {k: top["batched"][k] for k in ("p50_us", "p99_us", "p999_us")},
                "plain": {k: top["plain"][k] for k in ("p50_us", "p99_us", "p999_us")}}
            rec["serve"] = rows
            if parity:
                rec["serve_parity"] = parity
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
