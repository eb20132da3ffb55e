"""The oracle over many buffers at once, spread over worker processes (test
helper: the oracle itself is single-threaded Python)."""

import multiprocessing as mp
import os

from oracle import parse_buffer


def _one(args):
    buf, fmt, flags, delims = args
    bits, st = parse_buffer(buf, fmt, flags=flags, delims=delims)
    return bits, st


def parse_many(bufs, fmts, flags=0, delims=b"\n", workers=None):
    """[(bits, status)] of parse_buffer for every (buffer, format) pair."""
    jobs = [(b, f, flags, delims) for b, f in zip(bufs, fmts)]
    n = workers or max(1, min(16, os.cpu_count() or 1))
    if n == 1 or len(jobs) < 8:
        return [_one(j) for j in jobs]
    with mp.get_context("fork").Pool(n) as pool:
        return pool.map(_one, jobs, chunksize=max(1, len(jobs) // (4 * n)))
