"""ffp_parse_f64_noalloc (the entry point that allocates nothing, scratch in a
fixed device array) against ffp_parse_f64 on the same inputs, bit for bit:
two calls in a row, the second on a smaller input, both through the C-ABI;
and the size limit."""

import numpy as np
import pytest

from gen import workloads as W

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


def _text(seed, nmixed, nhard):
    rng = np.random.default_rng(seed)
    toks = W.mixed_tokens(rng, nmixed) + W.hard_tokens(rng, nhard)
    rng.shuffle(toks)
    return W.join_tokens(toks)


def test_noalloc_equals_parse_f64(ffpmod):
    dev = torch.device("cuda", 0)
    ctx = ffpmod.Context(0)
    try:
        # the second input is smaller and lies inside the first one's
        # footprint in the shared scratch
        for seed, nmixed, nhard, offset in ((91, 250_000, 3000, 0), (92, 30_000, 400, 3)):
            buf = _text(seed, nmixed, nhard)
            assert len(buf) <= ffpmod.NOALLOC_MAX_BYTES
            _log("case noalloc seed", seed, len(buf), "bytes")
            text = torch.frombuffer(bytearray(b"\n" * offset + buf), dtype=torch.uint8).to(dev)
            text = text[offset:]
            cap = len(buf) // 2 + 1
            out = {}
            for name in ("noalloc", "plain"):
                values = torch.full((cap,), -1.0, dtype=torch.float64, device=dev)
                status = torch.full((cap,), 255, dtype=torch.uint8, device=dev)
                count = torch.full((1,), -1, dtype=torch.int64, device=dev)
                if name == "noalloc":
                    ctx.parse_into_noalloc(text, values, status, count)
                else:
                    ctx.parse_into(text, values, status, count)
                torch.cuda.synchronize()
                assert ctx.last_device_error() == 0, name
                n = int(count.item())
                out[name] = (n, values[:n].view(torch.int64).cpu().numpy(),
                             status[:n].cpu().numpy())
            n0, v0, s0 = out["noalloc"]
            n1, v1, s1 = out["plain"]
            assert n0 == n1 == nmixed + nhard
            assert np.array_equal(v0, v1)
            assert np.array_equal(s0, s1)
            assert s0.max() <= 2  # every fallback decision landed
    finally:
        ctx.close()


def test_noalloc_rejects_larger_inputs(ffpmod):
    dev = torch.device("cuda", 0)
    ctx = ffpmod.Context(0)
    try:
        text = torch.full((ffpmod.NOALLOC_MAX_BYTES + 1,), ord("7"), dtype=torch.uint8,
                          device=dev)
        values = torch.empty(4, dtype=torch.float64, device=dev)
        status = torch.empty(4, dtype=torch.uint8, device=dev)
        count = torch.full((1,), -1, dtype=torch.int64, device=dev)
        with pytest.raises(ffpmod.FFPError) as e:
            ctx.parse_into_noalloc(text, values, status, count)
        assert e.value.code == ffpmod.FFP_E_SIZE
        torch.cuda.synchronize()
        assert int(count.item()) == -1  # nothing was queued
        # exactly the maximum is accepted: "25\n" repeated, plus "7" tokens
        n = ffpmod.NOALLOC_MAX_BYTES
        pat = torch.tensor(list(b"25\n"), dtype=torch.uint8, device=dev)
        full = pat.repeat(n // 3 + 1)[:n].contiguous()
        ntok = n // 3 + (1 if n % 3 else 0)
        values = torch.empty(ntok, dtype=torch.float64, device=dev)
        status = torch.full((ntok,), 255, dtype=torch.uint8, device=dev)
        ctx.parse_into_noalloc(full, values, status, count)
        torch.cuda.synchronize()
        assert int(count.item()) == ntok
        assert int(status.max().item()) == 0
        v = values.cpu().numpy()
        assert (v[:-1] == 25.0).all() and v[-1] in (2.0, 25.0)
    finally:
        ctx.close()
