"""Host-side helpers of bench.py: the reduction check against the oracle's
values, the per-launch sum of counter rows and the mismatch count (no GPU)."""

import importlib.util
import os
import struct

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test",
                                                  os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def f64(x):
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def test_expected_minmax_orders_by_value_and_skips_nan_and_errors(bench):
    bits = [f64(1.5), f64(-0.0), f64(0.0), f64(-2.0), f64(float("nan")), f64(7.0)]
    status = [0, 0, 0, 0, 0, 1]  # 7.0 has an error status: left out
    assert bench.expected_minmax(bits, status, "f64") == (f64(-2.0), f64(1.5), 4)


def test_expected_minmax_signed_zeros(bench):
    # -0 orders before +0: the minimum of {+0, -0} is -0, the maximum +0
    assert bench.expected_minmax([f64(0.0), f64(-0.0)], [0, 0], "f64") == \
        (f64(-0.0), f64(0.0), 2)
    assert bench.expected_minmax([f64(-0.0)], [0], "f64") == (f64(-0.0), f64(-0.0), 1)
    assert bench.expected_minmax([f64(0.0)], [0], "f64") == (0, 0, 1)


def test_expected_minmax_empty_sets_give_quiet_nan(bench):
    assert bench.expected_minmax([], [], "f64") == (0x7FF8000000000000, 0x7FF8000000000000, 0)
    nan_only = [f64(float("nan"))]
    assert bench.expected_minmax(nan_only, [0], "f64")[2] == 0
    assert bench.expected_minmax([], [], "f32")[:2] == (0x7FC00000, 0x7FC00000)
    assert bench.expected_minmax([], [], "f16")[:2] == (0x7E00, 0x7E00)
    assert bench.expected_minmax([], [], "bf16")[:2] == (0x7FC0, 0x7FC0)


def test_expected_minmax_narrow_formats(bench):
    # binary16: 1.0 = 0x3C00, -0 = 0x8000, -1.0 = 0xBC00, 65504 = 0x7BFF
    assert bench.expected_minmax([0x3C00, 0x8000, 0xBC00, 0x7BFF], [0] * 4, "f16") == \
        (0xBC00, 0x7BFF, 4)
    # bfloat16: the upper half of the binary32 encoding
    one, minus_three = 0x3F80, 0xC040
    assert bench.expected_minmax([one, minus_three], [0, 0], "bf16") == (minus_three, one, 2)
    # binary32
    b32 = lambda x: struct.unpack("<I", struct.pack("<f", x))[0]
    vals = [b32(3.5), b32(-1e-30), b32(2.0)]
    assert bench.expected_minmax(vals, [0, 0, 0], "f32") == (b32(-1e-30), b32(3.5), 3)


def test_expected_minmax_matches_numpy_on_random_values(bench):
    rng = np.random.default_rng(5)
    x = rng.standard_normal(5000) * 10.0 ** rng.integers(-30, 30, 5000)
    bits = x.view(np.uint64)
    status = (rng.random(5000) < 0.9).astype(np.uint8) ^ 1  # about 10% errors
    keep = status == 0
    mn, mx, n = bench.expected_minmax(bits, status, "f64")
    assert n == int(keep.sum())
    assert mn == int(bits[keep][np.argmin(x[keep])])
    assert mx == int(bits[keep][np.argmax(x[keep])])


def test_per_launch_sums_the_instances_of_a_launch(bench):
    # a 16 KiB-tile launch dispatches the plain instance and its dense twin
    vals = {"k_parse<4, true, false, 0>": [100.0, 102.0], "k_parse<4, true, false, 5>": [1.0, 3.0]}
    assert bench._per_launch(vals) == pytest.approx(101.0 + 2.0)


def test_count_mismatches(bench):
    a = np.array([1, 2, 3], dtype=np.uint64)
    s = np.array([0, 0, 1], dtype=np.uint8)
    assert bench.count_mismatches(a, s, a.copy(), s.copy()) == 0
    b = a.copy()
    b[1] = 7
    t = s.copy()
    t[0] = 2
    assert bench.count_mismatches(a, s, b, t) == 2
    assert bench.count_mismatches(a[:2], s[:2], a, s) == 3
