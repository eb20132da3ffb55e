"""Seeded synthetic inputs shared by the tests and the benchmark.

Holds no parsing arithmetic: it only prints numbers to text.
"""

from .workloads import (  # noqa: F401
    INVALID_EXAMPLES,
    config1,
    config2,
    config3,
    config4_sizes,
    config5_requests,
    coordinates,
    hard_tokens,
    join_tokens,
    mixed_tokens,
    random_bits_e17,
    slice_plan,
    token_pool,
    uniform_shortest,
)
