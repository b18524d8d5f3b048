"""The multiply-high division of the block decode (round-up method of
Granlund and Montgomery): for 1 <= d < 2^31 and 0 <= n < 2^31, with
l = ceil(log2 d) and m = ceil(2^(32+l) / d) - 2^32,
(mulhi(n, m) + n) >> l equals n // d.  Checked by brute force on small
divisors and numerators and on the extremes of both ranges (the kernels
decode block indexes with it, so a wrong quotient would misplace tiles)."""
import numpy as np


def make(d):
    l = 0
    while (1 << l) < d:
        l += 1
    return ((1 << (32 + l)) + d - 1) // d - (1 << 32), l


def fdiv(n, m, l):
    return ((n * m >> 32) + n) >> l


def test_fast_division_matches_integer_division():
    rng = np.random.default_rng(0)
    ns = np.concatenate([np.arange(0, 5000), rng.integers(0, 2 ** 31, 20000),
                         np.arange(2 ** 31 - 3000, 2 ** 31)]).astype(object)
    ds = list(range(1, 300)) + [2 ** k for k in range(31)] + [2 ** k + 1 for k in range(1, 31)] \
        + [2 ** k - 1 for k in range(2, 32)] + [int(x) for x in rng.integers(1, 2 ** 31, 200)]
    for d in ds:
        m, l = make(d)
        assert 0 <= m < 2 ** 32
        q = np.array([fdiv(int(n), m, l) for n in ns[:: max(1, len(ns) // 4000)]], dtype=object)
        ref = np.array([int(n) // d for n in ns[:: max(1, len(ns) // 4000)]], dtype=object)
        assert (q == ref).all(), d
