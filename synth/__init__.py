"""Seeded synthetic inputs shared by the oracle side and the device side.

This module only draws numbers.  It holds none of the arithmetic of the
loop-nest matmul or of the reduction, so the two implementations that are
compared in the tests can both take their operands from here without sharing
any of the code under test.

Every generator takes ``(seed, stream)`` and builds a fresh PCG64 generator
from ``SeedSequence([seed, stream])``, so each array has its own independent,
reproducible stream.  Value recipes follow the synthetic workloads that stand
in for the paper's matrix-multiplication benchmark (square row-major
``LEN*LEN`` operands, section "Matrix-Matrix Multiplication Example" and the
"Matrix Multiplication" paragraph of section 4.2) and for the reduction
clause (section 2.3, "Replacing the dummy OpenACC kernels region calls"):

* uniform[-1, 1] float32 as ``2*(u24 * 2**-24) - 1``: exact multiples of 2**-23;
* uniform[0, 1) float32 as ``u24 * 2**-24``: exact multiples of 2**-24, so a
  float64 serial sum of up to 2**28 of them is the exact real sum;
* integers uniform in ``[lo, hi]`` (inclusive) as int32;
* N(0, 1) times a per-row scale ``2**U`` with ``U ~ Uniform[-8, 8)``, drawn in
  float64 and rounded once to float32;
* sizes: LEN uniform over a list, ``n`` log-uniform over ``[a, b]``.
"""
from __future__ import annotations

import numpy as np

DEFAULT_SEED = 14121127

# Stream identifiers: one per logical array, so that e.g. A and B never share
# a stream and a change in one array's size does not shift the other's values.
STREAM_A = 1
STREAM_B = 2
STREAM_X = 3
STREAM_SIZES = 4
STREAM_ARRIVALS = 5


def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


def _u24(g: np.random.Generator, count: int) -> np.ndarray:
    # top 24 bits of 32-bit draws
    return (g.integers(0, 1 << 32, size=count, dtype=np.uint64) >> np.uint64(8)).astype(np.int64)


def uniform_pm1_f32(shape, seed: int, stream: int) -> np.ndarray:
    """uniform[-1, 1] as float32; every value is k * 2**-23 for an integer k."""
    count = int(np.prod(shape))
    u = _u24(rng(seed, stream), count).astype(np.float64) * 2.0 ** -24
    return (2.0 * u - 1.0).astype(np.float32).reshape(shape)


def uniform01_f32(n: int, seed: int, stream: int, chunk: int = 1 << 24) -> np.ndarray:
    """uniform[0, 1) as float32; every value is k * 2**-24, k < 2**24."""
    g = rng(seed, stream)
    out = np.empty(int(n), dtype=np.float32)
    for s in range(0, int(n), chunk):
        e = min(int(n), s + chunk)
        out[s:e] = (_u24(g, e - s).astype(np.float32) * np.float32(2.0 ** -24))
    return out


def int_uniform_i32(shape, lo: int, hi: int, seed: int, stream: int) -> np.ndarray:
    """Integers uniform in [lo, hi] inclusive, as int32."""
    g = rng(seed, stream)
    return g.integers(lo, hi + 1, size=shape, dtype=np.int64).astype(np.int32)


def full_range_i32(shape, seed: int, stream: int) -> np.ndarray:
    """Integers uniform over all of int32."""
    g = rng(seed, stream)
    return g.integers(-(1 << 31), 1 << 31, size=shape, dtype=np.int64).astype(np.int32)


def uniform_pm1_f64(n: int, seed: int, stream: int) -> np.ndarray:
    """uniform[-1, 1) as float64; every value is k * 2**-52 for an integer k."""
    g = rng(seed, stream)
    k = g.integers(-(1 << 52), 1 << 52, size=int(n), dtype=np.int64)
    return k.astype(np.float64) * 2.0 ** -52


def full_range_i64(n: int, seed: int, stream: int) -> np.ndarray:
    """Integers uniform over all of int64."""
    g = rng(seed, stream)
    return g.integers(-(1 << 63), (1 << 63) - 1, size=int(n), dtype=np.int64, endpoint=True)


def sparse_flags_i32(n: int, density: float, seed: int, stream: int) -> np.ndarray:
    """0/1 int32 flags, each 1 with probability `density` (a BFS frontier's
    "visit next" marks)."""
    g = rng(seed, stream)
    return (g.random(int(n)) < density).astype(np.int32)


def normal_rowscaled_f32(rows: int, cols: int, seed: int, stream: int,
                         umin: float = -8.0, umax: float = 8.0) -> np.ndarray:
    """N(0,1) * 2**U per row, U ~ Uniform[umin, umax), rounded once to float32."""
    g = rng(seed, stream)
    z = g.standard_normal((rows, cols))
    u = g.uniform(umin, umax, size=(rows, 1))
    return (z * np.exp2(u)).astype(np.float32)


def lens_uniform(count: int, choices, seed: int, stream: int = STREAM_SIZES) -> np.ndarray:
    g = rng(seed, stream)
    return np.asarray(choices, dtype=np.int64)[g.integers(0, len(choices), size=count)]


def log_uniform_int(count: int, lo: int, hi: int, seed: int, stream: int) -> np.ndarray:
    """floor(exp(U(ln lo, ln hi))), clipped to [lo, hi]."""
    g = rng(seed, stream)
    v = np.floor(np.exp(g.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)
    return np.clip(v, lo, hi)


def poisson_arrivals(count: int, rate_per_s: float, seed: int,
                     stream: int = STREAM_ARRIVALS) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    g = rng(seed, stream)
    return np.cumsum(g.exponential(1.0 / rate_per_s, size=count))
