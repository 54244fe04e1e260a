"""Seeded synthetic inputs for modular matrix products.

This module holds the input generators shared by the tests, the benchmark
and the oracle's callers.  It contains none of the modular-product
arithmetic: only a counter-based pseudo-random generator, prime search and
the workload recipes.

The paper generates its matrices "randomly" without naming a distribution
(Section 4.1, the paragraph before the two benchmark scenarios); entries here
are uniform integers in [0, p), which is the natural reading for elements of
F_p.

Generator: SplitMix64 used as a counter-based generator.  Element ``i`` of a
stream with key ``K`` is ``mix64(K + (i + 1) * 0x9E3779B97F4A7C15)`` where
``mix64`` is the SplitMix64 finaliser (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  Uniform draws in [0, p) use
rejection: a 64-bit word ``r`` is accepted when ``r < floor(2^64 / p) * p`` and
mapped to ``r mod p``; rejected positions are redrawn from the counters that
follow the stream's first ``count`` counters, in order.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN_GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1
BASE_SEED = 0x260107508

_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64_scalar(z: int) -> int:
    """SplitMix64 finaliser on a Python int (mod 2^64)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> np.uint64(30))
    z = z * _M1
    z = z ^ (z >> np.uint64(27))
    z = z * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> int:
    """Key of an independent stream derived from (seed, stream id)."""
    return mix64_scalar(mix64_scalar(seed) ^ ((stream * GOLDEN_GAMMA) & MASK64))


def raw_u64(key: int, start: int, count: int) -> np.ndarray:
    """64-bit words for counters start .. start+count-1 of a stream."""
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(key) + idx * np.uint64(GOLDEN_GAMMA)
        return _mix64(z)


def uniform_mod(seed: int, stream: int, count: int, p: int) -> np.ndarray:
    """``count`` integers uniform in [0, p) as uint64 (rejection sampling)."""
    if p <= 0 or p > (1 << 63):
        raise ValueError("p out of range")
    key = stream_key(seed, stream)
    limit = ((1 << 64) // p) * p  # accept r < limit
    out = raw_u64(key, 0, count)
    pp = np.uint64(p)
    if limit == (1 << 64):
        return out % pp
    lim = np.uint64(limit)
    bad = np.nonzero(out >= lim)[0]
    nxt = count
    while bad.size:
        r = raw_u64(key, nxt, bad.size)
        nxt += bad.size
        ok = r < lim
        out[bad[ok]] = r[ok]
        bad = bad[~ok]
    return out % pp


def uniform_bits(seed: int, stream: int, count: int, bits: int) -> np.ndarray:
    """``count`` integers uniform in [0, 2^bits) as uint64 (bits <= 64)."""
    r = raw_u64(stream_key(seed, stream), 0, count)
    if bits >= 64:
        return r
    return r >> np.uint64(64 - bits)


def random_matrix(seed: int, stream: int, rows: int, cols: int, p: int) -> np.ndarray:
    """rows x cols uint64 matrix, row-major, entries uniform in [0, p)."""
    return uniform_mod(seed, stream, rows * cols, p).reshape(rows, cols)


# ---------------------------------------------------------------- primes

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin; exact for n < 3.3e24 with these bases."""
    if n < 2:
        return False
    for b in _MR_BASES:
        if n % b == 0:
            return n == b
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def prev_prime(x: int) -> int:
    """Largest prime strictly below x."""
    n = x - 1
    while n >= 2 and not is_prime(n):
        n -= 1
    if n < 2:
        raise ValueError("no prime below x")
    return n


def largest_prime_below_pow2(bits: int) -> int:
    return prev_prime(1 << bits)


def random_prime_of_bits(seed: int, stream: int, bits: int, avoid=()) -> int:
    """Largest prime below a random x in [2^(bits-1), 2^bits), not in ``avoid``."""
    key = stream_key(seed, stream)
    c = 0
    while True:
        r = int(raw_u64(key, c, 1)[0])
        c += 1
        x = (1 << (bits - 1)) + (r >> (64 - (bits - 1)) if bits > 1 else 0)
        q = prev_prime(max(x, 3))
        if q.bit_length() == bits and q not in avoid:
            return q


# ---------------------------------------------------------------- workloads


@dataclass
class Problem:
    """One modular product C = A B mod p with seeded uniform inputs."""

    m: int
    n: int
    k: int
    p: int
    seed: int = BASE_SEED
    u: int = 0
    v: int = 0
    fill: str = "uniform"  # "uniform" | "pmax" (all entries p - 1)
    tag: str = ""

    def a(self) -> np.ndarray:
        if self.fill == "pmax":
            return np.full((self.m, self.k), self.p - 1, dtype=np.uint64)
        return random_matrix(self.seed, 1, self.m, self.k, self.p)

    def b(self) -> np.ndarray:
        if self.fill == "pmax":
            return np.full((self.k, self.n), self.p - 1, dtype=np.uint64)
        return random_matrix(self.seed, 2, self.k, self.n, self.p)


def config_problems(index: int) -> list[Problem]:
    """The benchmark workloads, by index 1..5 (square, 36-bit, 50-bit, sweep, CRT)."""
    s = BASE_SEED + index
    if index == 1:
        return [Problem(512, 512, 512, largest_prime_below_pow2(25), s, 1, 1, tag="sq512_b25_uv11")]
    if index == 2:
        return [
            Problem(4096, 4096, 4096, largest_prime_below_pow2(36), s, 0, 0, tag="sq4096_b36"),
            Problem(4096, 4096, 4096, largest_prime_below_pow2(26), s, 1, 1, tag="sq4096_b26_uv11"),
        ]
    if index == 3:
        p = largest_prime_below_pow2(50)
        return [
            Problem(8192, 8192, 8192, p, s, 2, 2, tag="sq8192_b50_uv22"),
            Problem(8192, 8192, 8192, p, s, 2, 2, fill="pmax", tag="sq8192_b50_uv22_pmax"),
        ]
    if index == 4:
        out = []
        for b in (23, 31, 40, 52):
            p = largest_prime_below_pow2(b)
            out.append(Problem(16384, 16384, 256, p, s, tag=f"tall16384x256_b{b}"))
            out.append(Problem(512, 512, 131072, p, s, tag=f"inner512x131072_b{b}"))
        return out
    raise ValueError("config index 1..4 are single products; use crt_job() / serve_stream()")


def unbalanced_problem(bits: int) -> Problem:
    """The paper's second workload (Section 4.1): m = 10923, k = 32768, n = 32,
    the iterated product of block-Wiedemann; uniform entries at the largest
    prime below 2^bits."""
    return Problem(10923, 32, 32768, largest_prime_below_pow2(bits), BASE_SEED + 7,
                   tag=f"unbal10923x32768x32_b{bits}")


@dataclass
class CrtJob:
    """One integer pair A, B (entries < 2^bits) reduced against many primes."""

    m: int
    n: int
    k: int
    primes: list[int]
    bits: int = 60
    seed: int = BASE_SEED + 5

    def a(self) -> np.ndarray:
        return uniform_bits(self.seed, 1, self.m * self.k, self.bits).reshape(self.m, self.k)

    def b(self) -> np.ndarray:
        return uniform_bits(self.seed, 2, self.k * self.n, self.bits).reshape(self.k, self.n)


def crt_primes(seed: int = BASE_SEED + 5, count: int = 32) -> list[int]:
    """Distinct primes; the i-th has bitsize 31 + (i mod 20)."""
    out: list[int] = []
    for i in range(count):
        b = 31 + (i % 20)
        out.append(random_prime_of_bits(seed, 100 + i, b, avoid=out))
    return out


def crt_job(m: int = 2048, n: int = 2048, k: int = 2048, count: int = 32) -> CrtJob:
    return CrtJob(m, n, k, crt_primes(count=count))


@dataclass
class Request:
    t_arrival: float
    problem: Problem


def serve_stream(count: int, rate_hz: float, seed: int = BASE_SEED + 6,
                 dim_lo: int = 64, dim_hi: int = 4096, bits_lo: int = 20,
                 bits_hi: int = 52) -> list[Request]:
    """Poisson arrivals; m, n, k log-uniform in [dim_lo, dim_hi]; bitsize uniform."""
    key = stream_key(seed, 7)
    r = raw_u64(key, 0, 6 * count).astype(np.float64) / 2.0**64
    t = 0.0
    out = []
    lo, hi = math.log(dim_lo), math.log(dim_hi)
    for i in range(count):
        u0, u1, u2, u3, u4, u5 = r[6 * i: 6 * i + 6]
        t += -math.log(max(1.0 - u0, 1e-300)) / rate_hz
        m = int(round(math.exp(lo + (hi - lo) * u1)))
        n = int(round(math.exp(lo + (hi - lo) * u2)))
        k = int(round(math.exp(lo + (hi - lo) * u3)))
        b = bits_lo + min(int(u4 * (bits_hi - bits_lo + 1)), bits_hi - bits_lo)
        p = random_prime_of_bits(seed, 1000 + i, b)
        out.append(Request(t, Problem(m, n, k, p, seed=seed * 7919 + i, tag=f"req{i}")))
    return out
