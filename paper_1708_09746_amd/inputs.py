"""Seeded synthetic workloads (no arithmetic of the multiplication method).

All inputs are drawn from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: output i of stream `seed` is mix(seed + (i + 1) * GAMMA).  Both the
tests (for the oracle and the GPU path) and the benchmark draw from here, so
the same seed gives the same polynomial everywhere.

Polynomials are packed little-endian into uint64 words (bit i -> word i // 64,
bit i % 64); bits at and above the length are zero and the top bit (length-1)
is forced to 1 so that the degree is exact.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Seeds of the configured workloads.
SEEDS = {
    "c1": (0x16A, 0x16B),  # 2^16 x 2^16 bits
    "c2": (0x20A, 0x20B),  # 2^20 x 2^20 bits
    "c3a": (0x28A, 0x28B),  # 2^28 x 2^28 bits
    "c3b": (0x29A, 0x29B),  # 2^29 x 2^29 bits
}
BATCH_LEN_SEED = 0x4096
BATCH_OPERAND_BASE = 0x4000_0000
SERVE_LEN_SEED = 0x5000
SERVE_OPERAND_BASE = 0x5000_0000
# Timing streams of many requests take operands as windows of one pool
# (stream SERVE_POOL_SEED) at offsets drawn from stream SERVE_POOL_SEED + 1.
SERVE_POOL_SEED = 0x5EED_0000


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Outputs offset .. offset+count-1 of the SplitMix64 stream `seed`."""
    with np.errstate(over="ignore"):
        i = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def words_for(nbits: int) -> int:
    return (nbits + 63) // 64


def random_poly(seed: int, nbits: int, force_top: bool = True) -> np.ndarray:
    """A dense uniform polynomial of exactly nbits bits (uint64 words)."""
    nw = words_for(nbits)
    if nw == 0:
        return np.zeros(0, dtype=np.uint64)
    w = splitmix64(seed, nw)
    r = nbits % 64
    if r:
        w[-1] &= np.uint64((1 << r) - 1)
    if force_top:
        w[-1] |= np.uint64(1 << ((nbits - 1) % 64))
    return w


def uniform01(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of each output."""
    z = splitmix64(seed, count, offset)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def log_uniform_lengths(seed: int, count: int, lo_log2: float, hi_log2: float) -> np.ndarray:
    """floor(2^u) with u ~ U[lo, hi] (one draw per length)."""
    u = lo_log2 + (hi_log2 - lo_log2) * uniform01(seed, count)
    return np.floor(np.exp2(u)).astype(np.int64)


def batch_workload(njobs: int = 4096, lo_log2: float = 12, hi_log2: float = 20):
    """Batched products: per job (na_bits, nb_bits, seed_a, seed_b)."""
    lens = log_uniform_lengths(BATCH_LEN_SEED, 2 * njobs, lo_log2, hi_log2)
    jobs = []
    for j in range(njobs):
        jobs.append((int(lens[2 * j]), int(lens[2 * j + 1]),
                     BATCH_OPERAND_BASE + 2 * j, BATCH_OPERAND_BASE + 2 * j + 1))
    return jobs


def serve_workload(nreq: int, rate_index: int = 0, lo_log2: float = 10, hi_log2: float = 24):
    """Serving requests: per request (na_bits, nb_bits, seed_a, seed_b, u)
    where u in [0,1) is the uniform draw for its exponential inter-arrival gap
    (gap = -ln(1-u) / rate, applied by the caller for the chosen rate)."""
    seed = SERVE_LEN_SEED + rate_index
    lens = log_uniform_lengths(seed, 2 * nreq, lo_log2, hi_log2)
    gaps = uniform01(seed, nreq, offset=2 * nreq)
    out = []
    for r in range(nreq):
        out.append((int(lens[2 * r]), int(lens[2 * r + 1]),
                    SERVE_OPERAND_BASE + 2 * r, SERVE_OPERAND_BASE + 2 * r + 1, float(gaps[r])))
    return out
