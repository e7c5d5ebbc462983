"""Seeded synthetic operands (shared by the tests, the oracle checks and the
benchmark).  This module draws random bits and builds fixed bit patterns; it
contains none of the multiplication method's arithmetic.

Operands are little-endian ``uint64`` limb arrays of length ``L = ceil(n/64)``
with every bit at position >= n cleared.
"""
import numpy as np


def nlimbs(n_bits):
    return (int(n_bits) + 63) // 64


def mask_top(limbs, n_bits):
    """Clear bits >= n_bits in place and return the array."""
    L = nlimbs(n_bits)
    r = int(n_bits) - 64 * (L - 1)
    if L and r < 64:
        limbs[L - 1] &= np.uint64((1 << r) - 1)
    return limbs


def random_limbs(n_bits, seed):
    """Uniform random n-bit operand from numpy's PCG64 stream ``seed``."""
    L = nlimbs(n_bits)
    g = np.random.Generator(np.random.PCG64(seed))
    a = g.integers(0, np.iinfo(np.uint64).max, size=L, dtype=np.uint64, endpoint=True)
    return mask_top(a, n_bits)


def operand_pair(n_bits, tag):
    """The (u, v) pair used for workload ``tag``: u from stream 2*tag, v from
    stream 2*tag + 1."""
    return random_limbs(n_bits, 2 * tag), random_limbs(n_bits, 2 * tag + 1)


def all_ones(n_bits):
    L = nlimbs(n_bits)
    return mask_top(np.full(L, np.iinfo(np.uint64).max, dtype=np.uint64), n_bits)


def small(n_bits, value):
    """The integer ``value`` (< 2^64) as an n-bit operand."""
    a = np.zeros(nlimbs(n_bits), dtype=np.uint64)
    a[0] = np.uint64(value)
    return mask_top(a, n_bits)


def power_of_two(n_bits, e):
    a = np.zeros(nlimbs(n_bits), dtype=np.uint64)
    if e < n_bits:
        a[e // 64] = np.uint64(1) << np.uint64(e % 64)
    return a


def digit_pattern(n_bits, b, value, shift=0):
    """Operand whose b-bit fields at positions i*b - shift all equal ``value``
    (an adversarial pattern when value = 2^(b-1): every balanced digit sits at
    the edge of its range)."""
    L = nlimbs(n_bits)
    bits = np.zeros(64 * L + b, dtype=np.uint8)
    field = np.array([(value >> j) & 1 for j in range(b)], dtype=np.uint8)
    start = (-shift) % b
    for pos in range(start, n_bits, b):
        m = min(b, n_bits - pos)
        bits[pos:pos + m] = field[:m]
    packed = np.packbits(bits[:64 * L], bitorder="little")
    return mask_top(np.frombuffer(packed.tobytes(), dtype="<u8").astype(np.uint64), n_bits)


def serving_mix(count, seed, log2_lo=12, log2_hi=22):
    """Request sizes and kinds of the mixed serving workload: n log-uniform
    over [2^log2_lo, 2^log2_hi] bits, rounded to whole 64-bit limbs; kind
    uniform over lo / hi / full.  Returns a list of (kind, n_bits)."""
    g = np.random.Generator(np.random.PCG64(seed))
    e = g.uniform(log2_lo, log2_hi, size=count)
    n = np.maximum(1, np.rint(np.exp2(e) / 64.0)).astype(np.int64) * 64
    kinds = g.integers(0, 3, size=count)
    names = ("lo", "hi", "full")
    return [(names[k], int(x)) for k, x in zip(kinds, n)]


def poisson_arrivals(count, rate, seed):
    """Arrival times (seconds) of a Poisson process of the given rate:
    cumulative exponential inter-arrival gaps, the first arrival at 0."""
    g = np.random.Generator(np.random.PCG64(seed))
    gaps = g.exponential(1.0 / rate, size=count)
    gaps[0] = 0.0
    return np.cumsum(gaps)


def operand_slices(mix, seed):
    """Operands for a request mix without one array per request: one random
    limb pool as long as the largest request, and per request the offsets of
    its u and v windows in it (seeded).  Returns (pool, [(ou, ov)])."""
    Lmax = max(nlimbs(n) for _, n in mix)
    pool = random_limbs(64 * 2 * Lmax, seed)
    g = np.random.Generator(np.random.PCG64(seed + 1))
    offs = []
    for _, n in mix:
        L = nlimbs(n)
        offs.append((int(g.integers(0, 2 * Lmax - L + 1)), int(g.integers(0, 2 * Lmax - L + 1))))
    return pool, offs
