"""Pins for the C oracle (plain definition of the full, low and high product,
Section 1).  Everything here runs on the CPU.

The oracle is checked against CPython's own integer multiplication (an
independent implementation), by brute force on tiny operands, and against the
closed forms of the edge cases."""
import random

import numpy as np
import pytest

import oracle
from paper_1703_00640_amd import inputs


def _py(u, v, n):
    uv = u * v
    return uv, uv % (1 << n), uv >> n, (uv % (1 << n)) != 0


def _check(u, v, n, threads=1):
    L = oracle.nlimbs(n)
    U, V = oracle.from_int(u, L), oracle.from_int(v, L)
    full, lo, q, nz = _py(u, v, n)
    assert oracle.to_int(oracle.mul_full(U, V, n, threads)) == full
    assert oracle.to_int(oracle.mul_lo(U, V, n, threads)) == lo
    qq, nnz = oracle.mul_hi(U, V, n, threads)
    assert oracle.to_int(qq) == q and nnz == nz


@pytest.mark.parametrize("n", range(1, 8))
def test_brute_force_all_pairs(n):
    for u in range(1 << n):
        for v in range(1 << n):
            _check(u, v, n)


def test_brute_force_n8_sampled():
    rng = random.Random(8)
    for _ in range(3000):
        _check(rng.getrandbits(8), rng.getrandbits(8), 8)


@pytest.mark.parametrize("n", [63, 64, 65, 127, 128, 129, 1000, 2047, 2048, 2049,
                               4096, 64 * 33 + 5, 64 * 97, 65536, 100003])
def test_random_against_cpython(n):
    rng = random.Random(n)
    for _ in range(3):
        _check(rng.getrandbits(n), rng.getrandbits(n), n)


def test_large_threaded_against_cpython():
    n = 1 << 20
    rng = random.Random(20)
    u, v = rng.getrandbits(n), rng.getrandbits(n)
    _check(u, v, n, threads=4)


@pytest.mark.parametrize("L", [31, 32, 33, 64, 65, 99, 130, 257])
def test_karatsuba_matches_schoolbook(L):
    g = np.random.Generator(np.random.PCG64(L))
    u = g.integers(0, 2 ** 64 - 1, size=L, dtype=np.uint64, endpoint=True)
    v = g.integers(0, 2 ** 64 - 1, size=L, dtype=np.uint64, endpoint=True)
    assert np.array_equal(oracle.mul_full(u, v, 64 * L), oracle.mul_school(u, v))


def test_bits_above_n_are_ignored():
    n = 200
    L = oracle.nlimbs(n)
    u = inputs.random_limbs(n, 1)
    v = inputs.random_limbs(n, 2)
    u2, v2 = u.copy(), v.copy()
    u2[-1] |= np.uint64(0xFF) << np.uint64(56)   # garbage above bit 200
    v2[-1] |= np.uint64(1) << np.uint64(63)
    assert np.array_equal(oracle.mul_full(u, v, n), oracle.mul_full(u2, v2, n))
    assert L == 4


@pytest.mark.parametrize("n", [1, 5, 64, 100, 1024, 4097])
def test_edge_closed_forms(n):
    """All-ones, 2^n-1 times 1, powers of two and zero (spec edge set)."""
    L = oracle.nlimbs(n)
    ones = inputs.all_ones(n)
    one = inputs.small(n, 1)
    zero = np.zeros(L, dtype=np.uint64)
    # (2^n-1)^2 = 2^n (2^n - 2) + 1: lo = 1, hi in {2^n - 2, 2^n - 1}
    assert oracle.to_int(oracle.mul_lo(ones, ones, n)) == 1
    q, nz = oracle.mul_hi(ones, ones, n)
    assert oracle.to_int(q) == (1 << n) - 2 and nz
    # (2^n-1) * 1: lo = 2^n - 1, hi in {0, 1}
    assert oracle.to_int(oracle.mul_lo(ones, one, n)) == (1 << n) - 1
    q, nz = oracle.mul_hi(ones, one, n)
    assert oracle.to_int(q) == 0 and nz == (n >= 1)
    # zero
    assert oracle.to_int(oracle.mul_lo(zero, ones, n)) == 0
    q, nz = oracle.mul_hi(zero, ones, n)
    assert oracle.to_int(q) == 0 and not nz
    # powers of two 2^a 2^c
    for a, c in [(0, 0), (n - 1, 0), (n - 1, n - 1), (n // 2, n // 3), (n - 1, 1)]:
        if a >= n or c >= n:
            continue
        pa, pc = inputs.power_of_two(n, a), inputs.power_of_two(n, c)
        e = a + c
        lo = oracle.to_int(oracle.mul_lo(pa, pc, n))
        assert lo == ((1 << e) if e < n else 0)
        q, nz = oracle.mul_hi(pa, pc, n)
        if e >= n:
            assert oracle.to_int(q) == 1 << (e - n) and not nz
        else:
            assert oracle.to_int(q) == 0 and nz


def test_invariants_random():
    """w_lo = uv mod 2^n and |uv - 2^n w_hi| < 2^n for both allowed values."""
    rng = random.Random(5)
    for n in (77, 640, 5000):
        u, v = rng.getrandbits(n), rng.getrandbits(n)
        L = oracle.nlimbs(n)
        U, V = oracle.from_int(u, L), oracle.from_int(v, L)
        lo = oracle.to_int(oracle.mul_lo(U, V, n))
        assert (lo - u * v) % (1 << n) == 0 and 0 <= lo < (1 << n)
        q, nz = oracle.mul_hi(U, V, n)
        for w in ([oracle.to_int(q)] + ([oracle.to_int(q) + 1] if nz else [])):
            assert abs(u * v - (w << n)) < (1 << n)
        assert oracle.hi_accepts(q, q, nz)


@pytest.mark.parametrize("L", [1, 2, 3, 17, 1000])
def test_residue_against_python_int(L):
    """residue(x, p) is x mod p by Python's own integer division, for random
    limb arrays (top limbs with every bit pattern) and moduli of different
    shapes: a Mersenne prime, a decimal prime, a tiny prime, an even number
    and the largest allowed modulus."""
    g = np.random.Generator(np.random.PCG64(4242 + L))
    for trial in range(4):
        x = g.integers(0, np.iinfo(np.uint64).max, size=L, dtype=np.uint64, endpoint=True)
        if trial == 1:
            x[-1] = np.uint64(0xFFFFFFFFFFFFFFFF)
        if trial == 2:
            x[:] = np.uint64(0xFFFFFFFFFFFFFFFF)
        xi = oracle.to_int(x)
        for p in (2 ** 61 - 1, 10 ** 9 + 7, 3, 2, 2 ** 62 + 6, 2 ** 63 - 25):
            assert oracle.residue(x, p) == xi % p, (L, trial, p)


def test_residue_check():
    n = 1 << 14
    u, v = inputs.operand_pair(n, 3)
    f = oracle.mul_full(u, v, n)
    for p in (2 ** 61 - 1, 1000000007, 2 ** 31 - 1):
        assert oracle.residue(f, p) == (oracle.residue(u, p) * oracle.residue(v, p)) % p
