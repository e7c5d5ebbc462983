"""Pins of the oracle's modular multiplication and Barrett reciprocal (CPU).

The oracle's mulmod is the plain definition (full product, then the
remainder of integer division).  It is pinned by facts that do not restate
that formula: Fermat's little theorem on Mersenne primes (a^(p-1) = 1 and
a^p = a mod p, by square-and-multiply through the oracle's mulmod only),
closed forms ((m-1)^2 = 1, a * 1 = a, 2^(n-1) * 2 = 1 mod 2^n - 1), and the
floor inequalities that define the reciprocal.
"""
import numpy as np
import pytest

import oracle
from paper_1703_00640_amd import inputs


def _modulus(n, seed):
    """Random n-bit modulus with the top bit set, not a power of two."""
    m = oracle.to_int(inputs.random_limbs(n, seed)) | (1 << (n - 1)) | 1
    return oracle.from_int(m, oracle.nlimbs(n))


def _pow_chain(a, e, m, n):
    """a^e mod m by square-and-multiply through oracle.mulmod."""
    L = oracle.nlimbs(n)
    r = oracle.from_int(1, L)
    base = a.copy()
    for bit in bin(e)[2:]:
        r = oracle.mulmod(r, r, m, n)
        if bit == "1":
            r = oracle.mulmod(r, base, m, n)
    return r


@pytest.mark.parametrize("n", [61, 127, 521])
def test_fermat_on_mersenne_primes(n):
    p = (1 << n) - 1  # 2^61-1, 2^127-1, 2^521-1 are prime
    L = oracle.nlimbs(n)
    m = oracle.from_int(p, L)
    for seed in (1, 2):
        a = oracle.from_int(oracle.to_int(inputs.random_limbs(n, seed)) % p, L)
        assert oracle.to_int(_pow_chain(a, p - 1, m, n)) == 1
        assert np.array_equal(_pow_chain(a, p, m, n), a)


@pytest.mark.parametrize("n", [2, 3, 64, 65, 200, 4099])
def test_closed_forms(n):
    L = oracle.nlimbs(n)
    m = _modulus(n, 7 + n)
    M = oracle.to_int(m)
    mm1 = oracle.from_int(M - 1, L)
    assert oracle.to_int(oracle.mulmod(mm1, mm1, m, n)) == 1
    a = oracle.from_int(oracle.to_int(inputs.random_limbs(n, n)) % M, L)
    assert np.array_equal(oracle.mulmod(a, oracle.from_int(1, L), m, n), a)
    assert oracle.to_int(oracle.mulmod(a, oracle.from_int(0, L), m, n)) == 0
    mers = oracle.from_int((1 << n) - 1, L)
    half = oracle.from_int(1 << (n - 1), L)
    assert oracle.to_int(oracle.mulmod(half, oracle.from_int(2, L), mers, n)) == 1


@pytest.mark.parametrize("n", [2, 64, 65, 1000, 1 << 14])
def test_barrett_reciprocal_is_the_floor(n):
    m = _modulus(n, 3 * n)
    mu = oracle.barrett_mu(m, n)
    assert len(mu) == oracle.nlimbs(n + 1)
    # mu m <= 2^(2n) < (mu + 1) m, products through the oracle's schoolbook
    lo = oracle.to_int(oracle.mul_school(mu, m))
    hi = oracle.to_int(oracle.mul_school(oracle.from_int(oracle.to_int(mu) + 1, len(mu)), m))
    assert lo <= (1 << (2 * n)) < hi
    assert (1 << n) < oracle.to_int(mu) < (1 << (n + 1))
