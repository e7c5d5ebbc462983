"""Exact series coefficients of the ring maps (test infrastructure only).

Each function returns a ``fractions.Fraction`` computed from the binomial
definition printed in the paper, with eps = 2^-b:

* beta_{k,r}  = binom(-k/N, r) (-eps)^r                      (Section 3.2)
* alpha_{k,r} = k/(k+r) binom((k+r)/N, r) (-eps)^r, r >= 1   (Lemma on the
  coefficients of alpha, via Lagrange inversion); alpha_{k,0} = 1
* delta_{k,r} = binom(k/N, r) (-eps)^r                       (Section 4.2)
* gamma_{k,r} = k/(k+r) binom(-(k+r)/N, r) (-eps)^r, r >= 1  (Lemma on the
  coefficients of gamma); gamma_{k,0} = 1

``binom(y, r) = y (y-1) ... (y-r+1) / r!`` for rational y.
"""
from fractions import Fraction
from math import factorial


def binom(y, r):
    y = Fraction(y)
    p = Fraction(1)
    for j in range(r):
        p *= (y - j)
    return p / factorial(r)


def _eps_pow(b, r, sign):
    return Fraction(sign, 2 ** b) ** r


def beta(k, r, N, b):
    return binom(Fraction(-k, N), r) * _eps_pow(b, r, -1)


def alpha(k, r, N, b):
    if r == 0:
        return Fraction(1)
    return Fraction(k, k + r) * binom(Fraction(k + r, N), r) * _eps_pow(b, r, -1)


def delta(k, r, N, b):
    return binom(Fraction(k, N), r) * _eps_pow(b, r, -1)


def gamma(k, r, N, b):
    if r == 0:
        return Fraction(1)
    return Fraction(k, k + r) * binom(Fraction(-(k + r), N), r) * _eps_pow(b, r, -1)


def series_power(kind, k, N, b, terms):
    """First ``terms`` coefficients of z^-k f(z)^k for f in {alpha, beta,
    gamma, delta}, i.e. [f_{k,0}, ..., f_{k,terms-1}]."""
    f = {"alpha": alpha, "beta": beta, "gamma": gamma, "delta": delta}[kind]
    return [f(k, r, N, b) for r in range(terms)]
