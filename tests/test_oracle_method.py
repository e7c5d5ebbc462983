"""Pins for the FP64 model of the paper's algorithms (oracle/method.py) and
the exact coefficient generators (oracle/coeffs.py).  CPU only.

Each test ties the model to something it does not compute itself: numbers
printed in the paper, identities the paper proves, exact rational arithmetic,
or CPython's integer product."""
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import coeffs, method as m

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _eval_poly_expr(expr, N):
    # the fixture holds arithmetic in N only; evaluate it with exact rationals
    allowed = set("N0123456789+-*/() ")
    assert set(expr) <= allowed, expr
    return eval(expr, {"__builtins__": {}}, {"N": Fraction(N)})


# ----------------------------------------------------- series coefficients


@pytest.mark.parametrize("N", [3, 7, 12, 1000])
def test_printed_first_terms(N):
    """Printed expansions of beta, alpha, delta, gamma (k = 1)."""
    b = 5
    eps = Fraction(1, 2 ** b)
    for kind, r, expr in _golden("printed_series_terms.txt"):
        r = int(r)
        printed = _eval_poly_expr(expr, N) * eps ** r
        exact = getattr(coeffs, kind)(1, r, N, b)
        assert exact == printed, (kind, r)
        fl = getattr(m, kind + "_c")(1, r, N, b)
        assert abs(fl - float(printed)) <= 4e-16 * abs(float(printed))


@pytest.mark.parametrize("N", [3, 4, 12, 100])
def test_coefficient_bounds(N):
    """|alpha|,|beta|,|delta| <= 2^-rb and |gamma| <= 2^-r(b-2) for 0 <= k < N."""
    b = 4
    for k in range(N):
        for r in range(8):
            assert abs(coeffs.alpha(k, r, N, b)) <= Fraction(1, 2 ** (r * b))
            assert abs(coeffs.beta(k, r, N, b)) <= Fraction(1, 2 ** (r * b))
            assert abs(coeffs.delta(k, r, N, b)) <= Fraction(1, 2 ** (r * b))
            assert abs(coeffs.gamma(k, r, N, b)) <= Fraction(1, 2 ** (r * (b - 2)))


def test_lagrange_identity():
    """n alpha_{k,n-k} = k beta_{-n,n-k} (proof of the alpha-coefficient Lemma)."""
    N, b = 7, 4
    for k in range(0, 6):
        for nn in range(k + 1, k + 7):
            assert nn * coeffs.alpha(k, nn - k, N, b) == k * coeffs.beta(-nn, nn - k, N, b)


def _compose(f, g, terms):
    """f(g(z)) for power series f = sum f_i z^(i+1), g = sum g_i z^(i+1)."""
    res = [Fraction(0)] * (terms + 1)
    gp = [Fraction(0)] * (terms + 1)
    gp[0] = Fraction(1)
    for i in range(terms):
        new = [Fraction(0)] * (terms + 1)
        for a, ca in enumerate(gp):
            if ca == 0:
                continue
            for j, cg in enumerate(g):
                if a + j + 1 <= terms:
                    new[a + j + 1] += ca * cg
        gp = new
        for d, c in enumerate(gp):
            res[d] += f[i] * c
    return res


@pytest.mark.parametrize("pair", [("alpha", "beta"), ("gamma", "delta")])
def test_formal_inverses(pair):
    """alpha(beta(z)) = z = beta(alpha(z)) and gamma(delta(z)) = z formally."""
    N, b, T = 5, 4, 7
    f = coeffs.series_power(pair[0], 1, N, b, T)
    g = coeffs.series_power(pair[1], 1, N, b, T)
    for a, c in ((f, g), (g, f)):
        comp = _compose(a, c, T)
        assert comp[1] == 1 and all(x == 0 for x in comp[2:]), comp


def test_figure_roots():
    """Roots of A(X) = X^12 + X/2 - 1 and B(X) = X^13 - 2X^12 + 2 as drawn in
    the figures (N = 12, b = 1); beta maps the roots of A onto 12th roots of
    unity (Lemma on beta)."""
    rows = _golden("figure_roots.txt")
    N, b = 12, 1
    A = np.zeros(N + 1); A[0] = 1.0; A[N - 1] = 2.0 ** -b; A[N] = -1.0    # highest first
    B = np.zeros(N + 2); B[0] = 1.0; B[1] = -(2.0 ** b); B[N + 1] = 2.0 ** b
    for name, poly in (("A", A), ("B", B)):
        printed = np.array([complex(float(x), float(y)) for p, x, y in rows if p == name])
        roots = np.roots(poly)
        assert len(roots) == len(printed)
        for z in printed:
            assert np.min(np.abs(roots - z)) < 1.5e-3
    for z in np.roots(A):
        beta_z = z * (1 - 2.0 ** -b * z) ** (-1.0 / N)
        assert abs(beta_z ** N - 1) < 1e-9


# ----------------------------------------------------- cancellation trick


def _poly_rem(P, D):
    """Exact remainder of P by monic D (Fraction coefficient lists, low first)."""
    P = list(P)
    n = len(D) - 1
    for d in range(len(P) - 1, n - 1, -1):
        c = P[d]
        if c:
            for j in range(n + 1):
                P[d - n + j] -= c * D[j]
    return P[:n]


@pytest.mark.parametrize("N", [3, 4, 9])
def test_low_cancellation_exact(N):
    """Prop. low-cancel: 2^b (W mod A) is integral, evaluates to
    sum_(i<N) w_i 2^(ib) at 2^b, and equals the closed form used for c_i."""
    b = 5
    rng = random.Random(N)
    W = [rng.randint(-2 ** 12, 2 ** 12) for _ in range(2 * N - 1)]
    A = [Fraction(-1), Fraction(1, 2 ** b)] + [Fraction(0)] * (N - 2) + [Fraction(1)]
    L = _poly_rem([Fraction(w) for w in W], A)
    scaled = [x * 2 ** b for x in L]
    assert all(x.denominator == 1 for x in scaled)
    assert sum(x * Fraction(2 ** b) ** i for i, x in enumerate(L)) == sum(
        W[i] * 2 ** (i * b) for i in range(N))
    assert [int(x) for x in scaled] == m.low_coeffs_exact(W, N, b)


@pytest.mark.parametrize("N", [3, 4, 9])
def test_high_cancellation_exact(N):
    """Prop. high-cancel: H = (1 - 2^-b X) W mod B has 2^b H integral and
    H(2^b) = sum_(i=N)^(2N) w_i 2^((i-N) b); matches the closed form."""
    b = 5
    rng = random.Random(100 + N)
    W = [rng.randint(-2 ** 12, 2 ** 12) for _ in range(2 * N + 1)]
    eps = Fraction(1, 2 ** b)
    P = [Fraction(0)] * (2 * N + 2)
    for i, w in enumerate(W):
        P[i] += w
        P[i + 1] -= eps * w
    Bm = [Fraction(2 ** b)] + [Fraction(0)] * (N - 1) + [Fraction(-(2 ** b)), Fraction(1)]
    H = _poly_rem(P, Bm)
    scaled = [x * 2 ** b for x in H]
    assert all(x.denominator == 1 for x in scaled)
    assert sum(x * Fraction(2 ** b) ** i for i, x in enumerate(H)) == sum(
        W[i] * 2 ** ((i - N) * b) for i in range(N, 2 * N + 1))
    assert [int(x) for x in scaled] == m.high_coeffs_exact(W, N, b)


# ------------------------------------------------------ ring isomorphisms


def test_alpha_beta_are_inverse_ring_maps():
    """beta* alpha* F = F and alpha*(F G mod A) = alpha*F alpha*G (Cor. on
    alpha*, beta* being mutually inverse ring isomorphisms)."""
    N, b, lam = 24, 8, 8
    g = np.random.Generator(np.random.PCG64(7))
    F = g.uniform(-1, 1, N)
    G = g.uniform(-1, 1, N)
    back = m.beta_star(m.alpha_star(F, N, b, lam), N, b, lam)
    assert np.max(np.abs(back - F)) < 1e-14
    FG = m.reduce_mod_A(np.convolve(F, G), N, b)
    lhs = m.alpha_star(FG, N, b, lam)
    rhs = m.convolution(m.alpha_star(F, N, b, lam), m.alpha_star(G, N, b, lam), N)
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_delta_dagger_multiply():
    """delta-dagger(gamma-dagger F * gamma-dagger G) = (1 - 2^-b X) F G mod B
    (Lemma delta-multiply), against exact rational reduction mod B."""
    N, b, lam = 6, 10, 9
    g = np.random.Generator(np.random.PCG64(11))
    F = g.integers(-512, 512, N + 1)
    G = g.integers(-512, 512, N + 1)
    rho = m.rho_newton(N, b)
    c = m.C_coeffs(N, b, rho)
    Fu, tF = m.gamma_dagger(F.astype(float), N, b, lam, rho, c)
    Gu, tG = m.gamma_dagger(G.astype(float), N, b, lam, rho, c)
    J = m.delta_dagger(m.convolution(Fu, Gu, N), tF * tG, N, b, lam, rho, c)
    eps = Fraction(1, 2 ** b)
    prod = [Fraction(int(x)) for x in np.convolve(F, G)]
    P = [Fraction(0)] * (len(prod) + 1)
    for i, w in enumerate(prod):
        P[i] += w
        P[i + 1] -= eps * w
    Bm = [Fraction(2 ** b)] + [Fraction(0)] * (N - 1) + [Fraction(-(2 ** b)), Fraction(1)]
    want = np.array([float(x) for x in _poly_rem(P, Bm)])
    assert np.max(np.abs(J - want)) < 1e-8 * np.max(np.abs(want))


def test_rho_interval():
    """2^b (1 - 2 * 2^-Nb) < rho < 2^b (Lemma on the real root), N = 12, b = 1."""
    N, b = 12, 1
    rho = m.rho_newton(N, b)
    assert 2.0 ** b * (1 - 2 * 2.0 ** (-N * b)) < rho < 2.0 ** b
    assert abs(rho ** (N + 1) - 2 ** b * rho ** N + 2 ** b) < 1e-9


# ------------------------------------------------------ digit splitting


@pytest.mark.parametrize("b", [4, 11, 16])
def test_balanced_digits(b):
    rng = random.Random(b)
    n = 997
    x = rng.getrandbits(n)
    N = -(-n // b)
    d = m.unsigned_digits(x, N, b)
    assert sum(di << (i * b) for i, di in enumerate(d)) == x
    for keep in (True, False):
        U = m.balanced_digits(d, b, keep)
        val = sum(ui << (i * b) for i, ui in enumerate(U))
        if keep:
            assert val == x
            assert all(abs(t) <= 2 ** (b - 1) for t in U[:-1]) and 0 <= U[-1] <= 2 ** b
        else:
            assert val % (1 << (N * b)) == x
            assert all(abs(t) <= 2 ** (b - 1) for t in U)


# ---------------------------------------------- end-to-end against CPython


@pytest.mark.parametrize("n,b,N,lam", [(1000, 11, 96, 6), (4096, 11, 384, 6),
                                       (4096, 12, 352, 5), (3001, 10, 301, 7),
                                       (777, 8, 100, 8)])
def test_model_products_against_cpython(n, b, N, lam):
    rng = random.Random(n * b)
    for _ in range(2):
        u, v = rng.getrandbits(n), rng.getrandbits(n)
        q, r = divmod(u * v, 1 << n)
        lo = m.low_product(u, v, n, b, N, lam)
        assert lo["w"] == r and lo["dist"] < 0.25
        assert lo["S"] % (1 << b) == 0
        Nh = N
        while (Nh + 1) * b < n + m.lg(Nh) + 2:
            Nh += 1
        hi = m.high_product(u, v, n, b, Nh, lam)
        assert hi["w"] == q or (r and hi["w"] == q + 1)
        assert abs(u * v - (hi["w"] << n)) < (1 << n)
        full = m.full_product(u, v, n, 16, -(-n // 16))
        assert full["w"] == u * v


def test_model_edge_operands():
    n, b, N, lam = 2048, 11, 192, 6
    ones = (1 << n) - 1
    for u, v in ((ones, ones), (ones, 1), (1 << (n - 1), 1 << (n - 1)), (0, ones)):
        q, r = divmod(u * v, 1 << n)
        assert m.low_product(u, v, n, b, N, lam)["w"] == r
        hi = m.high_product(u, v, n, b, N, lam)["w"]
        assert hi == q or (r and hi == q + 1)


def test_model_rounded_coefficients_match_closed_forms():
    """round(2^b W-bar_i) = 2^b L_i (proof of the low-product theorem) and
    round(2^b W-bar_i) = 2^b H_i (proof of the high-product theorem)."""
    n, b, N, lam = 6000, 11, 768, 6
    rng = random.Random(42)
    u, v = rng.getrandbits(n), rng.getrandbits(n)
    lo = m.low_product(u, v, n, b, N, lam)
    W = m.digit_product(lo["U"], lo["V"])
    assert list(lo["c"]) == m.low_coeffs_exact([int(t) for t in W], N, b)
    hi = m.high_product(u, v, n, b, N, lam)
    W = m.digit_product(hi["U"], hi["V"])
    assert list(hi["c"]) == m.high_coeffs_exact([int(t) for t in W], N, b)
    full = m.full_product(u, v, n, 16, 512)
    W = m.digit_product(full["U"], full["V"])
    assert list(full["c"][:len(W)]) == [int(t) for t in W]


@pytest.mark.parametrize("row", [0, 1])
def test_table2_parameters_are_correct_on_random_inputs(row):
    """The paper's own (N, b, lambda) rows of its parameter table give correct
    low, high and full products on random inputs (Section 5)."""
    n, N, b, lam, N2, bf = (int(t) for t in _golden("table2_parameters.txt")[row])
    rng = random.Random(row)
    u, v = rng.getrandbits(n), rng.getrandbits(n)
    q, r = divmod(u * v, 1 << n)
    lo = m.low_product(u, v, n, b, N, lam)
    assert lo["w"] == r and lo["dist"] < 0.5
    hi = m.high_product(u, v, n, b, N, lam)
    assert hi["w"] == q or (r and hi["w"] == q + 1)
    full = m.full_product(u, v, n, bf, N2 // 2)
    assert full["w"] == u * v
