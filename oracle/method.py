"""FP64 model of the paper's full, low and high product algorithms.

TEST INFRASTRUCTURE ONLY (see the package docstring).  It follows the
algorithms step by step in the paper's order and notation so that a reader
can check it against the paper by eye; the only library primitive is the
FFT used as the ``Convolution`` black box of Section 2.1 (numpy's real FFT).

Readings taken where the paper leaves a choice (each is listed in the design
notes):

* Digits are the balanced signed digits of Section 5 (|U_i| <= 2^(b-1)),
  formed from the unsigned b-bit digits d_i by
  ``U_i = d_i - 2^b [d_i >= 2^(b-1)] + [d_(i-1) >= 2^(b-1)]``.  The low
  product subtracts at every digit (the carry out of the top digit is
  dropped: only U(2^b) mod 2^(Nb) matters); the full and high products let
  the top digit keep its carry (so it lies in [0, 2^b]).
* The high product follows the Remark on Newton's method only where the
  arithmetic says so: rho is obtained by Newton's method on B from 2^b, C's
  coefficients are 2^b / rho^(j+1), and psi is evaluated from its defining
  formula; in double precision these reduce to rho = 2^b and psi = theta
  once N b exceeds the exponent range.
* Rounding uses round-half-to-even (ties may go either way, Section 2.2).
"""
import math

import numpy as np

# ----------------------------------------------------------------- helpers


def lg(x):
    """lg x = ceil(log2 x) for an integer x >= 1 (Section 2.1)."""
    x = int(x)
    if x < 1:
        raise ValueError("lg of %d" % x)
    return (x - 1).bit_length()


def overlap_add(c, b):
    """Exact integer sum_i c_i 2^(i b) of a sequence of integers."""
    c = [int(t) for t in c]

    def rec(lo, hi):
        if hi - lo <= 32:
            s = 0
            for i in range(hi - 1, lo - 1, -1):
                s = (s << b) + c[i]
            return s
        mid = (lo + hi) // 2
        return rec(lo, mid) + (rec(mid, hi) << ((mid - lo) * b))

    return rec(0, len(c)) if c else 0


def unsigned_digits(x, count, b, shift=0):
    """d_i = floor(x 2^shift / 2^(i b)) mod 2^b for i < count (Python ints).

    Bits are unpacked once (O(n)); digit i is bits [i b, i b + b)."""
    x = int(x) << shift
    nbits = count * b
    nbytes = (max(nbits, x.bit_length()) + 7) // 8 + 1
    bits = np.unpackbits(np.frombuffer(x.to_bytes(nbytes, "little"), np.uint8),
                         bitorder="little")[:nbits].astype(np.int64)
    weights = np.int64(1) << np.arange(b, dtype=np.int64)
    return [int(t) for t in bits.reshape(count, b) @ weights]


def balanced_digits(d, b, top_keeps_carry):
    """Balanced signed digits of Section 5 from unsigned digits d."""
    h = 1 << (b - 1)
    out = []
    for i, di in enumerate(d):
        carry_in = 1 if (i > 0 and d[i - 1] >= h) else 0
        last = i == len(d) - 1
        if last and top_keeps_carry:
            out.append(di + carry_in)
        else:
            out.append(di - (1 << b if di >= h else 0) + carry_in)
    return out


# ------------------------------------------------------ series coefficients


def _binom_float(y, r):
    p = 1.0
    for j in range(r):
        p *= (y - j)
    return p / math.factorial(r)


def alpha_c(k, r, N, b):
    """alpha_{k,r} = k/(k+r) binom((k+r)/N, r) (-2^-b)^r (Lemma, Sec. 3.2)."""
    if r == 0:
        return 1.0
    return k / (k + r) * _binom_float((k + r) / N, r) * (-(2.0 ** -b)) ** r


def beta_c(k, r, N, b):
    """beta_{k,r} = binom(-k/N, r) (-2^-b)^r (Section 3.2)."""
    return _binom_float(-k / N, r) * (-(2.0 ** -b)) ** r


def gamma_c(k, r, N, b):
    """gamma_{k,r} = k/(k+r) binom(-(k+r)/N, r) (-2^-b)^r (Lemma, Sec. 4.2)."""
    if r == 0:
        return 1.0
    return k / (k + r) * _binom_float(-(k + r) / N, r) * (-(2.0 ** -b)) ** r


def delta_c(k, r, N, b):
    """delta_{k,r} = binom(k/N, r) (-2^-b)^r (Section 4.2)."""
    return _binom_float(k / N, r) * (-(2.0 ** -b)) ** r


def _coef_vec(f, r, N, b):
    return np.array([f(k, r, N, b) for k in range(N)], dtype=np.float64)


# ------------------------------------------------------- polynomial moduli


def reduce_cyclic(P, N):
    """P mod X^N - 1 (coefficient vector of any length)."""
    out = np.zeros(N)
    for start in range(0, len(P), N):
        chunk = P[start:start + N]
        out[:len(chunk)] += chunk
    return out


def reduce_mod_A(P, N, b):
    """P mod A(X), A = X^N + 2^-b X - 1 (Proposition on low cancellation).

    Top-down elimination with X^d = X^(d-N) (1 - 2^-b X) for d >= N."""
    P = np.array(P, dtype=np.float64)
    eps = 2.0 ** -b
    for d in range(len(P) - 1, N - 1, -1):
        c = P[d]
        P[d] = 0.0
        P[d - N] += c
        P[d - N + 1] -= eps * c
    return P[:N].copy()


def rho_newton(N, b, iters=8):
    """Real root rho of B(X) = X^(N+1) - 2^b X^N + 2^b near 2^b (Lemma on
    the real root), by Newton's method started at 2^b (Proposition on
    approximating gamma-dagger).  Works with Y = X / 2^b, for which
    B(2^b Y) / 2^((N+1) b) = Y^(N+1) - Y^N + 2^(-N b)."""
    eps = 2.0 ** (-N * b) if N * b < 1070 else 0.0
    y = 1.0
    for _ in range(iters):
        f = y ** (N + 1) - y ** N + eps
        fp = (N + 1) * y ** N - N * y ** (N - 1)
        y = y - f / fp
    return (2.0 ** b) * y


def C_coeffs(N, b, rho):
    """Coefficients c_0..c_(N-1) of C(X) = B(X)/(X - rho) = X^N + sum_j c_j X^j,
    c_j = -(2^b / rho) rho^-j (explicit formula for C)."""
    j = np.arange(N, dtype=np.float64)
    with np.errstate(under="ignore"):
        return -(2.0 ** b / rho) * np.power(rho, -j)


def reduce_mod_C(P, N, c):
    """P mod C(X) using X^N = -sum_j c_j X^j, top-down."""
    P = np.array(P, dtype=np.float64)
    for d in range(len(P) - 1, N - 1, -1):
        t = P[d]
        if t == 0.0:
            continue
        P[d] = 0.0
        # X^d = X^(d-N) X^N = -sum_j c_j X^(d-N+j)
        P[d - N:d] -= t * c
    return P[:N].copy()


# ----------------------------------------------------------- the ring maps


def alpha_star(F, N, b, lam):
    """Truncated alpha* (Prop. on approximating alpha*): sum over r < lam of
    alpha*_r F = sum_k alpha_{k,r} F_k X^(k+r) mod X^N - 1."""
    P = np.zeros(N + lam)
    for r in range(lam):
        P[r:r + N] += _coef_vec(alpha_c, r, N, b) * F
    return reduce_cyclic(P, N)


def beta_star(F, N, b, lam):
    """Truncated beta* (Prop. on approximating beta*): sum over r < lam of
    sum_k beta_{k,r} F_k X^(k+r) mod A(X)."""
    P = np.zeros(N + lam)
    for r in range(lam):
        P[r:r + N] += _coef_vec(beta_c, r, N, b) * F
    return reduce_mod_A(P, N, b)


def gamma_star(F, N, b, lam):
    """Truncated gamma*: sum_k gamma_{k,r} F_k X^(k+r) mod X^N - 1."""
    P = np.zeros(N + lam)
    for r in range(lam):
        P[r:r + N] += _coef_vec(gamma_c, r, N, b) * F
    return reduce_cyclic(P, N)


def delta_star(F, N, b, lam, c):
    """Truncated delta*: sum_k delta_{k,r} F_k X^(k+r) mod C(X)."""
    P = np.zeros(N + lam)
    for r in range(lam):
        P[r:r + N] += _coef_vec(delta_c, r, N, b) * F
    return reduce_mod_C(P, N, c)


def gamma_dagger(F, N, b, lam, rho, c):
    """gamma-dagger F = (gamma*(F mod C), rho^-N F(rho)) for F of degree <= N
    (definition in Section 4.3; F mod C by eq. reduction-modC)."""
    F = np.asarray(F, dtype=np.float64)
    Fc = reduce_mod_C(F, N, c)
    G = gamma_star(Fc, N, b, lam)
    k = np.arange(N + 1, dtype=np.float64)
    with np.errstate(under="ignore"):
        theta = float(np.sum(F * np.power(rho, k - N)))
    return G, theta


def delta_dagger(W, theta, N, b, lam, rho, c):
    """delta-dagger(W, theta) by eq. crt-sum: J = (1 - 2^-b X) H + psi C(X)
    with H = delta* W mod C and psi from eq. psi-formula, evaluated after
    dividing numerator and denominator by rho^N (no overflow)."""
    H = delta_star(W, N, b, lam, c)
    j = np.arange(N, dtype=np.float64)
    with np.errstate(under="ignore"):
        rhoN_inv = rho ** (-N) if N * math.log2(rho) < 1070 else 0.0
        Hrho_scaled = float(np.sum(H * np.power(rho, j - N)))      # rho^-N H(rho)
        C_rho_scaled = 1.0 + float(np.sum(c * np.power(rho, j - N)))  # C(rho)/rho^N
    psi = (theta - rhoN_inv * Hrho_scaled) / C_rho_scaled
    J = np.zeros(N + 1)
    J[:N] += H
    J[1:N + 1] -= (2.0 ** -b) * H
    J[:N] += psi * c
    J[N] += psi
    return J


def convolution(F, G, N):
    """Cyclic convolution mod X^N - 1 (the Convolution black box of
    Section 2.1) by real FFTs."""
    return np.fft.irfft(np.fft.rfft(F, N) * np.fft.rfft(G, N), N)


# ------------------------------------------------------------ algorithms


def _round(x):
    return np.rint(x)


def full_product(u, v, n, b, N):
    """Algorithm full: N digits, length-2N convolution, round, overlap-add.
    Returns dict with digits, the convolution W-bar, rounded c and w = uv."""
    if N * b < n:
        raise ValueError("need N b >= n")
    U = balanced_digits(unsigned_digits(u % (1 << n), N, b), b, True)
    V = balanced_digits(unsigned_digits(v % (1 << n), N, b), b, True)
    Wb = convolution(np.array(U, float), np.array(V, float), 2 * N)
    c = _round(Wb)
    w = overlap_add(c[:2 * N - 1].astype(np.int64), b)
    return dict(U=U, V=V, x=Wb, c=c.astype(np.int64), w=w,
                dist=float(np.max(np.abs(Wb - c))), maxabs=float(np.max(np.abs(Wb))))


def low_product(u, v, n, b, N, lam):
    """Algorithm low: split, alpha*, convolution, beta*, round, overlap-add.
    Returns dict with U, V, x = 2^b W-bar, c = round(x), w = uv mod 2^n."""
    if N * b < n:
        raise ValueError("need N b >= n")
    U = balanced_digits(unsigned_digits(u % (1 << n), N, b), b, False)
    V = balanced_digits(unsigned_digits(v % (1 << n), N, b), b, False)
    Ut = alpha_star(np.array(U, float), N, b, lam)
    Vt = alpha_star(np.array(V, float), N, b, lam)
    Wt = convolution(Ut, Vt, N)
    Wbar = beta_star(Wt, N, b, lam)
    x = (2.0 ** b) * Wbar
    c = _round(x).astype(np.int64)
    S = overlap_add(c, b)
    w = (S >> b) % (1 << n)
    return dict(U=U, V=V, Ut=Ut, Vt=Vt, Wt=Wt, x=x, c=c, S=S, w=w,
                dist=float(np.max(np.abs(x - c))), maxabs=float(np.max(np.abs(x))))


def high_product(u, v, n, b, N, lam):
    """Algorithm high: split from the top (shift s = (N+1)b - n), gamma-dagger,
    convolution plus theta_W = theta_U theta_V, delta-dagger, round,
    t = sum 2^-b round(2^b W_i) 2^(ib - ((N+2)b - n)), return round(t)."""
    if (N + 1) * b < n + lg(N) + 2:
        raise ValueError("need (N+1) b >= n + lg N + 2")
    s = (N + 1) * b - n
    U = balanced_digits(unsigned_digits(u % (1 << n), N + 1, b, s), b, True)
    V = balanced_digits(unsigned_digits(v % (1 << n), N + 1, b, s), b, True)
    rho = rho_newton(N, b)
    cC = C_coeffs(N, b, rho)
    Gu, thu = gamma_dagger(np.array(U, float), N, b, lam, rho, cC)
    Gv, thv = gamma_dagger(np.array(V, float), N, b, lam, rho, cC)
    Wt = convolution(Gu, Gv, N)
    thW = thu * thv
    J = delta_dagger(Wt, thW, N, b, lam, rho, cC)
    x = (2.0 ** b) * J
    c = _round(x).astype(np.int64)
    S = overlap_add(c, b)
    D = (N + 3) * b - n            # t = S / 2^D
    w = (S + (1 << (D - 1))) >> D  # round half up
    return dict(U=U, V=V, Gu=Gu, Gv=Gv, Wt=Wt, theta=(thu, thv, thW), x=x, c=c,
                S=S, D=D, w=w, dist=float(np.max(np.abs(x - c))),
                maxabs=float(np.max(np.abs(x))))


# ------------------------------------------- exact rounded coefficients


def digit_product(U, V):
    """Exact integer coefficients w_i of W = U V (plain convolution)."""
    U = np.asarray(U, dtype=np.int64)
    V = np.asarray(V, dtype=np.int64)
    bound = int(np.max(np.abs(U), initial=0)) * int(np.max(np.abs(V), initial=0)) * min(len(U), len(V))
    if bound < 2 ** 62:
        return np.convolve(U, V).astype(np.int64)
    return np.convolve(U.astype(object), V.astype(object))


def low_coeffs_exact(W, N, b):
    """2^b L with L = W mod A written out as in the proof of the low
    cancellation proposition: L = sum_(i<N) w_i X^i
    + sum_(i<=N-2) w_(N+i) (1 - 2^-b X) X^i.  Integers, length N."""
    W = list(W) + [0] * max(0, 2 * N - 1 - len(W))
    c = [(W[i] << b) for i in range(N)]
    for i in range(N - 1):
        c[i] += W[N + i] << b
        c[i + 1] -= W[N + i]
    return c


def high_coeffs_exact(W, N, b):
    """2^b H with H = (1 - 2^-b X) W mod B written out as in the proof of
    the high cancellation proposition: H = sum_(i<N) w_i X^i (1 - 2^-b X)
    + sum_(i<=N) w_(N+i) X^i.  Integers, length N + 1."""
    W = list(W) + [0] * max(0, 2 * N + 1 - len(W))
    c = [0] * (N + 1)
    for i in range(N):
        c[i] += W[i] << b
        c[i + 1] -= W[i]
    for i in range(N + 1):
        c[i] += W[N + i] << b
    return c
