"""CPU oracle for the truncated-product library.

TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product: the GPU
library never imports, links or calls this package, and this package never
imports the library.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may use it.

Contents
--------
``bigmul.c`` (wrapped below)
    The plain definition of the three products of Section 1 on 64-bit limbs:
    full product ``uv``, low product ``uv mod 2^n``, and the high-product set
    ``{q, q+1 if uv mod 2^n != 0}`` with ``q = floor(uv / 2^n)``.
``method.py``
    An FP64 model of the paper's algorithms (full, low and high product) in
    the paper's order and notation, used for stage-level comparisons, plus
    the exact closed forms of the rounded coefficients (Propositions on the
    cancellation trick for the low and the high product).
``coeffs.py``
    Exact rational series coefficients alpha, beta, gamma, delta
    (Sections 3.2 and 4.2) from their binomial definitions.
``mulmod`` / ``barrett_mu`` (below)
    Modular multiplication, the consumer of the high and low products that
    Section 1 names, by its plain definition: the oracle's full product
    reduced mod m with integer division; and the Barrett reciprocal
    floor(2^(2n) / m).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=False):
    """Compile bigmul.c into liboracle.so with gcc (OpenMP on)."""
    src = os.path.join(_HERE, "bigmul.c")
    if (not force and os.path.exists(_LIB_PATH)
            and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(src)):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC",
                           "-o", tmp, src])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        p64 = ctypes.POINTER(ctypes.c_uint64)
        lib.oracle_mul_full.argtypes = [p64, p64, p64, ctypes.c_uint64, ctypes.c_int]
        lib.oracle_mul_lo.argtypes = [p64, p64, p64, ctypes.c_uint64, ctypes.c_int]
        lib.oracle_mul_hi.argtypes = [p64, ctypes.POINTER(ctypes.c_int), p64, p64,
                                      ctypes.c_uint64, ctypes.c_int]
        lib.oracle_mod.argtypes = [p64, ctypes.c_size_t, ctypes.c_uint64]
        lib.oracle_mod.restype = ctypes.c_uint64
        lib.oracle_mul_school.argtypes = [p64, p64, ctypes.c_size_t, p64, ctypes.c_size_t]
        for f in (lib.oracle_mul_full, lib.oracle_mul_lo, lib.oracle_mul_hi,
                  lib.oracle_mul_school):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _limbs(x, L):
    a = np.ascontiguousarray(x, dtype=np.uint64)
    if a.shape != (L,):
        raise ValueError("expected %d limbs, got shape %s" % (L, a.shape))
    return a


def nlimbs(n_bits):
    return (int(n_bits) + 63) // 64


def mul_full(u, v, n_bits, threads=1):
    """Full product of u mod 2^n and v mod 2^n: 2L limbs."""
    L = nlimbs(n_bits)
    u, v = _limbs(u, L), _limbs(v, L)
    w = np.zeros(2 * L, dtype=np.uint64)
    if _load().oracle_mul_full(_ptr(w), _ptr(u), _ptr(v), n_bits, threads):
        raise MemoryError("oracle_mul_full failed")
    return w


def mul_lo(u, v, n_bits, threads=1):
    """Low product uv mod 2^n: L limbs."""
    L = nlimbs(n_bits)
    u, v = _limbs(u, L), _limbs(v, L)
    w = np.zeros(L, dtype=np.uint64)
    if _load().oracle_mul_lo(_ptr(w), _ptr(u), _ptr(v), n_bits, threads):
        raise MemoryError("oracle_mul_lo failed")
    return w


def mul_hi(u, v, n_bits, threads=1):
    """High product set: returns (q, rem_nonzero); accepted are q and, when
    rem_nonzero, q + 1 (Section 1: |uv - 2^n w| < 2^n)."""
    L = nlimbs(n_bits)
    u, v = _limbs(u, L), _limbs(v, L)
    q = np.zeros(L, dtype=np.uint64)
    nz = ctypes.c_int(0)
    if _load().oracle_mul_hi(_ptr(q), ctypes.byref(nz), _ptr(u), _ptr(v), n_bits, threads):
        raise MemoryError("oracle_mul_hi failed")
    return q, bool(nz.value)


def mul_school(u, v):
    """Schoolbook product of two limb arrays of any lengths (cross-check)."""
    u = np.ascontiguousarray(u, dtype=np.uint64)
    v = np.ascontiguousarray(v, dtype=np.uint64)
    w = np.zeros(len(u) + len(v), dtype=np.uint64)
    _load().oracle_mul_school(_ptr(w), _ptr(u), len(u), _ptr(v), len(v))
    return w


def residue(x, p):
    """x mod p for a limb array x and p < 2^63."""
    x = np.ascontiguousarray(x, dtype=np.uint64)
    return int(_load().oracle_mod(_ptr(x), len(x), p))


def hi_accepts(w, q, rem_nonzero):
    """True iff limb array w is an allowed high product given (q, rem_nonzero)."""
    w = np.asarray(w, dtype=np.uint64)
    if np.array_equal(w, q):
        return True
    if not rem_nonzero:
        return False
    return to_int(w) == to_int(q) + 1


def to_int(limbs):
    """Little-endian uint64 limbs -> Python int."""
    return int.from_bytes(np.ascontiguousarray(limbs, dtype="<u8").tobytes(), "little")


def from_int(x, L):
    """Python int (non-negative, < 2^(64L)) -> L little-endian uint64 limbs."""
    return np.frombuffer(int(x).to_bytes(8 * L, "little"), dtype="<u8").astype(np.uint64)


def mulmod(a, b, m, n_bits, threads=1):
    """a b mod m (plain definition: the full product, then the remainder of
    integer division); a, b, m as limb arrays of ceil(n/64) limbs."""
    L = nlimbs(n_bits)
    full = to_int(mul_full(a, b, n_bits, threads))
    return from_int(full % to_int(_limbs(m, L)), L)


def barrett_mu(m, n_bits):
    """floor(2^(2n) / m) as ceil((n+1)/64) limbs (an input of the Barrett
    reduction, computed once per modulus)."""
    L = nlimbs(n_bits)
    mu = (1 << (2 * int(n_bits))) // to_int(_limbs(m, L))
    return from_int(mu, nlimbs(n_bits + 1))
