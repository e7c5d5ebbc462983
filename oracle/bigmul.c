/*
 * Reference big-integer products on little-endian 64-bit limbs.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the CPU oracle against which the
 * GPU library is checked; the library never links, loads or calls it, and it
 * shares no code, header or table with the library.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may use it.
 *
 * What it computes is the plain definition of the three products in the
 * paper's introduction (Section 1):
 *   full product  uv;
 *   low product   the unique w in [0, 2^n) with w = uv (mod 2^n);
 *   high product  any w in [0, 2^n] with |uv - 2^n w| < 2^n, i.e. one of
 *                 q = floor(uv / 2^n) and, when uv mod 2^n != 0, q + 1.
 * The oracle returns q together with the flag "uv mod 2^n != 0", so the
 * caller can test membership in that (at most two-element) set.
 *
 * The multiplication is schoolbook with 128-bit accumulation for short
 * operands and subtractive Karatsuba above a threshold; OpenMP tasks spread
 * the top recursion levels over cores.  Bits of u and v at positions >= n are
 * ignored (masked), as the library's interface specifies.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

#define KARATSUBA_THRESHOLD 32

/* ---------------------------------------------------------------- helpers */

/* r[0..n) = a[0..n) + b[0..n); returns carry */
static uint64_t add_n(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n)
{
    uint64_t c = 0;
    for (size_t i = 0; i < n; i++) {
        u128 s = (u128)a[i] + b[i] + c;
        r[i] = (uint64_t)s;
        c = (uint64_t)(s >> 64);
    }
    return c;
}

/* r[0..n) = a[0..n) - b[0..n); returns borrow */
static uint64_t sub_n(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n)
{
    uint64_t br = 0;
    for (size_t i = 0; i < n; i++) {
        uint64_t ai = a[i], bi = b[i];
        uint64_t d = ai - bi - br;
        br = (ai < bi) || (ai == bi && br) ? 1 : 0;
        r[i] = d;
    }
    return br;
}

/* add x (n limbs) into r (m >= n limbs), propagating the carry upward */
static void add_into(uint64_t *r, size_t m, const uint64_t *x, size_t n)
{
    uint64_t c = add_n(r, r, x, n);
    for (size_t i = n; c && i < m; i++) {
        r[i] += 1;
        c = (r[i] == 0);
    }
}

/* subtract x (n limbs) from r (m >= n limbs), propagating the borrow */
static void sub_into(uint64_t *r, size_t m, const uint64_t *x, size_t n)
{
    uint64_t b = sub_n(r, r, x, n);
    for (size_t i = n; b && i < m; i++) {
        b = (r[i] == 0);
        r[i] -= 1;
    }
}

/* compare a, b of n limbs: -1, 0, 1 */
static int cmp_n(const uint64_t *a, const uint64_t *b, size_t n)
{
    for (size_t i = n; i-- > 0;) {
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    }
    return 0;
}

/* r[0..na+nb) = a[0..na) * b[0..nb), schoolbook with 128-bit products */
static void mul_school(uint64_t *r, const uint64_t *a, size_t na,
                       const uint64_t *b, size_t nb)
{
    memset(r, 0, (na + nb) * sizeof(uint64_t));
    for (size_t i = 0; i < na; i++) {
        uint64_t c = 0;
        for (size_t j = 0; j < nb; j++) {
            u128 t = (u128)a[i] * b[j] + r[i + j] + c;
            r[i + j] = (uint64_t)t;
            c = (uint64_t)(t >> 64);
        }
        r[i + nb] = c;
    }
}

/*
 * r[0..2n) = a[0..n) * b[0..n), subtractive Karatsuba.
 * Split at h = ceil(n/2): a = a0 + a1 X^h, b = b0 + b1 X^h, X = 2^64.
 * a*b = a0b0 + (a0b0 + a1b1 + (a0-a1)(b1-b0)) X^h + a1b1 X^2h.
 */
static void mul_kara(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n,
                     int depth)
{
    if (n <= KARATSUBA_THRESHOLD) {
        mul_school(r, a, n, b, n);
        return;
    }
    size_t h = (n + 1) / 2, l = n - h;

    /* |a0 - a1| and |b1 - b0| as h-limb numbers (a1, b0 zero-extended) */
    uint64_t *da = calloc(h, sizeof(uint64_t));
    uint64_t *db = calloc(h, sizeof(uint64_t));
    uint64_t *a1x = calloc(h, sizeof(uint64_t));
    uint64_t *b1x = calloc(h, sizeof(uint64_t));
    memcpy(a1x, a + h, l * sizeof(uint64_t));
    memcpy(b1x, b + h, l * sizeof(uint64_t));
    int neg = 0;
    if (cmp_n(a, a1x, h) >= 0) sub_n(da, a, a1x, h);
    else { sub_n(da, a1x, a, h); neg ^= 1; }
    if (cmp_n(b1x, b, h) >= 0) sub_n(db, b1x, b, h);
    else { sub_n(db, b, b1x, h); neg ^= 1; }

    uint64_t *z0 = malloc(2 * h * sizeof(uint64_t));
    uint64_t *z2 = malloc(2 * h * sizeof(uint64_t));
    uint64_t *z1 = malloc(2 * h * sizeof(uint64_t));

#ifdef _OPENMP
    if (depth < 4 && n > 4096) {
#pragma omp task shared(z0) firstprivate(a, b, h, depth)
        mul_kara(z0, a, b, h, depth + 1);
#pragma omp task shared(z2) firstprivate(a1x, b1x, h, depth)
        mul_kara(z2, a1x, b1x, h, depth + 1);
#pragma omp task shared(z1) firstprivate(da, db, h, depth)
        mul_kara(z1, da, db, h, depth + 1);
#pragma omp taskwait
    } else
#endif
    {
        mul_kara(z0, a, b, h, depth + 1);
        mul_kara(z2, a1x, b1x, h, depth + 1);
        mul_kara(z1, da, db, h, depth + 1);
    }

    /* r = z0 + z2 X^2h (z2 has only 2l significant limbs) */
    memset(r, 0, 2 * n * sizeof(uint64_t));
    memcpy(r, z0, 2 * h * sizeof(uint64_t));
    add_into(r + 2 * h, 2 * n - 2 * h, z2, 2 * l);
    /* middle term z0 + z2 +/- z1 at X^h; it is non-negative, so apply the
       additions before the (possible) subtraction */
    add_into(r + h, 2 * n - h, z0, 2 * h);
    add_into(r + h, 2 * n - h, z2, 2 * l);
    if (neg) sub_into(r + h, 2 * n - h, z1, 2 * h);
    else     add_into(r + h, 2 * n - h, z1, 2 * h);

    free(da); free(db); free(a1x); free(b1x);
    free(z0); free(z1); free(z2);
}

/* copy the low n bits of src (L limbs) into dst (L limbs), clearing the rest */
static void mask_bits(uint64_t *dst, const uint64_t *src, size_t L, uint64_t n)
{
    for (size_t i = 0; i < L; i++) {
        uint64_t lo = (uint64_t)i * 64;
        if (lo >= n) dst[i] = 0;
        else if (n - lo >= 64) dst[i] = src[i];
        else dst[i] = src[i] & ((UINT64_C(1) << (n - lo)) - 1);
    }
}

/* ------------------------------------------------------------- public API */

size_t oracle_limbs(uint64_t n_bits) { return (size_t)((n_bits + 63) / 64); }

/* full product: w[0..2L) = (u mod 2^n) * (v mod 2^n), L = ceil(n/64) */
int oracle_mul_full(uint64_t *w, const uint64_t *u, const uint64_t *v,
                    uint64_t n_bits, int threads)
{
    size_t L = oracle_limbs(n_bits);
    if (L == 0) return 0;
    uint64_t *um = malloc(L * sizeof(uint64_t));
    uint64_t *vm = malloc(L * sizeof(uint64_t));
    if (!um || !vm) { free(um); free(vm); return -1; }
    mask_bits(um, u, L, n_bits);
    mask_bits(vm, v, L, n_bits);
#ifdef _OPENMP
    if (threads > 1) {
        omp_set_num_threads(threads);
#pragma omp parallel
#pragma omp single
        mul_kara(w, um, vm, L, 0);
    } else
#endif
    {
        (void)threads;
        mul_kara(w, um, vm, L, 99);   /* depth 99: no tasks */
    }
    free(um); free(vm);
    return 0;
}

/* low product: w[0..L) = uv mod 2^n */
int oracle_mul_lo(uint64_t *w, const uint64_t *u, const uint64_t *v,
                  uint64_t n_bits, int threads)
{
    size_t L = oracle_limbs(n_bits);
    uint64_t *f = malloc(2 * L * sizeof(uint64_t) + 8);
    if (!f) return -1;
    if (oracle_mul_full(f, u, v, n_bits, threads)) { free(f); return -1; }
    mask_bits(w, f, L, n_bits);
    free(f);
    return 0;
}

/*
 * high product: q[0..L) = floor(uv / 2^n) and *rem_nonzero = (uv mod 2^n != 0).
 * The accepted outputs are q, and q + 1 when *rem_nonzero is set.
 */
int oracle_mul_hi(uint64_t *q, int *rem_nonzero, const uint64_t *u,
                  const uint64_t *v, uint64_t n_bits, int threads)
{
    size_t L = oracle_limbs(n_bits);
    uint64_t *f = malloc(2 * L * sizeof(uint64_t) + 8);
    if (!f) return -1;
    if (oracle_mul_full(f, u, v, n_bits, threads)) { free(f); return -1; }
    /* remainder test: any of the low n bits set */
    int nz = 0;
    for (size_t i = 0; i < L && !nz; i++) {
        uint64_t lo = (uint64_t)i * 64;
        uint64_t word = f[i];
        if (n_bits - lo < 64) word &= (UINT64_C(1) << (n_bits - lo)) - 1;
        nz = word != 0;
    }
    *rem_nonzero = nz;
    /* q = f >> n, L limbs (uv < 2^2n so q < 2^n fits) */
    size_t sh_l = (size_t)(n_bits / 64);
    unsigned sh_b = (unsigned)(n_bits % 64);
    for (size_t i = 0; i < L; i++) {
        size_t s = i + sh_l;
        uint64_t lo = s < 2 * L ? f[s] : 0;
        uint64_t hi = s + 1 < 2 * L ? f[s + 1] : 0;
        q[i] = sh_b ? (lo >> sh_b) | (hi << (64 - sh_b)) : lo;
    }
    free(f);
    return 0;
}

/* x mod p for x of L limbs and p < 2^63 (Horner in 128-bit arithmetic) */
uint64_t oracle_mod(const uint64_t *x, size_t L, uint64_t p)
{
    u128 r = 0;
    for (size_t i = L; i-- > 0;) r = ((r << 64) | x[i]) % p;
    return (uint64_t)r;
}

/* schoolbook only, for cross-checking the Karatsuba path in tests */
int oracle_mul_school(uint64_t *w, const uint64_t *u, size_t nu,
                      const uint64_t *v, size_t nv)
{
    mul_school(w, u, nu, v, nv);
    return 0;
}
