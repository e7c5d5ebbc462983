"""Write the oracle's digests of the n = 2^30 products (largest single
instance) to ``large_products.json`` beside this script.

Test infrastructure.  The expected values come from ``oracle/`` only: the
plain Karatsuba product of the seeded operand pair (the same pair the GPU
test builds from ``paper_1703_00640_amd.inputs``), then the definitions of
Section 1: low product = the low n bits, high-product set = {q, q + 1 if the
low n bits are not all zero} with q = the high n bits.  A full product at
n = 2^30 takes minutes on the CPU, so the GPU test compares SHA-256 digests
of its outputs with these, which is an element-by-element comparison of
every limb; a few sampled limbs are stored too, so a mismatch names where.

Run:  python tests/golden/make_large_digests.py [threads]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1703_00640_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "large_products.json")
LOG2N = 30
TAG = 5          # operand_pair tag of the n = 2^30 workload
NSAMPLE = 64     # sampled limb positions per output


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


def plus_one(a):
    """a + 1 for a little-endian limb array (no overflow out of the top limb
    is possible here: q < 2^n - 1 whenever the remainder is non-zero)."""
    r = a.copy()
    i = 0
    while True:
        r[i] = np.uint64(int(r[i]) + 1 & 0xFFFFFFFFFFFFFFFF)
        if r[i] != 0:
            return r
        i += 1


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    n = 1 << LOG2N
    L = n // 64
    u, v = inputs.operand_pair(n, TAG)
    t0 = time.time()
    full = oracle.mul_full(u, v, n, threads)
    dt = time.time() - t0
    lo = full[:L]          # n is a multiple of 64: the low n bits are L limbs
    q = full[L:]           # floor(uv / 2^n)
    nz = bool(np.any(lo != 0))
    g = np.random.Generator(np.random.PCG64(12345))
    pos_full = sorted(int(x) for x in g.integers(0, 2 * L, size=NSAMPLE))
    rec = {
        "n_bits": n, "tag": TAG,
        "u_sha256": sha(u), "v_sha256": sha(v),
        "full_sha256": sha(full), "lo_sha256": sha(lo),
        "hi_q_sha256": sha(q), "hi_rem_nonzero": nz,
        "hi_q_plus_1_sha256": sha(plus_one(q)) if nz else None,
        "full_samples": [[p, "%016x" % int(full[p])] for p in pos_full],
        "oracle_seconds": round(dt, 1), "oracle_threads": threads,
    }
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print("wrote %s (oracle %.1f s on %d threads)" % (OUT, dt, threads))


if __name__ == "__main__":
    main()
