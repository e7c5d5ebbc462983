"""GPU parity of the FP32 path (tm_mul_fp32c: double-float FFT passes) against
the CPU oracle, through the C ABI.

The FP32 path computes the same low, high and full products with digit sizes
chosen for its smaller working precision (b = 9 truncated, 13 full, lengths
powers of two).  Low and full products must equal the oracle bit for bit,
high products must lie in the allowed set and equal the plan-exact value,
and the rounded coefficients must equal the exact closed forms of the
cancellation propositions for the FP32 path's own (N, b).
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import method as m
from paper_1703_00640_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _tm():
    import paper_1703_00640_amd as tm
    return tm


def dev():
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to(dev())


def to_host(t):
    return t.cpu().numpy().view(np.uint64)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_fp32c(kind, u, v, n):
    tm = _tm()
    g = tm.new_guard(dev())
    out = tm.mul(kind, to_dev(u), to_dev(v), n, guard=g, fp32c=True)
    torch.cuda.synchronize()
    return to_host(out), tm.read_guard(g)


def check_all(u, v, n, threads=16):
    out = {}
    for kind in ("lo", "hi", "full"):
        w, g = run_fp32c(kind, u, v, n)
        assert g.flags == 0 and g.max_dist < 0.25, (kind, n, g.as_dict())
        out[kind] = (w, g)
    assert np.array_equal(out["full"][0], oracle.mul_full(u, v, n, threads)), "full n=%d" % n
    assert np.array_equal(out["lo"][0], oracle.mul_lo(u, v, n, threads)), "lo n=%d" % n
    q, nz = oracle.mul_hi(u, v, n, threads)
    assert oracle.hi_accepts(out["hi"][0], q, nz), "hi n=%d" % n
    return {k: g for k, (w, g) in out.items()}


@pytest.mark.parametrize("n", [1000, 4097, 1 << 16, 100003, 1 << 20, (1 << 22) + 4160])
def test_fp32c_random_parity(n):
    say("[fp32c] n=%d" % n)
    u, v = inputs.operand_pair(n, 400 + n % 89)
    g = check_all(u, v, n)
    say("  dist lo %.3g hi %.3g full %.3g" % (g["lo"].max_dist, g["hi"].max_dist, g["full"].max_dist))


def test_fp32c_edge_operands():
    """All-ones, (2^n - 1) x 1, zero and powers of two at n = 2^16."""
    n = 1 << 16
    ones, one = inputs.all_ones(n), inputs.small(n, 1)
    zero = np.zeros_like(ones)
    for a, b_ in ((ones, ones), (ones, one), (zero, ones),
                  (inputs.power_of_two(n, n - 1), inputs.power_of_two(n, 12345))):
        check_all(a, b_, n)


@pytest.mark.parametrize("n", [4096, 1 << 16, 100003])
def test_fp32c_rounded_coefficients_bit_exact(n):
    """c_i of the FP32 path equal 2^b L_i, 2^b H_i (Props low-cancel and
    high-cancel) and w_i for its own (N, b), exactly; the high product equals
    the plan-exact round(S / 2^D)."""
    tm = _tm()
    u, v = inputs.operand_pair(n, 17)
    ui, vi = oracle.to_int(u), oracle.to_int(v)
    for kind in ("lo", "hi", "full"):
        say("[fp32c coeffs] n=%d %s" % (n, kind))
        pl = tm.plan(kind, n, fp32c=True)
        c, x, g = tm.coefficients(kind, to_dev(u), to_dev(v), n, fp32c=True)
        c = c.cpu().numpy()
        N, b = pl["N"], pl["b"]
        if kind == "lo":
            U = m.balanced_digits(m.unsigned_digits(ui, N, b), b, False)
            V = m.balanced_digits(m.unsigned_digits(vi, N, b), b, False)
            want = m.low_coeffs_exact([int(t) for t in m.digit_product(U, V)], N, b)
        elif kind == "hi":
            s = (N + 1) * b - n
            U = m.balanced_digits(m.unsigned_digits(ui, N + 1, b, s), b, True)
            V = m.balanced_digits(m.unsigned_digits(vi, N + 1, b, s), b, True)
            want = m.high_coeffs_exact([int(t) for t in m.digit_product(U, V)], N, b)
            D = (N + 3) * b - n
            S = m.overlap_add(want, b)
            hi, _ = run_fp32c("hi", u, v, n)
            assert oracle.to_int(hi) == (S + (1 << (D - 1))) >> D
        else:
            nd = pl["digits"]
            U = m.balanced_digits(m.unsigned_digits(ui, nd, b), b, True)
            V = m.balanced_digits(m.unsigned_digits(vi, nd, b), b, True)
            W = [int(t) for t in m.digit_product(U, V)]
            want = W + [0] * (N - len(W))
        assert [int(t) for t in c] == [int(t) for t in want], kind
        assert g.flags == 0 and g.max_dist < 0.25


@pytest.mark.parametrize("lm", [2, 8])
def test_fp32c_three_pass_split(monkeypatch, lm):
    """The FP32 path's middle pass (forced middle length) at n = 2^20."""
    monkeypatch.setenv("TM_FORCE_LM", str(lm))
    tm = _tm()
    n = 1 << 20
    assert tm.plan("hi", n, fp32c=True)["Lm"] == lm
    u, v = inputs.operand_pair(n, 430 + lm)
    check_all(u, v, n)


def test_fp32c_precision_config_n2_26_high():
    """The precision comparison size: the high product at n = 2^26 on both
    paths, each against the oracle, with its rounding distance below the
    guard's 1/4."""
    n = 1 << 26
    u, v = inputs.operand_pair(n, 4)
    q, nz = oracle.mul_hi(u, v, n, 16)
    w32, g32 = run_fp32c("hi", u, v, n)
    tm = _tm()
    g = tm.new_guard(dev())
    w64 = to_host(tm.mul("hi", to_dev(u), to_dev(v), n, guard=g))
    g64 = tm.read_guard(g)
    say("[fp32c] n=2^26 hi: fp32c b=%d N=%d dist %.4g; fp64 b=%d N=%d dist %.4g"
        % (g32.b, g32.N, g32.max_dist, g64.b, g64.N, g64.max_dist))
    assert g32.flags == 0 and g32.max_dist < 0.25 and g64.flags == 0
    assert oracle.hi_accepts(w32, q, nz) and oracle.hi_accepts(w64, q, nz)
