"""The allocation-free entry point (tm_mul_noalloc) against tm_mul.

tm_mul_noalloc runs the same plan and kernels as tm_mul with the library's
static per-GPU scratch array as its workspace.  Its products must equal
tm_mul's bit for bit (and the oracle's), on two calls in a row, the second
with a smaller input, so that what the first call left in the shared array
cannot leak into the second.  Sizes beyond the static maximum are refused.
"""
import numpy as np
import pytest

import oracle
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


def _pair(kind, n, tag):
    tm = _tm()
    u, v = inputs.operand_pair(n, tag)
    L = inputs.nlimbs(n)
    nout = 2 * L if kind == "full" else L
    tm.prepare(kind, n)
    return u, v, torch.zeros(nout, dtype=torch.int64, device=dev())


def _check_oracle(kind, u, v, n, w):
    if kind == "lo":
        assert np.array_equal(w, oracle.mul_lo(u, v, n, 8))
    elif kind == "full":
        assert np.array_equal(w, oracle.mul_full(u, v, n, 8))
    else:
        q, nz = oracle.mul_hi(u, v, n, 8)
        assert oracle.hi_accepts(w, q, nz)


@pytest.mark.parametrize("kind", ["lo", "hi", "full"])
def test_noalloc_matches_tm_mul_twice_shrinking(kind):
    """Two calls in a row on the shared scratch, the second smaller (and
    with a smaller transform), each equal to tm_mul and the oracle, guards
    included."""
    tm = _tm()
    for n, tag in (((1 << 22) + 4160, 300), (100003, 301)):
        print("[noalloc] %s n=%d" % (kind, n), flush=True)
        u, v, out = _pair(kind, n, tag)
        du, dv = to_dev(u), to_dev(v)
        g = tm.new_guard(dev())
        tm.mul_noalloc(kind, du, dv, n, out, guard=g)
        ref_g = tm.new_guard(dev())
        ref = tm.mul(kind, du, dv, n, guard=ref_g)
        torch.cuda.synchronize()
        w = to_host(out)
        assert np.array_equal(w, to_host(ref)), (kind, n)
        assert tm.read_guard(g).as_dict() == tm.read_guard(ref_g).as_dict()
        assert tm.read_guard(g).flags == 0
        _check_oracle(kind, u, v, n, w)


def test_noalloc_largest_and_refusals():
    """The largest size the static maximum covers (every kind at n = 2^24)
    runs and equals tm_mul; one size beyond it, and a size whose tables were
    never built, are refused with an error and launch nothing."""
    tm = _tm()
    n = 1 << 24
    assert tm.plan("full", n)["workspace_bytes"] <= tm.noalloc_max_bytes()
    u, v, out = _pair("full", n, 302)
    du, dv = to_dev(u), to_dev(v)
    tm.mul_noalloc("full", du, dv, n, out)
    ref = tm.mul("full", du, dv, n)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(out), to_host(ref))
    big = 1 << 26
    assert tm.plan("full", big)["workspace_bytes"] > tm.noalloc_max_bytes()
    L = inputs.nlimbs(big)
    z = torch.zeros(L, dtype=torch.int64, device=dev())
    o = torch.zeros(2 * L, dtype=torch.int64, device=dev())
    with pytest.raises(tm.TmulError):
        tm.mul_noalloc("full", z, z, big, o)
    # a transform length no other test builds: tables missing, refused
    n2 = 9500000  # low product N = 7 2^17: no other call here builds that length
    L2 = inputs.nlimbs(n2)
    z2 = torch.zeros(L2, dtype=torch.int64, device=dev())
    o2 = torch.zeros(L2, dtype=torch.int64, device=dev())
    with pytest.raises(tm.TmulError):
        tm.mul_noalloc("lo", z2, z2, n2, o2)
