"""GPU tests of packed batches (tm_mul_batched / tm_mul_packed): every stage
of a batch of independent multiplications runs as one launch per kernel
instance.  Each request's result and guard must be bit-identical to the
same multiplication run alone (tm_mul), and products must match the oracle
(low / full bit for bit, high within the allowed set).
"""
import ctypes
import sys

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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def guards_of(buf, count):
    tm = _tm()
    raw = bytes(buf.cpu().numpy().tobytes())
    sz = ctypes.sizeof(tm.Guard)
    return [tm.Guard.from_buffer_copy(raw[i * sz:(i + 1) * sz]) for i in range(count)]


def alone(kind, du, dv, n):
    tm = _tm()
    g = tm.new_guard(dev())
    out = tm.mul(kind, du, dv, n, guard=g)
    torch.cuda.synchronize()
    return to_host(out), tm.read_guard(g)


def run_batch(mix, seed, square_every=0):
    """Packed batch over mix [(kind, n)]; returns per-request
    (kind, n, u, v, packed result, packed guard, device u, device v)."""
    tm = _tm()
    reqs, ops = [], []
    for i, (kind, n) in enumerate(mix):
        u, v = inputs.operand_pair(n, seed + i)
        du = to_dev(u)
        dv = du if square_every and i % square_every == 0 else to_dev(v)
        if dv is du:
            v = u
        L = inputs.nlimbs(n)
        out = torch.zeros(2 * L if kind == "full" else L, dtype=torch.int64, device=dev())
        reqs.append((kind, du, dv, n, out))
        ops.append((u, v))
    gbuf = torch.zeros(len(mix) * ctypes.sizeof(tm.Guard), dtype=torch.uint8, device=dev())
    tm.mul_batched(reqs, guards=gbuf)
    torch.cuda.synchronize()
    gs = guards_of(gbuf, len(mix))
    return [(k, n, ops[i][0], ops[i][1], to_host(reqs[i][4]), gs[i], reqs[i][1], reqs[i][2])
            for i, (k, n) in enumerate(mix)]


def check_oracle(kind, u, v, n, w):
    if kind == "lo":
        assert np.array_equal(w, oracle.mul_lo(u, v, n, 8)), "low product n=%d" % n
    elif kind == "full":
        assert np.array_equal(w, oracle.mul_full(u, v, n, 8)), "full product n=%d" % n
    else:
        q, nz = oracle.mul_hi(u, v, n, 8)
        assert oracle.hi_accepts(w, q, nz), "high product n=%d" % n


def check_batch(res, oracle_every=1):
    for i, (k, n, u, v, w, g, du, dv) in enumerate(res):
        w1, g1 = alone(k, du, dv, n)
        assert np.array_equal(w, w1), "request %d (%s, n=%d) differs from tm_mul" % (i, k, n)
        assert g.as_dict() == g1.as_dict(), (i, k, n, g.as_dict(), g1.as_dict())
        assert g.flags == 0 and g.max_dist < 0.25, g.as_dict()
        if i % oracle_every == 0:
            check_oracle(k, u, v, n, w)


def test_packed_mixed_sizes_and_kinds():
    """48 requests, n log-uniform over [2^8, 2^18] bits, kinds mixed, every
    fifth one a squaring: many kernel instances per stage, several
    requests per instance."""
    mix = inputs.serving_mix(48, seed=31, log2_lo=8, log2_hi=18)
    say("[packed] mixed 48 requests")
    check_batch(run_batch(mix, seed=300, square_every=5), oracle_every=3)


def test_packed_more_than_one_group_per_instance():
    """70 requests of one shape: the stage tables split into launches of at
    most 64 requests."""
    mix = [("lo", 4096)] * 35 + [("hi", 4160)] * 35
    say("[packed] 70 requests of two shapes")
    check_batch(run_batch(mix, seed=500), oracle_every=7)


def test_packed_three_pass_split(monkeypatch):
    """Forced middle passes (Lm = 4) inside a packed batch, with ragged
    sizes; the split changes the schedule, not the products."""
    monkeypatch.setenv("TM_FORCE_LM", "4")
    tm = _tm()
    mix = [("lo", 1 << 16), ("hi", 100003), ("full", 70000), ("lo", 20000),
           ("full", 1 << 16), ("hi", 1 << 16), ("lo", 99999), ("full", 30000)]
    say("[packed] forced Lm=4", [tm.plan(k, n)["Lm"] for k, n in mix])
    check_batch(run_batch(mix, seed=700))


def test_packed_single_empty_and_tiny():
    """An empty batch, a batch of one, and the smallest sizes (routed
    through the full product) packed with larger ones."""
    tm = _tm()
    tm.mul_batched([])
    check_batch(run_batch([("full", 12345)], seed=900))
    check_batch(run_batch([("hi", 1), ("lo", 65), ("full", 1), ("lo", 1 << 14), ("hi", 64),
                           ("hi", 1 << 15)], seed=950))


def test_packed_fused_small_pass(monkeypatch):
    """A packed batch of small requests with the fused small-size pass on
    (TM_FUSED=1: one K0 workgroup per request, then K4) equals the
    four-step products, request by request, and the oracle."""
    mix = [("lo", 5000), ("hi", 20000), ("full", 3000), ("lo", 1 << 16), ("hi", 1 << 16),
           ("full", 1 << 16), ("hi", 89000), ("lo", 1100)]
    want = [r[4] for r in run_batch(mix, seed=960)]
    monkeypatch.setenv("TM_FUSED", "1")
    tm = _tm()
    say("[packed fused]", [(k, n, tm.plan(k, n)["fused"]) for k, n in mix])
    assert sum(tm.plan(k, n)["fused"] for k, n in mix) >= 6
    res = run_batch(mix, seed=960)
    for i, (k, n, u, v, w, g, du, dv) in enumerate(res):
        assert g.flags == 0
        assert np.array_equal(w, want[i]), "request %d (%s, n=%d) fused differs" % (i, k, n)
        check_oracle(k, u, v, n, w)
    monkeypatch.delenv("TM_FUSED")


def test_graph_capture_replays_match_eager():
    """tm_mul captured into a HIP graph (torch stream capture) after
    tm_prepare: every replay, with new operands copied in eagerly between
    replays, equals an eager call and the oracle.  A size whose tables do
    not exist yet is refused inside the capture, before any launch."""
    tm = _tm()
    for kind, n in (("lo", 1 << 16), ("hi", 100003), ("full", 70000)):
        say("[graph] %s n=%d" % (kind, n))
        tm.prepare(kind, n)
        L = inputs.nlimbs(n)
        du = torch.zeros(L, dtype=torch.int64, device=dev())
        dv = torch.zeros(L, dtype=torch.int64, device=dev())
        out = torch.zeros(2 * L if kind == "full" else L, dtype=torch.int64, device=dev())
        ws = torch.empty(tm.plan(kind, n)["workspace_bytes"], dtype=torch.uint8, device=dev())
        gbuf = tm.new_guard(dev())
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            tm.mul(kind, du, dv, n, out=out, workspace=ws, guard=gbuf)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            tm.mul(kind, du, dv, n, out=out, workspace=ws, guard=gbuf)
        for rep in range(3):
            u, v = inputs.operand_pair(n, 1200 + rep)
            du.copy_(to_dev(u))
            dv.copy_(to_dev(v))
            graph.replay()
            torch.cuda.synchronize()
            w = to_host(out)
            g = tm.read_guard(gbuf)
            w1, g1 = alone(kind, to_dev(u), to_dev(v), n)
            assert np.array_equal(w, w1), (kind, n, rep)
            assert g.as_dict() == g1.as_dict(), (kind, n, rep)
            check_oracle(kind, u, v, n, w)
        del graph
    # a size whose transform length no earlier test uses (M = 2^19): its
    # tables cannot be built inside a capture
    n = 9000000
    L = inputs.nlimbs(n)
    du = torch.zeros(L, dtype=torch.int64, device=dev())
    out = torch.zeros(L, dtype=torch.int64, device=dev())
    ws = torch.empty(tm.plan("lo", n)["workspace_bytes"], dtype=torch.uint8, device=dev())
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        with pytest.raises(tm.TmulError):
            tm.mul("lo", du, du, n, out=out, workspace=ws)
    torch.cuda.synchronize()
