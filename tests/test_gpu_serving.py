"""GPU tests of the continuous-batching server (tm_server_*, tm_serve_trace).

Every request's result must be the same bit for bit alone (tm_mul on the
device) and in the mix (served while other requests of other sizes and kinds
run), and low / full products must equal the oracle (high products: one of
the two allowed values).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1703_00640_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _tm():
    import paper_1703_00640_amd as tm
    return tm


def alone(kind, u, v, n):
    tm = _tm()
    d = torch.device("cuda:0")
    du = torch.from_numpy(np.ascontiguousarray(u).view(np.int64)).to(d)
    dv = torch.from_numpy(np.ascontiguousarray(v).view(np.int64)).to(d)
    out = tm.mul(kind, du, dv, n)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64)


def check_oracle(kind, u, v, n, w):
    if kind == "lo":
        assert np.array_equal(w, oracle.mul_lo(u, v, n, 8)), "low product n=%d" % n
    elif kind == "full":
        assert np.array_equal(w, oracle.mul_full(u, v, n, 8)), "full product n=%d" % n
    else:
        q, nz = oracle.mul_hi(u, v, n, 8)
        assert oracle.hi_accepts(w, q, nz), "high product n=%d" % n


def test_same_alone_and_in_the_mix():
    from paper_1703_00640_amd import serving
    mix = inputs.serving_mix(96, seed=11, log2_lo=12, log2_hi=18)
    say("serving mix: 96 requests, n in [2^12, 2^18]")
    m = serving.Mix(mix, seed=12)
    # arrivals far faster than service: requests join while others run
    arr = inputs.poisson_arrivals(len(mix), rate=2e5, seed=13)
    stats, lat, guards = serving.run(m, arr, pool_bytes=64 << 20, n_streams=4)
    say("served", stats)
    assert stats["failed"] == 0 and stats["guard_flags"] == 0
    for i, (k, n) in enumerate(mix):
        u, v = m.operands(i)
        w = m.result(i)
        assert np.array_equal(w, alone(k, u, v, n)), "request %d (%s, n=%d) differs alone" % (i, k, n)
        if i % 4 == 0:
            check_oracle(k, u, v, n, w)


def test_config_range_alone_and_in_the_mix():
    """The serving workload's full size range, n log-uniform over [2^12,
    2^22] bits with all three kinds: every request equals its result alone,
    and every third one (all kinds, up to the largest sizes) the oracle."""
    from paper_1703_00640_amd import serving
    mix = inputs.serving_mix(64, seed=31, log2_lo=12, log2_hi=22)
    say("serving mix: 64 requests, n in [2^12, 2^22], largest %d" % max(n for _, n in mix))
    m = serving.Mix(mix, seed=32)
    arr = inputs.poisson_arrivals(len(mix), rate=5e4, seed=33)
    stats, lat, guards = serving.run(m, arr, pool_bytes=256 << 20, n_streams=4)
    say("served", stats)
    assert stats["failed"] == 0 and stats["guard_flags"] == 0
    for i, (k, n) in enumerate(mix):
        u, v = m.operands(i)
        w = m.result(i)
        assert np.array_equal(w, alone(k, u, v, n)), "request %d (%s, n=%d) differs alone" % (i, k, n)
        if i % 3 == 0:
            check_oracle(k, u, v, n, w)


@pytest.mark.parametrize("graphs", [True, "auto"])
def test_graph_mode_same_results(graphs):
    """Batches captured into HIP graphs (server graph mode 1: every batch of
    two or more; "auto": batches of 16 or more) give the same results as
    alone, over the serving workload's size range with multi-request
    batches."""
    from paper_1703_00640_amd import serving
    mix = inputs.serving_mix(48, seed=41, log2_lo=12, log2_hi=22)
    say("graph mode %s: 48 requests, n in [2^12, 2^22]" % graphs)
    m = serving.Mix(mix, seed=42)
    stats, lat, guards = serving.run(m, np.zeros(len(mix)), pool_bytes=256 << 20, n_streams=2,
                                     graphs=graphs)
    say("graph mode", stats)
    assert stats["failed"] == 0 and stats["guard_flags"] == 0
    for i, (k, n) in enumerate(mix):
        u, v = m.operands(i)
        w = m.result(i)
        assert np.array_equal(w, alone(k, u, v, n)), "request %d (%s, n=%d) differs alone" % (i, k, n)
        if i % 4 == 0:
            check_oracle(k, u, v, n, w)


def test_server_submit_poll_and_small_pool():
    """Incremental API with a pool that holds about two of the largest
    requests: admission waits for memory, results stay exact, with pinned
    and pageable host buffers mixed in one batch."""
    tm = _tm()
    mix = inputs.serving_mix(24, seed=21, log2_lo=12, log2_hi=16)
    biggest = max(tm.server_footprint(k, n) for k, n in mix)
    srv = tm.Server(pool_bytes=2 * biggest + 4096, n_streams=3)
    pool, offs = inputs.operand_slices(mix, seed=22)
    bufs = {}
    for i, (k, n) in enumerate(mix):
        L = inputs.nlimbs(n)
        u = torch.from_numpy(pool[offs[i][0]:offs[i][0] + L].view(np.int64).copy())
        v = torch.from_numpy(pool[offs[i][1]:offs[i][1] + L].view(np.int64).copy())
        out = torch.zeros((2 if k == "full" else 1) * L, dtype=torch.int64)
        if i % 3:
            # pinned buffers are copied by the server's kernels; pageable
            # ones (every third request) with hipMemcpyAsync
            u, v, out = u.pin_memory(), v.pin_memory(), out.pin_memory()
        rid = srv.submit(k, u, v, n, out)
        bufs[rid] = (k, n, u, v, out)
    say("submitted", len(bufs), "pending", srv.pending())
    done = {}
    while len(done) < len(bufs):
        for rid, st, g in srv.poll():
            assert st == 0 and g.flags == 0
            done[rid] = True
    assert srv.pending() == 0
    for rid, (k, n, u, v, out) in bufs.items():
        uu, vv = u.numpy().view(np.uint64), v.numpy().view(np.uint64)
        w = out.numpy().view(np.uint64)
        assert np.array_equal(w, alone(k, uu, vv, n))
        check_oracle(k, uu, vv, n, w)
    # a request larger than the whole pool is refused, not queued forever
    big = 1 << 20
    ub = torch.zeros(inputs.nlimbs(big), dtype=torch.int64)
    with pytest.raises(tm.TmulError):
        srv.submit("full", ub, ub, big, torch.zeros(2 * inputs.nlimbs(big), dtype=torch.int64))
    srv.close()
