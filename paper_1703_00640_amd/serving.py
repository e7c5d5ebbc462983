"""Mixed-request serving runs through the library's continuous-batching
server (``tm_serve_trace``): marshalling of a request mix into pinned host
buffers, and latency / throughput statistics of a replayed arrival trace.
"""
import numpy as np
import torch

from . import inputs, nlimbs, serve_trace


class Mix:
    """A request mix with its operands and result buffers in pinned host
    memory.  Request i reads u, v as windows of one random limb pool and
    writes its own slice of one result buffer."""

    def __init__(self, mix, seed):
        self.mix = list(mix)
        pool, offs = inputs.operand_slices(self.mix, seed)
        self.pool = torch.from_numpy(pool.view(np.int64)).pin_memory()
        sizes = [(2 if k == "full" else 1) * nlimbs(n) for k, n in self.mix]
        self.out_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        self.out = torch.zeros(int(self.out_off[-1]), dtype=torch.int64).pin_memory()
        self.offs = offs
        self.requests = []
        for i, (k, n) in enumerate(self.mix):
            L = nlimbs(n)
            ou, ov = offs[i]
            self.requests.append((k, self.pool[ou:ou + L], self.pool[ov:ov + L], n,
                                  self.out[int(self.out_off[i]):int(self.out_off[i + 1])]))

    def operands(self, i):
        """(u, v) of request i as numpy uint64 arrays (copies)."""
        _, u, v, _, _ = self.requests[i]
        return u.numpy().view(np.uint64).copy(), v.numpy().view(np.uint64).copy()

    def result(self, i):
        return self.requests[i][4].numpy().view(np.uint64).copy()

    def total_bits(self):
        return sum(n for _, n in self.mix)


def run(mix, arrival_s, pool_bytes=1 << 30, n_streams=4, max_inflight=0, graphs=False):
    """Replay ``arrival_s`` over a Mix (graphs: batches as captured HIP
    graphs); returns a dict of statistics and the per-request latencies and
    guards."""
    lat, guards, makespan = serve_trace(mix.requests, arrival_s, pool_bytes, n_streams,
                                        max_inflight, graphs)
    lat = np.array(lat)
    ok = lat >= 0
    return {
        "requests": len(lat),
        "failed": int((~ok).sum()),
        "makespan_s": makespan,
        "throughput_rps": len(lat) / makespan,
        "operand_mbit_s": mix.total_bits() / makespan / 1e6,
        "p50_ms": float(np.percentile(lat[ok], 50) * 1e3) if ok.any() else None,
        "p99_ms": float(np.percentile(lat[ok], 99) * 1e3) if ok.any() else None,
        "max_guard_dist": max(g.max_dist for g in guards),
        "guard_flags": int(np.bitwise_or.reduce([g.flags for g in guards])),
    }, lat, guards
