"""Truncated integer multiplication on AMD MI355X: Python binding of libtmul.

Thin ctypes marshalling over the C ABI in ``include/tmul.h``: every step of
the computation runs in the library's HIP kernels.  PyTorch provides device
memory and streams only.  Operands are contiguous ``torch.uint64`` (or
``torch.int64``, same bits) tensors of ``ceil(n/64)`` little-endian limbs on
one GPU.

The library must have been built (``paper_1703_00640_amd.build.build()`` or
``__graft_entry__.build()``); importing works without it, calling does not.
"""
import ctypes
import os

import torch

__all__ = ["mul", "mul_lo", "mul_hi", "mul_full", "mul_batched", "mul_checked",
           "coefficients", "profile_stages", "plan", "workspace_bytes", "Guard",
           "TmulError", "KINDS", "library_path", "prepare", "Server", "serve_trace",
           "server_footprint", "autotune", "mulmod", "mul_noalloc", "noalloc_max_bytes"]

KINDS = {"full": 0, "lo": 1, "hi": 2}
_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libtmul.so")
_lib = None


class TmulError(RuntimeError):
    pass


class Guard(ctypes.Structure):
    """Rounding guard written by every multiplication (see tmul.h)."""
    _fields_ = [("max_dist", ctypes.c_double), ("max_abs", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("b", ctypes.c_uint32),
                ("lam", ctypes.c_uint32), ("kind", ctypes.c_uint32),
                ("N", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class _PlanInfo(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("via_full", ctypes.c_uint32),
                ("b", ctypes.c_uint32), ("lam", ctypes.c_uint32),
                ("n_bits", ctypes.c_uint64), ("N", ctypes.c_uint64),
                ("digits", ctypes.c_uint64), ("M", ctypes.c_uint64),
                ("L1", ctypes.c_uint32), ("L2", ctypes.c_uint32),
                ("workspace_bytes", ctypes.c_uint64), ("Lm", ctypes.c_uint32),
                ("guaranteed", ctypes.c_uint32), ("rounding_bound", ctypes.c_double),
                ("fused", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class _Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("n_bits", ctypes.c_uint64), ("u", ctypes.c_void_p),
                ("v", ctypes.c_void_p), ("w", ctypes.c_void_p)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(library_path):
        raise TmulError("libtmul.so is not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(library_path)
    P = ctypes.c_void_p
    U64, SZ, I32 = ctypes.c_uint64, ctypes.c_size_t, ctypes.c_int
    lib.tm_workspace_bytes.argtypes = [I32, U64]
    lib.tm_workspace_bytes.restype = SZ
    lib.tm_workspace_bytes_checked.argtypes = [I32, U64]
    lib.tm_workspace_bytes_checked.restype = SZ
    lib.tm_workspace_bytes_batched.argtypes = [P, SZ]
    lib.tm_workspace_bytes_batched.restype = SZ
    lib.tm_plan_query.argtypes = [I32, U64, ctypes.POINTER(_PlanInfo)]
    lib.tm_autotune.argtypes = [I32, U64, P, ctypes.POINTER(_PlanInfo)]
    lib.tm_autotune.restype = I32
    lib.tm_plan_query_guaranteed.argtypes = [I32, U64, ctypes.POINTER(_PlanInfo)]
    lib.tm_plan_query_guaranteed.restype = I32
    lib.tm_workspace_bytes_guaranteed.argtypes = [I32, U64]
    lib.tm_workspace_bytes_guaranteed.restype = SZ
    lib.tm_mul_guaranteed.argtypes = [I32, P, P, P, U64, P, SZ, P, P]
    lib.tm_mul_guaranteed.restype = I32
    lib.tm_workspace_bytes_fp32c.argtypes = [I32, U64]
    lib.tm_workspace_bytes_fp32c.restype = SZ
    lib.tm_plan_query_fp32c.argtypes = [I32, U64, ctypes.POINTER(_PlanInfo)]
    lib.tm_plan_query_fp32c.restype = I32
    lib.tm_mul_fp32c.argtypes = [I32, P, P, P, U64, P, SZ, P, P]
    lib.tm_mul_fp32c.restype = I32
    lib.tm_coefficients_fp32c.argtypes = [I32, P, P, U64, P, P, U64, P, SZ, P, P]
    lib.tm_coefficients_fp32c.restype = I32
    lib.tm_mul.argtypes = [I32, P, P, P, U64, P, SZ, P, P]
    for name in ("tm_mul_full", "tm_mul_lo", "tm_mul_hi"):
        getattr(lib, name).argtypes = [P, P, P, U64, P, SZ, P, P]
    lib.tm_mul_batched.argtypes = [P, SZ, P, SZ, P, P]
    lib.tm_batch_meta_bytes.argtypes = [SZ]
    lib.tm_batch_meta_bytes.restype = SZ
    lib.tm_mul_packed.argtypes = [P, SZ, P, P, P, SZ, P, P]
    lib.tm_mul_packed.restype = I32
    lib.tm_mul_checked.argtypes = [I32, P, P, P, U64, P, SZ, P, ctypes.POINTER(Guard)]
    lib.tm_mul_noalloc.argtypes = [I32, P, P, P, U64, P, P]
    lib.tm_mul_noalloc.restype = I32
    lib.tm_noalloc_max_bytes.argtypes = []
    lib.tm_noalloc_max_bytes.restype = SZ
    lib.tm_coefficients.argtypes = [I32, P, P, U64, P, P, U64, P, SZ, P, P]
    lib.tm_profile_stages.argtypes = [I32, P, P, P, U64, P, SZ, P,
                                      ctypes.POINTER(ctypes.c_float),
                                      ctypes.POINTER(ctypes.c_char_p), I32,
                                      ctypes.POINTER(I32)]
    for name in ("tm_plan_query", "tm_mul", "tm_mul_full", "tm_mul_lo", "tm_mul_hi",
                 "tm_mul_batched", "tm_mul_checked", "tm_coefficients", "tm_profile_stages"):
        getattr(lib, name).restype = I32
    lib.tm_workspace_bytes_mulmod.argtypes = [U64]
    lib.tm_workspace_bytes_mulmod.restype = SZ
    lib.tm_mulmod.argtypes = [P, P, P, P, P, U64, P, SZ, P]
    lib.tm_mulmod.restype = I32
    lib.tm_prepare.argtypes = [I32, U64, P]
    lib.tm_prepare.restype = I32
    lib.tm_server_footprint.argtypes = [I32, U64]
    lib.tm_server_footprint.restype = SZ
    lib.tm_server_create.argtypes = [SZ, I32, I32, ctypes.POINTER(P)]
    lib.tm_server_create.restype = I32
    lib.tm_server_submit.argtypes = [P, ctypes.POINTER(_Request), ctypes.POINTER(Guard),
                                     ctypes.POINTER(U64)]
    lib.tm_server_submit.restype = I32
    lib.tm_server_poll.argtypes = [P, ctypes.POINTER(U64), ctypes.POINTER(I32), I32]
    lib.tm_server_poll.restype = I32
    lib.tm_server_pending.argtypes = [P]
    lib.tm_server_pending.restype = SZ
    lib.tm_server_drain.argtypes = [P]
    lib.tm_server_drain.restype = I32
    lib.tm_server_destroy.argtypes = [P]
    lib.tm_server_destroy.restype = None
    lib.tm_serve_trace.argtypes = [ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_double), SZ,
                                   SZ, I32, I32, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(Guard), ctypes.POINTER(ctypes.c_double)]
    lib.tm_serve_trace.restype = I32
    lib.tm_serve_trace_ex.argtypes = lib.tm_serve_trace.argtypes + [I32]
    lib.tm_serve_trace_ex.restype = I32
    lib.tm_server_use_graphs.argtypes = [P, I32]
    lib.tm_server_use_graphs.restype = I32
    lib.tm_status_string.argtypes = [I32]
    lib.tm_status_string.restype = ctypes.c_char_p
    lib.tm_last_error.argtypes = []
    lib.tm_last_error.restype = ctypes.c_char_p
    lib.tm_release_caches.argtypes = []
    lib.tm_release_caches.restype = None
    _lib = lib
    return lib


def _check(status, what):
    if status != 0:
        lib = _load()
        raise TmulError("%s: %s (%s)" % (what, lib.tm_status_string(status).decode(),
                                          lib.tm_last_error().decode()))


def _kind(kind):
    if isinstance(kind, str):
        return KINDS[kind]
    return int(kind)


def nlimbs(n_bits):
    return (int(n_bits) + 63) // 64


def plan(kind, n_bits, guaranteed=False, fp32c=False):
    """The plan (b, lambda, N, FFT split, workspace, rounding bound) used for
    (kind, n_bits); guaranteed=True: the plan of tm_mul_guaranteed;
    fp32c=True: the plan of the FP32 path (tm_mul_fp32c)."""
    info = _PlanInfo()
    lib = _load()
    f = lib.tm_plan_query_guaranteed if guaranteed else lib.tm_plan_query_fp32c if fp32c \
        else lib.tm_plan_query
    _check(f(_kind(kind), int(n_bits), ctypes.byref(info)), "plan")
    return {k: getattr(info, k) for k, _ in _PlanInfo._fields_}


def workspace_bytes(kind, n_bits, checked=False):
    lib = _load()
    f = lib.tm_workspace_bytes_checked if checked else lib.tm_workspace_bytes
    nb = f(_kind(kind), int(n_bits))
    if nb == 0:
        raise TmulError("unsupported (kind, n_bits) = (%s, %d)" % (kind, n_bits))
    return nb


def _dev_ptr(t, L, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TmulError("%s must be a CUDA/HIP tensor" % name)
    if t.dtype not in (torch.uint64, torch.int64) or not t.is_contiguous():
        raise TmulError("%s must be a contiguous 64-bit integer tensor" % name)
    if t.numel() < L:
        raise TmulError("%s has %d limbs, needs %d" % (name, t.numel(), L))
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream, device):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def _workspace(nbytes, device, workspace):
    if workspace is None:
        return torch.empty(nbytes, dtype=torch.uint8, device=device)
    if workspace.numel() * workspace.element_size() < nbytes:
        raise TmulError("workspace too small: %d < %d bytes" % (
            workspace.numel() * workspace.element_size(), nbytes))
    return workspace


def new_guard(device):
    """A device buffer for one tm_guard (read it with read_guard)."""
    return torch.zeros(ctypes.sizeof(Guard), dtype=torch.uint8, device=device)


def read_guard(buf):
    raw = bytes(buf.detach().cpu().numpy().tobytes())
    return Guard.from_buffer_copy(raw[:ctypes.sizeof(Guard)])


def mul(kind, u, v, n_bits, out=None, workspace=None, stream=None, guard=None,
        guaranteed=False, fp32c=False):
    """w = product of ``kind`` ('lo', 'hi' or 'full') of u and v (n_bits each).

    Returns the output tensor (L limbs for lo/hi, 2L for full), enqueued on
    ``stream`` (default: torch's current stream).  ``guard`` may be a tensor
    from new_guard() to receive the rounding guard.  ``guaranteed``: use the
    digit size of the worst-case rounding bound (tm_mul_guaranteed).
    ``fp32c``: the FP32 path with double-float FFT passes (tm_mul_fp32c).
    Passing the same tensor as u and v computes a square with one forward
    transform."""
    k = _kind(kind)
    L = nlimbs(n_bits)
    dev = u.device
    pu, pv = _dev_ptr(u, L, "u"), _dev_ptr(v, L, "v")
    nout = 2 * L if k == 0 else L
    if out is None:
        out = torch.empty(nout, dtype=torch.uint64, device=dev)
    pw = _dev_ptr(out, nout, "out")
    lib = _load()
    if guaranteed or fp32c:
        nb = (lib.tm_workspace_bytes_guaranteed if guaranteed else lib.tm_workspace_bytes_fp32c)(
            k, int(n_bits))
        if nb == 0:
            raise TmulError("no %s plan for (%s, %d)" % ("guaranteed" if guaranteed else "FP32",
                                                        kind, n_bits))
    else:
        nb = workspace_bytes(k, n_bits)
    ws = _workspace(nb, dev, workspace)
    g = ctypes.c_void_p(guard.data_ptr()) if guard is not None else None
    f = lib.tm_mul_guaranteed if guaranteed else lib.tm_mul_fp32c if fp32c else lib.tm_mul
    _check(f(k, pw, pu, pv, int(n_bits), ctypes.c_void_p(ws.data_ptr()),
             ws.numel() * ws.element_size(), _stream_ptr(stream, dev), g), "tm_mul")
    return out


def mul_noalloc(kind, u, v, n_bits, out, stream=None, guard=None):
    """tm_mul_noalloc: the product into the caller's ``out`` with the
    library's static per-GPU scratch as workspace (no device allocation;
    tm_prepare the size first).  Calls overlapping on one GPU race."""
    k = _kind(kind)
    L = nlimbs(n_bits)
    dev = u.device
    nout = 2 * L if k == 0 else L
    g = ctypes.c_void_p(guard.data_ptr()) if guard is not None else None
    _check(_load().tm_mul_noalloc(k, _dev_ptr(out, nout, "out"), _dev_ptr(u, L, "u"),
                                  _dev_ptr(v, L, "v"), int(n_bits), _stream_ptr(stream, dev), g),
           "tm_mul_noalloc")
    return out


def noalloc_max_bytes():
    return _load().tm_noalloc_max_bytes()


def mul_lo(u, v, n_bits, **kw):
    return mul("lo", u, v, n_bits, **kw)


def mul_hi(u, v, n_bits, **kw):
    return mul("hi", u, v, n_bits, **kw)


def mul_full(u, v, n_bits, **kw):
    return mul("full", u, v, n_bits, **kw)


def _request_array(requests):
    arr = (_Request * len(requests))()
    for i, (kind, u, v, n_bits, out) in enumerate(requests):
        L = nlimbs(n_bits)
        k = _kind(kind)
        arr[i].kind = k
        arr[i].n_bits = int(n_bits)
        arr[i].u = _dev_ptr(u, L, "u").value
        arr[i].v = _dev_ptr(v, L, "v").value
        arr[i].w = _dev_ptr(out, 2 * L if k == 0 else L, "out").value
    return arr


def workspace_bytes_batched(requests):
    """Workspace bytes of mul_batched for ``requests`` (tm_workspace_bytes_batched)."""
    nb = _load().tm_workspace_bytes_batched(ctypes.byref(_request_array(requests)), len(requests))
    if nb == 0:
        raise TmulError("unsupported request in batch")
    return nb


def mul_batched(requests, workspace=None, stream=None, guards=None):
    """requests: list of (kind, u, v, n_bits, out) with device tensors of
    independent multiplications; runs them on one stream in packed launches
    (one launch per stage and kernel instance), each request with its own
    slice of one workspace."""
    if not requests:
        return
    arr = _request_array(requests)
    dev = requests[0][1].device
    lib = _load()
    nb = lib.tm_workspace_bytes_batched(ctypes.byref(arr), len(requests))
    if nb == 0:
        raise TmulError("unsupported request in batch")
    ws = _workspace(nb, dev, workspace)
    g = ctypes.c_void_p(guards.data_ptr()) if guards is not None else None
    _check(lib.tm_mul_batched(ctypes.byref(arr), len(requests), ctypes.c_void_p(ws.data_ptr()),
                              ws.numel() * ws.element_size(), _stream_ptr(stream, dev), g),
           "tm_mul_batched")


def mul_checked(kind, u, v, n_bits, out=None, workspace=None, stream=None):
    """Multiply, synchronise, and fall back to smaller digits if the rounding
    guard tripped.  Returns (out, Guard)."""
    k = _kind(kind)
    L = nlimbs(n_bits)
    dev = u.device
    nout = 2 * L if k == 0 else L
    if out is None:
        out = torch.empty(nout, dtype=torch.uint64, device=dev)
    ws = _workspace(workspace_bytes(k, n_bits, checked=True), dev, workspace)
    g = Guard()
    _check(_load().tm_mul_checked(k, _dev_ptr(out, nout, "out"), _dev_ptr(u, L, "u"),
                                  _dev_ptr(v, L, "v"), int(n_bits),
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                  _stream_ptr(stream, dev), ctypes.byref(g)), "tm_mul_checked")
    return out, g


def coefficients(kind, u, v, n_bits, with_x=True, workspace=None, stream=None, fp32c=False):
    """Rounded coefficients c_i (int64) and unrounded x_i (float64) of the
    plan for (kind, n_bits) (of the FP32 path with fp32c=True), plus the
    guard (synchronises)."""
    k = _kind(kind)
    L = nlimbs(n_bits)
    dev = u.device
    pl = plan(k, n_bits, fp32c=fp32c)
    ncoef = pl["N"] + (1 if (k == 2 and not pl["via_full"]) else 0)
    c = torch.empty(ncoef, dtype=torch.int64, device=dev)
    x = torch.empty(ncoef, dtype=torch.float64, device=dev) if with_x else None
    ws = _workspace(pl["workspace_bytes"], dev, workspace)
    gb = new_guard(dev)
    f = _load().tm_coefficients_fp32c if fp32c else _load().tm_coefficients
    _check(f(k, ctypes.c_void_p(c.data_ptr()),
             ctypes.c_void_p(x.data_ptr()) if x is not None else None,
             ncoef, _dev_ptr(u, L, "u"), _dev_ptr(v, L, "v"), int(n_bits),
             ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
             _stream_ptr(stream, dev), ctypes.c_void_p(gb.data_ptr())),
           "tm_coefficients")
    torch.cuda.synchronize(dev)
    return c, x, read_guard(gb)


def profile_stages(kind, u, v, n_bits, out, workspace, stream=None):
    """One multiplication with HIP events between its kernels on ``stream``;
    returns [(stage_name, ms), ...] (synchronises)."""
    k = _kind(kind)
    L = nlimbs(n_bits)
    cap = 8
    ms = (ctypes.c_float * cap)()
    names = (ctypes.c_char_p * cap)()
    nst = ctypes.c_int(0)
    nout = 2 * L if k == 0 else L
    _check(_load().tm_profile_stages(k, _dev_ptr(out, nout, "out"), _dev_ptr(u, L, "u"),
                                     _dev_ptr(v, L, "v"), int(n_bits),
                                     ctypes.c_void_p(workspace.data_ptr()),
                                     workspace.numel() * workspace.element_size(),
                                     _stream_ptr(stream, u.device), ms, names, cap,
                                     ctypes.byref(nst)), "tm_profile_stages")
    return [(names[i].decode(), float(ms[i])) for i in range(nst.value)]


# ------------------------------------------------------------------ serving

def prepare(kind, n_bits, stream=None):
    """Build the per-device caches of (kind, n_bits) now (optional)."""
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(_load().tm_prepare(_kind(kind), int(n_bits), ctypes.c_void_p(st.cuda_stream)),
           "prepare")


def autotune(kind, n_bits, stream=None, device=None):
    """Time the FFT splits of (kind, n_bits) on the GPU and keep the fastest
    for this process (tm_autotune); returns the tuned plan."""
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    info = _PlanInfo()
    _check(_load().tm_autotune(_kind(kind), int(n_bits), _stream_ptr(stream, dev),
                               ctypes.byref(info)), "autotune")
    return {k: getattr(info, k) for k, _ in _PlanInfo._fields_}


def mulmod(a, b, m, mu, n_bits, out=None, workspace=None, stream=None):
    """Barrett modular multiplication r = a b mod m on the GPU (tm_mulmod):
    a, b, m device tensors of ceil(n/64) limbs with 2^(n-1) < m < 2^n, mu of
    ceil((n+1)/64) limbs holding floor(2^(2n) / m).  Returns r (n-bit)."""
    lib = _load()
    L, L1 = nlimbs(n_bits), nlimbs(n_bits + 1)
    dev = a.device
    nb = lib.tm_workspace_bytes_mulmod(int(n_bits))
    if nb == 0:
        raise TmulError("mulmod: unsupported size %d" % n_bits)
    if out is None:
        out = torch.empty(L, dtype=torch.int64, device=dev)
    ws = _workspace(nb, dev, workspace)
    _check(lib.tm_mulmod(_dev_ptr(out, L, "out"), _dev_ptr(a, L, "a"), _dev_ptr(b, L, "b"),
                         _dev_ptr(m, L, "m"), _dev_ptr(mu, L1, "mu"), int(n_bits),
                         ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                         _stream_ptr(stream, dev)), "tm_mulmod")
    return out


def server_footprint(kind, n_bits):
    """Device pool bytes one request of (kind, n_bits) occupies in a Server."""
    nb = _load().tm_server_footprint(_kind(kind), int(n_bits))
    if nb == 0:
        raise TmulError("unsupported (kind, n_bits) = (%s, %d)" % (kind, n_bits))
    return nb


def _host_buf(t, L, name):
    if t.device.type != "cpu" or t.dtype not in (torch.uint64, torch.int64) \
            or not t.is_contiguous() or t.numel() < L:
        raise TmulError("%s must be a contiguous CPU int64/uint64 tensor of >= %d limbs" % (name, L))
    return t.data_ptr()


class Server:
    """Continuous-batching server (tm_server_* in tmul.h): requests with
    host tensors are admitted by device memory and overlap on the device.
    Keep every submitted tensor alive until its request is polled."""

    def __init__(self, pool_bytes=1 << 30, n_streams=4, max_inflight=0, graphs=False):
        lib = _load()
        h = ctypes.c_void_p()
        _check(lib.tm_server_create(int(pool_bytes), int(n_streams), int(max_inflight),
                                    ctypes.byref(h)), "server create")
        self._h = h
        self._keep = {}
        if graphs:
            _check(lib.tm_server_use_graphs(h, 2 if graphs == "auto" else 1), "server graphs")

    def submit(self, kind, u, v, n_bits, out):
        k, L = _kind(kind), nlimbs(n_bits)
        nout = 2 * L if k == 0 else L
        req = _Request(k, 0, int(n_bits), _host_buf(u, L, "u"), _host_buf(v, L, "v"),
                       _host_buf(out, nout, "out"))
        g = Guard()
        rid = ctypes.c_uint64()
        _check(_load().tm_server_submit(self._h, ctypes.byref(req), ctypes.byref(g),
                                        ctypes.byref(rid)), "submit")
        self._keep[rid.value] = (u, v, out, g)
        return rid.value

    def poll(self, cap=256):
        """[(id, status, Guard)] of requests finished since the last poll."""
        ids = (ctypes.c_uint64 * cap)()
        sts = (ctypes.c_int * cap)()
        n = _load().tm_server_poll(self._h, ids, sts, cap)
        if n < 0:
            raise TmulError("poll on a closed server")
        return [(ids[i], sts[i], self._keep.pop(ids[i])[3]) for i in range(n)]

    def pending(self):
        return _load().tm_server_pending(self._h)

    def drain(self):
        _check(_load().tm_server_drain(self._h), "drain")

    def close(self):
        if self._h:
            _load().tm_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve_trace(requests, arrival_s, pool_bytes=1 << 30, n_streams=4, max_inflight=0,
                graphs=False):
    """Replay an arrival trace (tm_serve_trace).  requests: list of
    (kind, u, v, n_bits, out) with CPU tensors (pinned for overlap).
    graphs: True runs every batch as a captured HIP graph (TM_SERVE_GRAPHS),
    "auto" only batches of 16 or more (TM_SERVE_GRAPHS_AUTO).
    Returns (latency_s list, guards list, makespan_s)."""
    lib = _load()
    cnt = len(requests)
    reqs = (_Request * cnt)()
    for i, (kind, u, v, n_bits, out) in enumerate(requests):
        k, L = _kind(kind), nlimbs(n_bits)
        reqs[i] = _Request(k, 0, int(n_bits), _host_buf(u, L, "u"), _host_buf(v, L, "v"),
                           _host_buf(out, 2 * L if k == 0 else L, "out"))
    arr = (ctypes.c_double * cnt)(*[float(a) for a in arrival_s])
    lat = (ctypes.c_double * cnt)()
    guards = (Guard * cnt)()
    mk = ctypes.c_double()
    _check(lib.tm_serve_trace_ex(reqs, arr, cnt, int(pool_bytes), int(n_streams), int(max_inflight),
                                 lat, guards, ctypes.byref(mk),
                                 2 if graphs == "auto" else 1 if graphs else 0), "serve_trace")
    return list(lat), [guards[i] for i in range(cnt)], mk.value
