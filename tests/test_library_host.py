"""Host-side checks of the HIP library (no GPU needed): it loads, exports
every entry point declared in include/tmul.h, plans every benchmark size
within the theorems' constraints, and rejects bad arguments before touching
the device."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tmul.h")
LIB = os.path.join(ROOT, "paper_1703_00640_amd", "libtmul.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libtmul.so not built")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tm_[a-z_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("tm_mul", "tm_mul_lo", "tm_mul_hi", "tm_mul_full", "tm_mul_batched",
                 "tm_workspace_bytes", "tm_plan_query", "tm_mul_checked"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name


def _plan(kind, n):
    import paper_1703_00640_amd as tm
    return tm.plan(kind, n)


def lg(x):
    return (x - 1).bit_length()


@pytest.mark.parametrize("n", [1 << 16, 1 << 24, 1 << 26, 1 << 30, 12345, 2049, 1000003])
def test_plans_satisfy_theorem_constraints(n):
    lo, hi, full = _plan("lo", n), _plan("hi", n), _plan("full", n)
    # low product: b >= 4, N >= 3, N b >= n (Theorem on the low product)
    assert lo["b"] >= 4 and lo["N"] >= 3 and lo["N"] * lo["b"] >= n
    # high product: (N + 1) b >= n + lg N + 2 (Theorem on the high product)
    assert hi["N"] * hi["b"] + hi["b"] >= n + lg(hi["N"]) + 2
    # full product: N digits with N b >= n, length 2N
    assert full["digits"] * full["b"] >= n and full["N"] == 2 * full["digits"]
    for p in (lo, hi, full):
        assert p["M"] * 2 == p["N"] and p["L1"] * p["Lm"] * p["L2"] == p["M"]
        assert p["L1"] <= 1024 or p["Lm"] == 1
        odd = p["N"]
        while odd % 2 == 0:
            odd //= 2
        assert odd in (1, 3, 5, 7)


def test_every_small_size_has_kernels():
    """Every plan for n up to 2^17 (and a sample beyond) has a row length
    with a K2 instance (16..1024) and a column length in the instance list."""
    import paper_1703_00640_amd as tm
    l1_ok = {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024,
             5, 10, 20, 40, 80, 160, 320, 640, 7, 14, 28, 56, 112, 224, 448, 896}
    sizes = list(range(1, 4097)) + list(range(4097, 1 << 17, 97)) + [10 ** 6, 3 * 10 ** 6, 10 ** 7]
    for n in sizes:
        for kind in ("lo", "hi", "full"):
            p = _plan(kind, n)
            assert 16 <= p["L2"] <= 1024 and p["L1"] in l1_ok, (kind, n, p)


def test_config_plans():
    """n = 2^24: truncated b = 11 at N = 3 * 2^19, full b = 16 at 2N = 2^21
    (transform length ratio 0.75)."""
    lo, full = _plan("lo", 1 << 24), _plan("full", 1 << 24)
    assert (lo["b"], lo["N"]) == (11, 3 << 19)
    assert (full["b"], full["N"]) == (16, 1 << 21)
    assert lo["N"] / full["N"] == 0.75
    assert 5 <= lo["lam"] <= 7


def test_small_n_routes_to_full():
    for n in (1, 64, 1000):
        assert _plan("lo", n)["via_full"] == 1
        assert _plan("hi", n)["via_full"] == 1
    assert _plan("lo", 4096)["via_full"] == 0


def test_invalid_arguments_rejected_without_gpu():
    import paper_1703_00640_amd as tm
    lib = tm._load()
    ws = tm.workspace_bytes("lo", 4096)
    # null operands
    assert lib.tm_mul(1, None, None, None, 4096, None, ws, None, None) == 1
    # bad kind, n = 0
    assert lib.tm_workspace_bytes(7, 4096) == 0
    assert lib.tm_workspace_bytes(1, 0) == 0
    info = tm._PlanInfo()
    assert lib.tm_plan_query(1, 0, ctypes.byref(info)) == 1
    assert lib.tm_status_string(3) == b"rounding guard tripped"
    assert lib.tm_autotune(7, 4096, None, None) == 1


def test_packed_batch_sizes_and_checks():
    """Workspace of a packed batch = the requests' workspaces (256-byte
    rounded) + the metadata area; malformed packed calls are rejected before
    any device work."""
    import paper_1703_00640_amd as tm
    lib = tm._load()
    mix = [("lo", 4096), ("hi", 100000), ("full", 777), ("lo", 1 << 20)]
    reqs = (tm._Request * len(mix))()
    for i, (k, n) in enumerate(mix):
        reqs[i].kind = tm._kind(k)
        reqs[i].n_bits = n
    meta = lib.tm_batch_meta_bytes(len(mix))
    assert meta > 0 and meta % 256 == 0
    assert lib.tm_batch_meta_bytes(64) >= lib.tm_batch_meta_bytes(4)
    want = sum((tm.workspace_bytes(k, n) + 255) // 256 * 256 for k, n in mix) + meta
    assert lib.tm_workspace_bytes_batched(ctypes.byref(reqs), len(mix)) == want
    reqs[1].kind = 9
    assert lib.tm_workspace_bytes_batched(ctypes.byref(reqs), len(mix)) == 0
    reqs[1].kind = 2
    ws = (ctypes.c_void_p * len(mix))()
    wsb = (ctypes.c_size_t * len(mix))()
    # empty batch: nothing to do
    assert lib.tm_mul_packed(None, 0, None, None, None, 0, None, None) == 0
    assert lib.tm_mul_batched(None, 0, None, 0, None, None) == 0
    # null metadata / workspace arrays, misaligned or short metadata area
    assert lib.tm_mul_packed(ctypes.byref(reqs), len(mix), ws, wsb, None, meta, None, None) == 1
    assert lib.tm_mul_packed(ctypes.byref(reqs), len(mix), None, wsb, 256, meta, None, None) == 1
    assert lib.tm_mul_packed(ctypes.byref(reqs), len(mix), ws, wsb, 260, meta, None, None) == 1
    assert lib.tm_mul_packed(ctypes.byref(reqs), len(mix), ws, wsb, 256, meta - 256, None, None) == 1
    # a request with null operands
    assert lib.tm_mul_packed(ctypes.byref(reqs), len(mix), ws, wsb, 256, meta, None, None) == 1
    assert lib.tm_mul_batched(ctypes.byref(reqs), len(mix), None, 1 << 30, None, None) == 1


def test_mulmod_host_checks():
    """Barrett modular multiplication: workspace sizes (0 below two bits,
    growing with n) and argument checks before any device work."""
    import paper_1703_00640_amd as tm
    lib = tm._load()
    assert lib.tm_workspace_bytes_mulmod(0) == 0 and lib.tm_workspace_bytes_mulmod(1) == 0
    small, big = lib.tm_workspace_bytes_mulmod(2), lib.tm_workspace_bytes_mulmod(1 << 20)
    assert 0 < small < big and big % 256 == 0
    # the workspace holds the largest of the three products' workspaces
    assert big >= max(tm.workspace_bytes("full", 1 << 20), tm.workspace_bytes("hi", (1 << 20) + 1),
                      tm.workspace_bytes("lo", (1 << 20) + 2))
    assert lib.tm_mulmod(None, None, None, None, None, 521, None, 0, None) == 1
    assert lib.tm_mulmod(8, 8, 8, 8, 8, 1, 256, 1 << 20, None) == 1          # n < 2
    assert lib.tm_mulmod(8, 8, 8, 8, 8, 521, 256, 16, None) == 1             # workspace too small
    assert lib.tm_mulmod(8, 8, 8, 8, 8, 521, 260, 1 << 20, None) == 1        # misaligned workspace


def test_three_pass_split_for_large_n():
    """n = 2^30: M = L1 * Lm * L2 with a middle pass; n = 2^24 stays two-pass."""
    lo, full = _plan("lo", 1 << 30), _plan("full", 1 << 30)
    assert (lo["L1"], lo["Lm"], lo["L2"]) == (768, 64, 1024)
    assert (full["L1"], full["Lm"], full["L2"]) == (1024, 64, 1024)
    assert lo["N"] / full["N"] == 0.75
    assert _plan("lo", 1 << 24)["Lm"] == 1 and _plan("full", 1 << 24)["Lm"] == 1


def test_server_host_checks():
    """Footprints and argument checks of the serving entry points (no GPU
    work: every call below returns before touching the device)."""
    import paper_1703_00640_amd as tm
    lib = tm._load()
    for kind, n in (("lo", 1 << 22), ("hi", 4096), ("full", 1 << 20)):
        fp = tm.server_footprint(kind, n)
        L = (n + 63) // 64
        assert fp >= tm.workspace_bytes(kind, n) + (4 if kind == "full" else 3) * 8 * L
        assert fp % 256 == 0
    h = ctypes.c_void_p()
    assert lib.tm_server_create(0, 4, 0, ctypes.byref(h)) == 1
    assert lib.tm_server_create(1 << 20, 0, 0, ctypes.byref(h)) == 1
    assert lib.tm_server_create(1 << 20, 2, -1, ctypes.byref(h)) == 1
    assert lib.tm_server_poll(None, None, None, 0) == -1
    assert lib.tm_server_pending(None) == 0
    # arrivals must be non-decreasing
    reqs = (tm._Request * 2)()
    arr = (ctypes.c_double * 2)(1.0, 0.5)
    lat = (ctypes.c_double * 2)()
    assert lib.tm_serve_trace(reqs, arr, 2, 1 << 20, 2, 0, lat, None, None) == 1


def test_guaranteed_plans():
    """Guaranteed mode: the largest digit size whose worst-case rounding
    bound is below 0.45; sizes shrink as n grows, and where no b >= 8
    qualifies the size is refused, never silently planned."""
    import paper_1703_00640_amd as tm
    prev = {"lo": 99, "hi": 99, "full": 99}
    for lg in range(12, 23):
        n = 1 << lg
        for kind in ("lo", "hi", "full"):
            try:
                g = tm.plan(kind, n, guaranteed=True)
            except tm.TmulError:
                assert kind == "hi" and lg >= 22
                continue
            assert g["guaranteed"] == 1 and 0 < g["rounding_bound"] <= 0.45
            assert 8 <= g["b"] <= tm.plan(kind, n)["b"] and g["b"] <= prev[kind]
            prev[kind] = g["b"]
    with pytest.raises(tm.TmulError):
        tm.plan("lo", 1 << 24, guaranteed=True)
    assert tm.plan("full", 1 << 30, guaranteed=True)["b"] >= 8
    # the statistical defaults are not covered by the worst-case bound at
    # large n (the rounding guard covers them instead)
    assert tm.plan("lo", 1 << 24)["guaranteed"] == 0
    assert tm._load().tm_workspace_bytes_guaranteed(1, 1 << 24) == 0


@pytest.mark.parametrize("log2n", [16, 20, 24, 26, 30])
def test_checked_workspace_covers_an_exact_fallback(log2n):
    """tm_mul_checked always has a fallback that is exact by its bound: the
    guaranteed truncated plan where one exists (up to about 2^22 bits), else
    the full product's guaranteed plan, whose workspace (two spectra of its
    length) tm_workspace_bytes_checked must cover."""
    import paper_1703_00640_amd as tm
    n = 1 << log2n
    gf = tm.plan("full", n, guaranteed=True)
    assert gf["guaranteed"] == 1 and gf["rounding_bound"] <= 0.45
    for kind in ("lo", "hi", "full"):
        need = tm.workspace_bytes(kind, n, checked=True)
        assert need >= tm.workspace_bytes(kind, n)
        try:
            g = tm.plan(kind, n, guaranteed=True)
        except tm.TmulError:
            g = None
        if g is not None and (kind == "full" or g["b"] < tm.plan(kind, n)["b"]):
            assert need >= g["workspace_bytes"]
        else:
            assert kind != "full" or g is None or g["b"] >= tm.plan(kind, n)["b"]
            assert need >= 2 * gf["M"] * 16


def test_odd_factor_in_rows_split(monkeypatch):
    """Forcing the odd factor into the row length: at n = 2^30 with Lm = 256
    the truncated products split 256 x 256 x 768 and the full product (a
    power-of-two length) keeps its own split; lengths whose odd factor has no
    row instance (5, 7) are refused."""
    import paper_1703_00640_amd as tm
    n = 1 << 30
    monkeypatch.setenv("TM_FORCE_ODD_ROW", "1")
    monkeypatch.setenv("TM_FORCE_LM", "256")
    for kind in ("lo", "hi"):
        p = tm.plan(kind, n)
        assert (p["L1"], p["Lm"], p["L2"]) == (256, 256, 768)
    p = tm.plan("full", n)
    assert p["L1"] * p["Lm"] * p["L2"] == p["M"] and p["L2"] & (p["L2"] - 1) == 0
    monkeypatch.delenv("TM_FORCE_LM")
    p = tm.plan("lo", 1 << 20)
    assert (p["L1"], p["Lm"], p["L2"]) == (64, 1, 768)
    with pytest.raises(tm.TmulError):
        tm.plan("lo", 3000000)  # N = 5 2^16


def test_fp32c_plans():
    """Digit sizes 9 (truncated) and 13 (full), power-of-two lengths, the
    theorems' size constraints (Nb >= n low, (N+1)b >= n + lg N + 2 high)."""
    import paper_1703_00640_amd as tm
    for n in (5000, 1 << 16, 100003, 1 << 22, 1 << 26, 1 << 30):
        for kind in ("lo", "hi", "full"):
            p = tm.plan(kind, n, fp32c=True)
            if p["via_full"]:
                continue
            N, b = p["N"], p["b"]
            assert N & (N - 1) == 0 and p["L1"] * p["Lm"] * p["L2"] == p["M"]
            assert b == (13 if kind == "full" else 9)
            if kind == "lo":
                assert N * b >= n
            elif kind == "hi":
                assert (N + 1) * b >= n + (N - 1).bit_length() + 2
