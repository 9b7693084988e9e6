"""Python binding of the MI355X RFR library (librfr.so).

Argument marshalling only: every step of the factorisation runs in the C++ host
core and the HIP kernels of librfr.so.  PyTorch supplies device memory and
streams for the kernel-level entry points.  Importing this package never falls
back to another implementation: if librfr.so is missing the import of the
library raises.
"""
from __future__ import annotations

import ctypes as C
import itertools
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "librfr.so")

RFR_OK = 0
RFR_EBUSY = -8
STATUS = {0: "RFR_OK", -1: "RFR_EINVAL", -2: "RFR_ENOTSQFREE", -3: "RFR_ENOMEM",
          -4: "RFR_EPRECISION", -5: "RFR_EOVERFLOW", -6: "RFR_ECANDIDATES",
          -7: "RFR_EDEVICE", -8: "RFR_EBUSY"}

# every symbol include/rfr.h declares
EXPORTS = [
    "rfr_create", "rfr_destroy", "rfr_set_candidate_cap", "rfr_factor", "rfr_factor_batch",
    "rfr_serve_start", "rfr_submit", "rfr_poll", "rfr_serve_stop", "rfr_result_free",
    "rfr_strerror", "rfr_last_error", "rfr_weights", "rfr_recombine_workspace_bytes",
    "rfr_recombine_dev", "rfr_expand_workspace_bytes", "rfr_expand_dev",
    "rfr_profile", "rfr_profile_read", "rfr_recombine_min_workspace_bytes",
    "rfr_autotune", "rfr_load_tuning", "rfr_prepare_batch", "rfr_results_pack", "rfr_results_free",
    "rfr_squarefree", "rfr_recombine_dev_noalloc", "rfr_recombine_noalloc_scratch_bytes",
    "rfr_recombine_e_workspace_bytes", "rfr_recombine_e_dev", "rfr_set_design",
]


class RFRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status
        self.name = STATUS.get(status, str(status))


class Profile(C.Structure):
    _fields_ = [("searches", C.c_uint64), ("keys", C.c_uint64), ("stage_ms", C.c_double * 6),
                ("launches", C.c_uint64), ("graph_captures", C.c_uint64), ("graph_replays", C.c_uint64)]


STAGES = ["count", "scan", "enum_partition", "tile_sort", "sort_join", "recover"]


class Result(C.Structure):
    _fields_ = [
        ("content", C.c_int64), ("nfactors", C.c_int32), ("n_elements", C.c_int32),
        ("n_real", C.c_int32), ("trace_folded", C.c_int32),
        ("degrees", C.POINTER(C.c_int32)), ("coeffs", C.POINTER(C.c_int64)),
        ("n_candidates", C.c_uint64), ("n_confirmed", C.c_uint64),
        ("t_lo", C.c_uint64), ("t_hi", C.c_uint64),
        ("ms_roots", C.c_double), ("ms_search", C.c_double), ("ms_confirm", C.c_double),
    ]


_lib = None


def lib():
    """The loaded librfr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("librfr.so not built at %s (run python -m paper_2410_15880_amd.build)" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    u64, i64, i32, sz = C.c_uint64, C.c_int64, C.c_int32, C.c_size_t
    RP = C.POINTER(Result)
    sig = {
        "rfr_create": ([C.c_int, sz, C.POINTER(P)], C.c_int),
        "rfr_destroy": ([P], None),
        "rfr_set_candidate_cap": ([P, u64], C.c_int),
        "rfr_set_design": ([P, C.c_int], C.c_int),
        "rfr_factor": ([P, C.POINTER(i64), C.c_int, C.POINTER(RP)], C.c_int),
        "rfr_factor_batch": ([P, C.c_int, C.POINTER(i64), C.POINTER(i32), C.POINTER(RP), C.POINTER(C.c_int)], C.c_int),
        "rfr_serve_start": ([P, C.c_int, C.c_int], C.c_int),
        "rfr_submit": ([P, C.POINTER(i64), C.c_int, C.POINTER(u64)], C.c_int),
        "rfr_poll": ([P, u64, C.POINTER(RP), C.POINTER(C.c_double)], C.c_int),
        "rfr_serve_stop": ([P], C.c_int),
        "rfr_result_free": ([RP], None),
        "rfr_results_pack": ([C.POINTER(RP), C.c_int, P, P, P, sz, P, sz, C.POINTER(sz), C.POINTER(sz)], C.c_int),
        "rfr_results_free": ([C.POINTER(RP), C.c_int], None),
        "rfr_squarefree": ([C.POINTER(i64), C.c_int, C.POINTER(i64), C.POINTER(i64), C.POINTER(i32),
                            C.POINTER(i32), C.POINTER(C.c_int)], C.c_int),
        "rfr_strerror": ([C.c_int], C.c_char_p),
        "rfr_last_error": ([], C.c_char_p),
        "rfr_weights": ([C.POINTER(i64), C.c_int, C.POINTER(u64), C.POINTER(i32), C.POINTER(i32),
                         C.POINTER(u64), C.POINTER(u64)], C.c_int),
        "rfr_recombine_workspace_bytes": ([C.c_int], sz),
        "rfr_recombine_min_workspace_bytes": ([C.c_int], sz),
        "rfr_recombine_dev": ([C.POINTER(u64), C.c_int, u64, u64, P, sz, P, P, u64, P], C.c_int),
        "rfr_recombine_dev_noalloc": ([C.POINTER(u64), C.c_int, u64, u64, P, P, u64, P], C.c_int),
        "rfr_recombine_noalloc_scratch_bytes": ([], sz),
        "rfr_recombine_e_workspace_bytes": ([C.c_int], sz),
        "rfr_recombine_e_dev": ([C.POINTER(u64), C.c_int, u64, u64, P, sz, P, P, u64, P], C.c_int),
        "rfr_expand_workspace_bytes": ([C.c_int], sz),
        "rfr_expand_dev": ([C.POINTER(u64), C.c_int, C.c_int, P, sz, P, P], C.c_int),
        "rfr_profile": ([P, C.c_int], C.c_int),
        "rfr_autotune": ([P, C.c_int, C.c_int, C.c_char_p], C.c_int),
        "rfr_prepare_batch": ([P, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(u64),
                               C.POINTER(C.c_int32), C.POINTER(u64), C.POINTER(u64), C.POINTER(C.c_int32),
                               C.POINTER(C.c_int)], C.c_int),
        "rfr_load_tuning": ([C.c_char_p], C.c_int),
        "rfr_profile_read": ([P, C.POINTER(Profile)], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(st: int):
    if st != RFR_OK:
        raise RFRError(st, lib().rfr_last_error().decode(errors="replace"))


def _i64(coeffs: Sequence[int]):
    """int64 array for the C ABI (raises OverflowError for values outside int64)."""
    arr = np.fromiter((int(c) for c in coeffs), dtype=np.int64)
    if arr.size == 0:
        arr = np.zeros(1, dtype=np.int64)
    return np.ctypeslib.as_ctypes(arr)


def _unpack(rp) -> dict:
    r = rp.contents
    nf = int(r.nfactors)
    degs = np.ctypeslib.as_array(r.degrees, shape=(nf,)).tolist() if nf else []
    total = sum(d + 1 for d in degs)
    co = np.ctypeslib.as_array(r.coeffs, shape=(total,)).tolist() if total else []
    facs, k = [], 0
    for d in degs:
        facs.append(tuple(co[k:k + d + 1]))
        k += d + 1
    out = {"content": int(r.content), "factors": facs, "n": int(r.n_elements), "r": int(r.n_real),
           "n_candidates": int(r.n_candidates), "n_confirmed": int(r.n_confirmed),
           "trace_folded": int(r.trace_folded),
           "t_lo": int(r.t_lo), "t_hi": int(r.t_hi), "ms_roots": r.ms_roots,
           "ms_search": r.ms_search, "ms_confirm": r.ms_confirm}
    lib().rfr_result_free(rp)
    return out


def squarefree(coeffs: Sequence[int]) -> Tuple[int, List[Tuple[Tuple[int, ...], int]]]:
    """Square-free decomposition (host, Yun): (content, [(part, multiplicity)])
    with p = content * prod part**multiplicity, parts sorted by (multiplicity,
    degree, coefficients)."""
    d = len(coeffs) - 1
    cs = _i64(coeffs)
    cont = C.c_int64()
    parts = (C.c_int64 * (2 * max(d, 0) + 2))()
    degs = (C.c_int32 * (max(d, 0) + 1))()
    mult = (C.c_int32 * (max(d, 0) + 1))()
    np_ = C.c_int()
    _check(lib().rfr_squarefree(cs, d, C.byref(cont), parts, degs, mult, C.byref(np_)))
    out, k = [], 0
    for j in range(np_.value):
        out.append((tuple(parts[k:k + degs[j] + 1]), int(mult[j])))
        k += degs[j] + 1
    return int(cont.value), out


def _flatten(polys: Sequence[Sequence[int]]):
    """Degrees (int32) and all coefficients back to back (int64) of a batch
    (raises OverflowError for values outside int64)."""
    n = len(polys)
    degs = np.fromiter((len(p) - 1 for p in polys), dtype=np.int32, count=n)
    total = int(degs.sum(dtype=np.int64)) + n
    flat = np.fromiter(itertools.chain.from_iterable(polys), dtype=np.int64, count=total)
    if flat.size == 0:
        flat = np.zeros(1, dtype=np.int64)
    return degs, flat


def _unpack_many(outs, sts, n: int) -> List:
    """(content, factors) or RFRError per entry of a batch's results (one
    flattening call instead of one conversion per result)."""
    L = lib()
    nd, nc = C.c_size_t(), C.c_size_t()
    _check(L.rfr_results_pack(outs, n, None, None, None, 0, None, 0, C.byref(nd), C.byref(nc)))
    content = np.zeros(max(n, 1), dtype=np.int64)
    nfac = np.zeros(max(n, 1), dtype=np.int32)
    dg = np.zeros(max(nd.value, 1), dtype=np.int32)
    co = np.zeros(max(nc.value, 1), dtype=np.int64)
    _check(L.rfr_results_pack(outs, n, content.ctypes.data, nfac.ctypes.data, dg.ctypes.data, dg.size,
                              co.ctypes.data, co.size, C.byref(nd), C.byref(nc)))
    st = np.ctypeslib.as_array(sts, shape=(max(n, 1),))[:n].tolist()
    content, nfac, dg, co = content.tolist(), nfac.tolist(), dg.tolist(), co.tolist()
    res, kd, kc = [], 0, 0
    for i in range(n):
        if st[i] != RFR_OK:
            res.append(RFRError(st[i], "batch entry %d" % i))
            continue
        facs = []
        for d in dg[kd:kd + nfac[i]]:
            facs.append(tuple(co[kc:kc + d + 1]))
            kc += d + 1
        kd += nfac[i]
        res.append((content[i], facs))
    return res


TUNING_PATH = os.path.join(_PKG, "tuning", "mi355x.txt")


def load_tuning(path: str = TUNING_PATH):
    _check(lib().rfr_load_tuning(path.encode()))


def weights(coeffs: Sequence[int]) -> dict:
    """Host stage only: elements' weights and the accept window (no GPU needed)."""
    d = len(coeffs) - 1
    w = (C.c_uint64 * max(d, 1))()
    n, r = C.c_int32(), C.c_int32()
    tlo, thi = C.c_uint64(), C.c_uint64()
    _check(lib().rfr_weights(_i64(coeffs), d, w, C.byref(n), C.byref(r), C.byref(tlo), C.byref(thi)))
    return {"w": [int(w[i]) for i in range(n.value)], "n": n.value, "r": r.value,
            "t_lo": tlo.value, "t_hi": thi.value}


class Context:
    """One device context (plain, batched and served factorisation)."""

    def __init__(self, device: int = 0, mem_budget: int = 0, cap: Optional[int] = None):
        self._h = C.c_void_p()
        _check(lib().rfr_create(device, mem_budget, C.byref(self._h)))
        if cap is not None:
            _check(lib().rfr_set_candidate_cap(self._h, cap))

    def close(self):
        if self._h:
            lib().rfr_destroy(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def factor_full(self, coeffs: Sequence[int]) -> dict:
        rp = C.POINTER(Result)()
        _check(lib().rfr_factor(self._h, _i64(coeffs), len(coeffs) - 1, C.byref(rp)))
        return _unpack(rp)

    def factor(self, coeffs: Sequence[int]) -> Tuple[int, List[Tuple[int, ...]]]:
        r = self.factor_full(coeffs)
        return r["content"], r["factors"]

    def factor_batch(self, polys: Sequence[Sequence[int]]) -> List:
        """List of (content, factors) or RFRError per polynomial."""
        n = len(polys)
        degs, flat = _flatten(polys)
        outs = (C.POINTER(Result) * max(n, 1))()
        sts = (C.c_int * max(n, 1))()
        _check(lib().rfr_factor_batch(self._h, n, flat.ctypes.data_as(C.POINTER(C.c_int64)),
                                      degs.ctypes.data_as(C.POINTER(C.c_int32)), outs, sts))
        try:
            return _unpack_many(outs, sts, n)
        finally:
            lib().rfr_results_free(outs, n)

    def prepare_batch(self, polys: Sequence[Sequence[int]]) -> List:
        """Host stages of the batched path with device roots: per polynomial a
        dict (w, n, t_lo, t_hi, device_roots) or an RFRError."""
        n = len(polys)
        flat = [int(c) for p in polys for c in p]
        degs = [len(p) - 1 for p in polys]
        w = (C.c_uint64 * max(sum(degs), 1))()
        nn = (C.c_int32 * n)()
        tlo = (C.c_uint64 * n)()
        thi = (C.c_uint64 * n)()
        dr = (C.c_int32 * n)()
        sts = (C.c_int * n)()
        _check(lib().rfr_prepare_batch(self._h, n, _i64(flat), (C.c_int32 * n)(*degs), w, nn, tlo, thi, dr, sts))
        out, off = [], 0
        for i in range(n):
            if sts[i] == RFR_OK:
                out.append({"w": [int(w[off + k]) for k in range(nn[i])], "n": nn[i], "t_lo": tlo[i],
                            "t_hi": thi[i], "device_roots": bool(dr[i])})
            else:
                out.append(RFRError(sts[i], "batch entry %d" % i))
            off += degs[i]
        return out

    # ---- tuning
    def autotune(self, lg_lo: int = 12, lg_hi: int = 27, path: Optional[str] = None):
        """Time every radix split per size class (halves of 2^lg keys, lg in
        [8, 32]; lg = 32 needs about 80 GB of tables) on this device; install
        the best."""
        _check(lib().rfr_autotune(self._h, lg_lo, lg_hi, path.encode() if path else None))

    def set_design(self, design: int):
        """Search design of the plain and served paths: 0 per size class (tuning
        table), 1 Horowitz-Sahni (Algorithm C), 2 the query design (Algorithm E)."""
        _check(lib().rfr_set_design(self._h, design))

    # ---- profiling
    def profile(self, enable: bool = True):
        _check(lib().rfr_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        pr = Profile()
        _check(lib().rfr_profile_read(self._h, C.byref(pr)))
        return {"searches": int(pr.searches), "keys": int(pr.keys), "launches": int(pr.launches),
                "graph_captures": int(pr.graph_captures), "graph_replays": int(pr.graph_replays),
                "stage_ms": {k: float(pr.stage_ms[i]) for i, k in enumerate(STAGES)}}

    # ---- serving
    def serve_start(self, max_active: int = 8, host_threads: int = 16):
        _check(lib().rfr_serve_start(self._h, max_active, host_threads))

    def submit(self, coeffs: Sequence[int]) -> int:
        t = C.c_uint64()
        _check(lib().rfr_submit(self._h, _i64(coeffs), len(coeffs) - 1, C.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """None while running; else (result dict or RFRError, latency_ms)."""
        rp = C.POINTER(Result)()
        lat = C.c_double()
        st = lib().rfr_poll(self._h, ticket, C.byref(rp), C.byref(lat))
        if st == RFR_EBUSY:
            return None
        if st != RFR_OK:
            return RFRError(st, lib().rfr_last_error().decode(errors="replace")), lat.value
        return _unpack(rp), lat.value

    def serve_stop(self):
        _check(lib().rfr_serve_stop(self._h))


# ---------------------------------------------------------------- kernel level


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def recombine_dev(w: Sequence[int], t_lo: int, t_hi: int, cap: int = 4096, stream=None,
                  workspace=None, sync: bool = True, ws_bytes: Optional[int] = None):
    """Search on the device over caller-owned torch buffers.

    Returns the list of patterns s (ints, bit i = element i of the first n-1),
    or raises RFRError(RFR_ECANDIDATES) when the capacity overflowed.
    """
    import numpy as np
    import torch
    n = len(w)
    L = lib()
    if ws_bytes is None:
        ws_bytes = L.rfr_recombine_workspace_bytes(n)
    if workspace is None:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device="cuda")
    cand = torch.empty(2 * cap, dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    wv = (C.c_uint64 * n)(*[int(x) & ((1 << 64) - 1) for x in w])
    _check(L.rfr_recombine_dev(wv, n, t_lo, t_hi, C.c_void_p(workspace.data_ptr()), workspace.numel(),
                               _stream_ptr(stream), C.c_void_p(cand.data_ptr()), cap,
                               C.c_void_p(count.data_ptr())))
    if not sync:
        return cand, count, workspace
    torch.cuda.synchronize()
    cnt = int(count.cpu().numpy().view(np.uint64)[0])
    if cnt == (1 << 64) - 1:
        raise RFRError(-6, "candidate capacity exceeded")
    arr = cand[: 2 * cnt].cpu().numpy().view(np.uint64).reshape(-1, 2)
    na = (n - 1 + 1) // 2
    return sorted(int(a) | (int(b) << na) for a, b in arr)


def recombine_dev_noalloc(w: Sequence[int], t_lo: int, t_hi: int, cand, count, stream=None):
    """The search through the allocation-free entry point: `cand` (2*cap int64)
    and `count` (one int64) are caller-owned device tensors; the call only
    enqueues work on `stream` (read `count` after synchronising)."""
    n = len(w)
    cap = cand.numel() // 2
    wv = (C.c_uint64 * n)(*[int(x) & ((1 << 64) - 1) for x in w])
    _check(lib().rfr_recombine_dev_noalloc(wv, n, t_lo, t_hi, _stream_ptr(stream), C.c_void_p(cand.data_ptr()),
                                           cap, C.c_void_p(count.data_ptr())))


def recombine_e_dev(w: Sequence[int], t_lo: int, t_hi: int, cap: int = 4096, stream=None):
    """The search by the query design (Algorithm E variant) over torch buffers:
    the sorted list of patterns, RFRError(RFR_ECANDIDATES) on overflow, or
    None when B''s sums were too clustered for the design (use recombine_dev)."""
    import numpy as np
    import torch
    n = len(w)
    L = lib()
    ws_bytes = L.rfr_recombine_e_workspace_bytes(n)
    if ws_bytes == 0:
        raise RFRError(-1, "n out of range for the query design")
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    cand = torch.empty(2 * cap, dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    wv = (C.c_uint64 * n)(*[int(x) & ((1 << 64) - 1) for x in w])
    _check(L.rfr_recombine_e_dev(wv, n, t_lo, t_hi, C.c_void_p(ws.data_ptr()), ws_bytes, _stream_ptr(stream),
                                 C.c_void_p(cand.data_ptr()), cap, C.c_void_p(count.data_ptr())))
    torch.cuda.synchronize()
    if int(count.cpu().numpy().view(np.uint64)[0]) == (1 << 64) - 2:
        return None
    return read_patterns(n, cand, count)


def read_patterns(n: int, cand, count):
    """Patterns of a finished search (cand/count as filled by the device
    entry points), sorted; raises RFRError(RFR_ECANDIDATES) on overflow."""
    import numpy as np
    cnt = int(count.cpu().numpy().view(np.uint64)[0])
    if cnt == (1 << 64) - 1:
        raise RFRError(-6, "candidate capacity exceeded")
    arr = cand[: 2 * cnt].cpu().numpy().view(np.uint64).reshape(-1, 2)
    na = (n - 1 + 1) // 2
    return sorted(int(a) | (int(b) << na) for a, b in arr)


def expand_dev(w: Sequence[int], negate: bool = False, stream=None):
    """EXPAND on the device: sorted subset sums of w as a numpy uint64 array."""
    import numpy as np
    import torch
    m = len(w)
    L = lib()
    ws_bytes = L.rfr_expand_workspace_bytes(m)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device="cuda")
    out = torch.empty(1 << m, dtype=torch.int64, device="cuda")
    wv = (C.c_uint64 * m)(*[int(x) & ((1 << 64) - 1) for x in w])
    _check(L.rfr_expand_dev(wv, m, 1 if negate else 0, C.c_void_p(ws.data_ptr()), ws.numel(),
                            _stream_ptr(stream), C.c_void_p(out.data_ptr())))
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64)
