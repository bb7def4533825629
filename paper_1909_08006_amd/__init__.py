"""Python binding of the MI355X record sorter (``lib/libleyenda.so``).

Argument marshalling only: every step of every sort runs in the HIP library
(``csrc/``) behind the C ABI declared in ``include/leyenda.h``.  PyTorch
supplies device memory, pinned host memory and streams.  There is no CPU
fallback: if the library is missing, :func:`load` raises.

Records are 100 bytes (10-byte key, 90-byte value, Section 4.1 of the paper);
tensors are ``torch.uint8`` of shape ``(n, 100)`` (or flat, ``n * 100``).
"""
from __future__ import annotations

import atexit
import ctypes
import os
from typing import Iterable, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libleyenda.so")
RECORD_BYTES = 100
KEY_BYTES = 10
MAX_LEVELS = 20  # LEYENDA_MAX_LEVELS: partition levels of the narrowest (4-bit) digit

_lib = None

STATUS = {0: "LEYENDA_OK", -1: "LEYENDA_EINVAL", -2: "LEYENDA_ENOMEM", -3: "LEYENDA_EBUDGET",
          -4: "LEYENDA_EHIP", -5: "LEYENDA_ETOOBIG", -6: "LEYENDA_EINTERNAL"}


class LeyendaError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")


class Params(ctypes.Structure):
    _fields_ = [("digit_bits", ctypes.c_uint32), ("tile_items", ctypes.c_uint32),
                ("big_threshold", ctypes.c_uint32), ("tiny_threshold", ctypes.c_uint32),
                ("local_capacity", ctypes.c_uint32), ("scatter_threads", ctypes.c_uint32),
                ("local_threads", ctypes.c_uint32), ("first_pass", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_uint32), ("segments", ctypes.c_uint32 * MAX_LEVELS),
                ("moved", ctypes.c_uint64 * MAX_LEVELS), ("tasks", ctypes.c_uint64), ("guard", ctypes.c_uint32)]


class Segment(ctypes.Structure):
    _fields_ = [("inp", ctypes.c_void_p), ("out", ctypes.c_void_p), ("n", ctypes.c_uint64)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("slots", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("max_batch_records", ctypes.c_uint64), ("batched", ctypes.c_int32)]


class Done(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("out_dev", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("submit_s", ctypes.c_double), ("start_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("status", ctypes.c_int32)]


def load():
    """Load the HIP library (built by ``build.py``); raise if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    P64 = ctypes.POINTER(ctypes.c_uint64)
    sig = {
        "leyenda_sort": ([vp, u64, vp, vp], i32),
        "leyenda_sort_noalloc": ([vp, u64, vp, vp], i32),
        "leyenda_noalloc_max_records": ([], u64),
        "leyenda_sort_keyed": ([vp, u64, ctypes.c_uint32, vp, vp], i32),
        "leyenda_workspace_bytes": ([u64], u64),
        "leyenda_sort_parts": ([u64], ctypes.c_uint32),
        "leyenda_first_pass": ([u64], ctypes.c_uint32),
        "leyenda_sort_runs": ([vp, u64, u64, vp, P64, u64, P64, vp], i32),
        "leyenda_merge": ([vp, P64, u64, vp, u64, vp], i32),
        "leyenda_sort_external_keys": ([vp, u64, u64, vp, vp], i32),
        "leyenda_sort_external": ([vp, u64, u64, vp, vp, vp], i32),
        "leyenda_plan_runs": ([u64, u64, P64, P64], i32),
        "leyenda_plan_external": ([u64, u64, P64, P64, P64], i32),
        "leyenda_sort_batch": ([ctypes.POINTER(Segment), u64, vp], i32),
        "leyenda_get_params": ([ctypes.POINTER(Params)], i32),
        "leyenda_set_params": ([ctypes.POINTER(Params)], i32),
        "leyenda_load_params": ([ctypes.c_char_p], i32),
        "leyenda_sort_stats": ([vp, ctypes.POINTER(Stats)], i32),
        "leyenda_status_string": ([i32], ctypes.c_char_p),
        "leyenda_last_error": ([], ctypes.c_char_p),
        "leyenda_release_workspaces": ([], i32),
        "leyenda_debug_extract": ([vp, u64, ctypes.c_uint32, vp, vp, vp, vp], i32),
        "leyenda_debug_gather": ([vp, u64, vp, u64, vp, vp], i32),
        "leyenda_debug_first_pass": ([vp, u64, ctypes.c_uint32, ctypes.c_uint32, vp, vp, vp, vp, vp], i32),
        "leyenda_server_create": ([ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)], i32),
        "leyenda_server_submit": ([vp, vp, u64, u64], i32),
        "leyenda_server_poll": ([vp, ctypes.POINTER(Done), u64, P64, ctypes.c_double], i32),
        "leyenda_server_release": ([vp, u64], i32),
        "leyenda_server_destroy": ([vp], i32),
        "leyenda_serve_replay": ([ctypes.POINTER(ServerConfig), u64, ctypes.POINTER(vp), P64,
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)], i32),
        "leyenda_host_alloc": ([u64, ctypes.POINTER(vp)], i32),
        "leyenda_host_free": ([vp], i32),
        "leyenda_profile_enable": ([i32], i32),
        "leyenda_profile_read": ([ctypes.POINTER(ctypes.c_double), P64], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    # registered after torch's own exit handlers, so it runs before them
    atexit.register(_release_at_exit)
    return lib


def _release_at_exit() -> None:
    """Frees the library's pooled workspaces, side streams and captured graphs
    while the HIP runtime is still up, instead of leaving them to process
    teardown (a no-op when nothing is held)."""
    if _lib is not None:
        try:
            _lib.leyenda_release_workspaces()
        except Exception:
            pass


def _check(rc: int, where: str) -> None:
    if rc != 0:
        raise LeyendaError(rc, where, load().leyenda_last_error().decode(errors="replace"))


def _stream_ptr(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _nrec(t) -> int:
    if t.dtype.itemsize != 1 or t.numel() % RECORD_BYTES:
        raise ValueError("record tensors are uint8 with a multiple of 100 bytes")
    if not t.is_contiguous():
        raise ValueError("record tensors must be contiguous")
    return t.numel() // RECORD_BYTES


# ---- sorting -------------------------------------------------------------------

def sort(records, out=None, stream=None):
    """Stable sort of device-resident records by key; returns ``out``.

    Asynchronous on ``stream`` (default: torch's current stream)."""
    import torch
    n = _nrec(records)
    if not records.is_cuda:
        raise ValueError("sort() takes a device tensor; use sort_runs()/merge() for host data")
    if out is None:
        out = torch.empty_like(records)
    elif _nrec(out) != n or not out.is_cuda:
        raise ValueError("out must be a device tensor of the same size")
    _check(load().leyenda_sort(records.data_ptr(), n, out.data_ptr(), _stream_ptr(stream)), "leyenda_sort")
    return out


def sort_keyed(records, key_bytes: int, out=None, stream=None):
    """Stable sort of device-resident records by a key of their first
    ``key_bytes`` bytes (1..100); returns ``out``.  For key_bytes > 10 the call
    returns after ``stream`` has drained."""
    import torch
    n = _nrec(records)
    if not records.is_cuda:
        raise ValueError("sort_keyed() takes a device tensor")
    if out is None:
        out = torch.empty_like(records)
    elif _nrec(out) != n or not out.is_cuda:
        raise ValueError("out must be a device tensor of the same size")
    _check(load().leyenda_sort_keyed(records.data_ptr(), n, key_bytes, out.data_ptr(), _stream_ptr(stream)),
           "leyenda_sort_keyed")
    return out


def workspace_bytes(n: int) -> int:
    return int(load().leyenda_workspace_bytes(n))


def sort_parts(n: int) -> int:
    """Output parts a sort of n records runs in (local sorts and gathers are
    launched once per part; the gathers overlap later parts' local sorts)."""
    return int(load().leyenda_sort_parts(n))


def first_pass(n: int) -> int:
    """First pass a sort of n records takes under the current parameters
    (0: extraction then partition; 1: one fused pass; 2: fused with the
    record copy)."""
    return int(load().leyenda_first_pass(n))


def plan_runs(n: int, budget_bytes: int) -> tuple[int, int]:
    r, k = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(load().leyenda_plan_runs(n, budget_bytes, ctypes.byref(r), ctypes.byref(k)), "leyenda_plan_runs")
    return int(r.value), int(k.value)


def plan_external(n: int, budget_bytes: int) -> tuple[int, int, int]:
    """(records per run, runs, runs kept on the device) of :func:`sort_external`."""
    r, k, kept = ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(load().leyenda_plan_external(n, budget_bytes, ctypes.byref(r), ctypes.byref(k), ctypes.byref(kept)),
           "leyenda_plan_external")
    return int(r.value), int(k.value), int(kept.value)


_PINNED: dict = {}


def pinned_empty(nbytes: int):
    """CPU uint8 tensor of exactly ``nbytes`` in pinned (hipHostMalloc) memory.

    Free it with :func:`pinned_free`; the tensor must not be used afterwards."""
    import numpy as np
    import torch
    ptr = ctypes.c_void_p(0)
    _check(load().leyenda_host_alloc(nbytes, ctypes.byref(ptr)), "leyenda_host_alloc")
    arr = np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ctypes.c_uint8)), shape=(nbytes,))
    t = torch.from_numpy(arr)
    _PINNED[t.data_ptr()] = ptr.value
    return t


def pinned_free(t) -> None:
    p = _PINNED.pop(t.data_ptr(), None)
    if p:
        _check(load().leyenda_host_free(p), "leyenda_host_free")


def sort_runs(host_records, budget_bytes: int, host_runs=None, k_max: int = 4096, stream=None):
    """Sorted runs of pinned host records within a device budget.

    Returns ``(host_runs, run_bounds)``; ``host_runs`` may be ``host_records``
    itself (runs are written over their own input ranges)."""
    import torch
    n = _nrec(host_records)
    if host_runs is None:
        host_runs = torch.empty_like(host_records, pin_memory=True)
    bounds = (ctypes.c_uint64 * (k_max + 1))()
    k = ctypes.c_uint64(0)
    _check(load().leyenda_sort_runs(host_records.data_ptr(), n, budget_bytes, host_runs.data_ptr(), bounds, k_max,
                                    ctypes.byref(k), _stream_ptr(stream)), "leyenda_sort_runs")
    return host_runs, [int(bounds[i]) for i in range(k.value + 1)]


def merge(host_runs, run_bounds: Sequence[int], budget_bytes: int, host_out=None, stream=None):
    """K-way merge of sorted runs (pinned host memory) into ``host_out``
    (pinned or pageable; a new pageable tensor by default)."""
    import torch
    n = _nrec(host_runs)
    if host_out is None:
        host_out = torch.empty_like(host_runs, pin_memory=False)
    k = len(run_bounds) - 1
    b = (ctypes.c_uint64 * len(run_bounds))(*run_bounds)
    if run_bounds[-1] != n:
        raise ValueError("run_bounds must end at the record count")
    _check(load().leyenda_merge(host_runs.data_ptr(), b, k, host_out.data_ptr(), budget_bytes, _stream_ptr(stream)),
           "leyenda_merge")
    return host_out


def sort_external(host_records, budget_bytes: int, host_runs=None, host_out=None, stream=None):
    """Runs + merge in one call (the last two runs stay on the device between the
    two stages).  ``host_runs``: pinned scratch for the runs, by default
    ``host_records`` itself (overwritten); ``host_out``: pinned or pageable (a
    new pageable tensor by default).  Returns ``host_out``."""
    import torch
    n = _nrec(host_records)
    if host_runs is None:
        host_runs = host_records
    if host_out is None:
        host_out = torch.empty_like(host_records, pin_memory=False)
    elif _nrec(host_out) != n or _nrec(host_runs) != n:
        raise ValueError("host_runs and host_out must hold as many records as host_records")
    _check(load().leyenda_sort_external(host_records.data_ptr(), n, budget_bytes, host_runs.data_ptr(),
                                        host_out.data_ptr(), _stream_ptr(stream)), "leyenda_sort_external")
    return host_out


def sort_external_keys(host_records, budget_bytes: int, host_out=None, stream=None):
    """Keys-only external sort of pinned host records: every (key, index)
    tuple sorted on the device at once, then the records written into
    ``host_out``: a pinned output takes a second in-order read of the input
    that puts every record in its place; a pageable one (a new pageable tensor
    by default) gets the records gathered from the pinned input in sorted
    order.  Needs ``workspace_bytes(n) + 256`` of device budget."""
    import torch
    n = _nrec(host_records)
    if host_out is None:
        host_out = torch.empty_like(host_records, pin_memory=False)
    elif _nrec(host_out) != n:
        raise ValueError("host_out must hold as many records as host_records")
    _check(load().leyenda_sort_external_keys(host_records.data_ptr(), n, budget_bytes, host_out.data_ptr(),
                                             _stream_ptr(stream)), "leyenda_sort_external_keys")
    return host_out


def sort_batch(pairs: Iterable, stream=None) -> None:
    """Sort many independent requests in one launch sequence.

    ``pairs``: iterable of ``(in_tensor, out_tensor)`` device tensors."""
    segs = []
    for a, b in pairs:
        n = _nrec(a)
        if _nrec(b) != n:
            raise ValueError("segment output size differs from its input")
        segs.append((a.data_ptr(), b.data_ptr(), n))
    arr = (Segment * max(1, len(segs)))()
    for i, (a, b, n) in enumerate(segs):
        arr[i].inp, arr[i].out, arr[i].n = a, b, n
    _check(load().leyenda_sort_batch(arr, len(segs), _stream_ptr(stream)), "leyenda_sort_batch")


# ---- serving ------------------------------------------------------------------------

def _config(budget_bytes: int, slots: int, max_batch: int, max_batch_records: int, batched: bool) -> ServerConfig:
    return ServerConfig(budget_bytes, slots, max_batch, max_batch_records, 1 if batched else 0)


class Server:
    """Continuous-batching sort server on the current GPU (see leyenda_server_* in leyenda.h)."""

    def __init__(self, budget_bytes: int, slots: int = 3, max_batch: int = 256,
                 max_batch_records: int = 10_000_000, batched: bool = True):
        self._h = ctypes.c_void_p(0)
        cfg = _config(budget_bytes, slots, max_batch, max_batch_records, batched)
        _check(load().leyenda_server_create(ctypes.byref(cfg), ctypes.byref(self._h)), "leyenda_server_create")

    def submit(self, records, tag: int) -> None:
        """Queue a device tensor of records; it must stay unchanged until the request completes."""
        _check(load().leyenda_server_submit(self._h, records.data_ptr(), _nrec(records), tag),
               "leyenda_server_submit")

    def poll(self, timeout_s: float = 0.0, cap: int = 256) -> list:
        buf = (Done * cap)()
        k = ctypes.c_uint64(0)
        _check(load().leyenda_server_poll(self._h, buf, cap, ctypes.byref(k), timeout_s), "leyenda_server_poll")
        return [{"tag": int(d.tag), "out_dev": int(d.out_dev or 0), "n": int(d.n), "submit_s": d.submit_s,
                 "start_s": d.start_s, "done_s": d.done_s, "status": int(d.status)} for d in buf[:k.value]]

    def output(self, done: dict):
        """Copy of a completed request's sorted records as a (n, 100) uint8 device tensor."""
        import torch
        out = torch.empty((done["n"], RECORD_BYTES), dtype=torch.uint8, device="cuda")
        src = _DevView(done["out_dev"], done["n"] * RECORD_BYTES)
        out.view(-1).copy_(torch.as_tensor(src, device="cuda"))
        return out

    def release(self, tag: int) -> None:
        _check(load().leyenda_server_release(self._h, tag), "leyenda_server_release")

    def close(self) -> None:
        if self._h:
            load().leyenda_server_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _DevView:
    """__cuda_array_interface__ view of engine-owned device memory (uint8)."""

    def __init__(self, ptr: int, nbytes: int):
        self.__cuda_array_interface__ = {"shape": (nbytes,), "typestr": "|u1", "data": (ptr, False),
                                         "version": 3, "strides": None}


def serve_replay(inputs: Sequence, arrivals_s, budget_bytes: int, slots: int = 3, max_batch: int = 256,
                 max_batch_records: int = 10_000_000, batched: bool = True):
    """Replay an arrival stream natively; returns (latencies_s list, makespan_s).

    ``inputs``: list of (device_ptr, n_records); ``arrivals_s``: non-decreasing seconds."""
    cnt = len(inputs)
    cfg = _config(budget_bytes, slots, max_batch, max_batch_records, batched)
    ptrs = (ctypes.c_void_p * max(cnt, 1))(*[p for p, _ in inputs])
    ns = (ctypes.c_uint64 * max(cnt, 1))(*[n for _, n in inputs])
    arr = (ctypes.c_double * max(cnt, 1))(*[float(a) for a in arrivals_s])
    lat = (ctypes.c_double * max(cnt, 1))()
    mk = ctypes.c_double(0)
    _check(load().leyenda_serve_replay(ctypes.byref(cfg), cnt, ptrs, ns, arr, lat, ctypes.byref(mk)),
           "leyenda_serve_replay")
    return [lat[i] for i in range(cnt)], mk.value


# ---- parameters and diagnostics -----------------------------------------------------

def get_params() -> dict:
    p = Params()
    _check(load().leyenda_get_params(ctypes.byref(p)), "leyenda_get_params")
    return p.as_dict()


def set_params(**kw) -> dict:
    p = Params()
    _check(load().leyenda_get_params(ctypes.byref(p)), "leyenda_get_params")
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, int(v))
    _check(load().leyenda_set_params(ctypes.byref(p)), "leyenda_set_params")
    return p.as_dict()


def load_params(path: str) -> dict:
    _check(load().leyenda_load_params(path.encode()), "leyenda_load_params")
    return get_params()


def stats(stream=None) -> dict:
    s = Stats()
    _check(load().leyenda_sort_stats(_stream_ptr(stream), ctypes.byref(s)), "leyenda_sort_stats")
    return {"levels": int(s.levels), "segments": list(s.segments), "moved": [int(x) for x in s.moved],
            "tasks": int(s.tasks), "guard": int(s.guard)}


PHASES = ("extract", "partition", "local", "gather")


def profile_enable(on: bool = True) -> None:
    _check(load().leyenda_profile_enable(1 if on else 0), "leyenda_profile_enable")


def profile_read() -> tuple[dict, int]:
    """Summed per-phase milliseconds (HIP events) and the number of sorts timed."""
    ms = (ctypes.c_double * 4)()
    calls = ctypes.c_uint64(0)
    _check(load().leyenda_profile_read(ms, ctypes.byref(calls)), "leyenda_profile_read")
    return {k: float(ms[i]) for i, k in enumerate(PHASES)}, int(calls.value)


def release_workspaces() -> None:
    _check(load().leyenda_release_workspaces(), "leyenda_release_workspaces")


def debug_extract(records, key_bytes: int = KEY_BYTES, stream=None):
    """(hi, lo, hist) of the sort's own extraction kernel: int64 tuple words and
    the int32 histogram of the leading ``digit_bits`` key bits (256 counters);
    key bytes at and past ``key_bytes`` (1..10) are cleared."""
    import torch
    n = _nrec(records)
    dev = records.device
    hi = torch.empty(n, dtype=torch.int64, device=dev)
    lo = torch.empty(n, dtype=torch.int64, device=dev)
    hist = torch.empty(256, dtype=torch.int32, device=dev)
    _check(load().leyenda_debug_extract(records.data_ptr(), n, key_bytes, hi.data_ptr(), lo.data_ptr(),
                                        hist.data_ptr(), _stream_ptr(stream)), "leyenda_debug_extract")
    return hi, lo, hist


def debug_first_pass(records, first_pass: int = 1, key_bytes: int = KEY_BYTES, stream=None):
    """(hi, lo, count, recs) of the sort's fused first pass: the level-0 buckets
    copied out in bucket order (int64 tuple words), the 256 bucket counts
    (int32) and, for first_pass 2, the records of the record pool in the same
    order (else None)."""
    import torch
    n = _nrec(records)
    dev = records.device
    hi = torch.empty(n, dtype=torch.int64, device=dev)
    lo = torch.empty(n, dtype=torch.int64, device=dev)
    count = torch.empty(256, dtype=torch.int32, device=dev)
    recs = torch.empty((n, RECORD_BYTES), dtype=torch.uint8, device=dev) if first_pass == 2 else None
    _check(load().leyenda_debug_first_pass(records.data_ptr(), n, first_pass, key_bytes, hi.data_ptr(),
                                           lo.data_ptr(), count.data_ptr(),
                                           recs.data_ptr() if recs is not None else None, _stream_ptr(stream)),
           "leyenda_debug_first_pass")
    return hi, lo, count, recs


def debug_gather(records, idx, stream=None):
    """out[j] = records[idx[j]] with the sort's gather kernel (idx: int32 device tensor)."""
    import torch
    n_rec = _nrec(records)
    n = idx.numel()
    out = torch.empty((n, RECORD_BYTES), dtype=torch.uint8, device=records.device)
    _check(load().leyenda_debug_gather(records.data_ptr(), n_rec, idx.data_ptr(), n, out.data_ptr(),
                                       _stream_ptr(stream)), "leyenda_debug_gather")
    return out
