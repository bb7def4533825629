"""CPU oracle for the record sort -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library (``paper_1909_08006_amd``)
never imports it, and it imports nothing from the GPU library.

What is computed (see ``oracle.c`` for the passages followed): the stable sort
of 100-byte records by memcmp order on their 10-byte key (bytes 0..9), equal
keys kept in input order; with ``key_bytes`` the same sort on a key of the
first K bytes (Section 5's flexible key sizes).  Every schedule of the paper's method -- MSD radix
passes, big/small/tiny buckets, sorted runs plus a k-way merge, batching --
reaches exactly this result.

Pinned by ``tests/test_oracle.py`` against the worked example of Section 2.2,
brute force over all permutations of tiny inputs, numpy's stable lexsort and
Python's stable ``sorted``, and planted mistakes for every checker.
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

REC, KEY = 100, 10


def build() -> str:
    """Compile liboracle.so with gcc (OpenMP for the O(n) scans).  Always recompiles."""
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-o", _LIB + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    vp, u64 = ctypes.c_void_p, ctypes.c_uint64
    lib.oracle_sort.argtypes = [vp, u64, vp, vp]
    lib.oracle_sort.restype = ctypes.c_int
    lib.oracle_sort_par.argtypes = [vp, u64, vp, vp, ctypes.c_int]
    lib.oracle_sort_par.restype = ctypes.c_int
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_sort_key.argtypes = [vp, u64, ctypes.c_uint32, vp, vp]
    lib.oracle_sort_key.restype = ctypes.c_int
    lib.oracle_output_rank.argtypes = [vp, u64, vp, u64, vp]
    lib.oracle_first_unsorted.argtypes = [vp, u64]
    lib.oracle_first_unsorted.restype = ctypes.c_int64
    lib.oracle_multiset_hash.argtypes = [vp, u64, vp]
    lib.oracle_ties_in_order.argtypes = [vp, vp, u64]
    lib.oracle_ties_in_order.restype = ctypes.c_int
    lib.oracle_count_less.argtypes = [vp, u64, vp, u64, vp]
    lib.oracle_equal_neighbours.argtypes = [vp, u64]
    lib.oracle_equal_neighbours.restype = ctypes.c_uint64
    _lib = lib
    return lib


def _as_records(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint8)
    if a.size % REC:
        raise ValueError("record buffer size is not a multiple of 100 bytes")
    return a.reshape(-1, REC)


def _ptr(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


def sort(records, return_perm: bool = False, key_bytes: int = KEY, threads: int = 1):
    """Stable sort of records by their key (memcmp order): the 10-byte key, or
    the first ``key_bytes`` bytes (1..100, the flexible key sizes of Section 5).

    ``threads`` != 1 (0: every host thread) sorts the 10-byte key with
    ``oracle_sort_par``: slices sorted by the same comparison, then merged --
    the same result, pinned against the one-thread sort."""
    rec = _as_records(records)
    n = rec.shape[0]
    if not 1 <= key_bytes <= REC:
        raise ValueError("key_bytes must be in 1..100")
    out = np.empty_like(rec)
    perm = np.empty(n, dtype=np.uint32)
    if n:
        if key_bytes == KEY and threads != 1:
            rc = 0 if _load().oracle_sort_par(_ptr(rec), n, _ptr(out), _ptr(perm), int(threads)) > 0 else -1
        elif key_bytes == KEY:
            rc = _load().oracle_sort(_ptr(rec), n, _ptr(out), _ptr(perm))
        else:
            rc = _load().oracle_sort_key(_ptr(rec), n, key_bytes, _ptr(out), _ptr(perm))
        if rc != 0:
            raise MemoryError("oracle sort failed")
    return (out, perm) if return_perm else out


def host_threads() -> int:
    """Threads the parallel oracle runs on when asked for all of them."""
    return int(_load().oracle_threads())


def output_rank(records, samples) -> np.ndarray:
    """Output position of each sampled input record under the stable sort."""
    rec = _as_records(records)
    s = np.ascontiguousarray(samples, dtype=np.uint64)
    if s.size and int(s.max()) >= rec.shape[0]:
        raise IndexError("sample index out of range")
    ranks = np.zeros(s.size, dtype=np.uint64)
    if s.size:
        _load().oracle_output_rank(_ptr(rec), rec.shape[0], _ptr(s), s.size, _ptr(ranks))
    return ranks


def count_less(records, probes) -> np.ndarray:
    """For each probe record, the number of records whose key is below the probe's key."""
    rec, pr = _as_records(records), _as_records(probes)
    out = np.zeros(pr.shape[0], dtype=np.uint64)
    if pr.shape[0]:
        _load().oracle_count_less(_ptr(rec), rec.shape[0], _ptr(pr), pr.shape[0], _ptr(out))
    return out


def equal_neighbours(records) -> int:
    """Adjacent pairs with equal keys (zero: stability is vacuous for this output)."""
    rec = _as_records(records)
    return int(_load().oracle_equal_neighbours(_ptr(rec), rec.shape[0]))


def first_unsorted(records) -> int:
    """Index j of the first pair with key[j] > key[j+1], or -1."""
    rec = _as_records(records)
    return int(_load().oracle_first_unsorted(_ptr(rec), rec.shape[0]))


def multiset_hash(records) -> tuple[int, int]:
    rec = _as_records(records)
    h = np.zeros(2, dtype=np.uint64)
    _load().oracle_multiset_hash(_ptr(rec), rec.shape[0], _ptr(h))
    return int(h[0]), int(h[1])


def ties_in_order(inp, out) -> bool:
    """Every equal-key run of `out` lists exactly the input records with that key, in input order."""
    a, b = _as_records(inp), _as_records(out)
    if a.shape != b.shape:
        raise ValueError("input and output sizes differ")
    rc = _load().oracle_ties_in_order(_ptr(a), _ptr(b), a.shape[0])
    if rc < 0:
        raise MemoryError("oracle_ties_in_order failed")
    return rc == 0


def verify_sorted_output(inp, out) -> None:
    """Raise AssertionError unless `out` is the stable key sort of `inp`.

    Uses the uniqueness of a stable sort: keys non-decreasing, the same record
    multiset, and equal keys in input order together fix the output."""
    j = first_unsorted(out)
    assert j == -1, f"keys out of order at output {j}"
    assert multiset_hash(inp) == multiset_hash(out), "record multiset differs"
    assert ties_in_order(inp, out), "equal keys not in input order"


# ---- pure-Python references for tiny inputs ----------------------------------

def brute_force_order(keys: list[bytes]) -> list[int]:
    """The one permutation p of range(n) for which keys[p] is non-decreasing
    (byte-string order) and equal keys keep increasing index, found by trying
    every permutation.  For n <= 7 only."""
    n = len(keys)
    if n > 7:
        raise ValueError("brute force is for n <= 7")
    found = None
    for p in itertools.permutations(range(n)):
        ok = True
        for a, b in zip(p, p[1:]):
            if keys[a] > keys[b] or (keys[a] == keys[b] and a > b):
                ok = False
                break
        if ok:
            if found is not None:
                raise AssertionError("two permutations satisfy the definition")
            found = list(p)
    return found


def corank_brute(runs_keys: list[list[bytes]], r: int) -> list[int]:
    """Split counts (s_0..s_{k-1}), sum r, such that the first s_i records of every
    run i are exactly the r smallest under (key, run, position) order; found by
    listing and sorting all (key, run, pos) triples.  For small inputs only."""
    triples = [(k, i, p) for i, keys in enumerate(runs_keys) for p, k in enumerate(keys)]
    triples.sort()
    s = [0] * len(runs_keys)
    for _, i, _ in triples[:r]:
        s[i] += 1
    return s
