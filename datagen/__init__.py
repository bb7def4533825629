"""Seeded synthetic record generators shared by the oracle side and the GPU side.

Records are 100 bytes: a 10-byte key (bytes 0..9) and a 90-byte payload
(bytes 10..99), the record format of the paper's workloads (Section 4.1).  The
workloads themselves (sortbenchmark.org generator output) are not available;
these seeded generators stand in for them with the shapes and key
distributions of the five workload configurations:

* uniform keys and payload (internal 10 GB and external 60 GB workloads),
* Zipf(s=1.2) 4-byte key prefixes over 65,536 values plus 5% exact-duplicate
  keys (the skewed 20 GB workload),
* keys of ten printable ASCII bytes, each uniform over 0x20..0x7E (the key
  format the paper gives its 20 GB dataset),
* log-uniform request sizes and Poisson arrivals (the serving workload).

Nothing here sorts or compares keys.  The C library ``libdatagen.so`` is built
by :func:`build` with gcc; the word generator is re-implemented in numpy
(:func:`words`) for the small request-size and arrival streams.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "datagen.c")
_LIB = os.path.join(_HERE, "libdatagen.so")
_lib = None

RECORD_BYTES = 100
KEY_BYTES = 10

# Workload seeds (one per configuration; request r of the serving stream uses 1000 + r).
SEED_SMALL, SEED_INTERNAL, SEED_SKEWED, SEED_EXTERNAL = 1, 2, 3, 4
SEED_ARRIVALS, SEED_SIZES, SEED_REQUEST_BASE = 5, 6, 1000
SEED_ASCII = 7
ASCII_LO, ASCII_VALUES = 0x20, 95
ZIPF_VALUES, ZIPF_S, DUP_FRAC = 65536, 1.2, 0.05


def build() -> str:
    """Compile libdatagen.so (gcc, OpenMP).  Always recompiles."""
    cmd = ["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
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
    u64, vp = ctypes.c_uint64, ctypes.c_void_p
    lib.dg_records_uniform.argtypes = [vp, u64, u64, u64]
    lib.dg_records_indexed.argtypes = [vp, u64, u64, u64]
    lib.dg_records_skewed.argtypes = [vp, u64, u64, u64, ctypes.c_uint32, ctypes.c_double, ctypes.c_double]
    lib.dg_records_skewed.restype = ctypes.c_int
    lib.dg_records_ascii.argtypes = [vp, u64, u64, u64]
    lib.dg_word.argtypes = [u64, u64, u64]
    lib.dg_word.restype = u64
    lib.dg_zipf_pmf.argtypes = [ctypes.c_uint32, ctypes.c_double, ctypes.c_uint32]
    lib.dg_zipf_pmf.restype = ctypes.c_double
    lib.dg_zipf_value.argtypes = [u64, ctypes.c_uint32]
    lib.dg_zipf_value.restype = ctypes.c_uint32
    _lib = lib
    return lib


# ---- raw-pointer fills (used to generate straight into pinned/host buffers) ----

def fill_uniform(ptr: int, count: int, seed: int, first: int = 0) -> None:
    _load().dg_records_uniform(ctypes.c_void_p(ptr), count, seed, first)


def fill_indexed(ptr: int, count: int, seed: int, first: int = 0) -> None:
    _load().dg_records_indexed(ctypes.c_void_p(ptr), count, seed, first)


def fill_ascii(ptr: int, count: int, seed: int, first: int = 0) -> None:
    _load().dg_records_ascii(ctypes.c_void_p(ptr), count, seed, first)


def fill_skewed(ptr: int, count: int, seed: int, first: int = 0, nvals: int = ZIPF_VALUES,
                s: float = ZIPF_S, dup_frac: float = DUP_FRAC) -> None:
    rc = _load().dg_records_skewed(ctypes.c_void_p(ptr), count, seed, first, nvals, s, dup_frac)
    if rc != 0:
        raise MemoryError("dg_records_skewed: allocation failed")


# ---- numpy conveniences ------------------------------------------------------

def _empty(count: int) -> np.ndarray:
    return np.empty((count, RECORD_BYTES), dtype=np.uint8)


def uniform(count: int, seed: int, first: int = 0) -> np.ndarray:
    a = _empty(count)
    if count:
        fill_uniform(a.ctypes.data, count, seed, first)
    return a


def indexed(count: int, seed: int, first: int = 0) -> np.ndarray:
    a = _empty(count)
    if count:
        fill_indexed(a.ctypes.data, count, seed, first)
    return a


def skewed(count: int, seed: int, first: int = 0, nvals: int = ZIPF_VALUES, s: float = ZIPF_S,
           dup_frac: float = DUP_FRAC) -> np.ndarray:
    a = _empty(count)
    if count:
        fill_skewed(a.ctypes.data, count, seed, first, nvals, s, dup_frac)
    return a


def ascii(count: int, seed: int, first: int = 0) -> np.ndarray:
    a = _empty(count)
    if count:
        fill_ascii(a.ctypes.data, count, seed, first)
    return a


def word(seed: int, i: int, k: int) -> int:
    return int(_load().dg_word(seed, i, k))


def zipf_pmf(r: int, nvals: int = ZIPF_VALUES, s: float = ZIPF_S) -> float:
    return float(_load().dg_zipf_pmf(nvals, s, r))


def zipf_value(seed: int, r: int) -> int:
    return int(_load().dg_zipf_value(seed, r))


# ---- the same counter-based word stream in numpy (small streams only) ----------

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)


def _sm64_out(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def words(seed: int, count: int, k: int = 0) -> np.ndarray:
    """Word k of records 0..count-1 for a seed (same values as the C generator)."""
    with np.errstate(over="ignore"):
        key = _sm64_out(np.array([seed], dtype=np.uint64) + _GOLDEN)[0]
        i = np.arange(count, dtype=np.uint64)
        return _sm64_out(key + (i * np.uint64(16) + np.uint64(k + 1)) * _GOLDEN)


def unit(seed: int, count: int, k: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of the word stream."""
    return (words(seed, count, k) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def request_sizes(count: int, seed: int = SEED_SIZES, lo: int = 1000, hi: int = 10_000_000) -> np.ndarray:
    """Log-uniform request sizes in [lo, hi] records."""
    u = unit(seed, count)
    s = np.floor(np.exp(np.log(lo) + u * (np.log(hi + 1) - np.log(lo)))).astype(np.int64)
    return np.clip(s, lo, hi)


def arrival_times(count: int, rate_per_s: float, seed: int = SEED_ARRIVALS) -> np.ndarray:
    """Poisson arrival times (seconds from 0): cumulative exponential gaps."""
    u = unit(seed, count)
    gaps = -np.log1p(-u) / rate_per_s
    return np.cumsum(gaps)
