"""Parity of the fused first passes (parameter first_pass 1 and 2) with the CPU oracle.

A single sort of at least 8 Mi records can make its first-digit buckets in one
pass over the records: the tuples (and, with first_pass 2, the records too) go
straight into per-bucket chains of chunks, a tile's place inside each bucket
coming from a look-back over the tiles before it.  The output must be the same
bytes as the oracle's stable sort whatever the first pass.
"""
import numpy as np
import pytest

import datagen
import oracle
from tests.test_gpu_sort import _want_tuples, assert_same, pattern, run_sort

pytestmark = pytest.mark.gpu

N = 8_388_608 + 12_345  # above the 8 Mi threshold: four output parts; a ragged last tile


def _with_params(gpu, params, fn):
    old = gpu.get_params()
    try:
        gpu.set_params(**params)
        return fn()
    finally:
        gpu.set_params(**old)


def _stats(gpu):
    import torch
    return gpu.stats(torch.cuda.current_stream())


@pytest.mark.parametrize("first_pass", [1, 2])
@pytest.mark.parametrize("name", ["uniform", "skewed", "skewed_narrow", "all_equal", "one_big_bucket",
                                  "few_distinct", "ascii", "sorted"])
def test_first_pass_patterns(gpu, first_pass, name):
    """Equal keys across tiles and chunks (all_equal: one bucket of every
    record, its chunks taken by one tile after another), one bucket of 90% of
    the records, Zipf prefixes with 20% duplicates, printable keys."""
    rec = datagen.uniform(N, 94) if name == "uniform" else pattern(name, N)
    want = oracle.sort(rec)
    got = _with_params(gpu, dict(first_pass=first_pass), lambda: run_sort(gpu, rec))
    assert_same(got, want, f"first_pass={first_pass} {name}")
    st = _stats(gpu)
    assert st["guard"] == 0
    assert st["moved"][0] == N


@pytest.mark.parametrize("params", [
    dict(first_pass=1, digit_bits=4), dict(first_pass=2, digit_bits=5), dict(first_pass=1, digit_bits=7),
    dict(first_pass=2, tile_items=16, scatter_threads=512),  # record copy: 4,096-key tiles fit 4,096-key chunks
    dict(first_pass=1, tile_items=16),  # 8,192-key fused tiles do not fit: the split passes run
    dict(first_pass=2, big_threshold=64, tiny_threshold=5),
])
def test_first_pass_params(gpu, params):
    rec = pattern("skewed_narrow", N)
    want = oracle.sort(rec)
    got = _with_params(gpu, params, lambda: run_sort(gpu, rec))
    assert_same(got, want, str(params))
    assert _stats(gpu)["guard"] == 0


def test_first_pass_below_threshold_and_repeats(gpu):
    """Below 8 Mi records the split passes run whatever the parameter; repeated
    sorts of different sizes reuse the workspace (look-back words and chunk
    table are cleared per sort)."""
    small = datagen.skewed(500_000, 61)
    big = datagen.skewed(N, 62)
    bigger = datagen.uniform(N + 3_000_000, 63)

    def body():
        assert_same(run_sort(gpu, small), oracle.sort(small), "below threshold")
        a = run_sort(gpu, big)
        assert_same(a, oracle.sort(big), "first")
        assert_same(run_sort(gpu, bigger), oracle.sort(bigger), "bigger")
        assert_same(run_sort(gpu, big), a, "repeat")

    for fp in (1, 2):
        _with_params(gpu, dict(first_pass=fp), body)


@pytest.mark.parametrize("key_bytes", [4, 10, 20])
def test_first_pass_keyed(gpu, key_bytes):
    """Shorter keys (masked tuples) and longer ones (the gather marks ties, so
    the record copy gives way to the tuple-only fused pass)."""
    import torch
    rec = pattern("skewed_narrow", N)
    rec[::3, 10:30] = rec[0, 10:30]  # ties past byte 10 for the 20-byte key
    want = oracle.sort(rec, key_bytes=key_bytes)

    def body():
        dev = torch.from_numpy(rec).cuda()
        out = gpu.sort_keyed(dev, key_bytes)
        torch.cuda.synchronize()
        return out.cpu().numpy()

    for fp in (1, 2):
        assert_same(_with_params(gpu, dict(first_pass=fp), body), want, f"K={key_bytes} first_pass={fp}")


@pytest.mark.parametrize("first_pass,key_bytes,digit_bits,n", [
    (1, 10, 8, 3 * 8192 + 77), (1, 10, 8, 200_003), (2, 10, 8, 200_003), (1, 4, 8, 100_000),
    (1, 9, 5, 150_001), (2, 10, 6, 90_001), (2, 3, 8, 70_001), (1, 10, 8, 1), (2, 10, 4, 5)])
def test_first_pass_step(gpu, first_pass, key_bytes, digit_bits, n):
    """The fused pass alone (as the sort launches it): bucket d holds the
    tuples of the records whose leading digit is d, in input order, i.e. the
    tuples stably sorted by that digit; with the record copy the records come
    in the same order and a tuple carries its position inside its bucket.  A
    third of the records share a 3-byte prefix, so one bucket spans many
    chunks and most tiles' runs start inside a chunk another tile took."""
    import torch
    rec = datagen.uniform(n, 33)
    rec[: n // 3, :3] = rec[0, :3]

    def body():
        out = gpu.debug_first_pass(torch.from_numpy(rec).cuda(), first_pass, key_bytes)
        torch.cuda.synchronize()
        return [None if x is None else x.cpu().numpy() for x in out]

    hi, lo, count, recs = _with_params(gpu, dict(digit_bits=digit_bits), body)
    want_hi, want_lo = _want_tuples(rec, key_bytes)
    lead = (want_hi >> np.uint64(64 - digit_bits)).astype(np.int64)
    order = np.argsort(lead, kind="stable")
    want_count = np.bincount(lead, minlength=256)
    np.testing.assert_array_equal(count, want_count)
    np.testing.assert_array_equal(hi.view(np.uint64), want_hi[order])
    if first_pass == 1:
        np.testing.assert_array_equal(lo.view(np.uint64), want_lo[order])
    else:
        base = np.concatenate([[0], np.cumsum(want_count)[:-1]])
        pos = (np.arange(n) - base[lead[order]]).astype(np.uint64)
        np.testing.assert_array_equal(lo.view(np.uint64), (want_lo[order] & np.uint64(0xFFFF00000000)) | pos)
        np.testing.assert_array_equal(recs, rec[order])
