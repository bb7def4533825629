"""Pins for the CPU oracle, independent of the oracle's own code.

Each pin would fail for a plausible mistake in the oracle: a comparator that
ignores the last key bytes (hi/lo split at byte 8), compares signed bytes,
reverses ties, drops the payload in the gather, or checkers that miss a
planted swap, bit flip or duplicate.
"""
import itertools

import numpy as np
import pytest

import datagen
import oracle
from tests.golden import pad_key, worked_example


def records_from_keys(keys, seed=7):
    rec = datagen.uniform(len(keys), seed)
    for i, k in enumerate(keys):
        rec[i, :10] = np.frombuffer(pad_key(k), dtype=np.uint8)
    return rec


def keys_of(rec):
    return [bytes(r[:10]) for r in rec]


# ---- Section 2.2 worked example ---------------------------------------------

def test_worked_example_every_input_order():
    ex = worked_example()
    for order in itertools.permutations(range(len(ex["keys"]))):
        keys = [ex["keys"][i] for i in order]
        rec = records_from_keys(keys, seed=11 + sum(order))
        out, perm = oracle.sort(rec, return_perm=True)
        assert [k.rstrip(b"\x00") for k in keys_of(out)] == ex["sorted"]
        # the gather moves whole records: payloads follow their keys
        np.testing.assert_array_equal(out, rec[perm])


def test_worked_example_buckets():
    ex = worked_example()
    rec = records_from_keys(ex["keys"])
    counts = np.bincount(rec[:, 0], minlength=256)
    assert {b: int(c) for b, c in enumerate(counts) if c} == ex["counts"]
    offs = np.concatenate([[0], np.cumsum(counts)[:-1]])
    assert {b: int(offs[b]) for b in ex["offsets"]} == ex["offsets"]
    out = oracle.sort(rec)
    c_bucket = out[ex["offsets"][0x63]: ex["offsets"][0x63] + ex["counts"][0x63]]
    assert list(c_bucket[:, 1]) == ex["c_second"]


# ---- brute force over all permutations ------------------------------------------

ALPHABET = [0x00, 0x01, 0xFF]


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_brute_force_tiny(n):
    rng = np.random.default_rng(100 + n)
    for trial in range(40 if n < 7 else 12):
        keys = []
        for _ in range(n):
            k = bytearray(10)
            for pos in (0, 7, 8, 9):  # byte 7/8 is the hi/lo split of the 16-byte tuple
                k[pos] = ALPHABET[rng.integers(3)]
            keys.append(bytes(k))
        rec = records_from_keys(keys, seed=1000 + trial)
        _, perm = oracle.sort(rec, return_perm=True)
        assert list(perm) == oracle.brute_force_order(keys)


def test_signed_byte_order_pinned():
    # 0x80.. must sort after 0x7F.. (unsigned bytes)
    rec = records_from_keys([b"\x80", b"\x7f", b"\xff\x00", b"\x00\xff"])
    assert keys_of(oracle.sort(rec))[0][:1] == b"\x00"
    assert [k[0] for k in keys_of(oracle.sort(rec))] == [0x00, 0x7F, 0x80, 0xFF]


# ---- library special cases -------------------------------------------------------

def _lexsort_perm(rec):
    hi = np.zeros(rec.shape[0], dtype=np.uint64)
    for b in range(8):
        hi = (hi << np.uint64(8)) | rec[:, b].astype(np.uint64)
    lo = (rec[:, 8].astype(np.uint64) << np.uint64(8)) | rec[:, 9].astype(np.uint64)
    idx = np.arange(rec.shape[0], dtype=np.uint64)
    return np.lexsort((idx, lo, hi))  # last key is primary; stable


def test_matches_numpy_lexsort_with_duplicates():
    rec = datagen.uniform(20000, 21)
    rng = np.random.default_rng(3)
    # plant exact duplicates and keys equal in bytes 0..7 only
    src = rng.integers(0, 20000, 3000)
    dst = rng.integers(0, 20000, 3000)
    rec[dst, :10] = rec[src, :10]
    dst2 = rng.integers(0, 20000, 500)
    rec[dst2, :8] = rec[0, :8]
    _, perm = oracle.sort(rec, return_perm=True)
    np.testing.assert_array_equal(perm.astype(np.int64), _lexsort_perm(rec))


def test_matches_python_sorted_skewed():
    rec = datagen.skewed(5000, 3)
    _, perm = oracle.sort(rec, return_perm=True)
    ref = sorted(range(rec.shape[0]), key=lambda i: (bytes(rec[i, :10]), i))
    assert list(perm) == ref


def test_empty_and_single():
    assert oracle.sort(np.zeros((0, 100), np.uint8)).shape == (0, 100)
    r = datagen.uniform(1, 5)
    np.testing.assert_array_equal(oracle.sort(r), r)


# ---- the multithreaded oracle -----------------------------------------------------

@pytest.mark.parametrize("threads", [2, 3, 5, 8, 16])
@pytest.mark.parametrize("n", [2, 3, 7, 9, 31, 1000, 65537])
def test_parallel_sort_matches_one_thread(n, threads):
    # more threads than records, odd slice counts, and many equal keys (ties
    # across slice boundaries must still come out in input order)
    rec = datagen.skewed(n, 40 + n % 7, nvals=16, dup_frac=0.4) if n > 8 else datagen.uniform(n, 41)
    rec[: n // 2, :10] = rec[0, :10]
    a, pa = oracle.sort(rec, return_perm=True)
    b, pb = oracle.sort(rec, return_perm=True, threads=threads)
    np.testing.assert_array_equal(pb, pa)
    np.testing.assert_array_equal(b, a)


def test_parallel_sort_matches_numpy_lexsort():
    rec = datagen.skewed(200_000, 43, nvals=256, dup_frac=0.2)
    _, perm = oracle.sort(rec, return_perm=True, threads=0)
    np.testing.assert_array_equal(perm.astype(np.int64), _lexsort_perm(rec))


@pytest.mark.parametrize("n", [3, 5, 7])
def test_parallel_sort_brute_force_tiny(n):
    rng = np.random.default_rng(200 + n)
    for trial in range(10):
        keys = []
        for _ in range(n):
            k = bytearray(10)
            for pos in (0, 8, 9):
                k[pos] = ALPHABET[rng.integers(3)]
            keys.append(bytes(k))
        rec = records_from_keys(keys, seed=2000 + trial)
        _, perm = oracle.sort(rec, return_perm=True, threads=4)
        assert list(perm) == oracle.brute_force_order(keys)


# ---- one-by-one ranks ------------------------------------------------------------

def test_output_rank_matches_full_sort():
    rec = datagen.skewed(4000, 9, nvals=50)  # many equal keys
    _, perm = oracle.sort(rec, return_perm=True)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size, dtype=perm.dtype)
    samples = np.arange(0, 4000, 7)
    np.testing.assert_array_equal(oracle.output_rank(rec, samples), inv[samples].astype(np.uint64))


def test_count_less_is_position_of_unique_keys():
    rec = datagen.uniform(3000, 13)
    out = oracle.sort(rec)
    probes = rec[[0, 17, 2999, 1500]]
    pos = oracle.count_less(rec[::-1].copy(), probes)  # any permutation of the input
    for p, r in zip(pos, probes):
        np.testing.assert_array_equal(out[int(p)], r)
    # brute force on a tiny input with ties: strict "less" count
    keys = [b"b", b"a", b"b", b"c"]
    tiny = records_from_keys(keys)
    assert list(oracle.count_less(tiny, tiny)) == [1, 0, 1, 3]


def test_equal_neighbours():
    rec = datagen.uniform(1000, 14)
    assert oracle.equal_neighbours(oracle.sort(rec)) == 0
    rec[[3, 9, 700], :10] = rec[3, :10]
    assert oracle.equal_neighbours(oracle.sort(rec)) == 2


# ---- checkers catch planted mistakes ------------------------------------------------

def test_checkers_accept_oracle_output():
    rec = datagen.skewed(30000, 4)
    out = oracle.sort(rec)
    oracle.verify_sorted_output(rec, out)


def test_first_unsorted_detects_swap():
    rec = datagen.uniform(1000, 5)
    out = oracle.sort(rec)
    assert oracle.first_unsorted(out) == -1
    bad = out.copy()
    bad[[100, 101]] = bad[[101, 100]]
    assert oracle.first_unsorted(bad) == 100


def test_multiset_hash_detects_flip_and_duplicate():
    rec = datagen.uniform(1000, 6)
    perm = np.random.default_rng(0).permutation(1000)
    assert oracle.multiset_hash(rec) == oracle.multiset_hash(rec[perm])
    flip = rec.copy()
    flip[500, 77] ^= 0x04
    assert oracle.multiset_hash(flip) != oracle.multiset_hash(rec)
    dup = rec.copy()
    dup[3] = dup[4]
    assert oracle.multiset_hash(dup) != oracle.multiset_hash(rec)


def test_ties_in_order_detects_swapped_equal_keys():
    rec = datagen.uniform(200, 8)
    rec[[10, 50, 150], :10] = rec[10, :10]
    out = oracle.sort(rec)
    assert oracle.ties_in_order(rec, out)
    j = int(np.nonzero((out[:, :10] == rec[10, :10]).all(axis=1))[0][0])
    bad = out.copy()
    bad[[j, j + 1]] = bad[[j + 1, j]]
    assert oracle.first_unsorted(bad) == -1  # still sorted by key ...
    assert oracle.multiset_hash(bad) == oracle.multiset_hash(rec)  # ... same multiset ...
    assert not oracle.ties_in_order(rec, bad)  # ... but ties out of input order


def test_verify_rejects_payload_loss():
    rec = datagen.uniform(300, 9)
    out = oracle.sort(rec)
    bad = out.copy()
    bad[17, 10:] = 0
    with pytest.raises(AssertionError):
        oracle.verify_sorted_output(rec, bad)


# ---- merge co-rank reference ------------------------------------------------------

def test_corank_brute_small():
    runs = [[b"a", b"c", b"c"], [b"b", b"c"], [b"c", b"d"]]
    assert oracle.corank_brute(runs, 0) == [0, 0, 0]
    assert oracle.corank_brute(runs, 2) == [1, 1, 0]
    # ties on "c": run 0 first, then run 1, then run 2
    assert oracle.corank_brute(runs, 4) == [3, 1, 0]
    assert oracle.corank_brute(runs, 5) == [3, 2, 0]
    assert oracle.corank_brute(runs, 6) == [3, 2, 1]
    assert oracle.corank_brute(runs, 7) == [3, 2, 2]


# ---- flexible key sizes (Section 5): the first K bytes are the key ----------------

def _tied_records(n, seed):
    """Records whose key bytes take few values at chosen positions, so prefixes
    of every length tie: bytes 0..11 from {0x00, 0xFF}, byte 40 from three
    values, byte 99 from two; the rest uniform."""
    rec = datagen.uniform(n, seed)
    rng = np.random.default_rng(seed)
    rec[:, :12] = np.where(rng.integers(0, 2, (n, 12)) == 1, 0xFF, 0x00)
    rec[:, 40] = rng.integers(0, 3, n) * 0x70
    rec[:, 99] = rng.integers(0, 2, n)
    return rec


@pytest.mark.parametrize("kb", [1, 2, 7, 8, 9, 11, 12, 13, 41, 99, 100])
def test_key_bytes_matches_python_sorted(kb):
    rec = _tied_records(3000, 50 + kb)
    _, perm = oracle.sort(rec, return_perm=True, key_bytes=kb)
    ref = sorted(range(rec.shape[0]), key=lambda i: bytes(rec[i, :kb]))  # stable
    assert list(perm) == ref


@pytest.mark.parametrize("kb", [3, 10, 16, 100])
def test_key_bytes_matches_numpy_lexsort(kb):
    rec = _tied_records(5000, 70 + kb)
    cols = tuple(rec[:, b] for b in range(kb - 1, -1, -1))  # last key is primary
    want = np.lexsort((np.arange(rec.shape[0]),) + cols)
    _, perm = oracle.sort(rec, return_perm=True, key_bytes=kb)
    np.testing.assert_array_equal(perm.astype(np.int64), want)


@pytest.mark.parametrize("n", [2, 4, 6])
def test_key_bytes_brute_force_tiny(n):
    rng = np.random.default_rng(200 + n)
    for trial in range(20):
        rec = _tied_records(n, 300 + trial)
        kb = int(rng.integers(1, 101))
        _, perm = oracle.sort(rec, return_perm=True, key_bytes=kb)
        assert list(perm) == oracle.brute_force_order([bytes(r[:kb]) for r in rec])


def test_key_bytes_ten_agrees_with_fixed_key_sort():
    rec = _tied_records(4000, 9)
    lib = oracle._load()
    out_a = np.empty_like(rec)
    out_b = np.empty_like(rec)
    perm_a = np.empty(rec.shape[0], dtype=np.uint32)
    perm_b = np.empty(rec.shape[0], dtype=np.uint32)
    assert lib.oracle_sort(oracle._ptr(rec), rec.shape[0], oracle._ptr(out_a), oracle._ptr(perm_a)) == 0
    assert lib.oracle_sort_key(oracle._ptr(rec), rec.shape[0], 10, oracle._ptr(out_b), oracle._ptr(perm_b)) == 0
    np.testing.assert_array_equal(perm_a, perm_b)
    np.testing.assert_array_equal(out_a, out_b)


def test_key_bytes_range():
    rec = datagen.uniform(10, 1)
    for bad in (0, 101):
        with pytest.raises(ValueError):
            oracle.sort(rec, key_bytes=bad)
    assert oracle._load().oracle_sort_key(oracle._ptr(rec), 10, 0, oracle._ptr(rec.copy()), None) == -2
    # a key of all 100 bytes orders whole records; a 1-byte key keeps input order inside each byte value
    out = oracle.sort(_tied_records(500, 4), key_bytes=100)
    assert all(bytes(out[i]) <= bytes(out[i + 1]) for i in range(499))
    rec = _tied_records(500, 5)
    _, perm = oracle.sort(rec, return_perm=True, key_bytes=1)
    for v in (0x00, 0xFF):
        p = perm[rec[perm, 0] == v]
        assert np.all(np.diff(p.astype(np.int64)) > 0)
