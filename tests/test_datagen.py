"""Input generator: determinism, range independence and workload statistics."""
import os
import subprocess
import sys

import numpy as np

import datagen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_deterministic_and_seeded():
    a = datagen.uniform(1000, 2)
    b = datagen.uniform(1000, 2)
    c = datagen.uniform(1000, 3)
    np.testing.assert_array_equal(a, b)
    assert (a != c).any()


def test_range_independent():
    full = datagen.uniform(5000, 4)
    part = datagen.uniform(1000, 4, first=2500)
    np.testing.assert_array_equal(full[2500:3500], part)
    sk = datagen.skewed(3000, 3)
    np.testing.assert_array_equal(sk[1000:2000], datagen.skewed(1000, 3, first=1000))


def test_thread_count_invariant():
    code = ("import sys; sys.path.insert(0, %r); import datagen, hashlib;"
            "print(hashlib.sha256(datagen.skewed(20000, 3).tobytes()).hexdigest())") % ROOT
    outs = []
    for t in ("1", "5"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                                   text=True, check=True).stdout.strip())
    assert outs[0] == outs[1]


def test_numpy_words_match_c():
    w = datagen.words(17, 50, k=3)
    assert [int(x) for x in w[:5]] == [datagen.word(17, i, 3) for i in range(5)]


def test_uniform_bytes_look_uniform():
    a = datagen.uniform(200000, 2)
    counts = np.bincount(a[:, 0], minlength=256)
    exp = a.shape[0] / 256
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert chi2 < 400  # 255 dof: mean 255, sd ~22.6


def test_indexed_payload_holds_index():
    a = datagen.indexed(100, 2, first=77)
    idx = a[:, 10:18].copy().view(np.uint64).ravel()
    np.testing.assert_array_equal(idx, np.arange(77, 177, dtype=np.uint64))
    np.testing.assert_array_equal(a[:, :10], datagen.uniform(100, 2, first=77)[:, :10])


def test_skewed_statistics():
    n = 400000
    a = datagen.skewed(n, 3)
    pref = (a[:, 0].astype(np.uint32) << 24) | (a[:, 1].astype(np.uint32) << 16) | \
           (a[:, 2].astype(np.uint32) << 8) | a[:, 3].astype(np.uint32)
    top = datagen.zipf_value(3, 1)
    p1 = datagen.zipf_pmf(1)
    assert 0.19 < p1 < 0.21  # Zipf(1.2) over 65,536 values: ~19.8% on rank 1
    frac = float((pref == top).mean())
    assert abs(frac - p1) < 0.005
    # exact-duplicate keys: about 5% of records copy an earlier record's key
    keys = a[:, :10].copy().view(np.dtype((np.void, 10))).ravel()
    _, first_idx, counts = np.unique(keys, return_index=True, return_counts=True)
    dup_records = n - first_idx.size
    assert 0.045 < dup_records / n < 0.056


def test_request_sizes_and_arrivals():
    s = datagen.request_sizes(20000)
    assert s.min() >= 1000 and s.max() <= 10_000_000
    med = float(np.median(s))
    assert 7e4 < med < 1.4e5  # log-uniform on [1e3, 1e7]: median 1e5
    t = datagen.arrival_times(20000, rate_per_s=50.0)
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] / 20000 - 1 / 50.0) < 0.002


def test_ascii_keys_printable_and_uniform():
    n = 200000
    a = datagen.ascii(n, datagen.SEED_ASCII)
    k = a[:, :10]
    assert k.min() == datagen.ASCII_LO and k.max() == datagen.ASCII_LO + datagen.ASCII_VALUES - 1
    # the payload is the uniform generator's; the range of records is independent
    np.testing.assert_array_equal(a[:, 10:], datagen.uniform(n, datagen.SEED_ASCII)[:, 10:])
    np.testing.assert_array_equal(a[500:900], datagen.ascii(400, datagen.SEED_ASCII, first=500))
    exp = n / datagen.ASCII_VALUES
    for b in (0, 3, 4, 9):  # chunks from each of the three words and both ends of one
        counts = np.bincount(k[:, b], minlength=256)[datagen.ASCII_LO:datagen.ASCII_LO + datagen.ASCII_VALUES]
        chi2 = float(((counts - exp) ** 2 / exp).sum())
        assert chi2 < 170  # 94 dof: mean 94, sd ~13.7
    # byte positions are independent: the first two bytes take all 95 x 95 pairs
    assert np.unique(k[:, 0].astype(np.int32) * 256 + k[:, 1]).size == 95 * 95
