"""Flexible key sizes (Section 5's next step): leyenda_sort_keyed against the
oracle's stable sort on the first K bytes, byte for byte.

Inputs tie on prefixes of every length, so the prefix sort (K <= 10, with the
bytes past the key cleared) and every tie round (K > 10: runs of equal
leading bytes ordered by six more key bytes per round) are exercised."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


def _sort_keyed(gpu, rec, kb):
    import torch
    dev = torch.from_numpy(np.ascontiguousarray(rec)).cuda()
    out = gpu.sort_keyed(dev, kb)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _same(got, want, what):
    if not np.array_equal(got, want):
        diff = np.nonzero((got != want).any(axis=1))[0]
        raise AssertionError(f"{what}: {diff.size} records differ, first at {int(diff[0])}")


def tied(n, seed):
    """Bytes 0..11 from {0x00, 0xFF} (4,096 prefixes of 12 bytes), byte 40 from
    three values, byte 99 from two; the rest uniform."""
    rec = datagen.uniform(n, seed)
    rng = np.random.default_rng(seed)
    rec[:, :12] = np.where(rng.integers(0, 2, (n, 12)) == 1, 0xFF, 0x00)
    rec[:, 40] = rng.integers(0, 3, n) * 0x70
    rec[:, 99] = rng.integers(0, 2, n)
    return rec


def long_runs(n, seed):
    """Copies of 40 distinct records with a few bytes varied: ties run through
    most of the 100 bytes (bytes 17, 58 and 95 take 2-3 values each), so a
    100-byte key needs every round."""
    rng = np.random.default_rng(seed)
    base = datagen.uniform(40, seed)
    rec = base[rng.integers(0, 40, n)].copy()
    rec[:, 17] = rng.integers(0, 2, n)
    rec[:, 58] = rng.integers(0, 3, n) + 0x80
    rec[:, 95] = rng.integers(0, 2, n) * 0xFF
    return rec


KEYS = [1, 2, 7, 8, 9, 10, 11, 12, 15, 16, 17, 22, 23, 41, 59, 96, 99, 100]


@pytest.mark.parametrize("kb", KEYS)
def test_keyed_tied_prefixes(gpu, kb):
    rec = tied(20_003, 60 + kb)
    _same(_sort_keyed(gpu, rec, kb), oracle.sort(rec, key_bytes=kb), f"tied kb={kb}")


@pytest.mark.parametrize("kb", [10, 16, 18, 59, 60, 95, 96, 100])
def test_keyed_long_runs(gpu, kb):
    rec = long_runs(30_011, 80 + kb)
    _same(_sort_keyed(gpu, rec, kb), oracle.sort(rec, key_bytes=kb), f"long runs kb={kb}")


@pytest.mark.parametrize("n", [1, 2, 3, 5, 1000, 4097])
@pytest.mark.parametrize("kb", [3, 10, 33, 100])
def test_keyed_small_and_ragged(gpu, n, kb):
    rec = long_runs(n, n + kb)
    _same(_sort_keyed(gpu, rec, kb), oracle.sort(rec, key_bytes=kb), f"n={n} kb={kb}")


def test_keyed_equal_keys_keep_input_order(gpu):
    """Every record has the same 60 leading bytes: one run through all rounds up
    to the key's end; the output must be the input order."""
    rec = datagen.uniform(50_000, 13)
    rec[:, :60] = 0x3C
    got = _sort_keyed(gpu, rec, 60)
    _same(got, rec, "all keys equal")
    _same(got, oracle.sort(rec, key_bytes=60), "all keys equal (oracle)")


def test_keyed_ten_is_leyenda_sort(gpu):
    import torch
    rec = datagen.skewed(100_000, 3)
    dev = torch.from_numpy(rec).cuda()
    a = gpu.sort(dev)
    b = gpu.sort_keyed(dev, 10)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("kb", [4, 20])
def test_keyed_output_parts_skewed(gpu, kb):
    """8,400,953 records (four output parts): Zipf prefixes with 5% duplicate
    10-byte keys, so a 20-byte key resolves many two-record runs by payload
    bytes, and a 4-byte key ties whole Zipf buckets."""
    n = 8_388_608 + 12_345
    rec = datagen.skewed(n, 8)
    _same(_sort_keyed(gpu, rec, kb), oracle.sort(rec, key_bytes=kb), f"skewed kb={kb}")


def test_keyed_bad_key_size(gpu):
    import torch
    dev = torch.from_numpy(datagen.uniform(10, 1)).cuda()
    for bad in (0, 101):
        with pytest.raises(gpu.LeyendaError):
            gpu.sort_keyed(dev, bad)
