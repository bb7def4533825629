"""leyenda_sort_noalloc (scratch in a fixed device array, no allocation per
call) against leyenda_sort, through the C ABI: two calls in a row on the
same array, the second smaller, each bit-exact with the allocating entry
point and with the oracle."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


def _call_both(gpu, rec: np.ndarray):
    import torch
    lib = gpu.load()
    n = rec.shape[0]
    dev = torch.from_numpy(np.ascontiguousarray(rec)).cuda()
    a = torch.empty_like(dev)
    b = torch.empty_like(dev)
    s = torch.cuda.current_stream().cuda_stream
    rc = lib.leyenda_sort(dev.data_ptr(), n, a.data_ptr(), s)
    assert rc == 0, lib.leyenda_last_error()
    rc = lib.leyenda_sort_noalloc(dev.data_ptr(), n, b.data_ptr(), s)
    assert rc == 0, lib.leyenda_last_error()
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_noalloc_matches_sort_twice_second_smaller(gpu):
    # a skewed input with duplicate keys (ties, deep levels), then a smaller
    # uniform one: the second call runs on the array the first left behind
    first = datagen.skewed(1_200_000, 61, nvals=512, dup_frac=0.1)
    second = datagen.uniform(300_001, 62)
    for rec in (first, second):
        want = oracle.sort(rec)
        a, b = _call_both(gpu, rec)
        np.testing.assert_array_equal(a, want)
        np.testing.assert_array_equal(b, a)


def test_noalloc_small_and_edge_sizes(gpu):
    for n in (1, 2, 2047, 2048, 2049, 8193):
        rec = datagen.skewed(n, 63 + n, nvals=8, dup_frac=0.5) if n > 2 else datagen.uniform(n, 63)
        a, b = _call_both(gpu, rec)
        np.testing.assert_array_equal(b, a)
        np.testing.assert_array_equal(b, oracle.sort(rec))


def test_noalloc_rejects_sizes_beyond_its_array(gpu):
    import torch
    lib = gpu.load()
    cap = int(lib.leyenda_noalloc_max_records())
    assert cap >= 1_000_000
    n = cap + 1
    a = torch.empty(n * 100, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    s = torch.cuda.current_stream().cuda_stream
    assert lib.leyenda_sort_noalloc(a.data_ptr(), n, b.data_ptr(), s) == -3  # LEYENDA_EBUDGET
    assert b"scratch" in lib.leyenda_last_error()
    assert lib.leyenda_sort_noalloc(a.data_ptr(), 0, b.data_ptr(), s) == 0
    torch.cuda.synchronize()
