"""Parity of the in-HBM GPU sort (leyenda_sort and its steps) with the CPU oracle.

Every comparison is byte for byte: the output of a stable key sort is unique.
"""
import numpy as np
import pytest

import datagen
import oracle
from tests.golden import pad_key, worked_example

pytestmark = pytest.mark.gpu


def run_sort(ley, rec: np.ndarray) -> np.ndarray:
    import torch
    dev = torch.from_numpy(np.ascontiguousarray(rec)).cuda()
    out = ley.sort(dev)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def assert_same(got: np.ndarray, want: np.ndarray, what: str = ""):
    if not np.array_equal(got, want):
        diff = np.nonzero((got != want).any(axis=1))[0]
        raise AssertionError(f"{what}: {diff.size} records differ, first at {int(diff[0])}")


# ---- step-level parity ------------------------------------------------------------

def _want_tuples(rec: np.ndarray, key_bytes: int):
    """Expected key-pointer tuple words written out from the definition: key
    bytes 0..7 big-endian, key bytes 8..9 big-endian above the record index,
    bytes at and past key_bytes cleared."""
    key = rec[:, :10].astype(np.uint64).copy()
    key[:, key_bytes:] = 0
    hi = np.zeros(rec.shape[0], dtype=np.uint64)
    for b in range(8):
        hi = (hi << np.uint64(8)) | key[:, b]
    k16 = (key[:, 8] << np.uint64(8)) | key[:, 9]
    lo = (k16 << np.uint64(32)) | np.arange(rec.shape[0], dtype=np.uint64)
    return hi, lo


# 3 * 8192 + 77 records: three full extraction tiles of the default shape and
# a ragged fourth; 2,048-key tiles (tile_items 8) make it thirteen
@pytest.mark.parametrize("key_bytes,digit_bits,tile_items", [
    (10, 8, 32), (9, 8, 32), (4, 8, 32), (10, 5, 32), (1, 4, 8), (10, 8, 8), (8, 7, 16)])
def test_extract_step(gpu, key_bytes, digit_bits, tile_items):
    """The sort's own extraction kernel (first stage of leyenda_sort): tuples
    and the histogram of the leading digit, with the key masks of shorter keys."""
    import torch
    n = 3 * 8192 + 77
    rec = datagen.uniform(n, 31)
    rec[: n // 3, :3] = rec[0, :3]  # a third of the keys share a 3-byte prefix
    old = gpu.get_params()
    try:
        gpu.set_params(digit_bits=digit_bits, tile_items=tile_items)
        hi, lo, hist = gpu.debug_extract(torch.from_numpy(rec).cuda(), key_bytes)
        torch.cuda.synchronize()
    finally:
        gpu.set_params(**old)
    want_hi, want_lo = _want_tuples(rec, key_bytes)
    np.testing.assert_array_equal(hi.cpu().numpy().view(np.uint64), want_hi)
    np.testing.assert_array_equal(lo.cpu().numpy().view(np.uint64), want_lo)
    lead = (want_hi >> np.uint64(64 - digit_bits)).astype(np.int64)
    np.testing.assert_array_equal(hist.cpu().numpy(), np.bincount(lead, minlength=256))


def test_extract_worked_example_histogram(gpu):
    import torch
    ex = worked_example()
    rec = datagen.uniform(len(ex["keys"]), 5)
    for i, k in enumerate(ex["keys"]):
        rec[i, :10] = np.frombuffer(pad_key(k), dtype=np.uint8)
    _, _, hist = gpu.debug_extract(torch.from_numpy(rec).cuda())
    h = hist.cpu().numpy()
    assert {b: int(c) for b, c in enumerate(h) if c} == ex["counts"]


def test_gather_step(gpu):
    import torch
    rec = datagen.uniform(5000, 32)
    idx = np.random.default_rng(1).permutation(5000).astype(np.int32)
    out = gpu.debug_gather(torch.from_numpy(rec).cuda(), torch.from_numpy(idx).cuda())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), rec[idx])


# ---- end-to-end parity ------------------------------------------------------------

SIZES = [1, 2, 3, 7, 255, 256, 257, 2047, 2048, 2049, 4095, 4096, 4097, 8193, 65537, 300_001]


@pytest.mark.parametrize("n", SIZES)
def test_sort_uniform_sizes(gpu, n):
    rec = datagen.uniform(n, 40 + n % 97)
    assert_same(run_sort(gpu, rec), oracle.sort(rec), f"uniform n={n}")


def _keys(n, seed):
    return datagen.uniform(n, seed)


def pattern(name: str, n: int) -> np.ndarray:
    rec = datagen.uniform(n, 77)
    rng = np.random.default_rng(5)
    if name == "all_equal":
        rec[:, :10] = 0x5A
    elif name == "only_byte9":
        rec[:, :9] = 0x11
    elif name == "bytes_7_8_only":  # keys differ only across the hi/lo tuple split
        rec[:, :7] = 0x22
        rec[:, 9] = 0x33
        rec[:, 7] = rng.integers(0, 3, n)
        rec[:, 8] = rng.integers(0, 3, n)
    elif name == "sorted":
        rec = oracle.sort(rec)
    elif name == "reverse":
        rec = oracle.sort(rec)[::-1].copy()
    elif name == "few_distinct":
        vals = datagen.uniform(16, 3)[:, :10]
        rec[:, :10] = vals[rng.integers(0, 16, n)]
    elif name == "shared_prefix":  # first 5 bytes constant: constant digits are skipped
        rec[:, :5] = 0xC3
    elif name == "extremes":
        rec[:, :10] = np.where(rng.integers(0, 2, (n, 10)) == 1, 0xFF, 0x00)
    elif name == "skewed":
        rec = datagen.skewed(n, 3)
    elif name == "skewed_narrow":  # Zipf over 64 values: huge equal-prefix buckets + duplicates
        rec = datagen.skewed(n, 8, nvals=64, dup_frac=0.2)
    elif name == "one_big_bucket":  # 90% of keys share 8 bytes, differing in bytes 8..9
        m = int(n * 0.9)
        rec[:m, :8] = 0x7E
    elif name == "ascii":  # printable keys: 95 of the 256 digit values occur at every level
        rec = datagen.ascii(n, datagen.SEED_ASCII)
    else:
        raise KeyError(name)
    return rec


PATTERNS = ["all_equal", "only_byte9", "bytes_7_8_only", "sorted", "reverse", "few_distinct", "shared_prefix",
            "extremes", "skewed", "skewed_narrow", "one_big_bucket", "ascii"]


@pytest.mark.parametrize("name", PATTERNS)
def test_sort_patterns(gpu, name):
    rec = pattern(name, 200_003)
    assert_same(run_sort(gpu, rec), oracle.sort(rec), name)


def test_sort_worked_example(gpu):
    ex = worked_example()
    rec = datagen.uniform(len(ex["keys"]), 9)
    for i, k in enumerate(reversed(ex["keys"])):
        rec[i, :10] = np.frombuffer(pad_key(k), dtype=np.uint8)
    got = run_sort(gpu, rec)
    assert [bytes(r[:10]).rstrip(b"\x00") for r in got] == ex["sorted"]
    assert_same(got, oracle.sort(rec), "worked example")


@pytest.mark.parametrize("params", [
    dict(big_threshold=1), dict(big_threshold=64), dict(big_threshold=2048),
    dict(tiny_threshold=1), dict(tiny_threshold=64), dict(tile_items=8),
    dict(tile_items=8, big_threshold=300, tiny_threshold=5), dict(scatter_threads=256),
    dict(scatter_threads=256, tile_items=8, big_threshold=1), dict(local_threads=512),
    dict(local_threads=512, tiny_threshold=1), dict(local_threads=512, tiny_threshold=64, big_threshold=2048),
    dict(tile_items=16, scatter_threads=512), dict(tile_items=32, scatter_threads=512),
    dict(tile_items=16, scatter_threads=1024, big_threshold=100), dict(tiny_threshold=256),
    dict(tiny_threshold=160, big_threshold=300),
    dict(digit_bits=4), dict(digit_bits=5), dict(digit_bits=6, big_threshold=64),
    dict(digit_bits=7, tile_items=8), dict(digit_bits=4, big_threshold=1, tiny_threshold=5),
    dict(digit_bits=6, tile_items=16, scatter_threads=512, local_threads=256),
])
def test_params_do_not_change_output(gpu, params):
    rec = pattern("skewed_narrow", 150_000)
    want = oracle.sort(rec)
    old = gpu.get_params()
    try:
        gpu.set_params(**params)
        assert_same(run_sort(gpu, rec), want, str(params))
    finally:
        gpu.set_params(**old)


@pytest.mark.parametrize("digit_bits", [4, 5, 6, 7])
@pytest.mark.parametrize("name", ["uniform", "bytes_7_8_only", "shared_prefix", "one_big_bucket", "ascii"])
def test_digit_widths(gpu, digit_bits, name):
    """Narrower partition digits (Algorithm 1 with 2^digit_bits buckets per
    level): digits straddle the byte boundaries and the two tuple words, and
    the level count grows to ceil(80 / digit_bits)."""
    import torch
    n = 1_000_003
    rec = datagen.uniform(n, 95) if name == "uniform" else pattern(name, n)
    want = oracle.sort(rec)
    old = gpu.get_params()
    try:
        gpu.set_params(digit_bits=digit_bits)
        assert_same(run_sort(gpu, rec), want, f"{name} digit_bits={digit_bits}")
        st = gpu.stats(torch.cuda.current_stream())
    finally:
        gpu.set_params(**old)
    assert st["guard"] == 0
    if name == "uniform":
        assert st["moved"][0] == n and st["levels"] >= 2


def test_deterministic_repeats(gpu):
    rec = datagen.skewed(400_000, 12)
    a = run_sort(gpu, rec)
    for _ in range(3):
        assert_same(run_sort(gpu, rec), a, "repeat")


def test_small_config_full_compare(gpu):
    """1,000,000 uniform records (100 MB): the whole output against the oracle."""
    rec = datagen.uniform(1_000_000, datagen.SEED_SMALL)
    got = run_sort(gpu, rec)
    assert_same(got, oracle.sort(rec), "1e6 uniform")


@pytest.mark.parametrize("kind", ["uniform", "skewed"])
def test_tile_offsets_across_scan_chunks(gpu, kind):
    """3,000,000 records: the level-0 bucket spans six chunks of the tile-offset
    scan (carries between chunks) and level-1 chunks hold many buckets."""
    n = 3_000_000
    rec = datagen.uniform(n, 91) if kind == "uniform" else datagen.skewed(n, 92)
    assert_same(run_sort(gpu, rec), oracle.sort(rec), f"3e6 {kind}")


def test_small_tiles_many_chunks(gpu):
    """2,048-key tiles: 1,200,000 records make 586 level-0 tiles (ten scan chunks)."""
    rec = datagen.skewed(1_200_000, 93, nvals=256, dup_frac=0.1)
    want = oracle.sort(rec)
    old = gpu.get_params()
    try:
        gpu.set_params(tile_items=8)
        assert_same(run_sort(gpu, rec), want, "tile_items=8")
    finally:
        gpu.set_params(**old)


@pytest.mark.parametrize("name", ["uniform", "few_distinct", "all_equal", "one_big_bucket", "skewed_narrow", "ascii"])
def test_output_parts(gpu, name):
    """8,400,953 records: above the 8 Mi threshold the local sorts run per output
    part (four) with each part's gather on a side stream.  Equal-key ranges
    (16 keys; one key) span part boundaries; one bucket of 90% of the keys and
    Zipf prefixes put tasks of deep levels on both sides of them."""
    import torch
    n = 8_388_608 + 12_345
    rec = datagen.uniform(n, 94) if name == "uniform" else pattern(name, n)
    got = run_sort(gpu, rec)
    assert_same(got, oracle.sort(rec), f"parts {name}")
    st = gpu.stats(torch.cuda.current_stream())
    assert st["guard"] == 0 and st["tasks"] > 0


@pytest.mark.parametrize("n", [2049, 300_001, 3_000_017, 20_000_003])
def test_sort_ascii_levels(gpu, n):
    """Printable keys (95 values per byte): buckets shrink 95-fold per digit, so
    these sizes end after one, two, two and three device-wide levels (the last
    with about 2,216 records per second-level bucket, above the 2,048 limit)."""
    import torch
    rec = datagen.ascii(n, datagen.SEED_ASCII + n % 5)
    assert_same(run_sort(gpu, rec), oracle.sort(rec), f"ascii n={n}")
    st = gpu.stats(torch.cuda.current_stream())
    assert st["guard"] == 0
    if n == 20_000_003:
        assert st["moved"][2] > 0


def test_stats_uniform(gpu):
    import torch
    rec = datagen.uniform(1_000_000, 1)
    run_sort(gpu, rec)
    st = gpu.stats(torch.cuda.current_stream())
    assert st["guard"] == 0
    assert st["moved"][0] == 1_000_000  # the whole array is partitioned on byte 0
    assert st["tasks"] > 0


def test_error_codes(gpu):
    import torch
    lib = gpu.load()
    a = torch.empty(1000 * 100, dtype=torch.uint8, device="cuda")
    b = torch.empty(1000 * 100, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert lib.leyenda_sort(None, 10, b.data_ptr(), s) == -1
    assert lib.leyenda_sort(a.data_ptr(), 10, a.data_ptr() + 500, s) == -1  # overlap
    assert lib.leyenda_sort(a.data_ptr() + 1, 10, b.data_ptr(), s) == -1  # misaligned
    assert lib.leyenda_sort(a.data_ptr(), 1 << 33, b.data_ptr(), s) == -5
    assert lib.leyenda_sort(a.data_ptr(), 0, b.data_ptr(), s) == 0
    with pytest.raises(gpu.LeyendaError):
        gpu.set_params(big_threshold=0)
    torch.cuda.synchronize()


def test_concurrent_sorts_share_the_side_stream(gpu):
    """Sorts of 8 Mi records or more on two caller streams at once, from two
    threads: their output-part gathers share the library's one side stream per
    device (each stream's sorts keep their own events), and both outputs must
    equal the oracle's."""
    import threading
    import torch
    n = 8_388_608 + 4_321
    recs = [datagen.uniform(n, 140), pattern("skewed_narrow", n)]
    wants = [oracle.sort(r, threads=0) for r in recs]
    errors = []

    def work(k):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                dev = torch.from_numpy(recs[k]).cuda()
                out = torch.empty_like(dev)
                for _ in range(3):
                    gpu.sort(dev, out=out, stream=s)
                    s.synchronize()
                    if not np.array_equal(out.cpu().numpy(), wants[k]):
                        errors.append(f"stream {k}: output differs")
        except Exception as exc:  # reported below
            errors.append(f"stream {k}: {exc!r}")

    threads = [threading.Thread(target=work, args=(k,)) for k in (0, 1)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=240)
    assert not errors, errors
