"""Parity at the full sizes of the five workload configurations, in the launch
configuration bench.py times (default parameters).

The in-HBM workloads (10 GB uniform, 20 GB skewed, 20 GB printable keys) are
compared record for record with the oracle's sort, run on every host thread.
The 60 GB external output, which a host sort would have to hold twice over,
is checked through the properties that fix a stable sort's output uniquely --
keys non-decreasing, the same record multiset (order-free hash), equal keys in
input order -- plus output positions of sampled records computed one by one
by the oracle.
"""
import time

import numpy as np
import pytest

import datagen
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _internal(gpu, n, fill, seed):
    import torch
    host = gpu.pinned_empty(n * 100)
    fill(host.data_ptr(), n, seed)
    dev = host.to("cuda:0", non_blocking=True)
    out = gpu.sort(dev)
    torch.cuda.synchronize()
    st = gpu.stats(torch.cuda.current_stream())
    assert st["guard"] == 0
    del dev
    got = out.cpu().numpy().reshape(n, 100)
    del out
    torch.cuda.empty_cache()
    rec = host.numpy().reshape(n, 100)
    t0 = time.perf_counter()
    want = oracle.sort(rec, threads=0)
    print(f"oracle: {n:,} records in {time.perf_counter() - t0:.1f} s on {oracle.host_threads()} threads", flush=True)
    if not np.array_equal(got, want):
        bad = np.nonzero((got != want).any(axis=1))[0]
        raise AssertionError(f"{bad.size} records differ from the oracle, first at {int(bad[0])}")
    del rec, got, want
    gpu.pinned_free(host)
    return st


@pytest.mark.timeout(900)
def test_internal_10gb_uniform(gpu):
    """100,000,000 x 100-byte records (10 GB), uniform keys, seed 2."""
    st = _internal(gpu, 100_000_000, datagen.fill_uniform, datagen.SEED_INTERNAL)
    assert st["moved"][0] == 100_000_000


@pytest.mark.timeout(1200)
def test_internal_20gb_skewed(gpu):
    """200,000,000 records (20 GB): Zipf(1.2) 4-byte prefixes over 65,536 values, 5% duplicate keys."""
    _internal(gpu, 200_000_000, datagen.fill_skewed, datagen.SEED_SKEWED)


@pytest.mark.timeout(1200)
def test_internal_20gb_ascii(gpu):
    """200,000,000 records (20 GB) with printable ASCII keys (95 values per byte)."""
    _internal(gpu, 200_000_000, datagen.fill_ascii, datagen.SEED_ASCII)


@pytest.mark.timeout(1500)
def test_external_60gb_30gb_budget(gpu):
    """600,000,000 records (60 GB) in pinned host memory, device budget 30 GB: runs + merge."""
    import torch
    n = 600_000_000
    budget = 30 * 10**9
    # exact-size pinned buffers (60 GB each, no allocator rounding)
    a = gpu.pinned_empty(n * 100)
    datagen.fill_uniform(a.data_ptr(), n, datagen.SEED_EXTERNAL)
    rec = a.numpy().reshape(n, 100)
    h_in = oracle.multiset_hash(rec)
    probes_idx = np.random.default_rng(4).integers(0, n, 32)
    probes = rec[probes_idx].copy()
    _, k = gpu.plan_runs(n, budget)
    t0 = time.perf_counter()
    runs, bounds = gpu.sort_runs(a, budget, host_runs=a)  # runs written over the input
    t_runs = time.perf_counter() - t0
    assert len(bounds) - 1 == k and k > 1
    # output in pageable memory: the pinned limit of the host (64 GiB) holds the input only
    out = np.empty((n, 100), dtype=np.uint8)
    t0 = time.perf_counter()
    gpu.merge(runs, bounds, budget, host_out=torch.from_numpy(out).view(-1))
    t_merge = time.perf_counter() - t0
    print(f"external 60 GB: {k} runs in {t_runs:.2f} s, merge in {t_merge:.2f} s "
          f"({n * 100 / (t_runs + t_merge) / 1e9:.1f} GB/s of records end to end)", flush=True)
    assert oracle.first_unsorted(out) == -1
    assert oracle.multiset_hash(out) == h_in
    # 10-byte uniform keys: equal keys are not expected among 6e8 (about 1.5e-7
    # pairs), so stability is vacuous and a probe's position is its count of smaller keys
    assert oracle.equal_neighbours(out) == 0
    pos = oracle.count_less(out, probes)
    for p, r in zip(pos, probes):
        np.testing.assert_array_equal(out[int(p)], r)
    del rec, out, runs
    gpu.pinned_free(a)


@pytest.mark.timeout(1500)
def test_external_60gb_one_call(gpu):
    """The same 60 GB workload through leyenda_sort_external (runs + merge, the
    last two runs kept on the device), runs written over the input."""
    import torch
    n = 600_000_000
    budget = 30 * 10**9
    a = gpu.pinned_empty(n * 100)
    datagen.fill_uniform(a.data_ptr(), n, datagen.SEED_EXTERNAL)
    rec = a.numpy().reshape(n, 100)
    h_in = oracle.multiset_hash(rec)
    probes = rec[np.random.default_rng(5).integers(0, n, 32)].copy()
    out = np.empty((n, 100), dtype=np.uint8)
    t0 = time.perf_counter()
    gpu.sort_external(a, budget, host_out=torch.from_numpy(out).view(-1))
    dt = time.perf_counter() - t0
    print(f"external 60 GB in one call: {dt:.2f} s ({n * 100 / dt / 1e9:.1f} GB/s of records)", flush=True)
    assert oracle.first_unsorted(out) == -1
    assert oracle.multiset_hash(out) == h_in
    assert oracle.equal_neighbours(out) == 0
    pos = oracle.count_less(out, probes)
    for p, r in zip(pos, probes):
        np.testing.assert_array_equal(out[int(p)], r)
    del rec, out
    gpu.pinned_free(a)


@pytest.mark.timeout(1500)
def test_external_60gb_keys_only(gpu):
    """The same 60 GB input, keys-only: all 600,000,000 tuples sorted on the
    device within the 30 GB budget, records gathered from the pinned input."""
    import torch
    n = 600_000_000
    budget = 30 * 10**9
    a = gpu.pinned_empty(n * 100)
    datagen.fill_uniform(a.data_ptr(), n, datagen.SEED_EXTERNAL)
    rec = a.numpy().reshape(n, 100)
    h_in = oracle.multiset_hash(rec)
    probes = rec[np.random.default_rng(5).integers(0, n, 32)].copy()
    out = np.empty((n, 100), dtype=np.uint8)
    t0 = time.perf_counter()
    gpu.sort_external_keys(a, budget, host_out=torch.from_numpy(out).view(-1))
    dt = time.perf_counter() - t0
    print(f"external 60 GB keys-only: {dt:.2f} s ({n * 100 / dt / 1e9:.1f} GB/s of records)", flush=True)
    del rec
    gpu.pinned_free(a)
    assert oracle.first_unsorted(out) == -1
    assert oracle.multiset_hash(out) == h_in
    assert oracle.equal_neighbours(out) == 0  # uniform 10-byte keys: no equal pair expected
    pos = oracle.count_less(out, probes)
    for p, r in zip(pos, probes):
        np.testing.assert_array_equal(out[int(p)], r)
    del out


@pytest.mark.timeout(900)
def test_serving_stream_config(gpu):
    """Requests log-uniform in [1e3, 1e7] records from the serving workload, 32 GB budget,
    batched server: each output equals its oracle sort, and equals the request sorted alone."""
    import torch
    pool_n = 10_000_000
    pool = datagen.uniform(pool_n, datagen.SEED_REQUEST_BASE)
    d = torch.from_numpy(pool).cuda().view(-1)
    count = 40
    sizes = datagen.request_sizes(count)
    offs = (datagen.words(datagen.SEED_REQUEST_BASE + 1, count) % np.uint64(pool_n)).astype(np.int64)
    offs = np.minimum(offs, pool_n - sizes)
    srv = gpu.Server(budget_bytes=32 * 10**9, slots=3, max_batch=256, max_batch_records=10_000_000)
    got = {}
    try:
        for t in range(count):
            srv.submit(d[int(offs[t]) * 100:(int(offs[t]) + int(sizes[t])) * 100], t)
        while len(got) < count:
            for dn in srv.poll(timeout_s=2.0):
                assert dn["status"] == 0
                got[dn["tag"]] = srv.output(dn).cpu().numpy()
                srv.release(dn["tag"])
    finally:
        srv.close()
    for t in range(count):
        o, n = int(offs[t]), int(sizes[t])
        np.testing.assert_array_equal(got[t], oracle.sort(pool[o:o + n]))
    for t in np.argsort(sizes)[-3:]:
        o, n = int(offs[t]), int(sizes[t])
        alone = gpu.sort(d[o * 100:(o + n) * 100])
        torch.cuda.synchronize()
        np.testing.assert_array_equal(alone.cpu().numpy().reshape(-1, 100), got[int(t)])
