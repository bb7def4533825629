"""Serving engine: every request's output equals its oracle sort and its alone-sorted bytes,
under a memory budget that forces queueing, in batched and per-request modes."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

POOL = 300_000


@pytest.fixture(scope="module")
def pool(gpu):
    import torch
    rec = datagen.uniform(POOL, 4242)
    return rec, torch.from_numpy(rec).cuda().view(-1)


def request_plan(count, seed, hi=60_000):
    sizes = datagen.request_sizes(count, seed=seed, lo=50, hi=hi)
    offs = (datagen.words(seed + 1, count) % np.uint64(POOL - hi)).astype(np.int64)
    return [(int(o), int(n)) for o, n in zip(offs, sizes)]


@pytest.mark.parametrize("batched", [True, False])
def test_server_outputs_match_oracle(gpu, pool, batched):
    import torch
    rec, d = pool
    plan = request_plan(120, 77)
    # budget: workspaces + room for only a few large outputs at once -> admission must wait
    budget = gpu.load().leyenda_workspace_bytes(60_000) * (3 if batched else 1) + 60_000 * 100 * 3 + (64 << 20)
    srv = gpu.Server(budget_bytes=budget, slots=3, max_batch=32, max_batch_records=60_000, batched=batched)
    try:
        for tag, (o, n) in enumerate(plan):
            srv.submit(d[o * 100:(o + n) * 100], tag)
        seen = {}
        while len(seen) < len(plan):
            for dn in srv.poll(timeout_s=1.0):
                assert dn["status"] == 0
                o, n = plan[dn["tag"]]
                assert dn["n"] == n and dn["done_s"] >= dn["start_s"] >= dn["submit_s"]
                seen[dn["tag"]] = srv.output(dn).cpu().numpy()
                srv.release(dn["tag"])
        torch.cuda.synchronize()
    finally:
        srv.close()
    for tag, (o, n) in enumerate(plan):
        want = oracle.sort(rec[o:o + n])
        np.testing.assert_array_equal(seen[tag], want)
        if tag % 20 == 0:  # the same request sorted alone gives the same bytes
            alone = gpu.sort(d[o * 100:(o + n) * 100])
            torch.cuda.synchronize()
            np.testing.assert_array_equal(alone.cpu().numpy().reshape(-1, 100), seen[tag])


def test_replay_reports_latencies(gpu, pool):
    _, d = pool
    plan = request_plan(200, 91)
    arrivals = datagen.arrival_times(len(plan), rate_per_s=4000.0, seed=5)
    inputs = [(d.data_ptr() + o * 100, n) for o, n in plan]
    for batched in (True, False):
        lat, mk = gpu.serve_replay(inputs, arrivals, budget_bytes=8 << 30, max_batch_records=60_000, batched=batched)
        assert len(lat) == len(plan) and min(lat) > 0 and mk >= arrivals[-1]


def test_server_errors(gpu, pool):
    _, d = pool
    with pytest.raises(gpu.LeyendaError) as ei:
        gpu.Server(budget_bytes=1 << 20, max_batch_records=1_000_000)
    assert ei.value.status == -3
    with pytest.raises(gpu.LeyendaError) as ei:
        gpu.Server(budget_bytes=1 << 30, slots=0)
    assert ei.value.status == -1
    srv = gpu.Server(budget_bytes=1 << 30, slots=2, max_batch=8, max_batch_records=10_000)
    try:
        with pytest.raises(gpu.LeyendaError):
            srv.submit(d[: 20_000 * 100], 1)  # above max_batch_records
        srv.submit(d[:1000], 5)
        with pytest.raises(gpu.LeyendaError):
            srv.submit(d[:1000], 5)  # tag in use
        got = []
        while not got:
            got = srv.poll(timeout_s=1.0)
        srv.release(5)
        with pytest.raises(gpu.LeyendaError):
            srv.release(5)
    finally:
        srv.close()


def _deep_records(n, seed):
    """Keys that keep big buckets past the third partition level: 90% share key
    bytes 0..7 (they differ in bytes 8..9 only), the rest uniform."""
    rec = datagen.uniform(n, seed)
    m = int(n * 0.9)
    rec[:m, :8] = 0x3C
    return rec


def test_server_second_part_for_deep_buckets(gpu):
    """The batched server's launch sequence runs the first partition levels, then its local
    sorts stand down and a second part runs the deeper levels when big buckets remain;
    outputs of such requests, mixed with ordinary ones in one batch, equal the oracle's."""
    import torch
    deep = _deep_records(1_000_000, 301)
    flat = datagen.uniform(200_000, 302)
    d_deep = torch.from_numpy(deep).cuda().view(-1)
    d_flat = torch.from_numpy(flat).cuda().view(-1)
    srv = gpu.Server(budget_bytes=4 << 30, slots=2, max_batch=8, max_batch_records=1_500_000)
    try:
        srv.submit(d_flat[: 150_000 * 100], 0)
        srv.submit(d_deep, 1)
        srv.submit(d_flat[150_000 * 100:], 2)
        got = {}
        while len(got) < 3:
            for dn in srv.poll(timeout_s=2.0):
                assert dn["status"] == 0
                got[dn["tag"]] = srv.output(dn).cpu().numpy()
                srv.release(dn["tag"])
        torch.cuda.synchronize()
    finally:
        srv.close()
    np.testing.assert_array_equal(got[1], oracle.sort(deep))
    np.testing.assert_array_equal(got[0], oracle.sort(flat[:150_000]))
    np.testing.assert_array_equal(got[2], oracle.sort(flat[150_000:]))
