"""Batched sort (one captured launch sequence for many requests): parity with the oracle,
each request identical alone and in the mix, and repeated graph replays."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_batch(gpu, recs):
    import torch
    ins = [dev(r) for r in recs]
    outs = [torch.empty_like(t) for t in ins]
    gpu.sort_batch(zip(ins, outs))
    torch.cuda.synchronize()
    return [o.cpu().numpy().reshape(-1, 100) for o in outs]


def mixed_requests(seed):
    sizes = [0, 1, 5, 2048, 2049, 4096, 70_000, 250_001, 9_000]
    out = []
    for i, n in enumerate(sizes):
        if i % 3 == 0:
            out.append(datagen.skewed(n, seed + i, nvals=200) if n else np.zeros((0, 100), np.uint8))
        else:
            out.append(datagen.uniform(n, seed + i))
    return out


def test_batch_matches_oracle_and_alone(gpu):
    recs = mixed_requests(500)
    mixed = run_batch(gpu, recs)
    for r, got in zip(recs, mixed):
        np.testing.assert_array_equal(got, oracle.sort(r))
        if r.shape[0]:
            alone = run_batch(gpu, [r])[0]
            np.testing.assert_array_equal(alone, got)  # same bytes alone and in the mix


def test_many_small_requests(gpu):
    rng = np.random.default_rng(7)
    sizes = rng.integers(1, 120, 3000)
    recs = [datagen.skewed(int(n), 2000 + i, nvals=30) for i, n in enumerate(sizes)]
    for r, got in zip(recs, run_batch(gpu, recs)):
        np.testing.assert_array_equal(got, oracle.sort(r))


def test_graph_replays_with_eager_work_between(gpu):
    """The captured sequence is replayed for several batches of different shapes that
    fit its capacity; eager sorts and synchronizations run between the replays."""
    import torch
    first = mixed_requests(900)
    run_batch(gpu, first)  # builds and captures
    for rep in range(4):
        recs = [datagen.uniform(n, 3000 + 10 * rep + j) for j, n in enumerate([333, 50_000 + rep, 17, 2049 * rep])]
        got = run_batch(gpu, recs)
        eager = gpu.sort(dev(recs[1]))  # eager single sort between replays
        torch.cuda.synchronize()
        np.testing.assert_array_equal(eager.cpu().numpy().reshape(-1, 100), oracle.sort(recs[1]))
        for r, g in zip(recs, got):
            np.testing.assert_array_equal(g, oracle.sort(r))


def test_batch_grows_capacity(gpu):
    small = [datagen.uniform(100, 1)]
    run_batch(gpu, small)
    big = [datagen.uniform(600_000, 2), datagen.skewed(400_000, 3)] + [datagen.uniform(10, 4 + i) for i in range(300)]
    for r, g in zip(big, run_batch(gpu, big)):
        np.testing.assert_array_equal(g, oracle.sort(r))


def test_batch_errors(gpu):
    import torch
    a = torch.empty(1000, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        gpu.sort_batch([(a[:500], a[:400])])
    with pytest.raises(gpu.LeyendaError):
        gpu.sort_batch([(a[:500], a[100:600])])  # overlapping input and output
    gpu.sort_batch([])  # empty batch is a no-op
