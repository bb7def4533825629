"""Parity of the limited-memory path (sorted runs + k-way merge) with the CPU oracle."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


def pinned(a: np.ndarray):
    import torch
    t = torch.empty(a.size, dtype=torch.uint8, pin_memory=True)
    t.numpy()[:] = a.reshape(-1)
    return t


def budget_for_runs(gpu, n, k):
    """Smallest budget giving at most k runs (found with the library's own planner)."""
    lo, hi = 1 << 16, 1 << 40
    while lo < hi:
        m = (lo + hi) // 2
        try:
            _, kk = gpu.plan_runs(n, m)
            ok = kk <= k
        except gpu.LeyendaError:
            ok = False
        if ok:
            hi = m
        else:
            lo = m + 1
    return lo


@pytest.mark.parametrize("runs", [1, 3, 10])
def test_runs_then_merge_uniform(gpu, runs):
    n = 150_001
    rec = datagen.uniform(n, 60 + runs)
    host = pinned(rec)
    budget = budget_for_runs(gpu, n, runs)
    out_runs, bounds = gpu.sort_runs(host, budget)
    assert bounds[0] == 0 and bounds[-1] == n and len(bounds) - 1 == runs
    got_runs = out_runs.numpy().reshape(n, 100)
    for a, b in zip(bounds, bounds[1:]):
        np.testing.assert_array_equal(got_runs[a:b], oracle.sort(rec[a:b]))
    merged = gpu.merge(out_runs, bounds, budget_bytes=3_000_000)  # forces many chunks
    np.testing.assert_array_equal(merged.numpy().reshape(n, 100), oracle.sort(rec))


def test_ties_straddle_runs_in_place(gpu):
    """Many exact-duplicate keys spread over every run; runs written over their input."""
    n = 120_000
    rec = datagen.skewed(n, 9, nvals=40, dup_frac=0.3)
    host = pinned(rec)
    budget = budget_for_runs(gpu, n, 7)
    runs, bounds = gpu.sort_runs(host, budget, host_runs=host)  # in place
    assert len(bounds) - 1 == 7
    merged = gpu.merge(runs, bounds, budget_bytes=2_000_000)
    np.testing.assert_array_equal(merged.numpy().reshape(n, 100), oracle.sort(rec))


@pytest.mark.parametrize("k", [2, 5, 33])
def test_merge_of_given_runs(gpu, k):
    """Merge of runs cut at uneven bounds (including empty runs), sorted by the oracle."""
    n = 90_000
    rec = datagen.skewed(n, 11 + k, nvals=300)
    rng = np.random.default_rng(k)
    cuts = np.sort(rng.integers(0, n, k - 1))
    bounds = [0] + [int(c) for c in cuts] + [n]
    if k > 2:
        bounds[2] = bounds[1]  # one empty run
    runs = np.concatenate([oracle.sort(rec[a:b]) for a, b in zip(bounds, bounds[1:])])
    merged = gpu.merge(pinned(runs), bounds, budget_bytes=1_500_000)
    # stable merge of runs = stable sort of the original input (runs are input ranges)
    np.testing.assert_array_equal(merged.numpy().reshape(n, 100), oracle.sort(rec))


def test_merge_into_pageable_output(gpu):
    import torch
    n = 80_000
    rec = datagen.uniform(n, 71)
    budget = budget_for_runs(gpu, n, 4)
    runs, bounds = gpu.sort_runs(pinned(rec), budget)
    out = np.empty((n, 100), dtype=np.uint8)
    gpu.merge(runs, bounds, budget_bytes=2_000_000, host_out=torch.from_numpy(out).view(-1))
    np.testing.assert_array_equal(out, oracle.sort(rec))


def test_tiny_and_single(gpu):
    for n in (1, 2, 37):
        rec = datagen.uniform(n, 3)
        runs, bounds = gpu.sort_runs(pinned(rec), 64 << 20)
        merged = gpu.merge(runs, bounds, budget_bytes=64 << 20)
        np.testing.assert_array_equal(merged.numpy().reshape(n, 100), oracle.sort(rec))


def test_external_errors(gpu):
    import torch
    lib = gpu.load()
    rec = datagen.uniform(1000, 4)
    pageable = torch.from_numpy(rec.reshape(-1).copy())
    with pytest.raises(gpu.LeyendaError) as ei:
        gpu.sort_runs(pageable, 64 << 20)
    assert ei.value.status == -1
    with pytest.raises(gpu.LeyendaError) as ei:
        gpu.sort_runs(pinned(rec), 1000)  # far below one run's footprint
    assert ei.value.status == -3
    with pytest.raises(gpu.LeyendaError) as ei:
        gpu.sort_runs(pinned(rec), budget_for_runs(gpu, 1000, 9), k_max=3)
    assert ei.value.status == -3
    assert lib is not None


# ---- keys-only variant: all tuples sorted on the device; records scattered into a pinned output
#      by a second in-order read, or gathered from the pinned input for a pageable one ----

@pytest.mark.parametrize("kind,pinned_out", [("uniform", True), ("uniform", False), ("ties", True),
                                             ("ties", False), ("few", True)])
def test_keys_only_matches_oracle(gpu, kind, pinned_out):
    """The input streams in about twelve chunks (twice for a pinned output)
    and a pageable output leaves in about seven, so equal keys straddle chunk
    boundaries on both sides."""
    import torch
    n = 250_007
    if kind == "uniform":
        rec = datagen.uniform(n, 81)
    elif kind == "ties":
        rec = datagen.skewed(n, 82, nvals=40, dup_frac=0.3)
    else:  # eight distinct keys: every bucket is far above the local capacity
        rec = datagen.uniform(n, 83)
        rec[:, :10] = datagen.uniform(8, 84)[np.arange(n) % 8, :10]
    host = pinned(rec)
    out = torch.empty(n * 100, dtype=torch.uint8, pin_memory=pinned_out)
    gpu.sort_external_keys(host, gpu.workspace_bytes(n) + 256, host_out=out)
    np.testing.assert_array_equal(out.numpy().reshape(n, 100), oracle.sort(rec))
    np.testing.assert_array_equal(host.numpy().reshape(n, 100), rec)  # the input is left as it was


def test_keys_only_tiny(gpu):
    import torch
    for n in (1, 2, 3, 12, 13, 101, 2049):
        rec = datagen.skewed(n, 85, nvals=4, dup_frac=0.5) if n > 3 else datagen.uniform(n, 85)
        out = gpu.sort_external_keys(pinned(rec), 64 << 20)
        np.testing.assert_array_equal(out.numpy().reshape(n, 100), oracle.sort(rec))
        pout = torch.empty(n * 100, dtype=torch.uint8, pin_memory=True)
        gpu.sort_external_keys(pinned(rec), 64 << 20, host_out=pout)
        np.testing.assert_array_equal(pout.numpy().reshape(n, 100), oracle.sort(rec))


def test_keys_only_pageable_many_pieces(gpu):
    """A pageable output: the gather writes pieces of 1,342,177 records into
    the four pinned bounce buffers, which the host empties oldest first; six
    million records fill five pieces (every buffer used, the first reused)
    and end in a ragged one."""
    n = 6_000_001
    rec = datagen.skewed(n, 95, nvals=200, dup_frac=0.2)
    out = gpu.sort_external_keys(pinned(rec), gpu.workspace_bytes(n) + 256)
    np.testing.assert_array_equal(out.numpy().reshape(n, 100), oracle.sort(rec))


def test_keys_only_pinned_output_repeats(gpu):
    """A pinned output takes the scatter: the places table and the staging
    areas are sort buffers reused from call to call, a larger call after a
    smaller one and back; every byte of the output is written (it starts
    filled with 0xEE)."""
    import torch
    for n, seed in ((300_001, 87), (40_000, 88), (300_001, 89)):
        rec = datagen.skewed(n, seed, nvals=60, dup_frac=0.2)
        out = torch.full((n * 100,), 0xEE, dtype=torch.uint8).pin_memory()
        gpu.sort_external_keys(pinned(rec), gpu.workspace_bytes(n) + 256, host_out=out)
        np.testing.assert_array_equal(out.numpy().reshape(n, 100), oracle.sort(rec))


def test_keys_only_budget_and_errors(gpu):
    import torch
    n = 5_000
    rec = datagen.uniform(n, 86)
    need = gpu.workspace_bytes(n) + 256
    with pytest.raises(gpu.LeyendaError) as ei:
        gpu.sort_external_keys(pinned(rec), need - 1)
    assert ei.value.status == -3
    out = gpu.sort_external_keys(pinned(rec), need)
    np.testing.assert_array_equal(out.numpy().reshape(n, 100), oracle.sort(rec))
    with pytest.raises(gpu.LeyendaError) as ei:  # pageable input: the gather reads it from the device
        gpu.sort_external_keys(torch.from_numpy(rec.reshape(-1).copy()), need)
    assert ei.value.status == -1


# ---- runs + merge in one call, the last two runs kept on the device ----

@pytest.mark.parametrize("runs,kind,in_place,pinned_out", [
    (1, "uniform", True, False), (2, "ties", True, True), (3, "uniform", False, False),
    (7, "ties", True, False), (10, "uniform", True, True), (23, "few", False, True)])
def test_sort_external_matches_oracle(gpu, runs, kind, in_place, pinned_out):
    """The last two runs' slices reach the merge by device copies and their
    keys are read from device memory by the co-rank; ties straddle every run
    (the resident runs included), and with many runs the merge has many
    chunks."""
    import torch
    n = 150_001
    if kind == "uniform":
        rec = datagen.uniform(n, 90 + runs)
    elif kind == "ties":
        rec = datagen.skewed(n, 91 + runs, nvals=40, dup_frac=0.3)
    else:
        rec = datagen.uniform(n, 92)
        rec[:, :10] = datagen.uniform(8, 93)[np.arange(n) % 8, :10]
    host = pinned(rec)
    budget = budget_for_runs(gpu, n, runs)
    _, k = gpu.plan_runs(n, budget)
    assert k <= runs
    host_runs = None if in_place else torch.empty(n * 100, dtype=torch.uint8, pin_memory=True)
    out = torch.empty(n * 100, dtype=torch.uint8, pin_memory=pinned_out)
    gpu.sort_external(host, budget, host_runs=host_runs, host_out=out)
    np.testing.assert_array_equal(out.numpy().reshape(n, 100), oracle.sort(rec))
    if not in_place:
        np.testing.assert_array_equal(host.numpy().reshape(n, 100), rec)  # the input is left as it was


@pytest.mark.parametrize("n,runs,budget,kept", [
    (120_007, 2, None, 2), (120_007, 3, None, 2), (120_007, 6, None, 2),
    (7111, 19, 200_000, 1), (7111, 21, 186_000, 0)])
def test_sort_external_keeps_the_last_runs(gpu, n, runs, budget, kept):
    """The runs the plan keeps on the device (two when the merge fits beside
    them; one, or none, for many tiny runs under a budget near one run's
    footprint) never reach host_runs: their ranges keep the bytes the buffer
    held, and every other run is written there."""
    import torch
    rec = datagen.skewed(n, 150 + runs, nvals=40, dup_frac=0.3)
    if budget is None:
        budget = budget_for_runs(gpu, n, runs)
    r, k, kk = gpu.plan_external(n, budget)
    assert (k, kk) == (runs, kept)
    host_runs = torch.full((n * 100,), 0xEE, dtype=torch.uint8).pin_memory()
    out = gpu.sort_external(pinned(rec), budget, host_runs=host_runs)
    np.testing.assert_array_equal(out.numpy().reshape(n, 100), oracle.sort(rec))
    hr = host_runs.numpy().reshape(n, 100)
    for i in range(k):
        untouched = bool((hr[i * r:min(n, (i + 1) * r)] == 0xEE).all())
        assert untouched == (i >= k - kept), f"run {i} of {k}, {kept} kept"


def test_sort_external_tiny_and_errors(gpu):
    import torch
    for n in (1, 2, 5, 2049):
        rec = datagen.skewed(n, 95, nvals=4, dup_frac=0.5) if n > 2 else datagen.uniform(n, 95)
        out = gpu.sort_external(pinned(rec), 64 << 20)
        np.testing.assert_array_equal(out.numpy().reshape(n, 100), oracle.sort(rec))
    rec = datagen.uniform(1000, 96)
    with pytest.raises(gpu.LeyendaError) as ei:  # pageable input
        gpu.sort_external(torch.from_numpy(rec.reshape(-1).copy()), 64 << 20)
    assert ei.value.status == -1
    with pytest.raises(gpu.LeyendaError) as ei:
        gpu.sort_external(pinned(rec), 1000)  # below one run's footprint
    assert ei.value.status == -3
    h = pinned(rec)
    with pytest.raises(gpu.LeyendaError) as ei:  # the output over the runs
        gpu.sort_external(h, 64 << 20, host_runs=h, host_out=h)
    assert ei.value.status == -1


def test_sort_external_many_tiny_runs(gpu):
    """21 runs of about 340 records under a budget near one run's footprint:
    the budget less one or two kept runs is too small for the merge's tables,
    so the call downloads every run and merges within the whole budget (found
    by a random case)."""
    import torch
    n = 7111
    rec = oracle.sort(datagen.uniform(n, 97))  # sorted input
    host = pinned(rec)
    budget = budget_for_runs(gpu, n, 21)
    _, k = gpu.plan_runs(n, budget)
    assert k == 21
    runs = torch.empty(n * 100, dtype=torch.uint8, pin_memory=True)
    out = gpu.sort_external(host, budget, host_runs=runs)
    np.testing.assert_array_equal(out.numpy().reshape(n, 100), rec)


def test_external_calls_reuse_and_share_their_memory(gpu):
    """The external calls keep a device arena and bounce buffers between calls:
    calls with growing and shrinking budgets reuse or replace them, and two
    calls at once on different threads (one takes the kept set, the other
    makes its own) both sort correctly."""
    import threading
    import torch
    recs = [datagen.skewed(60_000 + 7_000 * i, 130 + i, nvals=50, dup_frac=0.2) for i in range(4)]
    for i, rec in enumerate(recs):  # budgets up and down: the kept arena is reused or replaced
        n = rec.shape[0]
        budget = budget_for_runs(gpu, n, [3, 9, 2, 5][i])
        out = gpu.sort_external(pinned(rec), budget)
        np.testing.assert_array_equal(out.numpy().reshape(n, 100), oracle.sort(rec))
        runs, bounds = gpu.sort_runs(pinned(rec), budget)
        merged = gpu.merge(runs, bounds, budget)
        np.testing.assert_array_equal(merged.numpy().reshape(n, 100), oracle.sort(rec))
    results, errors = {}, []

    def work(k):
        try:
            rec = recs[k]
            n = rec.shape[0]
            budget = budget_for_runs(gpu, n, 4)
            for _ in range(3):
                out = gpu.sort_external(pinned(rec), budget, stream=torch.cuda.Stream())
                results[k] = out.numpy().reshape(n, 100).copy()
                if not np.array_equal(results[k], oracle.sort(rec)):
                    errors.append(f"thread {k}: output differs")
        except Exception as exc:  # reported below
            errors.append(f"thread {k}: {exc!r}")

    threads = [threading.Thread(target=work, args=(k,)) for k in (0, 1)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=240)
    assert not errors, errors
    assert set(results) == {0, 1}
    gpu.release_workspaces()


def test_keys_only_calls_at_once(gpu):
    """Three calls on three threads at once: keys-only into a pageable output
    (the gather fills bounce buffers: one thread takes the kept set, another
    makes its own), keys-only into a pinned output (the scatter), and runs +
    merge into a pageable output; each twice."""
    import threading
    import torch
    n = 1_500_001  # two bounce pieces
    recs = [datagen.skewed(n, 140 + i, nvals=80, dup_frac=0.2) for i in range(3)]
    wants = [oracle.sort(r) for r in recs]
    errors = []

    def work(k):
        try:
            rec = recs[k]
            for _ in range(2):
                s = torch.cuda.Stream()
                if k == 0:
                    out = gpu.sort_external_keys(pinned(rec), gpu.workspace_bytes(n) + 256, stream=s)
                elif k == 1:
                    out = torch.empty(n * 100, dtype=torch.uint8, pin_memory=True)
                    gpu.sort_external_keys(pinned(rec), gpu.workspace_bytes(n) + 256, host_out=out, stream=s)
                else:
                    out = gpu.sort_external(pinned(rec), budget_for_runs(gpu, n, 3), stream=s)
                if not np.array_equal(out.numpy().reshape(n, 100), wants[k]):
                    errors.append(f"thread {k}: output differs")
        except Exception as exc:  # reported below
            errors.append(f"thread {k}: {exc!r}")

    threads = [threading.Thread(target=work, args=(k,)) for k in (0, 1, 2)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=240)
    assert not any(th.is_alive() for th in threads)
    assert not errors, errors
    gpu.release_workspaces()
