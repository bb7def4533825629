"""Seeded random cases against the CPU oracle: random sizes, key structures,
tuning parameters and key lengths, random batches, and random cases of the
limited-memory path, of the sort that allocates nothing and of the serving
engine.

Each case draws its size log-uniformly (1 to 2.5 M records, plus two cases
above the 8 Mi threshold of the fused first pass), a key structure (uniform,
Zipf prefixes of random width and duplicate share, a few distinct keys, a
constant prefix of random length, small per-byte alphabets, printable keys,
sorted or reversed input), a parameter set from the whole accepted space and,
for a third of the cases, a key length K from 1 to 100 with ties planted past
byte 10.  The output must equal the oracle's stable sort byte for byte; every
case prints what it is before it runs.
"""
import numpy as np
import pytest

import datagen
import oracle
from tests.test_gpu_sort import assert_same

pytestmark = pytest.mark.gpu

SEED = 20261203
N_CASES = 200


def _records(rng, n: int) -> tuple[np.ndarray, str]:
    kind = rng.choice(["uniform", "zipf", "few", "prefix", "alphabet", "ascii", "sorted", "reverse"])
    seed = int(rng.integers(1, 1 << 30))
    if kind == "zipf":
        nvals = int(np.exp(rng.uniform(np.log(2), np.log(65536))))
        dup = float(rng.uniform(0.0, 0.5))
        return datagen.skewed(n, seed, nvals=nvals, dup_frac=dup), f"zipf(nvals={nvals},dup={dup:.2f})"
    if kind == "ascii":
        return datagen.ascii(n, seed), "ascii"
    rec = datagen.uniform(n, seed)
    if kind == "few":
        k = int(rng.integers(1, 40))
        vals = datagen.uniform(k, seed + 1)[:, :10]
        rec[:, :10] = vals[rng.integers(0, k, n)]
        return rec, f"few({k})"
    if kind == "prefix":
        p = int(rng.integers(1, 10))
        rec[:, :p] = rng.integers(0, 256, p, dtype=np.uint8)
        return rec, f"prefix({p})"
    if kind == "alphabet":
        sizes = rng.integers(1, 5, 10)
        for b in range(10):
            alpha = rng.integers(0, 256, int(sizes[b]), dtype=np.uint8)
            rec[:, b] = alpha[rng.integers(0, int(sizes[b]), n)]
        return rec, f"alphabet({''.join(map(str, sizes))})"
    if kind in ("sorted", "reverse"):
        rec = oracle.sort(rec)
        return (rec if kind == "sorted" else rec[::-1].copy()), kind
    return rec, "uniform"


def _params(rng) -> dict:
    return dict(digit_bits=int(rng.integers(4, 9)), tile_items=int(rng.choice([8, 16, 32])),
                big_threshold=int(np.exp(rng.uniform(0, np.log(2048)))),
                tiny_threshold=int(rng.integers(1, 257)), scatter_threads=int(rng.choice([256, 512, 1024])),
                local_threads=int(rng.choice([256, 512])), first_pass=int(rng.integers(0, 3)))


def _cases():
    rng = np.random.default_rng(SEED)
    cases = []
    for i in range(N_CASES):
        n = max(1, int(np.exp(rng.uniform(0, np.log(2_500_000)))))
        if i in (7, 23):
            n = int(rng.integers(8_388_608, 9_000_000))
        keyed = rng.uniform() < 1 / 3 and i != 7
        k = int(rng.integers(1, 101)) if keyed else None
        cases.append((i, n, int(rng.integers(1 << 30)), k))
    return cases


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"case{c[0]}")
def test_fuzz_sort(gpu, case):
    import torch
    i, n, seed, key_bytes = case
    rng = np.random.default_rng(seed)
    rec, what = _records(rng, n)
    params = _params(rng)
    if i == 7:  # the large cases take the fused first passes (records copied / tuples only)
        params.update(first_pass=2)
    elif i == 23:
        params.update(first_pass=1, tile_items=32)
    if key_bytes is not None and key_bytes > 10 and n > 1:
        # ties past byte 10: a share of the records copy bytes 10..10+L of a few templates
        L = int(rng.integers(1, 91))
        share = rng.uniform(0.1, 0.9)
        sel = rng.uniform(size=n) < share
        tmpl = rec[rng.integers(0, n, 3), 10:10 + L]
        rec[sel, 10:10 + L] = tmpl[rng.integers(0, 3, int(sel.sum()))]
        rec[sel, :10] = rec[0, :10]
    print(f"fuzz case {i}: n={n} keys={what} key_bytes={key_bytes} params={params}", flush=True)
    want = oracle.sort(rec, threads=0) if key_bytes is None else oracle.sort(rec, key_bytes=key_bytes)
    old = gpu.get_params()
    try:
        gpu.set_params(**params)
        if i in (7, 23):
            assert gpu.first_pass(n) == params["first_pass"]
        d = _dev(rec)
        out = gpu.sort(d) if key_bytes is None else gpu.sort_keyed(d, key_bytes)
        torch.cuda.synchronize()
        st = gpu.stats(torch.cuda.current_stream())
    finally:
        gpu.set_params(**old)
    assert_same(out.cpu().numpy().reshape(-1, 100), want, f"case {i}")
    if key_bytes is None:
        assert st["guard"] == 0


@pytest.mark.parametrize("seed", range(11, 19))
def test_fuzz_batch(gpu, seed):
    """Random batches: 1 to 40 requests of 0 to 300,000 records, mixed key
    structures, one launch sequence; each request must equal its oracle sort."""
    import torch
    rng = np.random.default_rng(SEED + seed)
    count = int(rng.integers(1, 41))
    recs, whats = [], []
    for _ in range(count):
        n = int(np.exp(rng.uniform(0, np.log(300_001)))) - 1
        if n == 0:
            recs.append(np.zeros((0, 100), np.uint8))
            whats.append("empty")
            continue
        r, w = _records(rng, n)
        recs.append(r)
        whats.append(f"{n}:{w}")
    print(f"fuzz batch {seed}: {count} requests {whats}", flush=True)
    ins = [_dev(r) for r in recs]
    outs = [torch.empty_like(t) for t in ins]
    gpu.sort_batch(zip(ins, outs))
    torch.cuda.synchronize()
    for k, (r, o) in enumerate(zip(recs, outs)):
        assert_same(o.cpu().numpy().reshape(-1, 100), oracle.sort(r), f"batch {seed} request {k}")


@pytest.mark.parametrize("seed", range(24))
def test_fuzz_external(gpu, seed):
    """The limited-memory path with random sizes (1,000 to 600,000 records),
    run counts (1 to 24), merge budgets (1.5 to 48 MB, so 1 to hundreds of
    chunks), runs in place or apart, pinned or pageable output, through the
    two calls, the one call and the keys-only call."""
    import torch
    from tests.test_gpu_external import budget_for_runs, pinned
    rng = np.random.default_rng(SEED + 100 + seed)
    n = int(np.exp(rng.uniform(np.log(1000), np.log(600_000))))
    rec, what = _records(rng, n)
    runs = int(rng.integers(1, 25))
    path = ["two_calls", "one_call", "keys_only"][seed % 3]
    in_place = bool(rng.integers(0, 2))
    pinned_out = bool(rng.integers(0, 2))
    merge_budget = int(np.exp(rng.uniform(np.log(1.5e6), np.log(48e6))))
    params = _params(rng)
    print(f"fuzz external {seed}: n={n} keys={what} runs<={runs} path={path} in_place={in_place} "
          f"pinned_out={pinned_out} merge_budget={merge_budget} params={params}", flush=True)
    want = oracle.sort(rec)
    host = pinned(rec)
    out = torch.empty(n * 100, dtype=torch.uint8, pin_memory=pinned_out)
    old = gpu.get_params()
    try:
        gpu.set_params(**params)
        if path == "keys_only":
            gpu.sort_external_keys(host, gpu.workspace_bytes(n) + 256 + (1 << 20), host_out=out)
        else:
            budget = budget_for_runs(gpu, n, runs)
            host_runs = host if in_place else torch.empty(n * 100, dtype=torch.uint8, pin_memory=True)
            if path == "one_call":
                gpu.sort_external(host, budget, host_runs=host_runs, host_out=out)
            else:
                got_runs, bounds = gpu.sort_runs(host, budget, host_runs=host_runs)
                assert bounds[0] == 0 and bounds[-1] == n and len(bounds) - 1 <= runs
                gpu.merge(got_runs, bounds, merge_budget, host_out=out)
    finally:
        gpu.set_params(**old)
    assert_same(out.numpy().reshape(n, 100), want, f"external {seed}")


@pytest.mark.parametrize("seed", range(12))
def test_fuzz_noalloc(gpu, seed):
    """leyenda_sort_noalloc through the C ABI with random parameters and sizes
    up to what its fixed array holds under them; calls follow each other on
    the same array."""
    import torch
    rng = np.random.default_rng(SEED + 200 + seed)
    params = _params(rng)
    lib = gpu.load()
    old = gpu.get_params()
    try:
        gpu.set_params(**params)
        cap = int(lib.leyenda_noalloc_max_records())
        n = int(np.exp(rng.uniform(0, np.log(cap))))
        rec, what = _records(rng, n)
        print(f"fuzz noalloc {seed}: n={n} (cap {cap}) keys={what} params={params}", flush=True)
        d = _dev(rec)
        out = torch.empty_like(d)
        rc = lib.leyenda_sort_noalloc(d.data_ptr(), n, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        assert rc == 0, lib.leyenda_last_error()
        torch.cuda.synchronize()
    finally:
        gpu.set_params(**old)
    assert_same(out.cpu().numpy().reshape(-1, 100), oracle.sort(rec), f"noalloc {seed}")


@pytest.mark.parametrize("seed", range(12))
def test_fuzz_server(gpu, seed):
    """The serving engine with random slots, batch limits, budgets and
    parameters, batched or not; requests of random sizes and key structures
    arrive in waves while earlier ones run, and completed outputs are held a
    while before release (so admission waits on the output arena).  Every
    output must equal its oracle sort."""
    import time
    import torch
    rng = np.random.default_rng(SEED + 300 + seed)
    params = _params(rng)
    batched = bool(rng.integers(0, 2))
    slots = int(rng.integers(1, 5))
    max_batch = int(rng.integers(1, 49))
    mbr = int(rng.integers(50_000, 400_001))
    count = int(rng.integers(60, 151))
    sizes = [int(np.exp(rng.uniform(0, np.log(mbr)))) for _ in range(count)]
    recs, whats = [], []
    for n in sizes:
        r, w = _records(rng, n)
        recs.append(r)
        whats.append(w)
    print(f"fuzz server {seed}: batched={batched} slots={slots} max_batch={max_batch} max_batch_records={mbr} "
          f"requests={count} records={sum(sizes)} params={params}", flush=True)
    ins = [_dev(r).view(-1) for r in recs]
    old = gpu.get_params()
    outs = {}
    try:
        gpu.set_params(**params)
        ws = gpu.workspace_bytes(mbr)
        budget = slots * (2 * ws + (64 << 20)) + mbr * 100 * int(rng.integers(1, 5))
        srv = gpu.Server(budget_bytes=budget, slots=slots, max_batch=max_batch, max_batch_records=mbr,
                         batched=batched)
        try:
            nxt, held, idle_since = 0, [], time.monotonic()
            while len(outs) < count:
                # a wave of submissions
                wave = int(rng.integers(0, 25))
                for _ in range(wave):
                    if nxt < count:
                        srv.submit(ins[nxt], nxt)
                        nxt += 1
                got = srv.poll(timeout_s=0.2)
                for dn in got:
                    assert dn["status"] == 0, dn
                    assert dn["n"] == sizes[dn["tag"]]
                    outs[dn["tag"]] = srv.output(dn).cpu().numpy()
                    held.append(dn["tag"])
                hold = int(rng.integers(0, 9))
                if not got or len(held) > hold:
                    for t in held[: len(held) - (hold if got else 0)]:
                        srv.release(t)
                    held = held[len(held) - (hold if got else 0):]
                if got:
                    idle_since = time.monotonic()
                elif nxt >= count and time.monotonic() - idle_since > 60:
                    raise AssertionError(f"no completion for 60 s with {count - len(outs)} requests left")
            for t in held:
                srv.release(t)
            torch.cuda.synchronize()
        finally:
            srv.close()
    finally:
        gpu.set_params(**old)
    for i, r in enumerate(recs):
        assert_same(outs[i], oracle.sort(r), f"server {seed} request {i} ({whats[i]}, n={sizes[i]})")
