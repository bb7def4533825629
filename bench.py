#!/usr/bin/env python3
"""Throughput of the in-HBM record sort on one MI355X.

Workload: 100,000,000 records x 100 bytes (10 GB), 10-byte keys of i.i.d.
uniform bytes and 90-byte uniform payloads from seed 2 (synthetic stand-in for
the paper's 10 GB internal-sort dataset, Section 4.1).  Input and output are
resident in HBM before the timed region; one step = one full leyenda_sort
(extraction, partition levels, local sorts, record gather).

Prints one JSON line: GB/s of records sorted, the roofline of the dominant
kernel (from HIP events recorded around each phase on the sort's stream),
and the CPU oracle timed on a bounded sample of the same workload.  Further
objects on the same line (each can be skipped by a flag): `serving` (batched
vs per-request serving of 2,000 requests), `copy_ceiling`, `flexible_keys`
(leyenda_sort_keyed with 4- and 20-byte keys), `ascii_keys` (the 20 GB
printable-key workload) and `external` (60 GB through a 30 GB device budget).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GB/s of 100-byte records sorted (10 GB, in-HBM); p50/p99 latency batched"
HBM_PEAK_GBS = 8000.0
PMC_FILE = os.path.join(ROOT, "profiles", "sort_internal_1e8_pmc.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1909_08006_amd", "csrc", "sort_kernels.hip")

# Algorithmic bytes per record of each phase (element granularity, no line overfetch):
#   extract   reads the 10 key bytes, writes a 16-byte (key, index) tuple (with the
#             fused first pass the tuple goes straight into its level-0 bucket, so
#             level 0 moves no tuple a second time)
#   partition per device-wide partition pass: reads + writes 16-byte tuples (32 B)
#             for every moved key, and levels >= 1 first read 8 key bytes per key
#             for their histograms
#   local     reads 16-byte tuples, writes a 4-byte index
#   gather    reads the 4-byte index and the 100-byte record, writes 100 bytes
ALG_BYTES = {"extract": 26, "local": 20, "gather": 204}
KERNEL_OF = {"extract": "k_extract", "partition": "k_hist+k_plan+k_scatter", "local": "k_local",
             "gather": "k_gather_plain"}
FIRST_PASS_KERNEL = {0: "k_extract", 1: "k_fuse0", 2: "k_fuse0"}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pmc_fields(n: int):
    """Fields of the committed rocprofv3 counter summary, or None if it is
    absent, for another size or taken on a different kernel source."""
    if not os.path.exists(PMC_FILE):
        return None
    fields = {}
    for line in open(PMC_FILE):
        if "=" in line and not line.startswith("#"):
            k, _, v = line.strip().partition("=")
            fields[k.strip()] = v.strip()
    src_hash = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]
    if fields.get("kernel_source_sha256_16") != src_hash or int(fields.get("n_records", -1)) != n:
        return None
    return fields


def pmc_traffic(n: int, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None if absent, for another kernel, or taken on a different
    kernel source."""
    if not os.path.exists(PMC_FILE):
        return None
    fields = {}
    for line in open(PMC_FILE):
        if "=" in line and not line.startswith("#"):
            k, _, v = line.strip().partition("=")
            fields[k.strip()] = v.strip()
    src_hash = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]
    if (fields.get("kernel_source_sha256_16") != src_hash or int(fields.get("n_records", -1)) != n
            or fields.get("kernel") != kernel):
        return None
    return int(float(fields["hbm_bytes_per_launch"]))


def host_cpu() -> dict:
    """Host CPU facts for the baseline: logical CPUs visible, the CPUs this
    process may run on, and the model name."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


# The paper's CPU sort-phase times for 10 GB of uniform 100-byte records
# (Table 1, Section 2.2): its first radix sort and GNU's parallel sorts.  The
# paper does not name the machine for this table; its contest testbed (Table 2,
# Section 4.1) is two Xeon E5-2640 v4 (20 cores, 40 hardware threads), 30 GB.
PAPER_TABLE1_S = {"leyenda_radix_sort": 2.238, "gnu_parallel_sort": 7.443, "gnu_parallel_stable_sort": 17.917,
                  "hardware": "not stated for Table 1; the paper's testbed (Table 2) is 2x Xeon E5-2640 v4 "
                              "(20 cores, 40 threads), 30 GB"}


def cpu_baseline(host_u8, n: int, n_one: int):
    """The oracle on the host: the whole workload on every host thread
    (``oracle_sort_par``: per-thread qsort slices, merged), plus one thread on
    the first ``n_one`` records.  Returns (cpu_baseline object, oracle output)."""
    import oracle
    rec = host_u8[: n * 100].numpy().reshape(n, 100)
    threads = oracle.host_threads()
    log(f"cpu baseline: oracle sort of {n:,} records on {threads} threads ...")
    t0 = time.perf_counter()
    want = oracle.sort(rec, threads=0)
    dt = time.perf_counter() - t0
    log(f"cpu baseline: oracle sort of {n_one:,} records on one thread ...")
    t0 = time.perf_counter()
    oracle.sort(rec[:n_one])
    dt1 = time.perf_counter() - t0
    res = {"value": round(n * 100 / dt / 1e9, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
           "sample": f"the whole workload ({n:,} records, {n * 100 / 1e9:.1f} GB): (key, index) pairs sorted by "
                     f"memcmp then index in {threads} qsort slices merged on {threads} threads, then the record "
                     f"gather; {dt:.2f} s",
           "seconds": round(dt, 3), "host": host_cpu(),
           "one_thread": {"records": n_one, "seconds": round(dt1, 3), "gbs": round(n_one * 100 / dt1 / 1e9, 4)},
           "paper_table1_sort_s_10gb": PAPER_TABLE1_S}
    return res, want


def first_pass_ab(ley, torch, dev, ref, n: int, steps: int) -> dict:
    """The sort timed with each first pass (parameter first_pass 0, 1, 2) on
    the same input: HIP events around `steps` back-to-back sorts after one
    warm-up, the output compared with `ref` byte for byte."""
    old = ley.get_params()
    res = {}
    try:
        for fp in (0, 1, 2):
            ley.set_params(first_pass=fp)
            out = torch.empty_like(dev)
            ley.sort(dev, out)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                ley.sort(dev, out)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            res[str(fp)] = {"ms_per_sort": round(ms, 4), "gbs": round(n * 100 / (ms / 1e3) / 1e9, 2),
                            "taken": ley.first_pass(n), "same_output": bool(torch.equal(out, ref)),
                            "guard": ley.stats()["guard"]}
            del out
            torch.cuda.empty_cache()
    finally:
        ley.set_params(**old)
    return res


def serving(ley, count: int, warm: int, budget: int) -> dict:
    """Serving workload: Poisson arrivals of sort requests, sizes log-uniform in
    [1e3, 1e7] records, device admission budget 32 GB.  The same request stream
    is replayed natively against the continuous-batching engine and against one
    plain leyenda_sort per request (one stream, arrival order); latency =
    completion - arrival, including queueing; the first `warm` requests are
    excluded from the statistics."""
    import numpy as np
    import torch
    import datagen

    pool_n = 10_000_000
    host = torch.empty(pool_n * 100, dtype=torch.uint8, pin_memory=True)
    datagen.fill_uniform(host.data_ptr(), pool_n, datagen.SEED_REQUEST_BASE)
    d = host.to("cuda:0")
    torch.cuda.synchronize()
    sizes = datagen.request_sizes(count)
    offs = (datagen.words(datagen.SEED_REQUEST_BASE + 1, count) % np.uint64(pool_n)).astype(np.int64)
    offs = np.minimum(offs, pool_n - sizes)
    inputs = [(d.data_ptr() + int(o) * 100, int(n)) for o, n in zip(offs, sizes)]
    total_bytes = float(sizes[warm:].sum()) * 100
    cfg = dict(budget_bytes=budget, slots=3, max_batch=256, max_batch_records=10_000_000)

    def stats(lat, mk):
        L = np.asarray(lat[warm:]) * 1e3
        return {"p50_ms": round(float(np.percentile(L, 50)), 3), "p99_ms": round(float(np.percentile(L, 99)), 3),
                "mean_ms": round(float(L.mean()), 3), "gbs": round(total_bytes / mk / 1e9, 2)}

    log(f"serving: {count} requests, closed-loop capacity of both engines ...")
    zero = [0.0] * count
    lat, mk_plain = ley.serve_replay(inputs, zero, batched=False, **cfg)
    lat_b, mk_b = ley.serve_replay(inputs, zero, batched=True, **cfg)
    mu = count / mk_plain
    res = {"requests": count, "warmup_requests": warm, "size_records": "log-uniform [1e3, 1e7]",
           "budget_bytes": budget, "slots": cfg["slots"], "max_batch": cfg["max_batch"],
           "capacity_rps": {"per_request": round(mu, 1), "batched": round(count / mk_b, 1)},
           "closed_loop": {"per_request": stats(lat, mk_plain), "batched": stats(lat_b, mk_b)}, "loads": []}
    for rho in (0.5, 0.8, 0.95):
        arr = datagen.arrival_times(count, rho * mu, seed=datagen.SEED_ARRIVALS)
        row = {"rho": rho, "rate_rps": round(rho * mu, 1)}
        for name, batched in (("batched", True), ("per_request", False)):
            log(f"serving: rho={rho} {name} ...")
            lat, mk = ley.serve_replay(inputs, arr, batched=batched, **cfg)
            row[name] = stats(lat, mk)
        res["loads"].append(row)
    del d, host
    torch.cuda.empty_cache()
    return res


def copy_ceiling(torch) -> dict:
    """Device-to-device copy of 2,000,000,000 bytes (HIP events, best of 5): the
    practical HBM ceiling beside the 8 TB/s peak."""
    src = torch.empty(2_000_000_000, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    best = None
    for _ in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes": 2_000_000_000, "ms": round(best, 4), "gbs_read_plus_write": round(4e9 / best / 1e6, 1)}


def keys_ordered(torch, out, n: int) -> bool:
    """Output sanity: keys non-decreasing (device-side check of big-endian key words)."""
    keys = out.view(n, 100)[:, :10].to(torch.int64)
    hi = torch.zeros(n, dtype=torch.int64, device=out.device)
    for b in range(7):
        hi = hi * 256 + keys[:, b]
    lo = (keys[:, 7] * 256 + keys[:, 8]) * 256 + keys[:, 9]
    ok = bool(((hi[1:] > hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] >= lo[:-1]))).all().item())
    del keys, hi, lo
    return ok


def prefix_ordered(torch, out, n: int, kb: int) -> bool:
    """Adjacent records in memcmp order on their first kb bytes (device-side)."""
    o = out.view(n, 100)
    ok = True
    for a in range(0, n - 1, 25_000_000):
        b = min(n - 1, a + 25_000_000)
        x, y = o[a:b, :kb], o[a + 1:b + 1, :kb]
        ne = x != y
        col = ne.to(torch.uint8).argmax(dim=1, keepdim=True)
        xd, yd = x.gather(1, col).squeeze(1), y.gather(1, col).squeeze(1)
        ok = ok and bool((~ne.any(dim=1) | (xd < yd)).all().item())
    return ok


def flexible_keys(ley, torch, datagen, dev, steps: int) -> dict:
    """Keys of the first K bytes (leyenda_sort_keyed) on the 10 GB uniform
    records already in HBM (K = 4: a masked prefix; K = 20: one tie round,
    which finds no tie) and on 200,000,000 skewed records (Zipf prefixes and 5%
    duplicate 10-byte keys: K = 20 resolves the duplicates' runs by bytes
    10..15, then 16..19)."""
    res = {}
    n = dev.numel() // 100
    out = torch.empty_like(dev)

    def timed(src, dst, kb):
        ley.sort_keyed(src, kb, dst)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ley.sort_keyed(src, kb, dst)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    def guard():  # key sizes above 10 report a fired guard as an error; these read the prefix sort's
        return ley.stats(torch.cuda.current_stream())["guard"]

    for kb in (4, 20):
        ms = timed(dev, out, kb)
        res[f"uniform_1e8_k{kb}"] = {"ms_per_sort": round(ms, 3), "gbs": round(n * 100 / (ms / 1e3) / 1e9, 2),
                                      "ordered": prefix_ordered(torch, out, n, kb), "guard": guard()}
    del out
    torch.cuda.empty_cache()
    m = 200_000_000
    log(f"keys: generating {m:,} skewed records (20 GB, seed {datagen.SEED_SKEWED}) ...")
    host = ley.pinned_empty(m * 100)
    datagen.fill_skewed(host.data_ptr(), m, datagen.SEED_SKEWED)
    sk = host.to("cuda:0", non_blocking=True)
    torch.cuda.synchronize()
    ley.pinned_free(host)
    out = torch.empty_like(sk)
    ms10 = timed(sk, out, 10)
    ms = timed(sk, out, 20)
    res["skewed_2e8_k20"] = {"ms_per_sort": round(ms, 3), "gbs": round(m * 100 / (ms / 1e3) / 1e9, 2),
                             "ms_per_sort_k10": round(ms10, 3), "ordered": prefix_ordered(torch, out, m, 20),
                             "guard": guard()}
    del sk, out
    torch.cuda.empty_cache()
    res["steps"] = steps
    return res


def ascii_keys(ley, torch, datagen, steps: int) -> dict:
    """The paper's 20 GB dataset format: 200,000,000 records whose keys are ten
    printable ASCII bytes (95 values each), in HBM, sorted like the 10 GB
    workload (same parameters, same timing)."""
    n = 200_000_000
    log(f"ascii: generating {n:,} records (20 GB, seed {datagen.SEED_ASCII}) ...")
    host = ley.pinned_empty(n * 100)
    datagen.fill_ascii(host.data_ptr(), n, datagen.SEED_ASCII)
    dev = host.to("cuda:0", non_blocking=True)
    torch.cuda.synchronize()
    ley.pinned_free(host)
    out = torch.empty_like(dev)
    stream = torch.cuda.current_stream()
    ley.sort(dev, out, stream)
    torch.cuda.synchronize()
    st = ley.stats(stream)
    t0 = time.perf_counter()
    for _ in range(steps):
        ley.sort(dev, out, stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    guard = st["guard"] | ley.stats(stream)["guard"]
    ok = keys_ordered(torch, out, n)
    del dev, out
    torch.cuda.empty_cache()
    return {"workload": "200,000,000 x 100-byte records (20 GB) in HBM, keys of 10 printable ASCII bytes "
                        "uniform over 0x20..0x7E", "steps": steps, "ms_per_step": round(ms, 3),
            "gbs": round(n * 100 / (ms / 1e3) / 1e9, 2),
            "partition_passes": round(sum(st["moved"]) / n, 4), "levels": st["levels"],
            "output_keys_ordered": ok, "guard": guard}


def pcie_rates(ley, nbytes: int = 2_000_000_000, tries: int = 3) -> dict:
    """PCIe rates between pinned host memory and device memory, the way the
    external calls move data: hipMemcpyAsync on non-blocking streams of the
    HIP runtime the library uses (host clock, best of `tries`): each way alone,
    and both ways at once on two streams.  Streams share the process's few
    hardware queues and copy engines, so one pair can serialise its copies; the
    both-ways attempts go over every pair of four streams."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so.7")
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    hip.hipMalloc.argtypes = [ctypes.POINTER(vp), sz]
    hip.hipFree.argtypes = [vp]
    hip.hipStreamCreateWithFlags.argtypes = [ctypes.POINTER(vp), ctypes.c_uint]
    hip.hipStreamDestroy.argtypes = [vp]
    hip.hipStreamSynchronize.argtypes = [vp]
    hip.hipMemcpyAsync.argtypes = [vp, vp, sz, ctypes.c_int, vp]
    h2d_kind, d2h_kind = 1, 2
    host = [ley.pinned_empty(nbytes), ley.pinned_empty(nbytes)]
    dev = [vp(), vp()]
    streams = [vp() for _ in range(4)]
    try:
        for d in dev:
            if hip.hipMalloc(ctypes.byref(d), nbytes) != 0:
                raise RuntimeError("hipMalloc failed")
        for st in streams:
            if hip.hipStreamCreateWithFlags(ctypes.byref(st), 1) != 0:
                raise RuntimeError("hipStreamCreateWithFlags failed")
        h = [vp(t.data_ptr()) for t in host]

        def run(copies):
            t0 = time.perf_counter()
            for dst, src, kind, st in copies:
                if hip.hipMemcpyAsync(dst, src, nbytes, kind, st) != 0:
                    raise RuntimeError("hipMemcpyAsync failed")
            for st in streams:
                if hip.hipStreamSynchronize(st) != 0:
                    raise RuntimeError("hipStreamSynchronize failed")
            return time.perf_counter() - t0

        rates = {}
        for name, kind, dst, src in (("h2d", h2d_kind, dev[0], h[0]), ("d2h", d2h_kind, h[0], dev[0])):
            best = min(run([(dst, src, kind, streams[0])]) for _ in range(tries))
            rates[name] = round(nbytes / best / 1e9, 2)
        pairs = [(a, b) for a in range(4) for b in range(4) if a != b]
        best = min(run([(dev[0], h[0], h2d_kind, streams[a]), (h[1], dev[1], d2h_kind, streams[b])])
                   for a, b in pairs)
        rates["both_ways"] = round(2 * nbytes / best / 1e9, 2)
        return rates
    finally:
        for st in streams:
            if st.value:
                hip.hipStreamDestroy(st)
        for d in dev:
            if d.value:
                hip.hipFree(d)
        for t in host:
            ley.pinned_free(t)


def external(ley, torch, datagen, rates: dict, n: int = 600_000_000, budget: int = 30 * 10**9) -> dict:
    """The 60 GB limited-memory workload: 600,000,000 records in pinned host
    memory, 30 GB device budget, sorted runs written over the input, then the
    k-way merge into pageable host memory (and, in `pinned_output`, both paths
    again into a second pinned buffer when the host can pin it).  Bound: PCIe, 200 B/record each way, the two directions
    overlapped at their measured single-direction rates.  The merge runs twice
    into the same output: first into fresh memory (its first-touch page faults
    included), then into the now resident buffer (a reused output).  Then, each
    on the regenerated input, runs + merge in one call and the keys-only
    variant.  rates: pcie_rates() of this machine.  (n and budget: smaller
    instances of the same workload, e.g. under a profiler.)"""
    import numpy as np
    log(f"external: generating {n:,} records ({n * 100 / 1e9:.0f} GB, seed {datagen.SEED_EXTERNAL}) ...")
    a = ley.pinned_empty(n * 100)
    datagen.fill_uniform(a.data_ptr(), n, datagen.SEED_EXTERNAL)
    log("external: runs ...")
    t0 = time.perf_counter()
    runs, bounds = ley.sort_runs(a, budget, host_runs=a)
    t_runs = time.perf_counter() - t0
    out = np.empty((n, 100), dtype=np.uint8)
    t_merge = []
    for _ in range(2):
        log("external: merge ...")
        t0 = time.perf_counter()
        ley.merge(runs, bounds, budget, host_out=torch.from_numpy(out).view(-1))
        t_merge.append(time.perf_counter() - t0)
    step = 1_000_000  # sampled order check (every millionth neighbour pair)
    keys = out[::step, :10]
    ok = bool(all(bytes(keys[i]) <= bytes(keys[i + 1]) for i in range(len(keys) - 1)))
    del keys, runs
    # runs + merge in one call on the same (regenerated) input, the last two
    # runs kept on the device; runs over the input
    log("external: runs + merge in one call ...")
    datagen.fill_uniform(a.data_ptr(), n, datagen.SEED_EXTERNAL)
    t0 = time.perf_counter()
    ley.sort_external(a, budget, host_runs=a, host_out=torch.from_numpy(out).view(-1))
    t_one = time.perf_counter() - t0
    keys = out[::step, :10]
    ok_one = bool(all(bytes(keys[i]) <= bytes(keys[i + 1]) for i in range(len(keys) - 1)))
    del keys
    # keys-only variant on the same (regenerated) input, into the same output
    # buffer; after the copy-engine paths, so each of those starts from the
    # same state (a freshly written input)
    log("external: keys-only variant ...")
    datagen.fill_uniform(a.data_ptr(), n, datagen.SEED_EXTERNAL)
    keys_skip = None
    t_keys, ok_keys = float("nan"), False
    try:
        t0 = time.perf_counter()
        ley.sort_external_keys(a, budget, host_out=torch.from_numpy(out).view(-1))
        t_keys = time.perf_counter() - t0
        keys = out[::step, :10]
        ok_keys = bool(all(bytes(keys[i]) <= bytes(keys[i + 1]) for i in range(len(keys) - 1)))
        del keys
    except ley.LeyendaError as exc:  # e.g. a budget below the tuples of the whole input
        keys_skip = str(exc)
    # both paths again with a pinned output buffer (the copy engine writes the
    # host buffer directly, no bounce buffers or host copies), if the host can
    # pin a second 60 GB: keys-only on the input, then runs and merge
    pinned = {}
    try:
        pout = ley.pinned_empty(n * 100)
    except ley.LeyendaError as exc:
        pinned = {"skipped": str(exc)}
    else:
        datagen.fill_uniform(a.data_ptr(), n, datagen.SEED_EXTERNAL)  # the input again (runs were written over it)
        pview = pout.numpy().reshape(n, 100)
        t_keys_p, ok_kp = float("nan"), False
        if keys_skip is None:
            log("external: keys-only variant, pinned output ...")
            t0 = time.perf_counter()
            ley.sort_external_keys(a, budget, host_out=pout)
            t_keys_p = time.perf_counter() - t0
            ok_kp = bool(all(bytes(pview[i * step, :10]) <= bytes(pview[(i + 1) * step, :10])
                             for i in range(n // step - 1)))
        log("external: runs + merge, pinned output ...")
        t0 = time.perf_counter()
        runs, bounds = ley.sort_runs(a, budget, host_runs=a)
        t_runs_p = time.perf_counter() - t0
        t0 = time.perf_counter()
        ley.merge(runs, bounds, budget, host_out=pout)
        t_merge_p = time.perf_counter() - t0
        ok_mp = bool(all(bytes(pview[i * step, :10]) <= bytes(pview[(i + 1) * step, :10])
                         for i in range(n // step - 1)))
        del runs, pview
        ley.pinned_free(pout)
        del out
        pinned = {"t_runs_s": round(t_runs_p, 3), "t_merge_s": round(t_merge_p, 3),
                  "gbs_records_end_to_end": round(n * 100 / (t_runs_p + t_merge_p) / 1e9, 2),
                  "pcie_frac": None, "sampled_order_ok": ok_mp,
                  "keys_only": {"t_s": round(t_keys_p, 3), "gbs_records_end_to_end": round(n * 100 / t_keys_p / 1e9, 2),
                                "pcie_frac": None, "sampled_order_ok": ok_kp}}
    ley.pinned_free(a)
    # keys-only into a pinned output at half the size (30 GB in, 30 GB out),
    # when the host could not pin a second 60 GB: the pinned output takes the
    # scatter (a second in-order read of the input, every record written to
    # its place); the same input into a pageable output (the first half of the
    # resident 60 GB one) takes the gather, for comparison
    half = None
    if "skipped" in pinned and keys_skip is None:
        m = n // 2
        try:
            hin = ley.pinned_empty(m * 100)
        except ley.LeyendaError as exc:
            half = {"skipped": str(exc)}
        else:
            try:
                hout = ley.pinned_empty(m * 100)
            except ley.LeyendaError as exc:
                half = {"skipped": str(exc)}
            else:
                datagen.fill_uniform(hin.data_ptr(), m, datagen.SEED_EXTERNAL)
                hview = hout.numpy().reshape(m, 100)
                log("external: keys-only variant, 30 GB into a pinned output ...")
                t0 = time.perf_counter()
                ley.sort_external_keys(hin, budget, host_out=hout)
                t_sc = time.perf_counter() - t0
                ok_sc = bool(all(bytes(hview[i * step, :10]) <= bytes(hview[(i + 1) * step, :10])
                                 for i in range(m // step - 1)))
                del hview
                ley.pinned_free(hout)
                log("external: keys-only variant, the same 30 GB into a pageable output ...")
                t0 = time.perf_counter()
                ley.sort_external_keys(hin, budget, host_out=torch.from_numpy(out[:m]).view(-1))
                t_ga = time.perf_counter() - t0
                ok_ga = bool(all(bytes(out[i * step, :10]) <= bytes(out[(i + 1) * step, :10])
                                 for i in range(m // step - 1)))
                # 200 B/record up, 100 down for both
                hb = max(m * 200 / (rates["h2d"] * 1e9), m * 100 / (rates["d2h"] * 1e9))
                half = {"workload": "300,000,000 x 100-byte records (30 GB) in pinned host memory, 30 GB device budget, "
                                    "uniform keys",
                        "pcie_bound_s": round(hb, 3),
                        "pinned_output_scatter": {"t_s": round(t_sc, 3), "gbs_records_end_to_end": round(m * 100 / t_sc / 1e9, 2),
                                                  "pcie_frac": round(hb / t_sc, 3), "sampled_order_ok": ok_sc},
                        "pageable_output_gather": {"t_s": round(t_ga, 3), "gbs_records_end_to_end": round(m * 100 / t_ga / 1e9, 2),
                                                   "pcie_frac": round(hb / t_ga, 3), "sampled_order_ok": ok_ga}}
            ley.pinned_free(hin)
    if "skipped" in pinned:
        del out
    # 200 B/record each way (runs: up + down; merge: up + down); the two directions
    # at their own single-direction rates, fully overlapped, is a lower bound on
    # any box (two concurrent copies have reached 97 GB/s together, not the
    # 115 GB/s of the two single-direction rates)
    both_bound = max(n * 200 / (rates["h2d"] * 1e9), n * 200 / (rates["d2h"] * 1e9))
    # keys-only: 200 B/record up (the input read once in order, then every
    # record again by the gather) and 100 B/record down
    keys_bound = max(n * 200 / (rates["h2d"] * 1e9), n * 100 / (rates["d2h"] * 1e9))
    duplex = rates["both_ways"] > 1.2 * max(rates["h2d"], rates["d2h"])
    duplex_bound = n * 400 / (rates["both_ways"] * 1e9) if duplex else None
    # the one call keeps its last runs on the device (the library's plan says
    # how many): they are neither downloaded after their sorts nor uploaded
    # for the merge (r_kept = their records)
    _, k_one, kept = ley.plan_external(n, budget)
    r_kept = bounds[-1] - bounds[-1 - kept] if kept else 0
    one_each_way = (n * 200 - r_kept * 100) if k_one > 1 else n * 100
    one_bound = max(one_each_way / (rates["h2d"] * 1e9), one_each_way / (rates["d2h"] * 1e9))
    one_duplex = 2 * one_each_way / (rates["both_ways"] * 1e9) if duplex else None
    if "t_runs_s" in pinned:
        pinned["pcie_frac"] = round(both_bound / (pinned["t_runs_s"] + pinned["t_merge_s"]), 3)
        if keys_skip is None:
            pinned["keys_only"]["pcie_frac"] = round(keys_bound / pinned["keys_only"]["t_s"], 3)
        else:
            pinned["keys_only"] = {"skipped": keys_skip}
    return {"workload": "600,000,000 x 100-byte records (60 GB) in pinned host memory, 30 GB device budget, "
                        "uniform keys; runs over the input, merge into pageable host memory",
            "runs": len(bounds) - 1, "t_runs_s": round(t_runs, 3),
            "t_merge_s": round(t_merge[1], 3), "t_merge_first_touch_s": round(t_merge[0], 3),
            "gbs_records_end_to_end": round(n * 100 / (t_runs + t_merge[1]) / 1e9, 2),
            "gbs_records_end_to_end_first_touch": round(n * 100 / (t_runs + t_merge[0]) / 1e9, 2),
            "pcie_measured_gbs": rates,
            # both directions as the run stage used them (120 GB moved over its time)
            "runs_observed_gbs_both_ways": round(n * 200 / t_runs / 1e9, 1),
            "pcie_bound": {"bytes_per_record_each_way": 200, "bound_s_each_way_rates_overlapped": round(both_bound, 3),
                           "frac": round(both_bound / (t_runs + t_merge[1]), 3),
                           # the same bytes at the rate both directions reached together
                           # (only when the two copies did overlap: above 1.2x one way)
                           "bound_s_both_ways_rate": round(duplex_bound, 3) if duplex_bound else None,
                           "frac_both_ways_rate": round(duplex_bound / (t_runs + t_merge[1]), 3)
                           if duplex_bound else None},
            "sampled_order_ok": ok,
            "keys_only": {"skipped": keys_skip} if keys_skip is not None else
                         {"t_s": round(t_keys, 3), "gbs_records_end_to_end": round(n * 100 / t_keys / 1e9, 2),
                          "pcie_bound": {"bytes_per_record_up": 200, "bytes_per_record_down": 100,
                                         "bound_s": round(keys_bound, 3), "frac": round(keys_bound / t_keys, 3)},
                          "sampled_order_ok": ok_keys},
            "one_call": {"t_s": round(t_one, 3), "gbs_records_end_to_end": round(n * 100 / t_one / 1e9, 2),
                         "runs_kept_on_device": kept,
                         "bytes_per_record_each_way": round(one_each_way / n, 2),
                         "bound_s_each_way_rates_overlapped": round(one_bound, 3),
                         "pcie_frac": round(one_bound / t_one, 3),
                         "bound_s_both_ways_rate": round(one_duplex, 3) if one_duplex else None,
                         "pcie_frac_both_ways_rate": round(one_duplex / t_one, 3) if one_duplex else None,
                         "sampled_order_ok": ok_one},
            "pinned_output": pinned,
            "keys_only_half_size": half}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=100_000_000, help="records (default: the 10 GB workload)")
    ap.add_argument("--cpu-sample", type=int, default=10_000_000,
                    help="records the one-thread oracle run of cpu_baseline sorts")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving (batched vs per-request) comparison")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--no-external", action="store_true", help="skip the 60 GB runs + merge workload")
    ap.add_argument("--external-n", type=int, default=600_000_000, help="records of the external workload")
    ap.add_argument("--external-budget", type=int, default=30 * 10**9, help="device budget of the external workload")
    ap.add_argument("--workload", choices=["uniform", "skewed", "ascii"], default="uniform",
                    help="keys of the timed internal sort: uniform (the 10 GB workload), skewed (Zipf prefixes, "
                         "5%% duplicates) or printable ASCII; --n sets the size")
    ap.add_argument("--no-ascii", action="store_true", help="skip the 20 GB printable-key workload")
    ap.add_argument("--no-keys", action="store_true", help="skip the flexible key size (leyenda_sort_keyed) runs")
    ap.add_argument("--first-pass", type=int, choices=[0, 1, 2], default=None,
                    help="first pass of the sort (library parameter first_pass; default: the library's)")
    ap.add_argument("--no-first-pass-ab", action="store_true",
                    help="skip timing the sort with each of the three first passes")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 2 GB device copy (reference for HBM byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the sorter runs on one GPU; runs on several GPUs are not supported "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import datagen
    import paper_1909_08006_amd as ley

    ley.load()
    if args.first_pass is not None:
        ley.set_params(first_pass=args.first_pass)
    # PCIe rates first, while the process holds no streams of its own yet (a
    # property of the machine; the external workload's bound uses them)
    rates = pcie_rates(ley) if not args.no_external else None
    n = args.n
    fill, seed, keys = {
        "uniform": (datagen.fill_uniform, datagen.SEED_INTERNAL, "uniform 10-byte keys"),
        "skewed": (datagen.fill_skewed, datagen.SEED_SKEWED,
                   "skewed keys (Zipf(1.2) 4-byte prefixes over 65,536 values, 5% exact duplicates)"),
        "ascii": (datagen.fill_ascii, datagen.SEED_ASCII, "keys of 10 printable ASCII bytes"),
    }[args.workload]
    log(f"generating {n:,} records ({n * 100 / 1e9:.1f} GB, {args.workload}, seed {seed}) ...")
    host = torch.empty(n * 100, dtype=torch.uint8, pin_memory=True)
    fill(host.data_ptr(), n, seed)
    dev = host.to("cuda:0", non_blocking=True)
    out = torch.empty_like(dev)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    if args.calibrate_copy:
        src = torch.empty(2_000_000_000, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy: 2,000,000,000 bytes read + written")

    log(f"warmup {args.warmup} ...")
    for _ in range(args.warmup):
        ley.sort(dev, out, stream)
    torch.cuda.synchronize()
    st = ley.stats(stream)

    log(f"timing {args.steps} steps ...")
    ley.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ley.sort(dev, out, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases, calls = ley.profile_read()
    ley.profile_enable(False)
    ms = (t1 - t0) * 1e3 / args.steps
    gbs = n * 100 / (ms / 1e3) / 1e9
    avg = {k: v / max(calls, 1) for k, v in phases.items()}
    # device-side guards of the warm-up sort and of the last timed sort
    guards = {"warmup": st["guard"], "timed": ley.stats(stream)["guard"]}
    ok = guards["warmup"] == 0 and guards["timed"] == 0

    ordered = keys_ordered(torch, out, n)
    ok = ok and ordered

    first_pass = ley.first_pass(n)
    KERNEL_OF["extract"] = FIRST_PASS_KERNEL[first_pass]
    # keys moved by device-wide partition passes (a fused first pass writes each
    # tuple into its level-0 bucket once, as the extraction would: no pass)
    moved = sum(st["moved"]) - (st["moved"][0] if first_pass else 0)
    passes = moved / n
    b_alg = 250 + 32 * passes
    part_bytes = 32 * moved + 8 * sum(st["moved"][1:])
    alg = {"extract": ALG_BYTES["extract"] * n, "partition": part_bytes, "local": ALG_BYTES["local"] * n,
           "gather": ALG_BYTES["gather"] * n}
    dom = max(avg, key=lambda k: avg[k])
    # the local sorts and the gather are launched once per output part; the
    # gather phase is the sum of its launches' own durations
    launches = ley.sort_parts(n) if dom in ("local", "gather") else 1
    achieved = (alg[dom] / launches) / (avg[dom] / launches / 1e3) / 1e9
    traffic = pmc_traffic(n, KERNEL_OF[dom])

    res = {
        "metric": METRIC, "value": round(gbs, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"internal sort, {n:,} x 100-byte records ({n * 100 / 1e9:g} GB) in HBM, {keys}",
                   "n_records": n, "record_bytes": 100, "key_bytes": 10, "seed": seed,
                   "params": ley.get_params()},
        "roofline": {"bound": "hbm", "kernel": KERNEL_OF[dom],
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "launches_per_sort": launches, "records_per_launch_avg": n // launches,
                     "alg_bytes_per_launch_avg": int(alg[dom] / launches),
                     "avg_launch_ms": round(avg[dom] / launches, 4)},
        "phases_ms": {k: round(v, 4) for k, v in avg.items()},
        "phase_alg_gbs": {k: round(alg[k] / (avg[k] / 1e3) / 1e9, 1) for k in avg if avg[k] > 0},
        "first_pass": first_pass,
        "partition_passes": round(passes, 4),
        "b_alg_bytes_per_record": round(b_alg, 2),
        "sort_roofline_frac": round(b_alg * n / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        # the same time against the algorithmic bytes of the plan with a separate
        # extraction pass (250 + 32 * (passes + 1) with the fused first pass),
        # comparable across first passes
        "sort_roofline_frac_split_plan": round((b_alg + (32 if first_pass else 0)) * n / (ms / 1e3) / 1e9
                                               / HBM_PEAK_GBS, 4),
        "floor_frac_210B": round(210 * n / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "output_keys_ordered": ordered,
        "device_guards": guards,
    }
    pf = pmc_fields(n)
    if pf and "sort_hbm_bytes_per_record" in pf:
        # every kernel's counted HBM bytes of one sort, over the measured wall time
        bpr = float(pf["sort_hbm_bytes_per_record"])
        res["sort_hbm_traffic"] = {"bytes_per_record": bpr, "gbs": round(bpr * n / (ms / 1e3) / 1e9, 1),
                                   "source": os.path.relpath(PMC_FILE, ROOT)}
    # the three first passes on the same input (each output byte-equal to the timed one)
    if not args.no_first_pass_ab:
        res["first_pass_ab"] = first_pass_ab(ley, torch, dev, out, n, min(args.steps, 10))
        ok = ok and all(v["same_output"] and v["guard"] == 0 for v in res["first_pass_ab"].values())
    if not args.no_cpu_baseline:
        # the oracle on the host cores, and the timed sort's output against it record by record
        res["cpu_baseline"], want = cpu_baseline(host, n, min(args.cpu_sample, n))
        got = out.cpu().numpy().reshape(n, 100)
        res["output_matches_oracle"] = bool(np.array_equal(got, want))
        ok = ok and res["output_matches_oracle"]
        del got, want
    del out
    torch.cuda.empty_cache()
    if not args.no_serve:
        res["serving"] = serving(ley, args.serve_requests, 50, 32 * 10**9)
    res["copy_ceiling"] = copy_ceiling(torch)
    del host
    if hasattr(torch._C, "_host_emptyCache"):  # return the cached pinned block (host pinned limit)
        torch._C._host_emptyCache()
    if not args.no_keys:
        res["flexible_keys"] = flexible_keys(ley, torch, datagen, dev, min(args.steps, 5))
        ok = ok and all(v["ordered"] and v["guard"] == 0 for k, v in res["flexible_keys"].items() if k != "steps")
    if not args.no_ascii:
        res["ascii_keys"] = ascii_keys(ley, torch, datagen, args.steps)
        ok = ok and res["ascii_keys"]["output_keys_ordered"] and res["ascii_keys"]["guard"] == 0
    if not args.no_external:
        torch.cuda.empty_cache()
        if hasattr(torch._C, "_host_emptyCache"):  # return the cached pinned block (host pinned limit)
            torch._C._host_emptyCache()
        try:
            res["external"] = external(ley, torch, datagen, rates, args.external_n, args.external_budget)
        except ley.LeyendaError as exc:  # e.g. the host cannot pin 60 GB: report, keep the line
            res["external"] = {"skipped": str(exc)}
    print(json.dumps(res), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
