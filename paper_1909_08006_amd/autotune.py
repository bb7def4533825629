"""Autotuner for the sort's tuning parameters.

Sweeps the partition digit width (4..8 bits: 2^digit_bits buckets per level
of Algorithm 1), the partition tile (keys per thread), the big-bucket
threshold (Algorithm 1's bigBucketThreshold: buckets above it get another
device-wide pass), the radix-vs-comparison cutoff inside the local sort
(tinyBucketThreshold), the workgroup shapes and the first pass (separate
extraction and partition, or one fused pass), times each candidate on the GPU with HIP events on a
seeded workload, checks that every candidate returns exactly the bytes of the
default parameters (they may change speed only), and writes the fastest set
as a flat JSON object that ``leyenda_load_params`` reads.

    python -m paper_1909_08006_amd.autotune --n 20000000 --out params.json
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_SPACE = {
    "digit_bits": [4, 6, 8],
    "tile_items": [16, 32],
    "big_threshold": [1024, 2048],
    "tiny_threshold": [32, 64, 128, 192],
    "scatter_threads": [512, 1024],
    "local_threads": [256, 512],
    "first_pass": [0, 1],
}


def candidates(space: dict) -> list[dict]:
    keys = sorted(space)
    return [dict(zip(keys, vals)) for vals in itertools.product(*(space[k] for k in keys))]


def choose(timings: list[tuple[dict, float]]) -> dict:
    """Fastest candidate; ties go to the earlier candidate (deterministic)."""
    best = None
    for params, ms in timings:
        if best is None or ms < best[1]:
            best = (params, ms)
    if best is None:
        raise ValueError("no candidate was timed")
    return dict(best[0])


def write_params(path: str, params: dict, timings: list[tuple[dict, float]], workload: dict) -> None:
    doc = dict(params)
    doc["local_capacity"] = 2048
    doc["_workload"] = workload
    doc["_timings_ms"] = [{"params": p, "ms": round(ms, 4)} for p, ms in timings]
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)


def tune(n: int = 20_000_000, kind: str = "uniform", seed: int = 2, steps: int = 3,
         space: dict | None = None, out: str | None = None) -> dict:
    import torch
    import datagen
    import paper_1909_08006_amd as ley

    space = space or DEFAULT_SPACE
    host = torch.empty(n * 100, dtype=torch.uint8, pin_memory=True)
    (datagen.fill_skewed if kind == "skewed" else datagen.fill_uniform)(host.data_ptr(), n, seed)
    dev = host.to("cuda:0")
    out_t = torch.empty_like(dev)
    base = ley.get_params()
    ley.sort(dev, out_t)
    torch.cuda.synchronize()
    reference = out_t.clone()
    timings = []
    try:
        for cand in candidates(space):
            p = dict(base)
            p.update(cand)
            ley.set_params(**p)
            ley.sort(dev, out_t)  # warm-up (workspace sizing)
            torch.cuda.synchronize()
            if not torch.equal(out_t, reference):
                raise AssertionError(f"parameters {cand} changed the sorted bytes")
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                ley.sort(dev, out_t)
            e1.record()
            e1.synchronize()
            timings.append((cand, e0.elapsed_time(e1) / steps))
            print(f"[autotune] {cand} {timings[-1][1]:.3f} ms", file=sys.stderr, flush=True)
    finally:
        ley.set_params(**base)
    best = choose(timings)
    if out:
        write_params(out, best, timings, {"n": n, "kind": kind, "seed": seed, "steps": steps,
                                          "time": time.strftime("%Y-%m-%d %H:%M:%S")})
    return best


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=20_000_000)
    ap.add_argument("--kind", choices=["uniform", "skewed"], default="uniform")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--out", default="params.json")
    args = ap.parse_args()
    best = tune(args.n, args.kind, args.seed, args.steps, out=args.out)
    print(json.dumps(best))
    return 0


if __name__ == "__main__":
    sys.exit(main())
