"""bench.py's output checks (keys in order on the first 10 or K bytes) on the CPU:
they accept the oracle's sorted output and reject a planted swap."""
import os
import sys

import numpy as np
import pytest

import datagen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    import bench as b
    return b


def _tensor(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).reshape(-1))


def test_keys_ordered(bench):
    import torch
    rec = datagen.skewed(3000, 5)
    out = oracle.sort(rec)
    assert bench.keys_ordered(torch, _tensor(out), 3000)
    bad = out.copy()
    i = int(np.nonzero((bad[1:, :10] != bad[:-1, :10]).any(axis=1))[0][100])
    bad[[i, i + 1]] = bad[[i + 1, i]]
    assert not bench.keys_ordered(torch, _tensor(bad), 3000)


@pytest.mark.parametrize("kb", [1, 4, 10, 20, 100])
def test_prefix_ordered(bench, kb):
    import torch
    rec = datagen.uniform(2000, 6)
    rec[:, :12] = rec[:, :12] % 3  # ties on short prefixes
    out = oracle.sort(rec, key_bytes=kb)
    assert bench.prefix_ordered(torch, _tensor(out), 2000, kb)
    diff = np.nonzero((out[1:, :kb] != out[:-1, :kb]).any(axis=1))[0]
    i = int(diff[len(diff) // 2])
    bad = out.copy()
    bad[[i, i + 1]] = bad[[i + 1, i]]
    assert not bench.prefix_ordered(torch, _tensor(bad), 2000, kb)
