"""Autotuner: candidate space, deterministic choice, JSON the library loads; on the
GPU, a small sweep whose every candidate returns the oracle's bytes."""
import json

import numpy as np
import pytest

from paper_1909_08006_amd import autotune


def test_candidates_cover_the_space():
    space = {"tile_items": [8, 16], "big_threshold": [512, 2048], "tiny_threshold": [16], "digit_bits": [8]}
    c = autotune.candidates(space)
    assert len(c) == 4
    assert {(x["tile_items"], x["big_threshold"]) for x in c} == {(8, 512), (8, 2048), (16, 512), (16, 2048)}


def test_choose_is_fastest_and_deterministic():
    t = [({"a": 1}, 3.0), ({"a": 2}, 2.0), ({"a": 3}, 2.0)]
    assert autotune.choose(t) == {"a": 2}
    with pytest.raises(ValueError):
        autotune.choose([])


def test_written_params_load_into_library(tmp_path):
    import paper_1909_08006_amd as ley
    old = ley.get_params()
    try:
        f = tmp_path / "params.json"
        autotune.write_params(str(f), {"digit_bits": 8, "tile_items": 8, "big_threshold": 1024, "tiny_threshold": 16},
                              [({"tile_items": 8}, 1.0)], {"n": 10})
        doc = json.loads(f.read_text())
        assert doc["tile_items"] == 8 and doc["_timings_ms"][0]["ms"] == 1.0
        p = ley.load_params(str(f))
        assert p["big_threshold"] == 1024 and p["tiny_threshold"] == 16
    finally:
        ley.set_params(**old)


@pytest.mark.gpu
def test_small_sweep_on_gpu(gpu, tmp_path):
    import torch
    import datagen
    import oracle
    out = tmp_path / "params.json"
    space = {"digit_bits": [5, 8], "tile_items": [8, 16], "big_threshold": [256, 2048], "tiny_threshold": [4, 32],
             "local_threads": [256, 512]}
    old = gpu.get_params()
    try:
        best = autotune.tune(n=400_000, kind="skewed", seed=3, steps=1, space=space, out=str(out))
        assert best in autotune.candidates(space)
        gpu.load_params(str(out))
        rec = datagen.skewed(400_000, 3)
        got = gpu.sort(torch.from_numpy(rec).cuda())
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), oracle.sort(rec))
    finally:
        gpu.set_params(**old)
