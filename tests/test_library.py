"""The C-ABI library loads and exports every declared entry point (no GPU work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions() -> list[str]:
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(leyenda_\w+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["leyenda_sort", "leyenda_sort_runs", "leyenda_merge", "leyenda_sort_batch",
                 "leyenda_load_params", "leyenda_workspace_bytes", "leyenda_status_string"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1909_08006_amd as ley
    lib = ley.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_sort_parts_rule():
    import paper_1909_08006_amd as ley
    assert [ley.sort_parts(n) for n in (0, 1, 8 * 2**20 - 1)] == [1, 1, 1]
    assert [ley.sort_parts(n) for n in (8 * 2**20, 10**8, 10**9)] == [4, 4, 4]


def test_status_strings_and_param_checks():
    import paper_1909_08006_amd as ley
    lib = ley.load()
    assert lib.leyenda_status_string(-3) == b"does not fit the device budget"
    assert lib.leyenda_status_string(0) == b"ok"
    p = ley.get_params()
    assert p["digit_bits"] == 8 and p["local_capacity"] == 2048 and p["scatter_threads"] == 1024
    assert p["local_threads"] == 512 and p["tile_items"] == 32 and p["tiny_threshold"] == 128
    assert p["first_pass"] == 1
    for bad in [dict(tile_items=3), dict(big_threshold=0), dict(big_threshold=4096), dict(tiny_threshold=0),
                dict(tiny_threshold=257), dict(digit_bits=3), dict(digit_bits=9), dict(digit_bits=16),
                dict(scatter_threads=384), dict(first_pass=3),
                dict(local_threads=128)]:
        with pytest.raises(ley.LeyendaError):
            ley.set_params(**bad)
    assert ley.get_params() == p


def test_load_params_json(tmp_path):
    import paper_1909_08006_amd as ley
    old = ley.get_params()
    try:
        f = tmp_path / "params.json"
        f.write_text('{"tile_items": 8, "big_threshold": 1000, "tiny_threshold": 16, "scatter_threads": 256, '
                     '"comment": "x"}')
        p = ley.load_params(str(f))
        assert p["tile_items"] == 8 and p["big_threshold"] == 1000 and p["tiny_threshold"] == 16
        assert p["scatter_threads"] == 256
    finally:
        ley.set_params(**old)


def test_workspace_bytes_grows_with_n():
    import paper_1909_08006_amd as ley
    a, b = ley.workspace_bytes(1000), ley.workspace_bytes(100_000_000)
    assert 0 < a < b
    assert b < 100_000_000 * 64  # tuples (32 B) + index (4 B) + tables: well under 64 B per record


def test_missing_library_fails_loudly(monkeypatch):
    import paper_1909_08006_amd as ley
    monkeypatch.setattr(ley, "_lib", None)
    monkeypatch.setattr(ley, "LIB_PATH", "/nonexistent/libleyenda.so")
    with pytest.raises(RuntimeError, match="not built"):
        ley.load()


def test_plan_runs_budget_math():
    """Run planning is host arithmetic: equal runs covering n, fewer runs for more memory."""
    import paper_1909_08006_amd as ley
    for n, budget in [(600_000_000, 30 * 10**9), (10**6, 50 << 20), (5, 1 << 30)]:
        r, k = ley.plan_runs(n, budget)
        assert r * k >= n and r * (k - 1) < n
        assert ley.plan_runs(n, budget * 2)[1] <= k
    r, k = ley.plan_runs(600_000_000, 30 * 10**9)
    assert 5 <= k <= 20  # 60 GB of records through a 30 GB device budget
    with pytest.raises(ley.LeyendaError) as ei:
        ley.plan_runs(10**6, 1000)
    assert ei.value.status == -3
    assert ley.plan_runs(0, 1000) == (0, 0)


def test_plan_external_kept_runs():
    """The one-call external plan: the runs of leyenda_plan_runs, and the last
    two runs kept on the device when the merge fits beside them; many tiny runs
    under a budget near one run's footprint keep one run or none; one run is
    the output itself."""
    import paper_1909_08006_amd as ley
    assert ley.plan_external(600_000_000, 30 * 10**9) == (*ley.plan_runs(600_000_000, 30 * 10**9), 2)
    assert ley.plan_external(1000, 1 << 30) == (1000, 1, 1)
    assert ley.plan_external(0, 1000) == (0, 0, 0)
    n, tiers = 7111, set()
    for budget in range(150_000, 1_200_000, 2_000):
        try:
            r, k, kept = ley.plan_external(n, budget)
        except ley.LeyendaError as exc:
            assert exc.status == -3  # no run fits, or more runs than the merge takes
            continue
        assert (r, k) == ley.plan_runs(n, budget)
        assert kept in (0, 1, 2)
        tiers.add(kept)
    assert tiers == {0, 1, 2}
    with pytest.raises(ley.LeyendaError) as ei:
        ley.plan_external(10**6, 1000)
    assert ei.value.status == -3


def test_bench_refuses_several_gpus():
    """bench.py sorts on one GPU: --gpus above 1 exits with status 2 and says so."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_keyed_sort_argument_checks():
    """leyenda_sort_keyed rejects bad key sizes and buffers before any device work."""
    import paper_1909_08006_amd as ley
    lib = ley.load()
    einval = -1
    assert lib.leyenda_status_string(einval) != b"ok"
    for kb in (0, 101, 1000):
        assert lib.leyenda_sort_keyed(None, 10, kb, None, None) == einval
        assert b"key_bytes" in lib.leyenda_last_error()
    assert lib.leyenda_sort_keyed(None, 0, 20, None, None) == 0  # nothing to sort
    assert lib.leyenda_sort_keyed(None, 10, 20, None, None) == einval  # NULL buffers
    assert lib.leyenda_sort_keyed(ctypes.c_void_p(4096), 10, 20, ctypes.c_void_p(4098), None) == einval  # misaligned
    assert lib.leyenda_sort_keyed(ctypes.c_void_p(4096), 10, 20, ctypes.c_void_p(4096 + 500), None) == einval  # overlap


def test_first_pass_rule():
    """The fused first passes run only for sorts split into output parts whose
    partition tile holds a fused tile (8,192 keys; 4,096 with the record copy)."""
    import paper_1909_08006_amd as ley
    old = ley.get_params()
    try:
        ley.set_params(first_pass=1, tile_items=32)
        assert [ley.first_pass(n) for n in (1000, 8 * 2**20 - 1, 8 * 2**20, 10**8)] == [0, 0, 1, 1]
        ley.set_params(first_pass=1, tile_items=16)
        assert ley.first_pass(10**8) == 0
        ley.set_params(first_pass=2, tile_items=16)
        assert ley.first_pass(10**8) == 2
        ley.set_params(first_pass=2, tile_items=8)
        assert ley.first_pass(10**8) == 0
        ley.set_params(first_pass=0, tile_items=32)
        assert ley.first_pass(10**8) == 0
        import pytest
        with pytest.raises(ley.LeyendaError):
            ley.set_params(first_pass=3)
    finally:
        ley.set_params(**old)
