"""CPU model of the keyed sort's tie rounds (K > 10), checked against the
oracle's stable sort on K-byte keys.

The GPU path sorts by the 10-byte prefix, then resolves runs of equal leading
bytes six key bytes per round with one stable sort of (run number, window
bytes, position) entries; the rounds carry record indices, and the tied
positions take their records from the input once at the end.  This model
takes the same steps in numpy, so the
reasoning behind them (run numbering, windows masked to the key, only the
previous round's entries looked at, stability through positions) is checked on
many inputs without a GPU; the GPU tests compare the kernels with the oracle.
"""
import numpy as np
import pytest

import datagen
import oracle


def _stable_order(keys10: np.ndarray) -> np.ndarray:
    """Stable order of rows of a (m, 10) uint8 array (memcmp order)."""
    cols = tuple(keys10[:, b] for b in range(9, -1, -1))
    return np.lexsort((np.arange(keys10.shape[0]),) + cols)


def model_keyed(rec: np.ndarray, kb: int) -> np.ndarray:
    out, perm = oracle.sort(rec, return_perm=True)  # the 10-byte prefix sort (stable) and its order
    n = out.shape[0]
    # first round's tie marks: P[c] = record c ties record c - 1 on bytes 0..9
    P = np.zeros(n, dtype=bool)
    P[1:] = (out[1:, :10] == out[:-1, :10]).all(axis=1)
    cand_src = perm.astype(np.int64)  # candidate c -> input index of the record at its position
    cand_e0 = None                    # candidate c -> first-round entry owning its position
    slot0 = final_src = None          # per first-round entry: its position, its final record
    p = 10
    while p < kb:
        nc = cand_src.size
        eq_prev = P[:nc].copy()
        eq_next = np.zeros(nc, dtype=bool)
        eq_next[:-1] = P[1:nc]
        in_run = eq_prev | eq_next
        starts = eq_next & ~eq_prev
        if not in_run.any():
            break
        run = np.cumsum(starts) - 1  # the run holding c began at the latest start
        sel = np.nonzero(in_run)[0]
        src = cand_src[sel]
        if slot0 is None:  # first round: entries are output positions
            e0 = np.arange(sel.size)
            slot0 = sel.copy()
            final_src = src.copy()
        else:
            e0 = cand_e0[sel]
        ent = np.zeros((sel.size, 10), dtype=np.uint8)
        ent[:, :4] = run[sel].astype(">u4").view(np.uint8).reshape(-1, 4)
        for k, b in enumerate(range(p, p + 6)):
            if b < kb:
                ent[:, 4 + k] = rec[src, b]
        order = _stable_order(ent)  # entries in position order; the sort is stable
        s_sorted = src[order]
        # the q-th sorted entry takes the position of entry q (first-round entry e0[q])
        final_src[e0] = s_sorted
        e2 = ent[order]
        P = np.zeros(sel.size, dtype=bool)  # later rounds: neighbours of sorted entries
        P[1:] = (e2[1:] == e2[:-1]).all(axis=1)
        cand_src, cand_e0 = s_sorted, e0
        p += 6
    if slot0 is not None:  # the tied positions take their records from the input
        out[slot0] = rec[final_src]
    return out


def _records(n, seed, shared, variants):
    """n records copied from a few bases, the first `shared` bytes mostly equal,
    chosen bytes varied over a few values."""
    rng = np.random.default_rng(seed)
    base = datagen.uniform(7, seed)
    rec = datagen.uniform(n, seed + 1)
    rec[:, :shared] = base[rng.integers(0, 7, n), :shared]
    for b, vals in variants:
        rec[:, b] = rng.integers(0, vals, n)
    return rec


@pytest.mark.parametrize("kb", [11, 12, 15, 16, 17, 22, 23, 40, 41, 61, 95, 100])
def test_model_matches_oracle(kb):
    for trial in range(3):
        rec = _records(3000, 10 * kb + trial, 100, [(3, 2), (12, 3), (16, 2), (40, 2), (77, 3), (99, 2)])
        np.testing.assert_array_equal(model_keyed(rec, kb), oracle.sort(rec, key_bytes=kb))


def test_model_all_equal_keys_keep_input_order():
    rec = datagen.uniform(500, 3)
    rec[:, :60] = 0x41
    np.testing.assert_array_equal(model_keyed(rec, 60), rec)


def test_model_uniform_keys_need_no_round():
    rec = datagen.uniform(2000, 4)
    np.testing.assert_array_equal(model_keyed(rec, 30), oracle.sort(rec, key_bytes=30))
