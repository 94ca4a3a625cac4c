"""Pins of the per-curve reduction oracle (best scores over trial periods,
Sec. 2.1 and Sec. 3.2) against definitions computed another way: pure-Python
sorting, numpy's first-occurrence argmax and numpy's lexsort."""
import math

import numpy as np
import pytest

import oracle


def _brute(row, top, gate=None, gate_min=0.0):
    cand = [(float(v), i) for i, v in enumerate(row)
            if not math.isnan(v) and (gate is None or gate[i] >= gate_min)]
    cand.sort(key=lambda e: (-e[0], e[1]))
    cand = cand[:top]
    vals = [c[0] for c in cand] + [-math.inf] * (top - len(cand))
    idx = [c[1] for c in cand] + [-1] * (top - len(cand))
    return np.array(vals, np.float32), np.array(idx, np.int64)


def test_brute_force_with_ties_nan_and_gate():
    rng = np.random.default_rng(5)
    for trial in range(40):
        n = int(rng.integers(0, 60))
        top = int(rng.integers(1, 12))
        row = rng.integers(-3, 4, n).astype(np.float32)       # many ties
        row[rng.uniform(size=n) < 0.1] = np.nan
        row[rng.uniform(size=n) < 0.05] = -np.inf
        gate = rng.uniform(0, 10, n).astype(np.float32)
        gate[rng.uniform(size=n) < 0.1] = np.nan
        use_gate = trial % 2 == 1
        v, i = oracle.topk(row.reshape(1, n), top, gate if use_gate else None, 4.0)
        bv, bi = _brute(row, top, gate if use_gate else None, 4.0)
        np.testing.assert_array_equal(i[0], bi)
        np.testing.assert_array_equal(v[0], bv)


def test_top1_is_first_occurrence_argmax():
    rng = np.random.default_rng(6)
    x = rng.integers(0, 50, (7, 1000)).astype(np.float32)
    v, i = oracle.topk(x, 1)
    np.testing.assert_array_equal(i[:, 0], np.argmax(x, axis=1))
    np.testing.assert_array_equal(v[:, 0], x.max(axis=1))


def test_full_order_is_lexsort():
    rng = np.random.default_rng(7)
    x = (rng.normal(size=(3, 300)) * 4).round().astype(np.float32)
    v, i = oracle.topk(x, 300)
    for r in range(3):
        order = np.lexsort((np.arange(300), -x[r]))
        np.testing.assert_array_equal(i[r], order)
        np.testing.assert_array_equal(v[r], x[r][order])


def test_empty_rows_and_all_gated():
    v, i = oracle.topk(np.zeros((2, 0), np.float32), 3)
    assert (i == -1).all() and np.isneginf(v).all()
    x = np.ones((1, 5), np.float32)
    v, i = oracle.topk(x, 2, gate=np.zeros(5, np.float32), gate_min=1.0)
    assert (i == -1).all()
