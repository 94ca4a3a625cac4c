"""Pins of the two-tier equal-count fold oracle (Sec. 2.3 steps 1-5, Fig. 4)
against what fixes it independently: with at most one sample per
intermediate bin it is the classic fold the paper starts from (sort by
modular residual, cut into equal chunks, average: Sec. 2.3's three steps);
flux is conserved; a constant curve folds to that constant; points that all
share one residual give the overall mean in every bin; split parts carry the
bin mean in proportion to the points they take (hand-worked case)."""
import numpy as np
import pytest

import oracle


def _sort_chunk(t, f, P, nbins):
    x = t / P
    ph = x - np.floor(x)
    order = np.argsort(ph, kind="stable")
    return f.astype(np.float64)[order].reshape(nbins, -1).mean(axis=1)


@pytest.mark.parametrize("n,nbins", [(1024, 256), (4096, 256), (512, 64), (256, 256)])
def test_one_sample_per_mid_bin_is_sort_then_chunk(n, nbins):
    rng = np.random.default_rng(n + nbins)
    P = 0.75
    # residuals (i + 0.5) / n of a cycle, shuffled over 40 cycles: with n <= 4096
    # every intermediate bin holds at most one sample
    cyc = rng.integers(0, 40, n)
    t = (cyc + (rng.permutation(n) + 0.5) / n) * P
    f = (1.0 + rng.normal(0, 1e-3, n)).astype(np.float32)
    got = oracle.fold_eqcount(t, f, [P], nbins)[0]
    want = _sort_chunk(t, f, P, nbins)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)


def test_flux_conserved_and_constant_curve():
    rng = np.random.default_rng(3)
    n = 65000
    t = np.sort(rng.uniform(0, 1470, n))
    f = (1.0 + rng.normal(0, 3e-4, n)).astype(np.float32)
    periods = 1.0 / rng.uniform(1, 5, 7)
    m = oracle.fold_eqcount(t, f, periods)
    total = f.astype(np.float64).sum()
    for row in m:
        assert abs(row.sum() * n / 256 - total) <= 1e-9 * total
    c = np.full(n, 1.25, np.float32)
    assert np.all(oracle.fold_eqcount(t, c, periods) == 1.25)


def test_single_residual_gives_overall_mean():
    n = 1000
    t = np.arange(n) * 0.5            # period 0.5: every residual is 0
    f = np.linspace(0.9, 1.1, n).astype(np.float32)
    m = oracle.fold_eqcount(t, f, [0.5], 256)[0]
    np.testing.assert_allclose(m, f.astype(np.float64).mean(), rtol=1e-14)


def test_hand_worked_split():
    # 6 points, 4 final bins (1.5 points each), 8 intermediate bins:
    # residuals put 2 points (flux 1, 3) in bin 0, 1 point (flux 5) in bin 3,
    # 3 points (flux 7, 8, 9) in bin 6.
    P = 1.0
    t = np.array([0.01, 0.02, 0.40, 0.80, 0.81, 0.82])
    f = np.array([1, 3, 5, 7, 8, 9], np.float32)
    m = oracle.fold_eqcount(t, f, [P], nbins=4, n_mid=8)[0]
    # bin0 mean 2 (2 pts); bin3 mean 5; bin6 mean 8 (3 pts)
    # final 0: 1.5 pts of mean 2 -> 2
    # final 1: 0.5 pt of 2 + 1 pt of 5 -> (1 + 5) / 1.5 = 4
    # final 2: 1.5 pts of 8 -> 8; final 3: 1.5 pts of 8 -> 8
    np.testing.assert_allclose(m, [2.0, 4.0, 8.0, 8.0], rtol=1e-15)


def test_empty_and_invalid():
    m = oracle.fold_eqcount(np.zeros(0), np.zeros(0, np.float32), [0.5, 1.0], 16)
    assert np.isnan(m).all()
    m = oracle.fold_eqcount(np.arange(10.0), np.ones(10, np.float32), [0.0, -1.0, np.nan], 16)
    assert np.isnan(m).all()
