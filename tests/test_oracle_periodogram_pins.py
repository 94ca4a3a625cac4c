"""Pins of the periodogram post-processing oracle: SDE (Eq. 3) against a
closed form and its affine invariance; peaks (Sec. 4.2) against a
pure-Python run finder; harmonic codes on a constructed grid."""
import itertools
import math

import numpy as np
import pytest

import oracle


def test_sde_closed_form_single_spike():
    # n - 1 zeros and one value a: mean a/n, sd a sqrt(n-1)/n, SDE = sqrt(n-1)
    for n in (2, 10, 1000):
        v = np.zeros(n, np.float32)
        v[n // 3] = 7.0
        r = oracle.periodogram(v)
        assert r["sde"][0] == pytest.approx(math.sqrt(n - 1), rel=1e-6)


def test_sde_affine_invariant_and_degenerate():
    rng = np.random.default_rng(1)
    v = rng.normal(size=5000).astype(np.float32)
    a = oracle.periodogram(v)["sde"][0]
    b = oracle.periodogram((3.0 * v.astype(np.float64) + 11.0).astype(np.float32))["sde"][0]
    assert a == pytest.approx(b, rel=1e-5)
    assert oracle.periodogram(np.ones(10, np.float32))["sde"][0] == 0.0
    assert oracle.periodogram(np.zeros((1, 0), np.float32))["sde"][0] == 0.0


def _brute(v, nsigma, min_width, max_peaks):
    ok = [x for x in v if not math.isnan(x)]
    m = sum(ok) / len(ok)
    sd = math.sqrt(sum((x - m) ** 2 for x in ok) / len(ok))
    thr = m + nsigma * sd
    peaks = []
    i = 0
    for above, grp in itertools.groupby(enumerate(v), key=lambda e: (not math.isnan(e[1])) and e[1] > thr):
        grp = list(grp)
        if above and len(grp) > min_width:
            best = max(grp, key=lambda e: (e[1], -e[0]))
            peaks.append((float(best[1]), best[0], len(grp)))
    n = len(peaks)
    peaks.sort(key=lambda p: (-p[0], p[1]))
    return n, peaks[:max_peaks]


@pytest.mark.parametrize("seed", range(12))
def test_peaks_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(20, 400))
    v = np.round(rng.normal(size=n) * 2).astype(np.float32)    # ties, runs
    v[rng.uniform(size=n) < 0.03] = np.nan
    nsig = float(np.float32(rng.uniform(0.0, 1.0)))
    mw = int(rng.integers(0, 4))
    r = oracle.periodogram(v, nsigma=nsig, min_width=mw, max_peaks=5)
    npk, peaks = _brute(list(v.astype(np.float64)), nsig, mw, 5)
    assert r["n_peaks"][0] == npk
    for j, (pv, pi, pw) in enumerate(peaks):
        assert r["val"][0, j] == np.float32(pv) and r["idx"][0, j] == pi and r["width"][0, j] == pw
    for j in range(len(peaks), 5):
        assert r["idx"][0, j] == -1 and r["width"][0, j] == 0


def test_harmonic_codes():
    k = 20000
    periods = 1.0 / np.linspace(1.0, 5.0, k)
    v = np.zeros(k, np.float32)

    def bump(p, h):
        i = int(np.argmin(np.abs(periods - p)))
        v[i - 3:i + 4] = h
        return i
    bump(0.75, 10.0)     # best
    bump(0.375, 8.0)     # half the period
    bump(0.25, 6.0)      # a third
    bump(0.45, 7.0)      # unrelated
    r = oracle.periodogram(v, periods, nsigma=3.0, min_width=3, max_peaks=4)
    assert list(r["val"][0]) == [10.0, 8.0, 7.0, 6.0]
    assert list(r["harmonic"][0]) == [1, -2, 0, -3]
    assert list(r["width"][0]) == [7, 7, 7, 7]
