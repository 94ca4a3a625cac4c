"""Pins for the pre-processing oracle (Sec. 2.2, Fig. 3) against what the
paper's steps and independent library routines fix: segment boundaries of
constructed gaps and jumps, a continuum equal to scipy's own least-squares
spline (make_lsq_spline, a separate QR solve) on the points the oracle kept in
its fit, exact detrending of a trend inside the spline space, clipping of
injected outliers, masked transits left out of the fit and kept in the
output, BIC choosing fine knots for a fast trend and coarse knots for flat
noise, and the 30-point edge crop. The curves carry a trend, as real ones do:
on pure white noise the paper's 5-sigma flux-step test splits wherever two
neighbours differ by 3.5 of their own sigma (a few times per 10,000 samples)."""
import numpy as np
import pytest
from scipy.interpolate import make_lsq_spline

from oracle import detrend as od

DT = od.CADENCE


def _grid(n, t0=0.0):
    return t0 + DT * np.arange(n)


def _knots(t, h):
    span = t[-1] - t[0]
    L = max(1, int(np.ceil(span / h)))
    he = span / L
    return t[0] + he * np.arange(-3, L + 4)


def test_segments_at_gaps_and_jumps():
    rng = np.random.default_rng(1)
    t = np.concatenate([_grid(500), _grid(400, 12.0), _grid(300, 25.0)])   # gaps of ~1.8 d and ~4.8 d
    f = (1.0 + rng.normal(0, 1e-3, t.size)).astype(np.float32)
    f[700:720] += np.float32(0.05)          # a 50-sigma step up at 700 and back at 720
    seg = od.segments(t, f)
    assert seg == [(0, 500), (500, 700), (700, 720), (720, 900), (900, 1200)]
    # a long step inflates the curve's own sigma past a fifth of the step: no split
    g = f.copy()
    g[700:720] -= np.float32(0.05)
    g[600:] += np.float32(0.05)
    assert od.segments(t, g) == [(0, 500), (500, 900), (900, 1200)]
    # a step of exactly 30 cadences does not split; one just above does
    t2 = np.array([0.0, 30 * DT, 60 * DT + 1e-9])
    assert od.segments(t2, np.ones(3, np.float32)) == [(0, 2), (2, 3)]


def test_masked_transit_does_not_split_its_segment():
    rng = np.random.default_rng(2)
    t = _grid(2000)
    f = 1.0 + 5e-3 * np.sin(t / 3.0) + rng.normal(0, 1e-4, t.size)
    tr = np.zeros(t.size, bool)
    tr[1000:1010] = True
    f[tr] -= 0.2                                                            # deep: 200 sigma
    f = f.astype(np.float32)
    assert od.segments(t, f, tr) == [(0, 2000)]
    assert len(od.segments(t, f)) == 3                                      # unmasked, it splits


def test_trend_in_spline_space_detrends_exactly():
    # f32-exact linear trend (in every cubic spline space): the continuum is
    # the trend itself, every kept point detrends to 1
    t = np.arange(3000) * 2.0 ** -6
    f = (1.0 + 2.0 ** -10 * t / 64.0).astype(np.float32)
    assert np.array_equal(f.astype(np.float64), 1.0 + 2.0 ** -10 * t / 64.0)
    out, keep, recs = od.detrend(t, f, cadence=2.0 ** -6)
    assert keep.sum() > 0
    np.testing.assert_allclose(out[keep], 1.0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("h", [0.5, 1.5, 5.0])
def test_continuum_equals_independent_lsq_spline(h):
    rng = np.random.default_rng(3)
    t = _grid(2500)
    trend = 1.0 + 3e-3 * np.sin(t / 3.1) + 1e-3 * (t / t[-1]) ** 2
    f = (trend + rng.normal(0, 5e-4, t.size)).astype(np.float32)
    tr = np.zeros(t.size, bool)
    tr[800:830] = True
    r = od.fit_segment(t, f.astype(np.float64), tr, h)
    cont, clip = r[0], r[1]
    use = ~tr & ~clip
    ref = make_lsq_spline(t[use], f[use].astype(np.float64), _knots(t, h), k=3)
    np.testing.assert_allclose(cont, ref(t), rtol=0, atol=1e-9)
    # the clipped set is the 3-sigma set of this very fit (a fixed point)
    res = f.astype(np.float64) - cont
    sig = res[use].std()
    again = ~tr & (np.abs(res) > 3 * sig)
    assert np.array_equal(again, clip)


def test_outliers_clipped_and_dropped():
    rng = np.random.default_rng(4)
    t = _grid(3000)
    f = 1.0 + 4e-3 * np.cos(t / 5.0) + rng.normal(0, 3e-4, t.size)
    bad = np.array([200, 1234, 2222, 2700])
    f[bad] += np.array([4e-3, -5e-3, 4.5e-3, -4e-3])     # clipped, yet below the 5-sigma split
    f = f.astype(np.float32)
    out, keep, recs = od.detrend(t, f)
    assert not keep[bad].any()
    # the chosen fit is the fit of the data without the outliers
    h = recs[0][2]
    use = keep.copy()
    use[:30] = use[-30:] = True
    clean = od.fit_segment(np.delete(t, bad), np.delete(f, bad).astype(np.float64),
                           np.zeros(t.size - bad.size, bool), h)
    cont = f.astype(np.float64) / out
    np.testing.assert_allclose(np.delete(cont, bad), clean[0], rtol=0, atol=1e-9)


def test_masked_transit_kept_and_depth_preserved():
    rng = np.random.default_rng(5)
    t = _grid(4000)
    trend = 1.0 + 4e-3 * np.sin(t / 2.3)
    tr = ((t % 7.0) > 3.0) & ((t % 7.0) < 3.15)
    f = (trend * np.where(tr, 0.99, 1.0) + rng.normal(0, 2e-4, t.size)).astype(np.float32)
    out, keep, recs = od.detrend(t, f, tr)
    inner = np.zeros(t.size, bool)
    inner[30:-30] = True
    assert keep[tr & inner].all()
    assert abs(out[tr & keep].mean() - 0.99) < 3e-4
    assert abs(out[~tr & keep].mean() - 1.0) < 3e-5
    # leaving the masked points out of the fit is the same as deleting them
    h = recs[0][2]
    cont_ref = od.fit_segment(t[~tr], f[~tr].astype(np.float64), np.zeros((~tr).sum(), bool), h)[0]
    np.testing.assert_allclose((f.astype(np.float64) / out)[~tr], cont_ref, rtol=0, atol=1e-9)


def test_bic_prefers_fine_knots_for_fast_trends_and_coarse_for_noise():
    rng = np.random.default_rng(6)
    t = _grid(4000)
    fast = (1.0 + 1e-2 * np.sin(2 * np.pi * t / 2.0) + rng.normal(0, 1e-4, t.size)).astype(np.float32)
    flat = (1.0 + 1e-3 * t / t[-1] + rng.normal(0, 1e-4, t.size)).astype(np.float32)
    assert od.detrend(t, fast)[2][0][2] == 0.5
    assert od.detrend(t, flat)[2][0][2] == 5.0


def test_edges_cropped_and_short_segments_dropped():
    rng = np.random.default_rng(7)
    t = np.concatenate([_grid(60), _grid(61, 10.0), _grid(500, 20.0)])
    f = (1.0 + 5e-3 * np.sin(t / 3.0) + rng.normal(0, 1e-4, t.size)).astype(np.float32)
    out, keep, recs = od.detrend(t, f)
    assert [r[:2] for r in recs] == [(0, 60), (60, 121), (121, 621)]
    assert not keep[:60].any()                         # 60 points: nothing left
    assert keep[60:121].sum() <= 1 and not keep[60:90].any() and not keep[91:121].any()
    assert not keep[121:151].any() and not keep[591:].any()
    assert keep[151:591].sum() >= 430


def test_transit_after_a_gap_opens_the_next_segment():
    # a gap is a gap in the observations whether or not the samples after it are
    # masked: a known transit right after a 2-day gap starts the next segment
    # (kept with the segment before the gap, its continuum would be unconstrained)
    rng = np.random.default_rng(9)
    t = np.concatenate([_grid(1000), _grid(1000, 22.0)])
    f = (1.0 + 3e-3 * np.sin(t / 4.0) + rng.normal(0, 2e-4, t.size)).astype(np.float32)
    tr = np.zeros(t.size, bool)
    tr[1000:1008] = True
    assert od.segments(t, f, tr) == [(0, 1000), (1000, 2000)]
    # a masked sample does not serve as the previous sample of a flux step
    g = f.copy()
    g[500:504] -= np.float32(0.05)
    m = np.zeros(t.size, bool)
    m[500:504] = True
    assert od.segments(t, g, m) == [(0, 1000), (1000, 2000)]
