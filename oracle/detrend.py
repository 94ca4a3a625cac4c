"""CPU oracle of the light-curve pre-processing (Sec. 2.2, Fig. 3).

TEST INFRASTRUCTURE ONLY: the plain, slow FP64 statement of what the GPU
pre-processing computes. Only ``tests/`` and the benchmark's CPU leg may
import it; the product path never does, and the two share no code.

The paper's steps, in its order, with the readings its text leaves open:

1. Segments (Sec. 2.2): scanning in time order, a new segment starts where
   the time step exceeds 30 cadences (30 x 0.020428 d, about 14.7 h) or the
   flux step exceeds 5 standard deviations of the curve's flux. Reading: the
   curve is time-sorted; the time step is taken from the previous sample,
   known transit or not (a gap is a gap in the observations); the flux step
   is taken only between samples outside known transits, from the previous
   such sample (so a masked transit's dip does not split its segment); the
   standard deviation is the sample std (ddof 1) of the samples outside known
   transits.
2. Spline continuum of each segment with known transits masked, outliers
   beyond 3 sigma removed iteratively, the smoothing chosen by BIC. Reading:
   a least-squares cubic B-spline with uniform knots; the smoothing parameter
   is the knot spacing, tried from a candidate list (each spacing h gives
   L = max(1, ceil(span / h)) equal spans over the segment's time range and
   L + 3 basis functions). For each spacing: fit the points that are neither
   masked nor clipped, take the residuals of every segment point, their
   scatter sigma (ddof 0) over the fitted points, clip every unmasked point
   with |residual| > 3 sigma, and refit until the clipped set repeats (at
   most 10 fits; the last fit and the clipped set it used are kept).
   BIC = n ln(RSS / n) + m ln(n) over the n fitted points with m basis
   functions; the smallest wins (ties: the earlier candidate). A spacing
   with fewer than 2m fitted points is not tried; a segment where none can
   be tried is dropped.
3. Divide the segment's flux by its spline.
4. Drop 30 points at each end of each segment (a segment of 60 points or
   fewer vanishes), and the points clipped by the chosen fit (known-transit
   points are never clipped).
5. Stitch: the kept points in time order.
"""
from __future__ import annotations

import numpy as np
from scipy.interpolate import BSpline

CADENCE = 0.020428          # d: Kepler long cadence as Sec. 2.2 gives it
GAP_CADENCES = 30
JUMP_SIGMA = 5.0
CLIP_SIGMA = 3.0
EDGE = 30
MAX_FITS = 10
SPACINGS = (0.5, 0.75, 1.0, 1.5, 2.0, 3.0, 5.0)     # d


def segments(t, flux, transit=None, cadence=CADENCE, gap_cadences=GAP_CADENCES,
             jump_sigma=JUMP_SIGMA):
    """Step 1: [start, end) index ranges of the segments of a time-sorted curve."""
    t = np.asarray(t, np.float64)
    f = np.asarray(flux, np.float32).astype(np.float64)
    n = t.size
    tr = np.zeros(n, bool) if transit is None else np.asarray(transit, bool)
    if n == 0:
        return []
    free = f[~tr]
    sd = free.std(ddof=1) if free.size > 1 else 0.0
    out, start, prev = [], 0, -1
    for i in range(n):
        opens = i > 0 and t[i] - t[i - 1] > gap_cadences * cadence
        if not tr[i]:
            opens = opens or (prev >= 0 and abs(f[i] - f[prev]) > jump_sigma * sd)
            prev = i
        if opens:
            out.append((start, i))
            start = i
    out.append((start, n))
    return out


def design(tseg, a, span, h):
    """Cubic B-spline basis of a segment at spacing h: (B [n, m], m)."""
    L = max(1, int(np.ceil(span / h))) if span > 0 else 1
    he = span / L if span > 0 else 1.0
    knots = a + he * np.arange(-3, L + 4, dtype=np.float64)
    B = BSpline.design_matrix(tseg, knots, 3, extrapolate=True).toarray()
    return B, L + 3


def fit_segment(tseg, fseg, trseg, h, clip_sigma=CLIP_SIGMA, max_fits=MAX_FITS):
    """Step 2 at one spacing: (continuum, clipped mask, BIC, fitted count) or
    None when fewer than 2m points can be fitted."""
    a, span = tseg[0], tseg[-1] - tseg[0]
    B, m = design(tseg, a, span, h)
    clip = np.zeros(tseg.size, bool)
    for _ in range(max_fits):
        use = ~trseg & ~clip
        if use.sum() < 2 * m:
            return None
        coef = np.linalg.lstsq(B[use], fseg[use], rcond=None)[0]
        s = B @ coef
        r = fseg - s
        sig = r[use].std(ddof=0)
        new = ~trseg & (np.abs(r) > clip_sigma * sig)
        if np.array_equal(new, clip):
            break
        clip_used = clip
        clip = new
    else:
        clip = clip_used
    use = ~trseg & ~clip
    nfit = int(use.sum())
    rss = float(np.sum((fseg - s)[use] ** 2))
    bic = nfit * np.log(rss / nfit) + m * np.log(nfit) if rss > 0 else -np.inf
    return s, clip, bic, nfit


def detrend(t, flux, transit=None, spacings=SPACINGS, cadence=CADENCE, edge=EDGE):
    """Steps 1-5. Returns (detrended flux f64 [n], keep mask [n], per-segment
    records (start, end, chosen spacing or NaN))."""
    t = np.asarray(t, np.float64)
    f = np.asarray(flux, np.float32).astype(np.float64)
    n = t.size
    tr = np.zeros(n, bool) if transit is None else np.asarray(transit, bool)
    out = np.zeros(n)
    keep = np.zeros(n, bool)
    recs = []
    for s0, s1 in segments(t, f, tr, cadence=cadence):
        if s1 - s0 <= 2 * edge:
            recs.append((s0, s1, np.nan))
            continue
        ts, fs, trs = t[s0:s1], f[s0:s1], tr[s0:s1]
        best = None
        for h in spacings:
            r = fit_segment(ts, fs, trs, h)
            if r is not None and (best is None or r[2] < best[1][2]):
                best = (h, r)
        if best is None:
            recs.append((s0, s1, np.nan))
            continue
        h, (cont, clip, _, _) = best
        out[s0:s1] = fs / cont
        k = ~clip
        k[:edge] = False
        k[k.size - edge:] = False      # (k[-edge:] would clear every point when edge = 0)
        keep[s0:s1] = k
        recs.append((s0, s1, h))
    return out, keep, recs
