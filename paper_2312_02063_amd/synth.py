"""Seeded synthetic light curves and trial grids.

This module only makes inputs: timestamps, fluxes with injected transits, and
trial-period grids. It holds none of the fold or score arithmetic, and both
the GPU path and the CPU oracle's tests draw their inputs from it.

The shapes follow the paper's workloads: Kepler long cadence (29.4 min,
Sec. 2.2 and Sec. 3), up to four years of data with gaps, white plus
correlated noise, USP transit parameters of Table 2, box or trapezoid
transits (Sec. 2.6, Fig. 6), and trial grids spanning 0.2-1.0 d (Sec. 2.1).
Kepler DR25 light curves are not available here; these curves stand in for
them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CADENCE_D = 29.4 / 1440.0          # Kepler long cadence, days
BJD_OFFSET = 2454833.0             # Kepler BJD - 2454833 epoch offset


@dataclass
class Curve:
    t: np.ndarray                  # float64 [n], days
    flux: np.ndarray               # float32 [n], relative flux
    truth: dict = field(default_factory=dict)


def freq_grid(fmin: float, fmax: float, k: int) -> np.ndarray:
    """Trial periods uniform in frequency: P_j = 1 / (fmin + j (fmax - fmin) / (k - 1))."""
    if k == 1:
        return np.array([1.0 / fmin])
    j = np.arange(k, dtype=np.float64)
    f = fmin + j * ((fmax - fmin) / (k - 1))
    return 1.0 / f


def period_grid(pmin: float, pmax: float, k: int) -> np.ndarray:
    """Trial periods uniform in period (the paper's 100,000-period grid, Sec. 2.1)."""
    return np.linspace(pmin, pmax, k, dtype=np.float64)


def box_mask(t: np.ndarray, period: float, epoch: float, duration: float) -> np.ndarray:
    """In-transit samples of a box transit centred half a duration after each epoch."""
    ph = np.mod(t - epoch, period)
    return ph < duration


def trapezoid(t: np.ndarray, period: float, epoch: float, duration: float, depth: float,
              ratio: float) -> np.ndarray:
    """Trapezoid transit profile (Sec. 2.6, Fig. 6), negative in transit.

    ``duration`` is the width at half depth and ``ratio`` the short-base to
    long-base ratio; the transit is centred at ``epoch`` (mod ``period``).
    """
    long_b = 2.0 * duration / (1.0 + ratio)
    short_b = ratio * long_b
    x = np.abs(np.mod(t - epoch + 0.5 * period, period) - 0.5 * period)
    prof = np.zeros_like(t)
    flat = x <= 0.5 * short_b
    ramp = (x > 0.5 * short_b) & (x < 0.5 * long_b)
    prof[flat] = -depth
    if long_b > short_b:
        prof[ramp] = -depth * (0.5 * long_b - x[ramp]) / (0.5 * (long_b - short_b))
    return prof


def depth_for_snr(alpha: float, sigma: float, n: int, duration: float, period: float) -> float:
    """Transit depth that gives SNR alpha by Eq. 2 (Sec. 2.6), solved for d."""
    return alpha * sigma / np.sqrt(n * duration / period)


def plain_curve(seed: int = 1001, n: int = 4000, sigma: float = 1e-3, period: float = 0.5,
                depth: float = 5e-4, duration_h: float = 1.0, t0: float = 0.0) -> Curve:
    """Uniform-cadence curve, white noise and one box transit at a random epoch.

    With the defaults: 4,000 samples (~82 d), sigma 1e-3, P = 0.5 d, depth
    5e-4, 1 h duration.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.arange(n, dtype=np.float64) * CADENCE_D
    epoch = rng.uniform(0.0, period)
    dur = duration_h / 24.0
    f = 1.0 + rng.normal(0.0, sigma, n)
    inb = box_mask(t, period, epoch, dur)
    f[inb] -= depth
    return Curve(t + t0, f.astype(np.float32),
                 dict(period=period, epoch=epoch + t0, duration=dur, depth=depth, sigma=sigma,
                      n_in=int(inb.sum())))


def _drop_gaps(rng, ncad: int, keep: int, span: float, gap_min: float, gap_max: float) -> np.ndarray:
    """Cut gaps of U(gap_min, gap_max) days at uniform start times until exactly ``keep`` remain."""
    mask = np.ones(ncad, dtype=bool)
    remaining = ncad
    while remaining > keep:
        start = rng.uniform(0.0, span)
        length = rng.uniform(gap_min, gap_max)
        i0 = int(np.floor(start / CADENCE_D))
        i1 = min(ncad, int(np.ceil((start + length) / CADENCE_D)))
        idx = np.nonzero(mask[i0:i1])[0] + i0
        need = remaining - keep
        if idx.size > need:
            idx = idx[:need]
        mask[idx] = False
        remaining -= idx.size
    return mask


def kepler_long_curve(seed: int = 1002, n_keep: int = 65000, span_d: float = 1470.0,
                      white: float = 3e-4, ar_phi: float = 0.9, ar_sigma: float = 1e-4,
                      depth: float = 1e-4, pmin: float = 0.2, pmax: float = 1.0,
                      dur_h: tuple = (0.5, 2.0), t0: float = 0.0,
                      gap_d: tuple = (1.0, 5.0)) -> Curve:
    """Kepler-long-shaped curve: 65,000 samples over 1,470 d at 29.4-min cadence.

    About 10% of the 72,000 cadences are cut in gaps of 1-5 d; noise is white
    (sigma 3e-4) plus AR(1) red noise (phi 0.9, innovation sigma 1e-4,
    started from its stationary law over the full cadence grid); one box
    transit with P log-uniform in [0.2, 1] d, depth 1e-4, duration
    U(0.5, 2) h and a random epoch.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ncad = int(round(span_d / CADENCE_D))
    t = np.arange(ncad, dtype=np.float64) * CADENCE_D
    red = np.empty(ncad)
    innov = rng.normal(0.0, ar_sigma, ncad)
    red[0] = rng.normal(0.0, ar_sigma / np.sqrt(1.0 - ar_phi ** 2))
    for j in range(1, ncad):
        red[j] = ar_phi * red[j - 1] + innov[j]
    wn = rng.normal(0.0, white, ncad)
    period = float(np.exp(rng.uniform(np.log(pmin), np.log(pmax))))
    dur = rng.uniform(dur_h[0], dur_h[1]) / 24.0
    epoch = rng.uniform(0.0, period)
    f = 1.0 + wn + red
    inb = box_mask(t, period, epoch, dur)
    f[inb] -= depth
    keep = _drop_gaps(rng, ncad, n_keep, span_d, gap_d[0], gap_d[1])
    return Curve(t[keep] + t0, f[keep].astype(np.float32),
                 dict(period=period, epoch=epoch + t0, duration=dur, depth=depth,
                      n_in=int(inb[keep].sum())))


def trended_curve(seed: int = 2002, n: int = 12000, cadence: float = 0.020428, sigma: float = 2e-4,
                  n_gaps: int = 3, n_jumps: int = 1, n_outliers: int = 12, period: float = 3.7,
                  depth: float = 3e-3, duration: float = 0.15):
    """A raw (undetrended) Kepler-like curve for the pre-processing (Sec. 2.2):
    a slow multiplicative trend (a few sinusoids of 2-20 d), white noise,
    `n_gaps` gaps of 1-3 d, `n_jumps` flux steps of 5-10 % lasting to the
    next gap or the end, `n_outliers` single-cadence spikes of 8-20 sigma and
    a box transit whose samples are flagged as known. Returns (t f64, flux f32,
    transit mask bool)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = cadence * np.arange(n, dtype=np.float64)
    for _ in range(n_gaps):
        at = rng.integers(n // 10, 9 * n // 10)
        t[at:] += rng.uniform(1.0, 3.0)
    trend = np.ones(n)
    for _ in range(3):
        trend += rng.uniform(1e-3, 6e-3) * np.sin(2 * np.pi * t / rng.uniform(2.0, 20.0) + rng.uniform(0, 6.3))
    f = trend + rng.normal(0.0, sigma, n)
    for _ in range(n_jumps):
        at = rng.integers(n // 5, 4 * n // 5)
        f[at:] *= 1.0 + rng.uniform(0.05, 0.10) * rng.choice([-1.0, 1.0])
    epoch = rng.uniform(0, period)
    tr = box_mask(t, period, epoch, duration)
    f[tr] *= 1.0 - depth
    idx = rng.choice(np.flatnonzero(~tr), size=n_outliers, replace=False)
    f[idx] += rng.uniform(8.0, 20.0, n_outliers) * sigma * rng.choice([-1.0, 1.0], n_outliers)
    return t, f.astype(np.float32), tr


def multi_star(seed: int = 1005, n_stars: int = 512, nmin: int = 20000, nmax: int = 70000,
               n_transit: int = 51, alpha: tuple = (7.0, 20.0), pmin: float = 0.2,
               pmax: float = 1.0) -> list:
    """Stars of uneven length for the batched survey.

    Lengths U{nmin..nmax}; gaps as in ``kepler_long_curve`` on a baseline of
    n/0.9 cadences; white noise with sigma log-uniform in [1e-4, 1e-3];
    ``n_transit`` stars (a seeded choice) carry a box whose depth gives SNR
    alpha ~ U(alpha) by Eq. 2.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    has = np.zeros(n_stars, dtype=bool)
    has[rng.choice(n_stars, size=min(n_transit, n_stars), replace=False)] = True
    stars = []
    for s in range(n_stars):
        n = int(rng.integers(nmin, nmax + 1))
        ncad = int(np.ceil(n / 0.9))
        span = ncad * CADENCE_D
        t = np.arange(ncad, dtype=np.float64) * CADENCE_D
        sig = float(np.exp(rng.uniform(np.log(1e-4), np.log(1e-3))))
        f = 1.0 + rng.normal(0.0, sig, ncad)
        truth = dict(sigma=sig, has_transit=bool(has[s]))
        if has[s]:
            period = float(np.exp(rng.uniform(np.log(pmin), np.log(pmax))))
            dur = rng.uniform(0.5, 2.0) / 24.0
            epoch = rng.uniform(0.0, period)
            a = rng.uniform(*alpha)
            d = depth_for_snr(a, sig, n, dur, period)
            f[box_mask(t, period, epoch, dur)] -= d
            truth.update(period=period, epoch=epoch, duration=dur, depth=d, alpha=a)
        keep = _drop_gaps(rng, ncad, n, span, 1.0, 5.0)
        stars.append(Curve(t[keep], f[keep].astype(np.float32), truth))
    return stars


def training_curve(rng: np.random.Generator, n: int = 4000, positive: bool = True,
                   alpha_range: tuple = (3.0, 20.0), depth_range: tuple = (1e-5, 1e-3),
                   pmin: float = 0.2, pmax: float = 1.0, dur_h: tuple = (0.5, 3.0)) -> Curve:
    """One curve for the learned scorer's data set (Sec. 2.6-2.7 recipe).

    sigma ~ log-uniform [1e-4, 1e-3]; positives carry a trapezoid with
    P log-uniform in [pmin, pmax], duration U(dur_h) hours, base ratio
    r ~ U(0, 1), SNR alpha ~ U(alpha_range) turned into a depth by Eq. 2,
    redrawn until the depth lies in ``depth_range``.
    """
    t = np.arange(n, dtype=np.float64) * CADENCE_D
    sig = float(np.exp(rng.uniform(np.log(1e-4), np.log(1e-3))))
    f = 1.0 + rng.normal(0.0, sig, n)
    truth = dict(sigma=sig, label=int(positive))
    if positive:
        for _ in range(1000):
            period = float(np.exp(rng.uniform(np.log(pmin), np.log(pmax))))
            dur = rng.uniform(*dur_h) / 24.0
            a = rng.uniform(*alpha_range)
            d = depth_for_snr(a, sig, n, dur, period)
            if depth_range[0] <= d <= depth_range[1]:
                break
        epoch = rng.uniform(0.0, period)
        r = rng.uniform(0.0, 1.0)
        f = f + trapezoid(t, period, epoch, dur, d, r)
        truth.update(period=period, epoch=epoch, duration=dur, depth=d, alpha=a, ratio=r)
    return Curve(t, f.astype(np.float32), truth)


def direct_folds(rng: np.random.Generator, m: int, alpha_range: tuple = (6.0, 10.0),
                 transit: bool = True, nbins: int = 256, pmin: float = 0.2, pmax: float = 1.0,
                 dur_h: tuple = (0.5, 3.0)):
    """Folded curves made directly as length-``nbins`` vectors (Sec. 2.7):
    one unit of Gaussian noise per bin and, when ``transit``, a trapezoid dip
    of SNR alpha ~ U(alpha_range). The dip's width at half depth is the
    phase fraction q = duration / P (P log-uniform [pmin, pmax], duration
    U(dur_h) hours, q at most 1/2), its depth alpha / sqrt(nbins q) (Eq. 2 with
    one noise unit per bin and nbins q bins in transit), its base ratio
    r ~ U(0, 1) and its centre uniform in phase; the profile is evaluated at
    the bin centres. Returns (vectors f32 [m, nbins], alpha [m])."""
    v = rng.standard_normal((m, nbins))
    alpha = np.zeros(m)
    if transit and m:
        per = np.exp(rng.uniform(np.log(pmin), np.log(pmax), m))
        q = np.minimum(rng.uniform(dur_h[0], dur_h[1], m) / 24.0 / per, 0.5)
        alpha = rng.uniform(alpha_range[0], alpha_range[1], m)
        depth = alpha / np.sqrt(nbins * q)
        r = rng.uniform(0.0, 1.0, m)
        centre = rng.uniform(0.0, 1.0, m)
        x = (np.arange(nbins) + 0.5) / nbins
        dist = np.abs(np.mod(x[None, :] - centre[:, None] + 0.5, 1.0) - 0.5)
        long_b = (2.0 * q / (1.0 + r))[:, None]
        short_b = r[:, None] * long_b
        ramp = depth[:, None] * (0.5 * long_b - dist) / np.maximum(0.5 * (long_b - short_b), 1e-300)
        prof = np.where(dist <= 0.5 * short_b, depth[:, None], np.where(dist < 0.5 * long_b, ramp, 0.0))
        v = v - prof
    return v.astype(np.float32), alpha


# Learned-scorer parameter layout (canonical): per conv block l weight
# [Cout][Cin][5] then bias; fc weights [out][in] then bias.
CNN_LAYERS = [("conv", 1, 16), ("conv", 16, 32), ("conv", 32, 64), ("conv", 64, 64),
              ("fc", 1024, 256), ("fc", 256, 64), ("fc", 64, 1)]


def cnn_param_shapes():
    shapes = []
    for kind, cin, cout in CNN_LAYERS:
        shapes.append((cout, cin, 5) if kind == "conv" else (cout, cin))
        shapes.append((cout,))
    return shapes


def cnn_init(seed: int = 1003) -> np.ndarray:
    """He-normal initial weights (std sqrt(2 / fan_in)), zero biases, float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for kind, cin, cout in CNN_LAYERS:
        fan_in = cin * 5 if kind == "conv" else cin
        shape = (cout, cin, 5) if kind == "conv" else (cout, cin)
        parts.append(rng.normal(0.0, np.sqrt(2.0 / fan_in), size=shape).ravel())
        parts.append(np.zeros(cout))
    return np.concatenate(parts)


# Parameter tensors of the paper's own network, in its flat order: (name, shape, fan-in).
PNET_LAYERS = [("w1", (128, 1, 3, 3), 9), ("b1", (128,), 0), ("w2", (256, 128, 3, 3), 1152),
               ("b2", (256,), 0), ("w3", (128, 1, 5, 5), 25), ("b3", (128,), 0),
               ("w4", (256, 128, 5, 5), 3200), ("b4", (256,), 0), ("w5", (128, 256), 256),
               ("b5", (128,), 0), ("w6", (128,), 128), ("b6", (1,), 0)]


def pnet_init(seed: int = 1003) -> np.ndarray:
    """He-normal initial weights of the paper's network (std sqrt(2 / fan_in)),
    zero biases, float64, flat."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for _, shape, fan_in in PNET_LAYERS:
        n = int(np.prod(shape))
        parts.append(rng.normal(0.0, np.sqrt(2.0 / fan_in), size=n) if fan_in else np.zeros(n))
    return np.concatenate(parts)


def training_params(rng: np.random.Generator, m: int, n: int = 4000,
                    alpha_range: tuple = (3.0, 20.0), depth_range: tuple = (1e-5, 1e-3),
                    pmin: float = 0.2, pmax: float = 1.0, dur_h: tuple = (0.5, 3.0)) -> dict:
    """Per-curve parameters of ``m`` transit curves, vectorised (Sec. 2.6-2.7
    recipe): sigma log-uniform [1e-4, 1e-3]; P log-uniform [pmin, pmax];
    duration U(dur_h) hours; SNR alpha ~ U(alpha_range) turned into a depth by
    Eq. 2 and redrawn until it lies in ``depth_range``; trapezoid base ratio
    r ~ U(0, 1); epoch U[0, P)."""
    out = {k: np.empty(m) for k in ("sigma", "period", "duration", "alpha", "depth", "ratio", "epoch")}
    todo = np.arange(m)
    while todo.size:
        k = todo.size
        sig = np.exp(rng.uniform(np.log(1e-4), np.log(1e-3), k))
        per = np.exp(rng.uniform(np.log(pmin), np.log(pmax), k))
        dur = rng.uniform(dur_h[0], dur_h[1], k) / 24.0
        alp = rng.uniform(alpha_range[0], alpha_range[1], k)
        dep = alp * sig / np.sqrt(n * dur / per)
        ok = (dep >= depth_range[0]) & (dep <= depth_range[1])
        idx = todo[ok]
        for key, val in (("sigma", sig), ("period", per), ("duration", dur), ("alpha", alp), ("depth", dep)):
            out[key][idx] = val[ok]
        todo = todo[~ok]
    out["ratio"] = rng.uniform(0.0, 1.0, m)
    out["epoch"] = rng.uniform(0.0, 1.0, m) * out["period"]
    return out


def training_flux_torch(params: dict, positive: np.ndarray, noise_sigma: np.ndarray, n: int,
                        seed: int, device="cuda"):
    """Flux of a set of uniform-cadence curves (N = n) built on the GPU with a
    seeded torch generator: 1 + N(0, sigma) plus, where ``positive``, the
    trapezoid of ``params`` (same definition as ``trapezoid``). Returns
    (t f64[n] numpy, flux f32[m, n] torch tensor)."""
    import torch
    m = positive.size
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    t = np.arange(n, dtype=np.float64) * CADENCE_D
    tt = torch.tensor(t, dtype=torch.float64, device=device)[None, :]
    f = torch.randn((m, n), generator=g, dtype=torch.float64, device=device)
    f = 1.0 + f * torch.tensor(noise_sigma, dtype=torch.float64, device=device)[:, None]
    pos = np.nonzero(positive)[0]
    if pos.size:
        P = torch.tensor(params["period"][pos], dtype=torch.float64, device=device)[:, None]
        E = torch.tensor(params["epoch"][pos], dtype=torch.float64, device=device)[:, None]
        L = torch.tensor(params["duration"][pos], dtype=torch.float64, device=device)[:, None]
        D = torch.tensor(params["depth"][pos], dtype=torch.float64, device=device)[:, None]
        R = torch.tensor(params["ratio"][pos], dtype=torch.float64, device=device)[:, None]
        long_b = 2.0 * L / (1.0 + R)
        short_b = R * long_b
        x = torch.abs(torch.remainder(tt - E + 0.5 * P, P) - 0.5 * P)
        ramp = D * (0.5 * long_b - x) / torch.clamp(0.5 * (long_b - short_b), min=1e-300)
        prof = torch.where(x <= 0.5 * short_b, D, torch.where(x < 0.5 * long_b, ramp, torch.zeros_like(x)))
        f[torch.tensor(pos, device=device)] -= prof
    return t, f.to(torch.float32)
