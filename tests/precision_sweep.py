"""Precision sweep of the hot path against the FP64 oracle.

Fold sums: exact fixed-point integers (the default), FP32 plain and FP32
TwoSum-compensated float atomics; errors of bin means and of the box-SNR.
Learned scorer: FP32, bf16 and FP8 E4M3 (calibrated) inference; errors of the
logits against the FP64 network on the same normalised folds. Every error is
reported per result, on the Kepler-long curve (65,000 samples) at a seeded
sample of the 2,000,000-period grid plus the best periods.

This is test infrastructure (it runs the oracle): python tests/precision_sweep.py

    python tests/precision_sweep.py [--periods 20000] [--cnn-folds 2000]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2312_02063_amd import synth  # noqa: E402
from paper_2312_02063_amd._lib import CNN_BF16, CNN_FP32, Cnn, Plan  # noqa: E402

NBINS = 256


def _stats(err):
    err = np.abs(np.asarray(err, np.float64))
    err = err[np.isfinite(err)]
    return {"max": float(err.max()) if err.size else None,
            "rms": float(np.sqrt(np.mean(err ** 2))) if err.size else None}


def run(n_periods: int = 20000, n_top: int = 100, cnn_folds: int = 2000, params=None, seed: int = 1004):
    import torch

    import oracle   # the FP64 reference this sweep measures against
    dev = torch.device("cuda", 0)
    c = synth.kepler_long_curve(seed=1002)
    grid = synth.freq_grid(1.0, 5.0, 2_000_000)
    rng = np.random.Generator(np.random.PCG64(seed))
    plan = Plan(0)
    t = torch.tensor(c.t, dtype=torch.float64, device=dev)
    f = torch.tensor(c.flux, dtype=torch.float32, device=dev)
    # the best periods of the full grid by the box-SNR computed on the GPU, plus a seeded sample
    snr_all = plan.fold_score(t, f, torch.tensor(grid, dtype=torch.float64, device=dev), NBINS)[0]
    top = torch.topk(snr_all, n_top).indices.cpu().numpy()
    idx = np.unique(np.concatenate([rng.choice(grid.size, n_periods, replace=False), top]))
    periods = grid[idx]
    pp = torch.tensor(periods, dtype=torch.float64, device=dev)

    mean, sigma, _ = oracle.curve_stats(c.t, c.flux)
    osums, dsums, ocounts = oracle.fold(c.t, c.flux, periods, NBINS, ref=mean, nthreads=16)
    osnr, _, _, _ = oracle.score(ocounts, dsums, sigma)
    out = {"curve": "kepler-long 65,000 samples", "periods": int(periods.size), "nbins": NBINS,
           "sigma": sigma, "fold": {}, "cnn": {}}

    def fold_modes(flux_np, flux_dev, osums_, ocounts_, osnr_, sigma_):
        res = {}
        okm = ocounts_ > 0
        om = oracle.means(osums_, ocounts_)
        plan.prepare(t, flux_dev)
        modes = {"int64_exact": None, "fp32_plain": False, "fp32_twosum": True}
        for name, comp in modes.items():
            if comp is None:
                sums, counts, means = plan.fold_prepared(pp, NBINS)
            else:
                sums, counts, means = plan.fold_f32_prepared(pp, NBINS, comp)
            snr = plan.score(sums, counts, sigma_)[0]
            torch.cuda.synchronize()
            gm = means.cpu().numpy()
            res[name] = {
                "counts_bit_exact": bool(np.array_equal(counts.cpu().numpy(), ocounts_)),
                "bin_mean_abs_error": _stats(gm[okm] - om[okm]),
                "bin_mean_error_over_sigma": _stats((gm[okm] - om[okm]) / sigma_),
                "snr_rel_error": _stats((snr.cpu().numpy().astype(np.float64) - osnr_)
                                        / np.maximum(np.abs(osnr_), 1.0)),
            }
        return res

    out["fold"] = fold_modes(c.flux, f, osums, ocounts, osnr, sigma)
    # the same curve on a strongly variable star (a 30% sinusoid of period
    # 3.7 d): flux deviations now span more than 2^24 flux ulps, so FP32 sums
    # round and compensation matters
    fv = (c.flux.astype(np.float64) * (1.0 + 0.3 * np.sin(2 * np.pi * c.t / 3.7))).astype(np.float32)
    mean_v, sigma_v, _ = oracle.curve_stats(c.t, fv)
    osv, dsv, ocv = oracle.fold(c.t, fv, periods, NBINS, ref=mean_v, nthreads=16)
    osnr_v, _, _, _ = oracle.score(ocv, dsv, sigma_v)
    out["fold_variable_star"] = fold_modes(fv, torch.tensor(fv, dtype=torch.float32, device=dev), osv, ocv,
                                           osnr_v, sigma_v)

    if cnn_folds > 0:
        z = oracle.normalize(osums[:cnn_folds], ocounts[:cnn_folds])
        if params is None:
            params = synth.cnn_init(1003)
        zo = oracle.cnn_forward(params, z)
        xz = torch.tensor(z, dtype=torch.float32, device=dev)
        for name, prec in (("fp32", CNN_FP32), ("bf16", CNN_BF16)):
            net = Cnn(0, prec, max_batch=max(cnn_folds, 1))
            net.set_params(np.asarray(params, np.float32))
            zl = net.forward(xz).cpu().numpy()
            out["cnn"][name] = {"logit_abs_error": _stats(zl - zo),
                                "score_abs_error": _stats(1 / (1 + np.exp(-zl)) - 1 / (1 + np.exp(-zo)))}
            if prec == CNN_BF16:
                # calibrate on held-out folds of other periods of the same curve
                cal_idx = rng.choice(grid.size, min(10000, grid.size), replace=False)
                cal_p = torch.tensor(grid[cal_idx], dtype=torch.float64, device=dev)
                zc = torch.empty((cal_p.numel(), NBINS), dtype=torch.uint16, device=dev)
                plan.fold_score_prepared(cal_p, NBINS, zfold=zc)
                net2 = Cnn(0, CNN_BF16, max_batch=max(cnn_folds, zc.shape[0]))
                net2.set_params(np.asarray(params, np.float32))
                net2.calibrate_fp8(zc)
                z8 = net2.forward_fp8(xz).cpu().numpy()
                out["cnn"]["fp8_e4m3"] = {"logit_abs_error": _stats(z8 - zo),
                                          "score_abs_error": _stats(1 / (1 + np.exp(-z8)) - 1 / (1 + np.exp(-zo))),
                                          "calibration_folds": int(zc.shape[0])}
        out["cnn"]["folds"] = int(cnn_folds)
        out["cnn"]["logit_rms_fp64"] = float(np.sqrt(np.mean(zo ** 2)))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--periods", type=int, default=20000)
    ap.add_argument("--top", type=int, default=100)
    ap.add_argument("--cnn-folds", type=int, default=2000)
    ap.add_argument("--params", type=str, default="", help="trained network (.npy, FP32 canonical)")
    args = ap.parse_args()
    params = np.load(args.params).astype(np.float64) if args.params else None
    print(json.dumps(run(args.periods, args.top, args.cnn_folds, params)), flush=True)


if __name__ == "__main__":
    main()
