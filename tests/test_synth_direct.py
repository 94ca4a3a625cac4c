"""The directly made training vectors (folded curves simulated as length-256
vectors): noise statistics, the dip's SNR by Eq. 2, the labels of the SNR
cut-off."""
import numpy as np

from paper_2312_02063_amd import synth


def _pair(seed, m, alpha_range=(6.0, 10.0)):
    # the noise is drawn first, so the same seed gives the same noise with and
    # without the dip: their difference is the dip alone
    noise, _ = synth.direct_folds(np.random.default_rng(seed), m, transit=False)
    v, alpha = synth.direct_folds(np.random.default_rng(seed), m, alpha_range)
    return noise, noise.astype(np.float64) - v, alpha


def test_noise_is_unit_gaussian():
    noise, _ = synth.direct_folds(np.random.default_rng(1), 400, transit=False)
    assert noise.shape == (400, 256) and noise.dtype == np.float32
    assert abs(noise.mean()) < 0.01 and abs(noise.std() - 1.0) < 0.01


def test_dip_depth_follows_eq2():
    _, dip, alpha = _pair(2, 300)
    assert (dip >= -1e-6).all()                      # a dip only lowers the flux
    assert ((alpha >= 6.0) & (alpha < 10.0)).all()
    depth = dip.max(axis=1)
    width = (dip >= 0.5 * depth[:, None]).sum(axis=1)   # bins at or above half depth
    ok = width >= 8                                  # short dips are too coarse to measure
    est = depth[ok] * np.sqrt(width[ok])
    assert ok.sum() > 100
    assert np.median(np.abs(est / alpha[ok] - 1.0)) < 0.1


def test_dip_wraps_in_phase():
    # centres near the ends of the phase put part of the dip at the other end
    _, dip, _ = _pair(3, 400)
    both = (dip[:, 0] > 0) & (dip[:, -1] > 0)
    assert both.any()


def test_direct_training_set_labels_and_normalisation():
    import torch
    from paper_2312_02063_amd.learn import make_direct_set
    z, y, alpha = make_direct_set(60, 40, seed=5, device="cpu")
    assert z.shape == (100, 256) and z.dtype == torch.uint16
    y = y.numpy()
    assert (y[:60] == 1).all() and (y[60:] == 0).all()
    assert (alpha[60:80] == 0).all()                  # pure noise
    assert ((alpha[80:] >= 1.0) & (alpha[80:] < 5.0)).all()   # weak dips, below the cut
    x = z.view(torch.bfloat16).float().numpy()
    assert np.abs(x.mean(axis=1)).max() < 0.02
    assert np.abs(x.std(axis=1) - 1.0).max() < 0.02
