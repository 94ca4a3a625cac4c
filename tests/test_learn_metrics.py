"""CPU checks of the evaluation metrics used for the learned scorer."""
import numpy as np
import pytest

from paper_2312_02063_amd import learn


def test_recall_at_fpr_exact_threshold():
    neg = np.arange(100, dtype=float)           # 1% FPR lets through only 99
    pos = np.array([98.5, 99.5, 100.0, 50.0])
    stat = np.concatenate([pos, neg])
    label = np.concatenate([np.ones(4), np.zeros(100)])
    r, thr = learn.recall_at_fpr(stat, label, fpr=0.01)
    assert thr == 98.0
    assert r == pytest.approx(3 / 4)


def test_auc_against_pairwise_count():
    rng = np.random.default_rng(0)
    pos = rng.normal(1.0, 1.0, 200)
    neg = rng.normal(0.0, 1.0, 300)
    pos[:10] = neg[:10]                           # some ties
    stat = np.concatenate([pos, neg])
    label = np.concatenate([np.ones(200), np.zeros(300)])
    pairs = (pos[:, None] > neg[None, :]).mean() + 0.5 * (pos[:, None] == neg[None, :]).mean()
    assert learn.auc(stat, label) == pytest.approx(pairs, rel=1e-12)


def test_training_params_ranges():
    rng = np.random.default_rng(1)
    from paper_2312_02063_amd import synth
    prm = synth.training_params(rng, 5000)
    assert (prm["depth"] >= 1e-5).all() and (prm["depth"] <= 1e-3).all()
    assert (prm["alpha"] >= 3).all() and (prm["alpha"] <= 20).all()
    # Eq. 2 holds for every draw
    np.testing.assert_allclose(prm["alpha"], prm["depth"] / prm["sigma"] *
                               np.sqrt(4000 * prm["duration"] / prm["period"]), rtol=1e-12)
