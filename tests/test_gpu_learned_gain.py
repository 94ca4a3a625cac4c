"""What the trained network gains over the box statistic alone (runs on an
MI355X): a reduced version of the learned-scorer study. Train on folds the
fold kernel makes from injected transits and from noise, mine hard
negatives once, then compare, on held-out curves each searched over a
1,000-period grid, the recall at 1% false positives and the AUC of the best
network score per curve with those of the best box-SNR per curve. Both
numbers are printed; the network must not lose to the box statistic by more
than the sampling noise of a 3,000-curve evaluation."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_network_not_worse_than_box_snr():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_02063_amd import CNN_BF16, Cnn, Plan, learn, synth
    print("[gpu-case] learned gain: train 60k+60k, 1 hard round, eval 3k+3k x 1000", flush=True)
    periods = learn.grid(1000)
    plan = Plan(0)
    z, y, _ = learn.make_training_set(plan, 60000, 60000, seed=1103, periods=periods)
    net = Cnn(0, CNN_BF16, max_batch=65536)
    net.set_params(synth.cnn_init(1103).astype(np.float32))
    learn.train(net, z, y, epochs=4, batch=256, lr=1e-3)
    hard = learn.mine_hard_negatives(plan, net, 6000, 4, seed=2100, periods=periods)
    zp, yp, _ = learn.make_training_set(plan, hard.shape[0], 0, seed=3100, periods=periods)
    z = torch.cat([z, hard, zp])
    y = torch.cat([y, torch.zeros(hard.shape[0], dtype=torch.float32, device=z.device), yp])
    learn.train(net, z, y, epochs=2, batch=256, lr=5e-4, seed=12)
    ev = learn.evaluate(plan, net, 3000, 3000, seed=1113, periods=periods)
    res = learn.summarize(ev)
    c, b = res["cnn"], res["box"]
    print(f"recall@1%FPR cnn {c['recall_at_1pct_fpr']:.4f} box {b['recall_at_1pct_fpr']:.4f}; "
          f"AUC cnn {c['auc']:.4f} box {b['auc']:.4f}", flush=True)
    sys.stdout.flush()
    # 3,000 positives: one standard error of a recall near 0.75 is ~0.008
    assert c["recall_at_1pct_fpr"] >= b["recall_at_1pct_fpr"] - 0.025
    assert c["auc"] >= b["auc"] - 0.01
