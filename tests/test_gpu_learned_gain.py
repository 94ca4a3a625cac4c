"""What the trained network gains over the box statistic (runs on an
MI355X). The learned scorer is trained on folds the fold kernel makes from
injected transits and from noise (400,000 of each, then four rounds of
hard-negative mining), and judged as the paper judges its network (Sec. 3.2):
10,000 held-out transit curves and 10,000 noise curves are each searched over
a 1,000-period grid, and the best network score per curve is compared with
the best box-SNR per curve. The target: recall at 1% false positives and AUC
no worse than the box statistic's. Every step is seeded and every kernel is
deterministic, so the comparison is exact run to run."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_network_not_worse_than_box_snr():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_02063_amd import Plan, learn
    print("[gpu-case] learned gain: train 400k+400k, 4 hard rounds, eval 10k+10k x 1000", flush=True)
    plan = Plan(0)
    res = learn.learned_gain(plan, n_eval=10000)
    plan.close()
    c, b, j = res["cnn"], res["box"], res["judged"]
    print(f"recall@1%FPR cnn {c['recall_at_1pct_fpr']:.4f} box {b['recall_at_1pct_fpr']:.4f} "
          f"box-judged cnn {j['recall_at_1pct_fpr']:.4f}; AUC cnn {c['auc']:.4f} box {b['auc']:.4f}; "
          f"train {res['train_seconds']:.1f} s, eval {res['eval_seconds']:.1f} s", flush=True)
    sys.stdout.flush()
    assert c["recall_at_1pct_fpr"] >= b["recall_at_1pct_fpr"]
    assert c["auc"] >= b["auc"]
