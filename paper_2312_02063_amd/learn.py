"""Train and evaluate the learned scorer on folds the fold kernel produces.

The paper trains its CNN on synthetic folded curves and judges it, against a
BLS statistic, by the maximum score over trial periods of each light curve
(Sec. 2.5-2.7, Sec. 3.2). Here: training curves (C1-shaped: 4,000 samples at
29.4 min) with trapezoid transits at SNR 3-20 and curves without, folded by
the batch kernel at the grid period nearest the injected one (positives) or
at a random grid period (negatives), 256 bins, normalised to bfloat16
z-scores by the same kernel; the network is trained with Adam on the GPU by
the library's own forward/backward kernels. Evaluation folds held-out curves
over the whole trial grid and compares, at a 1% false-positive rate, the
recall of the best CNN score per curve with that of the best box-SNR per curve
(the box statistic is also the fallback scorer when no network is given).

The paper's own training set is also available (``--data direct``, Sec. 2.7):
vectors of length 256 made directly, noise plus a trapezoid at SNR 6-10 for
positives, pure noise and weak dips labelled by the SNR cut-off 5 for
negatives. ``--auc-vs-periods`` repeats the evaluation over several trial-grid
sizes (Sec. 3.2: detection quality against the number of trial periods).

    python -m paper_2312_02063_amd.learn --train 200000 --eval 10000 --epochs 4
    python -m paper_2312_02063_amd.learn --data direct --train 1000000 --eval 2000 \
        --auc-vs-periods 100,1000,10000
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import synth
from ._lib import CNN_BF16, Cnn, Plan

N_SAMPLES = 4000
NBINS = 256


def grid(k: int = 1000) -> np.ndarray:
    """Trial periods 0.2-1.0 d, uniform in frequency."""
    return synth.freq_grid(1.0, 5.0, k)


def _fold_chunk(plan, t, flux, periods_per_curve, k_per_curve, want_score=False):
    """Fold m curves (same times t, flux [m, n] on the GPU) each at its own
    k periods (periods_per_curve: f64 [m * k]); returns zfold [m*k, 256] and,
    if asked, the box-SNR [m*k]."""
    import torch
    m, n = flux.shape
    so = np.arange(m + 1, dtype=np.int64) * n
    po = np.arange(m + 1, dtype=np.int64) * k_per_curve
    plan.batch_setup(so, po)
    tt = torch.tensor(t, dtype=torch.float64, device=flux.device).repeat(m)
    pp = torch.as_tensor(periods_per_curve, dtype=torch.float64, device=flux.device)
    z = torch.empty((m * k_per_curve, NBINS), dtype=torch.uint16, device=flux.device)
    snr, start, width, depth = plan.batch_fold_score(tt, flux.reshape(-1).contiguous(), pp, NBINS,
                                                     zfold=z)
    return z, (snr if want_score else None)


def make_training_set(plan, n_pos: int, n_neg: int, seed: int, periods: np.ndarray,
                      chunk: int = 20000, snr_cut: float = 0.0):
    """Kernel-made training folds: (z uint16 [N, 256], labels f32 [N], alpha [N]).

    snr_cut > 0 follows the paper's labelling (Sec. 2.7): injections with SNR
    below the cut are labelled 0, so the network learns to tell weak
    fluctuations from significant transits."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    zs, ys, alphas = [], [], []
    freqs = 1.0 / periods
    for label, count in ((1, n_pos), (0, n_neg)):
        done = 0
        while done < count:
            m = min(chunk, count - done)
            if label:
                prm = synth.training_params(rng, m, n=N_SAMPLES)
                sig = prm["sigma"]
                fold_p = periods[np.abs(freqs[None, :] - 1.0 / prm["period"][:, None]).argmin(axis=1)]
                alpha = prm["alpha"]
            else:
                prm = None
                sig = np.exp(rng.uniform(np.log(1e-4), np.log(1e-3), m))
                fold_p = periods[rng.integers(0, periods.size, m)]
                alpha = np.zeros(m)
            t, flux = synth.training_flux_torch(prm or {}, np.full(m, bool(label)), sig, N_SAMPLES,
                                                seed=int(rng.integers(1 << 62)))
            z, _ = _fold_chunk(plan, t, flux, fold_p, 1)
            zs.append(z)
            lab = np.full(m, float(label))
            if label and snr_cut > 0:
                lab[alpha < snr_cut] = 0.0
            ys.append(torch.tensor(lab, dtype=torch.float32, device=z.device))
            alphas.append(alpha)
            done += m
    return torch.cat(zs), torch.cat(ys), np.concatenate(alphas)


def make_direct_set(n_pos: int, n_neg: int, seed: int, snr_cut: float = 5.0,
                    weak_range: tuple = (1.0, 5.0), chunk: int = 100000, device="cuda"):
    """Training vectors made directly rather than folded (Sec. 2.7): positives
    are noise plus a trapezoid at SNR 6-10; negatives are half pure noise and
    half noise plus a weak trapezoid (SNR in ``weak_range``), labelled by the
    SNR cut (at or above: 1, below: 0). Each vector is z-scored over its bins
    (ddof 0), as the fold kernel normalises folds, and kept as bf16 bits.
    Returns (z uint16 [N, 256], labels f32 [N], alpha [N])."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    zs, ys, alphas = [], [], []
    parts = ((n_pos, True, (6.0, 10.0)), (n_neg - n_neg // 2, False, (0.0, 0.0)),
             (n_neg // 2, True, weak_range))
    for count, transit, arange_ in parts:
        done = 0
        while done < count:
            m = min(chunk, count - done)
            v, a = synth.direct_folds(rng, m, arange_, transit=transit, nbins=NBINS)
            x = torch.tensor(v, device=device)
            mu = x.mean(dim=1, keepdim=True)
            sd = x.std(dim=1, unbiased=False, keepdim=True)
            z = torch.where(sd > 0, (x - mu) / sd, torch.zeros_like(x))
            zs.append(z.to(torch.bfloat16).view(torch.uint16))
            lab = (a >= snr_cut).astype(np.float32) if transit else np.zeros(m, np.float32)
            ys.append(torch.tensor(lab, device=device))
            alphas.append(a)
            done += m
    return torch.cat(zs), torch.cat(ys), np.concatenate(alphas)


def train(net, z, labels, epochs: int = 4, batch: int = 256, lr: float = 1e-3, seed: int = 7,
          log=None, graph: bool = True):
    """Adam on mini-batches of the kernel folds; returns the mean loss per epoch.
    With graph=True each step is one replay of a captured training step (the
    batch is gathered into the captured buffers first)."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    n = z.shape[0]
    hist = []
    xbuf = torch.empty((batch, z.shape[1]), dtype=z.dtype, device=z.device)
    ybuf = torch.empty(batch, dtype=torch.float32, device=z.device)
    if graph and n >= batch:
        net.train_capture(xbuf, ybuf, lr)
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(n), device=z.device)
        acc = torch.zeros(1, dtype=torch.float32, device=z.device)
        steps = 0
        for i in range(0, n - batch + 1, batch):
            idx = perm[i:i + batch]
            torch.index_select(z, 0, idx, out=xbuf)
            torch.index_select(labels, 0, idx, out=ybuf)
            acc += net.train_replay() if graph else net.train_step(xbuf, ybuf, lr)
            steps += 1
        tot = (acc / max(steps, 1)).item() if steps else float("nan")
        hist.append(tot)
        if log:
            log(f"epoch {ep}: mean loss {tot:.5f}")
    return hist


def mine_hard_negatives(plan, net, n_curves: int, per_curve: int, seed: int, periods: np.ndarray,
                        chunk: int = 250, cnn_batch: int = 65536):
    """Fold fresh no-transit curves over the whole grid, score every fold and
    keep each curve's `per_curve` best-scoring folds (per-curve best-K on the
    GPU): the folds the detection statistic's false positives come from."""
    import torch
    from ._lib import topk
    rng = np.random.Generator(np.random.PCG64(seed))
    k = periods.size
    out = []
    done = 0
    while done < n_curves:
        m = min(chunk, n_curves - done)
        sig = np.exp(rng.uniform(np.log(1e-4), np.log(1e-3), m))
        t, flux = synth.training_flux_torch({}, np.zeros(m, bool), sig, N_SAMPLES,
                                            seed=int(rng.integers(1 << 62)))
        z, _ = _fold_chunk(plan, t, flux, np.tile(periods, m), k)
        logits = torch.empty(m * k, dtype=torch.float32, device=z.device)
        for i in range(0, m * k, cnn_batch):
            net.forward(z[i:i + cnn_batch], out=logits[i:i + cnn_batch])
        _, idx = topk(logits.view(m, k), per_curve)
        rows = (idx + torch.arange(m, device=z.device)[:, None] * k).reshape(-1)
        out.append(z.index_select(0, rows))
        done += m
    return torch.cat(out)


def evaluate(plan, net, n_pos: int, n_neg: int, seed: int, periods: np.ndarray, chunk: int = 250,
             cnn_batch: int = 65536, log=None, judge_snr: float = 4.0):
    """Per held-out curve: best CNN logit and best box-SNR over all periods."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    k = periods.size
    out = {"cnn": [], "box": [], "judged": [], "label": [], "alpha": []}
    for label, count in ((1, n_pos), (0, n_neg)):
        done = 0
        while done < count:
            m = min(chunk, count - done)
            if label:
                prm = synth.training_params(rng, m, n=N_SAMPLES)
                sig, alpha = prm["sigma"], prm["alpha"]
            else:
                prm = None
                sig = np.exp(rng.uniform(np.log(1e-4), np.log(1e-3), m))
                alpha = np.zeros(m)
            t, flux = synth.training_flux_torch(prm or {}, np.full(m, bool(label)), sig, N_SAMPLES,
                                                seed=int(rng.integers(1 << 62)))
            z, snr = _fold_chunk(plan, t, flux, np.tile(periods, m), k, want_score=True)
            box = snr.view(m, k).max(dim=1).values
            if net is not None:
                logits = torch.empty(m * k, dtype=torch.float32, device=z.device)
                for i in range(0, m * k, cnn_batch):
                    net.forward(z[i:i + cnn_batch], out=logits[i:i + cnn_batch])
                lg = logits.view(m, k)
                cnn = lg.max(dim=1).values
                # the CNN's best period among those where the box statistic
                # sees a dip of at least judge_snr (box-SNR judging detections)
                judged = torch.where(snr.view(m, k) >= judge_snr, lg, torch.full_like(lg, -1e9)).max(dim=1).values
            else:
                cnn = box
                judged = box
            out["cnn"].append(cnn.cpu().numpy())
            out["box"].append(box.cpu().numpy())
            out["judged"].append(judged.cpu().numpy())
            out["label"].append(np.full(m, label))
            out["alpha"].append(alpha)
            done += m
            if log:
                log(f"eval label={label}: {done}/{count}")
    return {key: np.concatenate(v) for key, v in out.items()}


def train_scorer(plan, periods: np.ndarray, n_train: int = 400000, epochs: int = 8,
                 hard_rounds: int = 4, hard_curves: int = 30000, hard_per_curve: int = 4,
                 hard_epochs: int = 2, lr: float = 1e-3, batch: int = 256, snr_cut: float = 0.0,
                 seed: int = 1003, log=None):
    """The learned scorer's training recipe: n_train kernel folds of each class,
    `epochs` of Adam, then `hard_rounds` rounds of hard-negative mining (each
    adds the `hard_per_curve` best-scoring folds of `hard_curves` fresh noise
    curves searched over the whole grid, with as many fresh positives, and
    trains `hard_epochs` more at half the rate). Returns the network."""
    import torch
    z, y, _ = make_training_set(plan, n_train, n_train, seed=seed, periods=periods, snr_cut=snr_cut)
    net = Cnn(0, CNN_BF16, max_batch=65536)
    net.set_params(synth.cnn_init(seed).astype(np.float32))
    train(net, z, y, epochs, batch, lr, log=log)
    for rnd in range(hard_rounds):
        hard = mine_hard_negatives(plan, net, hard_curves, hard_per_curve, seed=2000 + rnd,
                                   periods=periods)
        zp, yp, _ = make_training_set(plan, hard.shape[0], 0, seed=3000 + rnd, periods=periods,
                                      snr_cut=snr_cut)
        z = torch.cat([z, hard, zp])
        y = torch.cat([y, torch.zeros(hard.shape[0], dtype=torch.float32, device=z.device), yp])
        if log:
            log(f"hard-negative round {rnd}: +{hard.shape[0]} negatives, +{zp.shape[0]} positives")
        train(net, z, y, hard_epochs, batch, lr * 0.5, seed=11 + rnd, log=log)
    return net


def train_pnet(plan, periods: np.ndarray, n_train: int = 100000, epochs: int = 3,
               hard_rounds: int = 1, hard_curves: int = 3000, hard_per_curve: int = 4,
               hard_epochs: int = 1, lr: float = 2e-4, batch: int = 256, dropout: float = 0.5,
               seed: int = 1003, log=None):
    """Train the paper's own network (Sec. 2.5, PNet) on kernel folds with
    dropout (keep masks drawn from a seeded generator and passed in), then
    hard-negative rounds as train_scorer does. Returns the network."""
    import torch
    from ._lib import PNet
    z, y, _ = make_training_set(plan, n_train, n_train, seed=seed, periods=periods)
    net = PNet(0, CNN_BF16, max_batch=batch)
    net.set_params(synth.pnet_init(seed).astype(np.float32))
    gen = torch.Generator(device=z.device)
    gen.manual_seed(seed)

    def run(z, y, n_ep, rate, rseed):
        rng = np.random.Generator(np.random.PCG64(rseed))
        xbuf = torch.empty((batch, z.shape[1]), dtype=z.dtype, device=z.device)
        ybuf = torch.empty(batch, dtype=torch.float32, device=z.device)
        for ep in range(n_ep):
            perm = torch.as_tensor(rng.permutation(z.shape[0]), device=z.device)
            acc, steps = torch.zeros(1, device=z.device), 0
            for i in range(0, z.shape[0] - batch + 1, batch):
                idx = perm[i:i + batch]
                torch.index_select(z, 0, idx, out=xbuf)
                torch.index_select(y, 0, idx, out=ybuf)
                keep = (torch.rand((batch, 128), generator=gen, device=z.device) >= dropout).float()
                keep /= (1.0 - dropout)
                acc += net.train_step(xbuf, ybuf, rate, keep=keep)
                steps += 1
            if log:
                log(f"pnet epoch {ep}: mean loss {(acc / max(steps, 1)).item():.5f}")

    run(z, y, epochs, lr, 7)
    for rnd in range(hard_rounds):
        hard = mine_hard_negatives(plan, net, hard_curves, hard_per_curve, seed=2000 + rnd,
                                   periods=periods, cnn_batch=batch)
        zp, yp, _ = make_training_set(plan, hard.shape[0], 0, seed=3000 + rnd, periods=periods)
        z = torch.cat([z, hard, zp])
        y = torch.cat([y, torch.zeros(hard.shape[0], dtype=torch.float32, device=z.device), yp])
        run(z, y, hard_epochs, lr * 0.5, 11 + rnd)
    return net


def compare_networks(plan, n_eval: int = 2000, periods: np.ndarray | None = None, log=None,
                     pnet_recipe: dict | None = None, cnn_recipe: dict | None = None):
    """The configured 1-D network and the paper's own 2-D network, each trained
    on kernel folds, judged with the box statistic on the same held-out curves
    (n_eval with a transit, n_eval without, each searched over the grid):
    recall at 1% false positives and AUC of each. Returns a dictionary."""
    import torch
    periods = grid(1000) if periods is None else periods
    t0 = time.time()
    cnn = train_scorer(plan, periods, log=log, **(cnn_recipe or {}))
    t1 = time.time()
    pnet = train_pnet(plan, periods, log=log, **(pnet_recipe or {}))
    torch.cuda.synchronize()
    t2 = time.time()
    ev_c = evaluate(plan, cnn, n_eval, n_eval, seed=1013, periods=periods)
    t3 = time.time()
    ev_p = evaluate(plan, pnet, n_eval, n_eval, seed=1013, periods=periods, cnn_batch=pnet.max_batch * 64)
    t4 = time.time()
    sc, sp = summarize(ev_c), summarize(ev_p)
    out = {"box": sc["box"], "cnn_1d": sc["cnn"], "cnn_1d_box_judged": sc["judged"],
           "pnet_2d": sp["cnn"], "pnet_2d_box_judged": sp["judged"],
           "seconds": {"train_cnn": t1 - t0, "train_pnet": t2 - t1, "eval_cnn": t3 - t2,
                       "eval_pnet": t4 - t3},
           "eval_curves": 2 * n_eval, "periods": int(periods.size)}
    cnn.close()
    pnet.close()
    return out


def learned_gain(plan, n_eval: int = 10000, periods: np.ndarray | None = None, log=None, **recipe):
    """What the trained network gains over the box statistic: train with
    train_scorer's recipe, then search n_eval held-out transit curves and n_eval
    noise curves over the grid and compare the best network score per curve
    with the best box-SNR per curve (recall at 1% false positives, AUC).
    Returns summarize()'s dictionary plus timings."""
    import torch
    periods = grid(1000) if periods is None else periods
    t0 = time.time()
    net = train_scorer(plan, periods, log=log, **recipe)
    torch.cuda.synchronize()
    t1 = time.time()
    ev = evaluate(plan, net, n_eval, n_eval, seed=1013, periods=periods)
    res = summarize(ev)
    res.update({"train_seconds": t1 - t0, "eval_seconds": time.time() - t1,
                "eval_curves": 2 * n_eval, "periods": int(periods.size)})
    net.close()
    return res


def auc_vs_periods(plan, net, ks, n_eval: int, seed: int = 1013, log=None):
    """Detection quality as the trial grid grows (Sec. 3.2): for each grid
    size k, the same held-out curves are folded over k periods and judged by
    their best CNN score and best box-SNR; more periods give noise more
    chances to look like a transit."""
    rows = []
    for k in ks:
        ev = evaluate(plan, net, n_eval, n_eval, seed=seed, periods=grid(int(k)))
        sm = summarize(ev)
        rows.append({"periods": int(k),
                     "cnn_auc": sm["cnn"]["auc"], "box_auc": sm["box"]["auc"],
                     "cnn_recall_at_1pct_fpr": sm["cnn"]["recall_at_1pct_fpr"],
                     "box_recall_at_1pct_fpr": sm["box"]["recall_at_1pct_fpr"]})
        if log:
            log(f"periods {k}: " + json.dumps(rows[-1]))
    return rows


def recall_at_fpr(stat, label, fpr=0.01):
    """Recall at the threshold that lets through at most `fpr` of the negatives."""
    neg = np.sort(stat[label == 0])
    pos = stat[label == 1]
    j = int(math.ceil((1.0 - fpr) * neg.size)) - 1
    thr = neg[min(max(j, 0), neg.size - 1)]
    return float((pos > thr).mean()), float(thr)


def auc(stat, label):
    """Area under the ROC curve (Mann-Whitney, ties counted half)."""
    pos = stat[label == 1]
    neg = stat[label == 0]
    allv = np.concatenate([pos, neg])
    order = allv.argsort(kind="mergesort")
    ranks = np.empty(allv.size)
    ranks[order] = np.arange(1, allv.size + 1)
    # average ranks of ties
    vals, inv, cnt = np.unique(allv, return_inverse=True, return_counts=True)
    sums = np.bincount(inv, weights=ranks)
    ranks = (sums / cnt)[inv]
    r_pos = ranks[: pos.size].sum()
    return float((r_pos - pos.size * (pos.size + 1) / 2) / (pos.size * neg.size))


def summarize(ev):
    res = {}
    for name in ("cnn", "box", "judged"):
        r, thr = recall_at_fpr(ev[name], ev["label"])
        res[name] = {"recall_at_1pct_fpr": r, "threshold": thr, "auc": auc(ev[name], ev["label"])}
        bins = [(3, 5), (5, 7), (7, 10), (10, 15), (15, 20)]
        per = {}
        for lo, hi in bins:
            sel = (ev["label"] == 1) & (ev["alpha"] >= lo) & (ev["alpha"] < hi)
            per[f"{lo}-{hi}"] = float((ev[name][sel] > thr).mean()) if sel.any() else None
        res[name]["recall_by_snr"] = per
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--train", type=int, default=200000, help="positives and negatives each")
    ap.add_argument("--eval", type=int, default=10000, help="held-out positives and negatives each")
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--periods", type=int, default=1000)
    ap.add_argument("--save", type=str, default="", help="write the trained FP32 parameters (.npy)")
    ap.add_argument("--snr-cut", type=float, default=0.0,
                    help="label injections below this SNR as negatives (the paper uses 5)")
    ap.add_argument("--hard-rounds", type=int, default=0,
                    help="rounds of hard-negative mining after the first training")
    ap.add_argument("--hard-curves", type=int, default=20000, help="no-transit curves mined per round")
    ap.add_argument("--hard-per-curve", type=int, default=4, help="best-scoring folds kept per curve")
    ap.add_argument("--hard-epochs", type=int, default=2, help="epochs after each mining round")
    ap.add_argument("--data", choices=("folds", "direct"), default="folds",
                    help="training set: kernel folds of synthetic curves, or vectors made directly "
                         "(noise + trapezoid at SNR 6-10, weak-transit and pure-noise negatives, cut 5)")
    ap.add_argument("--compare-pnet", action="store_true",
                    help="train the configured 1-D network and the paper's 2-D network and judge both "
                         "with box-SNR on the same --eval held-out curves")
    ap.add_argument("--auc-vs-periods", type=str, default="",
                    help="comma-separated grid sizes: AUC of CNN and box-SNR per size (--eval curves)")
    args = ap.parse_args()
    import torch

    def log(msg):
        print(f"[learn] {msg}", flush=True)

    periods = grid(args.periods)
    plan = Plan(0)
    if args.compare_pnet:
        res = compare_networks(plan, n_eval=args.eval, periods=periods, log=log)
        print(json.dumps(res), flush=True)
        return
    t0 = time.time()
    if args.data == "direct":
        z, y, _ = make_direct_set(args.train, args.train, seed=1003,
                                  snr_cut=args.snr_cut if args.snr_cut > 0 else 5.0)
    else:
        z, y, _ = make_training_set(plan, args.train, args.train, seed=1003, periods=periods,
                                    snr_cut=args.snr_cut)
    torch.cuda.synchronize()
    log(f"training folds {tuple(z.shape)} in {time.time() - t0:.1f} s")
    net = Cnn(0, CNN_BF16, max_batch=65536)
    net.set_params(synth.cnn_init(1003).astype(np.float32))
    t1 = time.time()
    hist = train(net, z, y, args.epochs, args.batch, args.lr, log=log)
    for rnd in range(args.hard_rounds):
        hard = mine_hard_negatives(plan, net, args.hard_curves, args.hard_per_curve,
                                   seed=2000 + rnd, periods=periods)
        # as many fresh positives as hard negatives keeps the classes balanced
        zp, yp, _ = make_training_set(plan, hard.shape[0], 0, seed=3000 + rnd, periods=periods,
                                      snr_cut=args.snr_cut)
        z = torch.cat([z, hard, zp])
        y = torch.cat([y, torch.zeros(hard.shape[0], dtype=torch.float32, device=z.device), yp])
        log(f"hard-negative round {rnd}: +{hard.shape[0]} negatives, +{zp.shape[0]} positives")
        hist += train(net, z, y, args.hard_epochs, args.batch, args.lr * 0.5, seed=11 + rnd, log=log)
    torch.cuda.synchronize()
    train_s = time.time() - t1
    del z, y
    if args.save:
        np.save(args.save, net.get_params().cpu().numpy())
    t2 = time.time()
    ev = evaluate(plan, net, args.eval, args.eval, seed=1013, periods=periods, log=None)
    eval_s = time.time() - t2
    res = summarize(ev)
    if args.auc_vs_periods:
        ks = [int(x) for x in args.auc_vs_periods.split(",") if x]
        res["auc_vs_periods"] = auc_vs_periods(plan, net, ks, args.eval, log=log)
    res.update({"data": args.data, "snr_cut": args.snr_cut, "hard_rounds": args.hard_rounds,
                "train_curves": 2 * args.train, "eval_curves": 2 * args.eval, "epochs": args.epochs,
                "loss_per_epoch": hist, "train_seconds": train_s, "eval_seconds": eval_s,
                "periods": args.periods, "folds_scored": 2 * args.eval * args.periods})
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
