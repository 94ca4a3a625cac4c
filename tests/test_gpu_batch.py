"""Normalised folds and the multi-curve persistent batch (runs on an MI355X).

The batch must reproduce, bit for bit, what the single-curve path gives for
each curve (same kernel body); both are checked against the oracle.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2312_02063_amd import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def plan(torch_dev):
    from paper_2312_02063_amd import Plan
    p = Plan(0)
    yield p
    p.close()


def _dev(torch, a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def bf16_to_f32(u16):
    return (u16.astype(np.uint32) << 16).view(np.float32)


def _single(torch, plan, t, f, periods, nbins, want_z=True):
    k = len(periods)
    plan.prepare(_dev(torch, t, torch.float64), _dev(torch, f, torch.float32))
    z = torch.empty((k, nbins), dtype=torch.uint16, device="cuda") if want_z else None
    out = plan.fold_score_prepared(_dev(torch, periods, torch.float64), nbins, zfold=z)
    torch.cuda.synchronize()
    res = [x.cpu().numpy() for x in out]
    return res, (z.cpu().numpy() if want_z else None)


def check_z(zg_u16, t, f, periods, nbins, label):
    sums, _, counts = oracle.fold(t, f, periods, nbins, nthreads=8)
    zo = oracle.normalize(sums, counts)
    zg = bf16_to_f32(zg_u16).astype(np.float64)
    err = np.abs(zg - zo)
    tol = 2.0 ** -8 * np.abs(zo) + 2e-3
    bad = np.argwhere(err > tol)
    assert bad.size == 0, f"{label}: z off at {bad[:5]}: {zg[tuple(bad[0])]} vs {zo[tuple(bad[0])]}"
    assert (zg[counts == 0] == 0).all()


@pytest.mark.parametrize("nbins", [16, 64, 256])
def test_normalised_fold_matches_oracle(torch_dev, plan, nbins):
    c = synth.plain_curve(1001)
    periods = synth.freq_grid(1.0, 5.0, 130)
    _say(f"zfold C1 nbins={nbins}")
    _, z = _single(torch_dev, plan, c.t, c.flux, periods, nbins)
    check_z(z, c.t, c.flux, periods, nbins, f"z-nb{nbins}")
    # sparse: many empty bins
    _say(f"zfold sparse nbins={nbins}")
    _, z = _single(torch_dev, plan, c.t[:150], c.flux[:150], periods, nbins)
    check_z(z, c.t[:150], c.flux[:150], periods, nbins, f"z-sparse-nb{nbins}")


def _batch_inputs(lengths, kcounts, seed=5):
    rng = np.random.default_rng(seed)
    ts, fs, ps = [], [], []
    for n, k in zip(lengths, kcounts):
        t = np.sort(rng.uniform(0, 1470.0 * n / 65000 + 1.0, n))
        f = (1.0 + rng.normal(0, 10 ** rng.uniform(-4, -3), n)).astype(np.float32)
        ts.append(t)
        fs.append(f)
        ps.append(1.0 / rng.uniform(1.0, 5.0, k))
    so = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    po = np.concatenate([[0], np.cumsum(kcounts)]).astype(np.int64)
    return ts, fs, ps, so, po


def test_batch_equals_single_curve_path(torch_dev, plan):
    torch = torch_dev
    lengths = [4000, 20000, 0, 1, 777, 65000, 300]
    kcounts = [130, 64, 5, 1, 0, 200, 70]
    ts, fs, ps, so, po = _batch_inputs(lengths, kcounts)
    nbins = 256
    _say(f"batch setup curves={len(lengths)} periods={po[-1]}")
    plan.batch_setup(so, po)
    t = _dev(torch, np.concatenate(ts), torch.float64)
    f = _dev(torch, np.concatenate(fs), torch.float32)
    p = _dev(torch, np.concatenate(ps), torch.float64)
    z = torch.empty((int(po[-1]), nbins), dtype=torch.uint16, device="cuda")
    _say("batch fold_score")
    out = plan.batch_fold_score(t, f, p, nbins, zfold=z)
    torch.cuda.synchronize()
    bo = [x.cpu().numpy() for x in out]
    bz = z.cpu().numpy()
    stats = plan.batch_curve_stats()
    for c in range(len(lengths)):
        a, b = po[c], po[c + 1]
        if lengths[c] > 0:
            mean, sigma, _ = oracle.curve_stats(ts[c], fs[c])
            assert stats[c]["n"] == lengths[c]
            assert stats[c]["sigma"] == pytest.approx(sigma, rel=1e-12, abs=1e-300)
        if b == a:
            continue
        _say(f"single curve {c} n={lengths[c]} k={b - a}")
        so_, sz = _single(torch, plan, ts[c], fs[c], ps[c], nbins)
        for x, y in zip(bo, so_):
            assert np.array_equal(x[a:b], y), f"curve {c}"
        assert np.array_equal(bz[a:b], sz)
        if lengths[c] >= 300:
            mean, sigma, _ = oracle.curve_stats(ts[c], fs[c])
            _, dsums, counts = oracle.fold(ts[c], fs[c], ps[c], nbins, ref=mean, nthreads=8)
            osnr, ostart, owidth, _ = oracle.score(counts, dsums, sigma)
            np.testing.assert_allclose(bo[0][a:b], osnr, rtol=1e-5, atol=1e-5)


def test_batch_graph_capture_replays(torch_dev, plan):
    torch = torch_dev
    lengths = [5000, 12000, 3000]
    kcounts = [300, 128, 65]
    ts, fs, ps, so, po = _batch_inputs(lengths, kcounts, seed=9)
    nbins = 64
    plan.batch_setup(so, po)
    t = _dev(torch, np.concatenate(ts), torch.float64)
    f = _dev(torch, np.concatenate(fs), torch.float32)
    p = _dev(torch, np.concatenate(ps), torch.float64)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        _say("batch capture")
        gout = plan.batch_capture(t, f, p, nbins)
    torch.cuda.synchronize()
    for rep in range(3):
        # eager work between replays: change the flux, run the eager batch
        f.mul_(1.0 + 1e-4 * (rep + 1)).add_(-1e-4 * (rep + 1))
        torch.cuda.synchronize()
        _say(f"eager batch rep {rep}")
        eo = [x.clone() for x in plan.batch_fold_score(t, f, p, nbins)]
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            _say(f"graph replay {rep}")
            plan.batch_replay()
        side.synchronize()
        for x, y in zip(gout, eo):
            assert torch.equal(x, y), f"replay {rep} differs from the eager run"


def test_batch_kepler_shaped_sampled(torch_dev, plan):
    """Uneven Kepler-shaped stars (20k-70k samples, gaps, noise 1e-4..1e-3,
    some with transits), 2,048 periods each, checked on sampled periods."""
    torch = torch_dev
    stars = synth.multi_star(seed=1005, n_stars=12, n_transit=4)
    k = 2048
    periods = synth.freq_grid(1.0, 5.0, k)
    so = np.concatenate([[0], np.cumsum([s.t.size for s in stars])]).astype(np.int64)
    po = np.arange(len(stars) + 1, dtype=np.int64) * k
    plan.batch_setup(so, po)
    t = _dev(torch, np.concatenate([s.t for s in stars]), torch.float64)
    f = _dev(torch, np.concatenate([s.flux for s in stars]), torch.float32)
    p = _dev(torch, np.tile(periods, len(stars)), torch.float64)
    _say(f"batch kepler-shaped stars={len(stars)} k={k}")
    out = plan.batch_fold_score(t, f, p, 256)
    torch.cuda.synchronize()
    snr = out[0].cpu().numpy()
    rng = np.random.default_rng(3)
    for c, s in enumerate(stars):
        idx = np.unique(np.concatenate([rng.choice(k, 40, replace=False),
                                        [int(np.argmax(snr[c * k:(c + 1) * k]))]]))
        mean, sigma, _ = oracle.curve_stats(s.t, s.flux)
        _, dsums, counts = oracle.fold(s.t, s.flux, periods[idx], 256, ref=mean, nthreads=8)
        osnr, _, _, _ = oracle.score(counts, dsums, sigma)
        np.testing.assert_allclose(snr[c * k + idx], osnr, rtol=1e-5, atol=1e-5)
