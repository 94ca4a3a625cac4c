"""Per-curve reduction and the chunked survey (runs on an MI355X).

gpfc_topk against the oracle bit for bit (values and indices). The survey:
box-SNR against the oracle (1e-5); the network's logits equal, bit for bit,
those of gpfc_cnn_forward on the single-curve normalised folds (same
kernels, deterministic); its reductions equal the oracle's reduction of its
own periodograms; a captured survey replays to the eager result.
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


def _dev(torch, a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("rows,n,top,gated", [(1, 0, 4, False), (3, 50, 64, False), (5, 777, 7, True),
                                              (600, 333, 1, False), (2, 100_003, 64, True),
                                              (1, 2_000_000, 16, False)])
def test_topk_matches_oracle(torch_dev, rows, n, top, gated):
    from paper_2312_02063_amd import topk
    torch = torch_dev
    rng = np.random.default_rng(rows * 7 + n)
    x = np.round(rng.normal(size=(rows, n)) * 8).astype(np.float32)   # many ties
    x[rng.uniform(size=(rows, n)) < 0.01] = np.nan
    if n > 10:
        x[0, 3] = -np.inf
    g = rng.uniform(0, 10, (rows, n)).astype(np.float32) if gated else None
    _say(f"topk rows={rows} n={n} top={top} gated={gated}")
    v, i = topk(_dev(torch, x, torch.float32), top,
                _dev(torch, g, torch.float32) if gated else None, 5.0)
    torch.cuda.synchronize()
    ov, oi = oracle.topk(x, top, g, 5.0)
    np.testing.assert_array_equal(i.cpu().numpy(), oi)
    np.testing.assert_array_equal(v.cpu().numpy(), ov)


def test_topk_split_row_mostly_empty(torch_dev):
    """A long row split over many blocks where most parts hold fewer than
    `top` valid scores (99.9% NaN): the merge sees empty places."""
    from paper_2312_02063_amd import topk
    torch = torch_dev
    rng = np.random.default_rng(77)
    x = np.round(rng.normal(size=(1, 1_500_000)) * 4).astype(np.float32)
    x[rng.uniform(size=x.shape) < 0.999] = np.nan
    _say("topk split row mostly NaN")
    v, i = topk(_dev(torch, x, torch.float32), 64)
    ov, oi = oracle.topk(x, 64)
    np.testing.assert_array_equal(i.cpu().numpy(), oi)
    np.testing.assert_array_equal(v.cpu().numpy(), ov)


@pytest.mark.parametrize("rows,n,top,nan_frac,gate_pass,seed", [
    (1, 1024, 64, 0.9, None, 1), (1, 1024, 64, 0.9, None, 2), (4, 1024, 64, 0.95, None, 3),
    (1, 1024, 64, 0.0, 0.7, 4), (3, 5000, 64, 0.3, 0.3, 5), (2, 1024, 48, 0.9, None, 6),
    (1, 900_000, 64, 0.9995, None, 7), (1, 600_000, 64, 0.0, 0.0003, 8)])
def test_topk_wave_lists_with_holes(torch_dev, rows, n, top, nan_frac, gate_pass, seed):
    """Rows where a wave's first 64 elements leave empty places at scattered
    lanes (NaN or gated out) and the wave sees fewer than `top` entries in
    all: the per-wave sorted lists must still be a permutation of the places.
    The long rows run split over many blocks whose parts leave holes too."""
    from paper_2312_02063_amd import topk
    torch = torch_dev
    rng = np.random.default_rng(seed)
    x = np.round(rng.normal(size=(rows, n)) * 6).astype(np.float32)
    x[rng.uniform(size=(rows, n)) < nan_frac] = np.nan
    g = None
    if gate_pass is not None:
        g = np.where(rng.uniform(size=(rows, n)) < gate_pass, 9.0, 1.0).astype(np.float32)
    _say(f"topk holes rows={rows} n={n} top={top} nan={nan_frac} gate={gate_pass} seed={seed}")
    v, i = topk(_dev(torch, x, torch.float32), top,
                None if g is None else _dev(torch, g, torch.float32), 5.0)
    torch.cuda.synchronize()
    ov, oi = oracle.topk(x, top, g, 5.0)
    np.testing.assert_array_equal(i.cpu().numpy(), oi)
    np.testing.assert_array_equal(v.cpu().numpy(), ov)


def test_topk_ascending_worst_case(torch_dev):
    """Ascending values make every element enter the candidate lists."""
    from paper_2312_02063_amd import topk
    torch = torch_dev
    x = np.arange(200_000, dtype=np.float32).reshape(1, -1)
    _say("topk ascending")
    v, i = topk(_dev(torch, x, torch.float32), 64)
    ov, oi = oracle.topk(x, 64)
    np.testing.assert_array_equal(i.cpu().numpy(), oi)


def _stars(n_stars, seed=21):
    return synth.multi_star(seed=seed, n_stars=n_stars, nmin=2000, nmax=7000,
                            n_transit=max(1, n_stars // 3), alpha=(10.0, 20.0))


def _survey(torch, stars, k, chunk_folds, net=None, top=8, judge=3.0, capture=False, fp8=False):
    from paper_2312_02063_amd import Plan
    plan = Plan(0)
    periods = synth.freq_grid(1.0, 5.0, k)
    so = np.concatenate([[0], np.cumsum([s.t.size for s in stars])]).astype(np.int64)
    plan.survey_setup(so, k, chunk_folds)
    t = _dev(torch, np.concatenate([s.t for s in stars]), torch.float64)
    f = _dev(torch, np.concatenate([s.flux for s in stars]), torch.float32)
    p = _dev(torch, periods, torch.float64)
    if capture:
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            r = plan.survey_capture(t, f, p, 256, cnn=net, top=top, judge_snr=judge, fp8=fp8)
        torch.cuda.synchronize()
        return plan, r, (t, f, p, side, periods)
    r = plan.survey_run(t, f, p, 256, cnn=net, top=top, judge_snr=judge, fp8=fp8)
    torch.cuda.synchronize()
    return plan, {a: b.cpu().numpy() for a, b in r.items()}, periods


def _net(torch, max_batch=1500):
    from paper_2312_02063_amd import CNN_BF16, Cnn
    net = Cnn(0, CNN_BF16, max_batch)
    net.set_params(synth.cnn_init(77).astype(np.float32))
    return net


def test_survey_box_only_matches_oracle(torch_dev):
    torch = torch_dev
    stars = _stars(7)
    k = 333
    _say(f"survey box-only stars={len(stars)} k={k}")
    _, r, periods = _survey(torch, stars, k, 0, top=5)
    for c, s in enumerate(stars):
        mean, sigma, _ = oracle.curve_stats(s.t, s.flux)
        _, dsums, counts = oracle.fold(s.t, s.flux, periods, 256, ref=mean, nthreads=8)
        osnr, _, _, _ = oracle.score(counts, dsums, sigma)
        np.testing.assert_allclose(r["snr"][c], osnr, rtol=1e-5, atol=1e-5)
    ov, oi = oracle.topk(r["snr"], 5)
    np.testing.assert_array_equal(r["box_idx"], oi)
    np.testing.assert_array_equal(r["box_val"], ov)


@pytest.mark.parametrize("chunk_folds", [333, 1000, 2600])
def test_survey_with_network(torch_dev, chunk_folds):
    """Chunks of 1, 3 and 7 curves; the network runs in batches of 1,500."""
    from paper_2312_02063_amd import Plan
    torch = torch_dev
    stars = _stars(8, seed=31)
    k = 333
    net = _net(torch)
    _say(f"survey + cnn stars={len(stars)} k={k} chunk_folds={chunk_folds}")
    _, r, periods = _survey(torch, stars, k, chunk_folds, net=net, top=8, judge=3.0)
    single = Plan(0)
    pp = _dev(torch, periods, torch.float64)
    for c, s in enumerate(stars):
        single.prepare(_dev(torch, s.t, torch.float64), _dev(torch, s.flux, torch.float32))
        z = torch.empty((k, 256), dtype=torch.uint16, device="cuda")
        out = single.fold_score_prepared(pp, 256, zfold=z)
        lg = net.forward(z)
        torch.cuda.synchronize()
        assert np.array_equal(r["snr"][c], out[0].cpu().numpy()), c
        assert np.array_equal(r["logits"][c], lg.cpu().numpy()), c
    ov, oi = oracle.topk(r["logits"], 8)
    np.testing.assert_array_equal(r["cnn_idx"], oi)
    np.testing.assert_array_equal(r["cnn_val"], ov)
    ov, oi = oracle.topk(r["logits"], 8, r["snr"], 3.0)
    np.testing.assert_array_equal(r["judged_idx"], oi)
    np.testing.assert_array_equal(r["judged_val"], ov)


def test_survey_capture_replays(torch_dev):
    torch = torch_dev
    stars = _stars(5, seed=41)
    k = 200
    net = _net(torch, max_batch=512)
    _say("survey capture")
    plan, gr, (t, f, p, side, _) = _survey(torch, stars, k, 450, net=net, top=4, capture=True)
    for rep in range(3):
        f.mul_(1.0 + 1e-4 * (rep + 1)).add_(-1e-4 * (rep + 1))
        torch.cuda.synchronize()
        _say(f"survey eager rep {rep}")
        er = plan.survey_run(t, f, p, 256, cnn=net, top=4, judge_snr=3.0)
        er = {a: b.clone() for a, b in er.items()}
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            _say(f"survey replay {rep}")
            plan.batch_replay()
        side.synchronize()
        for key in er:
            a, b = gr[key], er[key]
            if not torch.equal(a, b):
                af, bf = a.double(), b.double()
                nd = int((af != bf).sum())
                print(f"{key}: {nd} of {a.numel()} differ; nan {int(torch.isnan(af).sum())} "
                      f"{int(torch.isnan(bf).sum())}; max diff {float((af - bf).abs().nan_to_num().max())}; "
                      f"first rows {torch.nonzero(af != bf)[:5].tolist()}")
            assert torch.equal(a, b), f"replay {rep}: {key}"


def test_survey_fp8(torch_dev):
    torch = torch_dev
    stars = _stars(3, seed=51)
    k = 150
    net = _net(torch, max_batch=512)
    cal = torch.randn(400, 256, device="cuda")
    net.calibrate_fp8(cal)
    _say("survey fp8")
    _, r, periods = _survey(torch, stars, k, 300, net=net, top=2, fp8=True)
    from paper_2312_02063_amd import Plan
    single = Plan(0)
    pp = _dev(torch, periods, torch.float64)
    for c, s in enumerate(stars):
        single.prepare(_dev(torch, s.t, torch.float64), _dev(torch, s.flux, torch.float32))
        z = torch.empty((k, 256), dtype=torch.uint16, device="cuda")
        single.fold_score_prepared(pp, 256, zfold=z)
        lg = net.forward_fp8(z)
        torch.cuda.synchronize()
        assert np.array_equal(r["logits"][c], lg.cpu().numpy()), c


@pytest.mark.parametrize("rows,n,nsig,mw", [(1, 0, 3.0, 3), (3, 40, 0.5, 0), (4, 5000, 1.0, 3),
                                            (2, 100_003, 2.0, 2), (1, 2_000_000, 3.0, 3),
                                            (1, 300_001, 0.0, 3)])
def test_periodogram_peaks_match_oracle(torch_dev, rows, n, nsig, mw):
    """SDE, mean, sd, peak count and the best peaks against the oracle: values
    and indices exact, statistics to FP32 rounding. Smooth rows make long runs
    that cross the kernel's per-thread chunks; long rows are split over many
    blocks."""
    from paper_2312_02063_amd import periodogram_peaks
    torch = torch_dev
    rng = np.random.default_rng(rows * 31 + n)
    x = rng.normal(size=(rows, n))
    if n > 100:
        # red noise: runs of hundreds of points above threshold
        k = np.exp(-np.arange(200) / 40.0)
        x = np.array([np.convolve(r, k, mode="same") for r in x])
    x = x.astype(np.float32)
    if n > 10:
        x[0, n // 2] = np.nan
    periods = 1.0 / np.linspace(1.0, 5.0, max(n, 1))[:n]
    _say(f"periodogram rows={rows} n={n} nsigma={nsig} min_width={mw}")
    r = periodogram_peaks(_dev(torch, x, torch.float32), _dev(torch, periods, torch.float64), nsig, mw, 6)
    torch.cuda.synchronize()
    o = oracle.periodogram(x, periods, nsig, mw, 6)
    g = {k: v.cpu().numpy() for k, v in r.items()}
    np.testing.assert_array_equal(g["n_peaks"], o["n_peaks"])
    np.testing.assert_array_equal(g["idx"], o["idx"])
    np.testing.assert_array_equal(g["val"], o["val"])
    np.testing.assert_array_equal(g["width"], o["width"])
    np.testing.assert_array_equal(g["harmonic"], o["harmonic"])
    np.testing.assert_allclose(g["sde"], o["sde"], rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(g["mean"], o["mean"], rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(g["sd"], o["sd"], rtol=1e-5, atol=1e-6)


def test_periodogram_run_spanning_many_parts(torch_dev):
    """A long row split over many blocks with one plateau far above the
    threshold covering whole parts, and a second plateau ending at the row's
    last score: runs joined across parts, and a run touching the row's end."""
    from paper_2312_02063_amd import periodogram_peaks
    torch = torch_dev
    rng = np.random.default_rng(5)
    n = 2_000_000
    x = rng.normal(size=(1, n)).astype(np.float32)
    x[0, 50_000:180_000] = 20.0           # mean 1.45, sd 5.4: threshold 17.7
    x[0, 120_001] = 25.0                  # the plateau's maximum, inside a middle part
    x[0, 1_990_000:] = 30.0
    periods = 1.0 / np.linspace(1.0, 5.0, n)
    _say("periodogram plateau over many parts")
    r = periodogram_peaks(_dev(torch, x, torch.float32), _dev(torch, periods, torch.float64), 3.0, 3, 6)
    torch.cuda.synchronize()
    o = oracle.periodogram(x, periods, 3.0, 3, 6)
    g = {k: v.cpu().numpy() for k, v in r.items()}
    for key in ("n_peaks", "idx", "val", "width", "harmonic"):
        np.testing.assert_array_equal(g[key], o[key])
    assert g["idx"][0, 0] == 1_990_000 and g["width"][0, 0] == 10_000
    assert g["idx"][0, 1] == 120_001 and g["width"][0, 1] == 130_000
    np.testing.assert_allclose(g["sde"], o["sde"], rtol=1e-5, atol=1e-6)


def test_survey_replay_uses_current_weights(torch_dev):
    """A captured survey re-packs the network's weights on every replay: after
    new parameters are set, the replay's logits equal an eager run's."""
    torch = torch_dev
    stars = _stars(3, seed=61)
    k = 128
    net = _net(torch, max_batch=512)
    _say("survey capture, then new weights")
    plan, gr, (t, f, p, side, _) = _survey(torch, stars, k, 256, net=net, top=2, capture=True)
    net.set_params((synth.cnn_init(78) * 0.9).astype(np.float32))
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        plan.batch_replay()
    side.synchronize()
    er = plan.survey_run(t, f, p, 256, cnn=net, top=2, judge_snr=3.0)
    torch.cuda.synchronize()
    assert torch.equal(gr["logits"], er["logits"])
    assert torch.equal(gr["cnn_idx"], er["cnn_idx"])


def test_survey_autotune_keeps_results_and_caches(torch_dev, tmp_path):
    """The survey tuner times chunk sizes x network pass sizes, leaves the plan
    set up with the fastest; a survey with the tuned shape equals one with any
    other shape bit for bit, and a second call takes the shape from the cache."""
    from paper_2312_02063_amd import Plan
    torch = torch_dev
    stars = _stars(9, seed=41)
    k = 333
    net = _net(torch, max_batch=2048)
    periods = synth.freq_grid(1.0, 5.0, k)
    so = np.concatenate([[0], np.cumsum([s.t.size for s in stars])]).astype(np.int64)
    t = _dev(torch, np.concatenate([s.t for s in stars]), torch.float64)
    f = _dev(torch, np.concatenate([s.flux for s in stars]), torch.float32)
    p = _dev(torch, periods, torch.float64)
    cache = str(tmp_path / "tune.txt")
    plan = Plan(0)
    _say("survey autotune: 3 chunk sizes x 2 network pass sizes")
    c, nb, ms = plan.survey_autotune(so, t, f, p, 256, cnn=net, chunks=(333, 999, 3000), nets=(512, 2048),
                                     cache_path=cache)
    assert c in (333, 999, 3000) and nb in (512, 2048) and ms > 0
    r = plan.survey_run(t, f, p, 256, cnn=net, top=4, judge_snr=3.0)
    _, ref, _ = _survey(torch, stars, k, 999, net=net, top=4, judge=3.0)
    torch.cuda.synchronize()
    for key in ("snr", "logits", "box_idx", "cnn_idx", "judged_idx"):
        assert np.array_equal(r[key].cpu().numpy(), ref[key]), key
    again = Plan(0)
    c2, nb2, ms2 = again.survey_autotune(so, t, f, p, 256, cnn=net, chunks=(333, 999, 3000),
                                         nets=(512, 2048), cache_path=cache)
    assert (c2, nb2, ms2) == (c, nb, -1.0)
    assert open(cache).read().count(" survey ") == 1
