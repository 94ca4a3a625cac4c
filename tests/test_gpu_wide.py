"""Parity of the two-word fixed-point fold and of the general path (runs on
an MI355X).

Two-word curves: flux whose deviations need more than 27 bits of fixed-point
range (zero-centred flux, one near-zero cadence) is packed in two words, so
its bin sums stay exact integers; a curve spanning more than 53 bits keeps 53
bits (flagged inexact, error below count * maxdev * 2^-52 per bin). General
path: nbins 512-4096 and curves longer than 2^18 - 1 samples. Bar as in
test_gpu_parity: counts bit-exact; sums, means and SNR within 1e-5 relative
(SNR 1e-5 absolute below 1) with the near-tie rule; beyond that, two-word sums
against exact (math.fsum) bin sums within a few FP64 roundings.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2312_02063_amd import synth
from test_gpu_parity import RTOL, check_fold, check_score

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


def _inputs(torch, t, f, periods):
    return (_dev(torch, t, torch.float64), _dev(torch, f, torch.float32),
            _dev(torch, periods, torch.float64))


def _curve(kind):
    """Kepler-long times with flux that needs (kind) one or two words."""
    c = synth.kepler_long_curve(1002)
    rng = np.random.default_rng(4242)
    n = c.t.size
    if kind == "zero-centred":          # N(0, 3e-4): fine ulps near zero
        f = rng.normal(0.0, 3e-4, n).astype(np.float32)
    elif kind == "one-near-zero":       # flux ~ 1 and one cadence at 1e-6
        f = c.flux.copy()
        f[n // 3] = np.float32(1e-6)
    elif kind == "raw-counts":          # ~1e5 counts with a 30% eclipse
        ph = (c.t / 0.731) % 1.0
        f = (1e5 * (1.0 + rng.normal(0.0, 3e-4, n)) * np.where(ph < 0.05, 0.7, 1.0)).astype(np.float32)
    elif kind == "beyond-53-bits":      # flux ~ 1 and one cadence at 1e-20
        f = c.flux.copy()
        f[n // 2] = np.float32(1e-20)
    else:
        raise ValueError(kind)
    return c.t, f


EXPECT = {"zero-centred": (2, 1), "one-near-zero": (2, 1), "raw-counts": (1, 1),
          "beyond-53-bits": (2, 0)}


def _bins(t, P, nbins):
    x = t / P
    b = np.floor((x - np.floor(x)) * nbins)
    return np.clip(np.nan_to_num(b, nan=0.0), 0, nbins - 1).astype(np.int64)


@pytest.mark.parametrize("kind", list(EXPECT))
def test_wide_range_flux_fold(torch_dev, plan, kind):
    """Counts bit-exact and sums to the 1e-5 bar against the oracle; for the
    two-word exact curves the sums equal the exact bin sums up to the final
    FP64 roundings, and the inexact curve stays within its stated bound."""
    torch = torch_dev
    t, f = _curve(kind)
    _say(f"wide-range stats {kind}")
    st = plan.curve_stats(_dev(torch, t, torch.float64), _dev(torch, f, torch.float32))
    assert (st["words"], st["exact"]) == EXPECT[kind], st
    periods = synth.freq_grid(1.0, 5.0, 2_000_000)[::6000][:300]
    for nb in (256, 64):
        sums, counts = check_fold(torch, plan, t, f, periods, nb, f"{kind}-nb{nb}")
    fd = f.astype(np.float64)
    for j in (0, 77, 151, 299):
        b = _bins(t, periods[j], 64)
        for bin_ in range(64):
            vals = fd[b == bin_]
            exact = math.fsum(vals)
            err = abs(sums[j, bin_] - exact)
            if EXPECT[kind][1]:
                tol = 4 * 2.0 ** -53 * (np.abs(vals).sum() + vals.size * abs(st["ref"]))
            else:
                tol = vals.size * st["maxdev"] * 2.0 ** -51 + 4 * 2.0 ** -53 * np.abs(vals).sum()
            assert err <= tol, (kind, j, bin_, err, tol)


@pytest.mark.parametrize("kind", ["zero-centred", "one-near-zero", "raw-counts", "beyond-53-bits"])
def test_wide_range_flux_fold_score(torch_dev, kind):
    """Fused fold + score of the two-word curves (two 32-period passes per
    block), single-block and sample-split launches, against the oracle;
    every split bit-identical, normalised folds included."""
    from paper_2312_02063_amd import Plan
    torch = torch_dev
    t, f = _curve(kind)
    periods = synth.freq_grid(1.0, 5.0, 2_000_000)[::5000][:400]
    mean, sigma, _ = oracle.curve_stats(t, f)
    _, dsums, counts = oracle.fold(t, f, periods, 256, ref=mean, nthreads=8)
    ref = oracle.score(counts, dsums, sigma)
    p = Plan(0)
    tt, ff, pp = _inputs(torch, t, f, periods)
    p.prepare(tt, ff)
    first = None
    for split in (1, 2, 8):
        p.set_split(split)
        _say(f"wide-range fold_score {kind} split={split}")
        z = torch.empty((periods.size, 256), dtype=torch.uint16, device="cuda")
        out = p.fold_score_prepared(pp, 256, zfold=z)
        torch.cuda.synchronize()
        got = [x.cpu().numpy() for x in out] + [z.cpu().numpy()]
        if first is None:
            first = got
            check_score(got[0], got[1], got[2], got[3], ref, counts, dsums, sigma, f"{kind}")
            sums, _, ocounts = oracle.fold(t, f, periods, 256, nthreads=8)
            zo = oracle.normalize(sums, ocounts)
            zg = (got[4].astype(np.uint32) << 16).view(np.float32).astype(np.float64)
            assert (np.abs(zg - zo) <= 2.0 ** -8 * np.abs(zo) + 2e-3).all(), kind
        else:
            for a, b in zip(got, first):
                assert np.array_equal(a, b), f"{kind}: split {split} differs"
    p.close()


def test_wide_range_batch_equals_single(torch_dev, plan):
    """A batch mixing one-word and two-word curves equals the single-curve
    path bit for bit."""
    torch = torch_dev
    curves = [_curve("zero-centred"), _curve("raw-counts"), _curve("one-near-zero")]
    rng = np.random.default_rng(3)
    ks = [130, 64, 97]
    ps = [1.0 / rng.uniform(1.0, 5.0, k) for k in ks]
    so = np.concatenate([[0], np.cumsum([c[0].size for c in curves])]).astype(np.int64)
    po = np.concatenate([[0], np.cumsum(ks)]).astype(np.int64)
    _say("wide-range batch")
    plan.batch_setup(so, po)
    t = _dev(torch, np.concatenate([c[0] for c in curves]), torch.float64)
    f = _dev(torch, np.concatenate([c[1] for c in curves]), torch.float32)
    p = _dev(torch, np.concatenate(ps), torch.float64)
    z = torch.empty((int(po[-1]), 256), dtype=torch.uint16, device="cuda")
    out = [x.cpu().numpy() for x in plan.batch_fold_score(t, f, p, 256, zfold=z)]
    zb = z.cpu().numpy()
    stats = plan.batch_curve_stats()
    assert [s["words"] for s in stats] == [2, 1, 2]
    for i, (tc, fc) in enumerate(curves):
        plan.prepare(_dev(torch, tc, torch.float64), _dev(torch, fc, torch.float32))
        zs = torch.empty((ks[i], 256), dtype=torch.uint16, device="cuda")
        one = [x.cpu().numpy() for x in plan.fold_score_prepared(_dev(torch, ps[i], torch.float64), 256,
                                                                 zfold=zs)]
        sl = slice(int(po[i]), int(po[i + 1]))
        for a, b in zip(one, out):
            assert np.array_equal(a, b[sl]), f"curve {i}"
        assert np.array_equal(zs.cpu().numpy(), zb[sl])


def test_wide_range_equal_count_and_f32(torch_dev):
    """The equal-count fold and the FP32 precision-study fold of a two-word
    curve against the oracle."""
    from paper_2312_02063_amd import Plan
    torch = torch_dev
    t, f = _curve("zero-centred")
    rng = np.random.default_rng(11)
    periods = 1.0 / rng.uniform(1.0, 5.0, 66)
    p = Plan(0)
    tt, ff, pp = _inputs(torch, t, f, periods)
    p.prepare(tt, ff)
    _say("wide-range equal-count")
    m = p.fold_eqcount_prepared(pp, 256).cpu().numpy()
    mo = oracle.fold_eqcount(t, f, periods, 256)
    scale = float(np.abs(f.astype(np.float64) - f.mean()).max())
    assert np.abs(m - mo).max() <= 1e-5 * scale
    _say("wide-range fp32 fold")
    sums, counts, means = p.fold_f32_prepared(pp, 256, True)
    torch.cuda.synchronize()
    osums, _, ocounts = oracle.fold(t, f, periods, 256, nthreads=8)
    assert np.array_equal(counts.cpu().numpy(), ocounts)
    ok = ocounts > 0
    assert np.abs(means.cpu().numpy()[ok] - oracle.means(osums, ocounts)[ok]).max() < 1e-9
    p.close()


# ------------------------------------------------------------------ general path: nbins 512-4096

@pytest.mark.parametrize("nbins", [512, 1024, 2048, 4096])
def test_fold_large_nbins(torch_dev, plan, nbins):
    """Materialised fold at nbins up to 4096: counts bit-exact, sums 1e-5;
    a ragged period count and an invalid period."""
    c = synth.kepler_long_curve(1002)
    periods = synth.freq_grid(1.0, 5.0, 2_000_000)[::9001][:67].copy()
    periods[5] = -1.0
    check_fold(torch_dev, plan, c.t, c.flux, periods, nbins, f"nb{nbins}")


@pytest.mark.parametrize("nbins", [512, 4096])
def test_fold_score_large_nbins(torch_dev, plan, nbins):
    """Fold + score at large nbins with the default width set (up to 23
    widths): the general scorer against the oracle, and gpfc_score of the
    materialised fold giving the same boxes."""
    torch = torch_dev
    c = synth.kepler_long_curve(1002)
    periods = np.concatenate([[c.truth["period"]], synth.freq_grid(1.0, 5.0, 2_000_000)[::40001][:40]])
    tt, ff, pp = _inputs(torch, c.t, c.flux, periods)
    _say(f"fold_score nbins={nbins}")
    snr, start, width, depth = [x.cpu().numpy() for x in plan.fold_score(tt, ff, pp, nbins)]
    mean, sigma, _ = oracle.curve_stats(c.t, c.flux)
    _, dsums, counts = oracle.fold(c.t, c.flux, periods, nbins, ref=mean, nthreads=8)
    ref = oracle.score(counts, dsums, sigma)
    check_score(snr, start, width, depth, ref, counts, dsums, sigma, f"fs-nb{nbins}")
    _say(f"score materialised nbins={nbins}")
    sums, cnt, _ = plan.fold(tt, ff, pp, nbins)
    out = [x.cpu().numpy() for x in plan.score(sums, cnt, sigma)]
    check_score(out[0], out[1], out[2], out[3], ref, counts, dsums, sigma, f"score-nb{nbins}")


def test_large_nbins_chunked_workspace(torch_dev):
    """A workspace cap that forces many period chunks gives the same results."""
    from paper_2312_02063_amd import Plan
    torch = torch_dev
    c = synth.plain_curve(1001)
    periods = synth.freq_grid(1.0, 5.0, 700)
    tt, ff, pp = _inputs(torch, c.t, c.flux, periods)
    big = Plan(0)
    small = Plan(0, workspace_bytes=1 << 20)        # 64 periods per chunk at 1024 bins
    _say("chunked workspace nbins=1024")
    a = [x.cpu().numpy() for x in big.fold(tt, ff, pp, 1024)]
    b = [x.cpu().numpy() for x in small.fold(tt, ff, pp, 1024)]
    sa = [x.cpu().numpy() for x in big.fold_score(tt, ff, pp, 1024)]
    sb = [x.cpu().numpy() for x in small.fold_score(tt, ff, pp, 1024)]
    for x, y in zip(a + sa, b + sb):
        assert np.array_equal(x, y, equal_nan=x.dtype.kind == "f")
    big.close()
    small.close()


def test_more_widths_than_the_fused_scorer_holds(torch_dev, plan):
    """20 box widths at 256 bins: the general scorer, against the oracle."""
    torch = torch_dev
    c = synth.plain_curve(1002)
    periods = synth.freq_grid(1.0, 5.0, 90)
    widths = list(range(1, 21))
    tt, ff, pp = _inputs(torch, c.t, c.flux, periods)
    plan.set_widths(widths)
    _say("fold_score 20 widths")
    out = [x.cpu().numpy() for x in plan.fold_score(tt, ff, pp, 256)]
    plan.set_widths(None)
    mean, sigma, _ = oracle.curve_stats(c.t, c.flux)
    _, dsums, counts = oracle.fold(c.t, c.flux, periods, 256, ref=mean, nthreads=8)
    ref = oracle.score(counts, dsums, sigma, widths)
    check_score(out[0], out[1], out[2], out[3], ref, counts, dsums, sigma, "w20")


# ------------------------------------------------------------------ general path: long curves

def _long_curve(n, seed=31, two_word=False):
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(0.0, 1470.0 * n / 65000, n))
    f = rng.normal(0.0, 3e-4, n) if two_word else 1.0 + rng.normal(0.0, 3e-4, n)
    ph = (t / 0.4321) % 1.0
    f = np.where(ph < 0.02, f - 2e-4, f).astype(np.float32)
    return t, f


@pytest.mark.parametrize("n,nbins,two_word", [(300_000, 256, False), (300_000, 64, True),
                                              (262_144, 1024, False), (600_001, 128, False)])
def test_long_curve_fold(torch_dev, plan, n, nbins, two_word):
    """Curves past one packed pass (2^18 - 1 samples): parts accumulated in
    integer histograms; counts bit-exact, sums to the bar."""
    t, f = _long_curve(n, two_word=two_word)
    periods = synth.freq_grid(1.0, 5.0, 130)
    check_fold(torch_dev, plan, t, f, periods, nbins, f"long-n{n}")


def test_long_curve_fold_score_finds_transit(torch_dev, plan):
    torch = torch_dev
    n = 300_000
    t, f = _long_curve(n)
    periods = np.sort(np.concatenate([synth.freq_grid(1.0, 5.0, 199), [0.4321]]))
    tt, ff, pp = _inputs(torch, t, f, periods)
    _say(f"long fold_score n={n}")
    snr, start, width, depth = [x.cpu().numpy() for x in plan.fold_score(tt, ff, pp, 256)]
    mean, sigma, _ = oracle.curve_stats(t, f)
    _, dsums, counts = oracle.fold(t, f, periods, 256, ref=mean, nthreads=8)
    ref = oracle.score(counts, dsums, sigma)
    check_score(snr, start, width, depth, ref, counts, dsums, sigma, "long")
    assert periods[int(np.argmax(snr))] == 0.4321


# ------------------------------------------------------------------ non-finite input

def test_non_finite_input_reported(torch_dev):
    """A NaN flux or an infinite time is reported as GPFC_EINVAL by
    gpfc_curve_stats and by the next gpfc_sync (once); clean input is not."""
    from paper_2312_02063_amd import Plan, _lib
    torch = torch_dev
    c = synth.plain_curve(1001)
    periods = synth.freq_grid(1.0, 5.0, 70)
    p = Plan(0)
    try:                                       # a flag left by an earlier test
        p.sync()
    except _lib.GpfcError:
        pass
    _say("non-finite: clean")
    p.fold_score(*_inputs(torch, c.t, c.flux, periods), 64)
    p.sync()
    bad = c.flux.copy()
    bad[17] = np.nan
    _say("non-finite: NaN flux")
    p.fold_score(*_inputs(torch, c.t, bad, periods), 64)
    with pytest.raises(_lib.GpfcError) as e:
        p.sync()
    assert e.value.code == _lib.EINVAL
    p.sync()                                   # reported once
    tb = c.t.copy()
    tb[3] = np.inf
    _say("non-finite: inf time via curve_stats")
    with pytest.raises(_lib.GpfcError) as e:
        p.curve_stats(_dev(torch, tb, torch.float64), _dev(torch, c.flux, torch.float32))
    assert e.value.code == _lib.EINVAL
    p.sync()                                   # curve_stats reported it already
    p.close()
