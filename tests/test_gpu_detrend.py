"""Light-curve pre-processing on the GPU (gpfc_detrend, Sec. 2.2) against the
CPU statement of the same steps (oracle/detrend.py): segment count, the kept
points bit for bit and the detrended flux within 1e-9 on raw synthetic curves
with trends, gaps, flux jumps, outliers and masked transits; the edge crop of
0 and 30 points; short segments dropped; the empty curve; determinism."""
import numpy as np
import pytest

from oracle import detrend as od

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


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


def _run(torch, plan, t, f, tr, **kw):
    dev = torch.device("cuda", 0)
    tt = torch.tensor(t, dtype=torch.float64, device=dev)
    ff = torch.tensor(f, dtype=torch.float32, device=dev)
    mm = None if tr is None else torch.tensor(tr.astype(np.uint8), device=dev)
    out, keep, info = plan.detrend(tt, ff, mm, **kw)
    return out.cpu().numpy(), keep.cpu().numpy().astype(bool), info


def _check(t, f, tr, out, keep, info, edge=30):
    o_out, o_keep, recs = od.detrend(t, f, tr, edge=edge)
    assert info["n_segments"] == len(recs)
    assert info["n_kept_segments"] == sum(1 for r in recs if not np.isnan(r[2]))
    assert info["status"] == 0
    assert np.array_equal(keep, o_keep), f"{np.flatnonzero(keep != o_keep)[:10]}"
    live = o_out != 0.0
    assert np.array_equal(out == 0.0, ~live)
    np.testing.assert_allclose(out[live], o_out[live], rtol=1e-9, atol=0)


@pytest.mark.parametrize("seed", [2002, 2003, 2004, 2005, 2008])
def test_detrend_matches_oracle(torch_dev, plan, seed):
    from paper_2312_02063_amd import synth
    t, f, tr = synth.trended_curve(seed)
    _say(f"detrend seed {seed}: n={t.size}")
    out, keep, info = _run(torch_dev, plan, t, f, tr)
    _check(t, f, tr, out, keep, info)
    # deterministic: a second call gives the same bits
    out2, keep2, _ = _run(torch_dev, plan, t, f, tr)
    assert np.array_equal(out2.view(np.int64), out.view(np.int64)) and np.array_equal(keep2, keep)


def test_detrend_without_mask_and_edge_zero(torch_dev, plan):
    from paper_2312_02063_amd import synth
    t, f, _ = synth.trended_curve(2006, n=6000, n_jumps=0)
    _say("detrend: no mask, edge 0")
    out, keep, info = _run(torch_dev, plan, t, f, None, edge=0)
    _check(t, f, None, out, keep, info, edge=0)


def test_detrend_short_segments_and_empty(torch_dev, plan):
    rng = np.random.default_rng(7)
    dt = od.CADENCE
    t = np.concatenate([dt * np.arange(60), 10.0 + dt * np.arange(61), 20.0 + dt * np.arange(700)])
    f = (1.0 + 5e-3 * np.sin(t / 3.0) + rng.normal(0, 1e-4, t.size)).astype(np.float32)
    _say("detrend: segments of 60, 61 and 700 points")
    out, keep, info = _run(torch_dev, plan, t, f, None)
    _check(t, f, None, out, keep, info)
    assert info["n_segments"] == 3
    assert not keep[:60].any() and keep[60:121].sum() == 1
    _say("detrend: empty curve")
    out, keep, info = _run(torch_dev, plan, np.zeros(0), np.zeros(0, np.float32), None)
    assert out.size == 0 and info["n_segments"] == 0
