"""The allocation-free fold + score (gpfc_fold_score_noalloc) against
gpfc_fold_score on the same inputs, called through the C ABI: two calls in a
row, the second on a smaller curve and grid (and a two-word, zero-centred
flux), so the second call runs over the first call's leftover buffer
contents. Same kernels, so every output must be identical."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _outputs(torch, k, dev):
    return (torch.empty(k, dtype=torch.float32, device=dev), torch.empty(k, dtype=torch.int32, device=dev),
            torch.empty(k, dtype=torch.int32, device=dev), torch.empty(k, dtype=torch.float32, device=dev))


def _noalloc(lib, torch, t, f, p, nbins):
    k = p.numel()
    snr, st, wd, dp = _outputs(torch, k, t.device)
    ptr = lambda x: ctypes.c_void_p(x.data_ptr())
    rc = lib.gpfc_fold_score_noalloc(ptr(t), ptr(f), t.numel(), ptr(p), k, nbins, ptr(snr), ptr(st),
                                     ptr(wd), ptr(dp),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, f"gpfc_fold_score_noalloc returned {rc}"
    return snr, st, wd, dp


def test_noalloc_equals_fold_score_two_calls():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_02063_amd import Plan, _lib, synth
    lib = _lib.load()
    dev = torch.device("cuda", 0)
    plan = Plan(0)
    big = synth.kepler_long_curve(seed=1002)
    small = synth.plain_curve(seed=1001)
    cases = [
        # (t, flux, periods, nbins): 65,000 samples x 20,000 periods at 256 bins, then
        # 4,000 zero-centred samples (two packed words) x 1,000 periods at 64 bins
        (big.t, big.flux, synth.freq_grid(1.0, 5.0, 20_000), 256),
        (small.t, (small.flux - 1.0).astype(np.float32), synth.freq_grid(1.0, 5.0, 1_000), 64),
    ]
    for i, (t_np, f_np, p_np, nbins) in enumerate(cases):
        print(f"[gpu-case] noalloc call {i}: n={t_np.size} k={p_np.size} nbins={nbins}", flush=True)
        t = torch.tensor(t_np, dtype=torch.float64, device=dev)
        f = torch.tensor(f_np, dtype=torch.float32, device=dev)
        p = torch.tensor(p_np, dtype=torch.float64, device=dev)
        got = _noalloc(lib, torch, t, f, p, nbins)
        ref = plan.fold_score(t, f, p, nbins)
        torch.cuda.synchronize()
        assert lib.gpfc_sync(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)) == 0
        for name, a, b in zip(("snr", "start", "width", "depth"), got, ref):
            a, b = a.cpu().numpy(), b.cpu().numpy()
            assert np.array_equal(a.view(np.int32), b.view(np.int32)), f"call {i}: {name} differs"
        if i == 1:
            c = plan.curve_stats(t, f)
            assert c["words"] == 2, "the second curve must take the two-word packing"
    plan.close()
