"""Precision sweep, reduced (runs on an MI355X): exact integer sums beat FP32
sums, compensation beats plain FP32, and every mode keeps bit-exact counts
and the SNR within 1e-5; CNN errors shrink from FP8 to bf16 to FP32."""
import pytest

pytestmark = pytest.mark.gpu


def test_precision_sweep_small():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from precision_sweep import run
    print("[gpu-case] precision sweep periods=600 cnn_folds=300", flush=True)
    r = run(n_periods=600, n_top=20, cnn_folds=300)
    fold = r["fold"]
    for mode in fold.values():
        assert mode["counts_bit_exact"]
        assert mode["snr_rel_error"]["max"] < 1e-5
    assert fold["int64_exact"]["bin_mean_abs_error"]["max"] < 1e-15
    assert fold["fp32_twosum"]["bin_mean_abs_error"]["max"] <= fold["fp32_plain"]["bin_mean_abs_error"]["max"]
    var = r["fold_variable_star"]
    for mode in var.values():
        assert mode["counts_bit_exact"]
    assert var["int64_exact"]["bin_mean_abs_error"]["max"] < 1e-14
    assert var["fp32_twosum"]["bin_mean_abs_error"]["max"] <= var["fp32_plain"]["bin_mean_abs_error"]["max"]
    cnn = r["cnn"]
    assert cnn["fp32"]["logit_abs_error"]["max"] < cnn["bf16"]["logit_abs_error"]["max"]
    assert cnn["bf16"]["logit_abs_error"]["rms"] <= cnn["fp8_e4m3"]["logit_abs_error"]["rms"] * 1.5
    print(r)
