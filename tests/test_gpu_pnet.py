"""The paper's own network (Sec. 2.5, Fig. 5) on the GPU against the FP64
oracle (oracle/pnet_oracle.c): FP32 logits and every parameter gradient
(dropout mask included) within 1e-4, the bf16 error printed and bounded,
chunked inference equal to one pass, deterministic gradients, and a loss that
falls under training."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

NAMES = ["w1", "b1", "w2", "b2", "w3", "b3", "w4", "b4", "w5", "b5", "w6", "b6"]


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _inputs(seed, B):
    """z-scored random folds [B][256] (what the fold kernel hands the network)."""
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(B, 256))
    x = (x - x.mean(axis=1, keepdims=True)) / x.std(axis=1, keepdims=True)
    y = (np.arange(B) % 2).astype(np.float64)
    return x, y


def _net(torch, precision, params, max_batch=64):
    from paper_2312_02063_amd import PNet
    net = PNet(0, precision, max_batch=max_batch)
    net.set_params(torch.tensor(params, dtype=torch.float32, device="cuda"))
    return net


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_pnet_fp32_forward_matches_oracle(torch_dev):
    torch = torch_dev
    from paper_2312_02063_amd import CNN_FP32, synth
    # the GPU computes with FP32 weights: the oracle takes the same rounded values
    p = synth.pnet_init(11).astype(np.float32).astype(np.float64)
    x, _ = _inputs(12, 6)
    _say("pnet fp32 forward, 6 inputs")
    net = _net(torch, CNN_FP32, p)
    z = net.forward(torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy()
    zo = oracle.pnet_forward(p, x.astype(np.float32).astype(np.float64))
    print("fp32 logits", z, "oracle", zo)
    np.testing.assert_allclose(z, zo, rtol=1e-4, atol=1e-4 * np.abs(zo).max())
    net.close()


def test_pnet_fp32_gradients_match_oracle(torch_dev):
    torch = torch_dev
    from paper_2312_02063_amd import CNN_FP32, synth
    p = synth.pnet_init(13).astype(np.float32).astype(np.float64)
    B = 4
    x, y = _inputs(14, B)
    x = x.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(15)
    keep = (rng.random((B, 128)) >= 0.5).astype(np.float64) * 2.0     # dropout 0.5, scaled
    _say("pnet fp32 backward, 4 inputs with dropout")
    net = _net(torch, CNN_FP32, p)
    loss = net.backward(torch.tensor(x, dtype=torch.float32, device="cuda"),
                        torch.tensor(y, dtype=torch.float32, device="cuda"),
                        keep=torch.tensor(keep, dtype=torch.float32, device="cuda")).item()
    g = net.get_grads().cpu().numpy().astype(np.float64)
    lo, go = oracle.pnet_loss_grad(p, x, y, mask=keep)
    assert abs(loss - lo) <= 1e-5 * max(1.0, abs(lo)), (loss, lo)
    gs, gos = oracle.pnet_split(g), oracle.pnet_split(go)
    for name in NAMES:
        e = _rel(gs[name].ravel(), gos[name].ravel())
        print(f"grad {name}: relative error {e:.2e} (norm {np.linalg.norm(gos[name]):.3e})")
        assert e < 1e-4, name
    # determinism: the same step gives the same bits
    net.backward(torch.tensor(x, dtype=torch.float32, device="cuda"),
                 torch.tensor(y, dtype=torch.float32, device="cuda"),
                 keep=torch.tensor(keep, dtype=torch.float32, device="cuda"))
    g2 = net.get_grads().cpu().numpy()
    assert np.array_equal(g2.view(np.int32), g.astype(np.float32).view(np.int32))
    net.close()


def test_pnet_bf16_forward_error_and_chunking(torch_dev):
    torch = torch_dev
    from paper_2312_02063_amd import CNN_BF16, synth
    p = synth.pnet_init(16)
    x, _ = _inputs(17, 40)
    _say("pnet bf16 forward, 40 inputs in passes of 16")
    net = _net(torch, CNN_BF16, p, max_batch=16)
    xb = torch.tensor(x, dtype=torch.float32, device="cuda").to(torch.bfloat16).view(torch.uint16)
    z = net.forward(xb).cpu().numpy()
    zo = oracle.pnet_forward(p, x)
    e = _rel(z, zo)
    print(f"bf16 logits relative L2 error vs FP64: {e:.3e}")
    # bf16 keeps 8 significant bits (unit roundoff 2^-9); weights and activations of
    # six layers are rounded to it: about sqrt(12) * 2^-9 = 7e-3 of the logits' norm
    assert e < 3e-2
    net.close()
    big = _net(torch, CNN_BF16, p, max_batch=64)
    z1 = big.forward(xb).cpu().numpy()
    assert np.array_equal(z1.view(np.int32), z.view(np.int32)), "chunked passes differ from one pass"
    big.close()


def test_pnet_bf16_training_lowers_the_loss(torch_dev):
    torch = torch_dev
    from paper_2312_02063_amd import CNN_BF16, synth
    p = synth.pnet_init(18)
    rng = np.random.default_rng(19)
    B = 64
    x = rng.normal(size=(B, 256))
    y = (np.arange(B) % 2).astype(np.float32)
    x[y == 1, 120:136] -= 2.0            # a dip in the positives
    x = (x - x.mean(axis=1, keepdims=True)) / x.std(axis=1, keepdims=True)
    _say("pnet bf16 training, 40 steps")
    net = _net(torch, CNN_BF16, p, max_batch=B)
    xt = torch.tensor(x, dtype=torch.float32, device="cuda").to(torch.bfloat16).view(torch.uint16)
    yt = torch.tensor(y, device="cuda")
    first = net.backward(xt, yt).item()
    for _ in range(40):
        net.train_step(xt, yt, 1e-4)
    last = net.backward(xt, yt).item()
    print(f"training loss {first:.4f} -> {last:.4f}")
    assert last < 0.5 * first
    net.close()


def test_pnet_fused_pairs_equal_layer_path(torch_dev):
    """The fused convolution-pair kernels (activation tile in LDS, pooling in the
    epilogue) against the layer-by-layer path: identical logits for bf16 and
    FP32 inputs, identical gradients with a dropout mask."""
    torch = torch_dev
    from paper_2312_02063_amd import CNN_BF16, synth
    p = synth.pnet_init(21)
    x, y = _inputs(22, 37)
    rng = np.random.default_rng(23)
    keep = torch.tensor((rng.random((37, 128)) >= 0.5) * 2.0, dtype=torch.float32, device="cuda")
    _say("pnet fused pairs vs layer path, 37 inputs")
    net = _net(torch, CNN_BF16, p, max_batch=64)
    xf = torch.tensor(x, dtype=torch.float32, device="cuda")
    xb = xf.to(torch.bfloat16).view(torch.uint16)
    yt = torch.tensor(y, dtype=torch.float32, device="cuda")
    out = {}
    for fused in (True, False):
        net.set_fused(fused)
        zb = net.forward(xb).cpu().numpy()
        zf = net.forward(xf).cpu().numpy()
        net.backward(xb, yt, keep=keep)
        out[fused] = (zb, zf, net.get_grads().cpu().numpy())
    for a, b, name in zip(out[True], out[False], ("bf16 logits", "f32 logits", "gradients")):
        assert np.array_equal(a.view(np.int32), b.view(np.int32)), name
    net.close()
