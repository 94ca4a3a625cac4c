"""Learned scorer on the GPU against the FP64 CNN oracle (runs on an MI355X).

FP32 mode: logits and gradients to 1e-4 relative (norm-wise per tensor; a
ReLU or pooling decision that flips at a near-tie moves one term, allowed
for by the norm). bf16 mode: the measured error is printed and bounded
loosely; its accuracy is judged by what the trained network does.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2312_02063_amd import synth

pytestmark = pytest.mark.gpu

SEGMENTS = [("conv1", 0, 96), ("conv2", 96, 2688), ("conv3", 2688, 12992), ("conv4", 12992, 33536),
            ("fc1", 33536, 295936), ("fc2", 295936, 312384), ("fc3", 312384, 312449)]


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _params(seed):
    rng = np.random.default_rng(seed)
    p = synth.cnn_init(seed)
    return p + rng.normal(0, 0.02, p.size)


def _inputs(seed, B):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(B, 256))
    y = (rng.uniform(size=B) < 0.5).astype(np.float64)
    return x, y


def _net(torch, precision, params, max_batch=512):
    from paper_2312_02063_amd import Cnn
    net = Cnn(0, precision, max_batch)
    net.set_params(params.astype(np.float32))
    return net


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def test_forward_fp32_matches_oracle(torch_dev):
    torch = torch_dev
    from paper_2312_02063_amd import CNN_FP32
    p = _params(1)
    x, _ = _inputs(2, 70)
    _say("cnn forward fp32 B=70")
    net = _net(torch, CNN_FP32, p)
    z = net.forward(torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy()
    p32 = p.astype(np.float32).astype(np.float64)
    zo = oracle.cnn_forward(p32, x.astype(np.float32).astype(np.float64))
    assert np.max(np.abs(z - zo) / np.maximum(1.0, np.abs(zo))) < 1e-4


def test_forward_bf16_error_and_bf16_input(torch_dev):
    torch = torch_dev
    from paper_2312_02063_amd import CNN_BF16
    p = _params(3)
    x, _ = _inputs(4, 129)
    _say("cnn forward bf16 B=129")
    net = _net(torch, CNN_BF16, p)
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    z = net.forward(xt).cpu().numpy()
    zo = oracle.cnn_forward(p, x)
    err = _rel(z, zo)
    print(f"bf16 forward relative L2 error vs FP64: {err:.3e}")
    assert err < 5e-2
    # bfloat16-bit input (as the fold kernel writes it) = the f32 input rounded
    xb = xt.to(torch.bfloat16).view(torch.uint16)
    zb = net.forward(xb).cpu().numpy()
    z2 = net.forward(xb.view(torch.bfloat16).to(torch.float32)).cpu().numpy()
    assert np.array_equal(zb, z2)


@pytest.mark.parametrize("prec_name", ["fp32", "bf16"])
def test_gradient_matches_oracle(torch_dev, prec_name):
    torch = torch_dev
    from paper_2312_02063_amd import CNN_BF16, CNN_FP32
    prec = CNN_FP32 if prec_name == "fp32" else CNN_BF16
    p = _params(5)
    x, y = _inputs(6, 96)
    _say(f"cnn backward {prec_name} B=96")
    net = _net(torch, prec, p)
    g = torch.empty(net.n_params, dtype=torch.float32, device="cuda")
    loss = net.backward(torch.tensor(x, dtype=torch.float32, device="cuda"),
                        torch.tensor(y, dtype=torch.float32, device="cuda"), grad_out=g)
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    p32 = p.astype(np.float32).astype(np.float64)
    lo, go = oracle.cnn_loss_grad(p32, x.astype(np.float32).astype(np.float64), y)
    tol = 1e-4 if prec == CNN_FP32 else 1e-1
    assert abs(loss.item() - lo) <= tol * max(1.0, lo)
    for name, a, b in SEGMENTS:
        err = _rel(g[a:b], go[a:b])
        print(f"{prec_name} grad {name}: relative L2 error {err:.3e}")
        assert err < tol, name


def test_adam_step_matches_oracle(torch_dev):
    torch = torch_dev
    from paper_2312_02063_amd import CNN_FP32
    p = _params(7)
    x, y = _inputs(8, 64)
    net = _net(torch, CNN_FP32, p)
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    yt = torch.tensor(y, dtype=torch.float32, device="cuda")
    p_ref = p.astype(np.float32).astype(np.float64)
    m = np.zeros_like(p_ref)
    v = np.zeros_like(p_ref)
    g = torch.empty(net.n_params, dtype=torch.float32, device="cuda")
    for step in range(1, 4):
        _say(f"cnn adam step {step}")
        net.backward(xt, yt, grad_out=g)
        net.adam(1e-3)
        oracle.adam(p_ref, g.cpu().numpy().astype(np.float64), m, v, step, 1e-3)
        got = net.get_params().cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - p_ref)) < 1e-6
        p_ref = got.copy()   # continue from the GPU's (FP32) parameters


def test_training_on_folds_reduces_loss(torch_dev):
    """A few hundred Adam steps on normalised folds the fold kernel produces
    from curves with and without transits lower the loss well below log 2."""
    torch = torch_dev
    from paper_2312_02063_amd import CNN_BF16, Plan
    rng = np.random.default_rng(9)
    curves = [synth.training_curve(rng, n=2000, positive=bool(i % 2), alpha_range=(12.0, 20.0))
              for i in range(256)]
    plan = Plan(0)
    so = np.concatenate([[0], np.cumsum([c.t.size for c in curves])])
    po = np.arange(len(curves) + 1)
    periods = np.array([c.truth.get("period", rng.uniform(0.2, 1.0)) for c in curves])
    plan.batch_setup(so, po)
    t = torch.tensor(np.concatenate([c.t for c in curves]), dtype=torch.float64, device="cuda")
    f = torch.tensor(np.concatenate([c.flux for c in curves]), dtype=torch.float32, device="cuda")
    pp = torch.tensor(periods, dtype=torch.float64, device="cuda")
    z = torch.empty((len(curves), 256), dtype=torch.uint16, device="cuda")
    _say("training folds via batch")
    plan.batch_fold_score(t, f, pp, 256, zfold=z)
    labels = torch.tensor([c.truth["label"] for c in curves], dtype=torch.float32, device="cuda")
    net = _net(torch, CNN_BF16, synth.cnn_init(13))
    _say("cnn training 300 steps")
    first = net.backward(z, labels).item()
    for _ in range(300):
        net.train_step(z, labels, 1e-3)
    last = net.backward(z, labels).item()
    print(f"training loss {first:.4f} -> {last:.4f}")
    assert last < 0.5 * first


def test_fp8_forward_error(torch_dev):
    """FP8 E4M3 inference after calibration: error against FP64 printed and
    bounded; an uncalibrated FP8 call is rejected."""
    torch = torch_dev
    from paper_2312_02063_amd import CNN_BF16, GpfcError
    p = _params(15)
    xc, _ = _inputs(16, 256)
    x, _ = _inputs(17, 200)
    net = _net(torch, CNN_BF16, p)
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    with pytest.raises(GpfcError):
        net.forward_fp8(xt)
    _say("cnn fp8 calibrate + forward")
    net.calibrate_fp8(torch.tensor(xc, dtype=torch.float32, device="cuda"))
    z8 = net.forward_fp8(xt).cpu().numpy()
    zb = net.forward(xt).cpu().numpy()
    zo = oracle.cnn_forward(p, x)
    e8, eb = _rel(z8, zo), _rel(zb, zo)
    cc = np.corrcoef(z8, zo)[0, 1]
    print(f"fp8 forward relative L2 error vs FP64: {e8:.3e} (bf16 {eb:.3e}); correlation {cc:.5f}")
    # E4M3 keeps 3 fraction bits (unit roundoff 2^-4); each of the five matrix-core
    # layers rounds its activations and weights to it, and independent rounding
    # errors add in quadrature: about sqrt(5 * 2 / 3) * 2^-4 = 0.11 of the logits'
    # L2 norm, bounded here by 0.15.
    assert e8 < 0.15
    # The same bound on the logits' deviations from their mean: an error d with
    # |d| <= eps |a| keeps corr(a, a + d) >= (1 - eps) / (1 + eps). The random-init
    # network's logits vary little around their mean, so eps is several times 0.15.
    zc = zo - zo.mean()
    eps = 0.15 * np.linalg.norm(zo) / np.linalg.norm(zc)
    assert cc >= (1.0 - eps) / (1.0 + eps)


@pytest.mark.parametrize("B", [1, 7, 8, 9, 300, 4099, 65541])
def test_fused_inference_bit_identical(torch_dev, B):
    """The fused convolution-stack kernel against the layer-by-layer path:
    identical logits, ragged last tiles included (65,541 inputs: enough rows
    for the 256-row FC1 tiles, with a ragged last one)."""
    torch = torch_dev
    from paper_2312_02063_amd import CNN_BF16
    p = _params(19)
    x, _ = _inputs(20 + B, B)
    net = _net(torch, CNN_BF16, p, max_batch=max(B, 4099))
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    _say(f"cnn fused vs layered B={B}")
    zf = net.forward(xt).cpu().numpy()
    net.set_fused(False)
    zl = net.forward(xt).cpu().numpy()
    net.set_fused(True)
    xb = xt.to(torch.bfloat16).view(torch.uint16)
    zfb = net.forward(xb).cpu().numpy()
    net.set_fused(False)
    zlb = net.forward(xb).cpu().numpy()
    assert np.array_equal(zf, zl)
    assert np.array_equal(zfb, zlb)
    net.set_fused(2)
    zr = net.forward(xt).cpu().numpy()
    net.set_fused(1)
    assert np.array_equal(zr, zl)
    # the FP64 oracle on at most 600 inputs (the first 512 and the ragged tail)
    rows = np.arange(B) if B <= 600 else np.r_[0:512, B - 88:B]
    zo = oracle.cnn_forward(p, x[rows])
    assert _rel(zf[rows], zo) < 5e-2


def test_captured_training_step_equals_eager(torch_dev):
    """Graph replays of a training step (new batches copied into the captured
    buffers each time) give the same parameters and losses as eager steps."""
    torch = torch_dev
    from paper_2312_02063_amd import CNN_BF16
    p = _params(21)
    B = 128
    xs = [torch.tensor(_inputs(30 + i, B)[0], dtype=torch.float32, device="cuda") for i in range(4)]
    ys = [torch.tensor(_inputs(30 + i, B)[1], dtype=torch.float32, device="cuda") for i in range(4)]
    eager = _net(torch, CNN_BF16, p)
    graph = _net(torch, CNN_BF16, p)
    xbuf = torch.empty_like(xs[0])
    ybuf = torch.empty_like(ys[0])
    _say("cnn training graph capture")
    loss_buf = graph.train_capture(xbuf, ybuf, 1e-3)
    torch.cuda.synchronize()
    for i in range(4):
        le = eager.train_step(xs[i], ys[i], 1e-3).item()
        xbuf.copy_(xs[i])
        ybuf.copy_(ys[i])
        lg = graph.train_replay().item()
        assert lg == le, (i, lg, le)
    torch.cuda.synchronize()
    assert torch.equal(eager.get_params(), graph.get_params())


def test_save_load_round_trip(torch_dev, tmp_path):
    """A saved network loads back bit for bit; files that are not network
    files (wrong tag, wrong count, short, missing) are refused with
    GPFC_EIO and leave the network unchanged."""
    torch = torch_dev
    from paper_2312_02063_amd import CNN_BF16
    from paper_2312_02063_amd._lib import EIO, GpfcError
    p = _params(31).astype(np.float32)
    a = _net(torch, CNN_BF16, p, 64)
    path = tmp_path / "net.gpfc"
    _say("cnn save/load")
    a.save(path)
    raw = path.read_bytes()
    assert raw[:8] == b"GPFCCNN1" and int.from_bytes(raw[8:16], "little") == p.size
    assert np.array_equal(np.frombuffer(raw[16:], dtype="<f4"), p)
    b = _net(torch, CNN_BF16, _params(32).astype(np.float32), 64)
    b.load(path)
    x = torch.tensor(_inputs(3, 50)[0], dtype=torch.float32, device="cuda")
    assert torch.equal(a.forward(x), b.forward(x))
    bad = {"tag": b"GPFCCNN0" + raw[8:], "count": raw[:8] + (5).to_bytes(8, "little") + raw[16:],
           "short": raw[:-4], "long": raw + b"\0\0\0\0"}
    for name, blob in bad.items():
        f = tmp_path / name
        f.write_bytes(blob)
        with pytest.raises(GpfcError) as e:
            b.load(f)
        assert e.value.code == EIO, name
    with pytest.raises(GpfcError) as e:
        b.load(tmp_path / "missing")
    assert e.value.code == EIO
    assert np.array_equal(b.get_params().cpu().numpy(), p)


def test_train_step_equals_backward_then_adam(torch_dev):
    torch = torch_dev
    from paper_2312_02063_amd import CNN_BF16
    p = _params(33)
    x, y = _inputs(34, 128)
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    yt = torch.tensor(y, dtype=torch.float32, device="cuda")
    a = _net(torch, CNN_BF16, p, 256)
    b = _net(torch, CNN_BF16, p, 256)
    _say("cnn train_step vs backward + adam")
    for _ in range(3):
        la = a.train_step(xt, yt, 1e-3).clone()
        lb = b.backward(xt, yt).clone()
        b.adam(1e-3)
        assert torch.equal(la, lb)
    assert torch.equal(a.get_params(), b.get_params())


@pytest.mark.parametrize("B,xbf16", [(1, False), (7, False), (257, False), (300, False), (5000, False),
                                     (300, True), (4099, True)])
def test_fused_training_matches_layer_path(torch_dev, B, xbf16):
    """A bf16 training step through the fused kernels (the convolution stack
    forward, which also writes the activations and pooling masks; the
    backward data gradients carried down the blocks in one pass; per-block
    weight gradients over groups of 8 inputs) against the same step layer by
    layer: the loss and the fully connected layers' gradients are identical
    bit for bit, the convolution gradients differ only by FP32 summation
    order (the data gradients they are formed from are bit-identical, so a
    relative difference above 1e-5 would mean a wrong term). Inputs in FP32
    or as bf16 bits (block 1's weight gradients read either form)."""
    torch = torch_dev
    from paper_2312_02063_amd import CNN_BF16
    p = _params(35)
    x, y = _inputs(36, B)
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    if xbf16:
        xt = xt.to(torch.bfloat16).view(torch.uint16)
    yt = torch.tensor(y, dtype=torch.float32, device="cuda")
    a = _net(torch, CNN_BF16, p, max(B, 512))
    b = _net(torch, CNN_BF16, p, max(B, 512))
    b.set_fused(False)
    _say(f"cnn fused vs layered backward B={B} bf16 input {xbf16}")
    ga = torch.empty(a.n_params, dtype=torch.float32, device="cuda")
    gb = torch.empty(b.n_params, dtype=torch.float32, device="cuda")
    la = a.backward(xt, yt, grad_out=ga).clone()
    lb = b.backward(xt, yt, grad_out=gb).clone()
    torch.cuda.synchronize()
    assert torch.equal(la, lb)
    ga = ga.cpu().numpy().astype(np.float64)
    gb = gb.cpu().numpy().astype(np.float64)
    for name, lo, hi in SEGMENTS:
        if name.startswith("fc"):
            assert np.array_equal(ga[lo:hi], gb[lo:hi]), name
        else:
            err = _rel(ga[lo:hi], gb[lo:hi])
            print(f"B={B} {name}: fused vs layer path relative difference {err:.2e}")
            assert err < 1e-5, name
    # and the same holds through training steps: losses stay within rounding
    for _ in range(2):
        la = a.train_step(xt, yt, 1e-3).item()
        lb = b.train_step(xt, yt, 1e-3).item()
        assert abs(la - lb) <= 1e-5 * max(1.0, abs(lb)), (la, lb)


def test_bf16_gradients_follow_fp32_at_large_batch(torch_dev):
    """The bf16 training kernels at a batch that splits every weight-gradient
    reduction over many blocks (ragged last range, XCD-grouped tiles, the
    block-4 staged pipeline) against the FP32 layer path, an independent code
    path: every parameter segment agrees to bf16 accuracy (a wrong tile, range
    or term would be off by O(1), a missing one of 16 batch ranges by ~6%;
    measured 0.3-1.5%), and the loss to 2e-2."""
    torch = torch_dev
    from paper_2312_02063_amd import CNN_BF16, CNN_FP32
    p = _params(41)
    B = 4099
    x, y = _inputs(42, B)
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    yt = torch.tensor(y, dtype=torch.float32, device="cuda")
    _say(f"cnn bf16 vs fp32 gradients B={B}")
    out = {}
    for prec in (CNN_BF16, CNN_FP32):
        net = _net(torch, prec, p, B)
        g = torch.empty(net.n_params, dtype=torch.float32, device="cuda")
        loss = net.backward(xt, yt, grad_out=g).item()
        torch.cuda.synchronize()
        out[prec] = (loss, g.cpu().numpy().astype(np.float64))
        net.close()
    lb, gb = out[CNN_BF16]
    lf, gf = out[CNN_FP32]
    assert abs(lb - lf) <= 2e-2 * max(1.0, abs(lf)), (lb, lf)
    for name, a, b in SEGMENTS:
        err = _rel(gb[a:b], gf[a:b])
        print(f"B={B} {name}: bf16 vs fp32 relative difference {err:.2e}")
        assert err < 0.05, name
