"""CPU oracle for the GPFC fold + box-SNR path (arXiv:2312.02063).

TEST INFRASTRUCTURE ONLY. The oracle is the plain, slow, FP64 statement of
what the GPU library computes. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
(``paper_2312_02063_amd``) never does, and the two share no code.

The arithmetic lives in ``gpfc_oracle.c`` (plain C, binary64,
``-ffp-contract=off``); this module compiles it with gcc and wraps it with
ctypes over numpy arrays. Each wrapper names the passage of the paper it
follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gpfc_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "cnn_oracle.c"), os.path.join(_HERE, "pnet_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build() -> str:
    """Compile the oracle with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, *_SRCS, "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS):
        build()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    ip = ctypes.POINTER(ctypes.c_int32)
    i64 = ctypes.c_int64
    i32 = ctypes.c_int32
    lib.oracle_curve_stats.argtypes = [dp, fp, i64, dp, dp, dp]
    lib.oracle_curve_stats.restype = None
    lib.oracle_bin.argtypes = [ctypes.c_double, ctypes.c_double, i32]
    lib.oracle_bin.restype = i32
    lib.oracle_fold.argtypes = [dp, fp, i64, dp, i64, i32, ctypes.c_double, dp, dp, ip, ctypes.c_int]
    lib.oracle_fold.restype = None
    lib.oracle_means.argtypes = [dp, ip, i64, dp]
    lib.oracle_means.restype = None
    lib.oracle_default_widths.argtypes = [i32, ip, i32]
    lib.oracle_default_widths.restype = i32
    lib.oracle_fold_eqcount.argtypes = [dp, fp, i64, dp, i64, i32, i32, dp]
    lib.oracle_fold_eqcount.restype = None
    lib.oracle_periodogram.argtypes = [fp, dp, i64, i64, ctypes.c_float, i32, i32, fp, fp, fp, ip, fp,
                                       ctypes.POINTER(ctypes.c_int64), ip, ip]
    lib.oracle_periodogram.restype = None
    lib.oracle_topk.argtypes = [fp, fp, ctypes.c_float, i64, i64, i32, fp,
                                ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_topk.restype = None
    lib.oracle_score.argtypes = [ip, dp, i64, i32, ctypes.c_double, ip, i32, dp, ip, ip, dp]
    lib.oracle_score.restype = None
    lib.oracle_box_snr.argtypes = [ip, dp, i32, ctypes.c_double, i32, i32]
    lib.oracle_box_snr.restype = ctypes.c_double
    lib.oracle_normalize.argtypes = [dp, ip, i64, i32, dp]
    lib.oracle_normalize.restype = None
    lib.oracle_cnn_nparams.argtypes = []
    lib.oracle_cnn_nparams.restype = i64
    lib.oracle_conv1d_circ.argtypes = [dp, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
    lib.oracle_conv1d_circ.restype = None
    lib.oracle_maxpool2.argtypes = [dp, ctypes.c_int, dp, ip]
    lib.oracle_maxpool2.restype = None
    lib.oracle_cnn_forward.argtypes = [dp, dp, ctypes.c_int, dp]
    lib.oracle_cnn_forward.restype = None
    lib.oracle_cnn_loss_grad.argtypes = [dp, dp, dp, ctypes.c_int, dp]
    lib.oracle_cnn_loss_grad.restype = ctypes.c_double
    lib.oracle_adam.argtypes = [dp, dp, dp, dp, i64, i64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double]
    lib.oracle_adam.restype = None
    lib.oracle_grid_size.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.oracle_grid_size.restype = ctypes.c_double
    cfgp = ctypes.POINTER(PnetCfg)
    lib.oracle_pnet_nparams.argtypes = [cfgp]
    lib.oracle_pnet_nparams.restype = i64
    lib.oracle_pnet_conv2d_circ.argtypes = [dp, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, dp]
    lib.oracle_pnet_conv2d_circ.restype = None
    lib.oracle_pnet_forward.argtypes = [cfgp, dp, dp, i64, dp, dp]
    lib.oracle_pnet_forward.restype = None
    lib.oracle_pnet_features.argtypes = [cfgp, dp, dp, dp, dp, dp]
    lib.oracle_pnet_features.restype = None
    lib.oracle_pnet_loss_grad.argtypes = [cfgp, dp, dp, dp, i64, dp, dp]
    lib.oracle_pnet_loss_grad.restype = ctypes.c_double
    _lib = lib
    return lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def curve_stats(t, flux):
    """Mean, sample std (ddof 1) and max |t| of a curve; sigma is Eq. 2's per-point noise."""
    lib = _load()
    t = _f64(t)
    flux = _f32(flux)
    m = ctypes.c_double()
    s = ctypes.c_double()
    tm = ctypes.c_double()
    lib.oracle_curve_stats(_p(t, ctypes.c_double), _p(flux, ctypes.c_float), t.size,
                           ctypes.byref(m), ctypes.byref(s), ctypes.byref(tm))
    return m.value, s.value, tm.value


def phase_bin(t: float, period: float, nbins: int) -> int:
    """Bin of one sample at one period (Sec. 2.3 steps one and two)."""
    return int(_load().oracle_bin(float(t), float(period), int(nbins)))


def fold(t, flux, periods, nbins, ref=None, nthreads=1):
    """Fold at every period (Sec. 2.3 steps one to three).

    Returns ``(sums, dsums, counts)`` of shape ``[k, nbins]``: FP64 flux sums,
    FP64 sums of ``flux - ref`` and int32 counts. ``ref`` defaults to the
    curve mean.
    """
    lib = _load()
    t = _f64(t)
    flux = _f32(flux)
    periods = _f64(periods)
    if t.size != flux.size:
        raise ValueError("t and flux differ in length")
    if ref is None:
        ref = curve_stats(t, flux)[0]
    k = periods.size
    sums = np.empty((k, nbins), np.float64)
    dsums = np.empty((k, nbins), np.float64)
    counts = np.empty((k, nbins), np.int32)
    lib.oracle_fold(_p(t, ctypes.c_double), _p(flux, ctypes.c_float), t.size,
                    _p(periods, ctypes.c_double), k, int(nbins), float(ref),
                    _p(sums, ctypes.c_double), _p(dsums, ctypes.c_double),
                    _p(counts, ctypes.c_int32), int(nthreads))
    return sums, dsums, counts


def means(sums, counts):
    """Bin means (Sec. 2.3 step five); NaN for empty bins."""
    lib = _load()
    sums = _f64(sums)
    counts = np.ascontiguousarray(counts, dtype=np.int32)
    out = np.empty_like(sums)
    lib.oracle_means(_p(sums, ctypes.c_double), _p(counts, ctypes.c_int32), sums.size,
                     _p(out, ctypes.c_double))
    return out


def default_widths(nbins: int):
    """Distinct integers nearest sqrt(2)^j in [1, nbins/2]."""
    lib = _load()
    buf = np.zeros(64, np.int32)
    m = lib.oracle_default_widths(int(nbins), _p(buf, ctypes.c_int32), 64)
    return buf[:m].copy()


def score(counts, dsums, sigma, widths=None):
    """Box-SNR of each folded row (Eq. 2 with the BLS box of Sec. 3.1).

    Returns ``(snr, start, width, depth)``.
    """
    lib = _load()
    counts = np.ascontiguousarray(counts, dtype=np.int32)
    dsums = _f64(dsums)
    k, nbins = counts.shape
    w = default_widths(nbins) if widths is None else np.ascontiguousarray(widths, dtype=np.int32)
    snr = np.empty(k, np.float64)
    depth = np.empty(k, np.float64)
    start = np.empty(k, np.int32)
    width = np.empty(k, np.int32)
    lib.oracle_score(_p(counts, ctypes.c_int32), _p(dsums, ctypes.c_double), k, nbins,
                     float(sigma), _p(w, ctypes.c_int32), w.size, _p(snr, ctypes.c_double),
                     _p(start, ctypes.c_int32), _p(width, ctypes.c_int32), _p(depth, ctypes.c_double))
    return snr, start, width, depth


def box_snr(counts_row, dsums_row, sigma, s, w):
    """The statistic of one box on one folded row."""
    lib = _load()
    c = np.ascontiguousarray(counts_row, dtype=np.int32)
    d = _f64(dsums_row)
    return lib.oracle_box_snr(_p(c, ctypes.c_int32), _p(d, ctypes.c_double), c.size,
                              float(sigma), int(s), int(w))


def normalize(sums, counts):
    """Noise-normalised folds for the learned scorer (Sec. 2.1): z-scores of the
    bin means over non-empty bins (ddof 0); empty bins and zero spread give 0."""
    lib = _load()
    sums = _f64(sums)
    counts = np.ascontiguousarray(counts, dtype=np.int32)
    k, nbins = sums.shape
    z = np.empty_like(sums)
    lib.oracle_normalize(_p(sums, ctypes.c_double), _p(counts, ctypes.c_int32), k, nbins,
                         _p(z, ctypes.c_double))
    return z


def grid_size(n_o: float, span: float, width: float) -> float:
    """Eq. 1 (Sec. 2.1): number of trial periods N_o * T / L."""
    return _load().oracle_grid_size(float(n_o), float(span), float(width))


def fold_score(t, flux, periods, nbins, widths=None, nthreads=1):
    """Whole path on the CPU: stats, fold, box-SNR. Returns a dict."""
    mean, sigma, _ = curve_stats(t, flux)
    sums, dsums, counts = fold(t, flux, periods, nbins, ref=mean, nthreads=nthreads)
    snr, start, width, depth = score(counts, dsums, sigma, widths)
    return dict(mean=mean, sigma=sigma, sums=sums, dsums=dsums, counts=counts,
                snr=snr, start=start, width=width, depth=depth)


# ---------------------------------------------------------------- learned scorer (Sec. 2.5)

def fold_eqcount(t, flux, periods, nbins=256, n_mid=4096):
    """The two-tier equal-count fold of Sec. 2.3 (steps 1-5, Fig. 4): mean
    flux of nbins final bins holding N / nbins points each, from n_mid
    equal-width intermediate bins split in proportion at the boundaries.
    Returns f64 [k, nbins]."""
    t = _f64(t)
    flux = _f32(flux)
    periods = _f64(np.atleast_1d(periods))
    k = periods.size
    means = np.empty((k, nbins), np.float64)
    _load().oracle_fold_eqcount(_p(t, ctypes.c_double), _p(flux, ctypes.c_float), t.size,
                                _p(periods, ctypes.c_double), k, n_mid, nbins,
                                _p(means, ctypes.c_double))
    return means


def periodogram(values, periods=None, nsigma=3.0, min_width=3, max_peaks=8):
    """SDE (Eq. 3), peaks above mean + nsigma sd wider than min_width points
    (Sec. 4.2) and harmonic codes of the best max_peaks peaks, per row of
    values f32 [rows, len]. Returns a dict of arrays."""
    v = np.ascontiguousarray(values, dtype=np.float32)
    if v.ndim == 1:
        v = v[None, :]
    rows, n = v.shape
    per = None if periods is None else _f64(periods)
    out = {"sde": np.empty(rows, np.float32), "mean": np.empty(rows, np.float32),
           "sd": np.empty(rows, np.float32), "n_peaks": np.empty(rows, np.int32),
           "val": np.empty((rows, max_peaks), np.float32), "idx": np.empty((rows, max_peaks), np.int64),
           "width": np.empty((rows, max_peaks), np.int32), "harmonic": np.empty((rows, max_peaks), np.int32)}
    _load().oracle_periodogram(_p(v, ctypes.c_float), None if per is None else _p(per, ctypes.c_double),
                               rows, n, ctypes.c_float(nsigma), min_width, max_peaks,
                               _p(out["sde"], ctypes.c_float), _p(out["mean"], ctypes.c_float),
                               _p(out["sd"], ctypes.c_float), _p(out["n_peaks"], ctypes.c_int32),
                               _p(out["val"], ctypes.c_float), _p(out["idx"], ctypes.c_int64),
                               _p(out["width"], ctypes.c_int32), _p(out["harmonic"], ctypes.c_int32))
    return out


def topk(values, top, gate=None, gate_min=0.0):
    """Per-row best `top` entries of a periodogram (Sec. 2.1, Sec. 3.2): value
    descending, then index ascending; NaN values and entries whose gate is not
    >= gate_min are skipped; missing places are (-inf, -1).
    values f32 [rows, len] -> (f32 [rows, top], int64 [rows, top])."""
    v = np.ascontiguousarray(values, dtype=np.float32)
    if v.ndim == 1:
        v = v[None, :]
    rows, n = v.shape
    g = None if gate is None else np.ascontiguousarray(gate, dtype=np.float32).reshape(rows, n)
    ov = np.empty((rows, top), np.float32)
    oi = np.empty((rows, top), np.int64)
    _load().oracle_topk(_p(v, ctypes.c_float), None if g is None else _p(g, ctypes.c_float),
                        ctypes.c_float(gate_min), rows, n, top, _p(ov, ctypes.c_float),
                        _p(oi, ctypes.c_int64))
    return ov, oi


def cnn_nparams() -> int:
    return int(_load().oracle_cnn_nparams())


def conv1d_circ(x, w, b):
    """Circular conv1d, padding 2 by wrap-around: x [B][Cin][L], w [Cout][Cin][5], b [Cout]."""
    lib = _load()
    x = _f64(x)
    w = _f64(w)
    b = _f64(b)
    B, Cin, L = x.shape
    Cout = w.shape[0]
    y = np.empty((B, Cout, L))
    lib.oracle_conv1d_circ(_p(x, ctypes.c_double), _p(w, ctypes.c_double), _p(b, ctypes.c_double),
                           B, Cin, Cout, L, _p(y, ctypes.c_double))
    return y


def maxpool2(r):
    """Max-pool by 2 with the winner index (first on a tie)."""
    lib = _load()
    r = _f64(r)
    out = np.empty(r.size // 2)
    idx = np.empty(r.size // 2, np.int32)
    lib.oracle_maxpool2(_p(r, ctypes.c_double), out.size, _p(out, ctypes.c_double),
                        _p(idx, ctypes.c_int32))
    return out, idx


def cnn_forward(params, x):
    """Logits of the network for inputs x [B][256] (FP64)."""
    lib = _load()
    params = _f64(params)
    x = _f64(x)
    B = x.shape[0]
    out = np.empty(B)
    lib.oracle_cnn_forward(_p(params, ctypes.c_double), _p(x, ctypes.c_double), B,
                           _p(out, ctypes.c_double))
    return out


def cnn_loss_grad(params, x, y):
    """(mean BCE-with-logits loss, gradient [312449]) for inputs x [B][256], labels y [B]."""
    lib = _load()
    params = _f64(params)
    x = _f64(x)
    y = _f64(y)
    g = np.empty(params.size)
    loss = lib.oracle_cnn_loss_grad(_p(params, ctypes.c_double), _p(x, ctypes.c_double),
                                    _p(y, ctypes.c_double), x.shape[0], _p(g, ctypes.c_double))
    return loss, g


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step in place on p, m, v (FP64 arrays)."""
    lib = _load()
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    lib.oracle_adam(_p(p, ctypes.c_double), _p(g, ctypes.c_double), _p(m, ctypes.c_double),
                    _p(v, ctypes.c_double), p.size, int(step), float(lr), float(b1), float(b2),
                    float(eps))


# ---------------------------------------------------------------- the paper's network (Sec. 2.5)

class PnetCfg(ctypes.Structure):
    """Sizes of the paper's network (pnet_oracle.c): image side S, filters
    F1, F2 (= S*S), F3, F4, kernel sides K1, K2, hidden units H."""
    _fields_ = [(n, ctypes.c_int32) for n in ("S", "F1", "F2", "F3", "F4", "K1", "K2", "H")]


PNET_FULL = dict(S=16, F1=128, F2=256, F3=128, F4=256, K1=3, K2=5, H=128)


def _cfg(cfg):
    c = PnetCfg(**(cfg or PNET_FULL))
    assert c.F2 == c.S * c.S, "F2 must equal S*S (the pooled values form an S x S image)"
    return c


def pnet_nparams(cfg=None) -> int:
    c = _cfg(cfg)
    return int(_load().oracle_pnet_nparams(ctypes.byref(c)))


def pnet_conv2d_circ(x, w, b):
    """Circular 2-D convolution (cross-correlation, wrap-around padding, same
    size): x [Ci][S][S], w [Co][Ci][K][K], b [Co] -> [Co][S][S]."""
    x, w, b = _f64(x), _f64(w), _f64(b)
    ci, S, _ = x.shape
    co, _, K, _ = w.shape
    y = np.empty((co, S, S))
    _load().oracle_pnet_conv2d_circ(_p(x, ctypes.c_double), _p(w, ctypes.c_double),
                                    _p(b, ctypes.c_double), ci, co, K, S, _p(y, ctypes.c_double))
    return y


def pnet_forward(params, x, cfg=None, mask=None):
    """Logits of the paper's network for inputs x [B][S*S]; mask [B][H] is
    the dropout keep mask already scaled by 1/(1 - rate) (None: inference)."""
    c = _cfg(cfg)
    params, x = _f64(params), _f64(x)
    B = x.shape[0]
    out = np.empty(B)
    m = None if mask is None else _f64(mask)
    _load().oracle_pnet_forward(ctypes.byref(c), _p(params, ctypes.c_double), _p(x, ctypes.c_double), B,
                                None if m is None else _p(m, ctypes.c_double), _p(out, ctypes.c_double))
    return out


def pnet_features(params, x, cfg=None):
    """First and second global max-pool outputs and the hidden layer of one
    input x [S*S]: (g1 [F2], g2 [F4], h [H])."""
    c = _cfg(cfg)
    params, x = _f64(params), _f64(x)
    g1, g2, h = np.empty(c.F2), np.empty(c.F4), np.empty(c.H)
    _load().oracle_pnet_features(ctypes.byref(c), _p(params, ctypes.c_double), _p(x, ctypes.c_double),
                                 _p(g1, ctypes.c_double), _p(g2, ctypes.c_double), _p(h, ctypes.c_double))
    return g1, g2, h


def pnet_loss_grad(params, x, y, cfg=None, mask=None):
    """(mean BCE-with-logits loss, gradient) of the paper's network."""
    c = _cfg(cfg)
    params, x, y = _f64(params), _f64(x), _f64(y)
    g = np.empty(params.size)
    m = None if mask is None else _f64(mask)
    loss = _load().oracle_pnet_loss_grad(ctypes.byref(c), _p(params, ctypes.c_double),
                                         _p(x, ctypes.c_double), _p(y, ctypes.c_double), x.shape[0],
                                         None if m is None else _p(m, ctypes.c_double),
                                         _p(g, ctypes.c_double))
    return loss, g


def pnet_split(params, cfg=None):
    """The flat parameter vector as named arrays (views)."""
    c = cfg or PNET_FULL
    S, F1, F2, F3, F4, K1, K2, H = (c[k] for k in ("S", "F1", "F2", "F3", "F4", "K1", "K2", "H"))
    shapes = [("w1", (F1, 1, K1, K1)), ("b1", (F1,)), ("w2", (F2, F1, K1, K1)), ("b2", (F2,)),
              ("w3", (F3, 1, K2, K2)), ("b3", (F3,)), ("w4", (F4, F3, K2, K2)), ("b4", (F4,)),
              ("w5", (H, F4)), ("b5", (H,)), ("w6", (H,)), ("b6", (1,))]
    out, o = {}, 0
    for name, shp in shapes:
        n = int(np.prod(shp))
        out[name] = params[o:o + n].reshape(shp)
        o += n
    assert o == params.size
    return out
