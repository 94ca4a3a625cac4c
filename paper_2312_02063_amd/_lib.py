"""ctypes binding of ``libgpfc.so`` (the C ABI in ``include/gpfc.h``).

Argument marshalling only: every step of the fold and the score runs in the
library's HIP kernels. Tensors are torch tensors on the plan's GPU; outputs
are allocated here with ``torch.empty`` and filled by the library on the
current torch stream. If the library is missing this module raises: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpfc.so")

OK, EINVAL, ENOTSUP, ERANGE, ENOMEM, EDEVICE, EIO = 0, -1, -2, -3, -4, -5, -6
MAX_SAMPLES = 2147483647
MAX_PACKED = 262143
MAX_NBINS = 4096
FUSED_MAX_NBINS = 256
MAX_WIDTHS = 24

_lib = None


class GpfcError(RuntimeError):
    def __init__(self, code: int, what: str):
        lib = load()
        msg = lib.gpfc_strerror(code).decode()
        if code == EDEVICE:
            err = (lib.gpfc_cnn_last_error() if what.startswith("gpfc_cnn") else lib.gpfc_last_error())
            msg += ": " + err.decode()
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


class Curve(ctypes.Structure):
    """Host mirror of ``gpfc_curve``."""
    _fields_ = [("mean", ctypes.c_double), ("sigma", ctypes.c_double), ("ref", ctypes.c_double),
                ("qscale", ctypes.c_double), ("tmax", ctypes.c_double), ("maxdev", ctypes.c_double),
                ("n", ctypes.c_int64), ("exact", ctypes.c_int32), ("finite", ctypes.c_int32),
                ("words", ctypes.c_int32), ("pad", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


class PlanOpts(ctypes.Structure):
    """Host mirror of ``gpfc_plan_opts``."""
    _fields_ = [("device", ctypes.c_int32), ("nw", ctypes.c_int32),
                ("widths", ctypes.c_int32 * MAX_WIDTHS), ("split", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("tune_cache", ctypes.c_char_p),
                ("workspace_bytes", ctypes.c_int64)]


class DetrendOpts(ctypes.Structure):
    """Host mirror of ``gpfc_detrend_opts``."""
    _fields_ = [("cadence", ctypes.c_double), ("gap_cadences", ctypes.c_double),
                ("jump_sigma", ctypes.c_double), ("clip_sigma", ctypes.c_double),
                ("edge", ctypes.c_int32), ("max_fits", ctypes.c_int32), ("n_spacings", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("spacings", ctypes.c_double * 8)]


class DetrendInfo(ctypes.Structure):
    """Host mirror of ``gpfc_detrend_info``."""
    _fields_ = [("n_segments", ctypes.c_int32), ("n_kept_segments", ctypes.c_int32),
                ("status", ctypes.c_int32), ("pad", ctypes.c_int32)]


class SurveyOut(ctypes.Structure):
    """Host mirror of ``gpfc_survey_out`` (device pointers)."""
    _fields_ = [("snr", ctypes.c_void_p), ("start", ctypes.c_void_p), ("width", ctypes.c_void_p),
                ("depth", ctypes.c_void_p), ("logits", ctypes.c_void_p), ("cnn_fp8", ctypes.c_int32),
                ("top", ctypes.c_int32), ("box_val", ctypes.c_void_p), ("box_idx", ctypes.c_void_p),
                ("cnn_val", ctypes.c_void_p), ("cnn_idx", ctypes.c_void_p),
                ("judge_snr", ctypes.c_float), ("judged_val", ctypes.c_void_p),
                ("judged_idx", ctypes.c_void_p)]


def load():
    """Load ``libgpfc.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2312_02063_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "gpfc_version": ([], i32),
        "gpfc_strerror": ([i32], ctypes.c_char_p),
        "gpfc_last_error": ([], ctypes.c_char_p),
        "gpfc_plan_create": ([ctypes.POINTER(vp), i32], i32),
        "gpfc_plan_create_opts": ([ctypes.POINTER(vp), ctypes.POINTER(PlanOpts)], i32),
        "gpfc_plan_destroy": ([vp], i32),
        "gpfc_plan_set_widths": ([vp, ctypes.POINTER(ctypes.c_int32), i32], i32),
        "gpfc_curve_stats": ([vp, vp, vp, i64, ctypes.POINTER(Curve), vp], i32),
        "gpfc_fold": ([vp, vp, vp, i64, vp, i64, i32, vp, vp, vp, vp], i32),
        "gpfc_score": ([vp, vp, vp, i64, i32, f64, vp, vp, vp, vp, vp], i32),
        "gpfc_fold_score": ([vp, vp, vp, i64, vp, i64, i32, vp, vp, vp, vp, vp], i32),
        "gpfc_fold_naive": ([vp, vp, vp, i64, vp, i64, i32, vp, vp, vp], i32),
        "gpfc_prepare": ([vp, vp, vp, i64, vp], i32),
        "gpfc_fold_prepared": ([vp, vp, i64, i32, vp, vp, vp, vp], i32),
        "gpfc_fold_score_prepared": ([vp, vp, i64, i32, vp, vp, vp, vp, vp, vp], i32),
        "gpfc_fold_f32_prepared": ([vp, vp, i64, i32, i32, vp, vp, vp, vp], i32),
        "gpfc_batch_setup": ([vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64), i32], i32),
        "gpfc_batch_fold_score": ([vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp], i32),
        "gpfc_batch_capture": ([vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp], i32),
        "gpfc_batch_replay": ([vp, vp], i32),
        "gpfc_batch_curve_stats": ([vp, ctypes.POINTER(Curve), vp], i32),
        "gpfc_sync": ([vp], i32),
        "gpfc_topk": ([vp, i64, i64, vp, ctypes.c_float, i32, vp, vp, vp], i32),
        "gpfc_plan_set_split": ([vp, i32], i32),
        "gpfc_fold_eqcount_prepared": ([vp, vp, i64, i32, vp, vp, vp], i32),
        "gpfc_periodogram_peaks": ([vp, i64, i64, vp, ctypes.c_float, i32, i32, vp, vp, vp, vp, vp, vp,
                                    vp, vp, vp], i32),
        "gpfc_autotune": ([vp, vp, i64, i32, ctypes.c_char_p, ctypes.POINTER(i32),
                           ctypes.POINTER(ctypes.c_float), vp], i32),
        "gpfc_survey_setup": ([vp, ctypes.POINTER(ctypes.c_int64), i32, i64, i64], i32),
        "gpfc_survey_run": ([vp, vp, vp, vp, vp, i32, ctypes.POINTER(SurveyOut), vp], i32),
        "gpfc_survey_capture": ([vp, vp, vp, vp, vp, i32, ctypes.POINTER(SurveyOut), vp], i32),
        "gpfc_cnn_nparams": ([], i32),
        "gpfc_cnn_last_error": ([], ctypes.c_char_p),
        "gpfc_cnn_create": ([ctypes.POINTER(vp), i32, i32, i64], i32),
        "gpfc_cnn_destroy": ([vp], i32),
        "gpfc_cnn_set_params": ([vp, vp, vp], i32),
        "gpfc_cnn_get_params": ([vp, vp, vp], i32),
        "gpfc_cnn_set_fused": ([vp, i32], i32),
        "gpfc_cnn_forward": ([vp, vp, i32, i64, vp, vp], i32),
        "gpfc_cnn_backward": ([vp, vp, i32, vp, i64, vp, vp, vp], i32),
        "gpfc_cnn_adam": ([vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp], i32),
        "gpfc_cnn_calibrate_fp8": ([vp, vp, i32, i64, i32, vp], i32),
        "gpfc_cnn_forward_fp8": ([vp, vp, i32, i64, vp, vp], i32),
        "gpfc_cnn_train_capture": ([vp, vp, i32, vp, i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, vp, vp], i32),
        "gpfc_cnn_train_replay": ([vp, vp], i32),
        "gpfc_cnn_train_step": ([vp, vp, i32, vp, i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, vp, vp], i32),
        "gpfc_cnn_save": ([vp, ctypes.c_char_p, vp], i32),
        "gpfc_roof_probe": ([i32, i32, ctypes.POINTER(f64), ctypes.POINTER(f64), vp], i32),
        "gpfc_cnn_load": ([vp, ctypes.c_char_p, vp], i32),
        "gpfc_fold_score_noalloc": ([vp, vp, i64, vp, i64, i32, vp, vp, vp, vp, vp], i32),
        "gpfc_detrend": ([vp, vp, vp, vp, i64, ctypes.POINTER(DetrendOpts), vp, vp,
                          ctypes.POINTER(DetrendInfo), vp], i32),
        "gpfc_survey_autotune": ([vp, vp, ctypes.POINTER(ctypes.c_int64), i32, vp, vp, vp, i64, i32,
                                  ctypes.POINTER(ctypes.c_int64), i32, ctypes.POINTER(ctypes.c_int64), i32,
                                  ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_float), vp], i32),
        "gpfc_pnet_nparams": ([], i32),
        "gpfc_pnet_last_error": ([], ctypes.c_char_p),
        "gpfc_pnet_create": ([ctypes.POINTER(vp), i32, i32, i64], i32),
        "gpfc_pnet_destroy": ([vp], i32),
        "gpfc_pnet_set_fused": ([vp, i32], i32),
        "gpfc_pnet_set_params": ([vp, vp, vp], i32),
        "gpfc_pnet_get_params": ([vp, vp, vp], i32),
        "gpfc_pnet_forward": ([vp, vp, i32, i64, vp, vp], i32),
        "gpfc_pnet_backward": ([vp, vp, i32, vp, vp, i64, vp, vp, vp], i32),
        "gpfc_pnet_get_grads": ([vp, vp, vp], i32),
        "gpfc_pnet_adam": ([vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def exported_symbols():
    """Names the C ABI declares (see include/gpfc.h)."""
    return ["gpfc_version", "gpfc_strerror", "gpfc_last_error", "gpfc_plan_create",
            "gpfc_plan_create_opts",
            "gpfc_plan_destroy", "gpfc_plan_set_widths", "gpfc_curve_stats", "gpfc_fold",
            "gpfc_score", "gpfc_fold_score", "gpfc_fold_naive", "gpfc_sync", "gpfc_prepare",
            "gpfc_fold_prepared", "gpfc_fold_score_prepared", "gpfc_fold_f32_prepared",
            "gpfc_batch_setup",
            "gpfc_batch_fold_score", "gpfc_batch_capture", "gpfc_batch_replay",
            "gpfc_batch_curve_stats", "gpfc_cnn_nparams", "gpfc_cnn_last_error",
            "gpfc_cnn_create", "gpfc_cnn_destroy", "gpfc_cnn_set_params", "gpfc_cnn_get_params",
            "gpfc_cnn_forward", "gpfc_cnn_backward", "gpfc_cnn_adam", "gpfc_cnn_calibrate_fp8",
            "gpfc_cnn_forward_fp8", "gpfc_cnn_set_fused", "gpfc_cnn_train_capture",
            "gpfc_cnn_train_replay", "gpfc_topk", "gpfc_plan_set_split",
            "gpfc_autotune", "gpfc_fold_eqcount_prepared", "gpfc_periodogram_peaks", "gpfc_survey_setup", "gpfc_survey_run",
            "gpfc_survey_capture", "gpfc_cnn_train_step", "gpfc_cnn_save", "gpfc_cnn_load",
            "gpfc_roof_probe", "gpfc_fold_score_noalloc", "gpfc_pnet_nparams", "gpfc_pnet_last_error",
            "gpfc_pnet_create", "gpfc_pnet_destroy", "gpfc_pnet_set_fused", "gpfc_pnet_set_params", "gpfc_pnet_get_params",
            "gpfc_pnet_forward", "gpfc_pnet_backward", "gpfc_pnet_get_grads", "gpfc_pnet_adam",
            "gpfc_detrend", "gpfc_survey_autotune"]


ROOF_LDS_U64, ROOF_LDS_U32, ROOF_LDS_F32, ROOF_FP64_FMA, ROOF_HBM_COPY = 0, 1, 2, 3, 4


def roof_probe(kind: int, device: int = 0):
    """(rate, ms) of one roofline micro-benchmark (see gpfc_roof_probe)."""
    rate = ctypes.c_double(0.0)
    ms = ctypes.c_double(0.0)
    _check(load().gpfc_roof_probe(device, int(kind), ctypes.byref(rate), ctypes.byref(ms), _stream()),
           "gpfc_roof_probe")
    return rate.value, ms.value


def _check(rc, what):
    if rc != OK:
        raise GpfcError(rc, what)


def _ptr(x):
    return ctypes.c_void_p(x.data_ptr()) if x is not None else None


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(x, dtype, name, dev):
    import torch
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {x.dtype}")
    if x.device != dev:
        raise ValueError(f"{name} is on {x.device}, expected {dev}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Plan:
    """A library plan on one GPU (owns the device workspace and the width set)."""

    def __init__(self, device: int = 0, widths=None, split: int = 0, tune_cache: str | None = None,
                 workspace_bytes: int = 0):
        import torch
        self.lib = load()
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        if split or tune_cache or workspace_bytes:
            w = list(widths or [])
            o = PlanOpts(device=device, nw=len(w), split=int(split),
                         tune_cache=tune_cache.encode() if tune_cache else None,
                         workspace_bytes=int(workspace_bytes))
            for i, x in enumerate(w):
                o.widths[i] = int(x)
            _check(self.lib.gpfc_plan_create_opts(ctypes.byref(h), ctypes.byref(o)),
                   "gpfc_plan_create_opts")
            self.h = h
            return
        _check(self.lib.gpfc_plan_create(ctypes.byref(h), device), "gpfc_plan_create")
        self.h = h
        if widths is not None:
            self.set_widths(widths)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.gpfc_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_widths(self, widths):
        w = list(widths or [])
        arr = (ctypes.c_int32 * max(1, len(w)))(*w)
        _check(self.lib.gpfc_plan_set_widths(self.h, arr, len(w)), "gpfc_plan_set_widths")

    def _inputs(self, t, flux, periods=None):
        import torch
        _need(t, torch.float64, "t", self.device)
        _need(flux, torch.float32, "flux", self.device)
        if t.numel() != flux.numel():
            raise ValueError("t and flux differ in length")
        if periods is not None:
            _need(periods, torch.float64, "periods", self.device)

    def curve_stats(self, t, flux) -> dict:
        self._inputs(t, flux)
        c = Curve()
        _check(self.lib.gpfc_curve_stats(self.h, _ptr(t), _ptr(flux), t.numel(), ctypes.byref(c),
                                         _stream()), "gpfc_curve_stats")
        return c.as_dict()

    def fold(self, t, flux, periods, nbins: int, means: bool = True):
        """(sums f64[k, nbins], counts i32[k, nbins], means f64[k, nbins] or None)."""
        import torch
        self._inputs(t, flux, periods)
        k = periods.numel()
        sums = torch.empty((k, nbins), dtype=torch.float64, device=self.device)
        counts = torch.empty((k, nbins), dtype=torch.int32, device=self.device)
        mo = torch.empty((k, nbins), dtype=torch.float64, device=self.device) if means else None
        _check(self.lib.gpfc_fold(self.h, _ptr(t), _ptr(flux), t.numel(), _ptr(periods), k, nbins,
                                  _ptr(sums), _ptr(counts), _ptr(mo), _stream()), "gpfc_fold")
        return sums, counts, mo

    def _score_outputs(self, k):
        import torch
        return (torch.empty(k, dtype=torch.float32, device=self.device),
                torch.empty(k, dtype=torch.int32, device=self.device),
                torch.empty(k, dtype=torch.int32, device=self.device),
                torch.empty(k, dtype=torch.float32, device=self.device))

    def score(self, sums, counts, sigma: float):
        """Box-SNR of materialised folds: (snr f32[k], start i32[k], width i32[k], depth f32[k])."""
        import torch
        _need(sums, torch.float64, "sums", self.device)
        _need(counts, torch.int32, "counts", self.device)
        if sums.dim() != 2 or sums.shape != counts.shape:
            raise ValueError("sums and counts must both be [k, nbins]")
        k, nbins = sums.shape
        snr, start, width, depth = self._score_outputs(k)
        _check(self.lib.gpfc_score(self.h, _ptr(sums), _ptr(counts), k, nbins, float(sigma),
                                   _ptr(snr), _ptr(start), _ptr(width), _ptr(depth), _stream()),
               "gpfc_score")
        return snr, start, width, depth

    def fold_score(self, t, flux, periods, nbins: int, out=None):
        """Fused fold + box-SNR: (snr, start, width, depth), each [k]."""
        self._inputs(t, flux, periods)
        k = periods.numel()
        snr, start, width, depth = out if out is not None else self._score_outputs(k)
        _check(self.lib.gpfc_fold_score(self.h, _ptr(t), _ptr(flux), t.numel(), _ptr(periods), k,
                                        nbins, _ptr(snr), _ptr(start), _ptr(width), _ptr(depth),
                                        _stream()), "gpfc_fold_score")
        return snr, start, width, depth

    def prepare(self, t, flux):
        """Prepare a curve in the plan for the *_prepared folds."""
        self._inputs(t, flux)
        _check(self.lib.gpfc_prepare(self.h, _ptr(t), _ptr(flux), t.numel(), _stream()),
               "gpfc_prepare")

    def fold_prepared(self, periods, nbins: int, means: bool = True):
        import torch
        _need(periods, torch.float64, "periods", self.device)
        k = periods.numel()
        sums = torch.empty((k, nbins), dtype=torch.float64, device=self.device)
        counts = torch.empty((k, nbins), dtype=torch.int32, device=self.device)
        mo = torch.empty((k, nbins), dtype=torch.float64, device=self.device) if means else None
        _check(self.lib.gpfc_fold_prepared(self.h, _ptr(periods), k, nbins, _ptr(sums),
                                           _ptr(counts), _ptr(mo), _stream()), "gpfc_fold_prepared")
        return sums, counts, mo

    def fold_f32_prepared(self, periods, nbins: int, compensated: bool):
        """Fold of the prepared curve with FP32 (optionally TwoSum-compensated) bin sums."""
        import torch
        _need(periods, torch.float64, "periods", self.device)
        k = periods.numel()
        sums = torch.empty((k, nbins), dtype=torch.float64, device=self.device)
        counts = torch.empty((k, nbins), dtype=torch.int32, device=self.device)
        means = torch.empty((k, nbins), dtype=torch.float64, device=self.device)
        _check(self.lib.gpfc_fold_f32_prepared(self.h, _ptr(periods), k, nbins, int(compensated),
                                               _ptr(sums), _ptr(counts), _ptr(means), _stream()),
               "gpfc_fold_f32_prepared")
        return sums, counts, means

    def fold_score_prepared(self, periods, nbins: int, out=None, zfold=None):
        """Fused fold + score on the prepared curve; ``zfold`` (optional uint16
        tensor [k, nbins]) receives the normalised folds as bfloat16 bits."""
        import torch
        _need(periods, torch.float64, "periods", self.device)
        k = periods.numel()
        snr, start, width, depth = out if out is not None else self._score_outputs(k)
        if zfold is not None:
            _need(zfold, torch.uint16, "zfold", self.device)
            if zfold.numel() != k * nbins:
                raise ValueError("zfold must hold k * nbins values")
        _check(self.lib.gpfc_fold_score_prepared(self.h, _ptr(periods), k, nbins, _ptr(snr),
                                                 _ptr(start), _ptr(width), _ptr(depth),
                                                 _ptr(zfold), _stream()),
               "gpfc_fold_score_prepared")
        return snr, start, width, depth

    # ---------------------------------------------------------------- batches

    def batch_setup(self, sample_offsets, period_offsets):
        """Describe a batch of curves by host offsets (length n_curves + 1, from 0)."""
        so = [int(x) for x in sample_offsets]
        po = [int(x) for x in period_offsets]
        if len(so) != len(po) or len(so) < 1:
            raise ValueError("offset arrays must both have n_curves + 1 entries")
        a = (ctypes.c_int64 * len(so))(*so)
        b = (ctypes.c_int64 * len(po))(*po)
        _check(self.lib.gpfc_batch_setup(self.h, a, b, len(so) - 1), "gpfc_batch_setup")
        self.batch_n = len(so) - 1
        self.batch_k = po[-1]
        self.batch_samples = so[-1]

    def _batch_args(self, t, flux, periods, nbins, out, zfold):
        import torch
        _need(t, torch.float64, "t", self.device)
        _need(flux, torch.float32, "flux", self.device)
        _need(periods, torch.float64, "periods", self.device)
        if t.numel() != self.batch_samples or flux.numel() != self.batch_samples:
            raise ValueError("t / flux do not match the batch's sample offsets")
        if periods.numel() != self.batch_k:
            raise ValueError("periods do not match the batch's period offsets")
        outs = out if out is not None else self._score_outputs(self.batch_k)
        if zfold is not None:
            _need(zfold, torch.uint16, "zfold", self.device)
            if zfold.numel() != self.batch_k * nbins:
                raise ValueError("zfold must hold total periods * nbins values")
        return outs

    def batch_fold_score(self, t, flux, periods, nbins: int, out=None, zfold=None):
        snr, start, width, depth = self._batch_args(t, flux, periods, nbins, out, zfold)
        _check(self.lib.gpfc_batch_fold_score(self.h, _ptr(t), _ptr(flux), _ptr(periods), nbins,
                                              _ptr(snr), _ptr(start), _ptr(width), _ptr(depth),
                                              _ptr(zfold), _stream()), "gpfc_batch_fold_score")
        return snr, start, width, depth

    def batch_capture(self, t, flux, periods, nbins: int, out=None, zfold=None):
        """Capture the batch pipeline into a HIP graph on the current (non-default) stream."""
        snr, start, width, depth = self._batch_args(t, flux, periods, nbins, out, zfold)
        self._graph_keep = (t, flux, periods, snr, start, width, depth, zfold)
        _check(self.lib.gpfc_batch_capture(self.h, _ptr(t), _ptr(flux), _ptr(periods), nbins,
                                           _ptr(snr), _ptr(start), _ptr(width), _ptr(depth),
                                           _ptr(zfold), _stream()), "gpfc_batch_capture")
        return snr, start, width, depth

    def batch_replay(self):
        _check(self.lib.gpfc_batch_replay(self.h, _stream()), "gpfc_batch_replay")

    def batch_curve_stats(self):
        arr = (Curve * max(1, self.batch_n))()
        _check(self.lib.gpfc_batch_curve_stats(self.h, arr, _stream()), "gpfc_batch_curve_stats")
        return [arr[i].as_dict() for i in range(self.batch_n)]

    def fold_eqcount_prepared(self, periods, nbins: int = 256, means: bool = True, zfold=None):
        """The two-tier equal-count fold of the prepared curve: means f64 [k, nbins]
        (None if means=False) and, if given, zfold u16 [k, nbins] filled."""
        import torch
        _need(periods, torch.float64, "periods", self.device)
        k = periods.numel()
        m = torch.empty((k, nbins), dtype=torch.float64, device=self.device) if means else None
        if zfold is not None:
            _need(zfold, torch.uint16, "zfold", self.device)
            if zfold.numel() != k * nbins:
                raise ValueError("zfold must hold k * nbins values")
        _check(self.lib.gpfc_fold_eqcount_prepared(self.h, _ptr(periods), k, nbins, _ptr(m), _ptr(zfold),
                                                   _stream()), "gpfc_fold_eqcount_prepared")
        return m

    def set_split(self, split: int):
        """Sample split of the single-curve fold + score (0: automatic)."""
        _check(self.lib.gpfc_plan_set_split(self.h, int(split)), "gpfc_plan_set_split")

    def autotune(self, periods, nbins: int, cache_path: str | None = None):
        """Time the block shapes for the prepared curve at these periods; returns (split, ms)."""
        import torch
        _need(periods, torch.float64, "periods", self.device)
        sp = ctypes.c_int32(0)
        ms = ctypes.c_float(0.0)
        _check(self.lib.gpfc_autotune(self.h, _ptr(periods), periods.numel(), nbins,
                                      cache_path.encode() if cache_path else None,
                                      ctypes.byref(sp), ctypes.byref(ms), _stream()), "gpfc_autotune")
        return sp.value, ms.value

    # ---------------------------------------------------------------- surveys

    def survey_setup(self, sample_offsets, k: int, chunk_folds: int = 0):
        """Curves cut from concatenated t / flux by host offsets, all folded at
        the same k periods; chunk_folds > 0 reserves the workspace the network
        needs (curves are taken max(1, chunk_folds // k) at a time)."""
        so = [int(x) for x in sample_offsets]
        a = (ctypes.c_int64 * len(so))(*so)
        _check(self.lib.gpfc_survey_setup(self.h, a, len(so) - 1, int(k), int(chunk_folds)),
               "gpfc_survey_setup")
        self.survey_n = len(so) - 1
        self.survey_k = int(k)
        self.survey_samples = so[-1]

    def survey_autotune(self, sample_offsets, t, flux, periods, nbins: int = 256, cnn=None,
                        chunks=(2_000_000, 4_000_000, 8_000_000), nets=(), cache_path: str | None = None):
        """Time the survey's chunk sizes and network pass sizes, keep the fastest
        (the plan is left set up with it); returns (chunk, net_batch, ms)."""
        import torch
        _need(t, torch.float64, "t", self.device)
        _need(flux, torch.float32, "flux", self.device)
        _need(periods, torch.float64, "periods", self.device)
        so = [int(x) for x in sample_offsets]
        a = (ctypes.c_int64 * len(so))(*so)
        ch = (ctypes.c_int64 * len(chunks))(*[int(c) for c in chunks])
        nt = (ctypes.c_int64 * max(1, len(nets)))(*([int(v) for v in nets] or [0]))
        co, no, ms = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_float(0.0)
        _check(self.lib.gpfc_survey_autotune(self.h, cnn.h if cnn is not None else None, a, len(so) - 1,
                                             _ptr(t), _ptr(flux), _ptr(periods), periods.numel(), nbins,
                                             ch, len(chunks), nt, len(nets),
                                             cache_path.encode() if cache_path else None,
                                             ctypes.byref(co), ctypes.byref(no), ctypes.byref(ms),
                                             _stream()), "gpfc_survey_autotune")
        self.survey_n = len(so) - 1
        self.survey_k = int(periods.numel())
        self.survey_samples = so[-1]
        return co.value, no.value, ms.value

    def _survey_args(self, t, flux, periods, cnn, top, judge_snr, fp8):
        import torch
        _need(t, torch.float64, "t", self.device)
        _need(flux, torch.float32, "flux", self.device)
        _need(periods, torch.float64, "periods", self.device)
        if t.numel() != self.survey_samples or flux.numel() != self.survey_samples:
            raise ValueError("t / flux do not match the survey's sample offsets")
        if periods.numel() != self.survey_k:
            raise ValueError("periods must hold the survey's k periods")
        m, k = self.survey_n, self.survey_k
        e = lambda dt: torch.empty((m, k), dtype=dt, device=self.device)  # noqa: E731
        r = {"snr": e(torch.float32), "start": e(torch.int32), "width": e(torch.int32),
             "depth": e(torch.float32)}
        if cnn is not None:
            r["logits"] = e(torch.float32)
        o = SurveyOut(snr=_ptr(r["snr"]), start=_ptr(r["start"]), width=_ptr(r["width"]),
                      depth=_ptr(r["depth"]), logits=_ptr(r.get("logits")), cnn_fp8=int(bool(fp8)),
                      top=int(top), judge_snr=float(judge_snr))
        if top > 0:
            t2 = lambda dt: torch.empty((m, top), dtype=dt, device=self.device)  # noqa: E731
            r["box_val"], r["box_idx"] = t2(torch.float32), t2(torch.int64)
            o.box_val, o.box_idx = _ptr(r["box_val"]), _ptr(r["box_idx"])
            if cnn is not None:
                r["cnn_val"], r["cnn_idx"] = t2(torch.float32), t2(torch.int64)
                r["judged_val"], r["judged_idx"] = t2(torch.float32), t2(torch.int64)
                o.cnn_val, o.cnn_idx = _ptr(r["cnn_val"]), _ptr(r["cnn_idx"])
                o.judged_val, o.judged_idx = _ptr(r["judged_val"]), _ptr(r["judged_idx"])
        return r, o

    def survey_run(self, t, flux, periods, nbins: int = 256, cnn=None, top: int = 1,
                   judge_snr: float = 0.0, fp8: bool = False):
        """Fold, box-score and (with `cnn`) network-score every curve at every
        period; returns a dict of [n_curves, k] periodograms and, for top > 0,
        the [n_curves, top] best entries by box-SNR, by logit and by logit
        among periods with snr >= judge_snr."""
        r, o = self._survey_args(t, flux, periods, cnn, top, judge_snr, fp8)
        _check(self.lib.gpfc_survey_run(self.h, cnn.h if cnn is not None else None, _ptr(t),
                                        _ptr(flux), _ptr(periods), nbins, ctypes.byref(o),
                                        _stream()), "gpfc_survey_run")
        return r

    def survey_capture(self, t, flux, periods, nbins: int = 256, cnn=None, top: int = 1,
                       judge_snr: float = 0.0, fp8: bool = False):
        """Capture survey_run into the plan's HIP graph (replay with batch_replay)."""
        r, o = self._survey_args(t, flux, periods, cnn, top, judge_snr, fp8)
        self._graph_keep = (t, flux, periods, r, cnn)
        _check(self.lib.gpfc_survey_capture(self.h, cnn.h if cnn is not None else None, _ptr(t),
                                            _ptr(flux), _ptr(periods), nbins, ctypes.byref(o),
                                            _stream()), "gpfc_survey_capture")
        return r

    def detrend(self, t, flux, transit=None, cadence: float = 0.020428, gap_cadences: float = 30.0,
                jump_sigma: float = 5.0, clip_sigma: float = 3.0, edge: int = 30, max_fits: int = 10,
                spacings=(0.5, 0.75, 1.0, 1.5, 2.0, 3.0, 5.0)):
        """Pre-processing of a time-sorted curve (gpfc_detrend): returns
        (flux / continuum f64 [n], keep uint8 [n], info dict)."""
        import torch
        self._inputs(t, flux)
        if transit is not None:
            _need(transit, torch.uint8, "transit", self.device)
        n = t.numel()
        o = DetrendOpts(cadence=cadence, gap_cadences=gap_cadences, jump_sigma=jump_sigma,
                        clip_sigma=clip_sigma, edge=int(edge), max_fits=int(max_fits),
                        n_spacings=len(spacings))
        for i, h in enumerate(spacings):
            o.spacings[i] = float(h)
        out = torch.empty(n, dtype=torch.float64, device=self.device)
        keep = torch.empty(n, dtype=torch.uint8, device=self.device)
        info = DetrendInfo()
        _check(self.lib.gpfc_detrend(self.h, _ptr(t), _ptr(flux), _ptr(transit), n, ctypes.byref(o),
                                     _ptr(out), _ptr(keep), ctypes.byref(info), _stream()),
               "gpfc_detrend")
        return out, keep, {"n_segments": info.n_segments, "n_kept_segments": info.n_kept_segments,
                           "status": info.status}

    def fold_naive(self, t, flux, periods, nbins: int, out=None):
        """Plain global-atomic GPU fold (baseline): (sums, counts)."""
        import torch
        self._inputs(t, flux, periods)
        k = periods.numel()
        if out is None:
            sums = torch.empty((k, nbins), dtype=torch.float64, device=self.device)
            counts = torch.empty((k, nbins), dtype=torch.int32, device=self.device)
        else:
            sums, counts = out
        _check(self.lib.gpfc_fold_naive(self.h, _ptr(t), _ptr(flux), t.numel(), _ptr(periods), k,
                                        nbins, _ptr(sums), _ptr(counts), _stream()),
               "gpfc_fold_naive")
        return sums, counts

    def sync(self):
        _check(self.lib.gpfc_sync(_stream()), "gpfc_sync")


def fold_score_noalloc(t, flux, periods, nbins: int, out):
    """gpfc_fold_score_noalloc: fused fold + box-SNR on the current device with
    no allocation; ``out`` = (snr f32, start i32, width i32, depth f32), each [k],
    allocated by the caller."""
    import torch
    lib = load()
    dev = t.device
    _need(t, torch.float64, "t", dev)
    _need(flux, torch.float32, "flux", dev)
    _need(periods, torch.float64, "periods", dev)
    snr, start, width, depth = out
    _check(lib.gpfc_fold_score_noalloc(_ptr(t), _ptr(flux), t.numel(), _ptr(periods), periods.numel(),
                                       nbins, _ptr(snr), _ptr(start), _ptr(width), _ptr(depth),
                                       _stream()), "gpfc_fold_score_noalloc")
    return snr, start, width, depth


def topk(values, top: int = 1, gate=None, gate_min: float = 0.0):
    """Per-row best `top` (<= 64) entries of values f32 [rows, len] (value
    descending, index ascending; NaN and gated-out entries skipped; missing
    places -inf / -1): (f32 [rows, top], int64 [rows, top])."""
    import torch
    v = values if values.dim() == 2 else values.reshape(1, -1)
    _need(v, torch.float32, "values", v.device)
    if gate is not None:
        gate = gate.reshape(v.shape)
        _need(gate, torch.float32, "gate", v.device)
    rows, n = v.shape
    ov = torch.empty((rows, top), dtype=torch.float32, device=v.device)
    oi = torch.empty((rows, top), dtype=torch.int64, device=v.device)
    _check(load().gpfc_topk(_ptr(v), rows, n, _ptr(gate), float(gate_min), int(top), _ptr(ov),
                            _ptr(oi), _stream()), "gpfc_topk")
    return ov, oi


def periodogram_peaks(values, periods=None, nsigma: float = 3.0, min_width: int = 3,
                      max_peaks: int = 8):
    """SDE, mean, sd, peak count and the best max_peaks peaks (value, index,
    width, harmonic code) of each row of values f32 [rows, len]."""
    import torch
    v = values if values.dim() == 2 else values.reshape(1, -1)
    _need(v, torch.float32, "values", v.device)
    if periods is not None:
        _need(periods, torch.float64, "periods", v.device)
        if periods.numel() != v.shape[1]:
            raise ValueError("periods must hold one period per column")
    rows = v.shape[0]
    d = v.device
    r = {"sde": torch.empty(rows, dtype=torch.float32, device=d),
         "mean": torch.empty(rows, dtype=torch.float32, device=d),
         "sd": torch.empty(rows, dtype=torch.float32, device=d),
         "n_peaks": torch.empty(rows, dtype=torch.int32, device=d),
         "val": torch.empty((rows, max_peaks), dtype=torch.float32, device=d),
         "idx": torch.empty((rows, max_peaks), dtype=torch.int64, device=d),
         "width": torch.empty((rows, max_peaks), dtype=torch.int32, device=d),
         "harmonic": torch.empty((rows, max_peaks), dtype=torch.int32, device=d)}
    _check(load().gpfc_periodogram_peaks(_ptr(v), rows, v.shape[1], _ptr(periods), float(nsigma),
                                         int(min_width), int(max_peaks), _ptr(r["sde"]), _ptr(r["mean"]),
                                         _ptr(r["sd"]), _ptr(r["n_peaks"]), _ptr(r["val"]), _ptr(r["idx"]),
                                         _ptr(r["width"]), _ptr(r["harmonic"]), _stream()),
           "gpfc_periodogram_peaks")
    return r


CNN_BF16, CNN_FP32 = 0, 1


class Cnn:
    """The learned scorer on one GPU (gpfc_cnn_*): FP32 master weights,
    bf16 (or FP32) matrix-core forward and backward, Adam."""

    def __init__(self, device: int = 0, precision: int = CNN_BF16, max_batch: int = 4096):
        import torch
        self.lib = load()
        self.device = torch.device("cuda", device)
        self.max_batch = max_batch
        self.n_params = int(self.lib.gpfc_cnn_nparams())
        h = ctypes.c_void_p()
        _check(self.lib.gpfc_cnn_create(ctypes.byref(h), device, precision, max_batch), "gpfc_cnn_create")
        self.h = h
        self._loss = torch.zeros(1, dtype=torch.float32, device=self.device)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.gpfc_cnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        import torch
        p = torch.as_tensor(params, dtype=torch.float32, device=self.device).contiguous()
        if p.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        _check(self.lib.gpfc_cnn_set_params(self.h, _ptr(p), _stream()), "gpfc_cnn_set_params")
        torch.cuda.current_stream().synchronize()

    def get_params(self):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _check(self.lib.gpfc_cnn_get_params(self.h, _ptr(out), _stream()), "gpfc_cnn_get_params")
        return out

    def _x(self, x):
        import torch
        if x.dtype == torch.uint16:
            return 0
        if x.dtype == torch.float32:
            return 1
        raise TypeError("x must be uint16 (bfloat16 bits) or float32")

    def set_fused(self, on):
        """bf16 inference path: 1 / True fused convolution stack with wave-private inputs
        (default), 2 fused over tiles of 8 inputs in lockstep, 0 / False layer by layer."""
        _check(self.lib.gpfc_cnn_set_fused(self.h, int(on)), "gpfc_cnn_set_fused")

    def forward(self, x, out=None):
        """Logits f32[B] for x [B][256]."""
        import torch
        xf = self._x(x)
        _need(x, x.dtype, "x", self.device)
        B = x.shape[0]
        logits = out if out is not None else torch.empty(B, dtype=torch.float32, device=self.device)
        _check(self.lib.gpfc_cnn_forward(self.h, _ptr(x), xf, B, _ptr(logits), _stream()),
               "gpfc_cnn_forward")
        return logits

    def calibrate_fp8(self, x, reset: bool = True):
        """Record activation maxima of a bf16 network on calibration folds x."""
        xf = self._x(x)
        _need(x, x.dtype, "x", self.device)
        _check(self.lib.gpfc_cnn_calibrate_fp8(self.h, _ptr(x), xf, x.shape[0], int(reset), _stream()),
               "gpfc_cnn_calibrate_fp8")

    def forward_fp8(self, x, out=None):
        """Logits with FP8 E4M3 matrix-core layers (after calibrate_fp8)."""
        import torch
        xf = self._x(x)
        _need(x, x.dtype, "x", self.device)
        B = x.shape[0]
        logits = out if out is not None else torch.empty(B, dtype=torch.float32, device=self.device)
        _check(self.lib.gpfc_cnn_forward_fp8(self.h, _ptr(x), xf, B, _ptr(logits), _stream()),
               "gpfc_cnn_forward_fp8")
        return logits

    def backward(self, x, labels, grad_out=None):
        """Mean BCE loss (device tensor [1]); the gradient stays in the network
        (also copied to grad_out if given)."""
        import torch
        xf = self._x(x)
        _need(x, x.dtype, "x", self.device)
        _need(labels, torch.float32, "labels", self.device)
        _check(self.lib.gpfc_cnn_backward(self.h, _ptr(x), xf, _ptr(labels), x.shape[0],
                                          _ptr(self._loss), _ptr(grad_out), _stream()),
               "gpfc_cnn_backward")
        return self._loss

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        _check(self.lib.gpfc_cnn_adam(self.h, lr, beta1, beta2, eps, _stream()), "gpfc_cnn_adam")

    def train_capture(self, x, labels, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                      eps: float = 1e-8):
        """Record one training step on x / labels into a HIP graph (on a side
        stream); returns the device loss buffer each replay writes."""
        import torch
        xf = self._x(x)
        _need(x, x.dtype, "x", self.device)
        _need(labels, torch.float32, "labels", self.device)
        self._train_keep = (x, labels)
        self._train_loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self._train_stream = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(self._train_stream):
            _check(self.lib.gpfc_cnn_train_capture(self.h, _ptr(x), xf, _ptr(labels), x.shape[0], lr,
                                                   beta1, beta2, eps, _ptr(self._train_loss),
                                                   _stream()), "gpfc_cnn_train_capture")
        return self._train_loss

    def train_replay(self):
        """One captured training step, ordered after the current stream's work."""
        _check(self.lib.gpfc_cnn_train_replay(self.h, _stream()), "gpfc_cnn_train_replay")
        return self._train_loss

    def train_step(self, x, labels, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                   eps: float = 1e-8):
        """Backward then Adam in one call; returns the device loss buffer."""
        import torch
        xf = self._x(x)
        _need(x, x.dtype, "x", self.device)
        _need(labels, torch.float32, "labels", self.device)
        _check(self.lib.gpfc_cnn_train_step(self.h, _ptr(x), xf, _ptr(labels), x.shape[0], lr, beta1,
                                            beta2, eps, _ptr(self._loss), _stream()),
               "gpfc_cnn_train_step")
        return self._loss

    def save(self, path: str):
        """Write the parameters to a network file (tag, count, FP32 values)."""
        _check(self.lib.gpfc_cnn_save(self.h, str(path).encode(), _stream()), "gpfc_cnn_save")

    def load(self, path: str):
        """Read a network file written by save (resets the Adam state)."""
        _check(self.lib.gpfc_cnn_load(self.h, str(path).encode(), _stream()), "gpfc_cnn_load")


class PNet:
    """The paper's own network (gpfc_pnet_*): 16 x 16 image of the fold,
    circular 2-D convolutions of 128 and 256 filters (3 x 3, then 5 x 5) with
    global max-pools, a dense ReLU layer with dropout and a sigmoid output;
    FP32 master weights, bf16 (or FP32) matrix-core forward, Adam."""

    def __init__(self, device: int = 0, precision: int = CNN_BF16, max_batch: int = 1024):
        import torch
        self.lib = load()
        self.device = torch.device("cuda", device)
        self.max_batch = max_batch
        self.n_params = int(self.lib.gpfc_pnet_nparams())
        h = ctypes.c_void_p()
        rc = self.lib.gpfc_pnet_create(ctypes.byref(h), device, precision, max_batch)
        _check(rc, "gpfc_pnet_create")
        self.h = h
        self._loss = torch.zeros(1, dtype=torch.float32, device=self.device)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.gpfc_pnet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        import torch
        p = torch.as_tensor(params, dtype=torch.float32, device=self.device).contiguous()
        if p.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        _check(self.lib.gpfc_pnet_set_params(self.h, _ptr(p), _stream()), "gpfc_pnet_set_params")
        torch.cuda.current_stream().synchronize()

    def get_params(self):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _check(self.lib.gpfc_pnet_get_params(self.h, _ptr(out), _stream()), "gpfc_pnet_get_params")
        return out

    def set_fused(self, on: bool):
        """bf16 forward: fused convolution pairs (default) or layer by layer."""
        _check(self.lib.gpfc_pnet_set_fused(self.h, int(bool(on))), "gpfc_pnet_set_fused")

    def get_grads(self):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _check(self.lib.gpfc_pnet_get_grads(self.h, _ptr(out), _stream()), "gpfc_pnet_get_grads")
        return out

    @staticmethod
    def _xf(x):
        import torch
        if x.dtype == torch.uint16:
            return 0
        if x.dtype == torch.float32:
            return 1
        raise TypeError("x must be uint16 (bfloat16 bits) or float32")

    def forward(self, x, out=None):
        """Logits f32[B] for x [B][256] (no dropout)."""
        import torch
        xf = self._xf(x)
        _need(x, x.dtype, "x", self.device)
        B = x.shape[0]
        logits = out if out is not None else torch.empty(B, dtype=torch.float32, device=self.device)
        _check(self.lib.gpfc_pnet_forward(self.h, _ptr(x), xf, B, _ptr(logits), _stream()),
               "gpfc_pnet_forward")
        return logits

    def backward(self, x, labels, keep=None, logits=None):
        """Gradient of the mean BCE at x with dropout keep mask `keep` [B][128]
        (None: no dropout); returns the loss as a device scalar tensor."""
        import torch
        xf = self._xf(x)
        _need(x, x.dtype, "x", self.device)
        _need(labels, torch.float32, "labels", self.device)
        if keep is not None:
            _need(keep, torch.float32, "keep", self.device)
        B = x.shape[0]
        lg = logits if logits is not None else torch.empty(B, dtype=torch.float32, device=self.device)
        _check(self.lib.gpfc_pnet_backward(self.h, _ptr(x), xf, _ptr(labels), _ptr(keep), B, _ptr(lg),
                                           _ptr(self._loss), _stream()), "gpfc_pnet_backward")
        return self._loss

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        _check(self.lib.gpfc_pnet_adam(self.h, lr, beta1, beta2, eps, _stream()), "gpfc_pnet_adam")

    def train_step(self, x, labels, lr: float, keep=None):
        loss = self.backward(x, labels, keep)
        self.adam(lr)
        return loss
