"""MI355X-native GPU phase folding and box-SNR scoring (GPFC, arXiv:2312.02063).

The compute path is the HIP library ``libgpfc.so`` (gfx950) behind the C ABI
of ``include/gpfc.h``; ``Plan`` is its thin Python binding. ``synth`` makes
seeded synthetic light curves and trial grids.
"""
from ._lib import Cnn, CNN_BF16, CNN_FP32, GpfcError, Plan, PNet, load, periodogram_peaks, topk  # noqa: F401

__all__ = ["Plan", "Cnn", "PNet", "CNN_BF16", "CNN_FP32", "GpfcError", "load"]
