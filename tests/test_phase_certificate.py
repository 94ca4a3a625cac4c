"""The fold kernels' certified fast phase path, emulated exactly on the CPU.

The kernels compute y = fma(t, 256 RN(1/P), 1.5 * 2^36 - 2^-16) in FP64 and
read the bin from bits 16-23 of y's low word, trusting it only when the low
16 bits (the fraction field) are below 65534; other updates take the IEEE
sequence of the fold's bin definition (x = RN(t/P), f = x - floor(x),
b = floor(256 f)). Here the FMA is evaluated exactly with rationals and
rounded once (float() of a Fraction rounds correctly), and the claim is
checked: a certified bin always equals the IEEE one. Inputs include times
placed within a few ulps of bin edges, where a wrong certificate would show.
"""
from __future__ import annotations

import math
import struct
from fractions import Fraction

import numpy as np

C = 1.5 * 2.0 ** 36 - 2.0 ** -16
LIM = 65536 - 2


def _fast(t: float, P: float, nb: int = 256):
    rB = (1.0 / P) * float(nb)
    y = float(Fraction(t) * Fraction(rB) + Fraction(C))
    lo = struct.unpack("<Q", struct.pack("<d", y))[0] & 0xFFFFFFFF
    return (lo >> 16) & (nb - 1), lo & 0xFFFF, abs(t) * rB < 2.0 ** 34


def _ieee(t: float, P: float, nb: int = 256) -> int:
    x = t / P
    f = x - math.floor(x)
    b = math.floor(f * nb)
    return min(max(b, 0), nb - 1)


def _check(ts, ps, nb=256):
    certified = rejected = 0
    for t, P in zip(ts, ps):
        b, frac, on = _fast(float(t), float(P), nb)
        assert on
        if frac < LIM:
            assert b == _ieee(float(t), float(P), nb), (t, P)
            certified += 1
        else:
            rejected += 1
    return certified, rejected


def test_constant_is_exact():
    assert Fraction(C) == Fraction(3, 2) * 2 ** 36 - Fraction(1, 2 ** 16)


def test_random_times_and_periods():
    rng = np.random.default_rng(7)
    n = 4000
    ts = rng.uniform(0.0, 1500.0, n)
    ps = rng.uniform(0.2, 1.0, n)
    cert, rej = _check(ts, ps)
    assert rej <= 3          # about 2 in 65,536 are handed to the IEEE sequence


def test_bjd_sized_times():
    rng = np.random.default_rng(8)
    n = 3000
    ts = 2_454_833.0 + rng.uniform(0.0, 1500.0, n)
    ps = rng.uniform(0.2, 1.0, n)
    _check(ts, ps)


def test_times_next_to_bin_edges():
    # t = P (m + j/256) moved by a few ulps, or by fractions of the 2^-16 bin
    # grid, either way: the IEEE bin flips between neighbours here, and the
    # certificate must either match it or hand the update over
    rng = np.random.default_rng(9)
    ts, ps = [], []
    for _ in range(800):
        P = float(rng.uniform(0.2, 1.0))
        edge = P * (int(rng.integers(0, 4000)) + int(rng.integers(0, 256)) / 256.0)
        grid = P / 256.0 * 2.0 ** -16
        for k in (-3, -1, 0, 1, 3):
            ts.append(edge + k * math.ulp(edge))
            ps.append(P)
        for g in (-3.0, -2.0, -1.5, -1.0, -0.5, 0.5, 1.0, 1.5, 2.0, 3.0):
            ts.append(edge + g * grid)
            ps.append(P)
    cert, rej = _check(ts, ps)
    assert rej > 0 and cert > 0


def test_dyadic_exact_edges_are_rejected():
    # t/P exactly on a bin edge: the fraction field is 65535, never certified
    for j in range(6):
        P = 2.0 ** -j
        for i in range(0, 4096, 37):
            b, frac, _ = _fast(i * 2.0 ** -7, P)
            if (i * 2.0 ** -7 / P * 256) % 1 == 0:
                assert frac >= LIM


def test_4096_bins():
    rng = np.random.default_rng(10)
    ts = rng.uniform(0.0, 1500.0, 2000)
    ps = rng.uniform(0.2, 1.0, 2000)
    _check(ts, ps, nb=4096)
