"""The margin of the pair kernel's fp16 cutoff test (float form), emulated on
the CPU.

The float pair kernel tests each candidate against each target with fp16
coordinates relative to a point O of the group's cell, in cutoff units: the
target T rounded to nearest, the candidate C cut toward zero, and
W = fp16(|C|^2 - lim) cut toward zero; v = |T|^2 + W - 2 T.C, products
exact in float32. A pair inside the cutoff must give v < 0 (the hit loop
then decides exactly on the fixed-point separation), so lim carries a
margin bounded from the fp16 spacings (pp.hip, fp16_test_lim). This test
repeats that bound and checks it on the worst placements: targets anywhere
within one cell edge of O, candidates at 1 - 1e-7 cutoff from them in every
direction, so that a margin too small for the rounding fails here before it
could drop a pair on the GPU.
"""
import math

import numpy as np
import pytest


def ulp16_bound(x):
    """Spacing bound of fp16 values of magnitude <= x: 2^(e - 11) for x < 2^e."""
    _, e = math.frexp(x)
    return math.ldexp(1.0, max(e - 11, -24))


def fp16_test_lim(emax):
    flush = 2.0 ** -14
    tmax = emax * (1.0 + 1e-6)
    cmx = tmax + 1.0
    u_t = 0.5 * ulp16_bound(tmax) + flush
    u_c = ulp16_bound(cmx) + flush
    u_w = ulp16_bound(max(1.1, (cmx + u_c) ** 2)) + flush
    d = math.sqrt(3.0) * (u_t + u_c)
    return float(np.float32(1.0 + 2.0 * d + d * d + u_w + 1e-5 * max(1.0, 3.0 * cmx * cmx)))


def rtz16(x):
    """float32 values cut toward zero to fp16 (normal range: 11 significant
    bits; subnormal range: multiples of 2^-24)."""
    x = np.asarray(x, dtype=np.float32)
    cut = (x.view(np.uint32) & np.uint32(0xFFFFE000)).view(np.float32)
    sub = np.trunc(x.astype(np.float64) * 2.0 ** 24) / 2.0 ** 24
    return np.where(np.abs(x) < 2.0 ** -14, sub, cut.astype(np.float64))


def test_rtz16_is_fp16_toward_zero():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(100000) * 3).astype(np.float32)
    r = rtz16(x)
    assert np.all(np.float16(r).astype(np.float64) == r)           # representable
    assert np.all(np.abs(r) <= np.abs(x)) and np.all(np.sign(r) * np.sign(x) >= 0)
    away = np.where(x >= 0, np.inf, -np.inf).astype(np.float16)
    up = np.nextafter(np.float16(r), away).astype(np.float64)     # the next fp16 value away from zero
    assert np.all((np.abs(up) > np.abs(x)) | (r == x))             # nearest toward zero


@pytest.mark.parametrize("emax", [0.25, 0.5, 0.52, 0.7, 1.0, 1.3, 1.9])
def test_inside_pairs_always_pass(emax):
    rng = np.random.default_rng(int(emax * 1000))
    lim = fp16_test_lim(emax)
    n = 400000
    t = rng.uniform(-emax, emax, (n, 3))
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    c = t + (1.0 - 1e-7) * u
    # the kernel's float coordinates (units times the unit: rounded once)
    t32 = t.astype(np.float32)
    c32 = c.astype(np.float32)
    T = np.float16(t32).astype(np.float64)                         # to nearest
    C = rtz16(c32)                                                 # toward zero
    w32 = np.float32(np.sum(C * C, axis=1) - lim)
    W = rtz16(w32)
    tt = np.sum(T * T, axis=1)
    v = tt + W - 2.0 * np.sum(T * C, axis=1)                       # exact products, exact sum
    slack = 4 * 2.0 ** -24 * (tt + np.abs(W) + 2 * np.abs(np.sum(T * C, axis=1)))
    worst = np.max(v + slack)
    print(f"emax {emax}: lim - 1 = {lim - 1:.2e}, worst v {worst:.2e}", flush=True)
    assert worst < 0.0


def test_margin_stays_small():
    # a larger margin only admits more candidates for the exact test; for
    # cells up to a cutoff wide it stays near 1 %
    assert fp16_test_lim(0.5) - 1.0 < 0.008
    assert fp16_test_lim(1.0) - 1.0 < 0.015
