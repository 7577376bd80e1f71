"""The guided filter's fixed-point a and b (Eq. (6)) against the float64 oracle,
on the CPU.

The library forms a and b in FP64 from exact integer box sums, stores each as
rint(v * 2^k) (int32, or int64 when the int32 rounding is too coarse), and
takes the stage-2 box means of the stored integers.  This emulates that
storage with NumPy from the oracle's own a and b and measures the effect on
the refined t, for the scale rule the library uses:

  B = 1 + 1 / (4 sqrt(eps));  k32 = min(30, floor(log2((2^31 - 1) / B)))
  int32 while 2^-k32 <= 1e-6 t0, else int64 with
  k64 = min(52, floor(log2(9.2e18 / (B (2r+1)^2))))

The rounding moves t by at most 2^-k, so the rule keeps it at or below
1e-6 t0, a tenth of the 1e-5 relative tolerance of t.  The emulation shows
that int32 storage alone would break the tolerance at small eps and t0.
"""
import math

import numpy as np
import pytest

import oracle
from synth import make_frame


def rule(eps, t0, r):
    eps, t0 = float(np.float32(eps)), float(np.float32(t0))
    B = 1.0 + 0.25 / math.sqrt(eps)
    k = min(30, math.floor(math.log2(2147483647.0 / B)))
    if 2.0 ** -k <= 1e-6 * t0:
        return False, k
    n = (2 * r + 1) ** 2
    return True, min(52, math.floor(math.log2(9.2e18 / (B * n))))


def emulate(I, eps, t0, r, bits, wide):
    p = oracle.Params(mode="offline", gf_radius=r, gf_eps=eps, t0=t0)
    ref = oracle.dehaze(I, p)
    a, b = ref.aux["gf_a"], ref.aux["gf_b"]
    lim = 4.0e18 if wide else 2147483647.0
    ia = np.clip(np.rint(a * 2.0 ** bits), -lim, lim)
    ib = np.clip(np.rint(b * 2.0 ** bits), -lim, lim)
    assert np.abs(ia).max() < lim and np.abs(ib).max() < lim, "scale overflows the storage"
    G = oracle.luma(ref.aux.get("I", I))
    q = (oracle.box_mean(ia, r) * G + oracle.box_mean(ib, r)) * 2.0 ** -bits
    t = np.clip(q, float(np.float32(t0)), 1.0)
    return t, ref.aux["t"]


def _frame(dark):
    I = make_frame(96, 64, 21, beta=1.8).I
    return (I * dark).astype(np.uint8)


@pytest.mark.parametrize("eps,t0", [(1e-3, 0.1), (1e-3, 0.005), (1e-5, 0.01), (1e-8, 0.01), (1e-8, 0.1)])
def test_rule_keeps_the_rounding_inside_the_tolerance(eps, t0):
    r = 12
    wide, k = rule(eps, t0, r)
    assert 2.0 ** -k <= 1e-6 * float(np.float32(t0))
    t, t_ref = emulate(_frame(0.35), eps, t0, r, k, wide)
    err = np.abs(t - t_ref) / t_ref
    assert err.max() <= 2.0 ** -k / float(np.float32(t0)) + 1e-12
    assert err.max() <= 1e-6


def test_int32_alone_fails_at_small_eps_and_t0():
    eps, t0, r = 1e-8, 0.01, 12
    wide, k = rule(eps, t0, r)
    assert wide
    B = 1.0 + 0.25 / math.sqrt(float(np.float32(eps)))
    k32 = min(30, math.floor(math.log2(2147483647.0 / B)))
    assert k32 == 19
    # a bright flat frame: t = t0 everywhere, so a = 0 and b = t0, and the rounding of b
    # to a multiple of 2^-19 is the whole error (0.01 * 2^19 = 5242.88 rounds to 5243)
    I = np.full((40, 56, 3), 250, dtype=np.uint8)
    t, t_ref = emulate(I, eps, t0, r, k32, False)
    err = np.abs(t - t_ref) / t_ref
    assert err.max() > 1e-5
    t, t_ref = emulate(I, eps, t0, r, k, True)
    assert (np.abs(t - t_ref) / t_ref).max() <= 1e-9


def test_default_parameters_stay_on_int32():
    # the configurations' eps = 1e-3 and t0 in {0.1, 0.05} keep the compact 8-byte map
    for t0 in (0.1, 0.05):
        wide, k = rule(1e-3, t0, 60)
        assert not wide and k == 27
