"""GPU parity of the adaptive per-frame gamma against the oracle.

The frame's gamma comes from fixed-point luma sums of J on the GPU and from a
float64 mean in the oracle; the two gammas agree to ~1e-7 relative, far inside
the output tolerance, so the usual tolerances apply.  Cases are chosen so the
rule is exercised inside its clamp range, not only at the bounds.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2512_16609_amd as hzd
from synth import make_frame
from parity import compare, oracle_params, run_gpu, to_dev

pytestmark = pytest.mark.gpu


def _frame(w, h, seed, dark=1.0):
    I = make_frame(w, h, seed).I
    return (I * dark).astype(np.uint8) if dark != 1.0 else I


CASES = [(320, 240, 1, 1.0, 0.9), (320, 240, 2, 0.35, 0.5), (333, 197, 3, 0.5, 0.6), (97, 61, 4, 1.0, 0.5),
         (640, 480, 5, 0.3, 0.45), (1, 1, 6, 1.0, 0.5), (29, 1, 7, 0.6, 0.7)]


@pytest.mark.parametrize("w,h,seed,dark,tau", CASES)
@pytest.mark.parametrize("cb", [0, 1])
@pytest.mark.parametrize("tx", [hzd.TX_HE, hzd.TX_PAPER])
def test_realtime_adaptive_gamma(w, h, seed, dark, tau, cb, tx):
    I = _frame(w, h, seed, dark)
    p = hzd.Params(gamma_adaptive=1, gamma_target=tau, color_balance=cb, tx=tx)
    compare(I, p, run_gpu(I, p), label=f"rt {w}x{h} tau {tau}")


@pytest.mark.parametrize("w,h,seed,dark,tau", CASES[:5])
@pytest.mark.parametrize("cb", [0, 1])
@pytest.mark.parametrize("prec", [hzd.PREC_FP32, hzd.PREC_FP16])
def test_offline_adaptive_gamma(w, h, seed, dark, tau, cb, prec):
    I = _frame(w, h, seed, dark)
    p = hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=20, gamma_adaptive=1, gamma_target=tau, color_balance=cb,
                   precision=prec)
    compare(I, p, run_gpu(I, p), label=f"off {w}x{h} tau {tau}")


def test_cases_exercise_the_rule_inside_its_clamp():
    inside = 0
    for w, h, seed, dark, tau in CASES:
        g = oracle.dehaze(_frame(w, h, seed, dark), oracle_params(hzd.Params(gamma_adaptive=1, gamma_target=tau)))
        inside += 0.5 < g.aux["gamma"] < 2.0
    assert inside >= 4


def test_adaptive_gamma_1080p_offline_matches_oracle():
    I = _frame(1920, 1080, 2)
    p = hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=60, color_balance=1, gamma_adaptive=1, gamma_target=0.7)
    s = compare(I, p, run_gpu(I, p), label="1080p adaptive")
    print(s)


def test_degenerate_frames_take_the_clamped_gamma():
    for val in (0, 255, 117):
        I = np.full((48, 80, 3), val, dtype=np.uint8)
        for p in (hzd.Params(gamma_adaptive=1),
                  hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=9, color_balance=1, gamma_adaptive=1)):
            compare(I, p, run_gpu(I, p), label=f"const {val}")


def test_batch_mixing_adaptive_and_fixed_gamma_equals_frames():
    shapes = [(240, 320), (97, 130), (480, 640), (120, 160)]
    params = [hzd.Params(gamma_adaptive=1, gamma_target=0.8), hzd.Params(),
              hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=30, gamma_adaptive=1, gamma_target=0.6),
              hzd.Params(gamma_adaptive=1, gamma_target=0.4, color_balance=1)]
    frames = [_frame(w, h, 60 + i, 0.5) for i, (h, w) in enumerate(shapes)]
    srcs = [to_dev(I) for I in frames]
    dsts = [torch.zeros_like(s) for s in srcs]
    auxs = [hzd.make_aux(h, w) for (h, w) in shapes]
    hzd.dehaze_batch(srcs, dsts, hzd.Params(), per_frame_params=params, auxs=auxs)
    torch.cuda.synchronize()
    for i, I in enumerate(frames):
        alone = run_gpu(I, params[i])
        assert np.array_equal(dsts[i].cpu().numpy(), alone["out"]), i
        for k in ("A", "sel", "dark", "t", "J"):
            assert np.array_equal(auxs[i][k].cpu().numpy(), alone[k]), (i, k)
