"""Seeded random combinations of the optional stages (resize, adaptive gamma,
temporal airlight smoothing) with every other parameter, run as short frame
sequences through the C ABI and checked against the oracle frame by frame:
the tests that introduce each stage vary it mostly on its own."""
import numpy as np
import pytest

import oracle
import paper_2512_16609_amd as hzd
from synth import make_frame
from parity import compare, oracle_params, run_gpu

pytestmark = pytest.mark.gpu


def _case(rng, seed):
    h, w = int(rng.integers(1, 220)), int(rng.integers(1, 320))
    nf = int(rng.integers(1, 4))
    if h >= 16 and w >= 16:
        frames = [make_frame(w, h, seed + k, beta=float(rng.uniform(0.5, 2.0))).I for k in range(nf)]
    else:
        frames = [rng.integers(0, 256, size=(h, w, 3), dtype=np.uint8) for _ in range(nf)]
    if rng.random() < 0.3:
        frames = [(f * rng.uniform(0.2, 0.8)).astype(np.uint8) for f in frames]   # darker frames
    resize = rng.random() < 0.5
    p = hzd.Params(mode=int(rng.integers(0, 2)), patch=int(rng.choice(np.arange(1, 32, 2))),
                   omega=float(rng.uniform(0.5, 1.0)), t0=float(rng.uniform(0.05, 0.3)),
                   top_frac=float(rng.uniform(0.0005, 0.05)), alpha=float(rng.uniform(0.5, 1.0)),
                   gamma=float(rng.uniform(0.8, 2.5)), gf_radius=int(rng.integers(1, 65)),
                   gf_eps=float(rng.choice([1e-5, 1e-3, 1e-2])), color_balance=int(rng.integers(0, 2)),
                   tx=int(rng.integers(0, 2)), precision=int(rng.integers(0, 2)),
                   resize_width=int(rng.integers(1, 300)) if resize else 0,
                   resize_height=int(rng.integers(1, 200)) if resize else 0,
                   airlight_smoothing=float(rng.choice([0.0, rng.uniform(0.1, 0.95)])),
                   gamma_adaptive=int(rng.integers(0, 2)), gamma_target=float(rng.uniform(0.3, 0.8)))
    return frames, p


@pytest.mark.parametrize("case", range(60))
def test_random_feature_sweep(case):
    rng = np.random.default_rng(12000 + case)
    frames, p = _case(rng, 12000 + 10 * case)
    pad = int(rng.choice([0, 0, 1, 5]))
    state = hzd.make_airlight_state()
    ref = oracle.dehaze_sequence(frames, oracle_params(p))
    for k, (I, r) in enumerate(zip(frames, ref)):
        g = run_gpu(I, p, pitch_pad=pad, airlight_state=state)
        compare(I, p, g, ref=r, label=f"feature sweep {case}/{k} {I.shape} {p}")
