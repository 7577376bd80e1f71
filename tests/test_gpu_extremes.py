"""Parameters at the ends of their accepted ranges, against the oracle."""
import numpy as np
import pytest

import paper_2512_16609_amd as hzd
from synth import make_frame
from parity import compare, run_gpu

pytestmark = pytest.mark.gpu


def _frame(w, h, seed):
    return make_frame(w, h, seed).I


@pytest.mark.parametrize("gamma", [0.1, 0.3, 5.0, 10.0])
@pytest.mark.parametrize("mode", [hzd.MODE_REALTIME, hzd.MODE_OFFLINE])
def test_gamma_range_ends(gamma, mode):
    I = _frame(320, 240, 70)
    p = hzd.Params(mode=mode, gamma=gamma, gf_radius=30, color_balance=int(mode == hzd.MODE_OFFLINE))
    print(gamma, mode, compare(I, p, run_gpu(I, p), label=f"gamma {gamma}"))


@pytest.mark.parametrize("top_frac", [1.0, 0.5, 1e-9])   # K = N, half the frame, K = 1
def test_selection_extremes(top_frac):
    I = _frame(160, 120, 71)
    p = hzd.Params(top_frac=top_frac, alpha=1.0)
    g = run_gpu(I, p)
    compare(I, p, g, label=f"top_frac {top_frac}")
    n = 160 * 120
    assert int(g["sel"][0]) == max(1, int(np.floor(float(np.float32(top_frac)) * n)))


@pytest.mark.parametrize("eps", [1e-8, 1.0])
def test_guided_filter_eps_ends(eps):
    I = _frame(200, 150, 72)
    p = hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=64, gf_eps=eps)
    compare(I, p, run_gpu(I, p), label=f"eps {eps}")


def test_largest_patch_and_radius_on_small_frames():
    for (w, h) in [(17, 9), (70, 33), (129, 65)]:
        I = np.random.default_rng(w).integers(0, 256, (h, w, 3), dtype=np.uint8)
        p = hzd.Params(mode=hzd.MODE_OFFLINE, patch=31, gf_radius=64, color_balance=1)
        compare(I, p, run_gpu(I, p), label=f"patch 31 r 64 {w}x{h}")


@pytest.mark.parametrize("eps,t0", [(1e-8, 0.01), (1e-8, 0.1), (1e-5, 0.005), (1e-3, 0.002)])
def test_small_eps_and_t0_take_the_int64_a_b(eps, t0):
    """Where int32 a, b would move t by more than 1e-6 t0 the library stores them as
    int64: a bright flat frame (t = t0 everywhere, b = t0) and a hazy frame stay within
    the 1e-5 tolerance of the oracle's t."""
    flat = np.full((60, 90, 3), 250, dtype=np.uint8)
    for I in (flat, _frame(240, 160, 73)):
        p = hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=20, gf_eps=eps, t0=t0, color_balance=1)
        s = compare(I, p, run_gpu(I, p), label=f"eps {eps} t0 {t0}")
        assert s["t_rel_max"] <= 2e-6, s


def test_int64_a_b_do_not_depend_on_the_tile_height():
    I = _frame(320, 200, 74)
    p = hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=25, gf_eps=1e-8, t0=0.01)
    outs = []
    for rows in (8, 24, 64):
        hzd.tile_config_set(320, 200, rows)
        try:
            outs.append(run_gpu(I, p))
        finally:
            hzd.tile_config_set(320, 200, None)
    for o in outs[1:]:
        assert np.array_equal(o["out"], outs[0]["out"]) and np.array_equal(o["t"], outs[0]["t"])
