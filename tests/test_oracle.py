"""Pins for the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a hand-worked
example, brute force, an independent library routine (scipy.ndimage), a
closed form, or an invariant that a plausible slip (a dropped term, a wrong
sign, a transposed operand, a wrong tie-break) would break.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import ndimage

import oracle
from oracle import Params
from synth import make_frame

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rng(seed):
    return np.random.default_rng(seed)


# ------------------------------------------------------------ dark channel
SHAPES = [(1, 1), (1, 7), (7, 1), (5, 9), (16, 23), (3, 40), (12, 12)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("patch", [1, 3, 5, 15, 31])
def test_erode_matches_bruteforce(shape, patch):
    x = rng(hash((shape, patch)) & 0xffff).integers(0, 256, size=shape, dtype=np.uint8)
    assert np.array_equal(oracle.erode(x, patch), oracle.erode_bruteforce(x, patch))


@pytest.mark.parametrize("patch", [3, 7, 15])
def test_erode_matches_scipy(patch):
    # an independent library routine: padding with 255 equals a clipped window
    x = rng(patch).integers(0, 256, size=(37, 53), dtype=np.uint8)
    ref = ndimage.minimum_filter(x, size=patch, mode="constant", cval=255)
    assert np.array_equal(oracle.erode(x, patch), ref)


def test_erode_closed_forms():
    x = np.full((20, 30), 77, dtype=np.uint8)
    assert np.array_equal(oracle.erode(x, 15), x)                 # constant stays constant
    y = rng(0).integers(0, 256, size=(9, 11), dtype=np.uint8)
    assert np.array_equal(oracle.erode(y, 1), y)                  # p = 1 is the identity
    z = np.full((20, 30), 200, dtype=np.uint8)
    z[2, 27] = 5                                                  # one dark pixel near a corner
    e = oracle.erode(z, 7)
    expect = np.full((20, 30), 200, dtype=np.uint8)
    expect[0:6, 24:30] = 5                                        # clipped 7x7 square
    assert np.array_equal(e, expect)


def test_dark_is_min_of_channel_erosions():
    I = rng(1).integers(0, 256, size=(31, 45, 3), dtype=np.uint8)
    D = oracle.dark_channel(I, 15)
    E = oracle.channel_erosions(I, 15)
    assert np.array_equal(D, E.min(axis=2))


def test_hand_example_dark_and_airlight():
    g = json.load(open(os.path.join(GOLDEN, "hand_dark_airlight.json")))
    I = np.array(g["frame_rgb"], dtype=np.uint8)
    assert np.array_equal(oracle.channel_min(I), np.array(g["channel_min"]))
    D = oracle.dark_channel(I, g["patch"])
    assert np.array_equal(D, np.array(g["dark"]))
    for case in g["cases"]:
        air = oracle.airlight(I, D, case["top_frac"], g["alpha"])
        assert air.K == case["K"]
        assert air.vstar == case["vstar"]
        assert air.cutoff == case["cutoff"]
        assert list(air.sel) == case["set"]
        assert list(air.S) == case["S"]
        a32 = float(np.float32(g["alpha"]))
        assert np.array_equal(air.A, a32 * np.array(case["S"], dtype=np.float64) / case["K"])


# ---------------------------------------------------------------- airlight
def _python_topk(D, K):
    h, w = D.shape
    keyed = sorted(((-int(D[y, x]), y * w + x) for y in range(h) for x in range(w)))
    return [i for _, i in keyed[:K]]


@pytest.mark.parametrize("seed", range(6))
def test_airlight_set_matches_python_sort(seed):
    r = rng(100 + seed)
    h, w = int(r.integers(1, 24)), int(r.integers(1, 24))
    # few distinct values -> massive ties, as with real uint8 dark channels
    D = r.integers(0, 4, size=(h, w)).astype(np.uint8) * 60
    I = r.integers(0, 256, size=(h, w, 3), dtype=np.uint8)
    top = float(r.uniform(0.01, 0.5))
    air = oracle.airlight(I, D, top, 0.8)
    K = max(1, math.floor(float(np.float32(top)) * h * w))
    assert air.K == K
    assert list(air.sel) == _python_topk(D, K)


def test_airlight_set_is_lexicographic_threshold():
    r = rng(7)
    D = r.integers(180, 200, size=(64, 80)).astype(np.uint8)
    I = r.integers(0, 256, size=(64, 80, 3), dtype=np.uint8)
    air = oracle.airlight(I, D, 0.01, 0.8)
    d = D.reshape(-1)
    inset = np.zeros(d.size, bool)
    inset[air.sel] = True
    assert inset.sum() == air.K
    # every pixel outside the set is below (vstar, cutoff) in the (D desc, idx asc) order
    out_idx = np.nonzero(~inset)[0]
    assert np.all((d[out_idx] < air.vstar) | ((d[out_idx] == air.vstar) & (out_idx > air.cutoff)))
    in_idx = np.nonzero(inset)[0]
    assert np.all((d[in_idx] > air.vstar) | ((d[in_idx] == air.vstar) & (in_idx <= air.cutoff)))


def test_uniform_frame_selects_first_k_raster_pixels():
    I = np.full((20, 50, 3), (90, 120, 150), dtype=np.uint8)
    D = oracle.dark_channel(I, 15)
    air = oracle.airlight(I, D, 0.05, 0.8)
    assert air.K == 50
    assert list(air.sel) == list(range(50))
    a32 = float(np.float32(0.8))
    assert np.array_equal(air.A, a32 * np.array([90.0, 120.0, 150.0]))


def test_sky_region_gives_alpha_times_sky():
    fr = make_frame(320, 240, 11, beta=1.0)
    I = fr.I.copy()
    sky = np.array([217, 224, 229], dtype=np.uint8)
    I[:40, :, :] = sky                  # 12800 px > K + erosion margin
    D = oracle.dark_channel(I, 15)
    air = oracle.airlight(I, D, 0.001, 0.8)
    a32 = float(np.float32(0.8))
    assert np.array_equal(air.A, a32 * sky.astype(np.float64))


def test_unique_maxima_are_selected():
    I = np.full((30, 40, 3), 40, dtype=np.uint8)
    spots = [(3, 5), (20, 33), (27, 2)]
    for (y, x) in spots:
        I[max(0, y - 7):y + 8, max(0, x - 7):x + 8] = (200, 210, 220)
    D = oracle.dark_channel(I, 1)
    air = oracle.airlight(I, D, 3 / 1200 + 1e-6, 0.8)
    assert air.K == 3
    assert air.vstar == 200
    # the first three raster pixels of the bright squares
    bright = np.nonzero(D.reshape(-1) == 200)[0][:3]
    assert list(air.sel) == list(bright)


@pytest.mark.parametrize("wh,K", [((320, 240), 76), ((640, 480), 307), ((1280, 720), 921),
                                  ((1920, 1080), 2073), ((3840, 2160), 8294)])
def test_top_count_at_config_sizes(wh, K):
    assert oracle.top_count(0.001, wh[0] * wh[1]) == K


def test_bright_blob_captures_the_airlight():
    # the limitation the paper notes: a large bright region (a headlight)
    # takes over the top-K set and A follows it
    fr = make_frame(320, 240, 12, beta=1.0)
    I = fr.I.copy()
    I[100:140, 100:160] = 255
    D = oracle.dark_channel(I, 15)
    air = oracle.airlight(I, D, 0.001, 0.8)
    assert air.vstar == 255
    assert np.allclose(air.A, float(np.float32(0.8)) * 255.0)


# ------------------------------------------------------------ transmission
def test_transmission_bounds_and_omega_zero():
    fr = make_frame(96, 64, 3, beta=1.3)
    D = oracle.dark_channel(fr.I, 15)
    A = oracle.airlight(fr.I, D, 0.001, 0.8).A
    for tx in ("he", "paper"):
        for om in (0.0, 0.5, 0.95, 1.0):
            if tx == "he":
                t = oracle.transmission_he(fr.I, A, om, 0.1, 15)
            else:
                t = oracle.transmission_paper(fr.I, A, om, 0.1)
            assert t.min() >= float(np.float32(0.1)) and t.max() <= 1.0
            if om == 0.0:
                assert np.all(t == 1.0)


def test_transmission_he_commutes_with_erosion():
    # dark(I/A) = min_c erode(I^c)/A^c exactly: erosion commutes with a positive
    # per-channel scale and with the channel minimum
    I = rng(5).integers(0, 256, size=(40, 33, 3), dtype=np.uint8)
    A = np.array([180.3, 201.7, 222.9])
    E = oracle.channel_erosions(I, 15).astype(np.float64)
    via_E = (E / A[None, None, :]).min(axis=2)
    t1 = np.maximum(1.0 - float(np.float32(0.95)) * via_E, float(np.float32(0.1)))
    t2 = oracle.transmission_he(I, A, 0.95, 0.1, 15)
    assert np.array_equal(t1, t2)


def test_transmission_paper_hand_value():
    I = np.zeros((1, 1, 3), dtype=np.uint8)
    I[0, 0] = (100, 60, 200)
    A = np.array([150.0, 160.0, 170.0])
    t = oracle.transmission_paper(I, A, 0.5, 0.05)
    w = float(np.float32(0.5))
    assert t[0, 0] == 1.0 - w * 60.0 / 170.0


# ---------------------------------------------------------- exact recovery
def _zero_channel_scene(h, w, seed):
    r = rng(seed)
    J = r.uniform(0.05, 0.95, size=(h, w, 3)) * 255.0
    zc = r.integers(0, 3, size=(h, w))
    for c in range(3):
        J[:, :, c][zc == c] = 0.0
    return J


@pytest.mark.parametrize("t_const", [0.35, 0.8])
def test_exact_recovery_constant_t(t_const):
    # I = J t + A (1 - t) in float64 with a zero channel at every pixel: the prior
    # holds exactly, so dark(I/A) = 1 - t and, with omega = 1, J is recovered
    J = _zero_channel_scene(40, 56, 1)
    A = np.array([0.85, 0.88, 0.90]) * 255.0
    t = np.full(J.shape[:2], t_const)
    I = J * t[..., None] + A * (1.0 - t[..., None])
    p = Params(mode="realtime", omega=1.0, t0=0.01, gamma=1.0, tx="he")
    res = oracle.dehaze(I, p, A_inject=A)
    assert np.max(np.abs(res.aux["t"] - t)) <= 1e-12
    assert np.max(np.abs(res.aux["J"] - J)) <= 1e-12


def test_exact_recovery_piecewise_t_interior():
    J = _zero_channel_scene(64, 96, 2)
    A = np.array([0.84, 0.87, 0.91]) * 255.0
    t = np.full(J.shape[:2], 0.3)
    t[:, 48:] = 0.7
    t[32:, :] = 0.5
    I = J * t[..., None] + A * (1.0 - t[..., None])
    p = Params(mode="realtime", omega=1.0, t0=0.01, gamma=1.0, tx="he", patch=7)
    res = oracle.dehaze(I, p, A_inject=A)
    r = 3
    interior = np.ones(t.shape, bool)
    for edge in (48,):
        interior[:, edge - r:edge + r] = False
    interior[32 - r:32 + r, :] = False
    err_t = np.abs(res.aux["t"] - t)[interior]
    err_J = np.abs(res.aux["J"] - J)[interior]
    assert err_t.max() <= 1e-12 and err_J.max() <= 1e-12


def test_recovery_from_synth_uint8_is_close():
    # the quantised generator frame: the recovered t tracks the true t
    fr = make_frame(320, 240, 1, beta=1.0)
    p = Params(mode="realtime", omega=1.0, t0=0.05, gamma=1.0, tx="he")
    res = oracle.dehaze(fr.I, p, A_inject=fr.A * 255.0)
    err = np.abs(res.aux["t"] - fr.t)
    assert np.median(err) < 0.03


# ----------------------------------------------------------- guided filter
def test_box_mean_matches_bruteforce_and_scipy():
    x = rng(9).uniform(size=(23, 31))
    for r in (0, 1, 3, 8, 40):
        bm = oracle.box_mean(x, r)
        assert np.allclose(bm, oracle.box_mean_bruteforce(x, r), rtol=0, atol=1e-13)
        ones = np.ones_like(x)
        size = 2 * r + 1
        ref = (ndimage.uniform_filter(x, size=size, mode="constant", cval=0.0)
               / ndimage.uniform_filter(ones, size=size, mode="constant", cval=0.0))
        assert np.allclose(bm, ref, rtol=0, atol=1e-12)


def test_guided_filter_identity_on_constant_input():
    G = rng(3).uniform(size=(40, 50))
    p = np.full((40, 50), 0.42)
    q = oracle.guided_filter(p, G, 6, 1e-3).q
    assert np.max(np.abs(q - p)) <= 1e-12   # integral-image rounding only


def test_guided_filter_identity_when_input_is_guide():
    G = rng(4).uniform(size=(30, 30))   # var > 0 in every window
    q = oracle.guided_filter(G, G, 3, 0.0).q
    assert np.max(np.abs(q - G)) <= 1e-12


def test_guided_filter_constant_guide_is_box_of_box():
    G = np.full((25, 33), 0.5)
    p = rng(6).uniform(size=(25, 33))
    r = 4
    q = oracle.guided_filter(p, G, r, 1e-3).q
    ref = oracle.box_mean_bruteforce(oracle.box_mean_bruteforce(p, r), r)
    assert np.max(np.abs(q - ref)) <= 1e-13


def test_guided_filter_hand_scalar_case():
    # 1x1 frame: every window is the pixel itself, var = cov = 0, q = p
    G = np.array([[0.3]])
    p = np.array([[0.7]])
    gf = oracle.guided_filter(p, G, 5, 1e-3)
    assert gf.a[0, 0] == 0.0 and gf.b[0, 0] == 0.7 and gf.q[0, 0] == 0.7


def test_luma_weights():
    I = np.array([[[255, 0, 0], [0, 255, 0], [0, 0, 255], [255, 255, 255]]], dtype=np.uint8)
    g = oracle.luma(I)
    assert np.allclose(g[0], [0.299, 0.587, 0.114, 1.0], rtol=0, atol=1e-15)


# ------------------------------------------------- reconstruction and post
def test_reconstruct_hand_value_and_clamp():
    I = np.array([[[100, 200, 50]]], dtype=np.uint8)
    A = np.array([150.0, 150.0, 150.0])
    t = np.array([[0.5]])
    J = oracle.reconstruct(I, A, t)
    assert np.array_equal(J[0, 0], [50.0, 250.0, 0.0])   # (50-150)/.5+150 = -50 -> 0


def test_gamma_closed_forms():
    J = np.linspace(0, 255, 101)
    assert np.array_equal(oracle.gamma_correct(J, 1.0), J)
    assert abs(oracle.gamma_correct(np.array([127.5]), 2.0)[0] - 255.0 * math.sqrt(0.5)) < 1e-12
    g = float(np.float32(1.2))
    assert abs(oracle.gamma_correct(np.array([51.0]), 1.2)[0] - 255.0 * 0.2 ** (1.0 / g)) < 1e-12


def test_gray_world_identity_and_known_gains():
    gray = np.full((8, 8, 3), 100.0)
    out, gains = oracle.gray_world(gray)
    assert np.array_equal(out, gray) and np.array_equal(gains, [1, 1, 1])
    img = np.empty((4, 4, 3))
    img[..., 0], img[..., 1], img[..., 2] = 60.0, 120.0, 180.0
    out, gains = oracle.gray_world(img)
    assert np.allclose(gains, [2.0, 1.0, 2.0 / 3.0], rtol=0, atol=1e-15)
    assert np.allclose(out, 120.0)
    img[..., 2] = 0.0
    out, gains = oracle.gray_world(img)
    assert gains[2] == 1.0


def test_rne():
    x = np.array([0.5, 1.5, 2.5, 254.5, 255.4, -3.0, 300.0])
    assert list(oracle.rne_u8(x)) == [0, 2, 2, 254, 255, 0, 255]


# ----------------------------------------------------------- whole frame
@pytest.mark.parametrize("tx", ["he", "paper"])
def test_pipeline_is_identity_with_omega_zero(tx):
    fr = make_frame(64, 48, 8, beta=1.2)
    p = Params(mode="realtime", omega=0.0, gamma=1.0, tx=tx)
    res = oracle.dehaze(fr.I, p)
    assert np.array_equal(res.out, fr.I)


def test_pipeline_offline_runs_and_bounds():
    fr = make_frame(96, 80, 9)
    p = Params(mode="offline", gf_radius=8, color_balance=True)
    res = oracle.dehaze(fr.I, p)
    t = res.aux["t"]
    assert t.min() >= float(np.float32(0.1)) and t.max() <= 1.0
    assert res.out.dtype == np.uint8 and res.out.shape == fr.I.shape


# ------------------------------------------------------------ resize (Sec. V step 1)
RESIZE_CASES = [((16, 12), (16, 12)), ((16, 12), (8, 6)), ((1920, 1080), (640, 480)),
                ((37, 23), (11, 7)), ((11, 7), (37, 23)), ((9, 5), (1, 1)), ((1, 1), (5, 3)),
                ((1, 9), (4, 2)), ((64, 48), (63, 47)), ((40, 30), (40, 31))]


def test_resize_same_size_is_identity():
    I = rng(71).integers(0, 256, (23, 37, 3), dtype=np.uint8)
    assert np.array_equal(oracle.resize(I, 37, 23), I)


def test_resize_halving_is_the_rounded_block_mean():
    # at ratio 2 every output sits midway between four inputs: weights 1/2, 1/2
    I = rng(72).integers(0, 256, (12, 16, 3), dtype=np.uint8)
    block = I.astype(np.int64).reshape(6, 2, 8, 2, 3).sum(axis=(1, 3))
    assert np.array_equal(oracle.resize(I, 8, 6), ((block + 2) >> 2).astype(np.uint8))


def test_resize_constant_frame_stays_constant():
    I = np.full((21, 34, 3), (7, 130, 255), dtype=np.uint8)
    for w, h in [(5, 4), (34, 21), (70, 50), (1, 1)]:
        assert np.all(oracle.resize(I, w, h) == np.array([7, 130, 255], dtype=np.uint8))


@pytest.mark.parametrize("src,dst", RESIZE_CASES)
def test_resize_matches_library_bilinear(src, dst):
    # torch's bilinear interpolation (pixel centres aligned, no antialiasing) in
    # float64 is the exact value the oracle approximates: weights rounded to
    # 2^-11 move each one-axis interpolation by at most 255 * 2^-12, so the
    # value before the final rounding is within 2 * 255 * 2^-12 < 0.125 of it
    import torch
    w, h = src
    I = rng(73 + w + 1000 * h).integers(0, 256, (h, w, 3), dtype=np.uint8)
    ref = torch.nn.functional.interpolate(
        torch.from_numpy(I.astype(np.float64)).permute(2, 0, 1)[None], size=(dst[1], dst[0]),
        mode="bilinear", align_corners=False, antialias=False)[0].permute(1, 2, 0).numpy()
    out = oracle.resize(I, dst[0], dst[1]).astype(np.float64)
    assert out.shape == ref.shape
    assert np.max(np.abs(out - ref)) <= 0.5 + 0.125
    # away from a rounding boundary the integer result is the rounded exact value
    safe = np.abs(ref - np.floor(ref) - 0.5) > 0.125
    assert np.array_equal(out[safe], np.floor(ref[safe] + 0.5))


def test_resize_taps_bruteforce():
    # taps and weights from the coordinate formula evaluated in exact rationals
    from fractions import Fraction
    for n_in, n_out in [(1920, 640), (7, 3), (3, 7), (1, 4), (5, 1), (480, 1080)]:
        i0, i1, w1 = oracle.resize_taps(n_in, n_out)
        for i in range(n_out):
            s = max(Fraction(2 * i + 1, 2) * Fraction(n_in, n_out) - Fraction(1, 2), Fraction(0))
            f0 = math.floor(s)
            assert i0[i] == f0 and i1[i] == min(f0 + 1, n_in - 1)
            assert w1[i] == math.floor((s - f0) * 2048 + Fraction(1, 2))


def test_pipeline_with_resize_runs_at_the_target_size():
    I = make_frame(96, 64, 9).I
    p = Params(resize_width=48, resize_height=40)
    r = oracle.dehaze(I, p)
    assert r.out.shape == (40, 48, 3)
    assert np.array_equal(r.aux["I"], oracle.resize(I, 48, 40))
    assert np.array_equal(r.out, oracle.dehaze(oracle.resize(I, 48, 40), Params()).out)


# ------------------------------------------------------------ temporal airlight smoothing
def _clip(n, seed=0):
    return [make_frame(64, 48, seed + k, beta=0.5 + 0.2 * k).I for k in range(n)]


def test_smoothing_zero_keeps_frames_independent():
    frames = _clip(4)
    seq = oracle.dehaze_sequence(frames, Params(airlight_smoothing=0.0))
    for I, r in zip(frames, seq):
        alone = oracle.dehaze(I, Params())
        assert np.array_equal(r.aux["A"], alone.aux["A"])
        assert np.array_equal(r.out, alone.out)


def test_smoothing_of_a_repeated_frame_stays_at_its_estimate():
    I = _clip(1)[0]
    seq = oracle.dehaze_sequence([I] * 6, Params(airlight_smoothing=0.9))
    A_hat = seq[0].aux["A_hat"]
    for r in seq:
        assert np.allclose(r.aux["A"], A_hat, rtol=1e-6, atol=0)


def test_smoothing_matches_the_closed_form():
    # A_t = lam^t Ahat_0 + (1 - lam) sum_{k=1..t} lam^(t-k) Ahat_k, up to the float32 storage of
    # each A between frames
    lam = 0.6
    seq = oracle.dehaze_sequence(_clip(6, seed=10), Params(airlight_smoothing=lam))
    lam = float(np.float32(lam))
    hats = [r.aux["A_hat"] for r in seq]
    for t, r in enumerate(seq):
        closed = lam ** t * hats[0] + (1 - lam) * sum(lam ** (t - k) * hats[k] for k in range(1, t + 1))
        assert np.allclose(r.aux["A"], closed, rtol=1e-6, atol=0), t


def test_smoothing_step_response():
    # a frame with estimate a followed by frames with estimate b: A_t - b = lam^t (a - b)
    a_frame, b_frame = _clip(2, seed=20)
    lam = 0.5
    seq = oracle.dehaze_sequence([a_frame] + [b_frame] * 5, Params(airlight_smoothing=lam))
    a, b = seq[0].aux["A_hat"], seq[1].aux["A_hat"]
    for t in range(1, 6):
        assert np.allclose(seq[t].aux["A"] - b, lam ** t * (a - b), rtol=1e-5, atol=1e-4), t


def test_smoothed_airlight_drives_transmission_and_recovery():
    f0, f1 = _clip(2, seed=30)
    seq = oracle.dehaze_sequence([f0, f1], Params(airlight_smoothing=0.7, mode="offline", gf_radius=8))
    injected = oracle.dehaze(f1, Params(mode="offline", gf_radius=8), A_inject=seq[1].aux["A"])
    assert np.array_equal(seq[1].out, injected.out)
    assert not np.array_equal(seq[1].aux["A"], seq[1].aux["A_hat"])


# ------------------------------------------------------------ adaptive gamma
def test_adaptive_gamma_maps_a_constant_frame_to_the_target():
    # for a constant gray J = v the mean luma is v/255, and (v/255)^(1/gamma) = tau exactly
    for v, tau in [(60.0, 0.5), (128.0, 0.45), (200.0, 0.6), (90.0, 0.3), (10.0, 0.5), (250.0, 0.5)]:
        J = np.full((6, 9, 3), v)
        g = oracle.adaptive_gamma(J, tau)
        raw = math.log(v / 255.0) / math.log(float(np.float32(tau)))
        assert g == pytest.approx(min(max(raw, 0.5), 2.0), rel=1e-15)
        if 0.5 < g < 2.0:
            assert np.allclose(oracle.gamma_power(J, g), 255.0 * float(np.float32(tau)), rtol=1e-12)


def test_adaptive_gamma_weights_and_clamps():
    # one channel at a time: the BT.601 weight of that channel sets the mean luma
    for c, wgt in enumerate((0.299, 0.587, 0.114)):
        J = np.zeros((4, 4, 3))
        J[:, :, c] = 255.0
        # tau = 3/8 is exact in binary32
        assert oracle.adaptive_gamma(J, 0.375) == pytest.approx(
            min(max(math.log(wgt) / math.log(0.375), 0.5), 2.0), rel=1e-12)
    assert oracle.adaptive_gamma(np.zeros((3, 3, 3)), 0.5) == 2.0         # black: mu floored, gamma clamped
    assert oracle.adaptive_gamma(np.full((3, 3, 3), 255.0), 0.5) == 0.5   # white: ln(1) = 0, clamped
    # the mean is over every pixel: half black, half of a level
    J = np.zeros((2, 8, 3))
    J[:, :4] = 200.0
    assert oracle.adaptive_gamma(J, 0.5) == pytest.approx(math.log(100.0 / 255.0) / math.log(0.5), rel=1e-12)


def test_pipeline_with_adaptive_gamma_uses_the_frame_gamma():
    I = (make_frame(64, 48, 5).I * 0.35).astype(np.uint8)   # a darker frame: gamma inside the clamp
    r = oracle.dehaze(I, Params(gamma_adaptive=True, gamma_target=0.5))
    assert 0.5 < r.aux["gamma"] < 2.0
    g = r.aux["gamma"]
    assert g == oracle.adaptive_gamma(r.aux["J"], 0.5)
    assert np.allclose(r.aux["Jg"], 255.0 * (r.aux["J"] / 255.0) ** (1.0 / g), rtol=1e-14, atol=0)
    # brighter target -> lower gamma exponent 1/gamma -> brighter output on average
    r2 = oracle.dehaze(I, Params(gamma_adaptive=True, gamma_target=0.7))
    assert r2.aux["gamma"] > g and r2.out.mean() > r.out.mean()


# ------------------------------------------------- percentile ("simple") white balance
def test_percentile_points_hand_example():
    # ten codes, p = 0.1 -> k = 1: lo is the 2nd smallest, hi the 2nd largest (worked by hand)
    q = np.array([20, 3, 41, 7, 3, 40, 21, 9, 40, 20])
    assert oracle.percentile_points(q, 0.1) == (3, 40)
    # p = 0 -> the extremes; p = 0.3 -> k = 3: sorted 3 3 7 9 20 20 21 40 40 41
    assert oracle.percentile_points(q, 0.0) == (3, 41)
    assert oracle.percentile_points(q, 0.3) == (9, 21)


@pytest.mark.parametrize("seed", range(6))
def test_percentile_points_match_a_sort(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 5000))
    q = rng.integers(0, 256, size=n) if seed % 2 else np.clip(rng.normal(120, 30, n), 0, 255).astype(int)
    p = float(rng.choice([0.0, 0.001, 0.02, 0.1, 0.3]))
    k = math.floor(float(np.float32(p)) * n)
    srt = np.sort(q)
    assert oracle.percentile_points(q, p) == (int(srt[k]), int(srt[n - 1 - k]))


def test_percentile_stretch_of_a_ramp_is_the_closed_form():
    x = np.arange(256, dtype=np.float64)
    Jg = np.stack([x, x, x], axis=-1).reshape(16, 16, 3)
    p = 10 / 256                               # float32-exact: k = 10
    out, points, _ = oracle.percentile_stretch(Jg, p)
    assert points == [(10, 245)] * 3
    want = np.clip((x - 10) * 255.0 / 235.0, 0, 255).reshape(16, 16)
    for c in range(3):
        np.testing.assert_allclose(out[..., c], want, rtol=0, atol=1e-12)
    assert out[..., 0].reshape(-1)[10] == 0.0 and abs(out[..., 0].reshape(-1)[245] - 255.0) < 1e-9


def test_percentile_stretch_identity_and_flat_channel():
    rng = np.random.default_rng(3)
    Jg = rng.uniform(0, 255, size=(20, 30, 3))
    Jg[0, 0, :] = 0.0
    Jg[0, 1, :] = 255.0
    Jg[..., 2] = 77.3                          # a flat channel: hi == lo, left as it is
    out, points, _ = oracle.percentile_stretch(Jg, 0.0)
    assert points[0] == (0, 255) and points[1] == (0, 255) and points[2] == (77, 77)
    np.testing.assert_array_equal(out, Jg)


def test_percentile_candidates_widen_only_near_half_codes():
    x = np.full((1, 10), 50.2)
    x[0, :3] = 10.4999                         # within the band of a half-integer: code 10 or 11
    Jg = np.stack([x, x, x], axis=-1)
    _, points, cands = oracle.percentile_stretch(Jg, 0.2, band=1e-3)    # k = 2: lo = 3rd smallest
    assert points[0] == (10, 50)
    assert cands[0] == ((10, 11), (50, 50))
    _, _, cands0 = oracle.percentile_stretch(Jg, 0.2, band=0.0)
    assert cands0[0] == ((10, 10), (50, 50))


def test_pipeline_percentile_balance_stretches_each_channel():
    I = make_frame(96, 64, 5, beta=1.2).I
    base = oracle.dehaze(I, Params())
    r = oracle.dehaze(I, Params(color_balance=2, wb_percentile=0.02))
    q = oracle.rne_u8(base.aux["Jg"])
    n = q.shape[0] * q.shape[1]
    k = math.floor(float(np.float32(0.02)) * n)
    for c in range(3):
        srt = np.sort(q[..., c].reshape(-1))
        lo, hi = int(srt[k]), int(srt[n - 1 - k])
        assert r.aux["wb_points"][c] == (lo, hi)
        # pixels at or below the black point map to 0, at or above the white point to 255
        assert np.all(r.out[..., c][q[..., c] < lo] == 0)
        assert np.all(r.out[..., c][q[..., c] > hi] == 255)
    # the stretch is monotone per channel
    for c in range(3):
        order = np.argsort(base.aux["Jg"][..., c], axis=None)
        assert np.all(np.diff(r.aux["Jf"][..., c].reshape(-1)[order]) >= 0)
    # with p = 0 on a frame whose channels already span 0..255 nothing changes
    Jspan = base.aux["Jg"].copy()
    Jspan[0, 0, :], Jspan[0, 1, :] = 0.0, 255.0
    out0, _, _ = oracle.percentile_stretch(Jspan, 0.0)
    np.testing.assert_array_equal(out0, Jspan)
