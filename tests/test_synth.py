"""The seeded generator: deterministic, the prior holds, and the recipe's ranges."""
import numpy as np

import oracle
from synth import make_frame, make_scene, make_streams, make_video, sha256_u8


def test_generator_is_deterministic():
    a = make_frame(160, 120, 42)
    b = make_frame(160, 120, 42)
    c = make_frame(160, 120, 43)
    assert sha256_u8(a.I) == sha256_u8(b.I)
    assert sha256_u8(a.I) != sha256_u8(c.I)


def test_scene_ranges_and_prior():
    s = make_scene(128, 96, 7)
    assert s.J.min() >= 0.0 and s.J.max() <= 0.95 + 1e-12
    assert s.depth.min() >= 0.0 and s.depth.max() <= 3.0
    # every aligned 8x8 block has one channel <= 0.02, so a 15x15 window's dark channel is tiny
    dark = oracle.erode(s.J.min(axis=2), 15)
    assert dark.max() <= 0.02


def test_frame_shapes_and_airlight_range():
    f = make_frame(320, 240, 1, beta=1.0)
    assert f.I.shape == (240, 320, 3) and f.I.dtype == np.uint8
    assert np.all(np.abs(f.A - np.array([0.85, 0.88, 0.90])) <= 0.02)
    assert np.allclose(f.t, np.exp(-1.0 * -np.log(f.t)))


def test_video_pans_and_drifts():
    v = make_video(160, 96, nframes=12, seed=3, pan=40, y_off=8)
    f0, f5 = v.frame(0), v.frame(5)
    assert f0.I.shape == (96, 160, 3)
    b0, A0, x0, _ = v.params(0)
    b11, _, x11, _ = v.params(11)
    assert x0 == 0 and x11 == 40
    assert 0.6 <= b0 <= 1.6 and 0.6 <= b11 <= 1.6
    assert sha256_u8(f0.I) != sha256_u8(f5.I)


def test_streams_are_seeded():
    a = make_streams(8, seconds=2.0)
    b = make_streams(8, seconds=2.0)
    assert [(s.width, s.height, s.offline, len(s.arrivals)) for s in a] == \
           [(s.width, s.height, s.offline, len(s.arrivals)) for s in b]
    for s in a:
        assert np.all(np.diff(s.arrivals) > 0)
