"""Seeded synthetic hazy frames.

This module only *generates inputs*: it renders a clear scene J, a depth map,
a transmission t = exp(-beta * d) and an airlight A, and composes a hazy frame
with the atmospheric scattering model (paper Sec. III, Eq. (1)),
I = J * t + A * (1 - t), plus a little Gaussian sensor noise, quantised to
uint8.  It holds none of the dehazing arithmetic and is shared by the oracle
tests, the GPU parity tests and the benchmark so that both sides see identical
bytes.

Scene recipe (all values in [0, 1] until the final x255):
  * clear radiance J: per channel, 4 octaves of value noise on lattices of
    128/64/32/16 px with amplitude 0.5**o and quintic smoothstep interpolation,
    mapped affinely to [0.05, 0.95];
  * 16 constant-colour axis-aligned rectangles (5-30 % of each side) for edges;
  * the dark-channel prior is forced to hold: in every aligned 8x8 block one
    randomly chosen channel is replaced by U[0, 0.02];
  * depth: 6 Voronoi cells, each a plane d0 + gx*x/W + gy*y/H with
    d0 ~ U[0, 3], gx, gy ~ U[-1, 1], clipped to [0, 3];
  * airlight A = (0.85, 0.88, 0.90) + U[-0.02, 0.02]^3;
  * I = J t + A (1 - t) + N(0, 0.005), x255, round half to even, clip, uint8.

Frames are H x W x 3 (RGB, row-major, channel-interleaved).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np

A_BASE = np.array([0.85, 0.88, 0.90])
NOISE_SIGMA = 0.005


def _rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _quintic(u: np.ndarray) -> np.ndarray:
    return u * u * u * (u * (u * 6.0 - 15.0) + 10.0)


def _value_noise(rng: np.random.Generator, h: int, w: int, cell: int) -> np.ndarray:
    gh, gw = h // cell + 2, w // cell + 2
    lat = rng.random((gh, gw))
    ys = np.arange(h) / cell
    xs = np.arange(w) / cell
    y0 = np.floor(ys).astype(np.int64)
    x0 = np.floor(xs).astype(np.int64)
    fy = _quintic(ys - y0)[:, None]
    fx = _quintic(xs - x0)[None, :]
    v00 = lat[np.ix_(y0, x0)]
    v01 = lat[np.ix_(y0, x0 + 1)]
    v10 = lat[np.ix_(y0 + 1, x0)]
    v11 = lat[np.ix_(y0 + 1, x0 + 1)]
    top = v00 + (v01 - v00) * fx
    bot = v10 + (v11 - v10) * fx
    return top + (bot - top) * fy


@dataclass
class Scene:
    """A static clear scene: radiance J (H,W,3) and depth d (H,W), float64."""

    J: np.ndarray
    depth: np.ndarray


def make_scene(width: int, height: int, seed: int) -> Scene:
    rng = _rng(seed)
    h, w = height, width
    J = np.empty((h, w, 3))
    for c in range(3):
        acc = np.zeros((h, w))
        for o, cell in enumerate((128, 64, 32, 16)):
            acc += (0.5 ** o) * _value_noise(rng, h, w, cell)
        lo, hi = acc.min(), acc.max()
        J[:, :, c] = 0.05 + 0.9 * (acc - lo) / max(hi - lo, 1e-12)
    # edges: constant-colour rectangles
    for _ in range(16):
        rw = max(1, int(round(w * rng.uniform(0.05, 0.30))))
        rh = max(1, int(round(h * rng.uniform(0.05, 0.30))))
        x0 = int(rng.integers(0, max(1, w - rw + 1)))
        y0 = int(rng.integers(0, max(1, h - rh + 1)))
        J[y0:y0 + rh, x0:x0 + rw, :] = rng.uniform(0.05, 0.95, size=3)
    # the prior holds by construction: one channel per aligned 8x8 block is ~0
    bh, bw = (h + 7) // 8, (w + 7) // 8
    chan = rng.integers(0, 3, size=(bh, bw))
    dark = rng.uniform(0.0, 0.02, size=(h, w))
    cmap = np.repeat(np.repeat(chan, 8, axis=0), 8, axis=1)[:h, :w]
    for c in range(3):
        sel = cmap == c
        J[:, :, c][sel] = dark[sel]
    # depth: piecewise-planar Voronoi cells
    ncell = 6
    sx = rng.uniform(0, w, size=ncell)
    sy = rng.uniform(0, h, size=ncell)
    d0 = rng.uniform(0.0, 3.0, size=ncell)
    gx = rng.uniform(-1.0, 1.0, size=ncell)
    gy = rng.uniform(-1.0, 1.0, size=ncell)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    best = np.full((h, w), np.inf)
    lab = np.zeros((h, w), dtype=np.int64)
    for k in range(ncell):
        dk = (xx - sx[k]) ** 2 + (yy - sy[k]) ** 2
        closer = dk < best
        best[closer] = dk[closer]
        lab[closer] = k
    depth = d0[lab] + gx[lab] * xx / w + gy[lab] * yy / h
    depth = np.clip(depth, 0.0, 3.0)
    return Scene(J=J, depth=depth)


def haze(J: np.ndarray, t: np.ndarray, A: np.ndarray, noise_rng=None,
         sigma: float = NOISE_SIGMA) -> np.ndarray:
    """Compose I = J t + A (1 - t) (+ noise) in [0,1] float64 (scattering model)."""
    I = J * t[..., None] + A[None, None, :] * (1.0 - t[..., None])
    if noise_rng is not None and sigma > 0:
        I = I + noise_rng.normal(0.0, sigma, size=I.shape)
    return I


def quantize_u8(I01: np.ndarray) -> np.ndarray:
    return np.clip(np.rint(I01 * 255.0), 0, 255).astype(np.uint8)


@dataclass
class Frame:
    I: np.ndarray        # (H, W, 3) uint8 hazy frame
    J: np.ndarray        # (H, W, 3) float64 clear radiance in [0, 1]
    t: np.ndarray        # (H, W) float64 transmission
    A: np.ndarray        # (3,) float64 airlight in [0, 1]
    beta: float


def make_frame(width: int, height: int, seed: int, beta=None, A=None,
               noise: bool = True) -> Frame:
    """One hazy frame. beta defaults to U[0.5, 2.0] and A to A_BASE +- 0.02."""
    scene = make_scene(width, height, seed)
    rng = _rng((seed, 1))
    if beta is None:
        beta = float(rng.uniform(0.5, 2.0))
    if A is None:
        A = A_BASE + rng.uniform(-0.02, 0.02, size=3)
    A = np.asarray(A, dtype=np.float64)
    t = np.exp(-beta * scene.depth)
    I01 = haze(scene.J, t, A, noise_rng=_rng((seed, 2)) if noise else None)
    return Frame(I=quantize_u8(I01), J=scene.J, t=t, A=A, beta=beta)


# ---------------------------------------------------------------- video (C3)
@dataclass
class Video:
    scene: Scene
    width: int
    height: int
    nframes: int
    A0: np.ndarray
    seed: int
    pan: int = 320
    y_off: int = 90

    def params(self, f: int):
        phase = 2.0 * np.pi * f / self.nframes
        beta = 1.1 + 0.5 * np.sin(phase)
        A = self.A0 + 0.03 * np.sin(phase + 2.0 * np.pi * np.arange(3) / 3.0)
        x = int(round(f * self.pan / max(self.nframes - 1, 1)))
        return beta, A, x, self.y_off

    def frame(self, f: int) -> Frame:
        beta, A, x, y = self.params(f)
        J = self.scene.J[y:y + self.height, x:x + self.width]
        d = self.scene.depth[y:y + self.height, x:x + self.width]
        t = np.exp(-beta * d)
        I01 = haze(J, t, A, noise_rng=_rng((self.seed, 3, f)))
        return Frame(I=quantize_u8(I01), J=J, t=t, A=A, beta=beta)


def make_video(width: int = 1280, height: int = 720, nframes: int = 300,
               seed: int = 3, pan: int = 320, y_off: int = 90) -> Video:
    """A static seeded scene seen through a slowly panning crop.

    The canvas is (width + pan) x (height + 2*y_off); beta drifts as
    1.1 + 0.5 sin(2 pi f / n) and A^c as A0^c + 0.03 sin(2 pi f / n + 2 pi c / 3).
    """
    scene = make_scene(width + pan, height + 2 * y_off, seed)
    rng = _rng((seed, 4))
    A0 = A_BASE + rng.uniform(-0.02, 0.02, size=3)
    return Video(scene=scene, width=width, height=height, nframes=nframes,
                 A0=A0, seed=seed, pan=pan, y_off=y_off)


# ------------------------------------------------------------ streams (C5)
RESOLUTIONS = {"480p": (640, 480), "720p": (1280, 720),
               "1080p": (1920, 1080), "4k": (3840, 2160)}


@dataclass
class StreamSpec:
    index: int
    width: int
    height: int
    offline: bool
    arrivals: np.ndarray   # seconds, sorted
    seed: int


def make_streams(n: int = 32, seconds: float = 10.0, rate: float = 30.0,
                 seed: int = 5, p_offline: float = 0.2,
                 resolutions=("480p", "720p", "1080p", "4k")):
    """Per-stream resolution, mode and Poisson arrival times (seeded)."""
    rng = _rng(seed)
    out = []
    for s in range(n):
        res = resolutions[int(rng.integers(0, len(resolutions)))]
        w, h = RESOLUTIONS[res]
        offline = bool(rng.random() < p_offline)
        srng = _rng(5000 + s)
        ts, acc = [], 0.0
        while True:
            acc += srng.exponential(1.0 / rate)
            if acc >= seconds:
                break
            ts.append(acc)
        out.append(StreamSpec(index=s, width=w, height=h, offline=offline,
                              arrivals=np.asarray(ts), seed=5000 + s))
    return out


def batch_shapes_c4():
    """The uneven 64-frame batch: 16 each of 480p, 720p, 1080p and 4K."""
    shapes = []
    for res in ("480p", "720p", "1080p", "4k"):
        shapes += [RESOLUTIONS[res]] * 16
    return shapes


def sha256_u8(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
