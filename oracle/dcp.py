"""FP64 CPU oracle for the per-frame Dark-Channel-Prior dehazing path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, calls or links this module; only the tests, the
smoke check and the CPU-baseline leg of the benchmark do.  It shares no code,
tables or constants with the GPU implementation.

Every step follows the paper's statement of the method (Hazedefy, arXiv
2512.16609) in the paper's order, in plain float64 NumPy:

  Sec. IV-A, Eq. (2)   dark channel: per-pixel channel minimum, then the
                       minimum over a square patch (morphological erosion)
  Sec. IV-B, Eq. (3)   airlight: mean RGB of the K brightest dark-channel
                       pixels, scaled by alpha = 0.8
  Sec. IV-C, Eqs. (4)-(5)  transmission with a lower clamp
  Sec. IV-D, Eq. (6)   guided-filter refinement (He et al. 2013 box form)
  Sec. IV-E, Eqs. (7)-(8)  radiance recovery and gamma correction, then the
                       optional colour balance
  Sec. V               per-frame step order and the real-time/offline branch

Where the paper is silent the oracle takes these readings (each is also a
parameter or a documented choice of the GPU library):
  * parameters are binary32 values (the C ABI carries floats); the oracle
    converts each to its float32 value before computing in float64;
  * erosion and box windows are clipped at the frame border (a clipped box is
    normalised by its own pixel count);
  * K = max(1, floor(top_frac * W * H)); the K pixels are the first K in the
    order (D descending, raster index ascending), so the set is unique;
  * A^c is the alpha-scaled mean of the hazy input over the set; as a divisor
    it is guarded as max(A^c, 1) on the 0..255 scale;
  * default transmission ("he"): t = max(1 - omega * dark(I / A), t0), where
    dark(I / A) is the patch minimum of min_c I^c / A^c; the literal Eq. (4)
    ("paper"): t = max(1 - omega * min_c I^c(x) / max_c A^c, t0), pointwise;
  * the guided filter refines the clamped t with the BT.601 luma of the hazy
    input scaled to [0, 1] as guide, and its output is clamped to [t0, 1];
  * J is clamped to [0, 255] before the gamma of Eq. (8);
  * colour balance is gray-world on the gamma-corrected image:
    g_c = mean(mu) / mu_c (g_c = 1 when mu_c = 0), J_c <- min(255, g_c J_c);
  * the second balance (the "simple" white balance by percentiles): per
    channel, the black and white points are the low and high percentiles of
    the channel's unbalanced output codes q = RNE(J_gamma): with k =
    floor(p W H), lo is the (k+1)-th smallest and hi the (k+1)-th largest
    code; the channel is stretched linearly, J_c <- clamp((J_c - lo) 255 /
    (hi - lo), 0, 255), and left as it is when hi <= lo;
  * the output is rounded half to even and saturated to uint8;
  * the optional resize of Sec. V step 1 (the paper names no interpolation) is
    bilinear sampling with pixel centres aligned, source coordinates clamped
    below at 0 and taps clamped at the last row/column, weights rounded to
    multiples of 2^-11 (half up) and the result rounded half up to uint8;
    every step is exact integer arithmetic;
  * optional temporal smoothing of the airlight over a stream's frames (the
    flicker concern of Sec. V): A_t = lam A_{t-1} + (1 - lam) Ahat_t, where
    Ahat_t is the frame's own Eq. (3) estimate (float64) and A_{t-1} is the
    previous frame's A as stored (float32); the sum is formed in float64 as
    (lam * A_{t-1}) + ((1 - lam) * Ahat_t).  The first frame takes A = Ahat;
  * the "gamma-adaptive" correction named in the abstract has no rule in the
    paper; the reading here picks, per frame, the gamma that maps the mean
    BT.601 luma mu of the recovered J (on [0, 1]) to a target tau:
    mu^(1/gamma) = tau, i.e. gamma = ln(mu) / ln(tau), with mu floored at
    2^-20 and gamma clamped to [1/2, 2].
All functions are pinned by tests against brute force, closed forms,
invariants or independent library routines (scipy.ndimage).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def f32(x) -> float:
    """The float32 value of a parameter, as a float64 (the ABI carries binary32)."""
    return float(np.float32(x))


@dataclass
class Params:
    mode: str = "realtime"         # "realtime" (no guided filter) or "offline"
    patch: int = 15                # odd side of the square patch Omega
    omega: float = 0.95            # transmission weight of Eq. (4)
    t0: float = 0.1                # lower bound t_min of Eq. (5)
    top_frac: float = 0.001        # fraction of pixels averaged in Eq. (3)
    alpha: float = 0.8             # airlight scale of Eq. (3)
    gamma: float = 1.2             # gamma of Eq. (8)
    gf_radius: int = 60            # guided-filter box radius r
    gf_eps: float = 1e-3           # guided-filter regulariser epsilon
    color_balance: int = 0         # 0 none, 1 gray-world, 2 percentile stretch (True = 1)
    wb_percentile: float = 0.02    # fraction p of pixels ignored at each end of each channel (balance 2)
    tx: str = "he"                 # "he" (dark(I/A)) or "paper" (literal Eq. (4))
    resize_width: int = 0          # Sec. V step 1 target size; 0 x 0 = native size
    resize_height: int = 0
    airlight_smoothing: float = 0.0  # lam of the temporal airlight average; 0 = none
    gamma_adaptive: bool = False     # per-frame gamma from the mean luma of J (gamma unused)
    gamma_target: float = 0.5        # tau: the mean luma the adaptive gamma aims for

    def f(self, name):
        return f32(getattr(self, name))


# ------------------------------------------------------------- Sec. V, step 1
RESIZE_BITS = 11   # fractional bits of the bilinear weights


def resize_taps(n_in: int, n_out: int):
    """Source taps and weights of bilinear resampling along one axis.

    Output sample i sits at source coordinate s = (i + 1/2) n_in / n_out - 1/2
    (pixel centres aligned), with s < 0 taken as 0.  Its taps are i0 = floor(s)
    and i1 = min(i0 + 1, n_in - 1); the weight of i1 is the fractional part of
    s rounded half up to a multiple of 2^-RESIZE_BITS, returned as an integer
    numerator w1 (the weight of i0 is 2^RESIZE_BITS - w1).  s is carried as
    the exact rational ((2i + 1) n_in - n_out) / (2 n_out).
    """
    i = np.arange(n_out, dtype=np.int64)
    num = np.maximum((2 * i + 1) * n_in - n_out, 0)
    den = 2 * n_out
    i0 = num // den
    frac = num - i0 * den
    w1 = (frac * (1 << (RESIZE_BITS + 1)) + den) // (2 * den)
    i1 = np.minimum(i0 + 1, n_in - 1)
    return i0, i1, w1


def resize(I: np.ndarray, width: int, height: int) -> np.ndarray:
    """Sec. V step 1: the frame resized to width x height (uint8 RGB).

    Bilinear interpolation with the taps and weights of resize_taps, first
    along rows then along columns, in exact integers; the value
    sum w_y w_x I / 2^(2 RESIZE_BITS) is rounded half up.
    """
    assert I.dtype == np.uint8 and width >= 1 and height >= 1
    h, w, _ = I.shape
    x0, x1, wx = resize_taps(w, width)
    y0, y1, wy = resize_taps(h, height)
    one = 1 << RESIZE_BITS
    X = I.astype(np.int64)
    wx = wx[None, :, None]
    h0 = (one - wx) * X[y0][:, x0] + wx * X[y0][:, x1]
    h1 = (one - wx) * X[y1][:, x0] + wx * X[y1][:, x1]
    wy = wy[:, None, None]
    v = (one - wy) * h0 + wy * h1
    half = 1 << (2 * RESIZE_BITS - 1)
    return ((v + half) >> (2 * RESIZE_BITS)).astype(np.uint8)


# ------------------------------------------------------------- Sec. IV-A
def channel_min(I: np.ndarray) -> np.ndarray:
    """min over c in {r,g,b} of I^c(x): the inner minimum of Eq. (2)."""
    return I.min(axis=2)


def _pad_value(x: np.ndarray):
    if np.issubdtype(x.dtype, np.integer):
        return np.iinfo(x.dtype).max
    return np.inf


def erode(x: np.ndarray, patch: int) -> np.ndarray:
    """Minimum of x over the patch x patch window centred at each pixel.

    The window is clipped to the frame: the frame is padded with a value no
    smaller than any pixel, so padded cells never win.  Written as the
    definition (the minimum over every offset in the window), vectorised over
    pixels only.
    """
    assert patch >= 1 and patch % 2 == 1
    r = (patch - 1) // 2
    h, w = x.shape
    pv = _pad_value(x)
    pad = np.full((h + 2 * r, w + 2 * r), pv, dtype=x.dtype)
    pad[r:r + h, r:r + w] = x
    out = np.full((h, w), pv, dtype=x.dtype)
    for dy in range(patch):
        for dx in range(patch):
            np.minimum(out, pad[dy:dy + h, dx:dx + w], out=out)
    return out


def erode_bruteforce(x: np.ndarray, patch: int) -> np.ndarray:
    """Per-pixel loop over the clipped window (tiny inputs only)."""
    r = (patch - 1) // 2
    h, w = x.shape
    out = np.empty_like(x)
    for y in range(h):
        for xx in range(w):
            out[y, xx] = x[max(0, y - r):min(h, y + r + 1),
                           max(0, xx - r):min(w, xx + r + 1)].min()
    return out


def dark_channel(I: np.ndarray, patch: int) -> np.ndarray:
    """Eq. (2): D(x) = min over Omega(x) of min_c I^c."""
    return erode(channel_min(I), patch)


def channel_erosions(I: np.ndarray, patch: int) -> np.ndarray:
    """E^c = erosion of each colour plane (H, W, 3)."""
    return np.stack([erode(np.ascontiguousarray(I[:, :, c]), patch)
                     for c in range(3)], axis=2)


# ------------------------------------------------------------- Sec. IV-B
def top_count(top_frac: float, n: int) -> int:
    """K = max(1, floor(top_frac * N)), top_frac taken as its float32 value."""
    return max(1, int(math.floor(f32(top_frac) * n)))


@dataclass
class Airlight:
    A: np.ndarray          # (3,) float64, 0..255 scale
    K: int
    vstar: float           # dark-channel value of the last selected pixel
    cutoff: int            # raster index of the last selected pixel with D == vstar
    sel: np.ndarray        # (K,) raster indices of the selected pixels, in sort order
    S: np.ndarray          # (3,) sum of I over the set


def airlight(I: np.ndarray, D: np.ndarray, top_frac: float, alpha: float) -> Airlight:
    """Eq. (3): A = alpha * (1/K) * sum_{i<=K} I(p_i) over the top-K dark pixels.

    The pixels are fully sorted by (D descending, raster index ascending) and
    the first K are taken.
    """
    h, w = D.shape
    n = h * w
    K = top_count(top_frac, n)
    d = D.reshape(-1)
    idx = np.arange(n)
    order = np.lexsort((idx, -d.astype(np.float64)))
    sel = order[:K]
    last = sel[-1]
    vstar = d[last]
    cutoff = int(last)
    Iflat = I.reshape(n, 3)
    if np.issubdtype(I.dtype, np.integer):
        S = Iflat[sel].astype(np.int64).sum(axis=0).astype(np.float64)
    else:
        S = Iflat[sel].astype(np.float64).sum(axis=0)
    A = f32(alpha) * S / K
    return Airlight(A=A, K=K, vstar=vstar, cutoff=cutoff, sel=sel, S=S)


def airlight_smooth(A_prev: np.ndarray, A_hat: np.ndarray, lam: float) -> np.ndarray:
    """Temporal airlight average: lam * A_prev + (1 - lam) * A_hat in float64.

    A_prev is the previous frame's airlight as stored (float32 values), A_hat
    this frame's estimate of Eq. (3); lam is taken as its float32 value.
    """
    lam = f32(lam)
    A_prev = np.asarray(A_prev, dtype=np.float32).astype(np.float64)
    return lam * A_prev + (1.0 - lam) * np.asarray(A_hat, dtype=np.float64)


def airlight_divisor(A: np.ndarray) -> np.ndarray:
    """A^c guarded as a divisor: max(A^c, 1) on the 0..255 scale."""
    return np.maximum(A, 1.0)


# ------------------------------------------------------------- Sec. IV-C
def transmission_he(I: np.ndarray, A: np.ndarray, omega: float, t0: float,
                    patch: int) -> np.ndarray:
    """t = max(1 - omega * dark(I / A), t0), dark(I/A) = erode(min_c I^c / A^c)."""
    Ad = airlight_divisor(A)
    norm = (I.astype(np.float64) / Ad[None, None, :]).min(axis=2)
    t_hat = 1.0 - f32(omega) * erode(norm, patch)
    return np.maximum(t_hat, f32(t0))


def transmission_paper(I: np.ndarray, A: np.ndarray, omega: float, t0: float) -> np.ndarray:
    """Eqs. (4)-(5) as printed: t = max(1 - omega * min_c I^c(x) / max(A), t_min)."""
    Amax = airlight_divisor(A).max()
    m = channel_min(I).astype(np.float64)
    t_hat = 1.0 - f32(omega) * m / Amax
    return np.maximum(t_hat, f32(t0))


# ------------------------------------------------------------- Sec. IV-D
def luma(I: np.ndarray) -> np.ndarray:
    """Grayscale guide: BT.601 luma of the hazy input, scaled to [0, 1]."""
    I = I.astype(np.float64)
    return (0.299 * I[:, :, 0] + 0.587 * I[:, :, 1] + 0.114 * I[:, :, 2]) / 255.0


def box_sum(x: np.ndarray, r: int) -> np.ndarray:
    """Sum of x over the (2r+1)^2 window clipped to the frame (integral image)."""
    h, w = x.shape
    S = np.zeros((h + 1, w + 1))
    S[1:, 1:] = np.cumsum(np.cumsum(x.astype(np.float64), axis=0), axis=1)
    ys = np.arange(h)
    xs = np.arange(w)
    y0 = np.clip(ys - r, 0, h)
    y1 = np.clip(ys + r + 1, 0, h)
    x0 = np.clip(xs - r, 0, w)
    x1 = np.clip(xs + r + 1, 0, w)
    return (S[np.ix_(y1, x1)] - S[np.ix_(y0, x1)]
            - S[np.ix_(y1, x0)] + S[np.ix_(y0, x0)])


def box_count(h: int, w: int, r: int) -> np.ndarray:
    ys = np.arange(h)
    xs = np.arange(w)
    ch = np.minimum(ys + r, h - 1) - np.maximum(ys - r, 0) + 1
    cw = np.minimum(xs + r, w - 1) - np.maximum(xs - r, 0) + 1
    return np.outer(ch, cw).astype(np.float64)


def box_mean(x: np.ndarray, r: int) -> np.ndarray:
    """Mean of x over the clipped (2r+1)^2 window, normalised by its pixel count."""
    return box_sum(x, r) / box_count(x.shape[0], x.shape[1], r)


def box_mean_bruteforce(x: np.ndarray, r: int) -> np.ndarray:
    h, w = x.shape
    out = np.empty((h, w))
    for y in range(h):
        for xx in range(w):
            out[y, xx] = x[max(0, y - r):min(h, y + r + 1),
                           max(0, xx - r):min(w, xx + r + 1)].astype(np.float64).mean()
    return out


@dataclass
class GuidedOut:
    q: np.ndarray
    a: np.ndarray
    b: np.ndarray


def guided_filter(p: np.ndarray, G: np.ndarray, r: int, eps: float) -> GuidedOut:
    """Eq. (6) in the box-filter formulation of He et al. (2013):
    a = cov(G,p) / (var(G) + eps), b = mean(p) - a mean(G),
    q = mean(a) G + mean(b), every mean over the clipped (2r+1)^2 window.
    """
    mean_G = box_mean(G, r)
    mean_p = box_mean(p, r)
    corr_GG = box_mean(G * G, r)
    corr_Gp = box_mean(G * p, r)
    var_G = corr_GG - mean_G * mean_G
    cov_Gp = corr_Gp - mean_G * mean_p
    a = cov_Gp / (var_G + eps)
    b = mean_p - a * mean_G
    q = box_mean(a, r) * G + box_mean(b, r)
    return GuidedOut(q=q, a=a, b=b)


# ------------------------------------------------------------- Sec. IV-E
def reconstruct(I: np.ndarray, A: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Eq. (7): J^c = (I^c - A^c) / t + A^c, then clamped to [0, 255]."""
    I = I.astype(np.float64)
    J = (I - A[None, None, :]) / t[..., None] + A[None, None, :]
    return np.clip(J, 0.0, 255.0)


def gamma_correct(J: np.ndarray, gamma: float) -> np.ndarray:
    """Eq. (8): J_gamma = 255 (J / 255)^(1/gamma)."""
    return 255.0 * np.power(J / 255.0, 1.0 / f32(gamma))


GAMMA_ADAPTIVE_MIN, GAMMA_ADAPTIVE_MAX = 0.5, 2.0
MU_FLOOR = 2.0 ** -20


def adaptive_gamma(J: np.ndarray, target: float) -> float:
    """Per-frame gamma: ln(mu) / ln(tau) for the mean luma mu of J/255, clamped.

    mu is the mean over pixels of (0.299 R + 0.587 G + 0.114 B) / 255 of the
    clamped J of Eq. (7); tau is taken as its float32 value.
    """
    mu = float(np.mean(0.299 * J[:, :, 0] + 0.587 * J[:, :, 1] + 0.114 * J[:, :, 2])) / 255.0
    g = math.log(max(mu, MU_FLOOR)) / math.log(f32(target))
    return min(max(g, GAMMA_ADAPTIVE_MIN), GAMMA_ADAPTIVE_MAX)


def gamma_power(J: np.ndarray, gamma: float) -> np.ndarray:
    """Eq. (8) with a gamma given in float64 (the adaptive case)."""
    return 255.0 * np.power(J / 255.0, 1.0 / gamma)


def gray_world(Jg: np.ndarray):
    """Gray-world colour balance: g_c = mean(mu) / mu_c, output clamped to 255."""
    mu = Jg.reshape(-1, 3).mean(axis=0)
    mbar = mu.mean()
    gains = np.where(mu > 0.0, mbar / np.where(mu > 0.0, mu, 1.0), 1.0)
    return np.minimum(255.0, Jg * gains[None, None, :]), gains


def percentile_points(q: np.ndarray, p: float):
    """Black and white points of one channel's integer codes q (any shape).

    With N codes and k = floor(p N) (p as its float32 value), lo is the
    (k+1)-th smallest code and hi the (k+1)-th largest, read off the
    256-bin histogram: lo is the smallest v with #{q <= v} > k, hi the
    largest v with #{q >= v} > k.
    """
    q = np.asarray(q).reshape(-1).astype(np.int64)
    n = q.size
    k = int(math.floor(f32(p) * n))
    hist = np.bincount(q, minlength=256)
    below = np.cumsum(hist)                  # #{q <= v}
    above = np.cumsum(hist[::-1])[::-1]      # #{q >= v}
    lo = int(np.flatnonzero(below > k)[0])
    hi = int(np.flatnonzero(above > k)[-1])
    return lo, hi


def percentile_stretch(Jg: np.ndarray, p: float, band: float = 0.0):
    """The percentile ("simple") white balance on the gamma-corrected image.

    Per channel: q = RNE(J_gamma) are the unbalanced output codes, (lo, hi)
    = percentile_points(q, p), and J_c <- clamp((J_c - lo) 255 / (hi - lo),
    0, 255), unchanged when hi <= lo.  Returns (balanced image, points,
    candidates): points[c] = (lo, hi) from these codes, and candidates[c] =
    ((lo_min, lo_max), (hi_min, hi_max)), the range each point can take when
    every value may move by up to `band` before rounding (a computation with
    that error could round codes within band of a half-integer either way).
    """
    out = np.empty_like(Jg, dtype=np.float64)
    points, cands = [], []
    for c in range(3):
        x = Jg[..., c]
        lo, hi = percentile_points(rne_u8(x), p)
        lo_a, hi_a = percentile_points(rne_u8(x - band), p)
        lo_b, hi_b = percentile_points(rne_u8(x + band), p)
        points.append((lo, hi))
        cands.append(((lo_a, lo_b), (hi_a, hi_b)))
        out[..., c] = stretch_channel(x, lo, hi)
    return out, points, cands


def stretch_channel(x: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """clamp((x - lo) 255 / (hi - lo), 0, 255); x itself when hi <= lo."""
    if hi <= lo:
        return np.asarray(x, dtype=np.float64).copy()
    return np.clip((x - lo) * (255.0 / (hi - lo)), 0.0, 255.0)


def rne_u8(x: np.ndarray) -> np.ndarray:
    """Round half to even and saturate to uint8."""
    return np.clip(np.rint(x), 0, 255).astype(np.uint8)


# Rounding margin for the percentile decisions: a single-precision J_gamma
# may lie this far from the float64 value before rounding to a code (the
# tolerances of t and J bound the difference well below it).
WB_BAND = 2e-3


# ------------------------------------------------------------- Sec. V
@dataclass
class Result:
    out: np.ndarray
    aux: dict = field(default_factory=dict)


def dehaze(I: np.ndarray, p: Params, A_inject=None, A_prev=None) -> Result:
    """One frame through the per-frame algorithm of Sec. V (steps 1-7).

    I: (H, W, 3) uint8 RGB, or float64 on the 0..255 scale (for the
    exact-recovery checks; then A may be injected instead of estimated).
    With resize_width/resize_height set, step 1 resizes I first and every
    later step (and the output) is at that size.  A_prev: the previous
    frame's stored airlight (float32) of the same stream, blended in when
    p.airlight_smoothing > 0 (None = first frame).  aux["A_state"] is this
    frame's airlight as it would be stored for the next one.
    """
    aux = {}
    if p.resize_width or p.resize_height:
        I = resize(I, p.resize_width, p.resize_height)
        aux["I"] = I
    m = channel_min(I)
    D = erode(m, p.patch)
    aux.update(m=m, D=D)
    if A_inject is None:
        air = airlight(I, D, p.top_frac, p.alpha)
        A = air.A
        aux.update(K=air.K, vstar=air.vstar, cutoff=air.cutoff, sel=air.sel, S=air.S, A_hat=air.A)
        if p.airlight_smoothing > 0 and A_prev is not None:
            A = airlight_smooth(A_prev, A, p.airlight_smoothing)
    else:
        A = np.asarray(A_inject, dtype=np.float64)
    aux["A"] = A
    aux["A_state"] = np.asarray(A, dtype=np.float64).astype(np.float32)
    if p.tx == "he":
        t = transmission_he(I, A, p.omega, p.t0, p.patch)
    elif p.tx == "paper":
        t = transmission_paper(I, A, p.omega, p.t0)
    else:
        raise ValueError(p.tx)
    aux["t_coarse"] = t
    if p.mode == "offline":
        G = luma(I)
        gf = guided_filter(t, G, p.gf_radius, p.f("gf_eps"))
        t = np.clip(gf.q, p.f("t0"), 1.0)
        aux["gf_a"] = gf.a
        aux["gf_b"] = gf.b
    elif p.mode != "realtime":
        raise ValueError(p.mode)
    aux["t"] = t
    J = reconstruct(I, A, t)
    aux["J"] = J
    if p.gamma_adaptive:
        g = adaptive_gamma(J, p.gamma_target)
        aux["gamma"] = g
        Jg = gamma_power(J, g)
    else:
        Jg = gamma_correct(J, p.gamma)
    aux["Jg"] = Jg
    if p.color_balance == 2:
        Jf, points, cands = percentile_stretch(Jg, p.wb_percentile, band=WB_BAND)
        gains = np.ones(3)
        aux["wb_points"] = points
        aux["wb_candidates"] = cands
    elif p.color_balance:
        Jf, gains = gray_world(Jg)
    else:
        Jf, gains = Jg, np.ones(3)
    aux["gains"] = gains
    aux["Jf"] = Jf
    return Result(out=rne_u8(Jf), aux=aux)


def dehaze_sequence(frames, p: Params):
    """Frames of one stream in order, carrying the stored airlight between them."""
    out, A_prev = [], None
    for I in frames:
        r = dehaze(I, p, A_prev=A_prev)
        A_prev = r.aux["A_state"]
        out.append(r)
    return out
