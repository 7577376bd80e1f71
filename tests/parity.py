"""Shared helpers for the GPU parity tests: run one frame through the C ABI
with every optional output, run the FP64 oracle on the same bytes, and
compare to the stated tolerances.

Tolerances (single-precision path against the FP64 oracle):
  D, E-derived values, K, vstar, cutoff   bit-exact
  A                                       equal to float32(oracle A)
  t                                       |dt| <= RTOL * t_ref          (RTOL 1e-5; 1e-3 with FP16 t)
  J (Eq. (7), clamped, before gamma)      |dJ| <= RTOL * (|I - A| / t_ref + |A|) + 1e-4
                                          (relative to the magnitude of the terms J is formed from;
                                           J itself may sit at 0 after the clamp)
  output                                  |d out| <= 1 LSB
"""
from __future__ import annotations

import numpy as np
import torch

import oracle
import paper_2512_16609_amd as hzd

RTOL_FP32 = 1e-5
RTOL_FP16 = 1e-3


def oracle_params(p: hzd.Params) -> oracle.Params:
    return oracle.Params(mode="offline" if p.mode == hzd.MODE_OFFLINE else "realtime", patch=p.patch,
                         omega=p.omega, t0=p.t0, top_frac=p.top_frac, alpha=p.alpha, gamma=p.gamma,
                         gf_radius=p.gf_radius, gf_eps=p.gf_eps, color_balance=bool(p.color_balance),
                         tx="he" if p.tx == hzd.TX_HE else "paper")


def to_dev(I: np.ndarray, pitch_pad: int = 0) -> torch.Tensor:
    """Upload an (H, W, 3) uint8 frame; pitch_pad > 0 gives a row pitch > 3W."""
    h, w, _ = I.shape
    if pitch_pad:
        big = torch.zeros((h, 3 * w + pitch_pad), dtype=torch.uint8, device="cuda")
        big[:, :3 * w] = torch.from_numpy(I.reshape(h, 3 * w)).cuda()
        return torch.as_strided(big, (h, w, 3), (3 * w + pitch_pad, 3, 1))
    return torch.from_numpy(np.ascontiguousarray(I)).cuda()


def run_gpu(I: np.ndarray, p: hzd.Params, pitch_pad: int = 0, with_J: bool = True):
    h, w, _ = I.shape
    src = to_dev(I, pitch_pad)
    if pitch_pad:
        dbig = torch.zeros((h, 3 * w + pitch_pad), dtype=torch.uint8, device="cuda")
        dst = torch.as_strided(dbig, (h, w, 3), (3 * w + pitch_pad, 3, 1))
    else:
        dst = torch.zeros_like(src)
    aux = hzd.make_aux(h, w, J=with_J)
    hzd.dehaze_frame(src, dst, p, aux=aux)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in aux.items()}
    out["out"] = dst.cpu().numpy() if not pitch_pad else dst.contiguous().cpu().numpy()
    return out


def compare(I: np.ndarray, p: hzd.Params, g: dict, ref=None, label: str = "") -> dict:
    """Assert parity of GPU outputs g against the oracle; return error statistics."""
    if ref is None:
        ref = oracle.dehaze(I, oracle_params(p))
    a = ref.aux
    # dark channel and the airlight set: bit-exact
    assert np.array_equal(g["dark"], a["D"]), f"{label}: dark channel differs"
    assert int(g["sel"][0]) == a["K"], f"{label}: K {g['sel'][0]} != {a['K']}"
    assert int(g["sel"][1]) == int(a["vstar"]), f"{label}: vstar {g['sel'][1]} != {a['vstar']}"
    assert int(g["sel"][2]) == a["cutoff"], f"{label}: cutoff {g['sel'][2]} != {a['cutoff']}"
    A32 = a["A"].astype(np.float32)
    assert np.array_equal(g["A"], A32), f"{label}: A {g['A']} != {A32}"
    rtol = RTOL_FP16 if p.precision == hzd.PREC_FP16 else RTOL_FP32
    t_ref = a["t"]
    t_err = np.abs(g["t"].astype(np.float64) - t_ref) / t_ref
    assert t_err.max() <= rtol, f"{label}: t rel err {t_err.max():.3g} > {rtol}"
    stats = {"t_rel_max": float(t_err.max())}
    if "J" in g:
        Iref = I.astype(np.float64)
        A = a["A"]
        scale = np.abs(Iref - A[None, None, :]) / t_ref[..., None] + np.abs(A)[None, None, :]
        J_err = np.abs(g["J"].astype(np.float64) - a["J"])
        bound = rtol * scale + 1e-4
        worst = (J_err / bound).max()
        assert worst <= 1.0, f"{label}: J error {J_err.max():.3g} exceeds bound (ratio {worst:.3g})"
        stats["J_abs_max"] = float(J_err.max())
        stats["J_rel_scaled_max"] = float((J_err / scale).max())
    d = np.abs(g["out"].astype(np.int32) - ref.out.astype(np.int32))
    assert d.max() <= 1, f"{label}: output differs by {d.max()} LSB"
    stats["lsb_max"] = int(d.max())
    stats["lsb_frac1"] = float((d == 1).mean())
    return stats
