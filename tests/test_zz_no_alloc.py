"""hzd_dehaze_frame_noalloc (the entry point for callers that cannot allocate
device memory) against hzd_dehaze_frame: two calls in a row on the shared
static scratch, the second with a smaller frame, each bit-identical to the
workspace entry point's result (output, A, selection, dark channel, t).
The workspace results are in turn held to the FP64 oracle by the parity tests;
here the first frame is also checked against the oracle directly."""
import numpy as np
import pytest
import torch

import paper_2512_16609_amd as hzd
from synth import make_frame

from parity import compare, to_dev

pytestmark = pytest.mark.gpu


def _run(entry, I, p):
    h, w, _ = I.shape
    src = to_dev(I)
    ho, wo = p.output_shape(h, w)
    dst = torch.zeros((ho, wo, 3), dtype=torch.uint8, device="cuda")
    aux = hzd.make_aux(ho, wo, J=True)
    torch.cuda.synchronize()
    if entry == "noalloc":
        hzd.dehaze_frame_noalloc(src, dst, p, aux=aux)
    else:
        hzd.dehaze_frame(src, dst, p, aux=aux)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in aux.items()}
    out["out"] = dst.cpu().numpy()
    return out


def _same(a, b, label):
    for k in ("out", "A", "sel", "dark", "t", "J"):
        assert np.array_equal(a[k], b[k]), f"{label}: {k} differs"
    assert int(a["sel"][3]) == 0, f"{label}: selection status {a['sel'][3]}"


def test_noalloc_equals_workspace_entry_two_calls():
    cases = [
        # the largest workspace first: 1080p offline with the guided filter and colour balance
        (make_frame(1920, 1080, 2, beta=1.3).I, hzd.Params(mode=hzd.MODE_OFFLINE, color_balance=1)),
        # then a smaller frame on the same scratch, which still holds the first call's data
        (make_frame(640, 480, 11, beta=0.9).I, hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=20)),
        # and a small real-time frame with a ragged size
        (make_frame(336, 200, 12).I[:197, :331].copy(), hzd.Params()),
    ]
    for i, (I, p) in enumerate(cases):
        print(f"noalloc case {i}: {I.shape[1]}x{I.shape[0]} mode {p.mode}", flush=True)
        got = _run("noalloc", I, p)
        ref = _run("workspace", I, p)
        _same(got, ref, f"case {i}")
        if i == 0:
            compare(I, p, got, label="noalloc 1080p offline")


def test_noalloc_under_graph_capture_replays():
    # callers that cannot allocate include code under graph capture: the captured call zeroes the
    # frame state with the init kernel on every replay (direct calls do it in leading blocks of
    # k_dark); each replay equals the workspace entry point's direct result
    p = hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=20, color_balance=1)
    I1, I2 = make_frame(640, 480, 31).I, make_frame(640, 480, 32, beta=1.4).I
    ref1, ref2 = _run("workspace", I1, p)["out"], _run("workspace", I2, p)["out"]
    src = to_dev(I1)
    dst = torch.zeros((480, 640, 3), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=stream):
        hzd.dehaze_frame_noalloc(src, dst, p, stream=stream)
    for rep in range(4):
        src.copy_(to_dev(I1 if rep % 2 == 0 else I2))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(dst.cpu().numpy(), ref1 if rep % 2 == 0 else ref2), rep


def test_noalloc_rejects_oversized_frame():
    I = torch.zeros((2160, 3840, 3), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(I)
    with pytest.raises(hzd.HzdError) as e:
        hzd.dehaze_frame_noalloc(I, dst, hzd.Params(mode=hzd.MODE_OFFLINE))
    assert e.value.status == hzd.HZD_E_NOMEM
