"""GPU parity of the resize front end (Sec. V step 1) against the oracle.

The resampling is exact integer arithmetic on both sides, so the resized
frame is compared bit for bit: with omega = 0, gamma = 1 and no colour
balance the pipeline is the identity on its input, and the output is then the
resized frame itself.  Full-pipeline cases then follow the usual tolerances at
the working size.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2512_16609_amd as hzd
from synth import make_frame
from parity import compare, run_gpu, to_dev

pytestmark = pytest.mark.gpu


def P(**kw):
    return hzd.Params(**kw)


def _frame(w, h, seed, beta=1.0):
    return make_frame(w, h, seed, beta=beta).I


# (input w, h) -> (output w, h): the paper's default working size from common
# inputs, ratios below and above 1, odd sizes, single rows/columns, 1x1, and
# outputs wider than one block row (256 columns) with ragged tails
SIZE_PAIRS = [((1920, 1080), (640, 480)), ((3840, 2160), (640, 480)), ((1280, 720), (640, 480)),
              ((640, 480), (640, 480)), ((320, 240), (640, 480)), ((97, 61), (1000, 3)),
              ((333, 197), (257, 129)), ((1, 1), (5, 3)), ((9, 5), (1, 1)), ((1, 40), (3, 7)),
              ((40, 1), (7, 3)), ((1027, 769), (513, 385)), ((16, 12), (8, 6)), ((701, 3), (255, 2))]


@pytest.mark.parametrize("src,dst", SIZE_PAIRS)
@pytest.mark.parametrize("pad", [0, 1])
def test_resized_frame_is_bit_exact(src, dst, pad):
    # pad = 1 gives an odd row pitch, so rows start at every alignment mod 4
    I = _frame(src[0], src[1], 100 + src[0] + dst[0])
    p = P(omega=0.0, gamma=1.0, resize_width=dst[0], resize_height=dst[1])
    g = run_gpu(I, p, pitch_pad=pad)
    ref = oracle.resize(I, dst[0], dst[1])
    assert g["out"].shape == ref.shape
    assert np.array_equal(g["out"], ref)


@pytest.mark.parametrize("src,dst", [((1920, 1080), (640, 480)), ((333, 197), (257, 129)), ((97, 61), (128, 40))])
@pytest.mark.parametrize("mode", [hzd.MODE_REALTIME, hzd.MODE_OFFLINE])
def test_resized_pipeline_matches_oracle(src, dst, mode):
    I = _frame(src[0], src[1], 200 + src[0])
    p = P(mode=mode, gf_radius=60, color_balance=int(mode == hzd.MODE_OFFLINE),
          resize_width=dst[0], resize_height=dst[1])
    g = run_gpu(I, p)
    s = compare(I, p, g, label=f"resize {src}->{dst}")
    print(src, dst, s)


def test_paper_preset_at_the_default_working_size():
    # the shipped real-time values with the paper's default 640x480 working size
    I = _frame(1280, 720, 300)
    p = hzd.Params.preset(hzd.PRESET_PAPER_REALTIME)
    p.resize_width, p.resize_height = 640, 480
    compare(I, p, run_gpu(I, p), label="paper preset 640x480")


def test_batch_mixes_resized_and_native_frames():
    shapes = [(1080, 1920), (240, 320), (720, 1280), (97, 130)]
    params = [P(resize_width=640, resize_height=480), P(),
              P(mode=hzd.MODE_OFFLINE, gf_radius=30, color_balance=1, resize_width=320, resize_height=200),
              P(resize_width=64, resize_height=48)]
    frames = [_frame(w, h, 400 + i) for i, (h, w) in enumerate(shapes)]
    srcs = [to_dev(I) for I in frames]
    outs = [p.output_shape(h, w) for p, (h, w) in zip(params, shapes)]
    dsts = [torch.zeros((ho, wo, 3), dtype=torch.uint8, device="cuda") for ho, wo in outs]
    auxs = [hzd.make_aux(ho, wo) for ho, wo in outs]
    hzd.dehaze_batch(srcs, dsts, P(), per_frame_params=params, auxs=auxs)
    torch.cuda.synchronize()
    for i, I in enumerate(frames):
        alone = run_gpu(I, params[i])
        assert np.array_equal(dsts[i].cpu().numpy(), alone["out"]), i
        for k in ("A", "sel", "dark", "t", "J"):
            assert np.array_equal(auxs[i][k].cpu().numpy(), alone[k]), (i, k)


def test_served_stream_with_resize_equals_frame_call():
    I = [_frame(1280, 720, 500 + k) for k in range(3)]
    p = P(resize_width=640, resize_height=480)
    ws = hzd.workspace_size(p, [(720, 1280)])
    srv = hzd.Server(arena_bytes=2 * (ws + 256) + 4096 + (1 << 20))
    try:
        st = srv.open(p, 1280, 720)
        srcs = [to_dev(x) for x in I]
        dsts = [torch.zeros((480, 640, 3), dtype=torch.uint8, device="cuda") for _ in I]
        tickets = [st.submit(s, d) for s, d in zip(srcs, dsts)]
        for t in tickets:
            assert st.wait(t)[0] == hzd.HZD_OK
        for x, d in zip(I, dsts):
            assert np.array_equal(d.cpu().numpy(), run_gpu(x, p)["out"])
        st.close()
    finally:
        srv.close()


def test_graph_replay_with_resize():
    I1, I2 = _frame(1920, 1080, 601), _frame(1920, 1080, 602)
    p = P(resize_width=640, resize_height=480)
    ref1, ref2 = run_gpu(I1, p, with_J=False)["out"], run_gpu(I2, p, with_J=False)["out"]
    src, dst = to_dev(I1), torch.zeros((480, 640, 3), dtype=torch.uint8, device="cuda")
    ws = hzd.alloc_workspace(hzd.workspace_size(p, [(1080, 1920)]))
    stream = torch.cuda.Stream()
    try:
        hzd.graph_cache(8)
        with torch.cuda.stream(stream):
            for rep in range(4):
                src.copy_(to_dev(I1 if rep % 2 == 0 else I2))
                hzd.dehaze_frame(src, dst, p, workspace=ws, stream=stream)
                stream.synchronize()
                assert np.array_equal(dst.cpu().numpy(), ref1 if rep % 2 == 0 else ref2), rep
    finally:
        hzd.graph_cache(0)
