"""GPU parity of the temporal airlight average over a stream's frames.

The blended airlight is formed in double in a fixed operation order on both
sides, so A is compared exactly (as float32) frame by frame along a sequence;
t, J and the output then follow the usual tolerances.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2512_16609_amd as hzd
from synth import make_video
from parity import compare, oracle_params, run_gpu, to_dev

pytestmark = pytest.mark.gpu


def _clip(w, h, n, seed=3):
    v = make_video(w, h, nframes=n, seed=seed, pan=64, y_off=16)
    return [v.frame(f).I for f in range(n)]


def _sequence_gpu(frames, p, state=None):
    state = hzd.make_airlight_state() if state is None else state
    outs = [run_gpu(I, p, airlight_state=state) for I in frames]
    return outs, state


@pytest.mark.parametrize("mode,lam", [(hzd.MODE_REALTIME, 0.8), (hzd.MODE_REALTIME, 0.3),
                                      (hzd.MODE_OFFLINE, 0.5)])
def test_sequence_matches_oracle(mode, lam):
    frames = _clip(160, 120, 6)
    p = hzd.Params(mode=mode, gf_radius=20, color_balance=int(mode == hzd.MODE_OFFLINE), airlight_smoothing=lam)
    gpu, state = _sequence_gpu(frames, p)
    ref = oracle.dehaze_sequence(frames, oracle_params(p))
    for k, (I, g, r) in enumerate(zip(frames, gpu, ref)):
        assert np.array_equal(g["A"], r.aux["A"].astype(np.float32)), k
        compare(I, p, g, ref=r, label=f"frame {k}")
    st = state.cpu().numpy()
    assert np.array_equal(st[:3], ref[-1].aux["A_state"])
    assert st[3:].view(np.uint32)[0] == len(frames)
    # the average moved A away from the frames' own estimates
    assert any(not np.array_equal(r.aux["A"], r.aux["A_hat"]) for r in ref[1:])


def test_zero_weight_with_a_state_equals_frames_alone():
    frames = _clip(160, 120, 3)
    p = hzd.Params()
    gpu, state = _sequence_gpu(frames, p)
    for I, g in zip(frames, gpu):
        alone = run_gpu(I, p)
        for k in alone:
            assert np.array_equal(g[k], alone[k]), k
    assert state.cpu().numpy()[3:].view(np.uint32)[0] == 1   # no blending: the count restarts


def test_batch_of_streams_equals_per_stream_sequences():
    # three streams advance together, one frame of each per batch call
    clips = [_clip(160, 120, 3, seed=s) for s in (31, 32, 33)]
    params = [hzd.Params(airlight_smoothing=0.9), hzd.Params(airlight_smoothing=0.5, patch=7),
              hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=10, airlight_smoothing=0.7)]
    states = [hzd.make_airlight_state() for _ in clips]
    got = [[] for _ in clips]
    for f in range(3):
        srcs = [to_dev(c[f]) for c in clips]
        dsts = [torch.zeros_like(s) for s in srcs]
        auxs = [hzd.make_aux(120, 160) for _ in clips]
        hzd.dehaze_batch(srcs, dsts, hzd.Params(), per_frame_params=params, auxs=auxs, airlight_states=states)
        torch.cuda.synchronize()
        for i in range(3):
            got[i].append((dsts[i].cpu().numpy(), auxs[i]["A"].cpu().numpy()))
    for i, c in enumerate(clips):
        seq, _ = _sequence_gpu(c, params[i])
        for f in range(3):
            assert np.array_equal(got[i][f][0], seq[f]["out"]), (i, f)
            assert np.array_equal(got[i][f][1], seq[f]["A"]), (i, f)


def test_served_stream_with_smoothing_equals_frame_calls():
    frames = _clip(320, 240, 6, seed=40)
    p = hzd.Params(airlight_smoothing=0.75)
    q = hzd.Params()
    srv = hzd.Server(arena_bytes=hzd.stream_arena_size(p, 320, 240) + hzd.stream_arena_size(q, 320, 240) + 4096,
                     max_inflight=8, frames_per_launch=4, hip_streams=2)
    try:
        st = srv.open(p, 320, 240)
        other = srv.open(q, 320, 240)       # an unsmoothed stream sharing the launches
        srcs = [to_dev(I) for I in frames]
        dsts = [torch.zeros_like(s) for s in srcs]
        odsts = [torch.zeros_like(s) for s in srcs]
        tickets = []
        for s, d, od in zip(srcs, dsts, odsts):
            tickets.append((st, st.submit(s, d)))
            tickets.append((other, other.submit(s, od)))
        for x, t in tickets:
            assert x.wait(t)[0] == hzd.HZD_OK
        seq, _ = _sequence_gpu(frames, p)
        for k in range(len(frames)):
            assert np.array_equal(dsts[k].cpu().numpy(), seq[k]["out"]), k
            assert np.array_equal(odsts[k].cpu().numpy(), run_gpu(frames[k], q)["out"]), k
        A, _ = st.state()
        assert np.array_equal(np.array(A, dtype=np.float32), seq[-1]["A"])
        st.close()
        other.close()
    finally:
        srv.close()


def test_autotune_leaves_the_airlight_state_alone():
    frames = _clip(320, 240, 2, seed=50)
    p = hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=30, airlight_smoothing=0.8)
    _, state = _sequence_gpu(frames, p)
    before = state.clone()
    src = to_dev(frames[0])
    try:
        rows = hzd.autotune(src, torch.zeros_like(src), p, reps=2, airlight_state=state)
        assert rows in (8, 16, 24, 32, 48, 64, 96, 128)
        torch.cuda.synchronize()
        assert torch.equal(state, before)
    finally:
        hzd.tile_config_set(320, 240, None)
