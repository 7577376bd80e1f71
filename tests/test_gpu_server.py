"""The continuous-batching server on the GPU: every served frame equals the
same frame run alone through hzd_dehaze_frame, admission follows the arena
budget, and closing/destroying drains or cancels correctly."""
import numpy as np
import pytest
import torch

import oracle
import paper_2512_16609_amd as hzd
from synth import make_frame

from parity import oracle_params, run_gpu, to_dev

pytestmark = pytest.mark.gpu

RT = hzd.Params()
OFF = hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=60, color_balance=1)


def _need(p, w, h):
    return 2 * (hzd.workspace_size(p, [(h, w)]) + 256) + 512


def test_served_equals_alone_in_a_mix():
    specs = [(320, 240, RT), (640, 480, OFF), (160, 120, RT), (640, 480, RT), (320, 240, OFF),
             (1280, 720, RT)]
    arena = sum(_need(p, w, h) for w, h, p in specs) + (1 << 20)
    srv = hzd.Server(arena_bytes=arena, max_inflight=8, frames_per_launch=4, hip_streams=3)
    streams = [srv.open(p, w, h) for w, h, p in specs]
    frames = {i: [make_frame(w, h, 100 + 10 * i + k).I for k in range(4)] for i, (w, h, _) in enumerate(specs)}
    srcs = {i: [to_dev(I) for I in frames[i]] for i in frames}
    dsts = {i: [torch.zeros_like(s) for s in srcs[i]] for i in frames}
    tickets = []
    for k in range(4):                       # interleave the streams so launches mix them
        for i, st in enumerate(streams):
            tickets.append((i, k, st.submit(srcs[i][k], dsts[i][k])))
    for i, k, t in tickets:
        rc, lat = streams[i].wait(t)
        assert rc == 0 and lat > 0
    stats = srv.stats()
    assert stats["completed"] == len(tickets) and stats["failed"] == 0
    for i, (w, h, p) in enumerate(specs):
        for k in range(4):
            alone = run_gpu(frames[i][k], p, with_J=False)["out"]
            assert np.array_equal(dsts[i][k].cpu().numpy(), alone), (i, k)
    # per-stream device state: A and the airlight selection of the last frame
    A, sel = streams[0].state()
    ref = oracle.dehaze(frames[0][3], oracle_params(RT))
    assert sel[0] == ref.aux["K"] and sel[1] == int(ref.aux["vstar"])
    assert sel[2] == ref.aux["cutoff"] and sel[3] == 0
    assert np.allclose(A, ref.aux["A"].astype(np.float32))
    for st in streams:
        st.close()
    srv.close()


def test_admission_by_arena_budget():
    need = _need(OFF, 640, 480)
    srv = hzd.Server(arena_bytes=2 * need, max_inflight=4, frames_per_launch=2, hip_streams=2)
    a = srv.open(OFF, 640, 480)
    b = srv.open(OFF, 640, 480)
    with pytest.raises(hzd.HzdError) as e:
        srv.open(OFF, 640, 480)
    assert e.value.status == hzd.HZD_E_AGAIN
    a.close()
    c = srv.open(OFF, 640, 480)          # the released space is reused
    assert srv.stats()["open_streams"] == 2
    b.close()
    c.close()
    srv.close()


def test_close_waits_for_inflight_and_destroy_cancels_queued():
    I = make_frame(640, 480, 7).I
    src = to_dev(I)
    srv = hzd.Server(arena_bytes=_need(OFF, 640, 480) + (1 << 20), max_inflight=1, frames_per_launch=1,
                     hip_streams=1)
    st = srv.open(OFF, 640, 480)
    dsts = [torch.zeros_like(src) for _ in range(6)]
    ts = [st.submit(src, d) for d in dsts]
    st.close()                           # drains all six
    alone = run_gpu(I, OFF, with_J=False)["out"]
    for d in dsts:
        assert np.array_equal(d.cpu().numpy(), alone)
    st2 = srv.open(OFF, 640, 480)
    many = [st2.submit(src, dsts[k % 6]) for k in range(40)]
    srv.close()                          # cancels what is still queued
    # the stream object was freed by destroy; statuses are not observable after it, so only
    # check that destroy returned and the GPU is idle and consistent
    torch.cuda.synchronize()
    assert len(ts) == 6 and len(many) == 40


def test_submit_rejects_wrong_size():
    srv = hzd.Server(arena_bytes=_need(RT, 320, 240) + (1 << 20))
    st = srv.open(RT, 320, 240)
    bad = torch.zeros((100, 100, 3), dtype=torch.uint8, device="cuda")
    with pytest.raises(hzd.HzdError) as e:
        st.submit(bad, torch.zeros_like(bad))
    assert e.value.status == hzd.HZD_E_INVAL
    st.close()
    srv.close()


def test_random_stream_mix_equals_alone():
    # streams with random sizes and parameters, frames interleaved so launches mix them; every
    # served frame must equal the same frame run alone (results do not depend on batching)
    rng = np.random.default_rng(4242)
    specs = []
    for i in range(7):
        w, h = int(rng.integers(8, 400)), int(rng.integers(8, 300))
        p = hzd.Params(mode=int(rng.integers(0, 2)), patch=int(rng.choice([1, 7, 15, 31])),
                       gamma=float(rng.uniform(0.8, 2.5)), gf_radius=int(rng.integers(1, 65)),
                       color_balance=int(rng.integers(0, 2)), tx=int(rng.integers(0, 2)),
                       precision=int(rng.integers(0, 2)))
        specs.append((w, h, p))
    arena = sum(_need(p, w, h) for w, h, p in specs) + (1 << 20)
    srv = hzd.Server(arena_bytes=arena, max_inflight=8, frames_per_launch=4, hip_streams=3)
    streams = [srv.open(p, w, h) for w, h, p in specs]
    frames = {i: [make_frame(w, h, 800 + 10 * i + k).I if min(w, h) >= 16 else
                  rng.integers(0, 256, size=(h, w, 3), dtype=np.uint8) for k in range(3)]
              for i, (w, h, _) in enumerate(specs)}
    srcs = {i: [to_dev(I) for I in frames[i]] for i in frames}
    dsts = {i: [torch.zeros_like(s) for s in srcs[i]] for i in frames}
    tickets = [(i, k, streams[i].submit(srcs[i][k], dsts[i][k])) for k in range(3) for i in range(len(specs))]
    for i, k, t in tickets:
        rc, _ = streams[i].wait(t)
        assert rc == 0
    for i, (w, h, p) in enumerate(specs):
        for k in range(3):
            assert np.array_equal(dsts[i][k].cpu().numpy(), run_gpu(frames[i][k], p, with_J=False)["out"]), (i, k)
    for st in streams:
        st.close()
    srv.close()


def test_random_stream_mix_with_optional_stages_equals_frame_calls():
    # streams that resize, smooth the airlight over time or adapt gamma, mixed with plain ones;
    # a smoothed stream is compared with the same frames run in order through frame calls that
    # carry a state, every other stream with each frame run alone
    rng = np.random.default_rng(4343)
    specs = []
    for i in range(8):
        w, h = int(rng.integers(16, 400)), int(rng.integers(16, 300))
        resize = bool(rng.random() < 0.5)
        p = hzd.Params(mode=int(rng.integers(0, 2)), patch=int(rng.choice([1, 7, 15])),
                       gf_radius=int(rng.integers(1, 65)), color_balance=int(rng.integers(0, 2)),
                       precision=int(rng.integers(0, 2)),
                       resize_width=int(rng.integers(8, 300)) if resize else 0,
                       resize_height=int(rng.integers(8, 200)) if resize else 0,
                       airlight_smoothing=float(rng.choice([0.0, 0.8])),
                       gamma_adaptive=int(rng.integers(0, 2)), gamma_target=float(rng.uniform(0.4, 0.8)))
        specs.append((w, h, p))
    arena = sum(hzd.stream_arena_size(p, w, h) for w, h, p in specs) + (1 << 20)
    srv = hzd.Server(arena_bytes=arena, max_inflight=8, frames_per_launch=4, hip_streams=3)
    streams = [srv.open(p, w, h) for w, h, p in specs]
    nf = 4
    frames = {i: [make_frame(w, h, 900 + 10 * i + k).I for k in range(nf)] for i, (w, h, _) in enumerate(specs)}
    srcs = {i: [to_dev(I) for I in frames[i]] for i in frames}
    dsts = {}
    for i, (w, h, p) in enumerate(specs):
        ho, wo = p.output_shape(h, w)
        dsts[i] = [torch.zeros((ho, wo, 3), dtype=torch.uint8, device="cuda") for _ in range(nf)]
    tickets = [(i, k, streams[i].submit(srcs[i][k], dsts[i][k])) for k in range(nf) for i in range(len(specs))]
    for i, k, t in tickets:
        rc, _ = streams[i].wait(t)
        assert rc == 0
    for i, (w, h, p) in enumerate(specs):
        state = hzd.make_airlight_state() if p.airlight_smoothing > 0 else None
        for k in range(nf):
            ref = run_gpu(frames[i][k], p, with_J=False, airlight_state=state)["out"]
            assert np.array_equal(dsts[i][k].cpu().numpy(), ref), (i, k, p)
    for st in streams:
        st.close()
    srv.close()


def test_served_with_graph_cache_equals_frame_calls():
    # the server's launches captured and replayed as HIP graphs (a smoothed stream's first frame
    # and later frames differ in their launch arguments, so they take different graphs); repeated
    # rounds with the same buffers replay the cached graphs
    specs = [(320, 240, hzd.Params(airlight_smoothing=0.6)), (640, 480, OFF), (320, 240, RT)]
    arena = sum(hzd.stream_arena_size(p, w, h) for w, h, p in specs) + (1 << 20)
    frames = {i: [make_frame(w, h, 950 + 10 * i + k).I for k in range(3)] for i, (w, h, _) in enumerate(specs)}
    refs = {}   # per stream, both rounds: a smoothed stream's second round continues its average
    for i, (w, h, p) in enumerate(specs):
        state = hzd.make_airlight_state() if p.airlight_smoothing > 0 else None
        refs[i] = [run_gpu(frames[i][k % 3], p, with_J=False, airlight_state=state)["out"] for k in range(6)]
    try:
        hzd.graph_cache(64)
        srv = hzd.Server(arena_bytes=arena, max_inflight=4, frames_per_launch=2, hip_streams=2)
        streams = [srv.open(p, w, h) for w, h, p in specs]
        srcs = {i: [to_dev(I) for I in frames[i]] for i in frames}
        dsts = {i: [torch.zeros_like(s) for s in srcs[i]] for i in frames}
        for rnd in range(2):
            tickets = [(i, k, streams[i].submit(srcs[i][k], dsts[i][k])) for k in range(3) for i in range(len(specs))]
            for i, k, t in tickets:
                rc, _ = streams[i].wait(t)
                assert rc == 0
            for i in range(len(specs)):
                for k in range(3):
                    assert np.array_equal(dsts[i][k].cpu().numpy(), refs[i][3 * rnd + k]), (rnd, i, k)
        for st in streams:
            st.close()
        srv.close()
    finally:
        hzd.graph_cache(0)


def test_wait_twice_on_a_ticket_is_an_error():
    srv = hzd.Server(arena_bytes=_need(RT, 160, 120) + (1 << 20))
    st = srv.open(RT, 160, 120)
    src = to_dev(make_frame(160, 120, 3).I)
    dst = torch.zeros_like(src)
    t = st.submit(src, dst)
    rc, _ = st.wait(t)
    assert rc == 0
    assert st.wait(t)[0] == hzd.HZD_E_INVAL        # already collected: an error, not a wait forever
    assert st.wait(t + 100)[0] == hzd.HZD_E_INVAL  # never issued
    st.close()
    srv.close()


def test_submit_waits_for_the_producer_stream():
    """A frame written on another stream just before submit is read only after that stream's
    work: the submit records an event on the producer's stream and the launch waits for it."""
    w, h = 640, 480
    I = make_frame(w, h, 77).I
    alone = run_gpu(I, RT, with_J=False)["out"]
    srv = hzd.Server(arena_bytes=_need(RT, w, h) + (1 << 20), max_inflight=2, frames_per_launch=1, hip_streams=1)
    st = srv.open(RT, w, h)
    src = torch.zeros((h, w, 3), dtype=torch.uint8, device="cuda")
    dst = torch.full((h, w, 3), 7, dtype=torch.uint8, device="cuda")
    host = torch.from_numpy(I).pin_memory()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        a = torch.randn(4096, 4096, device="cuda")
        for _ in range(6):            # keeps the producer stream busy for milliseconds
            a = (a @ a) / 64.0
        src.copy_(host, non_blocking=True)
        dst.zero_()
    t = st.submit(src, dst, stream=side)
    rc, _ = st.wait(t)
    assert rc == 0
    torch.cuda.synchronize()
    assert np.array_equal(dst.cpu().numpy(), alone)
    st.close()
    srv.close()
