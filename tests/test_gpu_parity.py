"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded bytes (element by element), at the configuration sizes and at
ragged edge shapes."""
import numpy as np
import pytest
import torch

import oracle
import paper_2512_16609_amd as hzd
from synth import make_frame

from parity import compare, oracle_params, run_gpu, to_dev

pytestmark = pytest.mark.gpu


def P(**kw):
    return hzd.Params(**kw)


def _frame(w, h, seed, beta=1.0):
    return make_frame(w, h, seed, beta=beta).I


def test_c1_realtime_320x240():
    I = _frame(320, 240, 1)
    g = run_gpu(I, P())
    s = compare(I, P(), g, label="C1")
    print("C1", s)


@pytest.mark.parametrize("shape", [(1, 1), (1, 37), (29, 1), (5, 7), (23, 37), (33, 65), (97, 130), (197, 333)])
@pytest.mark.parametrize("patch", [1, 3, 15, 31])
def test_ragged_shapes_realtime(shape, patch):
    h, w = shape
    rng = np.random.default_rng(h * 1000 + w + patch)
    if h * w >= 64 * 64:
        I = _frame(w, h, 7)
    else:
        I = rng.integers(0, 256, size=(h, w, 3), dtype=np.uint8)
    p = P(patch=patch, top_frac=0.01)
    compare(I, p, run_gpu(I, p), label=f"{shape} p{patch}")


@pytest.mark.parametrize("shape", [(1, 1), (1, 37), (29, 1), (5, 7), (9, 130), (130, 9), (97, 130), (33, 300)])
@pytest.mark.parametrize("radius", [1, 32, 33, 64])
def test_ragged_shapes_offline(shape, radius):
    # guided-filter strips (128 output columns for r > 32, 192 for r <= 32), 8-row chunks and
    # clipped windows at every edge, against the oracle element by element
    h, w = shape
    rng = np.random.default_rng(h * 7919 + w * 31 + radius)
    I = rng.integers(0, 256, size=(h, w, 3), dtype=np.uint8)
    p = P(mode=hzd.MODE_OFFLINE, gf_radius=radius, color_balance=1, top_frac=0.01)
    compare(I, p, run_gpu(I, p), label=f"off {shape} r{radius}")


@pytest.mark.parametrize("radius", [31, 32, 33, 34])
def test_strip_width_boundary(radius):
    # both strip widths on a frame wider than several strips, with the window clipped
    I = _frame(448, 72, 13)
    p = P(mode=hzd.MODE_OFFLINE, gf_radius=radius)
    compare(I, p, run_gpu(I, p), label=f"strip r{radius}")


def test_pitch_larger_than_row():
    I = _frame(130, 97, 9)
    for pad in (1, 5, 64):
        compare(I, P(), run_gpu(I, P(), pitch_pad=pad), label=f"pad{pad}")
        compare(I, P(mode=hzd.MODE_OFFLINE, gf_radius=12, color_balance=1),
                run_gpu(I, P(mode=hzd.MODE_OFFLINE, gf_radius=12, color_balance=1), pitch_pad=pad),
                label=f"offline pad{pad}")


@pytest.mark.parametrize("tx", [hzd.TX_HE, hzd.TX_PAPER])
@pytest.mark.parametrize("cb", [0, 1])
@pytest.mark.parametrize("prec", [hzd.PREC_FP32, hzd.PREC_FP16])
def test_realtime_variants(tx, cb, prec):
    I = _frame(320, 240, 3, beta=1.4)
    p = P(tx=tx, color_balance=cb, precision=prec)
    compare(I, p, run_gpu(I, p), label=f"rt tx{tx} cb{cb} prec{prec}")


@pytest.mark.parametrize("tx", [hzd.TX_HE, hzd.TX_PAPER])
@pytest.mark.parametrize("cb", [0, 1])
@pytest.mark.parametrize("prec", [hzd.PREC_FP32, hzd.PREC_FP16])
@pytest.mark.parametrize("radius", [1, 8, 60, 64])
def test_offline_variants(tx, cb, prec, radius):
    I = _frame(203, 151, 4, beta=0.8)
    p = P(mode=hzd.MODE_OFFLINE, gf_radius=radius, tx=tx, color_balance=cb, precision=prec)
    compare(I, p, run_gpu(I, p), label=f"off r{radius} tx{tx} cb{cb} prec{prec}")


@pytest.mark.parametrize("gamma", [1.0, 1.2, 2.2])
def test_gamma_values(gamma):
    I = _frame(160, 120, 5)
    p = P(gamma=gamma)
    compare(I, p, run_gpu(I, p), label=f"gamma {gamma}")


def test_c2_offline_1080p():
    fr = make_frame(1920, 1080, 2)
    p = P(mode=hzd.MODE_OFFLINE, gf_radius=60, gf_eps=1e-3, color_balance=1)
    s = compare(fr.I, p, run_gpu(fr.I, p), label="C2")
    print("C2", s)


def test_4k_offline_frame():
    fr = make_frame(3840, 2160, 4000)
    p = P(mode=hzd.MODE_OFFLINE, gf_radius=60, gf_eps=1e-3)
    s = compare(fr.I, p, run_gpu(fr.I, p, with_J=False), label="4K")
    print("4K", s)


@pytest.mark.parametrize("mode", [hzd.MODE_REALTIME, hzd.MODE_OFFLINE])
@pytest.mark.parametrize("tx", [hzd.TX_HE, hzd.TX_PAPER])
def test_identity_when_omega_zero(mode, tx):
    I = _frame(211, 99, 6)
    p = P(mode=mode, tx=tx, omega=0.0, gamma=1.0, gf_radius=10)
    g = run_gpu(I, p)
    assert np.array_equal(g["out"], I)
    assert np.all(g["t"] == 1.0)


def test_degenerate_frames():
    # all black (the airlight divisor guard), all white, constant colour
    for val in (0, 255, 117):
        I = np.full((48, 80, 3), val, dtype=np.uint8)
        for p in (P(), P(mode=hzd.MODE_OFFLINE, gf_radius=9, color_balance=1)):
            compare(I, p, run_gpu(I, p), label=f"const {val}")


def test_bright_blob_limitation():
    I = _frame(320, 240, 12).copy()
    I[100:140, 100:160] = 255
    g = run_gpu(I, P())
    compare(I, P(), g, label="blob")
    assert int(g["sel"][1]) == 255


def test_run_to_run_determinism():
    I = _frame(640, 480, 8)
    for p in (P(), P(mode=hzd.MODE_OFFLINE, color_balance=1)):
        a, b = run_gpu(I, p), run_gpu(I, p)
        for k in a:
            assert np.array_equal(a[k], b[k]), k


def test_batch_equals_frame():
    shapes = [(120, 160), (97, 130), (240, 320), (31, 45), (480, 640)]
    params = [P(), P(patch=7), P(mode=hzd.MODE_OFFLINE, gf_radius=20, color_balance=1),
              P(tx=hzd.TX_PAPER), P(color_balance=1, precision=hzd.PREC_FP16)]
    frames = [_frame(w, h, 20 + i) for i, (h, w) in enumerate(shapes)]
    srcs = [to_dev(I) for I in frames]
    dsts = [torch.zeros_like(s) for s in srcs]
    auxs = [hzd.make_aux(h, w) for (h, w) in shapes]
    hzd.dehaze_batch(srcs, dsts, P(), per_frame_params=params, auxs=auxs)
    torch.cuda.synchronize()
    for i, I in enumerate(frames):
        alone = run_gpu(I, params[i])
        assert np.array_equal(dsts[i].cpu().numpy(), alone["out"]), i
        for k in ("A", "sel", "dark", "t", "J"):
            assert np.array_equal(auxs[i][k].cpu().numpy(), alone[k]), (i, k)


def test_row_record_selection_batch_of_sixteen():
    # sixteen frames too large for the one-block selection, of sixteen different heights (from
    # 4 rows to a 4K frame's 2160), in one launch: the row pass runs in 256-thread blocks and
    # each frame's last block ends its selection; a frame alone runs it in 512-thread blocks.
    # Every frame's selection, A and output equal its single-frame result, and two frames are
    # also checked against the FP64 oracle
    rng = np.random.default_rng(91)
    heights = [4, 17, 64, 65, 129, 200, 255, 256, 257, 511, 700, 1023, 1080, 1300, 2049, 2160]
    widths = [int(w) for w in rng.integers(1100, 2000, size=len(heights))]
    widths[-1] = 3840
    p = P()
    frames = [make_frame(w, h, 900 + i, beta=0.7 + 0.05 * i).I for i, (w, h) in enumerate(zip(widths, heights))]
    srcs = [to_dev(I) for I in frames]
    dsts = [torch.zeros_like(s) for s in srcs]
    auxs = [hzd.make_aux(h, w, J=False) for w, h in zip(widths, heights)]
    hzd.dehaze_batch(srcs, dsts, p, auxs=auxs)
    torch.cuda.synchronize()
    for i, I in enumerate(frames):
        alone = run_gpu(I, p, with_J=False)
        assert int(auxs[i]["sel"][3].item()) == 0, i
        assert np.array_equal(auxs[i]["sel"].cpu().numpy(), alone["sel"]), i
        assert np.array_equal(auxs[i]["A"].cpu().numpy(), alone["A"]), i
        assert np.array_equal(dsts[i].cpu().numpy(), alone["out"]), i
        if i in (3, 12):
            compare(I, p, alone, label=f"batch of sixteen, frame {i}")


def test_same_shape_batch_of_eight_720p_fp16():
    # one launch of 8 real-time 720p frames (FP16 t), every frame equal to its single-frame result
    from synth import make_video
    v = make_video(1280, 720, nframes=300, seed=3)
    idx = [0, 37, 74, 111, 148, 185, 222, 259]
    frames = [v.frame(f).I for f in idx]
    p = P(precision=hzd.PREC_FP16)
    srcs = [to_dev(I) for I in frames]
    dsts = [torch.zeros_like(s) for s in srcs]
    hzd.dehaze_batch(srcs, dsts, p)
    torch.cuda.synchronize()
    for i, I in enumerate(frames[:3]):
        ref = oracle.dehaze(I, oracle_params(p))
        d = np.abs(dsts[i].cpu().numpy().astype(int) - ref.out.astype(int))
        assert d.max() <= 1
    for i, I in enumerate(frames):
        assert np.array_equal(dsts[i].cpu().numpy(), run_gpu(I, p, with_J=False)["out"])


def test_results_do_not_depend_on_tile_rows():
    # exact integer box sums and integer colour-balance sums: every tile shape gives the same bits
    I = _frame(640, 480, 31)
    p = P(mode=hzd.MODE_OFFLINE, gf_radius=60, color_balance=1)
    outs = []
    try:
        for rows in (8, 16, 24, 32, 64, 128, 256):
            hzd.tile_config_set(640, 480, rows)
            outs.append(run_gpu(I, p))
    finally:
        hzd.tile_config_set(640, 480, None)
    for o in outs[1:]:
        for k in o:
            assert np.array_equal(o[k], outs[0][k]), k
    compare(I, p, outs[0], label="tile rows")


def test_autotune_picks_a_candidate(tmp_path, monkeypatch):
    # the choice goes into the table and is appended to the HZD_AUTOTUNE_CACHE file
    I = _frame(640, 480, 32)
    p = P(mode=hzd.MODE_OFFLINE, gf_radius=60, color_balance=1)
    src = to_dev(I)
    dst = torch.zeros_like(src)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("HZD_AUTOTUNE_CACHE", str(cache))
    try:
        rows = hzd.autotune(src, dst, p, reps=3)
        assert rows in (8, 16, 24, 32, 48, 64, 96, 128)
        assert hzd.tile_config_get(640, 480) == rows
        assert cache.read_text().split() == ["640", "480", str(rows)]
        compare(I, p, run_gpu(I, p), label="autotuned")
    finally:
        hzd.tile_config_set(640, 480, None)


def test_graph_replay_matches_direct_launch():
    I1, I2 = _frame(640, 480, 41), _frame(640, 480, 42)
    p = P(mode=hzd.MODE_OFFLINE, gf_radius=60, color_balance=1)
    ref1, ref2 = run_gpu(I1, p, with_J=False)["out"], run_gpu(I2, p, with_J=False)["out"]
    src, dst = to_dev(I1), torch.zeros((480, 640, 3), dtype=torch.uint8, device="cuda")
    ws = hzd.alloc_workspace(hzd.workspace_size(p, [(480, 640)]))
    stream = torch.cuda.Stream()
    try:
        hzd.graph_cache(8)
        with torch.cuda.stream(stream):
            for rep in range(4):      # capture once, then replays; new content in the same buffers
                src.copy_(to_dev(I1 if rep % 2 == 0 else I2))
                hzd.dehaze_frame(src, dst, p, workspace=ws, stream=stream)
                stream.synchronize()
                assert np.array_equal(dst.cpu().numpy(), ref1 if rep % 2 == 0 else ref2), rep
    finally:
        hzd.graph_cache(0)


@pytest.mark.parametrize("variant", ["offline_percentile_adaptive", "realtime_grayworld"])
def test_state_zeroing_does_not_depend_on_workspace_contents(variant):
    # Direct launches zero each frame's state in leading blocks of k_dark instead of with the
    # init kernel.  Run a batch on a workspace full of random
    # bytes, then again with the frames in another order (each frame's state now lies on what
    # another frame's maps held), and compare with the graph-replayed form, which zeroes the
    # state with the init kernel.  The selection's status checks that every histogram holds W H.
    if variant == "offline_percentile_adaptive":
        p = P(mode=hzd.MODE_OFFLINE, gf_radius=30, color_balance=2, gamma_adaptive=1, gamma_target=0.6)
    else:
        p = P(color_balance=1)
    shapes = [(480, 640), (720, 1280), (1080, 1920), (481, 655)]
    frames = [make_frame(w, h, 700 + i, beta=0.8 + 0.2 * i).I for i, (h, w) in enumerate(shapes)]
    srcs = [to_dev(I) for I in frames]
    stream = torch.cuda.Stream()

    def run(order, ws, graphs):
        dsts = [torch.zeros_like(srcs[i]) for i in order]
        auxs = [hzd.make_aux(shapes[i][0], shapes[i][1], J=False) for i in order]
        torch.cuda.synchronize()
        hzd.graph_cache(8 if graphs else 0)
        try:
            with torch.cuda.stream(stream):
                hzd.dehaze_batch([srcs[i] for i in order], dsts, p, auxs=auxs, workspace=ws, stream=stream)
            stream.synchronize()
        finally:
            hzd.graph_cache(0)
        out = {}
        for k, i in enumerate(order):
            assert int(auxs[k]["sel"][3].item()) == 0, (variant, order, i)
            out[i] = (dsts[k].cpu().numpy(), auxs[k]["A"].cpu().numpy(), auxs[k]["t"].cpu().numpy())
        return out

    order_a, order_b = [0, 1, 2, 3], [3, 2, 0, 1]
    ws_bytes = max(hzd.workspace_size(p, [shapes[i] for i in o]) for o in (order_a, order_b))
    ref = run(order_a, torch.zeros(ws_bytes, dtype=torch.uint8, device="cuda"), graphs=True)
    g = torch.Generator(device="cuda").manual_seed(5)
    ws = torch.randint(0, 256, (ws_bytes,), dtype=torch.uint8, device="cuda", generator=g)
    for order in (order_a, order_b, order_a):
        got = run(order, ws, graphs=False)
        for i in order:
            for a, b_ in zip(got[i], ref[i]):
                assert np.array_equal(a, b_), (variant, order, i)


@pytest.mark.parametrize("w,h", [(320, 240), (1280, 720)])
def test_stage_profiling_times_every_launch(w, h):
    # direct launches run no init kernel: a small frame takes the one-block selection, a larger
    # one has leading blocks of k_dark zero its state
    I = _frame(w, h, 51)
    p = P(mode=hzd.MODE_OFFLINE, gf_radius=60, color_balance=1)
    ref = run_gpu(I, p, with_J=False)["out"]
    hzd.profile_read(reset=True)
    hzd.profile_enable(True)
    try:
        for _ in range(2):
            out = run_gpu(I, p, with_J=False)["out"]
            assert np.array_equal(out, ref)
        stages = hzd.profile_read(reset=True)
    finally:
        hzd.profile_enable(False)
    names = {"event_pair", "dark", "select", "gf_prep", "gf_ab", "gf_q", "recon_apply"}
    for name in names:
        launches, ms = stages[name]
        assert launches == 2 and ms >= 0.0, (name, stages[name])
    assert set(stages) == names


@pytest.mark.parametrize("w,h", [(320, 240), (640, 480)])
def test_caller_graph_capture_replays_and_is_not_timed(w, h):
    # a call made while the caller captures its stream joins the caller's graph; profiling
    # stays off for it (its events would complete only when the graph runs).  640x480 takes the
    # row-record selection, whose captured form zeroes the state with the init kernel on every
    # replay
    I1, I2 = _frame(w, h, 52), _frame(w, h, 53)
    p = P(mode=hzd.MODE_OFFLINE, gf_radius=16, color_balance=1)
    ref1, ref2 = run_gpu(I1, p, with_J=False)["out"], run_gpu(I2, p, with_J=False)["out"]
    src, dst = to_dev(I1), torch.zeros((h, w, 3), dtype=torch.uint8, device="cuda")
    ws = hzd.alloc_workspace(hzd.workspace_size(p, [(h, w)]))
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    hzd.profile_read(reset=True)
    hzd.profile_enable(True)
    try:
        with torch.cuda.graph(graph, stream=stream):
            hzd.dehaze_frame(src, dst, p, workspace=ws, stream=stream)
        assert hzd.profile_read(reset=True) == {}
    finally:
        hzd.profile_enable(False)
    for rep in range(4):
        src.copy_(to_dev(I1 if rep % 2 == 0 else I2))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(dst.cpu().numpy(), ref1 if rep % 2 == 0 else ref2), rep


def test_concurrent_launch_groups_with_graph_cache_and_under_capture():
    # three launch groups (two parameter sets, one with more than 16 frames) run concurrently on
    # the library's group streams; with the graph cache on, each group is captured on its stream
    # and replayed; inside a caller's graph capture the groups join the caller's graph in order
    rng = np.random.default_rng(78)
    shapes = [(int(rng.integers(20, 90)), int(rng.integers(20, 130))) for _ in range(20)]
    params = [P() if i % 4 else P(mode=hzd.MODE_OFFLINE, gf_radius=7, color_balance=1) for i in range(20)]
    sets = [[rng.integers(0, 256, size=(h, w, 3), dtype=np.uint8) for (h, w) in shapes] for _ in range(2)]
    refs = [[run_gpu(I, params[i], with_J=False)["out"] for i, I in enumerate(fs)] for fs in sets]
    srcs = [to_dev(I) for I in sets[0]]
    dsts = [torch.zeros_like(s) for s in srcs]
    ws = hzd.alloc_workspace(hzd.workspace_size(P(), shapes, params))
    stream = torch.cuda.Stream()
    try:
        hzd.graph_cache(16)
        with torch.cuda.stream(stream):
            for rep in range(4):
                for s_, I in zip(srcs, sets[rep % 2]):
                    s_.copy_(to_dev(I))
                hzd.dehaze_batch(srcs, dsts, P(), per_frame_params=params, workspace=ws, stream=stream)
                stream.synchronize()
                for i in range(20):
                    assert np.array_equal(dsts[i].cpu().numpy(), refs[rep % 2][i]), (rep, i)
    finally:
        hzd.graph_cache(0)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        hzd.dehaze_batch(srcs, dsts, P(), per_frame_params=params, workspace=ws, stream=stream)
    for rep in range(3):
        for s_, I in zip(srcs, sets[rep % 2]):
            s_.copy_(to_dev(I))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for i in range(20):
            assert np.array_equal(dsts[i].cpu().numpy(), refs[rep % 2][i]), ("captured", rep, i)


def test_uneven_batch_each_size_matches_oracle():
    # the 64-frame configuration's four sizes in one batch call (offline r=60, no colour balance);
    # every frame is checked element by element against the FP64 oracle
    shapes = [(640, 480), (1280, 720), (1920, 1080), (3840, 2160)]
    p = P(mode=hzd.MODE_OFFLINE, gf_radius=60, gf_eps=1e-3, color_balance=0)
    frames = [make_frame(w, h, 4000 + 16 * i).I for i, (w, h) in enumerate(shapes)]
    srcs = [to_dev(I) for I in frames]
    dsts = [torch.zeros_like(s) for s in srcs]
    auxs = [hzd.make_aux(h, w, J=False) for (w, h) in shapes]
    hzd.dehaze_batch(srcs, dsts, p, auxs=auxs)
    torch.cuda.synchronize()
    for i, I in enumerate(frames):
        g = {k: v.cpu().numpy() for k, v in auxs[i].items()}
        g["out"] = dsts[i].cpu().numpy()
        s = compare(I, p, g, label=f"batch {shapes[i]}")
        print(shapes[i], s)


def test_batch_larger_than_one_launch_group():
    # 21 frames, two parameter groups, more than 16 frames in one group: several launches
    rng = np.random.default_rng(77)
    shapes = [(int(rng.integers(20, 90)), int(rng.integers(20, 130))) for _ in range(21)]
    params = [P() if i % 3 else P(mode=hzd.MODE_OFFLINE, gf_radius=9, color_balance=1) for i in range(21)]
    frames = [rng.integers(0, 256, size=(h, w, 3), dtype=np.uint8) for (h, w) in shapes]
    srcs = [to_dev(I) for I in frames]
    dsts = [torch.zeros_like(s) for s in srcs]
    hzd.dehaze_batch(srcs, dsts, P(), per_frame_params=params)
    torch.cuda.synchronize()
    for i, I in enumerate(frames):
        assert np.array_equal(dsts[i].cpu().numpy(), run_gpu(I, params[i], with_J=False)["out"]), i


def _random_case(rng, seed):
    h, w = int(rng.integers(1, 200)), int(rng.integers(1, 300))
    if h >= 16 and w >= 16:
        I = make_frame(w, h, seed, beta=float(rng.uniform(0.5, 2.0))).I
    else:
        I = rng.integers(0, 256, size=(h, w, 3), dtype=np.uint8)
    p = P(mode=int(rng.integers(0, 2)), patch=int(rng.choice(np.arange(1, 32, 2))),
          omega=float(rng.uniform(0.5, 1.0)), t0=float(rng.uniform(0.05, 0.3)),
          top_frac=float(rng.uniform(0.0005, 0.05)), alpha=float(rng.uniform(0.5, 1.0)),
          gamma=float(rng.uniform(0.8, 2.5)), gf_radius=int(rng.integers(1, 65)),
          gf_eps=float(rng.choice([1e-6, 1e-4, 1e-3, 1e-2, 0.1])), color_balance=int(rng.integers(0, 2)),
          tx=int(rng.integers(0, 2)), precision=int(rng.integers(0, 2)))
    return I, p


@pytest.mark.parametrize("case", range(100))
def test_random_parameter_sweep(case):
    # seeded random combinations of every parameter, size and pitch, each checked against the
    # oracle element by element (the other tests vary one or two knobs at a time)
    rng = np.random.default_rng(9000 + case)
    I, p = _random_case(rng, 9000 + case)
    pad = int(rng.choice([0, 0, 1, 7]))
    compare(I, p, run_gpu(I, p, pitch_pad=pad), label=f"sweep {case} {I.shape} {p}")


@pytest.mark.parametrize("case", range(12))
def test_random_batch_sweep(case):
    # random frames with random parameters in one hzd_dehaze_batch call (several launch groups,
    # ragged block lists); every frame against the oracle
    rng = np.random.default_rng(7000 + case)
    cases = [_random_case(rng, 7000 + 100 * case + i) for i in range(int(rng.integers(2, 8)))]
    srcs = [to_dev(I) for I, _ in cases]
    dsts = [torch.zeros_like(s) for s in srcs]
    auxs = [hzd.make_aux(I.shape[0], I.shape[1]) for I, _ in cases]
    hzd.dehaze_batch(srcs, dsts, P(), per_frame_params=[p for _, p in cases], auxs=auxs)
    torch.cuda.synchronize()
    for i, (I, p) in enumerate(cases):
        g = {k: v.cpu().numpy() for k, v in auxs[i].items()}
        g["out"] = dsts[i].cpu().numpy()
        compare(I, p, g, label=f"batch sweep {case}/{i} {I.shape} {p}")


@pytest.mark.parametrize("case", range(8))
def test_random_large_frames(case):
    # random parameters on frames large enough for many strips and tiles
    rng = np.random.default_rng(5100 + case)
    _, p = _random_case(rng, 5100 + case)
    w, h = int(rng.integers(300, 1200)), int(rng.integers(200, 800))
    I = make_frame(w, h, 5100 + case, beta=float(rng.uniform(0.5, 2.0))).I
    compare(I, p, run_gpu(I, p), label=f"large {case} {w}x{h} {p}")


@pytest.mark.parametrize("gamma", [0.5, 1.0, 1.2, 1.8, 2.2, 3.0])
def test_fp16_t_map_output_bound_per_gamma(gamma):
    """Offline mode with colour balance at FP16 precision stores the refined t as
    binary16: the output is held to the bound derived from that rounding (asserted
    element by element by compare), and the largest LSB difference is reported per
    gamma.  FP32 on the same frames stays within 1 LSB."""
    worst = 0
    for (w, h, seed, dark) in [(640, 480, 80, 1.0), (640, 480, 81, 0.4), (320, 240, 82, 0.25)]:
        I = make_frame(w, h, seed).I
        if dark != 1.0:
            I = (I * dark).astype(np.uint8)
        for prec in (hzd.PREC_FP16, hzd.PREC_FP32):
            p = P(mode=hzd.MODE_OFFLINE, gf_radius=60, color_balance=1, gamma=gamma, precision=prec)
            s = compare(I, p, run_gpu(I, p), label=f"gamma {gamma} prec {prec} {w}x{h} dark {dark}")
            if prec == hzd.PREC_FP16:
                worst = max(worst, s["lsb_max"])
            else:
                assert s["lsb_max"] <= 1
    print(f"FP16 t map, gamma {gamma}: largest output difference {worst} LSB")
