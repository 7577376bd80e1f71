#!/usr/bin/env python3
"""Benchmark of the per-frame dehazing path on one MI355X.

Metric: megapixels/s dehazed at 1080p, plain (hzd_dehaze_frame, one frame
after another on one stream) versus served (hzd_stream_submit through the
continuous-batching server), with p50/p99 frame latency.

Workload (one step = one pass of the whole path over one frame): a seeded
synthetic 1920x1080 RGB8 hazy frame, offline mode (dark channel patch 15,
airlight top 0.1 %, transmission omega 0.95 / t0 0.1, guided filter r = 60,
eps = 1e-3 on the BT.601 guide, gamma 1.2, gray-world colour balance), FP32
with exact fixed-point box sums.  Inputs are resident in HBM before timing;
the loop rotates over distinct src/dst/workspace sets whose total exceeds the
256 MB Infinity Cache, so each step reads cold data.

Prints ONE JSON line.  --gpus N > 1 exits: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "megapixels/sec dehazed at 1080p (plain vs served); p50/p99 frame latency"
HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per pixel of each kernel (what it must read and write,
# itemised per entry).  Keys are the library's stage names.
STAGE_BYTES_PER_PX = {
    "dark": 7.0,          # I (3) in; D (1) + per-channel erosions E (3) out
    "select": 1.0,        # D (1) in (+ I at the pixels with D >= vstar); two kernels
    "gf_prep": 17.0,      # I (3) + E (3) in; luma/t fixed point LP (8) + 8-row chunk sums (3) out
    "gf_ab": 18.0,        # LP (8) in; a/b fixed point (8) + chunk sums (2) out
    "gf_q": 15.0,         # a/b (8) + I (3) in; refined t (4) out
    "recon_apply": 10.0,  # I (3) + refined t (4) in; output (3) out
    "recon": 9.0,         # I (3) + E (3) in; output (3) out
    "recon_sums": 6.0,    # I (3) + E (3) in
    "init": 0.0,
}
# kernel symbols of this workload's stages, as rocprofv3 names them
# (the select stage is two kernels; its traffic entry is the row pass)
STAGE_KERNEL = {"init": "hzd::k_init", "dark": "hzd::k_dark<7,true>", "select": "hzd::k_select_rows",
                "gf_prep": "hzd::k_gf_prep<0>", "gf_ab": "hzd::k_gf_ab<2>", "gf_q": "hzd::k_gf_q<2,1,false,false>",
                "recon_apply": "hzd::k_recon<2,2,false,false>"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_1080p_offline.txt")
RESIZE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_resize_1080p_to_640x480_x8.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2512_16609_amd", "csrc", "hzd_kernels.hip")
EXTRAS = ("320", "video", "uneven", "offline8", "resize1", "resize8", "smooth", "gamma")


def kernel_source_hash(path=KERNEL_SRC):
    """sha256[:16] of the kernel source's code: line comments, trailing blanks and empty lines
    removed (no string literal in the file contains //), so editing comments does not mark the
    committed counter summaries as stale."""
    import hashlib
    lines = []
    for line in open(path).read().splitlines():
        code = line.split("//", 1)[0].rstrip()
        if code:
            lines.append(code)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()[:16]


def measured_traffic(kernel, path=TRAFFIC_FILE):
    """Calibrated HBM-side bytes per launch of `kernel` from a committed counter summary, or
    None if the kernels changed since the counters were taken."""
    try:
        text = open(path).read()
        src = kernel_source_hash()
    except OSError:
        return None
    raw, scale, recorded = {}, None, None
    for line in text.splitlines():
        f = line.split()
        if f and f[0] == "RAW":
            raw[f[1]] = (float(f[3]), float(f[5]))
        elif f and f[0] == "SCALE":
            scale = (float(f[2]), float(f[4]))
        elif f and f[0] == "SOURCE":
            recorded = f[1]
    if recorded != src or scale is None or kernel not in raw:
        return None
    fetch, write = raw[kernel]
    return round((fetch * scale[0] + write * scale[1]) * 1024.0)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def percentile(xs, q):
    if len(xs) == 0:
        return None
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q))


def rnd(v, k):
    return None if v is None else round(v, k)


def cpu_baseline(I, p_oracle, budget_s: float, gpu_out=None):
    """The FP64 oracle as it stands, single process, on a bounded sample.  With gpu_out (the
    library's output for the same frame) also returns its error against the oracle's output."""
    import oracle  # test infrastructure: used only for this reported baseline
    times = []
    t_start = time.perf_counter()
    ref = None
    while True:
        t0 = time.perf_counter()
        ref = oracle.dehaze(I, p_oracle)
        times.append(time.perf_counter() - t0)
        if len(times) >= 3 and time.perf_counter() - t_start >= budget_s:
            break
        if len(times) >= 20:
            break
    h, w, _ = I.shape
    mp = w * h / 1e6
    med = float(np.median(times))
    base = {"value": round(mp / med, 4), "unit": "MP/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(times)} runs of one {w}x{h} frame of this workload through the FP64 NumPy "
                      f"oracle (single thread), median {med:.2f} s/frame; host: {cpu_model()}, "
                      f"{os.cpu_count()} logical CPUs visible"}
    err = None
    if gpu_out is not None:
        d = np.abs(gpu_out.astype(np.int32) - ref.out.astype(np.int32))
        err = {"frame": f"{w}x{h}, this workload", "out_max_lsb": int(d.max()),
               "out_share_1lsb": float((d == 1).mean()), "out_share_equal": float((d == 0).mean())}
    return base, err


def timed(fn, reps, sync):
    sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    sync()
    return (time.perf_counter() - t0) / reps


def stage_us(hzd, run, reps, sync):
    """Average µs of each stage's launches over `reps` calls of run(), from HIP events on the
    launch stream, less the cost of an empty event pair."""
    hzd.profile_read(reset=True)
    hzd.profile_enable(True)
    try:
        for _ in range(reps):
            run()
        sync()
        st = hzd.profile_read(reset=True)
    finally:
        hzd.profile_enable(False)
    ev_n, ev_ms = st.pop("event_pair", (0, 0.0))
    ev_us = 1e3 * ev_ms / max(ev_n, 1)
    return {k: max(1e3 * ms / max(n, 1) - ev_us, 1e-3) for k, (n, ms) in st.items()}


def resize_workloads(hzd, torch, dev, which):
    """Sec. V step 1 at the paper's default working size: 1920x1080 inputs resized to 640x480,
    then the real-time path, from a pool of 16 distinct device-resident inputs."""
    from synth import make_frame
    out = {}
    sync = torch.cuda.synchronize
    W, H, Wo, Ho = 1920, 1080, 640, 480
    pool = [torch.from_numpy(make_frame(W, H, 700 + k).I).to(dev) for k in range(16)]
    outs = [torch.empty((Ho, Wo, 3), dtype=torch.uint8, device=dev) for _ in range(16)]
    p = hzd.Params(resize_width=Wo, resize_height=Ho)
    if "resize1" in which:
        ws = hzd.alloc_workspace(hzd.workspace_size(p, [(H, W)]), dev)
        calls = [hzd.FrameCall(pool[k], outs[k], p, ws) for k in range(16)]
        for k in range(20):
            calls[k % 16]()
        lat = []
        for k in range(300):
            t0 = time.perf_counter()
            calls[k % 16]()
            sync()
            lat.append((time.perf_counter() - t0) * 1e3)
        n = [0]

        def one():
            calls[n[0] % 16]()
            n[0] += 1
        per = timed(one, 480, sync)
        out["1920x1080_to_640x480_realtime"] = {
            "input_MP_per_s": round(W * H / 1e6 / per, 1), "output_MP_per_s": round(Wo * Ho / 1e6 / per, 1),
            "latency_ms": {"p50": rnd(percentile(lat, 50), 4), "p99": rnd(percentile(lat, 99), 4)}}
    if "resize8" in which:
        ws8 = hzd.alloc_workspace(hzd.workspace_size(p, [(H, W)] * 8), dev)
        L = [0]

        def batch8():
            idx = [(8 * L[0] + k) % 16 for k in range(8)]
            hzd.dehaze_batch([pool[i] for i in idx], [outs[i] for i in idx], p, workspace=ws8)
            L[0] += 1
        for _ in range(4):
            batch8()
        per = timed(batch8, 40, sync)
        us = stage_us(hzd, batch8, 40, sync)
        alg = 8 * (3 * W * H + 3 * Wo * Ho)   # read the inputs, write the working-size copies
        gbs = alg / (us["resize"] * 1e-6) / 1e9
        out["1920x1080_to_640x480_realtime_8_per_launch"] = {
            "input_MP_per_s": round(8 * W * H / 1e6 / per, 1), "output_MP_per_s": round(8 * Wo * Ho / 1e6 / per, 1),
            "ms_per_launch": round(per * 1e3, 4),
            "stage_us": {k: round(v, 3) for k, v in us.items()},
            "roofline": {"kernel": "hzd::k_resize", "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "traffic": measured_traffic("hzd::k_resize", RESIZE_TRAFFIC_FILE),
                         "alg_bytes_per_launch": alg, "avg_launch_us": round(us["resize"], 3)}}
    del pool, outs
    return out


def offline_1080p_8(hzd, torch, dev):
    """The headline workload (1920x1080 offline, r = 60, colour balance) at 8 frames per launch,
    from two alternating sets of 8 distinct device-resident frames: throughput, and every stage's
    launch time with its algorithmic HBM rate, so the kernels' rooflines can be read at a size
    that fills the chip several times over."""
    from synth import make_frame
    sync = torch.cuda.synchronize
    W, H = 1920, 1080
    p = hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=60, gf_eps=1e-3, color_balance=1)
    base = [torch.from_numpy(make_frame(W, H, 5000 + k).I).to(dev) for k in range(8)]
    sets = []
    for _ in range(2):
        srcs = [b.clone() for b in base]
        dsts = [torch.empty_like(b) for b in base]
        sets.append((srcs, dsts, hzd.alloc_workspace(hzd.workspace_size(p, [(H, W)] * 8), dev)))
    L = [0]

    def batch8():
        srcs, dsts, ws = sets[L[0] % 2]
        hzd.dehaze_batch(srcs, dsts, p, workspace=ws)
        L[0] += 1
    for _ in range(4):
        batch8()
    per = timed(batch8, 40, sync)
    us = stage_us(hzd, batch8, 40, sync)
    px = 8 * W * H
    rates = {k: round(STAGE_BYTES_PER_PX.get(k, 0.0) * px / (v * 1e-6) / 1e9, 1) for k, v in us.items()}
    dom = max(us, key=lambda k: us[k])
    path_bytes = sum(STAGE_BYTES_PER_PX.get(k, 0.0) for k in us) * px
    del sets, base
    return {"1920x1080_offline_8_per_launch": {
        "MP_per_s": round(px / 1e6 / per, 1), "ms_per_launch": round(per * 1e3, 4),
        "stage_us": {k: round(v, 3) for k, v in us.items()}, "stage_alg_GBps": rates,
        "path_alg_GBps": round(path_bytes / per / 1e9, 1),
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": rates[dom], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(rates[dom] / HBM_PEAK_GBS, 4), "traffic": None,
                     "alg_bytes_per_launch": STAGE_BYTES_PER_PX.get(dom, 0.0) * px,
                     "avg_launch_us": round(us[dom], 3)}}}


def realtime_320(hzd, torch, dev):
    """320x240 real-time single frame: launch-bound, so report latency."""
    from synth import make_frame
    sync = torch.cuda.synchronize
    I = make_frame(320, 240, 1, beta=1.0).I
    p = hzd.Params()
    src = torch.from_numpy(I).to(dev)
    dst = torch.empty_like(src)
    ws = hzd.alloc_workspace(hzd.workspace_size(p, [(240, 320)]), dev)
    call = hzd.FrameCall(src, dst, p, ws)
    for _ in range(20):
        call()
    lat = []
    for _ in range(300):
        t0 = time.perf_counter()
        call()
        sync()
        lat.append((time.perf_counter() - t0) * 1e3)
    per = timed(call, 500, sync)
    return {"320x240_realtime": {"MP_per_s": round(0.0768 / per, 1), "latency_ms": {
        "p50": rnd(percentile(lat, 50), 4), "p99": rnd(percentile(lat, 99), 4)}}}


def video_720p(hzd, torch, dev):
    """1280x720 video, real-time mode with FP16 t, 8 frames per launch; a 300-frame clip is 38
    launches, drawn from a 16-frame device-resident pool of the panning clip."""
    from synth import make_video
    sync = torch.cuda.synchronize
    v = make_video(1280, 720, nframes=300, seed=3)
    pool = [torch.from_numpy(v.frame(f).I).to(dev) for f in range(0, 300, 19)][:16]
    outs = [torch.empty_like(pool[0]) for _ in range(16)]
    p3 = hzd.Params(precision=hzd.PREC_FP16)
    ws3 = hzd.alloc_workspace(hzd.workspace_size(p3, [(720, 1280)] * 8), dev)

    def clip():
        for L in range(38):
            n = 8 if L < 37 else 4
            idx = [(8 * L + k) % 16 for k in range(n)]
            hzd.dehaze_batch([pool[i] for i in idx], [outs[i] for i in idx], p3, workspace=ws3)
    clip()
    per = timed(clip, 3, sync)
    # the same launches alternating over two HIP streams, each with its own workspace (the
    # frames are independent in real-time mode without airlight smoothing); launch L writes
    # outputs 8 (L % 2) .. 8 (L % 2) + 7, so the two streams never write the same buffer
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    wss = [ws3, hzd.alloc_workspace(hzd.workspace_size(p3, [(720, 1280)] * 8), dev)]

    def clip2():
        cur = torch.cuda.current_stream()
        for st in streams:
            st.wait_stream(cur)
        for L in range(38):
            n = 8 if L < 37 else 4
            idx = [(8 * L + k) % 16 for k in range(n)]
            hzd.dehaze_batch([pool[i] for i in idx], [outs[i] for i in idx], p3, workspace=wss[L % 2],
                             stream=streams[L % 2])
        for st in streams:
            cur.wait_stream(st)
    clip2()
    per2 = timed(clip2, 3, sync)
    return {"1280x720_video_rt_fp16_8_per_launch": {"MP_per_s": round(300 * 0.9216 / per, 1),
                                                    "ms_per_300_frames": round(per * 1e3, 3),
                                                    "two_streams_MP_per_s": round(300 * 0.9216 / per2, 1),
                                                    "two_streams_ms_per_300_frames": round(per2 * 1e3, 3)}}


def uneven_64(hzd, torch, dev):
    """64 uneven frames (16 each of 480p, 720p, 1080p, 4K), offline mode r=60, no colour balance,
    one batch call; one seeded frame per size, copied into 16 distinct buffers."""
    from synth import make_frame
    sync = torch.cuda.synchronize
    shapes = [(640, 480), (1280, 720), (1920, 1080), (3840, 2160)]
    srcs, dsts = [], []
    for i, (w, h) in enumerate(shapes):
        base = torch.from_numpy(make_frame(w, h, 4000 + 16 * i).I).to(dev)
        for _ in range(16):
            srcs.append(base.clone())
            dsts.append(torch.empty_like(base))
    p4 = hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=60, gf_eps=1e-3, color_balance=0)
    ws4 = hzd.alloc_workspace(hzd.workspace_size(p4, [(s.shape[0], s.shape[1]) for s in srcs]), dev)
    batch = lambda: hzd.dehaze_batch(srcs, dsts, p4, workspace=ws4)
    for _ in range(3):
        batch()
    per = timed(batch, 10, sync)
    mp4 = sum(s.shape[0] * s.shape[1] for s in srcs) / 1e6
    return {"64_uneven_frames_offline": {"MP_per_s": round(mp4 / per, 1), "ms_per_batch": round(per * 1e3, 3),
                                         "MP_per_batch": round(mp4, 2)}}


def smoothing_workload(hzd, torch, dev, lams=(0.0, 0.9), n=32, passes=5, streams=8):
    """Temporal airlight smoothing on the first frames of the 1280x720 panning clip (real time,
    FP16 t): sequential frame calls carrying the stream's airlight state, and a server with
    `streams` such streams, each at lam = 0 and lam > 0.  Reports throughput and the mean
    frame-to-frame change of A (0..255 scale), the flicker the smoothing damps."""
    from synth import make_video
    sync = torch.cuda.synchronize
    W, H = 1280, 720
    mp = W * H / 1e6
    v = make_video(W, H, nframes=300, seed=3)
    frames = [torch.from_numpy(v.frame(f).I).to(dev) for f in range(n)]
    out = {}
    for lam in lams:
        p = hzd.Params(precision=hzd.PREC_FP16, airlight_smoothing=lam)
        state = hzd.make_airlight_state(dev)
        ws = hzd.alloc_workspace(hzd.workspace_size(p, [(H, W)]), dev)
        dst = torch.empty_like(frames[0])
        As = torch.zeros((n, 4), dtype=torch.float32, device=dev)
        calls = [hzd.FrameCall(frames[k], dst, p, ws, aux={"A": As[k]}, airlight_state=state) for k in range(n)]
        for c in calls:
            c()
        sync()
        t0 = time.perf_counter()
        for _ in range(passes):
            for c in calls:
                c()
        sync()
        seq_mps = passes * n * mp / (time.perf_counter() - t0)
        A = As[:, :3].cpu().numpy().astype(np.float64)
        dA = np.abs(np.diff(A, axis=0)).mean()
        srv = hzd.Server(arena_bytes=streams * hzd.stream_arena_size(p, W, H) + 4096, max_inflight=16,
                         frames_per_launch=8, hip_streams=4)
        sts = [srv.open(p, W, H) for _ in range(streams)]
        dsts = [torch.empty_like(frames[0]) for _ in range(streams)]
        def served_pass():
            tk = [(st, st.submit(frames[k], dsts[i])) for k in range(n) for i, st in enumerate(sts)]
            for st, t in tk:
                rc, _ = st.wait(t)
                assert rc == 0, rc
        served_pass()   # warm: every HIP stream of the new server has run launches
        t0 = time.perf_counter()
        for _ in range(passes):
            served_pass()
        served_mps = passes * streams * n * mp / (time.perf_counter() - t0)
        for st in sts:
            st.close()
        srv.close()
        out[f"lambda_{lam:g}"] = {"sequential_frame_calls_MP_per_s": round(seq_mps, 1),
                                  "served_MP_per_s": round(served_mps, 1),
                                  "mean_abs_frame_to_frame_dA": round(float(dA), 4)}
    return {"1280x720_clip_airlight_smoothing": dict(out, frames=n, served_streams=streams)}


def adaptive_gamma_workload(hzd, torch, dev, reps=200):
    """Adaptive per-frame gamma against a fixed gamma on the 1920x1080 frame, one frame per call:
    offline (guided filter r=60, colour balance) and real time.  The adaptive rule needs the
    frame-wide luma sums of J before any pixel is corrected, so it adds a pass; its stage times
    come from HIP events on the launch stream."""
    from synth import make_frame
    sync = torch.cuda.synchronize
    W, H = 1920, 1080
    mp = W * H / 1e6
    src = torch.from_numpy(make_frame(W, H, 2).I).to(dev)
    dst = torch.empty_like(src)
    out = {}
    for mode, name in ((hzd.MODE_OFFLINE, "offline"), (hzd.MODE_REALTIME, "realtime")):
        row = {}
        for adaptive in (0, 1):
            p = hzd.Params(mode=mode, gf_radius=60, color_balance=int(mode == hzd.MODE_OFFLINE),
                           gamma_adaptive=adaptive, gamma_target=0.7)
            ws = hzd.alloc_workspace(hzd.workspace_size(p, [(H, W)]), dev)
            call = hzd.FrameCall(src, dst, p, ws)
            for _ in range(10):
                call()
            per = timed(call, reps, sync)
            us = stage_us(hzd, call, 50, sync)
            row["adaptive" if adaptive else "fixed"] = {"MP_per_s": round(mp / per, 1), "us_per_frame": round(per * 1e6, 2),
                                                        "stage_us": {k: round(v, 2) for k, v in us.items()}}
        out[name] = row
    return {"1920x1080_adaptive_gamma": out}


def extra_workloads(hzd, torch, dev, which=EXTRAS):
    """The other configurations, each timed on its own (inputs resident in HBM)."""
    out = {}
    if "320" in which:
        out.update(realtime_320(hzd, torch, dev))
    if "video" in which:
        out.update(video_720p(hzd, torch, dev))
    if "uneven" in which:
        out.update(uneven_64(hzd, torch, dev))
    if "offline8" in which:
        out.update(offline_1080p_8(hzd, torch, dev))
    if "resize1" in which or "resize8" in which:
        out.update(resize_workloads(hzd, torch, dev, which))
    if "smooth" in which:
        out.update(smoothing_workload(hzd, torch, dev))
    if "gamma" in which:
        out.update(adaptive_gamma_workload(hzd, torch, dev))
    torch.cuda.empty_cache()
    return out


def serving_mix(hzd, torch, dev, seconds: float, scales, pool: int = 4):
    """Many concurrent streams through the continuous-batching server.

    32 streams; resolution per stream from {640x480, 1280x720, 1920x1080, 3840x2160}; 20 % of
    streams offline (guided filter r=60, eps=1e-3, colour balance), the rest real-time; Poisson
    arrivals at 30 fps per stream (times `scale` for the saturation sweep).  Each stream cycles a
    `pool`-frame device-resident clip of a panning crop, so no host-to-device copy is timed.
    Latency runs from the scheduled arrival time to the scheduler observing completion."""
    import ctypes
    from synth import RESOLUTIONS, haze, make_scene, make_streams, quantize_u8
    L = hzd.lib()
    p_rt = hzd.Params()
    p_off = hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=60, gf_eps=1e-3, color_balance=1)
    specs = make_streams(32, seconds * max(scales), rate=30.0, seed=5)
    scenes = {}
    for sp in specs:
        key = (sp.width, sp.height)
        if key not in scenes:
            scenes[key] = make_scene(sp.width + 64, sp.height + 16, 5000 + sp.width)
    rng = np.random.Generator(np.random.PCG64(55))
    arena = sum(2 * (hzd.workspace_size(p_off if sp.offline else p_rt, [(sp.height, sp.width)]) + 256) + 4096
                for sp in specs) + (1 << 24)
    srv = hzd.Server(arena_bytes=arena, max_inflight=32, frames_per_launch=8, hip_streams=4)
    streams, frames = [], []
    for sp in specs:
        sc = scenes[(sp.width, sp.height)]
        fl = []
        for k in range(pool):
            x, y = int(rng.integers(0, 64)), int(rng.integers(0, 16))
            J = sc.J[y:y + sp.height, x:x + sp.width]
            d = sc.depth[y:y + sp.height, x:x + sp.width]
            beta = float(rng.uniform(0.6, 1.6))
            A = np.array([0.85, 0.88, 0.90]) + rng.uniform(-0.03, 0.03, size=3)
            I = quantize_u8(haze(J, np.exp(-beta * d), A, noise_rng=np.random.Generator(np.random.PCG64((sp.seed, k)))))
            src = torch.from_numpy(I).to(dev)
            dst = torch.empty_like(src)
            fl.append((src, dst, hzd._frame_struct(src, dst, p_off if sp.offline else p_rt)))
        frames.append(fl)
        streams.append(srv.open(p_off if sp.offline else p_rt, sp.width, sp.height))
    torch.cuda.synchronize()
    null_cb = hzd.DONE_FN()
    # warm every stream once
    for i, st in enumerate(streams):
        t = ctypes.c_uint64(0)
        L.hzd_stream_submit(st.handle, ctypes.byref(frames[i][0][2]), null_cb, None, ctypes.byref(t))
        st.wait(int(t.value))
    results = []
    for scale in scales:
        # the same seeded Poisson processes, time-compressed by `scale`, for `seconds` of arrivals
        events = sorted((t / scale, i) for i, sp in enumerate(specs) for t in sp.arrivals if t / scale < seconds)
        tickets = []
        t_base = time.perf_counter() + 0.05
        counters = [0] * len(specs)
        for when, i in events:
            target = t_base + when
            while True:
                now = time.perf_counter()
                if now >= target:
                    break
                if target - now > 0.002:
                    time.sleep(0.001)
            fr = frames[i][counters[i] % pool]
            counters[i] += 1
            t = ctypes.c_uint64(0)
            rc = L.hzd_stream_submit(streams[i].handle, ctypes.byref(fr[2]), null_cb, None, ctypes.byref(t))
            if rc != 0:
                raise RuntimeError(f"submit failed {rc}: {hzd.last_error()}")
            tickets.append((i, int(t.value), time.perf_counter() - target, fr[0].shape[0] * fr[0].shape[1]))
        lat, mp = [], 0.0
        for i, tk, lag, px in tickets:
            rc, ns = streams[i].wait(tk)
            if rc != 0:
                raise RuntimeError(f"frame failed {rc}")
            lat.append(ns / 1e6 + lag * 1e3)
            mp += px / 1e6
        span = time.perf_counter() - t_base
        results.append({"rate_scale": scale, "frames": len(tickets), "offered_MP_per_s": round(mp / seconds, 1),
                        "served_MP_per_s": round(mp / span, 1),
                        "latency_ms": {"p50": rnd(percentile(lat, 50), 3), "p99": rnd(percentile(lat, 99), 3),
                                       "max": rnd(float(max(lat)), 3)}})
        log(f"serving mix x{scale}: {results[-1]}")
    stats = srv.stats()
    for st in streams:
        st.close()
    srv.close()
    mix = {"streams": len(specs), "offline_streams": sum(sp.offline for sp in specs),
           "resolutions": {f"{w}x{h}": sum(1 for sp in specs if (sp.width, sp.height) == (w, h))
                           for (w, h) in RESOLUTIONS.values()},
           "seconds_per_point": seconds, "launches": int(stats["launches"])}
    ok = [r for r in results if r["latency_ms"]["p99"] is not None and r["latency_ms"]["p99"] <= 33.3]
    best = max(ok, key=lambda r: r["served_MP_per_s"]) if ok else None
    return {"mix": mix, "points": results,
            "max_sustained_MP_per_s_with_p99_under_33ms": best["served_MP_per_s"] if best else None}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--rotate", type=int, default=10, help="distinct buffer sets cycled by the timed loop")
    ap.add_argument("--served-streams", type=int, default=8)
    ap.add_argument("--served-frames", type=int, default=100, help="frames per served stream")
    ap.add_argument("--latency-frames", type=int, default=200)
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle time for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the other configurations")
    ap.add_argument("--extras", default=",".join(EXTRAS),
                    help="comma list of the other configurations to run: " + ", ".join(EXTRAS))
    ap.add_argument("--serving-seconds", type=float, default=1.5,
                    help="seconds of Poisson arrivals per point of the 32-stream serving mix (0 = skip)")
    ap.add_argument("--serving-scales", default="1,4,8,12,16", help="arrival-rate multipliers of the sweep")
    ap.add_argument("--graphs", type=int, default=1, help="replay captured HIP graphs (1) or launch directly (0)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="also run 5 device-to-device copies of this many MB (a kernel of known traffic for "
                         "scaling hardware byte counters)")
    args = ap.parse_args()
    which = set(x for x in args.extras.split(",") if x)
    if which - set(EXTRAS):
        print(f"unknown --extras {sorted(which - set(EXTRAS))}; choose from {EXTRAS}", file=sys.stderr)
        sys.exit(2)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the library has no multi-GPU path: frames and streams are independent and would shard "
              "across GPUs with no communication.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2512_16609_amd as hzd
    from synth import make_frame

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    hzd.lib()  # fail loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    W, H = 1920, 1080
    mp = W * H / 1e6
    log("generating the 1080p frame")
    fr = make_frame(W, H, 2)
    p = hzd.Params(mode=hzd.MODE_OFFLINE, patch=15, omega=0.95, t0=0.1, top_frac=0.001, alpha=0.8,
                   gamma=1.2, gf_radius=60, gf_eps=1e-3, color_balance=1, tx=hzd.TX_HE,
                   precision=hzd.PREC_FP32)
    ws_bytes = hzd.workspace_size(p, [(H, W)])
    src0 = torch.from_numpy(fr.I).to(dev)
    sets = []
    for _ in range(max(1, args.rotate)):
        src = src0.clone()
        dst = torch.empty_like(src)
        ws = hzd.alloc_workspace(ws_bytes, dev)
        sets.append((src, dst, ws))
    working_set = sum(s.numel() + d.numel() + w.numel() for s, d, w in sets)
    stream = torch.cuda.current_stream()
    calls = [hzd.FrameCall(s, d, p, w, stream=stream) for s, d, w in sets]

    if args.copy_calibration_mb:
        n = args.copy_calibration_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b2 = torch.empty_like(a)
        for _ in range(5):
            b2.copy_(a)
        torch.cuda.synchronize()
        del a, b2

    # ---- plain: timed region (production configuration: captured HIP graphs, no stage events)
    if args.graphs:
        hzd.graph_cache(256)
    log("plain: warmup")
    for i in range(args.warmup):
        calls[i % len(calls)]()
    torch.cuda.synchronize()
    log(f"plain: {args.steps} timed steps")
    t0 = time.perf_counter()
    for i in range(args.steps):
        calls[i % len(calls)]()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    plain_mps = args.steps * mp / elapsed
    ms_per_step = 1e3 * elapsed / args.steps

    # ---- the same steps with per-kernel HIP events on the launch stream (direct launches)
    hzd.profile_read(reset=True)
    hzd.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        calls[i % len(calls)]()
    torch.cuda.synchronize()
    plain_mps_events = args.steps * mp / (time.perf_counter() - t0)
    stages = hzd.profile_read(reset=True)
    hzd.profile_enable(False)

    # ---- plain: per-frame latency (one frame at a time, idle GPU)
    lat = []
    for i in range(args.latency_frames):
        t0 = time.perf_counter()
        calls[i % len(calls)]()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)

    # an empty event pair on the same stream measures the cost of bracketing a launch
    ev_n, ev_ms = stages.pop("event_pair", (0, 0.0))
    ev_us = 1e3 * ev_ms / max(ev_n, 1)
    stage_rows = {}
    for name, (n, tot_ms) in stages.items():
        avg_us = 1e3 * tot_ms / max(n, 1)
        kern_us = max(avg_us - ev_us, 1e-3)
        bpp = STAGE_BYTES_PER_PX.get(name, 0.0)
        gbs = bpp * W * H / (kern_us * 1e-6) / 1e9
        stage_rows[name] = {"launches": n, "avg_us_between_events": round(avg_us, 3), "avg_us": round(kern_us, 3),
                            "alg_bytes_per_px": bpp, "alg_GBps": round(gbs, 1)}
    dom = max(stage_rows, key=lambda k: stage_rows[k]["avg_us"])
    d = stage_rows[dom]
    traffic = measured_traffic(STAGE_KERNEL.get(dom))
    roofline = {"kernel": dom, "bound": "hbm", "achieved": d["alg_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(d["alg_GBps"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                "alg_bytes_per_launch": d["alg_bytes_per_px"] * W * H, "avg_launch_us": d["avg_us"],
                "event_pair_us": round(ev_us, 3)}
    # the whole path: every stage's algorithmic bytes per step over the timed step time
    path_bytes = sum(r["alg_bytes_per_px"] for r in stage_rows.values()) * W * H
    path_gbs = path_bytes / (ms_per_step * 1e-3) / 1e9
    path_roofline = {"alg_bytes_per_step": path_bytes, "achieved": round(path_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(path_gbs / HBM_PEAK_GBS, 4)}

    # ---- served
    served = None
    if not args.no_served:
        log("served: continuous batching")
        # served batches change composition from launch to launch, so graphs keyed by the
        # exact launch arguments would mostly be captured once and never replayed
        hzd.graph_cache(0)
        S, F = args.served_streams, args.served_frames
        per_stream_ws = 2 * (hzd.workspace_size(p, [(H, W)]) + 256) + 1024
        srv = hzd.Server(arena_bytes=S * per_stream_ws + (1 << 20), max_inflight=16, frames_per_launch=8,
                         hip_streams=4)
        sts = [srv.open(p, W, H) for _ in range(S)]
        srcs = [src0.clone() for _ in range(S)]
        dsts = [[torch.empty_like(src0) for _ in range(2)] for _ in range(S)]
        torch.cuda.synchronize()
        # warm: several saturated rounds, so every HIP stream of the new server has run
        # launches before the timed region
        for _ in range(4):
            tk = [(st, st.submit(srcs[i], dsts[i][f % 2])) for f in range(4) for i, st in enumerate(sts)]
            for st, t in tk:
                st.wait(t)
        # saturation throughput: every stream keeps its queue full
        t0 = time.perf_counter()
        tickets = []
        for f in range(F):
            for i, st in enumerate(sts):
                tickets.append((st, st.submit(srcs[i], dsts[i][f % 2])))
        for st, t in tickets:
            rc, _ = st.wait(t)
            assert rc == 0, rc
        t_sat = time.perf_counter() - t0
        served_mps = S * F * mp / t_sat
        # latency under a paced load: each stream submits at 30 fps
        rate = 30.0
        n_paced = 30
        t_base = time.perf_counter() + 0.01
        sched = sorted((t_base + k / rate + i / (rate * S), i) for i in range(S) for k in range(n_paced))
        paced = []
        for when, i in sched:
            while time.perf_counter() < when:
                pass
            paced.append((sts[i], sts[i].submit(srcs[i], dsts[i][len(paced) % 2])))
        lat_paced = []
        for st, t in paced:
            rc, ns = st.wait(t)
            assert rc == 0, rc
            lat_paced.append(ns / 1e6)
        stats = srv.stats()
        for st in sts:
            st.close()
        srv.close()
        served = {"MP_per_s": round(served_mps, 2), "streams": S, "frames": S * F,
                  "vs_plain": round(served_mps / plain_mps, 3),
                  "latency_ms_at_30fps_per_stream": {"p50": round(percentile(lat_paced, 50), 3),
                                                     "p99": round(percentile(lat_paced, 99), 3),
                                                     "offered_MP_per_s": round(S * rate * mp, 1)},
                  "launches": int(stats["launches"])}

    extra = None
    if not args.no_extra:
        log("other configurations")
        hzd.graph_cache(0)
        extra = extra_workloads(hzd, torch, dev, which)

    serving = None
    if args.serving_seconds > 0:
        log("serving mix: 32 streams")
        hzd.graph_cache(0)
        serving = serving_mix(hzd, torch, dev, args.serving_seconds,
                              [float(x) for x in args.serving_scales.split(",")])

    cpu = oracle_err = None
    if not args.no_cpu_baseline:
        log("cpu baseline: FP64 oracle")
        import oracle
        po = oracle.Params(mode="offline", patch=15, omega=0.95, t0=0.1, top_frac=0.001, alpha=0.8, gamma=1.2,
                           gf_radius=60, gf_eps=1e-3, color_balance=True, tx="he")
        gpu_out = sets[0][1].cpu().numpy()   # the timed loop's output for this frame
        cpu, oracle_err = cpu_baseline(fr.I, po, args.cpu_budget, gpu_out)

    out = {
        "metric": METRIC, "value": round(plain_mps, 2), "unit": "MP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "1920x1080 RGB8 synthetic hazy frame, offline mode: patch 15, top 0.1%, "
                               "omega 0.95, t0 0.1, guided filter r=60 eps=1e-3, gamma 1.2, colour balance; "
                               "one frame per step",
                   "global_batch": 1, "seq_len": None, "parallelism": "single GPU",
                   "rotating_buffer_sets": len(sets), "working_set_MB": round(working_set / 1e6, 1)},
        "plain": {"MP_per_s": round(plain_mps, 2), "graphs": bool(args.graphs),
                  "MP_per_s_with_stage_events_direct_launches": round(plain_mps_events, 2),
                  "latency_ms": {"p50": rnd(percentile(lat, 50), 4), "p99": rnd(percentile(lat, 99), 4)}},
        "served": served,
        "other_configs": extra,
        "serving_mix_32_streams": serving,
        "stages": stage_rows,
        "roofline": roofline,
        "path_roofline": path_roofline,
        "cpu_baseline": cpu,
        "oracle_error": oracle_err,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
