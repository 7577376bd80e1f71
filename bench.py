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
# Algorithmic bytes of the method per pixel: read the frame I (3 B) and write the output
# (3 B).  Every other map is an intermediate that the method does not require to leave the
# chip, so the roofline fraction of a launch (and of the whole path) is 6 B/px x pixels per
# launch over its time, against the 8 TB/s HBM peak.
ALG_BYTES_PER_PX = 6.0

# Designed HBM bytes per pixel of each kernel (what this implementation reads and writes,
# intermediates included, itemised per entry); reported beside the algorithmic figure.
# Keys are the library's stage names.
STAGE_BYTES_PER_PX = {
    "dark": 7.0,          # I (3) in; D (1) + per-channel erosions E (3) out
    "select": 1.0,        # D (1) in (+ I at the pixels with D >= vstar); row records are 32 B per row
    "gf_prep": 17.0,      # I (3) + E (3) in; luma/t fixed point LP (8) + 8-row chunk sums (3) out
    "gf_ab": 18.0,        # LP (8) in; a/b fixed point (8) + chunk sums (2) out
    "gf_q": 15.0,         # a/b (8) + I (3) in; refined t (4) out
    "recon_apply": 10.0,  # I (3) + refined t (4) in; output (3) out
    "recon": 9.0,         # I (3) + E (3) in; output (3) out
    "recon_sums": 6.0,    # I (3) + E (3) in
    "init": 0.0,
}
# kernel symbols of this workload's stages, as rocprofv3 names them
# (the select stage is one kernel: the row pass, then the final step in the frame's last row block)
STAGE_KERNEL = {"init": "hzd::k_init", "dark": "hzd::k_dark<7,true>", "select": "hzd::k_select_rows<512>",
                "gf_prep": "hzd::k_gf_prep<0>", "gf_ab": "hzd::k_gf_ab<2,false>",
                "gf_q": "hzd::k_gf_q<2,1,false,false,false>", "recon_apply": "hzd::k_recon<2,2,false,false>"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_1080p_offline.txt")
RESIZE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_resize_1080p_to_640x480_x8.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2512_16609_amd", "csrc", "hzd_kernels.hip")
EXTRAS = ("320", "video", "uneven", "offline8", "resize1", "resize8", "smooth", "gamma", "balance")


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


def roofline_obj(kernel, px, avg_us, designed_bpp=None, traffic=None, event_pair_us=None):
    """Roofline of one kernel's launch: algorithmic bytes (6 B/px x pixels per launch) over
    its average launch time, against the HBM peak; the designed bytes and the counter
    traffic of the same launch are reported beside it."""
    alg = ALG_BYTES_PER_PX * px
    gbs = alg / (avg_us * 1e-6) / 1e9
    r = {"kernel": kernel, "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "alg_bytes_per_launch": alg,
         "avg_launch_us": round(avg_us, 3)}
    if designed_bpp is not None:
        dgbs = designed_bpp * px / (avg_us * 1e-6) / 1e9
        r["designed_bytes_per_launch"] = designed_bpp * px
        r["designed_frac"] = round(dgbs / HBM_PEAK_GBS, 4)
    r["traffic_ratio"] = None if traffic is None else round(traffic / alg, 2)
    if event_pair_us is not None:
        r["event_pair_us"] = round(event_pair_us, 3)
    return r


def path_roofline_obj(px, seconds, designed_bytes=None):
    """The whole path: 6 B/px x pixels over the time of the step (or launch)."""
    alg = ALG_BYTES_PER_PX * px
    gbs = alg / seconds / 1e9
    r = {"alg_bytes_per_step": alg, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(gbs / HBM_PEAK_GBS, 4)}
    if designed_bytes is not None:
        r["designed_bytes_per_step"] = designed_bytes
        r["designed_frac"] = round(designed_bytes / seconds / 1e9 / HBM_PEAK_GBS, 4)
    return r


class Samples:
    """Frames whose GPU results are checked against the FP64 oracle in the CPU leg: for each
    benchmark row, a few of its frames with the library's outputs (output bytes and, where
    captured, A, the selection and t)."""

    def __init__(self):
        self.rows = {}

    def add(self, row, I, p, g, seq=None):
        self.rows.setdefault(row, []).append({"I": I, "p": p, "g": g, "seq": seq})


def aux_small(hzd, torch, h, w, dev, t=True):
    d = {"A": torch.zeros(3, dtype=torch.float32, device=dev),
         "sel": torch.zeros(4, dtype=torch.int32, device=dev)}
    if t:
        d["t"] = torch.zeros((h, w), dtype=torch.float32, device=dev)
    return d


def to_host(aux, out):
    g = {k: v.cpu().numpy() for k, v in aux.items()}
    g["out"] = out.cpu().numpy()
    return g


def capture_frame(hzd, torch, I, p, dev, airlight_state=None):
    """One frame call with aux outputs: the library's result for the oracle check."""
    src = torch.from_numpy(I).to(dev)
    ho, wo = p.output_shape(I.shape[0], I.shape[1])
    dst = torch.empty((ho, wo, 3), dtype=torch.uint8, device=dev)
    aux = aux_small(hzd, torch, ho, wo, dev)
    hzd.dehaze_frame(src, dst, p, aux=aux, airlight_state=airlight_state)
    torch.cuda.synchronize()
    return to_host(aux, dst)


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


def resize_workloads(hzd, torch, dev, which, samples):
    """Sec. V step 1 at the paper's default working size: 1920x1080 inputs resized to 640x480,
    then the real-time path, from a pool of 16 distinct device-resident inputs."""
    from synth import make_frame
    out = {}
    sync = torch.cuda.synchronize
    W, H, Wo, Ho = 1920, 1080, 640, 480
    frames = [make_frame(W, H, 700 + k).I for k in range(4)]
    pool = [torch.from_numpy(frames[k % 4]).to(dev) for k in range(16)]
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
        samples.add("1920x1080_to_640x480_realtime", frames[0], p, capture_frame(hzd, torch, frames[0], p, dev))
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
        # the resize kernel's own roofline: it reads the inputs and writes the working-size copies
        alg = 8 * (3 * W * H + 3 * Wo * Ho)
        gbs = alg / (us["resize"] * 1e-6) / 1e9
        traffic = measured_traffic("hzd::k_resize", RESIZE_TRAFFIC_FILE)
        out["1920x1080_to_640x480_realtime_8_per_launch"] = {
            "input_MP_per_s": round(8 * W * H / 1e6 / per, 1), "output_MP_per_s": round(8 * Wo * Ho / 1e6 / per, 1),
            "ms_per_launch": round(per * 1e3, 4),
            "stage_us": {k: round(v, 3) for k, v in us.items()},
            "resize_kernel": {"kernel": "hzd::k_resize", "bound": "hbm", "achieved": round(gbs, 1),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                              "traffic": traffic, "bytes_per_launch": alg, "avg_launch_us": round(us["resize"], 3),
                              "bytes_rule": "3 B per input pixel read + 3 B per working-size pixel written"}}
        # the batched result of frame 0, with aux outputs
        aux = [aux_small(hzd, torch, Ho, Wo, dev)] + [None] * 7
        hzd.dehaze_batch(pool[:8], outs[:8], p, auxs=aux, workspace=ws8)
        sync()
        samples.add("1920x1080_to_640x480_realtime_8_per_launch", frames[0], p, to_host(aux[0], outs[0]))
    del pool, outs
    return out


def offline_1080p_8(hzd, torch, dev, samples):
    """The headline workload (1920x1080 offline, r = 60, colour balance) at 8 frames per launch,
    from two alternating sets of 8 distinct device-resident frames: throughput, and every stage's
    launch time, so the kernels' rooflines can be read at a size that fills the chip several
    times over."""
    from synth import make_frame
    sync = torch.cuda.synchronize
    W, H = 1920, 1080
    p = hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=60, gf_eps=1e-3, color_balance=1)
    I0 = make_frame(W, H, 5000).I
    base = [torch.from_numpy(I0).to(dev) for k in range(8)]
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
    dom = max(us, key=lambda k: us[k])
    designed = sum(STAGE_BYTES_PER_PX.get(k, 0.0) for k in us) * px
    srcs, dsts, ws = sets[0]
    aux = [aux_small(hzd, torch, H, W, dev)] + [None] * 7
    hzd.dehaze_batch(srcs, dsts, p, auxs=aux, workspace=ws)
    sync()
    samples.add("1920x1080_offline_8_per_launch", I0, p, to_host(aux[0], dsts[0]))
    del sets, base
    return {"1920x1080_offline_8_per_launch": {
        "MP_per_s": round(px / 1e6 / per, 1), "ms_per_launch": round(per * 1e3, 4),
        "stage_us": {k: round(v, 3) for k, v in us.items()},
        "stage_alg_GBps": {k: round(ALG_BYTES_PER_PX * px / (v * 1e-6) / 1e9, 1) for k, v in us.items()},
        "stage_designed_GBps": {k: round(STAGE_BYTES_PER_PX.get(k, 0.0) * px / (v * 1e-6) / 1e9, 1)
                                for k, v in us.items()},
        "path_roofline": path_roofline_obj(px, per, designed),
        "roofline": roofline_obj(dom, px, us[dom], STAGE_BYTES_PER_PX.get(dom))}}


def realtime_320(hzd, torch, dev, samples):
    """320x240 real-time single frame: launch-bound, so report latency.  The call reuses its
    buffers, so the library replays its captured HIP graph (graph cache on), as a frame loop
    of a video application would."""
    from synth import make_frame
    sync = torch.cuda.synchronize
    I = make_frame(320, 240, 1, beta=1.0).I
    p = hzd.Params()
    src = torch.from_numpy(I).to(dev)
    dst = torch.empty_like(src)
    ws = hzd.alloc_workspace(hzd.workspace_size(p, [(240, 320)]), dev)
    stream = torch.cuda.Stream()
    call = hzd.FrameCall(src, dst, p, ws, stream=stream)
    ssync = stream.synchronize
    row = {}
    for graphs in (1, 0):
        hzd.graph_cache(64 if graphs else 0)
        for _ in range(20):
            call()
        ssync()
        lat = []
        for _ in range(300):
            t0 = time.perf_counter()
            call()
            ssync()
            lat.append((time.perf_counter() - t0) * 1e3)
        per = timed(call, 500, ssync)
        row["graphs" if graphs else "direct_launches"] = {
            "MP_per_s": round(0.0768 / per, 1),
            "latency_ms": {"p50": rnd(percentile(lat, 50), 4), "p99": rnd(percentile(lat, 99), 4)}}
    hzd.graph_cache(0)
    sync()
    us = stage_us(hzd, call, 100, ssync)
    samples.add("320x240_realtime", I, p, capture_frame(hzd, torch, I, p, dev))
    return {"320x240_realtime": dict(row["graphs"], direct_launches=row["direct_launches"],
                                     stage_us={k: round(v, 2) for k, v in us.items()})}


def video_720p(hzd, torch, dev, samples):
    """1280x720 video, real-time mode, 8 frames per launch; a 300-frame clip is 38 launches
    over a pool of 64 distinct device-resident input and output buffers (16 frames of the
    panning clip, each in 4 copies): 354 MB, more than the 256 MB Infinity Cache.  The
    precision setting is FP16, which in real time changes nothing: t never leaves registers and
    is binary32, so the output bits equal those of the FP32 setting."""
    from synth import make_video
    sync = torch.cuda.synchronize
    v = make_video(1280, 720, nframes=300, seed=3)
    fidx = list(range(0, 300, 19))[:16]
    frames = [v.frame(f).I for f in fidx]
    NP = 64
    pool = [torch.from_numpy(frames[k % 16]).to(dev) for k in range(NP)]
    outs = [torch.empty_like(pool[0]) for _ in range(NP)]
    p3 = hzd.Params(precision=hzd.PREC_FP16)
    ws3 = hzd.alloc_workspace(hzd.workspace_size(p3, [(720, 1280)] * 8), dev)
    working_set = sum(t.numel() for t in pool + outs) + ws3.numel()

    def clip():
        for L in range(38):
            n = 8 if L < 37 else 4
            idx = [(8 * L + k) % NP for k in range(n)]
            hzd.dehaze_batch([pool[i] for i in idx], [outs[i] for i in idx], p3, workspace=ws3)
    clip()
    per = timed(clip, 12, sync)
    # the same launches alternating over two HIP streams, each with its own workspace (the
    # frames are independent in real-time mode without airlight smoothing); consecutive
    # launches write disjoint output buffers
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    wss = [ws3, hzd.alloc_workspace(hzd.workspace_size(p3, [(720, 1280)] * 8), dev)]

    def clip2():
        cur = torch.cuda.current_stream()
        for st in streams:
            st.wait_stream(cur)
        for L in range(38):
            n = 8 if L < 37 else 4
            idx = [(8 * L + k) % NP for k in range(n)]
            hzd.dehaze_batch([pool[i] for i in idx], [outs[i] for i in idx], p3, workspace=wss[L % 2],
                             stream=streams[L % 2])
        for st in streams:
            cur.wait_stream(st)
    clip2()
    per2 = timed(clip2, 12, sync)
    L = [0]

    def launch8():
        idx = [(8 * L[0] + k) % NP for k in range(8)]
        hzd.dehaze_batch([pool[i] for i in idx], [outs[i] for i in idx], p3, workspace=ws3)
        L[0] += 1
    us = stage_us(hzd, launch8, 24, sync)
    px = 8 * 1280 * 720
    dom = max(us, key=lambda k: us[k])
    # the batched results of the first launch's frames 0 and 7, with aux outputs
    aux = [aux_small(hzd, torch, 720, 1280, dev) if k in (0, 7) else None for k in range(8)]
    hzd.dehaze_batch(pool[:8], outs[:8], p3, auxs=aux, workspace=ws3)
    sync()
    for k in (0, 7):
        samples.add("1280x720_video_rt_8_per_launch", frames[k], p3, to_host(aux[k], outs[k]))
    return {"1280x720_video_rt_8_per_launch": {
        "MP_per_s": round(300 * 0.9216 / per, 1), "ms_per_300_frames": round(per * 1e3, 3),
        "two_streams_MP_per_s": round(300 * 0.9216 / per2, 1),
        "two_streams_ms_per_300_frames": round(per2 * 1e3, 3),
        "precision_setting": "fp16 (real-time t stays binary32 in registers: same bits as fp32)",
        "working_set_MB": round(working_set / 1e6, 1),
        "stage_us_8_frame_launch": {k: round(v, 3) for k, v in us.items()},
        "path_roofline": path_roofline_obj(300 * 1280 * 720, per),
        "two_streams_path_roofline": path_roofline_obj(300 * 1280 * 720, per2),
        "roofline": roofline_obj(dom, px, us[dom], STAGE_BYTES_PER_PX.get(dom))}}


def uneven_64(hzd, torch, dev, samples):
    """64 uneven frames (16 each of 480p, 720p, 1080p, 4K), offline mode r=60, no colour balance,
    one batch call; one seeded frame per size, copied into 16 distinct buffers."""
    from synth import make_frame
    sync = torch.cuda.synchronize
    shapes = [(640, 480), (1280, 720), (1920, 1080), (3840, 2160)]
    srcs, dsts, firsts = [], [], []
    for i, (w, h) in enumerate(shapes):
        I = make_frame(w, h, 4000 + 16 * i).I
        firsts.append(I)
        base = torch.from_numpy(I).to(dev)
        for _ in range(16):
            srcs.append(base.clone())
            dsts.append(torch.empty_like(base))
    p4 = hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=60, gf_eps=1e-3, color_balance=0)
    ws4 = hzd.alloc_workspace(hzd.workspace_size(p4, [(s.shape[0], s.shape[1]) for s in srcs]), dev)
    batch = lambda: hzd.dehaze_batch(srcs, dsts, p4, workspace=ws4)
    for _ in range(3):
        batch()
    per = timed(batch, 10, sync)
    px = sum(s.shape[0] * s.shape[1] for s in srcs)
    # the batch's result for one frame of each size, with aux outputs
    aux = [aux_small(hzd, torch, s.shape[0], s.shape[1], dev) if k % 16 == 0 else None for k, s in enumerate(srcs)]
    hzd.dehaze_batch(srcs, dsts, p4, auxs=aux, workspace=ws4)
    sync()
    for i in range(4):
        samples.add("64_uneven_frames_offline", firsts[i], p4, to_host(aux[16 * i], dsts[16 * i]))
    return {"64_uneven_frames_offline": {"MP_per_s": round(px / 1e6 / per, 1), "ms_per_batch": round(per * 1e3, 3),
                                         "MP_per_batch": round(px / 1e6, 2),
                                         "path_roofline": path_roofline_obj(px, per)}}


def smoothing_workload(hzd, torch, dev, samples, lams=(0.0, 0.9), n=32, passes=5, streams=8):
    """Temporal airlight smoothing on the first frames of the 1280x720 panning clip (real time):
    sequential frame calls carrying the stream's airlight state, and a server with `streams`
    such streams, each at lam = 0 and lam > 0.  Reports throughput and the mean frame-to-frame
    change of A (0..255 scale), the flicker the smoothing damps."""
    from synth import make_video
    sync = torch.cuda.synchronize
    W, H = 1280, 720
    mp = W * H / 1e6
    v = make_video(W, H, nframes=300, seed=3)
    host = [v.frame(f).I for f in range(n)]
    frames = [torch.from_numpy(I).to(dev) for I in host]
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
        if lam > 0:
            # a fresh stream state over the clip's first 8 frames: every frame's result in order
            st8 = hzd.make_airlight_state(dev)
            seq = [capture_frame(hzd, torch, host[k], p, dev, airlight_state=st8) for k in range(8)]
            samples.add("1280x720_clip_airlight_smoothing", host[7], p, seq[-1], seq=(host[:8], seq))
    return {"1280x720_clip_airlight_smoothing": dict(out, frames=n, served_streams=streams)}


def adaptive_gamma_workload(hzd, torch, dev, samples, reps=200):
    """Adaptive per-frame gamma against a fixed gamma on the 1920x1080 frame, one frame per call:
    offline (guided filter r=60, colour balance) and real time.  The adaptive rule needs the
    frame-wide luma sums of J before any pixel is corrected, so it adds a pass; its stage times
    come from HIP events on the launch stream."""
    from synth import make_frame
    sync = torch.cuda.synchronize
    W, H = 1920, 1080
    mp = W * H / 1e6
    I = make_frame(W, H, 2).I
    src = torch.from_numpy(I).to(dev)
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
            if adaptive:
                samples.add(f"1920x1080_adaptive_gamma_{name}", I, p, capture_frame(hzd, torch, I, p, dev))
        out[name] = row
    return {"1920x1080_adaptive_gamma": out}


def percentile_balance_workload(hzd, torch, dev, samples, reps=200):
    """The balance stage's second reading, the percentile ("simple") white balance, against
    gray-world on the 1920x1080 frame, one frame per call, offline (guided filter r=60) and
    real time.  Both balances need a frame-wide reduction of J_gamma (channel sums or code
    histograms) before any pixel is written, so both take one more pass."""
    from synth import make_frame
    sync = torch.cuda.synchronize
    W, H = 1920, 1080
    mp = W * H / 1e6
    I = make_frame(W, H, 2).I
    src = torch.from_numpy(I).to(dev)
    dst = torch.empty_like(src)
    out = {}
    for mode, name in ((hzd.MODE_OFFLINE, "offline"), (hzd.MODE_REALTIME, "realtime")):
        row = {}
        for cb, cname in ((1, "gray_world"), (2, "percentile")):
            p = hzd.Params(mode=mode, gf_radius=60, color_balance=cb, wb_percentile=0.02)
            ws = hzd.alloc_workspace(hzd.workspace_size(p, [(H, W)]), dev)
            call = hzd.FrameCall(src, dst, p, ws)
            for _ in range(10):
                call()
            per = timed(call, reps, sync)
            us = stage_us(hzd, call, 50, sync)
            row[cname] = {"MP_per_s": round(mp / per, 1), "us_per_frame": round(per * 1e6, 2),
                          "stage_us": {k: round(v, 2) for k, v in us.items()}}
            if cb == 2:
                samples.add(f"1920x1080_percentile_balance_{name}", I, p, capture_frame(hzd, torch, I, p, dev))
        out[name] = row
    return {"1920x1080_percentile_white_balance": dict(out, wb_percentile=0.02)}


def extra_workloads(hzd, torch, dev, samples, which=EXTRAS):
    """The other configurations, each timed on its own (inputs resident in HBM)."""
    out = {}
    if "320" in which:
        out.update(realtime_320(hzd, torch, dev, samples))
    if "video" in which:
        out.update(video_720p(hzd, torch, dev, samples))
    if "uneven" in which:
        out.update(uneven_64(hzd, torch, dev, samples))
    if "offline8" in which:
        out.update(offline_1080p_8(hzd, torch, dev, samples))
    if "resize1" in which or "resize8" in which:
        out.update(resize_workloads(hzd, torch, dev, which, samples))
    if "smooth" in which:
        out.update(smoothing_workload(hzd, torch, dev, samples))
    if "gamma" in which:
        out.update(adaptive_gamma_workload(hzd, torch, dev, samples))
    if "balance" in which:
        out.update(percentile_balance_workload(hzd, torch, dev, samples))
    torch.cuda.empty_cache()
    return out


def serving_mix(hzd, torch, dev, seconds: float, scales, samples, pool: int = 4):
    """Many concurrent streams through the continuous-batching server.

    32 streams; resolution per stream from {640x480, 1280x720, 1920x1080, 3840x2160}; 20 % of
    streams offline (guided filter r=60, eps=1e-3, colour balance), the rest real-time; Poisson
    arrivals at 30 fps per stream, times `scale`.  The sweep raises the scale until the server
    saturates: p99 latency above one frame interval (33.3 ms), frames refused because a
    stream's queue is full, or served MP/s clearly below offered.  Each stream cycles a
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
    streams, frames, hosts = [], [], []
    for sp in specs:
        sc = scenes[(sp.width, sp.height)]
        fl, hl = [], []
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
            hl.append(I)
        frames.append(fl)
        hosts.append(hl)
        streams.append(srv.open(p_off if sp.offline else p_rt, sp.width, sp.height))
    torch.cuda.synchronize()
    null_cb = hzd.DONE_FN()
    ready = torch.cuda.current_stream().cuda_stream   # the stream that filled the frame pools
    # warm every stream once
    for i, st in enumerate(streams):
        t = ctypes.c_uint64(0)
        L.hzd_stream_submit(st.handle, ctypes.byref(frames[i][0][2]), ready, null_cb, None, ctypes.byref(t))
        st.wait(int(t.value))
    results = []
    for scale in scales:
        # the same seeded Poisson processes, time-compressed by `scale`, for `seconds` of arrivals
        events = sorted((t / scale, i) for i, sp in enumerate(specs) for t in sp.arrivals if t / scale < seconds)
        tickets = []
        refused = 0
        refused_mp = 0.0
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
            rc = L.hzd_stream_submit(streams[i].handle, ctypes.byref(fr[2]), ready, null_cb, None, ctypes.byref(t))
            if rc == hzd.HZD_E_AGAIN:          # the stream's queue is full: the frame is dropped
                refused += 1
                refused_mp += fr[0].shape[0] * fr[0].shape[1] / 1e6
                continue
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
        offered = (mp + refused_mp) / seconds
        served = mp / span
        p99 = percentile(lat, 99)
        saturated = (p99 is not None and p99 > 33.3) or refused > 0 or served < 0.9 * offered
        results.append({"rate_scale": scale, "frames": len(tickets), "refused_queue_full": refused,
                        "offered_MP_per_s": round(offered, 1), "served_MP_per_s": round(served, 1),
                        "latency_ms": {"p50": rnd(percentile(lat, 50), 3), "p99": rnd(p99, 3),
                                       "max": rnd(float(max(lat)), 3) if lat else None},
                        "saturated": saturated})
        log(f"serving mix x{scale}: {results[-1]}")
        if saturated:
            break
    # served results of one stream of each (resolution, mode), for the oracle check
    seen = set()
    for i, sp in enumerate(specs):
        key = (sp.width, sp.height, sp.offline)
        if key in seen:
            continue
        seen.add(key)
        t = ctypes.c_uint64(0)
        rc = L.hzd_stream_submit(streams[i].handle, ctypes.byref(frames[i][0][2]), ready, null_cb, None,
                                 ctypes.byref(t))
        if rc != 0 or streams[i].wait(int(t.value))[0] != 0:
            raise RuntimeError(f"sample frame failed {rc}: {hzd.last_error()}")
        A, sel = streams[i].state()
        samples.add("serving_mix_32_streams", hosts[i][0], p_off if sp.offline else p_rt,
                    {"out": frames[i][0][1].cpu().numpy(), "A": np.array(A, dtype=np.float32),
                     "sel": np.array(sel, dtype=np.int32)})
    stats = srv.stats()
    for st in streams:
        st.close()
    srv.close()
    mix = {"streams": len(specs), "offline_streams": sum(sp.offline for sp in specs),
           "resolutions": {f"{w}x{h}": sum(1 for sp in specs if (sp.width, sp.height) == (w, h))
                           for (w, h) in RESOLUTIONS.values()},
           "seconds_per_point": seconds, "launches": int(stats["launches"])}
    ok = [r for r in results if not r["saturated"]]
    best = max(ok, key=lambda r: r["served_MP_per_s"]) if ok else None
    first_sat = next((r for r in results if r["saturated"]), None)
    return {"mix": mix, "points": results,
            "capacity_MP_per_s_unsaturated": best["served_MP_per_s"] if best else None,
            "saturation_point": None if first_sat is None else {
                "rate_scale": first_sat["rate_scale"], "offered_MP_per_s": first_sat["offered_MP_per_s"],
                "served_MP_per_s": first_sat["served_MP_per_s"], "p99_ms": first_sat["latency_ms"]["p99"],
                "refused_queue_full": first_sat["refused_queue_full"]}}


# --------------------------------------------------------------------------- CPU oracle leg
# The FP64 NumPy oracle is test infrastructure; in this file it is used here only: it is
# timed as the CPU baseline, and it checks the sampled GPU results of every row above.

def oracle_params(hzd, p):
    import oracle
    return oracle.Params(mode="offline" if p.mode == hzd.MODE_OFFLINE else "realtime", patch=p.patch,
                         omega=p.omega, t0=p.t0, top_frac=p.top_frac, alpha=p.alpha, gamma=p.gamma,
                         gf_radius=p.gf_radius, gf_eps=p.gf_eps, color_balance=int(p.color_balance),
                         tx="he" if p.tx == hzd.TX_HE else "paper", resize_width=p.resize_width,
                         resize_height=p.resize_height, airlight_smoothing=p.airlight_smoothing,
                         gamma_adaptive=bool(p.gamma_adaptive), gamma_target=p.gamma_target,
                         wb_percentile=p.wb_percentile)


def _oracle_worker(args):
    """One process of the all-core leg: `reps` oracle frames; returns the seconds they took."""
    I, po, reps = args
    import oracle
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.dehaze(I, po)
    return time.perf_counter() - t0


def cpu_baseline(I, p_oracle, budget_s: float, procs: int):
    """The FP64 oracle as it stands on the headline frame: one process (single thread) on a
    bounded sample, then frames spread over `procs` processes (one per host core)."""
    import multiprocessing as mp
    import oracle
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
    mpx = w * h / 1e6
    med = float(np.median(times))
    single = {"value": round(mpx / med, 4), "unit": "MP/s", "cores": 1,
              "sample": f"{len(times)} runs of one {w}x{h} frame (single process), median {med:.2f} s/frame"}
    reps = 2
    ctx = mp.get_context("spawn")          # fresh interpreters: nothing of the GPU process is inherited
    with ctx.Pool(procs) as pool:
        pool.map(_oracle_worker, [(I, p_oracle, 0)] * procs)    # start-up and imports, untimed
        t0 = time.perf_counter()
        pool.map(_oracle_worker, [(I, p_oracle, reps)] * procs)
        wall = time.perf_counter() - t0
    allc = {"value": round(procs * reps * mpx / wall, 4), "unit": "MP/s", "cores": procs, "kind": "oracle",
            "sample": f"{procs * reps} runs of one {w}x{h} frame of this workload through the FP64 NumPy oracle, "
                      f"spread over {procs} processes (one per core, {reps} each), {wall:.2f} s wall; "
                      f"host: {cpu_model()}, {os.cpu_count()} logical CPUs visible",
            "single_process": single}
    return allc, ref


def error_vs_oracle(ref, g, p_is_fp16_map=False):
    """The library's result for one frame against the oracle's: output LSB difference, and
    where captured the airlight, the selection and the transmission."""
    a = ref.aux
    d = np.abs(g["out"].astype(np.int32) - ref.out.astype(np.int32))
    e = {"out_max_lsb": int(d.max()), "out_share_1lsb": float((d == 1).mean()),
         "out_share_equal": float((d == 0).mean())}
    if "A" in g:
        e["A_equal"] = bool(np.array_equal(np.asarray(g["A"])[:3], a["A"].astype(np.float32)))
    if "sel" in g:
        s = np.asarray(g["sel"])
        e["selection_equal"] = bool(int(s[0]) == a["K"] and int(s[1]) == int(a["vstar"])
                                    and int(s[2]) == a["cutoff"])
        e["selection_status"] = int(s[3])
    if "t" in g:
        e["t_rel_max"] = float((np.abs(g["t"].astype(np.float64) - a["t"]) / a["t"]).max())
    return e


def merge_errors(errs):
    out = {"frames_checked": len(errs), "out_max_lsb": max(e["out_max_lsb"] for e in errs),
           "out_share_1lsb_max": max(e["out_share_1lsb"] for e in errs)}
    for k in ("A_equal", "selection_equal"):
        v = [e[k] for e in errs if k in e]
        if v:
            out[k] = all(v)
    v = [e["selection_status"] for e in errs if "selection_status" in e]
    if v:
        out["selection_status_max"] = max(v)
    v = [e["t_rel_max"] for e in errs if "t_rel_max" in e]
    if v:
        out["t_rel_max"] = max(v)
    return out


def oracle_checks(hzd, samples, refs=None):
    """Error of every sampled GPU result against the FP64 oracle, per benchmark row."""
    import oracle
    refs = refs or {}
    out = {}
    for row, items in samples.rows.items():
        errs = []
        for it in items:
            po = oracle_params(hzd, it["p"])
            if it["seq"] is not None:       # a stream's frames in order (airlight smoothing)
                Is, gs = it["seq"]
                rs = oracle.dehaze_sequence(Is, po)
                errs.extend(error_vs_oracle(r, g) for r, g in zip(rs, gs))
                continue
            ref = refs.get(id(it["I"])) or oracle.dehaze(it["I"], po)
            errs.append(error_vs_oracle(ref, it["g"]))
        out[row] = merge_errors(errs)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--rotate", type=int, default=10, help="distinct buffer sets cycled by the timed loop")
    ap.add_argument("--served-streams", type=int, default=8)
    ap.add_argument("--served-frames", type=int, default=100, help="frames per served stream")
    ap.add_argument("--latency-frames", type=int, default=200)
    ap.add_argument("--cpu-budget", type=float, default=10.0, help="seconds of single-process oracle time")
    ap.add_argument("--cpu-procs", type=int, default=0, help="processes of the all-core oracle leg (0 = cores, <= 16)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU oracle leg (baseline and checks)")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the other configurations")
    ap.add_argument("--extras", default=",".join(EXTRAS),
                    help="comma list of the other configurations to run: " + ", ".join(EXTRAS))
    ap.add_argument("--serving-seconds", type=float, default=1.5,
                    help="seconds of Poisson arrivals per point of the 32-stream serving mix (0 = skip)")
    ap.add_argument("--serving-scales", default="1,8,16,20,24,32,48",
                    help="arrival-rate multipliers of the sweep (it stops at the first saturated point)")
    ap.add_argument("--graphs", type=int, default=0,
                    help="timed plain loop: replay captured HIP graphs (1) or launch directly (0, the library's "
                         "default; faster than graph replay on this ROCm build); the other mode is timed after it")
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
    samples = Samples()
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
        # every buffer is written once here, so that no set's first touch (page mapping)
        # falls into the timed region when the warmup is shorter than the rotation
        dst = torch.zeros_like(src)
        ws = hzd.alloc_workspace(ws_bytes, dev).zero_()
        sets.append((src, dst, ws))
    working_set = sum(s.numel() + d.numel() + w.numel() for s, d, w in sets)
    # a stream of its own: the library replays captured graphs on any stream but the null stream
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    calls = [hzd.FrameCall(s, d, p, w, stream=stream) for s, d, w in sets]

    if args.copy_calibration_mb:
        n = args.copy_calibration_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b2 = torch.empty_like(a)
        for _ in range(5):
            b2.copy_(a)
        torch.cuda.synchronize()
        del a, b2

    # ---- plain: timed region (direct launches by default, no stage events)
    hzd.graph_cache(256 if args.graphs else 0)
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
    samples.add("plain_1080p_offline", fr.I, p, {"out": sets[0][1].cpu().numpy()})

    # ---- the same steps in the other launch mode (graph replay after direct launches, or back)
    hzd.graph_cache(0 if args.graphs else 256)
    for i in range(len(calls)):      # captures the graphs outside the timed loop
        calls[i]()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        calls[i % len(calls)]()
    torch.cuda.synchronize()
    plain_mps_other = args.steps * mp / (time.perf_counter() - t0)
    hzd.graph_cache(256 if args.graphs else 0)

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
    hzd.graph_cache(0)
    g_aux = capture_frame(hzd, torch, fr.I, p, dev)
    samples.add("plain_1080p_offline", fr.I, p, g_aux)

    # an empty event pair on the same stream measures the cost of bracketing a launch
    ev_n, ev_ms = stages.pop("event_pair", (0, 0.0))
    ev_us = 1e3 * ev_ms / max(ev_n, 1)
    stage_rows = {}
    for name, (n, tot_ms) in stages.items():
        avg_us = 1e3 * tot_ms / max(n, 1)
        kern_us = max(avg_us - ev_us, 1e-3)
        bpp = STAGE_BYTES_PER_PX.get(name, 0.0)
        stage_rows[name] = {"launches": n, "avg_us_between_events": round(avg_us, 3), "avg_us": round(kern_us, 3),
                            "alg_GBps": round(ALG_BYTES_PER_PX * W * H / (kern_us * 1e-6) / 1e9, 1),
                            "designed_bytes_per_px": bpp,
                            "designed_GBps": round(bpp * W * H / (kern_us * 1e-6) / 1e9, 1)}
    dom = max(stage_rows, key=lambda k: stage_rows[k]["avg_us"])
    d = stage_rows[dom]
    roofline = roofline_obj(dom, W * H, d["avg_us"], d["designed_bytes_per_px"],
                            measured_traffic(STAGE_KERNEL.get(dom)), ev_us)
    designed_path = sum(r["designed_bytes_per_px"] for r in stage_rows.values()) * W * H
    path_roofline = path_roofline_obj(W * H, ms_per_step * 1e-3, designed_path)

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
        A_s, sel_s = sts[0].state()
        samples.add("served_1080p_offline", fr.I, p, {"out": dsts[0][(F - 1) % 2].cpu().numpy(),
                                                       "A": np.array(A_s, dtype=np.float32),
                                                       "sel": np.array(sel_s, dtype=np.int32)})
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
                  "path_roofline": path_roofline_obj(S * F * W * H, t_sat),
                  "latency_ms_at_30fps_per_stream": {"p50": round(percentile(lat_paced, 50), 3),
                                                     "p99": round(percentile(lat_paced, 99), 3),
                                                     "offered_MP_per_s": round(S * rate * mp, 1)},
                  "launches": int(stats["launches"])}

    extra = None
    if not args.no_extra:
        log("other configurations")
        hzd.graph_cache(0)
        extra = extra_workloads(hzd, torch, dev, samples, which)

    serving = None
    if args.serving_seconds > 0:
        log("serving mix: 32 streams")
        hzd.graph_cache(0)
        serving = serving_mix(hzd, torch, dev, args.serving_seconds,
                              [float(x) for x in args.serving_scales.split(",")], samples)

    cpu = errors = None
    if not args.no_cpu_baseline:
        log("cpu leg: FP64 oracle baseline")
        po = oracle_params(hzd, p)
        procs = args.cpu_procs or min(16, os.cpu_count() or 1)
        cpu, ref = cpu_baseline(fr.I, po, args.cpu_budget, procs)
        log("cpu leg: oracle checks of the sampled GPU results")
        errors = oracle_checks(hzd, samples, refs={id(fr.I): ref})
        for name, e in errors.items():
            for holder in (extra or {}, ):
                if name in holder:
                    holder[name]["oracle_error"] = e
            if name == "serving_mix_32_streams" and serving is not None:
                serving["oracle_error"] = e
            if name == "served_1080p_offline" and served is not None:
                served["oracle_error"] = e

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
                  ("MP_per_s_direct_launches" if args.graphs else "MP_per_s_graph_replay"): round(plain_mps_other, 2),
                  "MP_per_s_with_stage_events_direct_launches": round(plain_mps_events, 2),
                  "latency_ms": {"p50": rnd(percentile(lat, 50), 4), "p99": rnd(percentile(lat, 99), 4)}},
        "served": served,
        "other_configs": extra,
        "serving_mix_32_streams": serving,
        "stages": stage_rows,
        "roofline": roofline,
        "path_roofline": path_roofline,
        "cpu_baseline": cpu,
        "oracle_error": None if errors is None else errors.get("plain_1080p_offline"),
        "oracle_error_by_row": errors,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
