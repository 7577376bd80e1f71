"""Several host threads using the library at once, each with its own HIP stream, buffers and
workspace: batch calls whose launch groups run on the calling thread's group streams, and frame
calls, with the graph cache off and on.  Every result must equal the one-thread result."""
import threading

import numpy as np
import pytest
import torch

import paper_2512_16609_amd as hzd
from parity import run_gpu, to_dev

pytestmark = pytest.mark.gpu

P = hzd.Params


def _work(seed):
    # six frames of two parameter sets (two launch groups) plus one frame call
    rng = np.random.default_rng(seed)
    shapes = [(int(rng.integers(24, 100)), int(rng.integers(24, 140))) for _ in range(6)]
    params = [P() if i % 3 else P(mode=hzd.MODE_OFFLINE, gf_radius=5 + seed % 4, color_balance=1)
              for i in range(6)]
    frames = [rng.integers(0, 256, size=(h, w, 3), dtype=np.uint8) for (h, w) in shapes]
    single = rng.integers(0, 256, size=(120, 160, 3), dtype=np.uint8)
    return shapes, params, frames, single


@pytest.mark.parametrize("cache", [0, 32])
def test_threads_share_the_library(cache):
    T, reps = 4, 6
    works = [_work(90 + t) for t in range(T)]
    p1 = P(mode=hzd.MODE_OFFLINE, gf_radius=11, color_balance=1)
    refs = [([run_gpu(I, ps[i], with_J=False)["out"] for i, I in enumerate(fs)],
             run_gpu(one, p1, with_J=False)["out"]) for (_, ps, fs, one) in works]
    errors = []
    start = threading.Barrier(T)

    def worker(t):
        try:
            shapes, params, frames, one = works[t]
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                srcs = [to_dev(I) for I in frames]
                dsts = [torch.zeros_like(s) for s in srcs]
                src1 = to_dev(one)
                dst1 = torch.zeros_like(src1)
                ws = hzd.alloc_workspace(hzd.workspace_size(P(), shapes, params))
                ws1 = hzd.alloc_workspace(hzd.workspace_size(p1, [one.shape[:2]]))
            stream.synchronize()
            start.wait(timeout=60)
            for rep in range(reps):
                with torch.cuda.stream(stream):
                    for d in dsts + [dst1]:
                        d.zero_()
                hzd.dehaze_batch(srcs, dsts, P(), per_frame_params=params, workspace=ws, stream=stream)
                hzd.dehaze_frame(src1, dst1, p1, workspace=ws1, stream=stream)
                stream.synchronize()
                for i in range(len(frames)):
                    if not np.array_equal(dsts[i].cpu().numpy(), refs[t][0][i]):
                        errors.append(f"thread {t} rep {rep} batch frame {i}")
                if not np.array_equal(dst1.cpu().numpy(), refs[t][1]):
                    errors.append(f"thread {t} rep {rep} frame call")
        except Exception as e:  # reported by the main thread
            errors.append(f"thread {t}: {e!r}")
            start.abort()   # the others stop waiting at the start line

    try:
        hzd.graph_cache(cache)
        threads = [threading.Thread(target=worker, args=(t,), daemon=True) for t in range(T)]
        for th in threads:
            th.start()
        for th in threads:
            th.join(timeout=120)
        assert not any(th.is_alive() for th in threads), "a worker thread did not finish"
    finally:
        hzd.graph_cache(0)
    assert not errors, errors[:10]


def test_threads_submit_to_one_server():
    # three client threads, two streams each (a real-time and an offline size), submitting and
    # waiting at the same time; each served frame equals its frame-call result
    T, nf = 3, 8
    specs = []
    for t in range(T):
        rng = np.random.default_rng(120 + t)
        pa, pb = P(), P(mode=hzd.MODE_OFFLINE, gf_radius=7 + t, color_balance=1)
        fa = [rng.integers(0, 256, size=(120, 160, 3), dtype=np.uint8) for _ in range(nf)]
        fb = [rng.integers(0, 256, size=(80 + 8 * t, 96, 3), dtype=np.uint8) for _ in range(nf)]
        specs.append([(pa, fa), (pb, fb)])
    refs = [[[run_gpu(I, p, with_J=False)["out"] for I in fs] for (p, fs) in sp] for sp in specs]
    arena = sum(hzd.stream_arena_size(p, fs[0].shape[1], fs[0].shape[0]) for sp in specs for (p, fs) in sp)
    srv = hzd.Server(arena_bytes=arena + 4096, max_inflight=16, frames_per_launch=8, hip_streams=4)
    sts = [[srv.open(p, fs[0].shape[1], fs[0].shape[0]) for (p, fs) in sp] for sp in specs]
    errors = []
    start = threading.Barrier(T)

    def client(t):
        try:
            bufs = [([to_dev(I) for I in fs], [torch.zeros((I.shape[0], I.shape[1], 3), dtype=torch.uint8,
                                                         device="cuda") for I in fs]) for (_, fs) in specs[t]]
            torch.cuda.synchronize()
            start.wait(timeout=60)
            tickets = []
            for k in range(nf):
                for s, (srcs, dsts) in enumerate(bufs):
                    tickets.append((s, k, sts[t][s].submit(srcs[k], dsts[k])))
            for s, k, tk in tickets:
                rc, _ = sts[t][s].wait(tk, timeout_ns=60_000_000_000)
                if rc != 0:
                    errors.append(f"client {t} stream {s} frame {k}: status {rc}")
                elif not np.array_equal(bufs[s][1][k].cpu().numpy(), refs[t][s][k]):
                    errors.append(f"client {t} stream {s} frame {k}: differs from the frame call")
        except Exception as e:  # reported by the main thread
            errors.append(f"client {t}: {e!r}")
            start.abort()

    try:
        threads = [threading.Thread(target=client, args=(t,), daemon=True) for t in range(T)]
        for th in threads:
            th.start()
        for th in threads:
            th.join(timeout=120)
        assert not any(th.is_alive() for th in threads), "a client thread did not finish"
        assert srv.stats()["completed"] == T * 2 * nf
    finally:
        for row in sts:
            for st in row:
                st.close()
        srv.close()
    assert not errors, errors[:10]
