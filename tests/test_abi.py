"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/hzd.h declares, and rejects bad arguments before
any device work."""
import ctypes
import os
import re

import pytest

import paper_2512_16609_amd as hzd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hzd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(hzd_[a-z_]+)\s*\(", text))
    return sorted(n for n in names if not n.endswith("_fn"))


@pytest.fixture(scope="module")
def L():
    return hzd.lib()


def test_library_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(hzd.SYMBOLS), "binding and header disagree"
    assert L.hzd_abi_version() == hzd.ABI_VERSION == 4


def test_struct_sizes_match_header():
    assert ctypes.sizeof(hzd.hzd_params) == 4 * 19
    assert ctypes.sizeof(hzd.hzd_frame) == 8 + 8 + 8 + 8 + 4 + 4 + 8 + 8
    assert ctypes.sizeof(hzd.hzd_frame_aux) == 5 * 8


def test_presets(L):
    p = hzd.Params.preset(hzd.PRESET_REALTIME)
    assert (p.mode, p.patch, p.tx, p.color_balance) == (hzd.MODE_REALTIME, 15, hzd.TX_HE, 0)
    assert abs(p.omega - 0.95) < 1e-7 and abs(p.t0 - 0.1) < 1e-7 and abs(p.alpha - 0.8) < 1e-7
    q = hzd.Params.preset(hzd.PRESET_OFFLINE)
    assert (q.mode, q.gf_radius, q.color_balance) == (hzd.MODE_OFFLINE, 60, 1)
    r = hzd.Params.preset(hzd.PRESET_PAPER_REALTIME)
    assert r.tx == hzd.TX_PAPER and abs(r.omega - 0.5) < 1e-7 and abs(r.t0 - 0.05) < 1e-7
    with pytest.raises(hzd.HzdError):
        hzd.Params.preset(7)


FAKE_SRC = 0x10000000
FAKE_DST = 0x20000000


def call_frame(L, p: hzd.Params, w=64, h=48, src=FAKE_SRC, dst=FAKE_DST, sp=None, dp=None,
               ws=0x40000000, ws_bytes=1 << 40, size=None):
    pc = p.c()
    if size is not None:
        pc.size = size
    f = hzd.hzd_frame(src, sp if sp is not None else 3 * w, dst, dp if dp is not None else 3 * w, w, h, None)
    return L.hzd_dehaze_frame(ctypes.byref(pc), ctypes.byref(f), None, ws, ws_bytes, None)


@pytest.mark.parametrize("field,value,status", [
    ("patch", 14, hzd.HZD_E_INVAL), ("patch", 0, hzd.HZD_E_INVAL), ("patch", 33, hzd.HZD_E_UNSUPPORTED),
    ("omega", -0.1, hzd.HZD_E_INVAL), ("omega", 1.5, hzd.HZD_E_INVAL), ("omega", float("nan"), hzd.HZD_E_INVAL),
    ("t0", 0.0, hzd.HZD_E_INVAL), ("t0", 1.5, hzd.HZD_E_INVAL), ("top_frac", 0.0, hzd.HZD_E_INVAL),
    ("top_frac", 1.01, hzd.HZD_E_INVAL), ("alpha", 0.0, hzd.HZD_E_INVAL), ("gamma", 0.0, hzd.HZD_E_INVAL),
    ("mode", 3, hzd.HZD_E_INVAL), ("tx", 2, hzd.HZD_E_INVAL), ("precision", 5, hzd.HZD_E_INVAL),
    ("color_balance", 3, hzd.HZD_E_INVAL),
    ("color_balance", -1, hzd.HZD_E_INVAL),
])
def test_param_validation(L, field, value, status):
    p = hzd.Params()
    setattr(p, field, value)
    assert call_frame(L, p) == status
    assert hzd.last_error() != ""


def test_offline_param_validation(L):
    p = hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=0)
    assert call_frame(L, p) == hzd.HZD_E_INVAL
    p = hzd.Params(mode=hzd.MODE_OFFLINE, gf_radius=65)
    assert call_frame(L, p) == hzd.HZD_E_UNSUPPORTED
    p = hzd.Params(mode=hzd.MODE_OFFLINE, gf_eps=0.0)
    assert call_frame(L, p) == hzd.HZD_E_INVAL


def test_frame_validation(L):
    p = hzd.Params()
    assert call_frame(L, p, size=12) == hzd.HZD_E_INVAL                 # struct size mismatch
    assert call_frame(L, p, w=0) == hzd.HZD_E_INVAL
    assert call_frame(L, p, h=-3) == hzd.HZD_E_INVAL
    assert call_frame(L, p, w=65536, h=32768) == hzd.HZD_E_INVAL        # W*H >= 2^31
    assert call_frame(L, p, w=1 << 24, h=1) == hzd.HZD_E_UNSUPPORTED    # a row's sums must fit 32 bits
    assert call_frame(L, p, sp=100) == hzd.HZD_E_INVAL                  # pitch < 3W
    assert call_frame(L, p, src=0) == hzd.HZD_E_INVAL                   # NULL src
    assert call_frame(L, p, dst=FAKE_SRC + 100) == hzd.HZD_E_INVAL      # overlap
    assert call_frame(L, p, ws=0) == hzd.HZD_E_INVAL
    assert call_frame(L, p, ws=0x40000010) == hzd.HZD_E_INVAL           # misaligned workspace
    assert call_frame(L, p, ws_bytes=1000) == hzd.HZD_E_NOMEM
    assert L.hzd_dehaze_frame(None, None, None, None, 0, None) == hzd.HZD_E_INVAL
    pc = p.c()
    assert L.hzd_dehaze_batch(ctypes.byref(pc), None, 0, None, None, 0, None) == hzd.HZD_E_INVAL


def test_percentile_balance_validation(L):
    assert call_frame(L, hzd.Params(color_balance=2, wb_percentile=0.5)) == hzd.HZD_E_INVAL
    assert call_frame(L, hzd.Params(color_balance=2, wb_percentile=-0.01)) == hzd.HZD_E_INVAL
    # offline with a binary16 t map would move the codes the percentiles are taken on
    assert call_frame(L, hzd.Params(mode=hzd.MODE_OFFLINE, color_balance=2,
                                    precision=hzd.PREC_FP16)) == hzd.HZD_E_UNSUPPORTED
    assert "FP32" in hzd.last_error()
    # the percentile range is checked only when the balance uses it
    assert call_frame(L, hzd.Params(color_balance=1, wb_percentile=0.9), ws_bytes=10) == hzd.HZD_E_NOMEM
    assert hzd.Params.preset(hzd.PRESET_REALTIME).wb_percentile == pytest.approx(0.02)


def test_noalloc_rejects_before_device_work(L):
    """hzd_dehaze_frame_noalloc validates and checks the static scratch size before any HIP
    call, so on a machine without a GPU every rejection is observable."""
    assert L.hzd_dehaze_frame_noalloc(None, None, None, None) == hzd.HZD_E_INVAL
    pc = hzd.Params().c()
    f = hzd.hzd_frame(FAKE_SRC, 0, FAKE_DST, 192, 64, 48, None, None)      # pitch < 3W
    assert L.hzd_dehaze_frame_noalloc(ctypes.byref(pc), ctypes.byref(f), None, None) == hzd.HZD_E_INVAL
    # a 3840x2160 offline frame needs more workspace than the static scratch holds
    po = hzd.Params(mode=hzd.MODE_OFFLINE, color_balance=1)
    assert hzd.workspace_size(po, [(2160, 3840)]) > hzd.NOALLOC_SCRATCH_BYTES
    assert hzd.workspace_size(po, [(1080, 1920)]) <= hzd.NOALLOC_SCRATCH_BYTES
    # int64 a, b (small eps and t0) double the a, b map: a 1080p offline frame no longer fits
    p64 = hzd.Params(mode=hzd.MODE_OFFLINE, color_balance=1, gf_eps=1e-8, t0=0.01)
    assert hzd.workspace_size(p64, [(1080, 1920)]) > hzd.NOALLOC_SCRATCH_BYTES
    pc64 = p64.c()
    f64 = hzd.hzd_frame(FAKE_SRC, 3 * 1920, FAKE_DST, 3 * 1920, 1920, 1080, None, None)
    assert L.hzd_dehaze_frame_noalloc(ctypes.byref(pc64), ctypes.byref(f64), None, None) == hzd.HZD_E_NOMEM
    pc = po.c()
    f = hzd.hzd_frame(FAKE_SRC, 3 * 3840, FAKE_DST, 3 * 3840, 3840, 2160, None, None)
    assert L.hzd_dehaze_frame_noalloc(ctypes.byref(pc), ctypes.byref(f), None, None) == hzd.HZD_E_NOMEM
    assert "static scratch" in hzd.last_error()


def test_resize_validation(L):
    for rw, rh in [(640, 0), (0, 480), (-1, 480), (16385, 10), (10, 16385)]:
        assert call_frame(L, hzd.Params(resize_width=rw, resize_height=rh)) == hzd.HZD_E_INVAL, (rw, rh)
    p = hzd.Params(resize_width=640, resize_height=480)
    # input sides beyond 32768 are not supported when resizing
    assert call_frame(L, p, w=32769, h=2, dp=3 * 640) == hzd.HZD_E_UNSUPPORTED
    # dst pitch and the src/dst overlap are checked at the output size
    assert call_frame(L, p, w=64, h=48, dp=3 * 64) == hzd.HZD_E_INVAL
    assert call_frame(L, p, w=64, h=48, dp=3 * 640, dst=FAKE_SRC - 100000) == hzd.HZD_E_INVAL
    assert call_frame(L, p, w=64, h=48, dp=3 * 640, ws_bytes=1000) == hzd.HZD_E_NOMEM


def test_adaptive_gamma_validation(L):
    for flag, tau in [(2, 0.5), (-1, 0.5), (1, 0.0), (1, 1.0), (1, float("nan"))]:
        assert call_frame(L, hzd.Params(gamma_adaptive=flag, gamma_target=tau)) == hzd.HZD_E_INVAL, (flag, tau)
    # the target is only checked when the adaptive rule is on
    off = hzd.Params(mode=hzd.MODE_OFFLINE, gamma_adaptive=1)
    assert hzd.workspace_size(off, [(480, 640)]) == hzd.workspace_size(
        hzd.Params(mode=hzd.MODE_OFFLINE, color_balance=1), [(480, 640)])   # both store the t map


def test_airlight_smoothing_validation(L):
    for lam in (-0.1, 1.0, float("nan")):
        assert call_frame(L, hzd.Params(airlight_smoothing=lam)) == hzd.HZD_E_INVAL, lam
    # smoothing needs the stream's state; the state must be 16-byte aligned
    assert call_frame(L, hzd.Params(airlight_smoothing=0.5)) == hzd.HZD_E_INVAL
    p = hzd.Params(airlight_smoothing=0.5)
    pc = p.c()
    f = hzd.hzd_frame(FAKE_SRC, 192, FAKE_DST, 192, 64, 48, None, 0x30000008)
    assert L.hzd_dehaze_frame(ctypes.byref(pc), ctypes.byref(f), None, 0x40000000, 1 << 40, None) == hzd.HZD_E_INVAL
    # two frames of one call may not share a state
    arr = (hzd.hzd_frame * 2)()
    arr[0] = hzd.hzd_frame(FAKE_SRC, 192, FAKE_DST, 192, 64, 48, None, 0x30000000)
    arr[1] = hzd.hzd_frame(FAKE_SRC + (1 << 20), 192, FAKE_DST + (1 << 20), 192, 64, 48, None, 0x30000000)
    assert L.hzd_dehaze_batch(ctypes.byref(pc), arr, 2, None, 0x40000000, 1 << 40, None) == hzd.HZD_E_INVAL
    assert "share" in hzd.last_error()


def test_stream_arena_size(L):
    for p, (w, h) in [(hzd.Params(), (320, 240)), (hzd.Params(mode=hzd.MODE_OFFLINE, color_balance=1), (640, 480)),
                      (hzd.Params(resize_width=64, resize_height=48), (1920, 1080))]:
        n = hzd.stream_arena_size(p, w, h)
        ws = hzd.workspace_size(p, [(h, w)])
        assert n % 256 == 0 and n >= 2 * ws + 3 * 256


def test_workspace_size_with_resize(L):
    # every map at the output size, plus the resized copy of the input (pitch 1920, 480 rows)
    rs = hzd.workspace_size(hzd.Params(resize_width=640, resize_height=480), [(1080, 1920)])
    assert rs == hzd.workspace_size(hzd.Params(), [(480, 640)]) + 480 * 1920
    off = hzd.Params(mode=hzd.MODE_OFFLINE, color_balance=1, resize_width=640, resize_height=480)
    assert hzd.workspace_size(off, [(2160, 3840)]) == hzd.workspace_size(
        hzd.Params(mode=hzd.MODE_OFFLINE, color_balance=1), [(480, 640)]) + 480 * 1920


def test_workspace_size_grows_with_mode(L):
    rt = hzd.workspace_size(hzd.Params(), [(1080, 1920)])
    off = hzd.workspace_size(hzd.Params(mode=hzd.MODE_OFFLINE, color_balance=1), [(1080, 1920)])
    assert rt > 1920 * 1080 * 4      # D + E + state
    assert off > rt + 1920 * 1080 * 16
    two = hzd.workspace_size(hzd.Params(), [(1080, 1920), (480, 640)])
    assert two == rt + hzd.workspace_size(hzd.Params(), [(480, 640)])


def test_status_strings(L):
    for s in range(-7, 1):
        assert L.hzd_status_str(s).decode() != "unknown status"
    assert L.hzd_status_str(-99).decode() == "unknown status"


def test_server_create_rejects_bad_config(L):
    cfg = hzd.hzd_server_config(ctypes.sizeof(hzd.hzd_server_config), 0, 0x40000000, 1 << 20, 0, 4, 2)
    h = ctypes.c_void_p()
    assert L.hzd_server_create(ctypes.byref(cfg), ctypes.byref(h)) == hzd.HZD_E_INVAL   # max_inflight 0
    cfg.max_inflight = 4
    cfg.frames_per_launch = 17
    assert L.hzd_server_create(ctypes.byref(cfg), ctypes.byref(h)) == hzd.HZD_E_INVAL
    cfg.frames_per_launch = 4
    cfg.arena = 0x40000010
    assert L.hzd_server_create(ctypes.byref(cfg), ctypes.byref(h)) == hzd.HZD_E_INVAL
    cfg.size = 8
    assert L.hzd_server_create(ctypes.byref(cfg), ctypes.byref(h)) == hzd.HZD_E_INVAL


def test_tile_config_table(L):
    assert hzd.tile_config_get(1920, 1080) == 16          # built-in default
    hzd.tile_config_set(0, 0, 16)                         # new default
    assert hzd.tile_config_get(1920, 1080) == 16
    hzd.tile_config_set(1920, 1080, 64)                   # size-specific entry wins
    assert hzd.tile_config_get(1920, 1080) == 64 and hzd.tile_config_get(640, 480) == 16
    hzd.tile_config_set(1920, 1080, None)
    hzd.tile_config_set(0, 0, None)
    assert hzd.tile_config_get(1920, 1080) == 16
    for bad in (0, 7, 12, 257, 264):
        with pytest.raises(hzd.HzdError):
            hzd.tile_config_set(640, 480, bad)
    with pytest.raises(hzd.HzdError):
        hzd.tile_config_set(-1, 480, 16)


def test_autotune_cache_file_is_loaded(tmp_path):
    # HZD_AUTOTUNE_CACHE entries fill the tile table on its first use in a process; rows outside
    # the accepted range (multiples of 8 in 8..256) are skipped.  A fresh interpreter, since the
    # file is read once per process.
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    cache.write_text("640 480 32\n1280 720 12\n1920 1080 300\n0 0 24\n")
    code = ("import paper_2512_16609_amd as h; "
            "print(h.tile_config_get(640, 480), h.tile_config_get(1280, 720), h.tile_config_get(1920, 1080))")
    env = dict(os.environ, HZD_AUTOTUNE_CACHE=str(cache))
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert out.returncode == 0, out.stderr[-2000:]
    # 640x480 from its entry; the others fall back to the file's (0, 0) default of 24
    assert out.stdout.split() == ["32", "24", "24"]
