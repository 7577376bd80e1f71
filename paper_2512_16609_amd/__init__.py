"""Python binding of libhzd, the MI355X per-frame dark-channel-prior dehazing library.

Argument marshalling only: every step of the method runs in the library's
gfx950 kernels.  torch supplies device memory and HIP streams.  The names
follow the C ABI in include/hzd.h (hzd_dehaze_frame -> dehaze_frame, ...).

The library is loaded from this package directory (built in-tree by
build_lib.build()).  There is no fallback: if the library is missing or no
GPU is visible, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhzd.so")

HZD_OK, HZD_E_INVAL, HZD_E_NOMEM, HZD_E_DEVICE = 0, -1, -2, -3
HZD_E_AGAIN, HZD_E_CLOSED, HZD_E_UNSUPPORTED, HZD_E_TIMEOUT = -4, -5, -6, -7
MODE_REALTIME, MODE_OFFLINE = 0, 1
TX_HE, TX_PAPER = 0, 1
PREC_FP32, PREC_FP16 = 0, 1
PRESET_REALTIME, PRESET_OFFLINE, PRESET_PAPER_REALTIME = 0, 1, 2
ABI_VERSION = 4
NOALLOC_SCRATCH_BYTES = 64 << 20   # HZD_NOALLOC_SCRATCH_BYTES


class HzdError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str):
        super().__init__(f"{what}: status {status} ({detail})")
        self.status = status


class hzd_params(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("mode", ctypes.c_int32), ("patch", ctypes.c_int32),
                ("omega", ctypes.c_float), ("t0", ctypes.c_float), ("top_frac", ctypes.c_float),
                ("alpha", ctypes.c_float), ("gamma", ctypes.c_float), ("gf_radius", ctypes.c_int32),
                ("gf_eps", ctypes.c_float), ("color_balance", ctypes.c_int32), ("tx", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("resize_width", ctypes.c_int32),
                ("resize_height", ctypes.c_int32), ("airlight_smoothing", ctypes.c_float),
                ("gamma_adaptive", ctypes.c_int32), ("gamma_target", ctypes.c_float),
                ("wb_percentile", ctypes.c_float)]


class hzd_frame(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("src_pitch", ctypes.c_int64), ("dst", ctypes.c_void_p),
                ("dst_pitch", ctypes.c_int64), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("params", ctypes.POINTER(hzd_params)), ("airlight_state", ctypes.c_void_p)]


class hzd_frame_aux(ctypes.Structure):
    _fields_ = [("A_out", ctypes.c_void_p), ("sel_out", ctypes.c_void_p), ("dark_out", ctypes.c_void_p),
                ("t_out", ctypes.c_void_p), ("J_out", ctypes.c_void_p)]


class hzd_server_config(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint32), ("device", ctypes.c_int32), ("arena", ctypes.c_void_p),
                ("arena_bytes", ctypes.c_size_t), ("max_inflight", ctypes.c_int32),
                ("frames_per_launch", ctypes.c_int32), ("hip_streams", ctypes.c_int32)]


class hzd_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("arena_used", ctypes.c_uint64),
                ("arena_bytes", ctypes.c_uint64), ("open_streams", ctypes.c_int32),
                ("inflight", ctypes.c_int32)]


class hzd_tile_config(ctypes.Structure):
    _fields_ = [("gf_rows", ctypes.c_int32)]


class hzd_profile_entry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double)]


DONE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64)

_lib = None
_lib_lock = threading.Lock()

SYMBOLS = {
    "hzd_abi_version": (ctypes.c_int, []),
    "hzd_status_str": (ctypes.c_char_p, [ctypes.c_int32]),
    "hzd_last_error": (ctypes.c_char_p, []),
    "hzd_params_default": (ctypes.c_int, [ctypes.POINTER(hzd_params), ctypes.c_int32]),
    "hzd_workspace_size": (ctypes.c_int, [ctypes.POINTER(hzd_params), ctypes.POINTER(hzd_frame),
                                          ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "hzd_dehaze_frame": (ctypes.c_int, [ctypes.POINTER(hzd_params), ctypes.POINTER(hzd_frame),
                                        ctypes.POINTER(hzd_frame_aux), ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p]),
    "hzd_dehaze_frame_noalloc": (ctypes.c_int, [ctypes.POINTER(hzd_params), ctypes.POINTER(hzd_frame),
                                                ctypes.POINTER(hzd_frame_aux), ctypes.c_void_p]),
    "hzd_dehaze_batch": (ctypes.c_int, [ctypes.POINTER(hzd_params), ctypes.POINTER(hzd_frame),
                                        ctypes.c_int32, ctypes.POINTER(hzd_frame_aux), ctypes.c_void_p,
                                        ctypes.c_size_t, ctypes.c_void_p]),
    "hzd_server_create": (ctypes.c_int, [ctypes.POINTER(hzd_server_config), ctypes.POINTER(ctypes.c_void_p)]),
    "hzd_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "hzd_stream_open": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(hzd_params), ctypes.c_int32,
                                       ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "hzd_stream_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(hzd_frame), ctypes.c_void_p, DONE_FN,
                                         ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "hzd_stream_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64,
                                       ctypes.POINTER(ctypes.c_int64)]),
    "hzd_stream_arena_size": (ctypes.c_int, [ctypes.POINTER(hzd_params), ctypes.c_int32, ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_size_t)]),
    "hzd_stream_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "hzd_stream_close": (ctypes.c_int, [ctypes.c_void_p]),
    "hzd_server_stats_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(hzd_server_stats)]),
    "hzd_tile_config_set": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(hzd_tile_config)]),
    "hzd_tile_config_get": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(hzd_tile_config)]),
    "hzd_autotune": (ctypes.c_int, [ctypes.POINTER(hzd_params), ctypes.POINTER(hzd_frame), ctypes.c_void_p,
                                    ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.POINTER(hzd_tile_config)]),
    "hzd_graph_cache": (ctypes.c_int, [ctypes.c_int32]),
    "hzd_profile_enable": (ctypes.c_int, [ctypes.c_int32]),
    "hzd_profile_read": (ctypes.c_int, [ctypes.POINTER(hzd_profile_entry), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]),
}


def lib():
    """Load libhzd.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is not built; run paper_2512_16609_amd.build_lib.build()")
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SYMBOLS.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            if L.hzd_abi_version() != ABI_VERSION:
                raise ImportError(f"{LIB_PATH} has ABI {L.hzd_abi_version()}, the binding expects "
                                  f"{ABI_VERSION}; rebuild it")
            _lib = L
    return _lib


def last_error() -> str:
    return lib().hzd_last_error().decode()


def _check(rc: int, what: str):
    if rc != HZD_OK:
        raise HzdError(rc, what, f"{lib().hzd_status_str(rc).decode()}: {last_error()}")
    return rc


# ------------------------------------------------------------------ params
@dataclass
class Params:
    mode: int = MODE_REALTIME
    patch: int = 15
    omega: float = 0.95
    t0: float = 0.1
    top_frac: float = 0.001
    alpha: float = 0.8
    gamma: float = 1.2
    gf_radius: int = 60
    gf_eps: float = 1e-3
    color_balance: int = 0    # 0 none, 1 gray-world, 2 percentile white balance
    tx: int = TX_HE
    precision: int = PREC_FP32
    resize_width: int = 0     # Sec. V step 1 working size; 0 x 0 = the frame's own size
    resize_height: int = 0
    airlight_smoothing: float = 0.0   # temporal airlight weight lam; needs an airlight state
    gamma_adaptive: int = 0   # 1: per-frame gamma mapping the mean luma of J to gamma_target
    gamma_target: float = 0.5
    wb_percentile: float = 0.02   # percentile white balance: fraction ignored at each end

    def c(self) -> hzd_params:
        return hzd_params(ctypes.sizeof(hzd_params), self.mode, self.patch, self.omega, self.t0,
                          self.top_frac, self.alpha, self.gamma, self.gf_radius, self.gf_eps,
                          int(self.color_balance), self.tx, self.precision, self.resize_width,
                          self.resize_height, self.airlight_smoothing, int(self.gamma_adaptive),
                          self.gamma_target, self.wb_percentile)

    def output_shape(self, h: int, w: int) -> tuple:
        """(height, width) of the output of a frame of input shape (h, w)."""
        if self.resize_width or self.resize_height:
            return (self.resize_height, self.resize_width)
        return (h, w)

    @staticmethod
    def preset(preset: int) -> "Params":
        p = hzd_params()
        _check(lib().hzd_params_default(ctypes.byref(p), preset), "hzd_params_default")
        return Params(p.mode, p.patch, p.omega, p.t0, p.top_frac, p.alpha, p.gamma, p.gf_radius,
                      p.gf_eps, p.color_balance, p.tx, p.precision, p.resize_width, p.resize_height,
                      p.airlight_smoothing, p.gamma_adaptive, p.gamma_target, p.wb_percentile)


# ------------------------------------------------------------------ frames
def _frame_struct(src: torch.Tensor, dst: torch.Tensor, params: "Params", params_ptr=None,
                  airlight_state: torch.Tensor | None = None) -> hzd_frame:
    for name, t in (("src", src), ("dst", dst)):
        if t.dtype != torch.uint8 or t.dim() != 3 or t.shape[2] != 3:
            raise ValueError(f"{name} must be a uint8 (H, W, 3) tensor")
        if not t.is_cuda:
            raise ValueError(f"{name} must be on the GPU")
        if t.stride(2) != 1 or t.stride(1) != 3:
            raise ValueError(f"{name} must have packed RGB rows (strides (pitch, 3, 1))")
    h, w = int(src.shape[0]), int(src.shape[1])
    ho, wo = params.output_shape(h, w)
    if tuple(dst.shape[:2]) != (ho, wo):
        raise ValueError(f"dst shape {tuple(dst.shape[:2])} != output shape {(ho, wo)}")
    if airlight_state is not None and (not airlight_state.is_cuda or airlight_state.numel() * airlight_state.element_size() < 16):
        raise ValueError("airlight_state must be a device tensor of at least 16 bytes")
    f = hzd_frame(src.data_ptr(), src.stride(0) if h > 1 else 3 * w, dst.data_ptr(),
                  dst.stride(0) if ho > 1 else 3 * wo, w, h, params_ptr,
                  None if airlight_state is None else airlight_state.data_ptr())
    return f


def make_airlight_state(device="cuda") -> torch.Tensor:
    """A zeroed 16-byte airlight state {A[3], frames} for one stream of frame calls."""
    return torch.zeros(4, dtype=torch.float32, device=device)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _aux_struct(aux: dict | None) -> hzd_frame_aux | None:
    if not aux:
        return None
    return hzd_frame_aux(_ptr(aux.get("A")), _ptr(aux.get("sel")), _ptr(aux.get("dark")),
                         _ptr(aux.get("t")), _ptr(aux.get("J")))


def make_aux(h: int, w: int, device="cuda", J: bool = True) -> dict:
    """Device buffers for every optional per-frame output."""
    d = {"A": torch.zeros(3, dtype=torch.float32, device=device),
         "sel": torch.zeros(4, dtype=torch.int32, device=device),   # K, vstar, cutoff, status
         "dark": torch.zeros((h, w), dtype=torch.uint8, device=device),
         "t": torch.zeros((h, w), dtype=torch.float32, device=device)}
    if J:
        d["J"] = torch.zeros((h, w, 3), dtype=torch.float32, device=device)
    return d


def workspace_size(params: Params, shapes, per_frame_params=None) -> int:
    """Workspace bytes for frames of the given (height, width) shapes."""
    n = len(shapes)
    pcs = [p.c() for p in per_frame_params] if per_frame_params else None
    arr = (hzd_frame * n)()
    for i, (h, w) in enumerate(shapes):
        arr[i].width, arr[i].height = int(w), int(h)
        if pcs:
            arr[i].params = ctypes.pointer(pcs[i])
    out = ctypes.c_size_t(0)
    pc = params.c()
    _check(lib().hzd_workspace_size(ctypes.byref(pc), arr, n, ctypes.byref(out)), "hzd_workspace_size")
    return int(out.value)


def alloc_workspace(nbytes: int, device="cuda") -> torch.Tensor:
    # torch's caching allocator returns 512-byte aligned blocks
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
    assert ws.data_ptr() % 256 == 0
    return ws


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def dehaze_frame(src: torch.Tensor, dst: torch.Tensor, params: Params, aux: dict | None = None,
                 workspace: torch.Tensor | None = None, stream=None,
                 airlight_state: torch.Tensor | None = None) -> None:
    """hzd_dehaze_frame on a (H, W, 3) uint8 device tensor (asynchronous, stream-ordered);
    dst has the output shape params.output_shape(H, W).  airlight_state: the stream's
    state from make_airlight_state(), needed with params.airlight_smoothing > 0."""
    f = _frame_struct(src, dst, params, airlight_state=airlight_state)
    pc = params.c()
    if workspace is None:
        workspace = alloc_workspace(workspace_size(params, [(src.shape[0], src.shape[1])]), src.device)
    a = _aux_struct(aux)
    rc = lib().hzd_dehaze_frame(ctypes.byref(pc), ctypes.byref(f), ctypes.byref(a) if a else None,
                                workspace.data_ptr(), workspace.numel(), _stream_handle(stream))
    _check(rc, "hzd_dehaze_frame")


def dehaze_frame_noalloc(src: torch.Tensor, dst: torch.Tensor, params: Params, aux: dict | None = None,
                         stream=None, airlight_state: torch.Tensor | None = None) -> None:
    """hzd_dehaze_frame_noalloc: as dehaze_frame, with the workspace taken from the library's
    static device scratch (NOALLOC_SCRATCH_BYTES per device) instead of a caller buffer.
    Calls that overlap on one device race on that scratch."""
    f = _frame_struct(src, dst, params, airlight_state=airlight_state)
    pc = params.c()
    a = _aux_struct(aux)
    rc = lib().hzd_dehaze_frame_noalloc(ctypes.byref(pc), ctypes.byref(f), ctypes.byref(a) if a else None,
                                        _stream_handle(stream))
    _check(rc, "hzd_dehaze_frame_noalloc")


def dehaze_batch(srcs, dsts, params: Params, per_frame_params=None, auxs=None,
                 workspace: torch.Tensor | None = None, stream=None, airlight_states=None) -> None:
    """hzd_dehaze_batch over lists of (H_i, W_i, 3) uint8 device tensors; airlight_states: None or
    a list with a state tensor (or None) per frame."""
    n = len(srcs)
    pcs = [p.c() for p in per_frame_params] if per_frame_params else None
    arr = (hzd_frame * n)()
    for i in range(n):
        pi = per_frame_params[i] if per_frame_params else params
        arr[i] = _frame_struct(srcs[i], dsts[i], pi, ctypes.pointer(pcs[i]) if pcs else None,
                               airlight_states[i] if airlight_states else None)
    aarr = None
    if auxs is not None:
        aarr = (hzd_frame_aux * n)()
        for i in range(n):
            s = _aux_struct(auxs[i])
            if s is not None:
                aarr[i] = s
    pc = params.c()
    if workspace is None:
        shapes = [(s.shape[0], s.shape[1]) for s in srcs]
        workspace = alloc_workspace(workspace_size(params, shapes, per_frame_params), srcs[0].device)
    rc = lib().hzd_dehaze_batch(ctypes.byref(pc), arr, n, aarr, workspace.data_ptr(), workspace.numel(),
                                _stream_handle(stream))
    _check(rc, "hzd_dehaze_batch")


# ------------------------------------------------------------------ server
def stream_arena_size(params: Params, width: int, height: int) -> int:
    """hzd_stream_arena_size: arena bytes one opened stream reserves."""
    out = ctypes.c_size_t(0)
    pc = params.c()
    _check(lib().hzd_stream_arena_size(ctypes.byref(pc), width, height, ctypes.byref(out)),
           "hzd_stream_arena_size")
    return int(out.value)


class Server:
    """hzd_server_*: continuous batching of many frame streams on one GPU."""

    def __init__(self, arena_bytes: int, device: int = 0, max_inflight: int = 16,
                 frames_per_launch: int = 8, hip_streams: int = 4):
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=f"cuda:{device}")
        cfg = hzd_server_config(ctypes.sizeof(hzd_server_config), device, self.arena.data_ptr(), arena_bytes,
                                max_inflight, frames_per_launch, hip_streams)
        h = ctypes.c_void_p()
        _check(lib().hzd_server_create(ctypes.byref(cfg), ctypes.byref(h)), "hzd_server_create")
        self.handle = h

    def open(self, params: Params, width: int, height: int) -> "Stream":
        h = ctypes.c_void_p()
        pc = params.c()
        _check(lib().hzd_stream_open(self.handle, ctypes.byref(pc), width, height, ctypes.byref(h)),
               "hzd_stream_open")
        return Stream(self, h, width, height, params)

    def stats(self) -> dict:
        s = hzd_server_stats()
        _check(lib().hzd_server_stats_get(self.handle, ctypes.byref(s)), "hzd_server_stats_get")
        return {k: getattr(s, k) for k, _ in hzd_server_stats._fields_}

    def close(self):
        if self.handle:
            _check(lib().hzd_server_destroy(self.handle), "hzd_server_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Stream:
    def __init__(self, server: Server, handle, width, height, params: Params):
        self.server, self.handle, self.width, self.height = server, handle, width, height
        self.params = params

    def submit(self, src: torch.Tensor, dst: torch.Tensor, stream=None) -> int:
        """Queue one frame; no completion callback (completion and latency come from wait()).
        The frame is ordered after the work enqueued so far on `stream` (default: torch's
        current stream), which produced src and last used dst."""
        f = _frame_struct(src, dst, self.params)
        t = ctypes.c_uint64(0)
        rc = lib().hzd_stream_submit(self.handle, ctypes.byref(f), _stream_handle(stream), DONE_FN(), None,
                                     ctypes.byref(t))
        _check(rc, "hzd_stream_submit")
        return int(t.value)

    def wait(self, ticket: int, timeout_ns: int = -1):
        """(status, latency_ns) of a submitted frame; status HZD_E_TIMEOUT if not done in time."""
        lat = ctypes.c_int64(0)
        rc = lib().hzd_stream_wait(self.handle, ticket, timeout_ns, ctypes.byref(lat))
        return int(rc), int(lat.value)

    def state(self):
        """(A, [K, vstar, cutoff, status]) of the stream's last completed frame."""
        A = (ctypes.c_float * 3)()
        sel = (ctypes.c_int32 * 4)()
        _check(lib().hzd_stream_state(self.handle, A, sel), "hzd_stream_state")
        return list(A), list(sel)

    def close(self):
        if self.handle:
            _check(lib().hzd_stream_close(self.handle), "hzd_stream_close")
            self.handle = None


# ---------------------------------------------------------------- profiling
def profile_enable(on: bool = True) -> None:
    """hzd_profile_enable: bracket every kernel launch with HIP events on its stream."""
    _check(lib().hzd_profile_enable(1 if on else 0), "hzd_profile_enable")


def profile_read(reset: bool = True) -> dict:
    """hzd_profile_read: {stage: (launches, total_ms)} for the launches recorded so far."""
    cap = 32
    arr = (hzd_profile_entry * cap)()
    n = ctypes.c_int32(0)
    _check(lib().hzd_profile_read(arr, cap, ctypes.byref(n), 1 if reset else 0), "hzd_profile_read")
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(n.value)}


class FrameCall:
    """A prepared hzd_dehaze_frame call: ctypes arguments built once, so a
    timing loop measures the library and the GPU, not argument marshalling."""

    def __init__(self, src, dst, params: Params, workspace, aux: dict | None = None, stream=None,
                 airlight_state=None):
        self._keep = (src, dst, workspace, aux, airlight_state)
        self.f = _frame_struct(src, dst, params, airlight_state=airlight_state)
        self.pc = params.c()
        a = _aux_struct(aux)
        self.aux = ctypes.pointer(a) if a is not None else None
        self.ws = ctypes.c_void_p(workspace.data_ptr())
        self.ws_bytes = ctypes.c_size_t(workspace.numel())
        self.stream = ctypes.c_void_p(_stream_handle(stream))
        self.fn = lib().hzd_dehaze_frame
        self.fp = ctypes.byref(self.f)
        self.pp = ctypes.byref(self.pc)

    def __call__(self):
        rc = self.fn(self.pp, self.fp, self.aux, self.ws, self.ws_bytes, self.stream)
        if rc != HZD_OK:
            _check(rc, "hzd_dehaze_frame")


# ------------------------------------------------------------------- tuning
def tile_config_set(width: int, height: int, gf_rows: int | None) -> None:
    """hzd_tile_config_set; gf_rows None removes the entry."""
    c = hzd_tile_config(gf_rows) if gf_rows is not None else None
    _check(lib().hzd_tile_config_set(width, height, ctypes.byref(c) if c is not None else None),
           "hzd_tile_config_set")


def tile_config_get(width: int, height: int) -> int:
    c = hzd_tile_config()
    _check(lib().hzd_tile_config_get(width, height, ctypes.byref(c)), "hzd_tile_config_get")
    return int(c.gf_rows)


def autotune(src, dst, params: Params, workspace=None, reps: int = 20, stream=None, airlight_state=None) -> int:
    """hzd_autotune on one frame; returns the chosen gf_rows (now in the table)."""
    f = _frame_struct(src, dst, params, airlight_state=airlight_state)
    pc = params.c()
    if workspace is None:
        workspace = alloc_workspace(workspace_size(params, [(src.shape[0], src.shape[1])]), src.device)
    best = hzd_tile_config()
    _check(lib().hzd_autotune(ctypes.byref(pc), ctypes.byref(f), workspace.data_ptr(), workspace.numel(),
                              _stream_handle(stream), reps, ctypes.byref(best)), "hzd_autotune")
    return int(best.gf_rows)


def graph_cache(capacity: int) -> None:
    """hzd_graph_cache: replay captured HIP graphs for repeated launch arguments (0 = off)."""
    _check(lib().hzd_graph_cache(capacity), "hzd_graph_cache")
