// C ABI of the dehazing library: argument validation, workspace planning and
// the per-group launch sequence of the per-frame pipeline (paper Sec. V).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "hzd.h"
#include "hzd_internal.h"
#include "hzd_plan.h"

namespace hzd {

static thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

void clear_error() { g_last_error.clear(); }

static bool in_range(float v, float lo, float hi) { return v >= lo && v <= hi; }

int validate_params(const hzd_params* p) {
  if (!p) return fail(HZD_E_INVAL, "params is NULL");
  if (p->size != sizeof(hzd_params))
    return fail(HZD_E_INVAL, "params->size %u != sizeof(hzd_params) %zu", p->size, sizeof(hzd_params));
  if (p->mode != HZD_MODE_REALTIME && p->mode != HZD_MODE_OFFLINE)
    return fail(HZD_E_INVAL, "mode %d unknown", p->mode);
  if (p->patch < 1 || p->patch % 2 == 0) return fail(HZD_E_INVAL, "patch %d must be odd and >= 1", p->patch);
  if (p->patch > 2 * kMaxHalfPatch + 1)
    return fail(HZD_E_UNSUPPORTED, "patch %d > %d", p->patch, 2 * kMaxHalfPatch + 1);
  if (!in_range(p->omega, 0.0f, 1.0f)) return fail(HZD_E_INVAL, "omega %g outside [0,1]", p->omega);
  if (!(p->t0 > 0.0f && p->t0 <= 1.0f)) return fail(HZD_E_INVAL, "t0 %g outside (0,1]", p->t0);
  if (!(p->top_frac > 0.0f && p->top_frac <= 1.0f))
    return fail(HZD_E_INVAL, "top_frac %g outside (0,1]", p->top_frac);
  if (!(p->alpha > 0.0f && p->alpha <= 1.0f)) return fail(HZD_E_INVAL, "alpha %g outside (0,1]", p->alpha);
  if (!in_range(p->gamma, 0.1f, 10.0f)) return fail(HZD_E_INVAL, "gamma %g outside [0.1,10]", p->gamma);
  if (p->color_balance < 0 || p->color_balance > 2)
    return fail(HZD_E_INVAL, "color_balance %d must be 0, 1 or 2", p->color_balance);
  if (p->color_balance == 2) {
    if (!in_range(p->wb_percentile, 0.0f, 0.49f))
      return fail(HZD_E_INVAL, "wb_percentile %g outside [0,0.49]", p->wb_percentile);
  }
  if (p->tx != HZD_TX_HE && p->tx != HZD_TX_PAPER) return fail(HZD_E_INVAL, "tx %d unknown", p->tx);
  if (p->precision != HZD_PREC_FP32 && p->precision != HZD_PREC_FP16)
    return fail(HZD_E_INVAL, "precision %d unknown", p->precision);
  if (p->mode == HZD_MODE_OFFLINE) {
    if (p->gf_radius < 1) return fail(HZD_E_INVAL, "gf_radius %d < 1", p->gf_radius);
    if (p->gf_radius > kMaxRadius)
      return fail(HZD_E_UNSUPPORTED, "gf_radius %d > %d", p->gf_radius, kMaxRadius);
    if (!in_range(p->gf_eps, 1e-8f, 1.0f)) return fail(HZD_E_INVAL, "gf_eps %g outside [1e-8,1]", p->gf_eps);
    if (p->color_balance == 2 && p->precision == HZD_PREC_FP16)
      return fail(HZD_E_UNSUPPORTED, "the percentile white balance of offline mode needs FP32 precision");
  }
  if (p->gamma_adaptive != 0 && p->gamma_adaptive != 1)
    return fail(HZD_E_INVAL, "gamma_adaptive %d must be 0 or 1", p->gamma_adaptive);
  if (p->gamma_adaptive && !(p->gamma_target > 0.0f && p->gamma_target < 1.0f))
    return fail(HZD_E_INVAL, "gamma_target %g outside (0,1)", p->gamma_target);
  if (!(p->airlight_smoothing >= 0.0f && p->airlight_smoothing < 1.0f))
    return fail(HZD_E_INVAL, "airlight_smoothing %g outside [0,1)", p->airlight_smoothing);
  if (p->resize_width != 0 || p->resize_height != 0) {
    if (p->resize_width < 1 || p->resize_height < 1 || p->resize_width > kResizeMaxOut ||
        p->resize_height > kResizeMaxOut)
      return fail(HZD_E_INVAL, "resize %dx%d: both 0 or both in 1..%d", p->resize_width, p->resize_height,
                  kResizeMaxOut);
  }
  return HZD_OK;
}

void output_size(const hzd_params& p, int W, int H, int* Wo, int* Ho) {
  const bool rs = p.resize_width != 0;
  *Wo = rs ? p.resize_width : W;
  *Ho = rs ? p.resize_height : H;
}

int validate_size(const hzd_params& p, int W, int H, int idx) {
  if (W < 1 || H < 1) return fail(HZD_E_INVAL, "frame %d: size %dx%d", idx, W, H);
  if ((int64_t)W * (int64_t)H >= (int64_t(1) << 31))
    return fail(HZD_E_INVAL, "frame %d: width*height >= 2^31", idx);
  if (W > kMaxWidth) return fail(HZD_E_UNSUPPORTED, "frame %d: width %d beyond %d", idx, W, kMaxWidth);
  if (p.resize_width != 0 && (W > kResizeMaxIn || H > kResizeMaxIn))
    return fail(HZD_E_UNSUPPORTED, "frame %d: resize input %dx%d beyond %d per side", idx, W, H, kResizeMaxIn);
  return HZD_OK;
}

static bool ranges_overlap(const hzd_frame& f, int Wo, int Ho) {
  const uintptr_t s0 = (uintptr_t)f.src, d0 = (uintptr_t)f.dst;
  const uintptr_t s1 = s0 + (uintptr_t)((int64_t)(f.height - 1) * f.src_pitch + 3 * (int64_t)f.width);
  const uintptr_t d1 = d0 + (uintptr_t)((int64_t)(Ho - 1) * f.dst_pitch + 3 * (int64_t)Wo);
  return s0 < d1 && d0 < s1;
}

int validate_frame(const hzd_frame* f, const hzd_params& p, int idx) {
  if (!f) return fail(HZD_E_INVAL, "frame %d is NULL", idx);
  int rc = validate_size(p, f->width, f->height, idx);
  if (rc) return rc;
  int Wo, Ho;
  output_size(p, f->width, f->height, &Wo, &Ho);
  if (!f->src || !f->dst) return fail(HZD_E_INVAL, "frame %d: NULL pixel pointer", idx);
  if (f->src_pitch < 3 * (int64_t)f->width) return fail(HZD_E_INVAL, "frame %d: src_pitch < 3*width", idx);
  if (f->dst_pitch < 3 * (int64_t)Wo) return fail(HZD_E_INVAL, "frame %d: dst_pitch < 3*output width", idx);
  if (f->src_pitch >= (int64_t(1) << 40) || f->dst_pitch >= (int64_t(1) << 40))
    return fail(HZD_E_INVAL, "frame %d: pitch too large", idx);
  if (ranges_overlap(*f, Wo, Ho)) return fail(HZD_E_INVAL, "frame %d: src and dst overlap", idx);
  return HZD_OK;
}

static size_t a256(size_t v) { return (v + 255) & ~size_t(255); }
static int a16(int v) { return (v + 15) & ~15; }

AbFixed ab_fixed_point(float eps, float t0, int radius) {
  const double B = 1.0 + 0.25 / std::sqrt((double)eps);
  AbFixed f;
  f.bits = std::min(30, (int)std::floor(std::log2(2147483647.0 / B)));
  f.wide = std::ldexp(1.0, -f.bits) > 1e-6 * (double)t0;
  if (f.wide) {
    const double n = (2.0 * radius + 1.0) * (2.0 * radius + 1.0);
    f.bits = std::min(52, (int)std::floor(std::log2(9.2e18 / (B * n))));
  }
  return f;
}

GroupKey group_key(const hzd_params& p) {
  GroupKey g;
  g.mode = p.mode;
  g.half_patch = (p.patch - 1) / 2;
  g.tx = p.tx;
  g.cb = p.color_balance;
  g.fp16 = p.precision == HZD_PREC_FP16;
  g.radius = p.mode == HZD_MODE_OFFLINE ? p.gf_radius : 0;
  g.resize = p.resize_width != 0;
  g.gadapt = p.gamma_adaptive;
  g.ab64 = p.mode == HZD_MODE_OFFLINE ? (int)ab_fixed_point(p.gf_eps, p.t0, p.gf_radius).wide : 0;
  return g;
}

bool operator<(const GroupKey& a, const GroupKey& b) {
  return std::memcmp(&a, &b, sizeof(GroupKey)) < 0;
}

// W, H: the input size.  Every map is at the output size.
size_t frame_ws_bytes(const hzd_params& p, int Win, int Hin) {
  const bool offline = p.mode == HZD_MODE_OFFLINE;
  const bool needE = p.tx == HZD_TX_HE;
  int W, H;
  output_size(p, Win, Hin, &W, &H);
  size_t s = a256(sizeof(FrameState));
  if (p.resize_width != 0) s += a256((size_t)H * a16(3 * W));  // resized input
  s += a256((size_t)H * a16(W));                       // D
  if (needE) s += a256((size_t)H * a16(3 * W));        // E
  s += a256((size_t)H * sizeof(RowSel));               // per-row selection records
  if (select_one_fits(W, H)) s += a256((size_t)dark_tiles(W, H) * 256 * 2);   // per-tile histograms
  if (offline) {
    s += a256((size_t)W * H * 8);                      // LP
    s += a256((size_t)W * H * (ab_fixed_point(p.gf_eps, p.t0, p.gf_radius).wide ? 16 : 8));   // AB
    const size_t nch = (size_t)((H + 7) / 8);
    s += a256(nch * W * 16) + a256(nch * W * 16) + a256(nch * W * 16);  // 8-row chunk sums
    if (p.color_balance || p.gamma_adaptive) s += a256((size_t)W * H * (p.precision == HZD_PREC_FP16 ? 2 : 4));
  }
  return s;
}

// ------------------------------------------------------------ tile table
namespace {
std::mutex g_tune_mu;
std::map<std::pair<int, int>, hzd_tile_config> g_tune;
bool g_tune_loaded = false;

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("HZD_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* fp = std::fopen(path, "r");
  if (!fp) return;
  int w, h, rows;
  while (std::fscanf(fp, "%d %d %d", &w, &h, &rows) == 3) {
    if (w >= 0 && h >= 0 && rows >= kGfRowsMin && rows <= kGfRowsMax && rows % 8 == 0) g_tune[{w, h}] = hzd_tile_config{rows};
  }
  std::fclose(fp);
}

void tune_save(int w, int h, const hzd_tile_config& c) {
  const char* path = std::getenv("HZD_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* fp = std::fopen(path, "a");
  if (!fp) return;
  std::fprintf(fp, "%d %d %d\n", w, h, c.gf_rows);
  std::fclose(fp);
}
}  // namespace

hzd_tile_config tile_config_for(int W, int H, bool* from_table) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  auto it = g_tune.find({W, H});
  if (it == g_tune.end()) it = g_tune.find({0, 0});
  if (from_table) *from_table = it != g_tune.end();
  if (it != g_tune.end()) return it->second;
  return hzd_tile_config{kGfRowsDefault};
}

int device_cu_count() {
  static std::mutex mu;
  static std::map<int, int> per_dev;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return 256;
  }
  std::lock_guard<std::mutex> lk(mu);
  auto it = per_dev.find(dev);
  if (it != per_dev.end()) return it->second;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
    (void)hipGetLastError();
    cus = 256;
  }
  return per_dev[dev] = cus;
}

namespace {
// Guided-filter blocks resident at once on the current device (4 per CU).
int gf_round_blocks() { return 4 * device_cu_count(); }
}  // namespace

// Tile heights of an offline launch group.  Frames whose size has no table
// entry take the smallest height in {16, 32, 64, 128} at which the group's
// guided-filter blocks fit one round on the device: taller tiles amortise the
// initial window of each block, shorter ones keep a single frame's launch
// wide enough to fill the chip.  A group just over one round at 128 rows takes
// the smallest multiple of 8 up to kGfRowsMax that fits, when there is one.
// Results do not depend on the choice.
void fit_gf_rows(Batch& b) {
  bool fixed[kMaxBatch];
  int n_free = 0, fixed_blocks = 0;
  for (int i = 0; i < b.n; ++i) {
    const FrameDev& f = b.f[i];
    const hzd_tile_config c = tile_config_for(f.W, f.H, &fixed[i]);
    if (fixed[i]) {
      b.f[i].gf_rows = c.gf_rows;
      fixed_blocks += gf_blocks(f.W, f.H, f.radius, c.gf_rows);
    } else {
      ++n_free;
    }
  }
  if (!n_free) return;
  const int round = gf_round_blocks();
  auto blocks_at = [&](int rows) {
    int blocks = fixed_blocks;
    for (int i = 0; i < b.n; ++i)
      if (!fixed[i]) blocks += gf_blocks(b.f[i].W, b.f[i].H, b.f[i].radius, rows);
    return blocks;
  };
  int rows = 16;
  for (; rows < 128; rows *= 2)
    if (blocks_at(rows) <= round) break;
  if (rows == 128 && blocks_at(128) > round) {
    // just over one round at 128 rows (e.g. 8 x 1080p: 1080 blocks): a slightly
    // taller tile that fits one round is a little faster (136 rows: 484 against
    // 501 us per launch); beyond one round the cost is flat, so keep 128
    for (int r = 136; r <= kGfRowsMax; r += 8) {
      if (blocks_at(r) <= round) {
        rows = r;
        break;
      }
    }
  }
  for (int i = 0; i < b.n; ++i)
    if (!fixed[i]) b.f[i].gf_rows = rows;
}

// Fill the device descriptor of one frame; `ws` is the frame's workspace base.
// With a resize, *rz receives the resampling descriptor and the pipeline
// reads the working-size copy in the workspace instead of the caller's frame.
FrameDev make_frame_dev(const hzd_params& p, const hzd_frame& fr, const hzd_frame_aux* aux, uint8_t* ws,
                        ResizeDev* rz) {
  FrameDev d;
  std::memset(&d, 0, sizeof(d));
  int W, H;
  output_size(p, fr.width, fr.height, &W, &H);
  const bool offline = p.mode == HZD_MODE_OFFLINE;
  d.src = fr.src;
  d.dst = fr.dst;
  d.src_pitch = fr.src_pitch;
  d.dst_pitch = fr.dst_pitch;
  d.W = W;
  d.H = H;
  size_t off = 0;
  d.st = reinterpret_cast<FrameState*>(ws + off);
  off += a256(sizeof(FrameState));
  if (p.resize_width != 0) {
    uint8_t* copy = ws + off;
    off += a256((size_t)H * a16(3 * W));
    d.src = copy;
    d.src_pitch = a16(3 * W);
    if (rz) {
      rz->src = fr.src;
      rz->src_pitch = fr.src_pitch;
      rz->dst = copy;
      rz->dst_pitch = a16(3 * W);
      rz->Ws = fr.width;
      rz->Hs = fr.height;
      rz->Wo = W;
      rz->Ho = H;
    }
  }
  d.D_pitch = a16(W);
  d.D = ws + off;
  off += a256((size_t)H * d.D_pitch);
  d.E_pitch = a16(3 * W);
  if (p.tx == HZD_TX_HE) {
    d.E = ws + off;
    off += a256((size_t)H * d.E_pitch);
  }
  d.rowsel = reinterpret_cast<RowSel*>(ws + off);
  off += a256((size_t)H * sizeof(RowSel));
  if (select_one_fits(W, H)) {
    d.hpart = reinterpret_cast<uint16_t*>(ws + off);
    off += a256((size_t)dark_tiles(W, H) * 256 * 2);
  }
  if (offline) {
    d.LP = reinterpret_cast<uint2*>(ws + off);
    off += a256((size_t)W * H * 8);
    d.AB = ws + off;
    off += a256((size_t)W * H * (ab_fixed_point(p.gf_eps, p.t0, p.gf_radius).wide ? 16 : 8));
    const size_t nch = (size_t)((H + 7) / 8);
    d.PGa = reinterpret_cast<ulonglong2*>(ws + off);
    off += a256(nch * W * 16);
    d.PGb = reinterpret_cast<ulonglong2*>(ws + off);
    off += a256(nch * W * 16);
    d.S8ab = reinterpret_cast<longlong2*>(ws + off);
    off += a256(nch * W * 16);
    if (p.color_balance || p.gamma_adaptive) {  // the refined t waits for a frame-wide sum
      d.tmap = ws + off;
      off += a256((size_t)W * H * (p.precision == HZD_PREC_FP16 ? 2 : 4));
    }
  }
  if (aux) {
    d.A_out = aux->A_out;
    d.sel_out = aux->sel_out;
    d.dark_out = aux->dark_out;
    d.t_out = aux->t_out;
    d.J_out = aux->J_out;
  }
  const double n = (double)W * (double)H;
  d.K = (int32_t)std::max(1.0, std::floor((double)p.top_frac * n));
  d.radius = offline ? p.gf_radius : 0;
  d.omega = p.omega;
  d.t0 = p.t0;
  d.alpha = p.alpha;
  const double g = (double)p.gamma;
  d.inv_gamma = (float)(1.0 / g);
  d.gamma_log_bias = (float)(std::log2(255.0) * (1.0 - 1.0 / g));

  d.eps = p.gf_eps;
  if (offline) {
    const int k = ab_fixed_point(p.gf_eps, p.t0, p.gf_radius).bits;
    d.ab_scale = std::ldexp(1.0f, k);
  }
  d.gf_rows = tile_config_for(W, H).gf_rows;
  d.A_state = fr.airlight_state;
  d.ema = p.airlight_smoothing;
  d.gamma_target = p.gamma_target;
  const bool aligned = ((uintptr_t)d.src % 4 == 0) && ((uintptr_t)d.dst % 4 == 0) && (d.src_pitch % 4 == 0) &&
                       (d.dst_pitch % 4 == 0);
  d.flags = (p.gamma == 1.0f ? kFdGammaOne : 0u) | (aligned ? kFdAligned : 0u) |
            (p.gamma_adaptive ? kFdGammaAdaptive : 0u) | (p.color_balance == 2 ? kFdWbPercentile : 0u);
  // percentile white balance: k = floor(p W H) pixels ignored at each end of each channel
  d.wb_k = p.color_balance == 2 ? (int32_t)std::floor((double)p.wb_percentile * n) : 0;
  return d;
}

int check(hipError_t e, const char* what) {
  if (e == hipSuccess) return HZD_OK;
  return fail(HZD_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ------------------------------------------------------------ stage timing
namespace {
struct ProfRec {
  const char* stage;
  hipEvent_t a, b;
};
std::atomic<int> g_prof_on{0};
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof_pending;
std::vector<hipEvent_t> g_prof_pool;
std::map<std::string, std::pair<uint64_t, double>> g_prof_totals;

hipEvent_t prof_event() {
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_pool.empty()) {
      hipEvent_t e = g_prof_pool.back();
      g_prof_pool.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch one stage; with `prof`, bracket it with events on its stream.
template <typename F>
int stage(bool prof, const char* name, hipStream_t s, F&& launch) {
  if (!prof) return check(launch(), name);
  hipEvent_t a = prof_event(), b = prof_event();
  if (a) (void)hipEventRecord(a, s);
  const int rc = check(launch(), name);
  if (b) (void)hipEventRecord(b, s);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (a && b) {
    g_prof_pending.push_back({name, a, b});
  } else {
    if (a) g_prof_pool.push_back(a);
    if (b) g_prof_pool.push_back(b);
  }
  return rc;
}
}  // namespace

// A launch's epoch (kFdFresh): nonzero and unique in the process.  The start
// is random, so that state written by another process into the same memory is
// not mistaken for this launch's.
static unsigned long long next_epoch() {
  static std::atomic<unsigned long long> counter{[] {
    std::random_device rd;
    return ((unsigned long long)rd() << 32) ^ (unsigned long long)rd();
  }()};
  unsigned long long e;
  do e = counter.fetch_add(1, std::memory_order_relaxed) + 1; while (e == 0);
  return e;
}

bool stream_capturing(hipStream_t s) {
  if (s == nullptr) return false;   // the null stream cannot be captured
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return true;   // unknown: take the form that is safe to record
  }
  return cs != hipStreamCaptureStatusNone;
}

// The per-frame algorithm of Sec. V for one launch group of <= kMaxBatch frames;
// `prof` brackets every launch with timing events.  `fresh` (kFreshYes): the
// launches run once, directly (no graph records them), so leading blocks of
// k_dark zero the frames' state and the init kernel is not launched; kFreshAsk
// decides by whether s is being captured, asked only for frames that would
// take the init kernel.
int run_group(const GroupKey& g, const Batch& b, const ResizeBatch* rz, hipStream_t s, bool prof, int fresh) {
  int rc;
  // an empty event pair measures what bracketing itself costs
  if (prof) (void)stage(prof, "event_pair", s, [] { return hipSuccess; });
  if (g.resize && (rc = stage(prof, "resize", s, [&] { return launch_resize(*rz, s); })) != HZD_OK) return rc;
  const bool he = g.tx == HZD_TX_HE;
  // Small frames take the one-block selection: it builds the histogram from D
  // and zeroes the later passes' sums, so neither the init kernel nor the
  // histogram atomics of k_dark are needed.
  bool one = true;
  for (int i = 0; i < b.n; ++i) one = one && select_one_fits(b.f[i].W, b.f[i].H);
  if (one) {
    Batch bo = b;
    for (int i = 0; i < bo.n; ++i) bo.f[i].flags |= kFdNoHist;
    if ((rc = stage(prof, "dark", s, [&] { return launch_dark(bo, g, he, s); })) != HZD_OK) return rc;
    if ((rc = stage(prof, "select", s, [&] { return launch_select_one(bo, s); })) != HZD_OK) return rc;
  } else if (fresh == kFreshYes || (fresh == kFreshAsk && !stream_capturing(s))) {
    Batch bf = b;
    bf.epoch = next_epoch();
    for (int i = 0; i < bf.n; ++i) bf.f[i].flags |= kFdFresh;
    if ((rc = stage(prof, "dark", s, [&] { return launch_dark(bf, g, he, s); })) != HZD_OK) return rc;
    if ((rc = stage(prof, "select", s, [&] { return launch_select(bf, s); })) != HZD_OK) return rc;
  } else {
    if ((rc = stage(prof, "init", s, [&] { return launch_init(b, s); })) != HZD_OK) return rc;
    if ((rc = stage(prof, "dark", s, [&] { return launch_dark(b, g, he, s); })) != HZD_OK) return rc;
    if ((rc = stage(prof, "select", s, [&] { return launch_select(b, s); })) != HZD_OK) return rc;
  }
  if (g.mode == HZD_MODE_OFFLINE) {
    if ((rc = stage(prof, "gf_prep", s, [&] { return launch_gf_prep(b, g, s); })) != HZD_OK) return rc;
    if ((rc = stage(prof, "gf_ab", s, [&] { return launch_gf_ab(b, g, s); })) != HZD_OK) return rc;
    if ((rc = stage(prof, "gf_q", s, [&] { return launch_gf_q(b, g, s); })) != HZD_OK) return rc;
    if (g.gadapt) {  // the t map and luma sums are stored: gamma, then balance and output
      if (g.cb) {
        if ((rc = stage(prof, "recon_sums", s, [&] { return launch_recon(b, g, TSRC_TMAP, 1, s); })) != HZD_OK)
          return rc;
        if ((rc = stage(prof, "recon_apply", s, [&] { return launch_recon(b, g, TSRC_TMAP, 2, s); })) != HZD_OK)
          return rc;
      } else if ((rc = stage(prof, "recon", s, [&] { return launch_recon(b, g, TSRC_TMAP, 0, s); })) != HZD_OK) {
        return rc;
      }
    } else if (g.cb &&
               (rc = stage(prof, "recon_apply", s, [&] { return launch_recon(b, g, TSRC_TMAP, 2, s); })) != HZD_OK) {
      return rc;
    }
  } else {
    const int tsrc = he ? TSRC_HE : TSRC_PAPER;
    if (g.gadapt && (rc = stage(prof, "recon_luma", s, [&] { return launch_recon(b, g, tsrc, 3, s); })) != HZD_OK)
      return rc;
    if (g.cb) {
      if ((rc = stage(prof, "recon_sums", s, [&] { return launch_recon(b, g, tsrc, 1, s); })) != HZD_OK) return rc;
      if ((rc = stage(prof, "recon_apply", s, [&] { return launch_recon(b, g, tsrc, 2, s); })) != HZD_OK) return rc;
    } else {
      if ((rc = stage(prof, "recon", s, [&] { return launch_recon(b, g, tsrc, 0, s); })) != HZD_OK) return rc;
    }
  }
  return HZD_OK;
}

// ------------------------------------------------------------ graph cache
namespace {
struct GraphEntry {
  hipGraphExec_t exec;
  uint64_t last_use;
};
std::mutex g_graph_mu;
int g_graph_cap = 0;
uint64_t g_graph_clock = 0;
std::map<std::string, GraphEntry> g_graphs;

void graph_evict_locked(size_t keep) {
  if (g_graphs.size() <= keep) return;
  (void)hipDeviceSynchronize();  // an evicted graph may still be running somewhere
  while (g_graphs.size() > keep) {
    auto victim = g_graphs.begin();
    for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it)
      if (it->second.last_use < victim->second.last_use) victim = it;
    (void)hipGraphExecDestroy(victim->second.exec);
    g_graphs.erase(victim);
  }
}
}  // namespace

// Launch one group: replay a cached graph of its kernels when enabled.
int launch_group(const GroupKey& g, const Batch& bin, const ResizeBatch* rz, hipStream_t s) {
  if (g.resize && (!rz || rz->n != bin.n)) return fail(HZD_E_INVAL, "resize descriptors missing");
  Batch b = bin;
  if (g.mode == HZD_MODE_OFFLINE) fit_gf_rows(b);
  int cap;
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    cap = g_graph_cap;
  }
  const bool prof = g_prof_on.load(std::memory_order_relaxed);
  if (s == nullptr) return run_group(g, b, rz, s, prof, kFreshYes);
  if (cap == 0 && !prof) return run_group(g, b, rz, s, false, kFreshAsk);
  // the caller is capturing: our launches join its graph, in the form that
  // may be replayed, without timing events (they would complete only when
  // that graph runs)
  if (stream_capturing(s)) return run_group(g, b, rz, s, false, kFreshNo);
  if (cap == 0 || prof) return run_group(g, b, rz, s, prof, kFreshYes);
  // A graph is bound to the device it was captured on, and a freed device
  // address can come back on another device: the device is part of the key.
  int dev = -1;
  if (hipStreamGetDevice(s, &dev) != hipSuccess) {
    (void)hipGetLastError();
    return run_group(g, b, rz, s, false, kFreshYes);
  }
  std::string key(reinterpret_cast<const char*>(&dev), sizeof(dev));
  key.append(reinterpret_cast<const char*>(&g), sizeof(g));
  key.append(reinterpret_cast<const char*>(&b), sizeof(b));
  if (g.resize) key.append(reinterpret_cast<const char*>(rz), sizeof(*rz));
  hipGraphExec_t exec = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) {
      it->second.last_use = ++g_graph_clock;
      exec = it->second.exec;
    }
  }
  if (!exec) {
    int rc = check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
    if (rc) return rc;
    const int rrc = run_group(g, b, rz, s, false, kFreshNo);
    hipGraph_t graph = nullptr;
    rc = check(hipStreamEndCapture(s, &graph), "end capture");
    if (rrc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rrc;
    }
    if (rc) return rc;
    rc = check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate");
    (void)hipGraphDestroy(graph);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) {  // another thread captured the same key meanwhile
      (void)hipGraphExecDestroy(exec);
      exec = it->second.exec;
    } else {
      graph_evict_locked((size_t)std::max(0, g_graph_cap - 1));
      g_graphs[key] = GraphEntry{exec, ++g_graph_clock};
    }
  }
  return check(hipGraphLaunch(exec, s), "graph launch");
}

// ------------------------------------------------------------ concurrent launch groups
namespace {
struct GroupLaunch {
  GroupKey g;
  Batch b;
  ResizeBatch rz;
  double work;  // pixels of the group
};

constexpr int kGroupStreams = 4;
struct GroupStreams {
  hipStream_t s[kGroupStreams];
  hipEvent_t fork = nullptr;              // recorded on the caller's stream
  hipEvent_t join[kGroupStreams] = {};    // recorded on s[i]
  int n = 0;
  bool tried = false;
};

// Streams and fork/join events of the calling thread on device `dev` for
// concurrent launch groups.  Per thread, so that one thread's graph capture
// on such a stream never sees another thread's launches, and an event is
// re-recorded only by the thread that waits on it (a wait takes the record
// made before it).  They live until the process ends.
GroupStreams& group_streams(int dev) {
  thread_local std::map<int, GroupStreams> per_dev;
  GroupStreams& g = per_dev[dev];
  if (!g.tried) {
    g.tried = true;
    if (hipEventCreateWithFlags(&g.fork, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      g.fork = nullptr;
      return g;
    }
    for (int i = 0; i < kGroupStreams; ++i) {
      if (hipStreamCreateWithFlags(&g.s[i], hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        break;
      }
      if (hipEventCreateWithFlags(&g.join[i], hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamDestroy(g.s[i]);
        break;
      }
      ++g.n;
    }
  }
  return g;
}
}  // namespace

// Several launch groups of one call run concurrently on the thread's group
// streams, largest first, so that the short, latency-bound stages of one group
// overlap the work of another (the stream-ordered result is unchanged: groups
// touch disjoint frames and workspace slices).  The groups wait for the work
// enqueued on `s` before the call, and `s` waits for every group.  Returns
// HZD_E_UNSUPPORTED (nothing enqueued) where this does not apply: `s` is being
// captured into a graph, belongs to another device, or streams are missing.
int launch_concurrent(std::vector<GroupLaunch>& ls, hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return HZD_E_UNSUPPORTED;
  }
  if (s != nullptr) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    int sdev = -1;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone ||
        hipStreamGetDevice(s, &sdev) != hipSuccess || sdev != dev) {
      (void)hipGetLastError();
      return HZD_E_UNSUPPORTED;
    }
  }
  GroupStreams& gs = group_streams(dev);
  if (gs.n < 2) return HZD_E_UNSUPPORTED;
  const int k = std::min<int>(gs.n, (int)ls.size());
  int rc = check(hipEventRecord(gs.fork, s), "fork record");
  for (int i = 0; i < k && rc == HZD_OK; ++i) rc = check(hipStreamWaitEvent(gs.s[i], gs.fork, 0), "fork wait");
  if (rc != HZD_OK) return rc;
  std::stable_sort(ls.begin(), ls.end(),
                   [](const GroupLaunch& a, const GroupLaunch& b) { return a.work > b.work; });
  for (size_t j = 0; j < ls.size() && rc == HZD_OK; ++j)
    rc = launch_group(ls[j].g, ls[j].b, &ls[j].rz, gs.s[j % k]);
  // join even after a failure: `s` follows whatever was enqueued on the group streams
  for (int i = 0; i < k; ++i) {
    int jr = check(hipEventRecord(gs.join[i], gs.s[i]), "join record");
    if (jr == HZD_OK) jr = check(hipStreamWaitEvent(s, gs.join[i], 0), "join wait");
    if (rc == HZD_OK) rc = jr;
  }
  return rc;
}

int validate_call(const hzd_params* params, const hzd_frame* frames, int32_t n,
                  std::vector<const hzd_params*>& ps, std::vector<size_t>& offs, size_t* need) {
  if (n < 1) return fail(HZD_E_INVAL, "n = %d < 1", n);
  if (!frames) return fail(HZD_E_INVAL, "frames is NULL");
  ps.assign(n, nullptr);
  for (int i = 0; i < n; ++i) {
    ps[i] = frames[i].params ? frames[i].params : params;
    int rc = validate_params(ps[i]);
    if (rc) return rc;
    if ((rc = validate_frame(&frames[i], *ps[i], i)) != HZD_OK) return rc;
    if (ps[i]->airlight_smoothing > 0.0f && !frames[i].airlight_state)
      return fail(HZD_E_INVAL, "frame %d: airlight_smoothing > 0 needs an airlight_state", i);
    if ((uintptr_t)frames[i].airlight_state % 16)
      return fail(HZD_E_INVAL, "frame %d: airlight_state not 16-byte aligned", i);
  }
  {
    // frames of one call run concurrently: each stream state at most once
    std::vector<uintptr_t> states;
    for (int i = 0; i < n; ++i)
      if (frames[i].airlight_state) states.push_back((uintptr_t)frames[i].airlight_state);
    std::sort(states.begin(), states.end());
    if (std::adjacent_find(states.begin(), states.end()) != states.end())
      return fail(HZD_E_INVAL, "two frames of one call share an airlight_state");
  }
  offs.assign(n, 0);
  size_t total = 0;
  for (int i = 0; i < n; ++i) {
    offs[i] = total;
    total += frame_ws_bytes(*ps[i], frames[i].width, frames[i].height);
  }
  *need = total;
  return HZD_OK;
}

int run_frame_direct(const hzd_params* p, const hzd_frame& fr, const hzd_frame_aux* aux, void* ws,
                     hipStream_t s) {
  Batch b;
  ResizeBatch rz;
  std::memset(&b, 0, sizeof(b));
  std::memset(&rz, 0, sizeof(rz));
  b.n = rz.n = 1;
  b.f[0] = make_frame_dev(*p, fr, aux, reinterpret_cast<uint8_t*>(ws), &rz.f[0]);
  const GroupKey g = group_key(*p);
  if (g.mode == HZD_MODE_OFFLINE) fit_gf_rows(b);
  return run_group(g, b, &rz, s, false, kFreshAsk);
}

int dehaze_many(const hzd_params* params, const hzd_frame* frames, int32_t n, const hzd_frame_aux* aux,
                void* workspace, size_t ws_bytes, void* stream) {
  std::vector<const hzd_params*> ps;
  std::vector<size_t> offs;
  size_t need = 0;
  int vrc = validate_call(params, frames, n, ps, offs, &need);
  if (vrc) return vrc;
  if (!workspace) return fail(HZD_E_INVAL, "workspace is NULL");
  if ((uintptr_t)workspace % 256) return fail(HZD_E_INVAL, "workspace not 256-byte aligned");
  if (ws_bytes < need) return fail(HZD_E_NOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);

  std::map<GroupKey, std::vector<int>> groups;
  for (int i = 0; i < n; ++i) groups[group_key(*ps[i])].push_back(i);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<GroupLaunch> ls;
  for (auto& kv : groups) {
    const std::vector<int>& idx = kv.second;
    for (size_t c = 0; c < idx.size(); c += kMaxBatch) {
      ls.emplace_back();
      GroupLaunch& L = ls.back();
      std::memset(&L.b, 0, sizeof(L.b));
      std::memset(&L.rz, 0, sizeof(L.rz));
      L.g = kv.first;
      L.work = 0.0;
      L.b.n = L.rz.n = (int)std::min<size_t>(kMaxBatch, idx.size() - c);
      for (int j = 0; j < L.b.n; ++j) {
        const int i = idx[c + j];
        L.b.f[j] = make_frame_dev(*ps[i], frames[i], aux ? &aux[i] : nullptr,
                                  reinterpret_cast<uint8_t*>(workspace) + offs[i], &L.rz.f[j]);
        L.work += (double)frames[i].width * (double)frames[i].height;
      }
    }
  }
  if (ls.size() >= 2) {
    const int rc = launch_concurrent(ls, s);
    if (rc != HZD_E_UNSUPPORTED) return rc;
  }
  for (const GroupLaunch& L : ls) {
    const int rc = launch_group(L.g, L.b, &L.rz, s);
    if (rc) return rc;
  }
  return HZD_OK;
}

}  // namespace hzd

using namespace hzd;

extern "C" {

int hzd_abi_version(void) { return HZD_ABI_VERSION; }

const char* hzd_status_str(int32_t st) {
  switch (st) {
    case HZD_OK: return "ok";
    case HZD_E_INVAL: return "invalid argument";
    case HZD_E_NOMEM: return "workspace or arena too small";
    case HZD_E_DEVICE: return "device error";
    case HZD_E_AGAIN: return "try again";
    case HZD_E_CLOSED: return "closed";
    case HZD_E_UNSUPPORTED: return "unsupported";
    case HZD_E_TIMEOUT: return "timeout";
    default: return "unknown status";
  }
}

const char* hzd_last_error(void) { return g_last_error.c_str(); }

int hzd_params_default(hzd_params* p, int32_t preset) {
  if (!p) return fail(HZD_E_INVAL, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->size = sizeof(hzd_params);
  p->mode = HZD_MODE_REALTIME;
  p->patch = 15;
  p->omega = 0.95f;
  p->t0 = 0.1f;
  p->top_frac = 0.001f;
  p->alpha = 0.8f;
  p->gamma = 1.2f;
  p->gf_radius = 60;
  p->gf_eps = 1e-3f;
  p->color_balance = 0;
  p->tx = HZD_TX_HE;
  p->precision = HZD_PREC_FP32;
  p->gamma_adaptive = 0;
  p->gamma_target = 0.5f;
  p->wb_percentile = 0.02f;
  switch (preset) {
    case HZD_PRESET_REALTIME: break;
    case HZD_PRESET_OFFLINE:
      p->mode = HZD_MODE_OFFLINE;
      p->color_balance = 1;
      break;
    case HZD_PRESET_PAPER_REALTIME:
      p->omega = 0.5f;
      p->t0 = 0.05f;
      p->tx = HZD_TX_PAPER;
      break;
    default: return fail(HZD_E_INVAL, "preset %d unknown", preset);
  }
  clear_error();
  return HZD_OK;
}

int hzd_workspace_size(const hzd_params* params, const hzd_frame* frames, int32_t n, size_t* bytes) {
  if (!bytes) return fail(HZD_E_INVAL, "bytes is NULL");
  if (!frames || n < 1) return fail(HZD_E_INVAL, "no frames");
  size_t need = 0;
  for (int i = 0; i < n; ++i) {
    const hzd_params* p = frames[i].params ? frames[i].params : params;
    int rc = validate_params(p);
    if (rc) return rc;
    if ((rc = validate_size(*p, frames[i].width, frames[i].height, i)) != HZD_OK) return rc;
    need += frame_ws_bytes(*p, frames[i].width, frames[i].height);
  }
  *bytes = need;
  clear_error();
  return HZD_OK;
}

int hzd_tile_config_set(int32_t width, int32_t height, const hzd_tile_config* cfg) {
  if (width < 0 || height < 0) return fail(HZD_E_INVAL, "size %dx%d", width, height);
  if (cfg && (cfg->gf_rows < kGfRowsMin || cfg->gf_rows > kGfRowsMax || cfg->gf_rows % 8 != 0))
    return fail(HZD_E_INVAL, "gf_rows %d not a multiple of 8 in %d..%d", cfg->gf_rows, kGfRowsMin, kGfRowsMax);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  if (cfg) g_tune[{width, height}] = *cfg;
  else g_tune.erase({width, height});
  clear_error();
  return HZD_OK;
}

int hzd_tile_config_get(int32_t width, int32_t height, hzd_tile_config* cfg) {
  if (!cfg) return fail(HZD_E_INVAL, "cfg is NULL");
  *cfg = tile_config_for(width, height);
  clear_error();
  return HZD_OK;
}

int hzd_autotune(const hzd_params* params, const hzd_frame* frame, void* workspace, size_t ws_bytes,
                 void* hip_stream, int32_t reps, hzd_tile_config* best) {
  if (!frame || !best) return fail(HZD_E_INVAL, "NULL argument");
  if (reps < 1 || reps > 10000) return fail(HZD_E_INVAL, "reps %d outside 1..10000", reps);
  const hzd_params* p = frame->params ? frame->params : params;
  int rc = validate_params(p);
  if (rc) return rc;
  // the timed calls leave the stream's airlight state alone: same kernels,
  // no blend and no state write
  hzd_params tp = *p;
  tp.airlight_smoothing = 0.0f;
  hzd_frame tf = *frame;
  tf.params = &tp;
  tf.airlight_state = nullptr;
  int W, H;  // the guided filter runs at the output size
  output_size(*p, frame->width, frame->height, &W, &H);
  if (p->mode != HZD_MODE_OFFLINE) {  // no tile knob on the real-time path
    *best = tile_config_for(W, H);
    clear_error();
    return HZD_OK;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  hipEvent_t e0, e1;
  if ((rc = check(hipEventCreate(&e0), "event")) != HZD_OK) return rc;
  if ((rc = check(hipEventCreate(&e1), "event")) != HZD_OK) {
    (void)hipEventDestroy(e0);
    return rc;
  }
  const hzd_tile_config prev = tile_config_for(W, H);
  bool had_entry;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    had_entry = g_tune.count({W, H}) > 0;
  }
  static const int kCand[] = {8, 16, 24, 32, 48, 64, 96, 128};
  float best_ms = 1e30f;
  hzd_tile_config bestc = prev;
  for (int rows : kCand) {
    if (rows > H && rows != kCand[0]) break;
    hzd_tile_config c{rows};
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[{W, H}] = c;
    }
    rc = dehaze_many(&tp, &tf, 1, nullptr, workspace, ws_bytes, hip_stream);  // warm
    if (rc == HZD_OK) rc = check(hipEventRecord(e0, s), "event record");
    for (int i = 0; i < reps && rc == HZD_OK; ++i) rc = dehaze_many(&tp, &tf, 1, nullptr, workspace, ws_bytes, hip_stream);
    if (rc == HZD_OK) rc = check(hipEventRecord(e1, s), "event record");
    if (rc == HZD_OK) rc = check(hipEventSynchronize(e1), "event sync");
    float ms = 0.f;
    if (rc == HZD_OK) rc = check(hipEventElapsedTime(&ms, e0, e1), "event time");
    if (rc != HZD_OK) break;
    if (ms < best_ms) {
      best_ms = ms;
      bestc = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (rc == HZD_OK) g_tune[{W, H}] = bestc;
    else if (had_entry) g_tune[{W, H}] = prev;
    else g_tune.erase({W, H});
  }
  if (rc != HZD_OK) return rc;
  tune_save(W, H, bestc);
  *best = bestc;
  clear_error();
  return HZD_OK;
}

int hzd_graph_cache(int32_t capacity) {
  if (capacity < 0 || capacity > 4096) return fail(HZD_E_INVAL, "capacity %d outside 0..4096", capacity);
  std::lock_guard<std::mutex> lk(g_graph_mu);
  g_graph_cap = capacity;
  graph_evict_locked((size_t)capacity);
  clear_error();
  return HZD_OK;
}

int hzd_profile_enable(int32_t on) {
  g_prof_on.store(on ? 1 : 0);
  clear_error();
  return HZD_OK;
}

int hzd_profile_read(hzd_profile_entry* out, int32_t cap, int32_t* n, int32_t reset) {
  if (cap < 0 || (cap > 0 && !out)) return fail(HZD_E_INVAL, "bad output array");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  int rc = HZD_OK;
  for (const ProfRec& r : g_prof_pending) {
    float ms = 0.f;
    if (rc == HZD_OK) rc = check(hipEventSynchronize(r.b), "profile sync");
    if (rc == HZD_OK) rc = check(hipEventElapsedTime(&ms, r.a, r.b), "profile elapsed");
    auto& t = g_prof_totals[r.stage];
    t.first += 1;
    t.second += ms;
    g_prof_pool.push_back(r.a);
    g_prof_pool.push_back(r.b);
  }
  g_prof_pending.clear();
  int k = 0;
  for (auto& kv : g_prof_totals) {
    if (k < cap) {
      std::memset(out[k].name, 0, sizeof(out[k].name));
      std::strncpy(out[k].name, kv.first.c_str(), sizeof(out[k].name) - 1);
      out[k].launches = kv.second.first;
      out[k].total_ms = kv.second.second;
    }
    ++k;
  }
  if (n) *n = std::min(k, cap);
  if (reset) g_prof_totals.clear();
  if (rc == HZD_OK) clear_error();
  return rc;
}

int hzd_dehaze_frame(const hzd_params* params, const hzd_frame* frame, const hzd_frame_aux* aux,
                     void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!frame) return fail(HZD_E_INVAL, "frame is NULL");
  int rc = dehaze_many(params, frame, 1, aux, workspace, ws_bytes, hip_stream);
  if (rc == HZD_OK) clear_error();
  return rc;
}

int hzd_dehaze_batch(const hzd_params* params, const hzd_frame* frames, int32_t n,
                     const hzd_frame_aux* aux, void* workspace, size_t ws_bytes, void* hip_stream) {
  int rc = dehaze_many(params, frames, n, aux, workspace, ws_bytes, hip_stream);
  if (rc == HZD_OK) clear_error();
  return rc;
}

}  // extern "C"
