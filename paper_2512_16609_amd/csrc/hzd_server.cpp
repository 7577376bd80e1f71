// Continuous-batching server for streams of frames.
//
// One scheduler thread per server.  Streams reserve their device state and
// workspaces in the caller's arena at open (admission by HBM budget).
// Submitted frames wait in a FIFO; whenever a HIP stream and in-flight
// capacity are free, the scheduler takes the oldest frames that share one
// launch group (same kernels), up to frames_per_launch, and launches them as
// one batch; frames that arrive while others run join the next batch.  The
// method is feed-forward per frame (paper Sec. V) and every kernel reduces in
// an order fixed by the frame's own tiling, so a frame's result does not
// depend on which batch it rode in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "hzd.h"
#include "hzd_internal.h"
#include "hzd_plan.h"

using namespace hzd;

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// First-fit allocator over [0, size) of the arena, 256-byte granules.
struct Arena {
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(size_t n) {
    size = n & ~size_t(255);
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t n, size_t* off) {
    n = (n + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, roff = it->first + n;
        free_.erase(it);
        if (rest) free_[roff] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) & ~size_t(255);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const {
    size_t f = 0;
    for (auto& kv : free_) f += kv.second;
    return size - f;
  }
};

constexpr int kSlotsPerStream = 2;   // frames of one stream on the device at once

// Host-coherent pinned cells of 4 int32 that the selection writes a served
// frame's {K, vstar, cutoff, status} into, so that the scheduler reads the
// selection's consistency status when the launch completes, without a copy.
// Process-wide pool, allocated in blocks and never freed (a block is reused by
// later streams and servers).
struct StatusCells {
  std::mutex mu;
  std::vector<int32_t*> free_cells;
  int32_t* get() {
    std::lock_guard<std::mutex> lk(mu);
    if (free_cells.empty()) {
      constexpr int kBlock = 1024;
      void* p = nullptr;
      if (hipHostMalloc(&p, kBlock * 4 * sizeof(int32_t), hipHostMallocCoherent | hipHostMallocPortable) !=
              hipSuccess ||
          !p) {
        (void)hipGetLastError();
        return nullptr;
      }
      int32_t* c = static_cast<int32_t*>(p);
      for (int i = kBlock - 1; i >= 0; --i) free_cells.push_back(c + 4 * i);
    }
    int32_t* c = free_cells.back();
    free_cells.pop_back();
    return c;
  }
  void put(int32_t* c) {
    if (!c) return;
    std::lock_guard<std::mutex> lk(mu);
    free_cells.push_back(c);
  }
};
StatusCells& status_cells() {
  static StatusCells* s = new StatusCells();   // outlives every server
  return *s;
}
constexpr int kMaxQueuedPerStream = 256;

// A stream's arena block: per-slot airlight outputs (A; 256 B each), the stream's
// airlight state (256 B), then one workspace per slot.
constexpr size_t kAirlightStateOff = 256 * kSlotsPerStream;
constexpr size_t kWorkspacesOff = kAirlightStateOff + 256;

size_t stream_ws_bytes(const hzd_params& p, int W, int H) {
  return (frame_ws_bytes(p, W, H) + 255) & ~size_t(255);
}

struct Job;

}  // namespace

struct hzd_stream {
  hzd_server* srv = nullptr;
  hzd_params p{};
  int W = 0, H = 0;
  size_t arena_off = 0, arena_len = 0;
  size_t ws_bytes = 0;          // one slot's workspace
  uint8_t* state_dev = nullptr; // A (3 floats) of each slot, 256 B apart
  int32_t* status[kSlotsPerStream] = {nullptr, nullptr};  // pinned {K, vstar, cutoff, status} per slot
  bool slot_busy[kSlotsPerStream] = {false, false};
  uint64_t blocked_pass = 0;    // admission pass in which a frame of this stream was left queued
  int last_slot = -1;
  bool ema_primed = false;      // a frame has completed and stored the airlight state
  uint64_t next_ticket = 1;
  int queued = 0, inflight = 0;
  bool closing = false;
  std::set<uint64_t> pending;    // submitted tickets not yet completed
  std::map<uint64_t, std::pair<int32_t, int64_t>> done;  // completed tickets not yet waited for: status, latency
  std::condition_variable cv;
};

namespace {
struct Job {
  hzd_stream* st;
  hzd_frame fr;
  hzd_done_fn cb;
  void* user;
  uint64_t ticket;
  int64_t t_submit;
  hipEvent_t ready = nullptr;  // recorded on the producer's stream at submit
  int slot = -1;
};

struct Launch {
  hipEvent_t ev = nullptr;
  int hs = -1;
  std::vector<Job> jobs;
  int status = HZD_OK;
};
}  // namespace

struct hzd_server {
  hzd_server_config cfg{};
  std::vector<hipStream_t> hstreams;
  std::vector<bool> hs_busy;
  std::vector<hipEvent_t> events;
  std::mutex mu;
  std::condition_variable cv;
  std::thread thr;
  bool stop = false;
  Arena arena;
  std::vector<hzd_stream*> streams;
  std::deque<Job> queue;
  std::vector<Launch> inflight;
  int inflight_frames = 0;
  uint64_t admit_pass = 0;
  std::vector<hipEvent_t> ready_pool;  // events for the producers' streams, reused
  hzd_server_stats stats{};
};

namespace {

// Completed or failed jobs: callbacks, then (under the lock) the stream's
// completion record and its in-flight count.  The count drops only here, so a
// stream being closed cannot be freed while its completions are recorded.
void finish(hzd_server* s, std::vector<std::pair<Job, int32_t>>& done) {
  // called without the lock: completion callbacks may submit again
  const int64_t t = now_ns();
  for (auto& d : done) {
    if (d.first.cb) d.first.cb(d.first.user, d.first.ticket, d.second, t - d.first.t_submit);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  for (auto& d : done) {
    hzd_stream* st = d.first.st;
    st->done[d.first.ticket] = std::make_pair(d.second, t - d.first.t_submit);
    st->pending.erase(d.first.ticket);
    if (d.second == HZD_OK) st->ema_primed = true;
    st->inflight--;
    st->cv.notify_all();
  }
  done.clear();
  s->cv.notify_all();
}

// Launch the oldest compatible frames on a free HIP stream.  Lock held.
bool admit(hzd_server* s, std::vector<std::pair<Job, int32_t>>& done) {
  if (s->queue.empty() || s->inflight_frames >= s->cfg.max_inflight) return false;
  int hs = -1;
  for (size_t i = 0; i < s->hs_busy.size(); ++i)
    if (!s->hs_busy[i]) { hs = (int)i; break; }
  if (hs < 0) return false;
  Launch L;
  GroupKey key{};
  bool have_key = false;
  // keep a stream's frames in submission order: once a frame of a stream is
  // left in the queue, this pass skips the stream's later frames (one flag per
  // stream and pass, so a pass is linear in the queue length)
  const uint64_t pass = ++s->admit_pass;
  for (auto it = s->queue.begin(); it != s->queue.end();) {
    if ((int)L.jobs.size() >= s->cfg.frames_per_launch ||
        s->inflight_frames + (int)L.jobs.size() >= s->cfg.max_inflight)
      break;
    hzd_stream* st = it->st;
    int slot = -1;
    for (int k = 0; k < kSlotsPerStream; ++k)
      if (!st->slot_busy[k]) { slot = k; break; }
    const GroupKey gk = group_key(st->p);
    // with temporal airlight smoothing a frame needs its predecessor's
    // airlight: one frame of such a stream on the device at a time
    const bool ema_wait = st->p.airlight_smoothing > 0.0f && st->inflight > 0;
    if (st->blocked_pass == pass || slot < 0 || ema_wait || (have_key && (gk < key || key < gk))) {
      st->blocked_pass = pass;
      ++it;
      continue;
    }
    key = gk;
    have_key = true;
    Job j = *it;
    j.slot = slot;
    st->slot_busy[slot] = true;
    st->queued--;
    st->inflight++;
    L.jobs.push_back(j);
    it = s->queue.erase(it);
  }
  if (L.jobs.empty()) return false;
  Batch b;
  ResizeBatch rz;
  std::memset(&b, 0, sizeof(b));
  std::memset(&rz, 0, sizeof(rz));
  b.n = rz.n = (int)L.jobs.size();
  for (int i = 0; i < b.n; ++i) {
    const Job& j = L.jobs[i];
    hzd_stream* st = j.st;
    uint8_t* base = reinterpret_cast<uint8_t*>(s->cfg.arena) + st->arena_off;
    uint8_t* state = base + 256 * j.slot;
    hzd_frame_aux aux{};
    aux.A_out = reinterpret_cast<float*>(state);
    aux.sel_out = st->status[j.slot];
    st->status[j.slot][3] = -1;   // overwritten by the frame's selection kernel
    uint8_t* ws = base + kWorkspacesOff + st->ws_bytes * j.slot;
    hzd_frame fr = j.fr;
    const bool ema = st->p.airlight_smoothing > 0.0f;
    fr.airlight_state = ema ? reinterpret_cast<float*>(base + kAirlightStateOff) : nullptr;
    b.f[i] = make_frame_dev(st->p, fr, &aux, ws, &rz.f[i]);
    if (ema && !st->ema_primed) b.f[i].flags |= kFdEmaFirst;
  }
  (void)hipSetDevice(s->cfg.device);
  // the launch follows the producers' work on src and dst; an event can be
  // re-recorded as soon as a wait has been enqueued on it
  int rc = HZD_OK;
  for (auto& j : L.jobs) {
    if (j.ready) {
      if (rc == HZD_OK) rc = check(hipStreamWaitEvent(s->hstreams[hs], j.ready, 0), "ready wait");
      s->ready_pool.push_back(j.ready);
      j.ready = nullptr;
    }
  }
  if (rc == HZD_OK) rc = launch_group(key, b, &rz, s->hstreams[hs]);
  if (rc == HZD_OK) rc = check(hipEventRecord(s->events[hs], s->hstreams[hs]), "event record");
  s->stats.launches++;
  if (rc != HZD_OK) {
    for (auto& j : L.jobs) {
      j.st->slot_busy[j.slot] = false;
      s->stats.failed++;
      done.emplace_back(j, rc);
    }
    return true;
  }
  L.ev = s->events[hs];
  L.hs = hs;
  s->hs_busy[hs] = true;
  s->inflight_frames += (int)L.jobs.size();
  s->inflight.push_back(std::move(L));
  return true;
}

// Collect finished launches.  Lock held.
bool reap(hzd_server* s, std::vector<std::pair<Job, int32_t>>& done) {
  bool any = false;
  for (size_t i = 0; i < s->inflight.size();) {
    Launch& L = s->inflight[i];
    const hipError_t q = hipEventQuery(L.ev);
    if (q == hipErrorNotReady) { ++i; continue; }
    const int32_t launch_status = (q == hipSuccess) ? HZD_OK : HZD_E_DEVICE;
    for (auto& j : L.jobs) {
      // the selection's consistency status, written by the frame's kernels
      const volatile int32_t* cell = j.st->status[j.slot];
      const int32_t status = (launch_status == HZD_OK && cell[3] != 0) ? HZD_E_DEVICE : launch_status;
      j.st->slot_busy[j.slot] = false;
      j.st->last_slot = j.slot;
      if (status == HZD_OK) s->stats.completed++;
      else s->stats.failed++;
      done.emplace_back(j, status);
    }
    s->hs_busy[L.hs] = false;
    s->inflight_frames -= (int)L.jobs.size();
    s->inflight.erase(s->inflight.begin() + i);
    any = true;
  }
  return any;
}

void scheduler(hzd_server* s) {
  (void)hipSetDevice(s->cfg.device);
  std::vector<std::pair<Job, int32_t>> done;
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool progressed = reap(s, done);
    while (admit(s, done)) progressed = true;
    if (!done.empty()) {
      lk.unlock();
      finish(s, done);
      lk.lock();
      continue;
    }
    if (s->stop && s->queue.empty() && s->inflight.empty()) break;
    if (progressed) continue;
    if (s->inflight.empty()) {
      s->cv.wait(lk);
    } else {
      // device work in flight: poll its events at a fine grain
      s->cv.wait_for(lk, std::chrono::microseconds(20));
    }
  }
}

}  // namespace

extern "C" {

int hzd_server_create(const hzd_server_config* cfg, hzd_server** out) {
  if (!cfg || !out) return fail(HZD_E_INVAL, "NULL argument");
  if (cfg->size != sizeof(hzd_server_config)) return fail(HZD_E_INVAL, "config size mismatch");
  if (!cfg->arena || (uintptr_t)cfg->arena % 256) return fail(HZD_E_INVAL, "arena NULL or not 256-aligned");
  if (cfg->max_inflight < 1) return fail(HZD_E_INVAL, "max_inflight < 1");
  if (cfg->frames_per_launch < 1 || cfg->frames_per_launch > kMaxBatch)
    return fail(HZD_E_INVAL, "frames_per_launch outside 1..%d", kMaxBatch);
  if (cfg->hip_streams < 1 || cfg->hip_streams > 8) return fail(HZD_E_INVAL, "hip_streams outside 1..8");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev)
    return fail(HZD_E_INVAL, "device %d not available", cfg->device);
  hzd_server* s = new hzd_server();
  s->cfg = *cfg;
  s->arena.init(cfg->arena_bytes);
  (void)hipSetDevice(cfg->device);
  for (int i = 0; i < cfg->hip_streams; ++i) {
    hipStream_t hs = nullptr;
    hipEvent_t ev = nullptr;
    if (hipStreamCreateWithFlags(&hs, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      if (hs) (void)hipStreamDestroy(hs);
      for (auto h : s->hstreams) (void)hipStreamDestroy(h);
      for (auto e : s->events) (void)hipEventDestroy(e);
      delete s;
      return fail(HZD_E_DEVICE, "stream/event creation failed");
    }
    s->hstreams.push_back(hs);
    s->events.push_back(ev);
    s->hs_busy.push_back(false);
  }
  s->stats.arena_bytes = s->arena.size;
  s->thr = std::thread(scheduler, s);
  *out = s;
  clear_error();
  return HZD_OK;
}

int hzd_server_destroy(hzd_server* s) {
  if (!s) return fail(HZD_E_INVAL, "server is NULL");
  std::vector<std::pair<Job, int32_t>> cancelled;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto& j : s->queue) {
      j.st->queued--;
      j.st->inflight++;  // finish() records the cancellation and drops it again
      if (j.ready) s->ready_pool.push_back(j.ready);
      j.ready = nullptr;
      cancelled.emplace_back(j, HZD_E_CLOSED);
    }
    s->queue.clear();
    s->stop = true;
    s->cv.notify_all();
  }
  finish(s, cancelled);
  s->thr.join();
  (void)hipSetDevice(s->cfg.device);
  for (auto h : s->hstreams) (void)hipStreamSynchronize(h);
  for (hzd_stream* st : s->streams) {
    for (int k = 0; k < kSlotsPerStream; ++k) status_cells().put(st->status[k]);
    delete st;
  }
  for (auto h : s->hstreams) (void)hipStreamDestroy(h);
  for (auto e : s->events) (void)hipEventDestroy(e);
  for (auto e : s->ready_pool) (void)hipEventDestroy(e);
  delete s;
  clear_error();
  return HZD_OK;
}

int hzd_stream_open(hzd_server* s, const hzd_params* params, int32_t width, int32_t height,
                    hzd_stream** out) {
  if (!s || !out) return fail(HZD_E_INVAL, "NULL argument");
  int rc = validate_params(params);
  if (rc) return rc;
  if ((rc = validate_size(*params, width, height, 0)) != HZD_OK) return rc;
  hzd_stream* st = new hzd_stream();
  st->srv = s;
  st->p = *params;
  st->W = width;
  st->H = height;
  st->ws_bytes = stream_ws_bytes(*params, width, height);
  st->arena_len = kWorkspacesOff + st->ws_bytes * kSlotsPerStream;
  (void)hipSetDevice(s->cfg.device);
  for (int k = 0; k < kSlotsPerStream; ++k) {
    st->status[k] = status_cells().get();
    if (!st->status[k]) {
      for (int m = 0; m < k; ++m) status_cells().put(st->status[m]);
      delete st;
      return fail(HZD_E_DEVICE, "pinned status memory could not be allocated");
    }
  }
  auto drop = [&] {
    for (int k = 0; k < kSlotsPerStream; ++k) status_cells().put(st->status[k]);
    delete st;
  };
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      drop();
      return fail(HZD_E_CLOSED, "server is shutting down");
    }
    if (!s->arena.alloc(st->arena_len, &st->arena_off)) {
      drop();
      return fail(HZD_E_AGAIN, "arena has no room for %zu bytes (%zu used of %zu)", st->arena_len,
                  s->arena.used(), s->arena.size);
    }
    st->state_dev = reinterpret_cast<uint8_t*>(s->cfg.arena) + st->arena_off;
    s->streams.push_back(st);
    s->stats.open_streams = (int)s->streams.size();
    s->stats.arena_used = s->arena.used();
  }
  *out = st;
  clear_error();
  return HZD_OK;
}

int hzd_stream_submit(hzd_stream* st, const hzd_frame* frame, void* ready_stream, hzd_done_fn cb, void* user,
                      uint64_t* ticket) {
  if (!st || !frame) return fail(HZD_E_INVAL, "NULL argument");
  int rc = validate_frame(frame, st->p, 0);
  if (rc) return rc;
  if (frame->width != st->W || frame->height != st->H)
    return fail(HZD_E_INVAL, "frame %dx%d does not match stream %dx%d", frame->width, frame->height, st->W,
                st->H);
  hzd_server* s = st->srv;
  std::unique_lock<std::mutex> lk(s->mu);
  if (st->closing || s->stop) return fail(HZD_E_CLOSED, "stream is closing");
  if (st->queued >= kMaxQueuedPerStream) return fail(HZD_E_AGAIN, "stream queue full");
  // an event on the producer's stream, taken from the pool (or created)
  hipEvent_t ev = nullptr;
  if (!s->ready_pool.empty()) {
    ev = s->ready_pool.back();
    s->ready_pool.pop_back();
  }
  lk.unlock();
  (void)hipSetDevice(s->cfg.device);
  if (!ev && (rc = check(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "ready event")) != HZD_OK) return rc;
  if ((rc = check(hipEventRecord(ev, reinterpret_cast<hipStream_t>(ready_stream)), "ready record")) != HZD_OK) {
    lk.lock();
    s->ready_pool.push_back(ev);
    return rc;
  }
  lk.lock();
  if (st->closing || s->stop || st->queued >= kMaxQueuedPerStream) {   // changed while unlocked
    s->ready_pool.push_back(ev);
    return st->queued >= kMaxQueuedPerStream ? fail(HZD_E_AGAIN, "stream queue full")
                                             : fail(HZD_E_CLOSED, "stream is closing");
  }
  Job j;
  j.ready = ev;
  j.st = st;
  j.fr = *frame;
  j.fr.params = nullptr;
  j.cb = cb;
  j.user = user;
  j.ticket = st->next_ticket++;
  j.t_submit = now_ns();
  st->queued++;
  st->pending.insert(j.ticket);
  s->queue.push_back(j);
  s->stats.submitted++;
  if (ticket) *ticket = j.ticket;
  s->cv.notify_all();
  clear_error();
  return HZD_OK;
}

int hzd_stream_wait(hzd_stream* st, uint64_t ticket, int64_t timeout_ns, int64_t* latency_ns) {
  if (!st) return fail(HZD_E_INVAL, "stream is NULL");
  hzd_server* s = st->srv;
  std::unique_lock<std::mutex> lk(s->mu);
  if (ticket == 0 || ticket >= st->next_ticket || (!st->pending.count(ticket) && !st->done.count(ticket)))
    return fail(HZD_E_INVAL, "unknown or already collected ticket %llu", (unsigned long long)ticket);
  auto ready = [&] { return st->done.count(ticket) > 0; };
  if (timeout_ns < 0) {
    st->cv.wait(lk, ready);
  } else if (!st->cv.wait_for(lk, std::chrono::nanoseconds(timeout_ns), ready)) {
    return fail(HZD_E_TIMEOUT, "ticket %llu not complete", (unsigned long long)ticket);
  }
  const auto res = st->done[ticket];
  st->done.erase(ticket);
  if (latency_ns) *latency_ns = res.second;
  return res.first;
}

int hzd_stream_arena_size(const hzd_params* params, int32_t width, int32_t height, size_t* bytes) {
  if (!bytes) return fail(HZD_E_INVAL, "bytes is NULL");
  int rc = validate_params(params);
  if (rc) return rc;
  if ((rc = validate_size(*params, width, height, 0)) != HZD_OK) return rc;
  *bytes = kWorkspacesOff + stream_ws_bytes(*params, width, height) * kSlotsPerStream;
  clear_error();
  return HZD_OK;
}

int hzd_stream_state(hzd_stream* st, float* A_host, int32_t* sel_host) {
  if (!st) return fail(HZD_E_INVAL, "stream is NULL");
  int slot;
  {
    std::lock_guard<std::mutex> lk(st->srv->mu);
    slot = st->last_slot;
  }
  if (slot < 0) return fail(HZD_E_AGAIN, "no frame of this stream has completed yet");
  (void)hipSetDevice(st->srv->cfg.device);
  if (A_host) {
    int rc = check(hipMemcpy(A_host, st->state_dev + 256 * slot, 12, hipMemcpyDeviceToHost), "state copy");
    if (rc) return rc;
  }
  if (sel_host) {
    const volatile int32_t* cell = st->status[slot];
    for (int k = 0; k < 4; ++k) sel_host[k] = cell[k];
  }
  clear_error();
  return HZD_OK;
}

int hzd_stream_close(hzd_stream* st) {
  if (!st) return fail(HZD_E_INVAL, "stream is NULL");
  hzd_server* s = st->srv;
  std::unique_lock<std::mutex> lk(s->mu);
  st->closing = true;
  st->cv.wait(lk, [&] { return st->queued == 0 && st->inflight == 0; });
  s->arena.release(st->arena_off, st->arena_len);
  s->streams.erase(std::remove(s->streams.begin(), s->streams.end(), st), s->streams.end());
  s->stats.open_streams = (int)s->streams.size();
  s->stats.arena_used = s->arena.used();
  lk.unlock();
  for (int k = 0; k < kSlotsPerStream; ++k) status_cells().put(st->status[k]);
  delete st;
  clear_error();
  return HZD_OK;
}

int hzd_server_stats_get(hzd_server* s, hzd_server_stats* out) {
  if (!s || !out) return fail(HZD_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->inflight = s->inflight_frames;
  out->arena_used = s->arena.used();
  clear_error();
  return HZD_OK;
}

}  // extern "C"
