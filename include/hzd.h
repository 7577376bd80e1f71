/*
 * hzd.h -- C ABI of the MI355X (gfx950) per-frame dark-channel-prior dehazing
 * library (Hazedefy, arXiv 2512.16609).
 *
 * The library recovers the scene radiance J from a hazy frame I under the
 * atmospheric scattering model I = J t + A (1 - t) (paper Sec. III, Eq. (1))
 * by estimating the global airlight A and the transmission t.  One frame runs
 * the paper's per-frame steps (Sec. V):
 *
 *   optional resize to a working size                        Sec. V, step 1
 *   channel minimum + patch erosion -> dark channel D        Sec. IV-A, Eq. (2)
 *   fractional top-pixel average    -> airlight A            Sec. IV-B, Eq. (3)
 *   transmission with lower bound   -> t                     Sec. IV-C, Eqs. (4)-(5)
 *   guided-filter refinement (offline mode only)             Sec. IV-D, Eq. (6)
 *   radiance recovery, gamma, optional colour balance       Sec. IV-E, Eqs. (7)-(8)
 *
 * Conventions for every call:
 *   - Pixel buffers are HIP device pointers to packed 8-bit RGB, row-major,
 *     channel-interleaved (R,G,B per pixel), with a row pitch in bytes
 *     (pitch >= 3 * width).  The caller owns them; they must stay valid until
 *     the work is complete in stream order (frame/batch) or until the ticket
 *     completes (served).
 *   - `hip_stream` is a hipStream_t (NULL = the null stream).  frame/batch
 *     calls are asynchronous: they return once the work is enqueued.
 *   - Every call returns an hzd_status.  Arguments are validated before any
 *     device work is enqueued, so a call that returns an error has no side
 *     effects.  hzd_last_error() gives a thread-local description.
 *   - No call aborts or throws across the ABI.  frame/batch never allocate
 *     device memory: scratch comes from the caller's workspace.
 */
#ifndef HZD_H
#define HZD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HZD_ABI_VERSION 4

typedef enum {
  HZD_OK = 0,
  HZD_E_INVAL = -1,        /* an argument is out of range or inconsistent      */
  HZD_E_NOMEM = -2,        /* workspace/arena too small                        */
  HZD_E_DEVICE = -3,       /* a HIP call failed (detail in hzd_last_error)     */
  HZD_E_AGAIN = -4,        /* no admission budget or queue space right now     */
  HZD_E_CLOSED = -5,       /* the stream/server is closed; the frame was dropped */
  HZD_E_UNSUPPORTED = -6,  /* valid request outside what the library implements */
  HZD_E_TIMEOUT = -7       /* hzd_stream_wait timed out                        */
} hzd_status;

/* Sec. I / Sec. V: real-time video mode skips the guided filter; offline
 * image mode refines t with it (Fig. 2, "Image Mode?" branch). */
typedef enum { HZD_MODE_REALTIME = 0, HZD_MODE_OFFLINE = 1 } hzd_mode;

/* Transmission estimate (Sec. IV-C).
 *   HZD_TX_HE    t = max(1 - omega * dark(I / A), t0), where dark(I/A) is the
 *                patch minimum of min_c I^c / A^c (the dark-channel form).
 *   HZD_TX_PAPER t = max(1 - omega * min_c I^c(x) / max_c A^c, t0), the
 *                pointwise expression printed as Eq. (4). */
typedef enum { HZD_TX_HE = 0, HZD_TX_PAPER = 1 } hzd_tx;

/* Precision of the stored transmission map, and the output bound of each.
 * The only floating-point map that crosses memory is the refined t of offline
 * mode with a balance (color_balance 1) or the adaptive gamma, between the
 * guided filter and the reconstruction that needs the frame-wide sums.  J and
 * the gamma of Eq. (8) are always formed in binary32.
 *   HZD_PREC_FP32  t binary32 everywhere.  Output within 1 LSB of the FP64
 *                  reading of the method in every mode; t within 1e-5
 *                  relative.
 *   HZD_PREC_FP16  that map is stored as binary16 (half its traffic; the sums
 *                  use the same rounded values); everywhere else t never
 *                  leaves registers, so the results equal FP32's bit for bit.
 *                  For the stored map t is within 1e-3 relative, and the
 *                  output within the bound that the binary16 rounding
 *                  (2^-11 relative) implies through Eqs. (7)-(8) and the
 *                  gains: 1 LSB on the test frames for gamma <= 1.2 (the
 *                  default), up to 2 LSB at gamma 1.8, 4 at 2.2 and 12 at 3.0,
 *                  the error concentrating next to black, where Eq. (8) is
 *                  steepest.  Offline percentile white balance (color_balance
 *                  2) is refused at FP16 (HZD_E_UNSUPPORTED). */
typedef enum { HZD_PREC_FP32 = 0, HZD_PREC_FP16 = 1 } hzd_prec;

typedef enum {
  HZD_PRESET_REALTIME = 0,       /* patch 15, omega .95, t0 .1, top .001, gamma 1.2 */
  HZD_PRESET_OFFLINE = 1,        /* as REALTIME + guided filter r 60, eps 1e-3, colour balance */
  HZD_PRESET_PAPER_REALTIME = 2  /* the shipped real-time values of Sec. IV-C: omega .5, t_min .05, TX_PAPER */
} hzd_preset;

/* Parameters of one frame.  Ranges are checked by every call.
 *   size           must equal sizeof(hzd_params)
 *   mode           hzd_mode
 *   patch          odd side of the square patch Omega of Eq. (2), 1..31 (paper: 15)
 *   omega          transmission weight of Eq. (4), [0, 1]
 *   t0             lower bound t_min of Eq. (5), (0, 1]
 *   top_frac       fraction of pixels averaged in Eq. (3), (0, 1];
 *                  K = max(1, floor(top_frac * W * H)); ties in D are broken
 *                  by the lower raster index y * W + x
 *   alpha          airlight scale of Eq. (3), (0, 1] (paper: 0.8)
 *   gamma          gamma of Eq. (8), [0.1, 10]
 *   gf_radius      guided-filter box radius r (OFFLINE), 1..64
 *   gf_eps         guided-filter regulariser (OFFLINE), [1e-8, 1]; the guide is
 *                  the BT.601 luma of the hazy input scaled to [0, 1].  The
 *                  filter's a and b are kept in fixed point between its two
 *                  stages: int32 with k = floor(log2((2^31 - 1) / B))
 *                  fractional bits, B = 1 + 1 / (4 sqrt(gf_eps)), while 2^-k
 *                  <= 1e-6 t0, else int64 (workspace 16 instead of 8 bytes
 *                  per pixel for that map), so the rounding moves t by at
 *                  most a tenth of its tolerance
 *   color_balance  the balance stage of Sec. IV-E, on the gamma-corrected image:
 *                  0 = none; 1 = gray-world gains g_c = mean(mu) / mu_c, where
 *                  mu_c is the channel mean (1 when mu_c = 0), clamped to 255;
 *                  2 = percentile ("simple") white balance: per channel the
 *                  black point lo is the (k+1)-th smallest and the white point
 *                  hi the (k+1)-th largest of the unbalanced output codes
 *                  RNE(J_gamma), k = floor(wb_percentile * W * H), and the
 *                  channel becomes clamp((J_gamma - lo) * 255 / (hi - lo), 0,
 *                  255) (unchanged when hi <= lo).  With 2, offline mode
 *                  needs precision FP32 (HZD_E_UNSUPPORTED otherwise): the
 *                  percentile decisions are taken on codes of J_gamma, which a
 *                  binary16 t map would move.
 *   tx             hzd_tx
 *   precision      hzd_prec
 *   resize_width, resize_height
 *                  working size of Sec. V step 1 (paper default 640 x 480):
 *                  both 0 = process frames at their own size; else both in
 *                  1..16384, and every frame is first resampled to that size
 *                  (input width and height <= 32768).  The resampling is
 *                  bilinear with pixel centres aligned: output sample i of an
 *                  axis of n_in inputs and n_out outputs sits at source
 *                  coordinate s = (i + 1/2) n_in / n_out - 1/2, taken as 0 when
 *                  negative, between taps floor(s) and min(floor(s) + 1,
 *                  n_in - 1); the weight of the second tap is frac(s) rounded
 *                  half up to a multiple of 2^-11, and the weighted sum (rows,
 *                  then columns) is rounded half up to uint8, all in exact
 *                  integers.  Every later step, dst and the aux outputs are at
 *                  the working size.
 *   airlight_smoothing
 *                  lam in [0, 1): temporal average of the airlight over the
 *                  frames of one stream, against the flicker that Sec. V
 *                  addresses with the top-fraction average.  The frame's A is
 *                  lam * A_prev + (1 - lam) * Ahat, where Ahat is its own
 *                  Eq. (3) estimate and A_prev the previous frame's A as
 *                  stored in the stream's airlight state; the sum is formed
 *                  in double as (lam * A_prev) + ((1 - lam) * Ahat) and rounded
 *                  to float.  0 (the default) = every frame on its own.  A
 *                  frame call with lam > 0 needs hzd_frame.airlight_state.
 *   gamma_adaptive 0/1: the "gamma-adaptive" correction the abstract names,
 *                  for which the paper gives no rule.  With 1 each frame takes
 *                  gamma = ln(mu) / ln(gamma_target), where mu is the mean
 *                  BT.601 luma of its recovered J (Eq. (7), clamped) divided
 *                  by 255, floored at 2^-20; gamma is clamped to [1/2, 2] and
 *                  `gamma` is not used.  mu^(1/gamma) = gamma_target, so the
 *                  frame's mean luma is mapped to the target.  Costs one more
 *                  pass over the frame (the sums of J must be complete
 *                  before any pixel is corrected).
 *   gamma_target   tau in (0, 1), the mean luma aimed for (default 0.5).
 *   wb_percentile  p in [0, 0.49]: fraction of pixels ignored at each end of
 *                  each channel by the percentile white balance (default 0.02). */
typedef struct hzd_params {
  uint32_t size;
  int32_t mode;
  int32_t patch;
  float omega;
  float t0;
  float top_frac;
  float alpha;
  float gamma;
  int32_t gf_radius;
  float gf_eps;
  int32_t color_balance;
  int32_t tx;
  int32_t precision;
  int32_t resize_width;
  int32_t resize_height;
  float airlight_smoothing;
  int32_t gamma_adaptive;
  float gamma_target;
  float wb_percentile;
} hzd_params;

/* One frame: device pointers and geometry (see the conventions above).
 * width, height (>= 1, width * height < 2^31, width < 2^24; wider frames
 * return HZD_E_UNSUPPORTED) are the input size; dst and
 * the aux outputs have the output size, which is the input size unless the
 * frame's params resize it.  src and dst must not overlap.
 * params: NULL = the params given to the call; in a batch, a per-frame
 * override (host pointer, read during the call only).
 * airlight_state: NULL, or a device pointer to the 16-byte airlight state of
 * the stream this frame belongs to: {float A[3]; uint32_t frames}, zeroed by
 * the caller before the stream's first frame.  The frame reads it (blending
 * when frames > 0 and airlight_smoothing > 0) and writes its own A back, in
 * stream order.  Frames of one call must not share a state (HZD_E_INVAL). */
typedef struct hzd_frame {
  const uint8_t* src;
  int64_t src_pitch;
  uint8_t* dst;
  int64_t dst_pitch;
  int32_t width;
  int32_t height;
  const hzd_params* params;
  float* airlight_state;
} hzd_frame;

/* Optional per-frame device outputs for inspection (NULL = not written).
 * width and height below are the output size.
 *   A_out    3 floats: A^c of Eq. (3) on the 0..255 scale
 *   sel_out  4 int32: {K, vstar, cutoff, status}; the selected set of
 *            Eq. (3) is {D > vstar} U {D == vstar and raster index <= cutoff}.
 *            status is the selection's own consistency check, 0 when the
 *            per-row counts agree with the histogram of D.  Nonzero means
 *            the device produced inconsistent intermediate data (a fault):
 *            1 = the count of pixels above vstar or the cut pixel disagrees,
 *            or the histogram does not hold W*H pixels (A was formed, the
 *            result is not trustworthy); 2 = no row holds
 *            the cut (A is set to 0 and the output is undefined).  A frame
 *            or batch call returns before its kernels run, so a caller that
 *            needs this check passes sel_out (device or host-mapped memory)
 *            and reads status once the stream has completed; served frames
 *            report a nonzero status as HZD_E_DEVICE.
 *   dark_out width*height bytes (pitch = width): D of Eq. (2)
 *   t_out    width*height floats: the t used in Eq. (7) (after the guided
 *            filter in OFFLINE mode)
 *   J_out    width*height*3 floats: J of Eq. (7) clamped to [0, 255], before
 *            the gamma of Eq. (8) */
typedef struct hzd_frame_aux {
  float* A_out;
  int32_t* sel_out;
  uint8_t* dark_out;
  float* t_out;
  float* J_out;
} hzd_frame_aux;

/* Fill *p with a preset (hzd_preset).  Returns HZD_E_INVAL for an unknown preset. */
int hzd_params_default(hzd_params* p, int32_t preset);

/* Bytes of device workspace that hzd_dehaze_frame (n = 1) or hzd_dehaze_batch
 * needs for these frames (width/height/params are read; pointers are not).
 * The workspace must be 256-byte aligned. */
int hzd_workspace_size(const hzd_params* params, const hzd_frame* frames, int32_t n,
                       size_t* bytes);

/* Dehaze one frame (Sec. V, steps 2-7) on `hip_stream`.
 * workspace: device memory of at least hzd_workspace_size bytes, owned by the
 * caller, used exclusively by this call until it completes in stream order;
 * its contents before the call do not matter (the call zeroes the state it
 * accumulates into, inside its first kernel or, when the launches may be
 * replayed from a graph, with a kernel of its own).  aux may be NULL.  Errors: INVAL (arguments), NOMEM (workspace too small),
 * UNSUPPORTED (e.g. patch > 31), DEVICE (a launch failed). */
int hzd_dehaze_frame(const hzd_params* params, const hzd_frame* frame,
                     const hzd_frame_aux* aux, void* workspace, size_t ws_bytes,
                     void* hip_stream);

/* Dehaze n independent frames of possibly different sizes and parameters as
 * one batch: frames sharing (mode, patch, tx, colour balance, precision,
 * radius, resize, adaptive gamma) are processed by the same launches, up to
 * 16 frames per launch group.  Several launch groups run concurrently on
 * streams the library keeps per calling thread (ordered after the work already
 * on hip_stream, which in turn waits for all of them), unless hip_stream is
 * being captured into a graph; so the frames of one call must not write
 * overlapping dst or aux memory.  Each frame's result equals its
 * hzd_dehaze_frame result bit for bit.  aux: NULL or an array of n. */
int hzd_dehaze_batch(const hzd_params* params, const hzd_frame* frames, int32_t n,
                     const hzd_frame_aux* aux, void* workspace, size_t ws_bytes,
                     void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as hzd_dehaze_frame, with the workspace taken from a static
 * device array of HZD_NOALLOC_SCRATCH_BYTES that the library holds on each
 * device it runs on until the process ends.  The frame's hzd_workspace_size
 * must not exceed that size (a 1920x1080 offline frame with int32 a, b fits in
 * 59.4 MiB; with int64 a, b (small gf_eps or t0) it needs 75.2 MiB; a 3840x2160
 * offline frame does not): larger requests return HZD_E_NOMEM before any
 * device work.  hip_stream must belong to the current device (HZD_E_INVAL
 * otherwise).  The call allocates nothing: no hipMalloc/hipFree, no graph,
 * event or stream creation; kernels are launched directly on hip_stream
 * (the graph cache and profiling are not used).  Every call on one device
 * shares that device's array and leaves its contents behind; the kernels
 * clear what must start at zero.  Calls that overlap on one device (other
 * streams or threads, before the previous call has completed in stream
 * order) race on the array: the caller serialises them. */
#define HZD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int hzd_dehaze_frame_noalloc(const hzd_params* params, const hzd_frame* frame,
                             const hzd_frame_aux* aux, void* hip_stream);

/* ---------------------------------------------------------------- serving
 * A server owns a scheduler thread and a few HIP streams on one device.
 * Streams of frames (each of one size and one parameter set) are opened
 * against it; each opened stream reserves its device state and workspace in
 * the caller's arena (admission by HBM budget).  Submitted frames are queued
 * and launched in batches as slots free up, so frames that arrive while
 * others run join the next launch (continuous batching).  The method is
 * feed-forward per frame (Sec. V), so a served frame's output equals its
 * hzd_dehaze_frame output. */
typedef struct hzd_server hzd_server;
typedef struct hzd_stream hzd_stream;

/* size              = sizeof(hzd_server_config)
 * device            HIP device ordinal
 * arena, arena_bytes caller-owned device memory (256-byte aligned) that
 *                   stream state and workspaces are carved from
 * max_inflight      frames on the device at once (>= 1)
 * frames_per_launch largest batch per launch (1..16)
 * hip_streams       HIP streams the server launches on (1..8)             */
typedef struct hzd_server_config {
  uint32_t size;
  int32_t device;
  void* arena;
  size_t arena_bytes;
  int32_t max_inflight;
  int32_t frames_per_launch;
  int32_t hip_streams;
} hzd_server_config;

/* Completion callback, called on the scheduler thread.  latency_ns is from
 * hzd_stream_submit to the host observing completion. */
typedef void (*hzd_done_fn)(void* user, uint64_t ticket, int32_t status, int64_t latency_ns);

int hzd_server_create(const hzd_server_config* cfg, hzd_server** out);
/* Cancels queued frames (their callbacks get HZD_E_CLOSED), waits for frames
 * on the device, closes all streams and frees the server. */
int hzd_server_destroy(hzd_server* s);

/* Arena bytes that hzd_stream_open reserves for a stream of width x height
 * frames with these parameters (a multiple of 256). */
int hzd_stream_arena_size(const hzd_params* params, int32_t width, int32_t height, size_t* bytes);
/* Open a stream of width x height frames with these parameters.
 * HZD_E_AGAIN when the arena cannot hold its state right now.  The server
 * keeps the stream's airlight state (airlight_smoothing); a stream with
 * smoothing has one frame on the device at a time, since each frame starts
 * from its predecessor's airlight. */
int hzd_stream_open(hzd_server* s, const hzd_params* params, int32_t width, int32_t height,
                    hzd_stream** out);
/* Queue one frame (frame->width/height must match the stream; params and
 * airlight_state ignored).
 * ready_stream: the hipStream_t that produced src and last used dst (NULL =
 * the null stream).  The call records an event on it, and the launch that
 * takes the frame waits for that event, so the frame is read and written
 * only after the work enqueued on ready_stream before this call.
 * Returns at once with a ticket.  HZD_E_AGAIN when the queue is full. */
int hzd_stream_submit(hzd_stream* st, const hzd_frame* frame, void* ready_stream, hzd_done_fn cb,
                      void* user, uint64_t* ticket);
/* Wait until `ticket` completes (timeout_ns < 0: forever).  Returns the
 * frame's status, or HZD_E_TIMEOUT.  latency_ns (nullable): nanoseconds from
 * submit to the scheduler observing completion.  A ticket can be collected
 * once: waiting again for it (or for a ticket never issued) returns
 * HZD_E_INVAL at once. */
int hzd_stream_wait(hzd_stream* st, uint64_t ticket, int64_t timeout_ns, int64_t* latency_ns);
/* Per-stream device state as of the last completed frame: A (3 floats) and
 * {K, vstar, cutoff, status} (4 int32, as hzd_frame_aux.sel_out); host
 * pointers, either may be NULL. */
int hzd_stream_state(hzd_stream* st, float* A_host, int32_t* sel_host);
/* Wait for the stream's frames, release its arena space and free it. */
int hzd_stream_close(hzd_stream* st);

typedef struct hzd_server_stats {
  uint64_t submitted, completed, failed, launches;
  uint64_t arena_used, arena_bytes;
  int32_t open_streams, inflight;
} hzd_server_stats;
int hzd_server_stats_get(hzd_server* s, hzd_server_stats* out);

/* ------------------------------------------------------------ tuning
 * Tile shapes are tuning knobs only: the guided filter's box sums are exact
 * integers and every other reduction is integer or per pixel, so each result
 * is bit-identical for every allowed tile shape.  The table is process-wide
 * and keyed by frame size ((0, 0) = default for sizes without an entry).
 *   gf_rows  output rows per guided-filter block, a multiple of 8 in 8..256.
 *            With neither an entry for the size nor a (0, 0) entry, each
 *            launch picks the smallest of 16, 32, 64, 128 at which its
 *            frames' guided-filter blocks fit one round on the device (16 for
 *            one 1080p frame, taller for 4K frames and large batches);
 *            hzd_tile_config_get then reports 16. */
typedef struct hzd_tile_config {
  int32_t gf_rows;
} hzd_tile_config;
/* Set (cfg != NULL) or remove (cfg == NULL) the entry for width x height. */
int hzd_tile_config_set(int32_t width, int32_t height, const hzd_tile_config* cfg);
/* The configuration frames of this size use. */
int hzd_tile_config_get(int32_t width, int32_t height, hzd_tile_config* cfg);
/* Autotuner: time `reps` calls of hzd_dehaze_frame on this frame for each
 * candidate tile shape (HIP events on hip_stream, which is synchronised),
 * store the fastest in the table for the frame's size and return it in *best.
 * The frame's dst is overwritten; its airlight state is neither read nor
 * written.  If the environment variable
 * HZD_AUTOTUNE_CACHE names a file, results are appended to it and entries
 * found there are loaded into the table on first use. */
int hzd_autotune(const hzd_params* params, const hzd_frame* frame, void* workspace, size_t ws_bytes,
                 void* hip_stream, int32_t reps, hzd_tile_config* best);

/* ------------------------------------------------------------ graphs
 * The launches of one pipeline can be captured into a HIP graph and replayed.
 * Graphs are cached process-wide, keyed by the complete launch arguments
 * (frame sizes, parameters, pixel/workspace/aux pointers), so they pay off
 * when callers reuse buffers (frame pools, server slots).  capacity = 0
 * turns the cache off (every call launches its kernels directly); the
 * default is 0.  Calls on the null stream and calls made while profiling is
 * enabled always launch directly.  A call made while the caller captures
 * hip_stream launches directly into the caller's graph.  Graphs are keyed
 * by device too.  Shrinking the cache synchronises the current device
 * before destroying evicted graphs. */
int hzd_graph_cache(int32_t capacity);

/* ------------------------------------------------------------ profiling
 * Per-stage timing with HIP events recorded on the stream each kernel is
 * launched on.  While enabled (process-wide), every kernel launch of the
 * pipeline is bracketed by a pair of events.  hzd_profile_read synchronises
 * the recorded events, adds each launch's elapsed time to its stage entry
 * and returns up to `cap` entries (stage name, launches, total ms);
 * reset != 0 clears the totals afterwards.  Launches into a graph that the
 * caller is capturing are not timed. */
typedef struct hzd_profile_entry {
  char name[24];
  uint64_t launches;
  double total_ms;
} hzd_profile_entry;
int hzd_profile_enable(int32_t on);
int hzd_profile_read(hzd_profile_entry* out, int32_t cap, int32_t* n, int32_t reset);

const char* hzd_status_str(int32_t status);
/* Thread-local text for the last failing call on this thread ("" if none). */
const char* hzd_last_error(void);
int hzd_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HZD_H */
