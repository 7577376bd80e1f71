// Internal structures shared by the C-ABI layer (hzd_api.cpp) and the gfx950
// kernels (hzd_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hzd.h"

namespace hzd {

constexpr int kMaxBatch = 16;   // frames per launch (descriptors travel in kernel arguments)
constexpr int kMaxHalfPatch = 15;
constexpr int kMaxRadius = 64;  // guided-filter radius supported by the 256-column strip kernels

// Per-frame device state at the start of each frame's workspace.  Its sums
// start at zero in one of three ways:
//  - direct launches (kFdFresh): a leading block of k_dark per frame zeroes
//    the frame's state and then publishes the launch's epoch, a value no
//    earlier launch used, in it; the frame's tile blocks wait for that epoch
//    before merging their histograms;
//  - launches recorded into a graph (replays would repeat the epoch): the init
//    kernel zeroes everything before k_dark (the white-balance histograms only
//    for frames that use them);
//  - frames of the one-block selection: k_dark writes per-tile histograms
//    whole, and that selection zeroes the later sums itself.
// Sums that many blocks merge with integer atomics are spread over slots (block
// index mod slots), which keeps same-address contention low; integer sums make
// the slot choice irrelevant to the result.
constexpr int kHistSlots = 8;
constexpr int kCbSlots = 64;
struct FrameState {
  uint32_t hist[kHistSlots][256];       // histogram of the dark channel D, per slot
  float A[4];                           // airlight A^c (0..255 scale)
  int32_t sel[4];                       // K, vstar, cutoff, consistency flag (0 = ok)
  uint32_t rows_done;                   // row blocks of the selection that have written their records
  uint32_t rows_pad[3];
  unsigned long long cb[kCbSlots][4];   // sum of J_gamma^c in 2^-23 fixed point, per slot
  unsigned long long luma[kCbSlots];    // adaptive gamma: sum of the BT.601 luma of J in 2^-16 fixed point
  uint32_t wbh[kHistSlots][3][256];     // percentile white balance: histograms of the codes RNE(J_gamma^c), per slot
  unsigned long long epoch;             // direct launches: the launch's epoch once the state above is zero
  unsigned long long pad_;
};
static_assert(sizeof(FrameState) <= 40960, "FrameState too large");
static_assert(offsetof(FrameState, cb) % 16 == 0 && offsetof(FrameState, wbh) % 16 == 0 &&
                  offsetof(FrameState, epoch) % 16 == 0,
              "the state is zeroed with 16-byte stores");

// Per-row record of the airlight selection pass: the row's pixels with
// D == vstar (ties) and D > vstar, counted and summed per channel.  A row's
// sums stay below W * 255 < 2^32 (frames are at most kMaxWidth wide).
constexpr int kMaxWidth = (1 << 24) - 1;
struct RowSel {
  uint32_t ties, above;
  uint32_t tsum[3];
  uint32_t gsum[3];
};
static_assert(sizeof(RowSel) == 32, "RowSel layout");
static_assert((unsigned long long)kMaxWidth * 255ull < (1ull << 32), "a row's sums fit 32 bits");

// Everything one frame needs on the device, passed by value in kernel arguments.
struct FrameDev {
  const uint8_t* src;
  uint8_t* dst;
  int64_t src_pitch;
  int64_t dst_pitch;
  FrameState* st;
  uint8_t* D;        // dark channel, pitch D_pitch
  uint8_t* E;        // per-channel erosions (packed RGB8), pitch E_pitch
  RowSel* rowsel;    // per row: selection counts and sums (one record per row)
  uint16_t* hpart;   // small frames: each k_dark tile's 256-bin histogram of D (the one-block selection sums them)
  uint2* LP;         // offline: {luma*1000, t * 2^28} per pixel (pitch W)
  void* AB;          // offline: guided-filter a, b in fixed point, int2 or longlong2 (GroupKey.ab64), pitch W
  ulonglong2* PGa;   // offline: per column and aligned 8-row chunk, sums of {L, P} over the chunk's group of 8 up to it
  ulonglong2* PGb;   // offline: the same for {L^2, L*P}
  longlong2* S8ab;   // offline: per column and chunk, sums of {a, b} (fixed point)
  void* tmap;        // offline + colour balance: refined t (float or half, pitch W)
  float* A_out;
  int32_t* sel_out;
  uint8_t* dark_out;
  float* t_out;
  float* J_out;
  float* A_state;    // stream airlight state {A[3], frames} (NULL = none)
  int32_t W, H;
  int32_t D_pitch, E_pitch;
  int32_t K;
  int32_t radius;
  float omega, t0, alpha, inv_gamma, gamma_log_bias;  // gamma_log_bias = log2(255) (1 - 1/gamma)
  float eps;
  float ab_scale;                                    // fixed-point scale 2^k of a, b
  int32_t gf_rows;   // output rows per guided-filter block
  float ema;         // temporal airlight weight lam (0 = none)
  float gamma_target;  // tau of the adaptive gamma
  int32_t wb_k;      // percentile white balance: k = floor(p W H)
  uint32_t flags;    // kFd* bits
};

// FrameDev.flags
constexpr uint32_t kFdGammaOne = 1u;        // gamma == 1: Eq. (8) is the identity
constexpr uint32_t kFdAligned = 2u;         // src, dst and both pitches are multiples of 4
constexpr uint32_t kFdEmaFirst = 4u;        // the stream's first frame: ignore the stored airlight
constexpr uint32_t kFdGammaAdaptive = 8u;   // per-frame gamma from the luma sums of J
constexpr uint32_t kFdWbPercentile = 16u;   // balance by percentile stretch (else gray-world)
constexpr uint32_t kFdNoHist = 32u;         // k_dark skips the histogram (the one-block selection builds it)
constexpr uint32_t kFdFresh = 64u;          // no init kernel: leading k_dark blocks zero the frames' state

struct Batch {
  int32_t n;
  int32_t tile0[kMaxBatch + 1];  // per-launch prefix of blocks per frame
  unsigned long long epoch;      // kFdFresh: nonzero, unique to the launch
  FrameDev f[kMaxBatch];
};
static_assert(sizeof(Batch) <= 4000, "kernel argument block too large");

// Resampling of Sec. V step 1 for one frame: the caller's frame (Ws x Hs) to
// the working-size copy in the frame's workspace (Wo x Ho, pitch dst_pitch),
// which every later stage reads as its input.
constexpr int kResizeMaxOut = 16384;   // output width/height limit
constexpr int kResizeMaxIn = 32768;    // input width/height limit (keeps tap arithmetic in 32 bits)
constexpr int kResizeBits = 11;        // fractional bits of the bilinear weights
struct ResizeDev {
  const uint8_t* src;
  int64_t src_pitch;
  uint8_t* dst;
  int32_t dst_pitch;
  int32_t Ws, Hs, Wo, Ho;
};

struct ResizeBatch {
  int32_t n;
  int32_t tile0[kMaxBatch + 1];
  ResizeDev f[kMaxBatch];
};

// Group-wide kernel switches (identical for all frames of one launch).
struct GroupKey {
  int32_t mode, half_patch, tx, cb, fp16, radius, resize, gadapt, ab64;
};

// Fixed-point storage of the guided filter's a and b (Eq. (6)): a value v is
// kept as rint(v 2^k).  |a| <= 1 / (4 sqrt(eps)) for a guide and an input in
// [0, 1], and |b| <= 1 + |a|, so with B = 1 + 1 / (4 sqrt(eps)) int32 holds
// k = floor(log2((2^31 - 1) / B)) fractional bits.  The rounding moves the
// refined t by at most 2^-k (the box means of a and b each by 2^-(k+1), and
// the guide is at most 1).  That must stay far inside the 1e-5 relative
// tolerance of t >= t0: int32 is used while 2^-k <= 1e-6 t0, otherwise int64
// with k = floor(log2((2^63 - 1) / (B (2r+1)^2))), which keeps the stage-2 box
// sums of up to (2r+1)^2 values inside int64 (ab_fixed_point).
struct AbFixed {
  bool wide;   // int64 storage
  int bits;    // k
};
AbFixed ab_fixed_point(float eps, float t0, int radius);

// Compute units of the current device (cached per device; 256 if the query fails).
int device_cu_count();

// Launches (hzd_kernels.hip).  Each fills b.tile0 for its own tiling.
hipError_t launch_resize(ResizeBatch r, hipStream_t s);
hipError_t launch_init(Batch b, hipStream_t s);
hipError_t launch_dark(Batch b, const GroupKey& g, bool write_E, hipStream_t s);
hipError_t launch_select(Batch b, hipStream_t s);        // row records; the frame's last row block ends the selection
// One block per frame for small frames (select_one_fits); the frames' k_dark
// launch skips its histogram (kFdNoHist) and the init kernel is not needed.
hipError_t launch_select_one(Batch b, hipStream_t s);
constexpr int kOneVecMax = 8;    // 16-byte D vectors per thread of the one-block selection
__host__ __device__ inline int dark_tiles(int W, int H) { return ((W + 63) / 64) * ((H + 31) / 32); }   // k_dark's 64 x 32 tiles
// The one-block selection numbers D's vectors tile by tile (128 slots per
// k_dark tile) and gives each of its 1024 threads kOneVecMax slots.
inline bool select_one_fits(int W, int H) {
  return W <= 1024 && H <= 2048 && dark_tiles(W, H) * 128 <= 1024 * kOneVecMax;
}
hipError_t launch_gf_prep(Batch b, const GroupKey& g, hipStream_t s);
hipError_t launch_gf_ab(Batch b, const GroupKey& g, hipStream_t s);
hipError_t launch_gf_q(Batch b, const GroupKey& g, hipStream_t s);
// phase: 0 = write output, 1 = colour-balance sums only, 2 = apply gains and write
hipError_t launch_recon(Batch b, const GroupKey& g, int tsrc, int phase, hipStream_t s);

// Tiling shared by the workspace planner and the launches.
constexpr int kDarkTW = 64, kDarkTH = 32;
constexpr int kReconPx = 2048;   // pixels of one row per recon block (two groups of 4 per thread)
constexpr int kGfCols = 256;     // loaded columns per guided-filter strip block
constexpr int kGfRowsDefault = 16;  // output rows per guided-filter block unless tuned (a multiple of 8)
constexpr int kGfRowsMin = 8;
constexpr int kGfRowsMax = 256;    // one per-row table entry per thread of a 256-thread block
inline int recon_blocks(int W, int H) { return H * ((W + kReconPx - 1) / kReconPx); }
// Output columns of a guided-filter strip: the largest multiple of 64 that
// leaves room for the 2r halo columns in kGfCols (128 or 192 for r <= 64), so
// the 4 x gf_strip outputs of a 4-row phase split evenly over the 256 threads.
inline int gf_strip(int r) { return ((kGfCols - 2 * r) / 64) * 64; }
inline int gf_blocks(int W, int H, int r, int rows) {
  return ((W + gf_strip(r) - 1) / gf_strip(r)) * ((H + rows - 1) / rows);
}

enum { TSRC_HE = 0, TSRC_PAPER = 1, TSRC_TMAP = 2 };

}  // namespace hzd
