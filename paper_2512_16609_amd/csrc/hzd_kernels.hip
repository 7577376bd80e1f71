// gfx950 kernels of the per-frame dark-channel-prior dehazing path
// (Hazedefy, arXiv 2512.16609, Sec. IV and Sec. V).
//
// Stage map (every kernel processes a batch of frames; a block finds its
// frame from the per-launch block prefix in the kernel arguments):
//   k_resize   Sec. V step 1 (optional): bilinear resampling to the working
//              size in exact integers; the later stages read the copy
//   k_init     zero each frame's state (histogram, colour-balance and luma sums,
//              white-balance histograms when used) for launches recorded into
//              a graph; in direct launches leading blocks of k_dark do it, for
//              frames of the one-block selection k_select_one
//   k_dark     Eq. (2): channel minimum + patch erosion on LDS tiles with halo;
//              writes D (u8), optionally the per-channel erosions E, and a
//              256-bin histogram of D
//   k_select_rows   Eq. (3): vstar from the histogram, per-row counts and
//              exact sums of the ties and of the pixels above vstar; the
//              frame's last row block then finds the tie cut in raster order
//              and forms A from exact sums (optionally averaged with the
//              stream's previous airlight)
//   k_select_one    Eq. (3) for small frames in one block, from per-tile
//              histograms written by k_dark
//   k_gf_prep  offline: per-pixel luma and coarse t (Eqs. (4)-(5)) in fixed point,
//              with their column sums as prefixes inside 64-row groups
//   k_gf_ab    Eq. (6) stage 1: exact integer box sums -> a, b
//   k_gf_q     Eq. (6) stage 2: box means of a, b -> refined t (+ fused Eq. (7),
//              or the stored t map with colour-balance or luma sums)
//   k_recon    Eqs. (4)-(5) pointwise + Eq. (7) + Eq. (8) + colour balance;
//              phases for colour-balance sums, luma sums (adaptive gamma) and
//              the output
//
// Nothing here is a dense contraction, so no MFMA: the path is bound by HBM
// traffic and VALU work.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>

#include "hzd_internal.h"

namespace hzd {

// guided-filter column chunk sums (initial windows) and strip loop shape
constexpr int kChunk = 8;                                      // rows per chunk sum
constexpr int kGroupChunks = 8;                                // chunks per prefix group of the guided filter's L, P sums
constexpr int kEdgeBatch = 16;                                 // head/tail rows of a window loaded per round trip
static_assert((2 * kMaxRadius + 1) / kChunk <= 2 * kGroupChunks, "a window's whole chunks span at most three groups");
constexpr int kSelVec = 4;                                     // 16-byte D vectors per lane loaded at once

// ------------------------------------------------------------------ helpers
template <typename B>
__device__ __forceinline__ int frame_of(const B& b, int blk) {
  int f = 0;
  while (f + 1 < b.n && blk >= b.tile0[f + 1]) ++f;
  return f;
}

// Workgroups are dealt to the 8 XCDs round-robin.  Give each XCD a contiguous
// run of logical tiles so that neighbouring tiles (which share halo rows)
// meet in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  constexpr int X = 8;
  const int q = nb / X, r = nb % X;
  const int x = b % X, i = b / X;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

typedef unsigned short us2 __attribute__((ext_vector_type(2)));

// Two independent unsigned 16-bit minima in one VALU op (v_pk_min_u16).
__device__ __forceinline__ uint32_t pkmin(uint32_t a, uint32_t b) {
  us2 x = __builtin_bit_cast(us2, a), y = __builtin_bit_cast(us2, b);
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(x, y));
}

// Sliding minimum over windows of WIN consecutive values (van Herk /
// Gil-Werman): prefix minima g and suffix minima h inside aligned blocks of
// WIN values; window [i, i+WIN-1] spans at most two blocks, so its minimum is
// min(h[i], g[i+WIN-1]).  About 3 minima per output, independent of WIN.
template <int L, int WIN, int S>
__device__ __forceinline__ void sliding_min(const uint32_t (&v)[L], uint32_t (&o)[S]) {
  static_assert(L == S + WIN - 1, "window geometry");
  uint32_t g[L], h[L];
#pragma unroll
  for (int i = 0; i < L; ++i) g[i] = (i % WIN == 0) ? v[i] : pkmin(g[i > 0 ? i - 1 : 0], v[i]);
#pragma unroll
  for (int i = L - 1; i >= 0; --i)
    h[i] = (i % WIN == WIN - 1 || i == L - 1) ? v[i] : pkmin(h[i < L - 1 ? i + 1 : i], v[i]);
#pragma unroll
  for (int i = 0; i < S; ++i) o[i] = pkmin(h[i], g[i + WIN - 1]);
}


// DPP move with zero for lanes whose source is outside the row or whose row
// is masked off.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, true);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_add(uint32_t v) { return v + dpp32<CTRL, ROW_MASK>(v); }
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int32_t dpp_add(int32_t v) { return (int32_t)dpp_add<CTRL, ROW_MASK>((uint32_t)v); }
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned long long dpp_add(unsigned long long v) {
  const uint32_t lo = dpp32<CTRL, ROW_MASK>((uint32_t)v), hi = dpp32<CTRL, ROW_MASK>((uint32_t)(v >> 32));
  return v + (((unsigned long long)hi << 32) | lo);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ long long dpp_add(long long v) {
  return (long long)dpp_add<CTRL, ROW_MASK>((unsigned long long)v);
}

// Inclusive scan over the 64 lanes of a wave with DPP: Hillis-Steele inside
// each row of 16 lanes (row_shr 1, 2, 4, 8), then row_bcast:15 carries row
// totals into rows 1 and 3 and row_bcast:31 carries the first half's total
// into rows 2 and 3.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  v = dpp_add<0x111, 0xF>(v);
  v = dpp_add<0x112, 0xF>(v);
  v = dpp_add<0x114, 0xF>(v);
  v = dpp_add<0x118, 0xF>(v);
  v = dpp_add<0x142, 0xA>(v);
  v = dpp_add<0x143, 0xC>(v);
  return v;
}

// Sum over the 64 lanes of a wave, returned to every lane: the DPP scan, then
// lane 63's value read into scalar registers.  Integer types; the whole wave
// must be active.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit integers");
  const T s = wave_incl_scan(v);
  if constexpr (sizeof(T) == 8) {
    const unsigned long long u = (unsigned long long)s;
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), 63);
    return (T)(((unsigned long long)hi << 32) | lo);
  } else {
    return (T)__builtin_amdgcn_readlane((uint32_t)s, 63);
  }
}

// Sum over a 256-thread block in a fixed order; every thread gets the total.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* s_tmp) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  T x = wave_sum(v);
  if (lane == 0) s_tmp[w] = x;
  __syncthreads();
  T tot = (s_tmp[0] + s_tmp[1]) + (s_tmp[2] + s_tmp[3]);
  __syncthreads();
  return tot;
}

// Eqs. (7)-(8) for one pixel: J^c = (I^c - A^c)/t + A^c clamped to [0, 255],
// then J_gamma = 255 (J/255)^(1/gamma) = 2^(log2(J)/gamma + log2(255)(1 - 1/gamma)).
struct ReconConsts {
  float A[3];
  float inv_gamma, bias;
  int gamma_is_one;
};

__device__ __forceinline__ void recon_pixel(const ReconConsts& rc, const float I[3], float t,
                                            float J[3], float Jg[3]) {
  const float it = __builtin_amdgcn_rcpf(t);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float j = fmaf(I[c] - rc.A[c], it, rc.A[c]);
    j = __builtin_amdgcn_fmed3f(j, 0.0f, 255.0f);
    J[c] = j;
    Jg[c] = rc.gamma_is_one ? j
                            : __builtin_amdgcn_exp2f(fmaf(__builtin_amdgcn_logf(j), rc.inv_gamma, rc.bias));
  }
}

__device__ __forceinline__ uint32_t rne_u8(float v) {
  v = __builtin_amdgcn_fmed3f(v, 0.0f, 255.0f);
  return (uint32_t)__builtin_rintf(v);
}

__device__ __forceinline__ float round_half(float t) { return __half2float(__float2half_rn(t)); }

// ------------------------------------------------------------------ k_init
// Zero a frame's state up to its epoch word with 16-byte stores, spread over
// the 256 threads of a block; the white-balance histograms (the larger part of
// the state) only for frames that use them.
__device__ __forceinline__ void zero_state(const FrameDev& fd) {
  const int n16 = (int)(((fd.flags & kFdWbPercentile) ? offsetof(FrameState, epoch) : offsetof(FrameState, wbh)) / 16);
  uint4* s = reinterpret_cast<uint4*>(fd.st);
  for (int i = threadIdx.x; i < n16; i += 256) s[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ __launch_bounds__(256) void k_init(Batch b) { zero_state(b.f[blockIdx.x]); }

// ------------------------------------------------------------------ k_resize
// Sec. V step 1: bilinear resampling of the frame to the working size, in
// exact integers.  Along each axis output sample i lies at source coordinate
// s = (i + 1/2) n_in / n_out - 1/2 (0 when negative), carried as the rational
// ((2i + 1) n_in - n_out) / (2 n_out).  Its taps are floor(s) and the next
// sample, clamped to the last; the second tap's weight is frac(s) rounded half
// up to a multiple of 2^-11.  Rows are interpolated first, then columns, and
// the sum is rounded half up.
struct ResizeTap {
  int i0, i1;
  uint32_t w1;
};

__device__ __forceinline__ ResizeTap resize_tap(int i, int n_in, int n_out) {
  // (2i + 1) n_in < 2^31 for n_in <= 32768 and i < n_out <= 16384
  const int num = max((2 * i + 1) * n_in - n_out, 0);
  const uint32_t den = 2u * (uint32_t)n_out;
  const uint32_t i0 = (uint32_t)num / den;
  const uint32_t frac = (uint32_t)num - i0 * den;   // < den <= 2^15
  ResizeTap t;
  t.i0 = (int)i0;                                   // <= n_in - 1 since s < n_in - 1/2
  t.i1 = min((int)i0 + 1, n_in - 1);
  t.w1 = (frac * (2u << kResizeBits) + den) / (2u * den);
  return t;
}

// The RGB bytes of pixels x0 and x1 (x1 == x0 or x0 + 1) of a row, from
// aligned dword loads that each hold at least one needed byte (so no load
// leaves the row's allocation).
__device__ __forceinline__ void load_pixel_pair(const uint8_t* row, int x0, int x1, uint32_t& p0, uint32_t& p1) {
  const uintptr_t a = (uintptr_t)(row + 3 * (int64_t)x0);
  const uintptr_t a0 = a & ~(uintptr_t)3;
  const uintptr_t last = (a + (x1 > x0 ? 5 : 2)) & ~(uintptr_t)3;
  const uint32_t sh = (uint32_t)(a & 3);
  const uint32_t w0 = *reinterpret_cast<const uint32_t*>(a0);
  const uint32_t w1 = a0 + 4 <= last ? *reinterpret_cast<const uint32_t*>(a0 + 4) : 0u;
  const uint32_t w2 = a0 + 8 <= last ? *reinterpret_cast<const uint32_t*>(a0 + 8) : 0u;
  const uint32_t lo = __builtin_amdgcn_alignbyte(w1, w0, sh);   // bytes [a, a + 4)
  const uint32_t hi = __builtin_amdgcn_alignbyte(w2, w1, sh);   // bytes [a + 4, a + 8)
  p0 = lo & 0xFFFFFFu;
  p1 = x1 > x0 ? ((lo >> 24) | (hi << 8)) & 0xFFFFFFu : p0;
}

// One block: 4 output rows (one per wave) by 256 output columns.  The 256
// column taps are computed once per block into LDS.  Lane l of a wave
// produces columns l, l + 64, l + 128 and l + 192, so the 64 lanes of one
// load instruction read neighbouring source pixels.  Each row's bytes are
// staged in LDS and stored as consecutive dwords (the copy's pitch is a
// multiple of 16, so a dword that starts inside a row ends inside the pitch).
__global__ __launch_bounds__(256) void k_resize(ResizeBatch rb) {
  constexpr int kCols = 256, kRows = 4;
  __shared__ int s_x0[kCols];
  __shared__ uint32_t s_w[kCols];                 // weight of the second tap | (second tap != first) << 16
  __shared__ uint32_t s_row[kRows][3 * kCols / 4];
  const int blk = blockIdx.x;
  const int f = frame_of(rb, blk);
  const ResizeDev& fd = rb.f[f];
  const int tile = blk - rb.tile0[f];
  const int tiles_x = (fd.Wo + kCols - 1) / kCols;
  const int yb = (tile / tiles_x) * kRows, xb = (tile % tiles_x) * kCols;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int ncols = min(kCols, fd.Wo - xb);
  {
    const ResizeTap t = resize_tap(xb + min(tid, ncols - 1), fd.Ws, fd.Wo);
    s_x0[tid] = t.i0;
    s_w[tid] = t.w1 | ((uint32_t)(t.i1 > t.i0) << 16);
  }
  __syncthreads();
  const int y = yb + wv;
  uint8_t* srow = reinterpret_cast<uint8_t*>(s_row[wv]);
  if (y < fd.Ho) {
    const ResizeTap ty = resize_tap(y, fd.Hs, fd.Ho);
    const uint8_t* r0 = fd.src + (int64_t)ty.i0 * fd.src_pitch;
    const uint8_t* r1 = fd.src + (int64_t)ty.i1 * fd.src_pitch;
    constexpr uint32_t kOne = 1u << kResizeBits;
    const uint32_t wy1 = ty.w1, wy0 = kOne - wy1;
    uint32_t a0[4], a1[4], b0[4], b1[4], wx[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {   // every load of the lane first
      const int c = min(lane + 64 * k, ncols - 1);
      const int x0 = s_x0[c];
      wx[k] = s_w[c];
      const int x1 = x0 + (int)(wx[k] >> 16);
      load_pixel_pair(r0, x0, x1, a0[k], a1[k]);
      load_pixel_pair(r1, x0, x1, b0[k], b1[k]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int c = lane + 64 * k;
      const uint32_t wx1 = wx[k] & 0xFFFFu, wx0 = kOne - wx1;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const uint32_t h0 = wx0 * ((a0[k] >> (8 * ch)) & 255u) + wx1 * ((a1[k] >> (8 * ch)) & 255u);
        const uint32_t h1 = wx0 * ((b0[k] >> (8 * ch)) & 255u) + wx1 * ((b1[k] >> (8 * ch)) & 255u);
        const uint32_t q = (wy0 * h0 + wy1 * h1 + (1u << (2 * kResizeBits - 1))) >> (2 * kResizeBits);
        if (c < ncols) srow[3 * c + ch] = (uint8_t)q;
      }
    }
  }
  __syncthreads();
  if (y < fd.Ho) {
    uint32_t* out = reinterpret_cast<uint32_t*>(fd.dst + (int64_t)y * fd.dst_pitch + 3 * xb);
    const int nd = (3 * ncols + 3) / 4;
    for (int j = lane; j < nd; j += 64) out[j] = s_row[wv][j];
  }
}

// ------------------------------------------------------------------ k_dark
// One 64x32 output tile per block.  The (64+2h) x (32+2h) region goes to LDS
// as two planes of packed 16-bit pairs, (R | B << 16) and (G | 255 << 16), so
// each v_pk_min_u16 handles two channels; out-of-frame cells hold 255 (a
// clipped window).  Vertical van Herk per column segment, then horizontal van
// Herk per row segment, both in registers.
//
// The region is read as groups of 4 consecutive cells of one row: 12 bytes
// of the frame, covered by 3 or 4 aligned dwords (an aligned dword that holds
// a byte of the row lies in the same page as that byte), shifted into place
// with alignbyte and split into the two planes with one v_perm_b32 per plane
// and pixel.  Groups that touch the frame border take a per-cell path.  The
// outputs are packed with v_perm_b32 as well: per pixel [R, G, B, 0], then 4
// pixels into 3 dwords of E.
//
// Direct launches (kFdFresh) run without the init kernel.  The grid then
// starts with one block per frame that only zeroes that frame's state (as the
// init kernel would) with agent-scope atomic stores, waits until they have
// completed and publishes the launch's epoch in the state.  A tile block reads
// its frame's epoch after its staging and, if it does not match yet, polls it
// before its histogram merge (bounded: after kEpochSpins polls it merges
// anyway, and the final selection's check of the histogram total against W H
// flags the frame).  The zeroing blocks come first in the grid, so they are
// dispatched before any block that waits for them, and they wait for nothing:
// the wait cannot hold a slot they need.  At 8 x 720p per launch they publish
// about 4 us into the kernel, and fewer than 1% of the first round's tile
// blocks find the epoch missing after their vertical pass.
// The waiting blocks take no acquire fence: their only accesses to the zeroed
// state are the histogram's atomic adds, which the device performs at its
// point of coherence, issued after the epoch read has returned; an agent-scope
// acquire here would also invalidate cached lines that the other blocks are
// still reading (it made k_dark 5.6 us slower at 1080p).
constexpr int kEpochSpins = 1 << 15;
namespace dk {
typedef __attribute__((address_space(1))) const uint32_t gu32;   // global memory: global_load, not flat

// v_perm_b32(hi, lo, sel): result byte i = byte sel[i] of the pair {hi, lo}
// (0-3 from lo, 4-7 from hi), 0x0C gives 0x00 and 0x0D gives 0xFF.
__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}
// bytes b = R0 G0 B0 R1 | G1 B1 R2 G2 | B2 R3 G3 B3 -> the planes of 4 cells
__device__ __forceinline__ void split4(uint32_t b0, uint32_t b1, uint32_t b2, uint32_t rb[4], uint32_t g[4]) {
  rb[0] = perm(b0, b0, 0x0C020C00u);  // R0 | B0 << 16
  g[0] = perm(b0, b0, 0x0C0D0C01u);   // G0 | FF << 16
  rb[1] = perm(b1, b0, 0x0C050C03u);  // R1 (b0.3) | B1 (b1.1) << 16
  g[1] = perm(b1, b0, 0x0C0D0C04u);   // G1 (b1.0)
  rb[2] = perm(b2, b1, 0x0C040C02u);  // R2 (b1.2) | B2 (b2.0) << 16
  g[2] = perm(b2, b1, 0x0C0D0C03u);   // G2 (b1.3)
  rb[3] = perm(b2, b2, 0x0C030C01u);  // R3 (b2.1) | B3 (b2.3) << 16
  g[3] = perm(b2, b2, 0x0C0D0C02u);   // G3 (b2.2)
}
}  // namespace dk

template <int HP, bool WRITE_E>
__global__ __launch_bounds__(256) void k_dark(Batch b) {
  constexpr int TW = kDarkTW, TH = kDarkTH;
  constexpr int RW = TW + 2 * HP, RH = TH + 2 * HP, WIN = 2 * HP + 1;
  // plane rows are RWP = RW | 1 dwords apart (an odd stride), so the 32
  // lanes of a half-wave in the horizontal pass (8 rows x 4 segments 8
  // columns apart) read 32 distinct banks
  constexpr int RWP = RW | 1;
  constexpr int GPR = (RW + 3) / 4;            // 4-cell groups per region row
  // The staged region uses rows of RWA = RW rounded up to 4 dwords, so that
  // a group's 4 cells go to LDS as one 16-byte write; the vertical pass
  // writes its output rows in place with the odd stride RWP, which the
  // horizontal pass reads (all its inputs are in registers by then).
  constexpr int RWA = (RW + 3) & ~3;
  constexpr int PLN = ((RH * RWA > TH * RWP ? RH * RWA : TH * RWP) + 3) & ~3;   // dwords per plane
  __shared__ __align__(16) uint32_t s_pl[2][PLN];
  __shared__ uint32_t s_hist[256];
  __shared__ int s_epoch_ok;   // fresh launches: the frame's state was zeroed before the vertical pass ended
  uint32_t(&s_rb)[TH][RWP] = *reinterpret_cast<uint32_t(*)[TH][RWP]>(&s_pl[0][0]);
  uint32_t(&s_g)[TH][RWP] = *reinterpret_cast<uint32_t(*)[TH][RWP]>(&s_pl[1][0]);

  const bool fresh = (b.f[0].flags & kFdFresh) != 0;   // the same for every frame of a launch
  const int nzero = fresh ? b.n : 0;                    // leading blocks that zero the frames' state
  if ((int)blockIdx.x < nzero) {
    const FrameDev& fz = b.f[blockIdx.x];
    // agent-scope atomic stores are written through to the device's point of
    // coherence; once the wave's counter says they completed, they are
    // visible to every XCD, and no L2 write-back (what a release fence would
    // add) is needed before the epoch goes out
    const int n4 = (int)(((fz.flags & kFdWbPercentile) ? offsetof(FrameState, epoch) : offsetof(FrameState, wbh)) / 4);
    uint32_t* z = reinterpret_cast<uint32_t*>(fz.st);
    for (int i = threadIdx.x; i < n4; i += 256) __hip_atomic_store(&z[i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);   // every counter at zero: this wave's stores have completed
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(&fz.st->epoch, b.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  const int blk = xcd_remap(blockIdx.x - nzero, gridDim.x - nzero);
  const int f = frame_of(b, blk);
  const FrameDev& fd = b.f[f];
  const int tile = blk - b.tile0[f];
  const int W = fd.W, H = fd.H;
  const int tiles_x = (W + TW - 1) / TW;
  const int x0 = (tile % tiles_x) * TW, y0 = (tile / tiles_x) * TH;
  const int tid = threadIdx.x;
  // The frame's epoch is read once staging is done and compared before the
  // vertical pass's barrier, while no store of the block is in flight (a wait
  // for the read later would also wait for the block's output stores); the
  // merge polls only if that read came before the zeroing block published.
  unsigned long long seen = 0ull;

  s_hist[tid] = 0u;
  {
    // thread t < GPR * RPI takes group column gi = t % GPR of region rows
    // t / GPR, t / GPR + RPI, ...: its column, bounds and LDS offsets stay
    // fixed and its row address advances by RPI pitches; every load of the
    // block is issued before any cell is formed
    constexpr int RPI = 256 / GPR;                 // region rows per iteration
    constexpr int NIT = (RH + RPI - 1) / RPI;
    const bool act = tid < GPR * RPI;
    const int gi = tid % GPR, r_off = tid / GPR;
    const int xa = x0 - HP + 4 * gi;
    const bool colin = act && xa >= 0 && xa + 3 < W;   // all 4 cells inside the frame's columns
    const int64_t step = (int64_t)RPI * fd.src_pitch;
    const uint8_t* rowp = fd.src + (int64_t)(y0 - HP + r_off) * fd.src_pitch + 3 * xa;
    // Loads are unconditional, so that none is waited for before its use (a
    // group not wholly inside the frame reads the dword that holds the
    // frame's first byte, four times, and is redone per cell below).
    uint32_t w[NIT][4], sh[NIT];
    bool ok[NIT];
    const uint8_t* rp = rowp;
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int rr = r_off + RPI * k, y = y0 - HP + rr;
      ok[k] = colin && rr < RH && y >= 0 && y < H;
      const uintptr_t a = ok[k] ? (uintptr_t)rp : (uintptr_t)fd.src;
      rp += step;
      const uintptr_t a0 = a & ~(uintptr_t)3;
      sh[k] = (uint32_t)(a & 3);
      const uintptr_t o = ok[k] ? 4 : 0;
      const dk::gu32* q = reinterpret_cast<const dk::gu32*>(a0);
      w[k][0] = q[0];
      w[k][1] = *reinterpret_cast<const dk::gu32*>(a0 + o);
      w[k][2] = *reinterpret_cast<const dk::gu32*>(a0 + 2 * o);
      // the 4th dword only when the 12 bytes reach into it (it then holds byte a + 11)
      w[k][3] = *reinterpret_cast<const dk::gu32*>(a0 + (sh[k] ? 3 * o : 2 * o));
    }
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int rr = r_off + RPI * k, y = y0 - HP + rr;
      // the cells from the loaded bytes, formed unconditionally (the loads stay
      // ahead of this loop); groups not wholly inside the frame redo them per cell
      uint32_t rb[4], g[4];
      dk::split4(__builtin_amdgcn_alignbyte(w[k][1], w[k][0], sh[k]), __builtin_amdgcn_alignbyte(w[k][2], w[k][1], sh[k]),
                 __builtin_amdgcn_alignbyte(w[k][3], w[k][2], sh[k]), rb, g);
      if (!act || rr >= RH) continue;
      if (!ok[k]) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int x = xa + j;
          rb[j] = 0x00FF00FFu;
          g[j] = 0x00FF00FFu;
          if (y >= 0 && y < H && x >= 0 && x < W) {
            const uint8_t* p = fd.src + (int64_t)y * fd.src_pitch + 3 * (int64_t)x;
            rb[j] = (uint32_t)p[0] | ((uint32_t)p[2] << 16);
            g[j] = (uint32_t)p[1] | 0x00FF0000u;
          }
        }
      }
      // cells beyond RW land in the row's padding (RWA >= 4 GPR)
      *reinterpret_cast<uint4*>(&s_pl[0][rr * RWA + 4 * gi]) = make_uint4(rb[0], rb[1], rb[2], rb[3]);
      *reinterpret_cast<uint4*>(&s_pl[1][rr * RWA + 4 * gi]) = make_uint4(g[0], g[1], g[2], g[3]);
    }
  }
  __syncthreads();
  if (fresh && tid == 0) seen = __hip_atomic_load(&fd.st->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

  // vertical pass: RW columns x 2 segments of 16 output rows, one per
  // thread; the outputs replace rows [0, TH) of the planes in place
  {
    constexpr int SEG = 16, NSEG = TH / SEG, L = SEG + WIN - 1;
    static_assert(RW * NSEG <= 256, "one column segment per thread");
    const bool act = tid < RW * NSEG;
    const int sg = tid / RW, cc = tid - sg * RW, r0 = sg * SEG;
    uint32_t orb[SEG], og[SEG];
    if (act) {
      uint32_t vrb[L], vg[L];
#pragma unroll
      for (int i = 0; i < L; ++i) {
        vrb[i] = s_pl[0][(r0 + i) * RWA + cc];
        vg[i] = s_pl[1][(r0 + i) * RWA + cc];
      }
      sliding_min<L, WIN, SEG>(vrb, orb);
      sliding_min<L, WIN, SEG>(vg, og);
    }
    __syncthreads();  // every segment has read its rows before any is overwritten
    if (act) {
#pragma unroll
      for (int i = 0; i < SEG; ++i) {
        s_rb[r0 + i][cc] = orb[i];
        s_g[r0 + i][cc] = og[i];
      }
    }
  }
  if (fresh && tid == 0) s_epoch_ok = seen == b.epoch;
  __syncthreads();

  // horizontal pass: 32 rows x 8 segments of 8 output columns; wave w takes
  // rows 8w..8w+7, lane l row 8w + (l & 7) and segment l >> 3
  {
    constexpr int HS = 8, L = HS + WIN - 1;
    const int r = 8 * (tid >> 6) + (tid & 7), c0 = ((tid & 63) >> 3) * HS;
    uint32_t vrb[L], vg[L], orb[HS], og[HS];
#pragma unroll
    for (int i = 0; i < L; ++i) {
      vrb[i] = s_rb[r][c0 + i];
      vg[i] = s_g[r][c0 + i];
    }
    sliding_min<L, WIN, HS>(vrb, orb);
    sliding_min<L, WIN, HS>(vg, og);
    const int y = y0 + r, xb = x0 + c0;
    if (y < H && xb < W) {
      const int nx = min(HS, W - xb);
      uint32_t px[HS], d[HS];
#pragma unroll
      for (int i = 0; i < HS; ++i) {
        px[i] = dk::perm(og[i], orb[i], 0x0C020400u);   // [E^R, E^G, E^B, 0]
        const uint32_t m = pkmin(orb[i], og[i]);         // (min(R, G), min(B, 255))
        d[i] = min(m & 0xFFFFu, m >> 16);
      }
      uint8_t* Drow = fd.D + (int64_t)y * fd.D_pitch + xb;
      uint8_t* Erow = fd.E + (int64_t)y * fd.E_pitch + 3 * xb;
      if (nx == HS) {
        const uint32_t dlo = d[0] | (d[1] << 8) | (d[2] << 16) | (d[3] << 24);
        const uint32_t dhi = d[4] | (d[5] << 8) | (d[6] << 16) | (d[7] << 24);
        *reinterpret_cast<uint2*>(Drow) = make_uint2(dlo, dhi);
        if (WRITE_E) {
          uint2* e = reinterpret_cast<uint2*>(Erow);
          e[0] = make_uint2(dk::perm(px[1], px[0], 0x04020100u), dk::perm(px[2], px[1], 0x05040201u));
          e[1] = make_uint2(dk::perm(px[3], px[2], 0x06050402u), dk::perm(px[5], px[4], 0x04020100u));
          e[2] = make_uint2(dk::perm(px[6], px[5], 0x05040201u), dk::perm(px[7], px[6], 0x06050402u));
        }
      } else {
        for (int i = 0; i < nx; ++i) {
          Drow[i] = (uint8_t)d[i];
          if (WRITE_E) {
            Erow[3 * i + 0] = (uint8_t)(px[i] & 0xFFu);
            Erow[3 * i + 1] = (uint8_t)((px[i] >> 8) & 0xFFu);
            Erow[3 * i + 2] = (uint8_t)((px[i] >> 16) & 0xFFu);
          }
        }
      }
      if (fd.dark_out) {
        uint8_t* o = fd.dark_out + (int64_t)y * W + xb;
        for (int i = 0; i < nx; ++i) o[i] = (uint8_t)d[i];
      }
      // histogram with run-length aggregation (D is locally smooth)
      uint32_t cur = d[0], cnt = 1;
      if (nx == HS) {
#pragma unroll
        for (int i = 1; i < HS; ++i) {
          const bool same = d[i] == cur;
          if (!same) atomicAdd(&s_hist[cur], cnt);
          cnt = same ? cnt + 1 : 1;
          cur = d[i];
        }
      } else {
        for (int i = 1; i < nx; ++i) {
          const bool same = d[i] == cur;
          if (!same) atomicAdd(&s_hist[cur], cnt);
          cnt = same ? cnt + 1 : 1;
          cur = d[i];
        }
      }
      atomicAdd(&s_hist[cur], cnt);
    }
  }
  if (fresh && tid == 0 && !s_epoch_ok) {
    const unsigned long long* ep = &fd.st->epoch;
    for (int n = 0; seen != b.epoch && n < kEpochSpins; ++n) {
      __builtin_amdgcn_s_sleep(8);
      seen = __hip_atomic_load(ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();
  const uint32_t hv = s_hist[tid];
  if (fd.flags & kFdNoHist) {
    fd.hpart[tile * 256 + tid] = (uint16_t)hv;   // <= 2048: the tile's histogram, for the one-block selection
  } else if (hv) {
    atomicAdd(&fd.st->hist[tile % kHistSlots][tid], hv);
  }
}

// ------------------------------------------------------------ k_select_rows
// Eq. (3) with a unique top-K set: order pixels by (D descending, raster
// index ascending) and take the first K.
//   vstar  = largest v with #{D >= v} >= K (from the histogram)
//   need   = K - #{D > vstar} >= 1 pixels with D == vstar are taken, the
//            first `need` of them in raster order.
// Row pass: each wave reads one row of D, gathers I where D >= vstar and
// writes the row's record (counts and exact sums of the ties D == vstar and
// of D > vstar).  Final step, in the frame's last row block to finish: scan
// the row records, find the row holding the cut, find the cutoff pixel inside
// it with a block-wide scan of per-lane tie counts, and form
// A^c = alpha * S^c / K from exact integer sums.

// The end of Eq. (3) for one frame, by one thread: A^c = alpha S^c / K from the
// exact integer sums (in double; optionally averaged with the stream's stored
// airlight: (lam A_prev) + ((1 - lam) Ahat), each operation rounded on its
// own), then the frame's state, the stream state and the aux outputs.
// status: 0 = consistent, 1 = the counts disagree (A formed, not trusted).
__device__ void store_airlight(const FrameDev& fd, uint32_t K, uint32_t vstar, int32_t cutoff,
                               const unsigned long long S[3], int32_t status) {
  FrameState* st = fd.st;
  const double a = (double)fd.alpha;
  float* ast = fd.A_state;
  const bool blend = ast && fd.ema > 0.0f && !(fd.flags & kFdEmaFirst) && __float_as_uint(ast[3]) != 0u;
  const double lam = (double)fd.ema;
  for (int ch = 0; ch < 3; ++ch) {
    double Ad = a * (double)S[ch] / (double)K;
    if (blend) Ad = __dadd_rn(__dmul_rn(lam, (double)ast[ch]), __dmul_rn(__dsub_rn(1.0, lam), Ad));
    const float A = (float)Ad;
    st->A[ch] = A;
    if (fd.A_out) fd.A_out[ch] = A;
  }
  if (ast) {
    const uint32_t seen = blend ? __float_as_uint(ast[3]) : 0u;
    for (int ch = 0; ch < 3; ++ch) ast[ch] = st->A[ch];
    ast[3] = __uint_as_float(seen < 0xFFFFFFFFu ? seen + 1u : seen);
  }
  st->sel[0] = (int32_t)K;
  st->sel[1] = (int32_t)vstar;
  st->sel[2] = cutoff;
  st->sel[3] = status;
  if (fd.sel_out) {
    fd.sel_out[0] = (int32_t)K;
    fd.sel_out[1] = (int32_t)vstar;
    fd.sel_out[2] = cutoff;
    fd.sel_out[3] = status;
    __threadfence_system();   // sel_out may be host memory read when the stream completes
  }
}

// No cut row exists (the per-row counts hold fewer ties than the histogram):
// A is set to 0 and the frame flagged with status 2 instead of reading a row
// that is not there; the stream's stored airlight is left as it was.
__device__ void store_no_cut(const FrameDev& fd, uint32_t K, uint32_t vstar) {
  FrameState* st = fd.st;
  for (int ch = 0; ch < 3; ++ch) {
    st->A[ch] = 0.0f;
    if (fd.A_out) fd.A_out[ch] = 0.0f;
  }
  st->sel[0] = (int32_t)K;
  st->sel[1] = (int32_t)vstar;
  st->sel[2] = -1;
  st->sel[3] = 2;
  if (fd.sel_out) {
    fd.sel_out[0] = (int32_t)K;
    fd.sel_out[1] = (int32_t)vstar;
    fd.sel_out[2] = -1;
    fd.sel_out[3] = 2;
    __threadfence_system();
  }
}

// Inclusive scan over a block of NW waves; also returns the block total.
template <int NW, typename T>
__device__ __forceinline__ T block_scan_total(T v, T* s_tmp, T& total) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  T x = wave_incl_scan(v);
  if (lane == 63) s_tmp[w] = x;
  __syncthreads();
  T add = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const T t = s_tmp[i];
    if (i < w) add += t;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return x + add;
}

// vstar and #{D > vstar} in one wave from per-lane bin counts: lane l holds
// the counts of bins 4(63 - l) .. 4(63 - l) + 3 in c.x .. c.w, so the lanes in
// order, and each lane's bins from the top, hold the counts by descending
// value; an inclusive scan gives #{D >= v}, and vstar is the first v from the
// top at which it reaches K.  Counts that never reach K (an inconsistent
// state) give vstar 0, which the final consistency test flags.
__device__ __forceinline__ void vstar_from_lane_counts(uint4 c, uint32_t K, uint32_t& vstar, uint32_t& cnt_gt,
                                                       uint32_t* total = nullptr) {
  // in-lane counts of D >= b0 + 3, b0 + 2, b0 + 1, b0
  const uint32_t l3 = c.w, l2 = l3 + c.z, l1 = l2 + c.y, l0 = l1 + c.x;
  const uint32_t incl = wave_incl_scan(l0);
  if (total) *total = __builtin_amdgcn_readlane(incl, 63);   // every pixel counted once: W H
  const unsigned long long hit = __ballot(incl >= K);
  const int L = hit ? __ffsll((long long)hit) - 1 : 63;
  const uint32_t ex = __builtin_amdgcn_readlane(incl - l0, L);   // #{D > 4(63 - L) + 3}
  const uint32_t a3 = __builtin_amdgcn_readlane(l3, L), a2 = __builtin_amdgcn_readlane(l2, L),
                 a1 = __builtin_amdgcn_readlane(l1, L);
  const uint32_t top = 4u * (uint32_t)(63 - L);
  if (ex + a3 >= K) {
    vstar = top + 3; cnt_gt = ex;
  } else if (ex + a2 >= K) {
    vstar = top + 2; cnt_gt = ex + a3;
  } else if (ex + a1 >= K) {
    vstar = top + 1; cnt_gt = ex + a2;
  } else {
    vstar = top; cnt_gt = ex + a1;
  }
}

// The same from the frame's slotted histogram, with no LDS and no barrier.
__device__ __forceinline__ void wave_vstar(const FrameState* st, uint32_t K, uint32_t& vstar, uint32_t& cnt_gt,
                                           uint32_t* total = nullptr) {
  const int b0 = 4 * (63 - (int)(threadIdx.x & 63));
  uint4 c = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
  for (int k = 0; k < kHistSlots; ++k) {
    const uint4 h = *reinterpret_cast<const uint4*>(&st->hist[k][b0]);
    c.x += h.x; c.y += h.y; c.z += h.z; c.w += h.w;
  }
  vstar_from_lane_counts(c, K, vstar, cnt_gt, total);
}

// A row record as four 8-byte words, written and read with agent-scope atomic
// accesses: the frame's last row block reads every record in the same kernel.
__device__ __forceinline__ void store_rowsel(RowSel* p, const RowSel& r) {
  unsigned long long w[4];
  __builtin_memcpy(w, &r, sizeof(w));
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
#pragma unroll
  for (int i = 0; i < 4; ++i) __hip_atomic_store(q + i, w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ RowSel load_rowsel(const RowSel* p) {
  unsigned long long w[4];
  const unsigned long long* q = reinterpret_cast<const unsigned long long*>(p);
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = __hip_atomic_load(q + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  RowSel r;
  __builtin_memcpy(&r, w, sizeof(w));
  return r;
}
static_assert(sizeof(RowSel) == 32 && alignof(RowSel) <= 8, "a row record is four 8-byte words");

// A k_select_rows block has kFinT threads (512 for launches of one frame,
// whose final step then spreads over twice the threads; 256 for batches, so
// that their row pass has more, shorter blocks): one row per wave, and the
// final step of the frame's last block.
constexpr int kFinRows = 5;            // sweeps of kFinT rows per round of the final step

// The row pass of one block of k_select_rows: its kFinW rows' records.
template <int kFinT>
__device__ __forceinline__ void row_pass(const FrameDev& fd, int tile, uint32_t& s_vstar) {
  constexpr int kFinW = kFinT / 64;
  const int W = fd.W, H = fd.H;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;

  // one row per wave; each lane reads 16 consecutive bytes of D per step.
  // The first segment's D does not depend on vstar: it is loaded before the
  // histogram is read, so the two round trips overlap.
  const int y = tile * kFinW + wv;
  const bool row_ok = y < H;
  const uint8_t* Drow = fd.D + (int64_t)min(y, H - 1) * fd.D_pitch;
  uint4 dvs[kSelVec];  // all of this lane's D vectors of a segment, loaded up front
  auto load_d = [&](int seg) {
#pragma unroll
    for (int q = 0; q < kSelVec; ++q) {
      const int bq = seg + 1024 * q + 16 * lane;
      dvs[q] = (row_ok && bq < W) ? *reinterpret_cast<const uint4*>(Drow + bq) : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  load_d(0);
  // wave 0 forms vstar from the histogram and shares it (one histogram read
  // per block instead of per wave; the barrier wait overlaps the D loads)
  if (wv == 0) {
    uint32_t v, cnt_gt;
    wave_vstar(fd.st, (uint32_t)fd.K, v, cnt_gt);
    if (lane == 0) s_vstar = v;
  }
  __syncthreads();
  const uint32_t vstar = s_vstar;
  if (!row_ok) return;   // wave-uniform; the block's barriers come after the call
  uint32_t gR = 0, gG = 0, gB = 0, tR = 0, tG = 0, tB = 0;   // < W * 255 < 2^32
  uint32_t gN = 0, tN = 0;
  const uint8_t* Irow = fd.src + (int64_t)y * fd.src_pitch;
  for (int seg = 0; seg < W; seg += 1024 * kSelVec) {
    if (seg > 0) load_d(seg);
#pragma unroll
    for (int q = 0; q < kSelVec; ++q) {
      const int base = seg + 1024 * q + 16 * lane;
      if (base >= W) continue;
      const uint4 dv = dvs[q];  // rows are padded to 16 bytes
      const uint32_t dw[4] = {dv.x, dv.y, dv.z, dv.w};
      // most vectors hold no byte >= vstar: test all 16 at once first.  In
      // 16-bit halves, byte + (256 - vstar) carries into bit 8 iff byte >= vstar
      // (padding bytes past the row may pass; the exact test below drops them)
      {
        const uint32_t kk = (256u - vstar) * 0x00010001u;
        uint32_t any = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          any |= ((dw[i] & 0x00FF00FFu) + kk) | (((dw[i] >> 8) & 0x00FF00FFu) + kk);
        if (!(any & 0x01000100u)) continue;
      }
      const int nx = min(16, W - base);
      uint32_t cand = 0;  // pixels with D >= vstar
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const uint32_t d = (dw[k >> 2] >> (8 * (k & 3))) & 0xFFu;
        if (k < nx && d >= vstar) cand |= 1u << k;
      }
      if (!cand) continue;
      // the lane's 16 pixels of I in one round trip when the rows are dword aligned
      uint32_t iw[12];
      const bool vec = (fd.flags & kFdAligned) && nx == 16;
      if (vec) {
        const uint32_t* q4 = reinterpret_cast<const uint32_t*>(Irow + 3 * base);
#pragma unroll
        for (int j = 0; j < 12; ++j) iw[j] = q4[j];
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        if (!((cand >> k) & 1u)) continue;
        uint32_t r, g, bl;
        if (vec) {
          r = (iw[(3 * k) >> 2] >> (8 * ((3 * k) & 3))) & 0xFFu;
          g = (iw[(3 * k + 1) >> 2] >> (8 * ((3 * k + 1) & 3))) & 0xFFu;
          bl = (iw[(3 * k + 2) >> 2] >> (8 * ((3 * k + 2) & 3))) & 0xFFu;
        } else {
          const int x = base + k;
          r = Irow[3 * x]; g = Irow[3 * x + 1]; bl = Irow[3 * x + 2];
        }
        const uint32_t d = (dw[k >> 2] >> (8 * (k & 3))) & 0xFFu;
        if (d > vstar) {
          gR += r; gG += g; gB += bl; gN += 1;
        } else {
          tR += r; tG += g; tB += bl; tN += 1;
        }
      }
    }
  }
  tN = wave_sum(tN);
  gN = wave_sum(gN);
  if (tN) { tR = wave_sum(tR); tG = wave_sum(tG); tB = wave_sum(tB); }
  if (gN) { gR = wave_sum(gR); gG = wave_sum(gG); gB = wave_sum(gB); }
  if (lane == 0) {
    RowSel r;
    r.ties = tN; r.above = gN;
    r.tsum[0] = tR; r.tsum[1] = tG; r.tsum[2] = tB;
    r.gsum[0] = gR; r.gsum[1] = gG; r.gsum[2] = gB;
    store_rowsel(&fd.rowsel[y], r);
  }
}


// The final step of Eq. (3) for one frame, in one block.  Rows are dealt round-robin,
// row = base + t + kFinT u for sweep u of a round, so a wave loads consecutive
// records.  Per round of kFinRows sweeps:
//   1. the records (with, in the first round, vstar and #{D > vstar} from the
//      histogram) in one round trip; the tie counts go to LDS with the tie
//      total of every wave of every sweep;
//   2. after one barrier every wave finds, from those totals and one scan of
//      the 64 tie counts of the wave holding it, the row that holds the
//      need-th tie in raster order (need = K - #{D > vstar}) and the ties
//      before it;
// then 3. the cut row's D and I in one round trip, and an exclusive scan of
// the per-thread tie counts that gives each thread its share of the row's
// first need - (ties before) ties; 4. one block sum of the sums over
// D > vstar, the tie sums of the rows before the cut row and the cut row's
// share, from which thread 0 forms A.
template <int kFinT>
struct FinShared {
  static constexpr int kFinW = kFinT / 64;
  uint32_t ties[kFinRows][kFinT];   // tie counts of the round's rows, by sweep and thread
  uint32_t tw[kFinRows][kFinW];     // tie total of each wave of each sweep
  uint32_t cnt[kFinW];
  unsigned long long red[kFinW][5];
};

template <int kFinT>
__device__ void final_selection(const FrameDev& fd, FinShared<kFinT>& sh) {
  constexpr int kFinW = kFinT / 64;
  uint32_t(&s_ties)[kFinRows][kFinT] = sh.ties;
  uint32_t(&s_tw)[kFinRows][kFinW] = sh.tw;
  uint32_t(&s_cnt)[kFinW] = sh.cnt;
  unsigned long long(&s_red)[kFinW][5] = sh.red;
  const int W = fd.W, H = fd.H;
  const uint32_t K = (uint32_t)fd.K;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;

  RowSel r[kFinRows];
  auto load_round = [&](int base) {
#pragma unroll
    for (int u = 0; u < kFinRows; ++u) {
      const int y = base + tid + kFinT * u;
      if (y < H) {
        r[u] = load_rowsel(&fd.rowsel[y]);
      } else {
        r[u].ties = 0u;
        r[u].above = 0u;
#pragma unroll
        for (int c = 0; c < 3; ++c) r[u].tsum[c] = r[u].gsum[c] = 0u;
      }
    }
  };
  load_round(0);
  uint32_t vstar, cnt_gt, total;
  wave_vstar(fd.st, K, vstar, cnt_gt, &total);
  const uint32_t need = K - cnt_gt;  // >= 1

  int rstar = -1;          // the cut row (block-uniform once found)
  uint32_t before = 0;     // ties in the rows before it
  uint32_t carry = 0;      // ties in earlier rounds
  unsigned long long acc[4] = {0ull, 0ull, 0ull, 0ull};   // S^c so far, #{D > vstar}
  for (int base = 0; base < H; base += kFinT * kFinRows) {
    if (base > 0) {
      __syncthreads();  // s_ties and s_tw are rewritten
      load_round(base);
    }
#pragma unroll
    for (int u = 0; u < kFinRows; ++u) {
      s_ties[u][tid] = r[u].ties;
      const uint32_t wt = wave_sum(r[u].ties);
      if (lane == 0) s_tw[u][wv] = wt;
    }
    __syncthreads();
    // the round's wave totals in raster order, one per lane (sweep-major)
    static_assert(kFinRows * kFinW <= 64, "one lane per wave total");
    const uint32_t tw = lane < kFinRows * kFinW ? (&s_tw[0][0])[lane] : 0u;
    const uint32_t twi = wave_incl_scan(tw);
    if (rstar < 0) {
      const unsigned long long hit = __ballot(carry + twi >= need);
      if (hit) {  // block-uniform; the wave total at lane J holds the need-th tie
        const int J = __ffsll((long long)hit) - 1;
        const int us = J / kFinW, ws = J % kFinW;
        const uint32_t cum = carry + __builtin_amdgcn_readlane(twi - tw, J);
        const uint32_t tl = s_ties[us][64 * ws + lane];
        const uint32_t incl = wave_incl_scan(tl);
        const int L = __ffsll((long long)__ballot(cum + incl >= need)) - 1;
        before = cum + __builtin_amdgcn_readlane(incl - tl, L);
        rstar = base + 64 * ws + L + kFinT * us;
      }
    }
    // sums over D > vstar (every row) and tie sums of the rows before the cut row
#pragma unroll
    for (int u = 0; u < kFinRows; ++u) {
      const int y = base + tid + kFinT * u;
      const bool tb = rstar < 0 || y < rstar;
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] += (unsigned long long)r[u].gsum[c] + (tb ? r[u].tsum[c] : 0u);
      acc[3] += r[u].above;
    }
    carry += __builtin_amdgcn_readlane(twi, 63);
  }
  if (rstar < 0) {  // fewer ties in the records than the histogram promises
    if (tid == 0) store_no_cut(fd, K, vstar);
    return;
  }

  // 3. the first k = need - before ties of the cut row.  Thread t owns pixels
  // [16 t, 16 t + 16) of each kFinT*16-pixel segment, so thread order is
  // raster order inside a segment.  I is loaded with D, before the thread
  // knows whether it takes any of its ties.
  const uint32_t k = need - before;
  const uint8_t* Drow = fd.D + (int64_t)rstar * fd.D_pitch;
  const uint8_t* Irow = fd.src + (int64_t)rstar * fd.src_pitch;
  uint32_t run = 0;  // ties in earlier segments (block-uniform)
  int cut_x = -1;
  for (int seg = 0; seg < W && run < k; seg += 16 * kFinT) {
    const int x0 = seg + 16 * tid;
    const bool vec = (fd.flags & kFdAligned) && x0 + 16 <= W;
    uint32_t dw[4] = {0u, 0u, 0u, 0u}, iw[12] = {};
    if (x0 < W) {
      const uint4 dv = *reinterpret_cast<const uint4*>(Drow + x0);  // rows are padded to 16 bytes
      dw[0] = dv.x; dw[1] = dv.y; dw[2] = dv.z; dw[3] = dv.w;
    }
    if (vec) {
      const uint32_t* q4 = reinterpret_cast<const uint32_t*>(Irow + 3 * x0);
#pragma unroll
      for (int j = 0; j < 12; ++j) iw[j] = q4[j];
    }
    uint32_t mask = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const uint32_t d = (dw[j >> 2] >> (8 * (j & 3))) & 0xFFu;
      if (x0 + j < W && d == vstar) mask |= 1u << j;
    }
    const uint32_t cnt = (uint32_t)__popc(mask);
    const uint32_t ci = wave_incl_scan(cnt);
    if (lane == 63) s_cnt[wv] = ci;
    __syncthreads();
    uint32_t ex = ci - cnt, seg_total = 0;
    for (int w = 0; w < kFinW; ++w) {
      const uint32_t c = s_cnt[w];
      if (w < wv) ex += c;
      seg_total += c;
    }
    const uint32_t avail = (run + ex < k) ? min(cnt, k - run - ex) : 0u;
    // the thread's first `avail` ties: their bits, then their colours with
    // compile-time register indices (a data-dependent index into iw would
    // become a chain of selects per byte)
    uint32_t m = mask, take = 0u;
    for (uint32_t i = 0; i < avail; ++i) {
      const uint32_t low = m & (0u - m);
      take |= low;
      m ^= low;
    }
    if (avail && run + ex + avail == k) cut_x = x0 + 31 - __clz(take);   // the cut is the last tie taken
    if (vec) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        if (!((take >> j) & 1u)) continue;
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] += (iw[(3 * j + c) >> 2] >> (8 * ((3 * j + c) & 3))) & 0xFFu;
      }
    } else {
      while (take) {
        const int j = __ffs(take) - 1;
        take &= take - 1;
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] += Irow[3 * (x0 + j) + c];
      }
    }
    run += seg_total;
    if (seg + 16 * kFinT < W && run < k) __syncthreads();  // s_cnt is rewritten by the next segment
  }

  // 4. the block's sums
  const unsigned long long v[5] = {acc[0], acc[1], acc[2], acc[3], (unsigned long long)(cut_x + 1)};  // one thread holds the cut
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const unsigned long long x = wave_sum(v[i]);
    if (lane == 0) s_red[wv][i] = x;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long S[5] = {0, 0, 0, 0, 0};
    for (int w = 0; w < kFinW; ++w)
      for (int i = 0; i < 5; ++i) S[i] += s_red[w][i];
    const int cx = (int)S[4] - 1;
    // consistency: the rows' count over D > vstar must equal the histogram's
    const bool ok = S[3] == (unsigned long long)cnt_gt && cx >= 0 && total == (uint32_t)W * (uint32_t)H;
    store_airlight(fd, K, vstar, rstar * W + cx, S, ok ? 0 : 1);
  }
}

// The row pass, then, in the frame's last row block to finish, the final step.
// Every block's records are agent-scope atomic stores, complete (the wave's
// counters at zero) before the block counts itself in the frame's state; the
// block that counts last reads all of them with agent-scope atomic loads
// issued after its count returned.  Nothing else crosses blocks, so no L2
// write-back is needed (a release fence per block, which writes back the XCD's
// L2, made this 6 us slower than a kernel boundary).
template <int kFinT>
__global__ __launch_bounds__(kFinT) void k_select_rows(Batch b) {
  __shared__ uint32_t s_vstar;
  __shared__ int s_last;
  __shared__ FinShared<kFinT> s_fin;
  const int blk = blockIdx.x;
  const int f = frame_of(b, blk);
  const FrameDev& fd = b.f[f];
  const int tile = blk - b.tile0[f];
  row_pass<kFinT>(fd, tile, s_vstar);
  __builtin_amdgcn_s_waitcnt(0);   // every counter at zero: this wave's record stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t blocks = (uint32_t)(b.tile0[f + 1] - b.tile0[f]);
    s_last = atomicAdd(&fd.st->rows_done, 1u) == blocks - 1u;
  }
  __syncthreads();
  if (s_last) final_selection(fd, s_fin);
}

// ------------------------------------------------------------ k_select_one
// Eq. (3) for a small frame in one 1024-thread block.  D is read once: its
// 16-byte vectors are numbered tile by tile (k_dark's 64x32 tiles, 128 vector
// slots each: 32 rows x 4 vectors), and thread t holds the slots t, t + 1024,
// ..., so a wave holds half of one tile.  Thread t also loads bin t % 256 of
// the per-tile histograms k_dark wrote, for every fourth tile.  After one
// barrier (LDS holds each quarter's histogram sums and each tile's largest D,
// written without atomics), every wave
//   1. forms vstar and #{D > vstar} itself, and which tiles can hold members
//      of the set (largest D >= vstar: a wave-uniform test);
//   2. counts the ties per row in those tiles and sums I over their pixels
//      with D > vstar, which belong to the set whatever the cut;
// then, after a barrier, wave 0 scans the rows for the one holding the
// need-th tie and that row's ties (in LDS) for the cut pixel; after another,
// the ties up to the cut are summed, and thread 0 forms A = alpha S / K.  The
// kernel also zeroes the frame state's sums for the later passes (colour
// balance, luma, white balance); with the per-tile histograms written whole
// by k_dark, nothing of the frame's state needs zeroing before the frame, so
// the init kernel is not run.  Used when W <= 1024 (the cut row is one vector
// per lane of a wave) and the frame has at most kOneTiles tiles
// (select_one_fits).
constexpr int kOneT = 1024, kOneW = kOneT / 64;
constexpr int kOneRows = 2048;
constexpr int kOneTileLoads = 16;                 // per-tile histogram loads per thread
constexpr int kOneTiles = 4 * kOneTileLoads;      // tiles of a frame on this path (64)
static_assert(kOneTiles * 128 == kOneT * kOneVecMax, "every vector slot of every tile has a thread");

// Row y's tie count sits at y + y / 32, so that the 64 lanes of a wave that
// read rows 32 l + k hit distinct LDS banks.
__device__ __forceinline__ int one_row_slot(int y) { return y + (y >> 5); }

template <int NVT>
__global__ __launch_bounds__(kOneT) void k_select_one(Batch b) {
  __shared__ uint4 s_h4[4][64];                  // [tile quarter q][bins 4i .. 4i + 3]: histogram sums over the quarter's tiles
  __shared__ uint32_t s_tm4[4][kOneTiles];       // [bin quarter][tile]: 1 + the quarter's largest nonzero bin of the tile (0: none)
  __shared__ uint32_t s_tc[kOneRows + kOneRows / 32];   // ties per row (one_row_slot)
  __shared__ uint4 s_D[NVT * kOneT];             // D by slot, for the scan of the cut row
  __shared__ int s_misc[4];
  __shared__ unsigned long long s_red[kOneW][4];
  const FrameDev& fd = b.f[blockIdx.x];
  FrameState* st = fd.st;
  const int W = fd.W, H = fd.H;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const uint32_t K = (uint32_t)fd.K;
  const int tiles_x = (W + 63) / 64, nt = dark_tiles(W, H);

  for (int i = tid; i < kOneRows + kOneRows / 32; i += kOneT) s_tc[i] = 0u;
  // every load is issued before the first barrier
  uint4 dv[NVT];
  int vy[NVT], vx[NVT];   // vy < 0: no vector in this slot
#pragma unroll
  for (int i = 0; i < NVT; ++i) {
    const int slot = tid + kOneT * i, tile = slot >> 7, l = slot & 127;
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    vy[i] = ty * 32 + (l >> 2);
    vx[i] = tx * 64 + (l & 3) * 16;
    const bool ok = tile < nt && vy[i] < H && vx[i] < W;
    dv[i] = ok ? *reinterpret_cast<const uint4*>(fd.D + (int64_t)vy[i] * fd.D_pitch + vx[i]) : make_uint4(0u, 0u, 0u, 0u);
    if (!ok) vy[i] = -1;
  }
  const int bin = tid & 255, q = tid >> 8;
  uint32_t hv[kOneTileLoads];
#pragma unroll
  for (int u = 0; u < kOneTileLoads; ++u) {
    const int tt = q + 4 * u;
    hv[u] = tt < nt ? fd.hpart[tt * 256 + bin] : 0u;
  }
  // the frame state's sums of the later passes start at zero
  {
    uint32_t* z = reinterpret_cast<uint32_t*>(&st->cb[0][0]);
    constexpr int nz = (int)((offsetof(FrameState, epoch) - offsetof(FrameState, cb)) / 4);
    for (int i = tid; i < nz; i += kOneT) z[i] = 0u;
  }
  auto dbyte = [&](int i, int j) { return (((&dv[i].x)[j >> 2]) >> (8 * (j & 3))) & 0xFFu; };
  {
    // a wave holds 64 consecutive bins of the same tiles: the highest of its
    // nonzero bins per tile comes from one ballot
    uint32_t hsum = 0;
#pragma unroll
    for (int u = 0; u < kOneTileLoads; ++u) {
      hsum += hv[u];
      const uint64_t nzb = __ballot(hv[u] != 0u);
      if (lane == 0) s_tm4[bin >> 6][q + 4 * u] = nzb ? (uint32_t)((bin & ~63) + 64 - __clzll((long long)nzb)) : 0u;
    }
    reinterpret_cast<uint32_t*>(&s_h4[q][0])[bin] = hsum;
  }
#pragma unroll
  for (int i = 0; i < NVT; ++i) s_D[tid + kOneT * i] = dv[i];
  __syncthreads();   // histogram quarters, tile maxima, D and the zeroed row counts in LDS

  // 1. vstar and #{D > vstar}, in every wave
  uint32_t vstar, cnt_gt;
  {
    uint4 c = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint4 h = s_h4[k][63 - lane];
      c.x += h.x; c.y += h.y; c.z += h.z; c.w += h.w;
    }
    vstar_from_lane_counts(c, K, vstar, cnt_gt);
  }
  const uint32_t need = K - cnt_gt;   // >= 1
  // the slots of a wave lie in one tile: whether it can hold ties or members
  // of the set is wave-uniform (a tile's largest D is >= vstar iff one of its
  // bin quarters has a nonzero bin >= vstar)
  bool hot[NVT];
#pragma unroll
  for (int i = 0; i < NVT; ++i) {
    const int tile = (tid + kOneT * i) >> 7;
    hot[i] = false;
    if (tile < nt) {
#pragma unroll
      for (int k = 0; k < 4; ++k) hot[i] |= s_tm4[k][tile] > vstar;
    }
  }

  // 2. ties per row
  unsigned long long acc[4] = {0ull, 0ull, 0ull, 0ull};   // S^c, members
  auto sum_members = [&](int i, uint32_t mem) {
    const uint8_t* Irow = fd.src + (int64_t)max(vy[i], 0) * fd.src_pitch + 3 * vx[i];
    acc[3] += (unsigned long long)__popc(mem);
    if (!mem) return;
    if ((fd.flags & kFdAligned) && vx[i] + 16 <= W) {  // the lane's 16 pixels in one round trip
      uint32_t iw[12];
      const uint32_t* q4 = reinterpret_cast<const uint32_t*>(Irow);
#pragma unroll
      for (int j = 0; j < 12; ++j) iw[j] = q4[j];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        if (!((mem >> j) & 1u)) continue;
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] += (iw[(3 * j + c) >> 2] >> (8 * ((3 * j + c) & 3))) & 0xFFu;
      }
    } else {
      while (mem) {
        const int j = __ffs(mem) - 1;
        mem &= mem - 1;
        acc[0] += Irow[3 * j];
        acc[1] += Irow[3 * j + 1];
        acc[2] += Irow[3 * j + 2];
      }
    }
  };
  // member masks of the slots: D > vstar, and ties (D == vstar)
  uint32_t mg[NVT], mt[NVT];
#pragma unroll
  for (int i = 0; i < NVT; ++i) {
    mt[i] = mg[i] = 0u;
    if (!hot[i] || vy[i] < 0) continue;
    const int n = min(16, W - vx[i]);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const uint32_t d = dbyte(i, j);
      if (j < n && d == vstar) mt[i] |= 1u << j;
      if (j < n && d > vstar) mg[i] |= 1u << j;
    }
    if (mt[i]) atomicAdd(&s_tc[one_row_slot(vy[i])], (uint32_t)__popc(mt[i]));
  }
  __syncthreads();
  // while wave 0 finds the cut, the other waves sum I over their pixels with
  // D > vstar, which belong to the set whatever the cut (wave 0 adds its own
  // with its ties below)
  if (wv != 0) {
#pragma unroll
    for (int i = 0; i < NVT; ++i)
      if (hot[i] && __any(mg[i] != 0u)) sum_members(i, mg[i]);
  }
  // the cut row and the cut pixel, by wave 0: lane l sums rows [32 l, 32 l + 32),
  // a wave scan finds the lane, then the row, holding the need-th tie; then
  // lane l takes vector l of that row (W <= 1024) and a second scan finds the pixel
  if (wv == 0) {
    constexpr int RPL = kOneRows / 64;
    uint32_t tc[RPL], t = 0;   // the lane's rows' tie counts stay in registers for the search
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      tc[k] = s_tc[one_row_slot(RPL * lane + k)];   // zero past the last row
      t += tc[k];
    }
    const uint32_t incl = wave_incl_scan(t);
    uint32_t cum = incl - t;
    int ycut = -1;
    uint32_t before = 0;
    if (cum < need && need <= incl) {
#pragma unroll
      for (int k = 0; k < RPL; ++k) {
        if (ycut < 0 && cum + tc[k] >= need) {
          ycut = RPL * lane + k;
          before = cum;
        }
        if (ycut < 0) cum += tc[k];
      }
    }
    // the lane that found the row broadcasts it (-1 everywhere if none did)
    const uint64_t who = __ballot(ycut >= 0);
    if (who) {
      const int src = __ffsll((long long)who) - 1;
      ycut = __builtin_amdgcn_readlane(ycut, src);
      before = __builtin_amdgcn_readlane(before, src);
      const uint32_t kcut = need - before;   // the cut is the kcut-th tie of row ycut
      uint32_t m = 0u;
      if (16 * lane < W) {
        const int tile = (ycut >> 5) * tiles_x + (lane >> 2);
        const uint4 c = s_D[tile * 128 + (ycut & 31) * 4 + (lane & 3)];
        const int n = min(16, W - 16 * lane);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const uint32_t d = (((&c.x)[j >> 2]) >> (8 * (j & 3))) & 0xFFu;
          if (j < n && d == vstar) m |= 1u << j;
        }
      }
      const uint32_t cnt = (uint32_t)__popc(m);
      const uint32_t ci = wave_incl_scan(cnt), ce = ci - cnt;
      if (ce < kcut && kcut <= ci) {
        for (uint32_t k = ce + 1; k < kcut; ++k) m &= m - 1;   // drop the ties before the cut
        s_misc[2] = ycut * W + 16 * lane + (__ffs(m) - 1);
      }
    } else if (lane == 0) {
      s_misc[2] = -1;
    }
  }
  __syncthreads();
  const int cutoff = s_misc[2];
  if (cutoff < 0) {
    if (tid == 0) store_no_cut(fd, K, vstar);
    return;
  }

  // 3. the ties up to the cut (and wave 0's pixels with D > vstar)
#pragma unroll
  for (int i = 0; i < NVT; ++i) {
    if (!hot[i]) continue;
    uint32_t mem = wv == 0 ? mg[i] : 0u;
    if (mt[i]) {
      const int base = vy[i] * W + vx[i];
      const int last = cutoff - base;   // ties at j <= last are members
      mem |= last >= 15 ? mt[i] : (last < 0 ? 0u : mt[i] & ((2u << last) - 1u));
    }
    if (__any(mem != 0u)) sum_members(i, mem);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const unsigned long long x = wave_sum(acc[c]);
    if (lane == 0) s_red[wv][c] = x;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long S[4] = {0, 0, 0, 0};
    for (int w = 0; w < kOneW; ++w)
      for (int c = 0; c < 4; ++c) S[c] += s_red[w][c];
    // consistency: the set has exactly K members
    store_airlight(fd, K, vstar, cutoff, S, S[3] == (unsigned long long)K ? 0 : 1);
  }
}

// ----------------------------------------------------- transmission (device)
struct TxConsts {
  float iA[3];     // 1 / max(A^c, 1)
  float iAmax;     // 1 / max_c max(A^c, 1)
  float omega, t0;
};

__device__ __forceinline__ TxConsts tx_consts(const FrameDev& fd) {
  TxConsts k;
  float am = 1.0f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float a = fmaxf(fd.st->A[c], 1.0f);
    k.iA[c] = 1.0f / a;
    am = fmaxf(am, a);
  }
  k.iAmax = 1.0f / am;
  k.omega = fd.omega;
  k.t0 = fd.t0;
  return k;
}

// Eqs. (4)-(5), dark-channel form: t = max(1 - omega * min_c E^c / A^c, t0)
__device__ __forceinline__ float tx_he(const TxConsts& k, float er, float eg, float eb) {
  const float e = fminf(fminf(er * k.iA[0], eg * k.iA[1]), eb * k.iA[2]);
  return fmaxf(fmaf(-k.omega, e, 1.0f), k.t0);
}

// Eqs. (4)-(5) as printed: t = max(1 - omega * min_c I^c(x) / max(A), t0)
__device__ __forceinline__ float tx_paper(const TxConsts& k, float m) {
  return fmaxf(fmaf(-k.omega, m * k.iAmax, 1.0f), k.t0);
}

__device__ __forceinline__ ReconConsts recon_consts(const FrameDev& fd) {
  ReconConsts rc;
#pragma unroll
  for (int c = 0; c < 3; ++c) rc.A[c] = fd.st->A[c];
  rc.inv_gamma = fd.inv_gamma;
  rc.bias = fd.gamma_log_bias;
  rc.gamma_is_one = (fd.flags & kFdGammaOne) != 0;
  return rc;
}

// ---------------------------------------------------------------- k_gf_prep
// Offline mode, after the airlight: per pixel, the guide as an exact integer
// L = 299 R + 587 G + 114 B (= 255000 * BT.601 luma in [0,1]) and the coarse
// t of Eqs. (4)-(5) in fixed point P = rint(t * 2^28) (exact for t >= 1/16).
// A block covers 64 columns x one group of kGroupChunks aligned 8-row chunks;
// wave w takes chunk w, lane l one column.  Besides the LP map it writes, per
// column and chunk, the exact sums of L, P, L^2, L*P over the chunks of its
// group up to and including this one (a prefix inside the group), from which
// the guided-filter kernels form a window's whole-chunk sums with at most
// four loads.
template <int TX>
__global__ __launch_bounds__(64 * kGroupChunks) void k_gf_prep(Batch b) {
  __shared__ unsigned long long s_c[4][kGroupChunks][64];   // chunk sums of L, P, L^2, L*P
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int f = frame_of(b, blk);
  const FrameDev& fd = b.f[f];
  const int tile = blk - b.tile0[f];
  const int W = fd.W, H = fd.H;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int cblocks = (W + 63) / 64;
  const int grp = tile / cblocks;
  const int x = (tile - grp * cblocks) * 64 + lane;
  const int ch = grp * kGroupChunks + wv;
  const int y0 = ch * kChunk, n = max(0, min(kChunk, H - y0));
  const bool ok = x < W && n > 0;
  const TxConsts k = tx_consts(fd);
  uint32_t rgb[kChunk], e[kChunk];
#pragma unroll
  for (int i = 0; i < kChunk; ++i) {
    rgb[i] = 0u;
    e[i] = 0u;
    if (ok && i < n) {
      const uint8_t* ip = fd.src + (int64_t)(y0 + i) * fd.src_pitch + 3 * x;
      rgb[i] = (uint32_t)ip[0] | ((uint32_t)ip[1] << 8) | ((uint32_t)ip[2] << 16);
      if (TX == TSRC_HE) {
        const uint8_t* ep = fd.E + (int64_t)(y0 + i) * fd.E_pitch + 3 * x;
        e[i] = (uint32_t)ep[0] | ((uint32_t)ep[1] << 8) | ((uint32_t)ep[2] << 16);
      }
    }
  }
  uint32_t sL = 0;
  unsigned long long sP = 0, sLL = 0, sLP = 0;
#pragma unroll
  for (int i = 0; i < kChunk; ++i) {
    if (ok && i < n) {
      const uint32_t r = rgb[i] & 0xFFu, g = (rgb[i] >> 8) & 0xFFu, bl = (rgb[i] >> 16) & 0xFFu;
      float t;
      if (TX == TSRC_HE) {
        t = tx_he(k, (float)(e[i] & 0xFFu), (float)((e[i] >> 8) & 0xFFu), (float)((e[i] >> 16) & 0xFFu));
      } else {
        t = tx_paper(k, (float)min(min(r, g), bl));
      }
      const uint32_t L = 299u * r + 587u * g + 114u * bl;
      const uint32_t P = (uint32_t)__builtin_rintf(t * 268435456.0f);
      fd.LP[(int64_t)(y0 + i) * W + x] = make_uint2(L, P);
      sL += L;
      sP += P;
      sLL += (unsigned long long)L * L;
      sLP += (unsigned long long)L * P;
    }
  }
  s_c[0][wv][lane] = sL;
  s_c[1][wv][lane] = sP;
  s_c[2][wv][lane] = sLL;
  s_c[3][wv][lane] = sLP;
  __syncthreads();
  if (!ok) return;
  unsigned long long v[4] = {0ull, 0ull, 0ull, 0ull};
  for (int c = 0; c <= wv; ++c) {
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] += s_c[q][c][lane];
  }
  fd.PGa[(int64_t)ch * W + x] = make_ulonglong2(v[0], v[1]);
  fd.PGb[(int64_t)ch * W + x] = make_ulonglong2(v[2], v[3]);
}

// Rows [ya, yb] of one column as: head rows, whole aligned 8-row chunks
// (a chunk at the frame bottom may be short), tail rows.  Every load of the
// initial window is issued before any is consumed.
struct WindowSplit {
  int ya, head_end, c0, nch, tail_beg, yb;
};

__device__ __forceinline__ WindowSplit split_window(int ya, int yb, int H) {
  WindowSplit w;
  w.ya = ya;
  w.yb = yb;
  const int c0 = (ya + kChunk - 1) / kChunk;
  const int c1 = (yb == H - 1) ? (H - 1) / kChunk : (yb + 1) / kChunk - 1;
  if (c1 >= c0) {
    w.c0 = c0;
    w.nch = c1 - c0 + 1;
    w.head_end = c0 * kChunk;                   // head rows [ya, head_end)
    w.tail_beg = min(H, (c1 + 1) * kChunk);     // tail rows [tail_beg, yb]
  } else {
    w.c0 = 0;
    w.nch = 0;
    w.head_end = yb + 1;
    w.tail_beg = yb + 1;
  }
  return w;
}

// ------------------------------------------------------------------ k_gf_ab
// FP64 reciprocal: the hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// 64-bit integers to double with one rounding: hi * 2^32 + lo in one FMA.
__device__ __forceinline__ double u64_to_f64(unsigned long long x) {
  return fma((double)(uint32_t)(x >> 32), 4294967296.0, (double)(uint32_t)x);
}
__device__ __forceinline__ double i64_to_f64(long long x) {
  return fma((double)(int32_t)(x >> 32), 4294967296.0, (double)(uint32_t)x);
}

// Geometry of one guided-filter strip block: SW + 2r loaded columns (one per
// thread) starting at x0 - r, output columns [x0, x0 + SW) with SW = 128 or
// 192 (gf_strip), output rows [y0, y1) with y1 - y0 = fd.gf_rows (the tile
// height is a tuning knob; the integer sums make results independent of it).
struct GfTile {
  int W, H, r, SW, x0, y0, y1, xl;
  bool colin;
};

__device__ __forceinline__ GfTile gf_tile(const FrameDev& fd, int tile) {
  GfTile t;
  t.W = fd.W;
  t.H = fd.H;
  t.r = fd.radius;
  t.SW = ((kGfCols - 2 * t.r) / 64) * 64;
  // column-major: consecutive tiles are vertical neighbours, which share
  // 2r halo rows, and XCD-aware block mapping keeps runs of them in one L2
  const int chunks = (t.H + fd.gf_rows - 1) / fd.gf_rows;
  const int sx = tile / chunks, sy = tile - sx * chunks;
  t.x0 = sx * t.SW;
  t.y0 = sy * fd.gf_rows;
  t.y1 = min(t.H, t.y0 + fd.gf_rows);
  t.xl = t.x0 - t.r + (int)threadIdx.x;
  t.colin = (int)threadIdx.x < t.SW + 2 * t.r && t.xl >= 0 && t.xl < t.W;
  return t;
}

constexpr int kRpi = 4;          // rows per barrier phase in the guided-filter strip kernels
static_assert(kRpi == 4, "one wave of the 256-thread block per row of a phase");
static_assert(kGfRowsMax <= 256, "per-row table filled by one pass of the block's threads");

// Per output row of the block: the clipped window height ch and 1/ch (one
// table per block, filled before the first barrier of the row loop).
__device__ __forceinline__ void gf_row_table(const GfTile& g, double2* s_rows) {
  const int i = threadIdx.x;
  if (i < g.y1 - g.y0) {
    const int y = g.y0 + i;
    const int ch = min(y + g.r, g.H - 1) - max(y - g.r, 0) + 1;
    s_rows[i] = make_double2((double)ch, rcp_nr((double)ch));
  }
}
static_assert(kChunk % kRpi == 0, "phases must not straddle 8-row chunks");

// One step of an inclusive wave scan on NR 64-bit values at once: v += the
// DPP-routed v, as a VOP2 DPP add on the low halves and a DPP add-with-carry
// on the high halves (two VALU ops per value instead of two DPP moves and a
// 64-bit add).  Rows of a step are interleaved, so every DPP read is at least
// two VALU ops after the write of its source; s_nop 1 covers values written
// just before the block.  Lanes whose source is outside the row read 0
// (bound_ctrl); rows masked off by row_mask keep their value.
#define HZD_DPP64_2(mod)                                                                   \
  asm("s_nop 1\n\t"                                                                        \
      "v_add_co_u32_dpp %0, vcc, %0, %0 " mod "\n\t"                                       \
      "v_addc_co_u32_dpp %1, vcc, %1, %1, vcc " mod "\n\t"                                 \
      "v_add_co_u32_dpp %2, vcc, %2, %2 " mod "\n\t"                                       \
      "v_addc_co_u32_dpp %3, vcc, %3, %3, vcc " mod                                       \
      : "+v"(lo[0]), "+v"(hi[0]), "+v"(lo[1]), "+v"(hi[1])                                \
      :                                                                                  \
      : "vcc")
#define HZD_DPP64_4(mod)                                                                   \
  asm("s_nop 1\n\t"                                                                        \
      "v_add_co_u32_dpp %0, vcc, %0, %0 " mod "\n\t"                                       \
      "v_addc_co_u32_dpp %1, vcc, %1, %1, vcc " mod "\n\t"                                 \
      "v_add_co_u32_dpp %2, vcc, %2, %2 " mod "\n\t"                                       \
      "v_addc_co_u32_dpp %3, vcc, %3, %3, vcc " mod "\n\t"                                 \
      "v_add_co_u32_dpp %4, vcc, %4, %4 " mod "\n\t"                                       \
      "v_addc_co_u32_dpp %5, vcc, %5, %5, vcc " mod "\n\t"                                 \
      "v_add_co_u32_dpp %6, vcc, %6, %6 " mod "\n\t"                                       \
      "v_addc_co_u32_dpp %7, vcc, %7, %7, vcc " mod                                       \
      : "+v"(lo[0]), "+v"(hi[0]), "+v"(lo[1]), "+v"(hi[1]), "+v"(lo[2]), "+v"(hi[2]),     \
        "+v"(lo[3]), "+v"(hi[3])                                                          \
      :                                                                                  \
      : "vcc")

// Inclusive scans over the 64 lanes of NR (2 or 4) independent 64-bit values
// (two's complement, so signed and unsigned alike), the same lane pattern as
// wave_incl_scan.
template <int NR>
__device__ __forceinline__ void wave_incl_scan64(unsigned long long (&v)[NR]) {
  static_assert(NR == 2 || NR == 4, "2 or 4 rows per scan");
  uint32_t lo[NR], hi[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    lo[j] = (uint32_t)v[j];
    hi[j] = (uint32_t)(v[j] >> 32);
  }
  if constexpr (NR == 2) {
    HZD_DPP64_2("row_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    HZD_DPP64_2("row_shr:2 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    HZD_DPP64_2("row_shr:4 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    HZD_DPP64_2("row_shr:8 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    HZD_DPP64_2("row_bcast:15 row_mask:0xa bank_mask:0xf");
    HZD_DPP64_2("row_bcast:31 row_mask:0xc bank_mask:0xf");
  } else {
    HZD_DPP64_4("row_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    HZD_DPP64_4("row_shr:2 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    HZD_DPP64_4("row_shr:4 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    HZD_DPP64_4("row_shr:8 row_mask:0xf bank_mask:0xf bound_ctrl:1");
    HZD_DPP64_4("row_bcast:15 row_mask:0xa bank_mask:0xf");
    HZD_DPP64_4("row_bcast:31 row_mask:0xc bank_mask:0xf");
  }
#pragma unroll
  for (int j = 0; j < NR; ++j) v[j] = ((unsigned long long)hi[j] << 32) | lo[j];
}
#undef HZD_DPP64_2
#undef HZD_DPP64_4

// Prefix sums over the 256 columns of one LDS row, 4 columns per lane (one
// wave per row of the array).
// NR rows of 256 values each, `stride` elements apart: independent scans
// whose DPP steps interleave.
// Physical slot of strip column c in the scan buffers.  A lane of the scan
// owns 4 consecutive 8-byte columns (32 bytes); the two 16-byte halves are
// swapped in every other group of four lanes, so the 128-bit accesses of 8
// consecutive lanes cover all 32 LDS banks once (without the swap, lanes l
// and l + 4 hit the same banks).
__device__ __forceinline__ int qsw(int c) { return c ^ ((c >> 3) & 2); }

template <typename T, int NR>
__device__ __forceinline__ void wave_prefix256_rows(T* base, int stride) {
  static_assert(sizeof(T) == 8, "64-bit sums");
  const int lane = threadIdx.x & 63;
  const int h0 = 4 * lane + (((lane >> 2) & 1) << 1);   // slot of columns 4l, 4l+1 (qsw)
  const int h1 = h0 ^ 2;                                // slot of columns 4l+2, 4l+3
  T v[NR][4];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    const ulonglong2 lo = *reinterpret_cast<const ulonglong2*>(base + j * stride + h0);
    const ulonglong2 hi = *reinterpret_cast<const ulonglong2*>(base + j * stride + h1);
    v[j][0] = (T)lo.x; v[j][1] = (T)lo.y; v[j][2] = (T)hi.x; v[j][3] = (T)hi.y;
  }
  unsigned long long ex[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    v[j][1] += v[j][0];
    v[j][2] += v[j][1];
    v[j][3] += v[j][2];
    ex[j] = (unsigned long long)v[j][3];
  }
  wave_incl_scan64<NR>(ex);
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    const T e = (T)(ex[j] - (unsigned long long)v[j][3]);
    *reinterpret_cast<ulonglong2*>(base + j * stride + h0) =
        make_ulonglong2((unsigned long long)(v[j][0] + e), (unsigned long long)(v[j][1] + e));
    *reinterpret_cast<ulonglong2*>(base + j * stride + h1) =
        make_ulonglong2((unsigned long long)(v[j][2] + e), (unsigned long long)(v[j][3] + e));
  }
}

// Storage of the fixed-point a, b (see AbFixed): int32 pairs, or int64 pairs
// when the int32 rounding would move t by more than 1e-6 t0.
template <bool AB64> struct AbStore {
  using V = int2;
  using E = int;
  static constexpr double lim = 2147483647.0;
  __device__ static V make(double a, double b) { return make_int2((int)a, (int)b); }
};
template <> struct AbStore<true> {
  using V = longlong2;
  using E = long long;
  static constexpr double lim = 4.0e18;
  __device__ static V make(double a, double b) { return make_longlong2((long long)a, (long long)b); }
};

// Eq. (6), stage 1 (He et al. 2013 box form).  Each thread keeps exact u64
// vertical window sums of L, L^2, P, L*P for its column, sliding down the
// rows.  Rows are handled kRpi at a time: the window sums of kRpi rows go to
// LDS, one barrier, each wave prefix-sums one quantity of all kRpi rows
// across the strip (independent DPP scans), another barrier, and the
// kRpi x SW outputs of the phase, dealt NI to a thread, are formed from
// clipped (2r+1)^2 box sums as differences of two prefixes.  Operands of the
// next kRpi rows are loaded while the current ones are processed.  Means, var
// and cov are formed in FP64; a and b leave as int32 fixed point with the
// frame's scale, and their 8-row chunk sums per column (for stage 2's initial
// windows) are merged in LDS.
template <int NI, bool AB64>
__global__ __launch_bounds__(256) void k_gf_ab(Batch b) {
  using AB = AbStore<AB64>;
  __shared__ unsigned long long s_q[kRpi][4][kGfCols];
  __shared__ double2 s_rows[kGfRowsMax];
  __shared__ unsigned long long s_ch[2][64 * NI];  // a, b sums of each output column's current 8-row chunk
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int f = frame_of(b, blk);
  const FrameDev& fd = b.f[f];
  const GfTile g = gf_tile(fd, blk - b.tile0[f]);
  const int W = g.W, H = g.H, r = g.r;
  const int tid = threadIdx.x, wv = tid >> 6;
  // this thread's column; threads outside the frame read the nearest edge
  // column, whose sums land in prefix entries no in-frame box uses
  const uint2* col = fd.LP + min(max(g.xl, 0), W - 1);
  gf_row_table(g, s_rows);

  unsigned long long sL = 0, sLL = 0, sP = 0, sLP = 0;
  auto add = [&](uint2 v) {
    const unsigned long long L = v.x, P = v.y;
    sL += L; sLL += L * L; sP += P; sLP += L * P;
  };
  auto sub = [&](uint2 v) {
    const unsigned long long L = v.x, P = v.y;
    sL -= L; sLL -= L * L; sP -= P; sLP -= L * P;
  };
  if (g.colin) {  // the initial window from head rows, whole 8-row chunks and tail rows
    const WindowSplit w = split_window(max(0, g.y0 - r), min(H - 1, g.y0 + r), H);
    const int nhead = w.head_end - w.ya, nedge = nhead + (w.yb + 1 - w.tail_beg);
    // chunks c0..c1 from the prefixes inside their groups: + PG[c1]
    // - PG[c0 - 1] (when c0 does not start its group) + the last prefix of
    // every group before c1's.  A window of at most 2 kMaxRadius + 1 rows
    // spans at most three groups.  All of it, and the first kEdgeBatch edge
    // rows, is loaded in one round trip.
    const int c1 = w.c0 + w.nch - 1;
    const int g0 = w.c0 / kGroupChunks, g1 = c1 / kGroupChunks;
    const bool sub0 = w.nch > 0 && (w.c0 % kGroupChunks) != 0;
    const int64_t xl = g.xl;
    ulonglong2 pa[4], pb[4];   // + PG[c1], - PG[c0 - 1], + the ends of groups g0 and g0 + 1
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int c = -1;
      if (w.nch > 0) {
        if (i == 0) c = c1;
        else if (i == 1) c = sub0 ? w.c0 - 1 : -1;
        else if (g0 + (i - 2) < g1) c = (g0 + (i - 2)) * kGroupChunks + kGroupChunks - 1;
      }
      pa[i] = make_ulonglong2(0ull, 0ull);
      pb[i] = make_ulonglong2(0ull, 0ull);
      if (c >= 0) {
        pa[i] = fd.PGa[(int64_t)c * W + xl];
        pb[i] = fd.PGb[(int64_t)c * W + xl];
      }
    }
    for (int e0 = 0; e0 < nedge; e0 += kEdgeBatch) {
      uint2 ev[kEdgeBatch];
#pragma unroll
      for (int i = 0; i < kEdgeBatch; ++i) {
        const int e = e0 + i;
        const int yr = e < nhead ? w.ya + e : w.tail_beg + (e - nhead);
        ev[i] = (e < nedge) ? col[yr * W] : make_uint2(0u, 0u);
      }
#pragma unroll
      for (int i = 0; i < kEdgeBatch; ++i) add(ev[i]);
    }
    // entries not loaded are zero; modular u64 arithmetic keeps the sums exact
    sL += pa[0].x + pa[2].x + pa[3].x - pa[1].x;
    sP += pa[0].y + pa[2].y + pa[3].y - pa[1].y;
    sLL += pb[0].x + pb[2].x + pb[3].x - pb[1].x;
    sLP += pb[0].y + pb[2].y + pb[3].y - pb[1].y;
  }
  // entering/leaving rows of output row yn.  The loads are unconditional
  // (rows clamped into the frame) so that the number of loads in flight is
  // static and a prefetch is waited for only where it is used; rows that do
  // not enter or leave the window are skipped at the use (uniform branches).
  auto fetch = [&](int yn, uint2& vin, uint2& vout) {
    vin = col[min(yn + r, H - 1) * W];  // offsets < W*H < 2^31
    vout = col[min(max(yn - r - 1, 0), H - 1) * W];
  };
  auto enters = [&](int yn) { return yn > g.y0 && yn < g.y1 && yn + r < H; };
  auto leaves = [&](int yn) { return yn > g.y0 && yn < g.y1 && yn - r - 1 >= 0; };
  uint2 pin[kRpi], pout[kRpi];
#pragma unroll
  for (int u = 0; u < kRpi; ++u) fetch(g.y0 + u, pin[u], pout[u]);

  // output items of this thread in a phase: wave w owns row w of the phase,
  // lane l its columns l + 64 j (SW = 64 NI), so a wave's items read only the
  // scans it made itself (no barrier between scan and items) and every wave
  // gets the same share of the FP64 work
  constexpr int SWc = 64 * NI;
  const int lane = tid & 63;
  int ic[NI], iclo[NI], ichi[NI];
  double icw[NI], cwd[NI];
  bool iok[NI];
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    ic[j] = lane + 64 * j;
    const int x = g.x0 + ic[j];
    iok[j] = x < W;
    const int lo = max(x - r, 0), hi = min(x + r, W - 1);
    iclo[j] = lo - (g.x0 - r);
    ichi[j] = hi - (g.x0 - r);
    cwd[j] = (double)(hi - lo + 1);
    icw[j] = rcp_nr(cwd[j]);
  }
  for (int i = tid; i < 2 * SWc; i += 256) (&s_ch[0][0])[i] = 0ull;
  // Eq. (6) from the exact box sums S over n = cw * ch pixels (L = G / kG, P = t / kP):
  //   var = kG^2 / n (S_LL - S_L^2 / n),  cov = kG kP / n (S_LP - S_L S_P / n)
  //   a = cov / (var + eps) = (kP / kG) C / (V + n eps / kG^2)   with V, C the brackets
  //   b = mean(t) - a mean(G) = (kP / n) (S_P - (a kG / kP) S_L)
  const double kG = 1.0 / 255000.0, kP = 1.0 / 268435456.0;
  const double eps_n = (double)fd.eps / (kG * kG);
  const double s = (double)fd.ab_scale, lim = AB::lim;
  const double sa_k = s * kP / kG, sb_k = s * kP;
  for (int yb = g.y0; yb < g.y1; yb += kRpi) {
#pragma unroll
    for (int u = 0; u < kRpi; ++u) {
      if (enters(yb + u)) add(pin[u]);
      if (leaves(yb + u)) sub(pout[u]);
      fetch(yb + kRpi + u, pin[u], pout[u]);
      const int qt = qsw(tid);
      s_q[u][0][qt] = sL;
      s_q[u][1][qt] = sLL;
      s_q[u][2][qt] = sP;
      s_q[u][3][qt] = sLP;
    }
    __syncthreads();
    // wave wv prefix-sums the four quantities of row wv (independent DPP scans)
    wave_prefix256_rows<unsigned long long, 4>(&s_q[wv][0][0], kGfCols);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int u = wv, y = yb + u;
      if (iok[j] && y < g.y1) {
        const int clo = iclo[j], chi = qsw(ichi[j]), cl = qsw(max(clo - 1, 0));
        // box sums as differences of two prefixes; S_L < 2^32, so 32-bit wrap-around is exact
        const uint32_t sl = (uint32_t)s_q[u][0][chi] - (clo > 0 ? (uint32_t)s_q[u][0][cl] : 0u);
        const double SL = (double)sl;
        const double SLL = u64_to_f64(s_q[u][1][chi] - (clo > 0 ? s_q[u][1][cl] : 0ull));
        const double SP = u64_to_f64(s_q[u][2][chi] - (clo > 0 ? s_q[u][2][cl] : 0ull));
        const double SLP = u64_to_f64(s_q[u][3][chi] - (clo > 0 ? s_q[u][3][cl] : 0ull));
        const double2 rw = s_rows[y - g.y0];  // {ch, 1 / ch}
        const double inv_n = icw[j] * rw.y;
        const double t1 = SL * inv_n;
        const double V = fma(-t1, SL, SLL);
        const double C = fma(-t1, SP, SLP);
        const double a2 = C * rcp_nr(fma(cwd[j] * rw.x, eps_n, V));  // a kG / kP
        const double ia = fmin(fmax(__builtin_rint(a2 * sa_k), -lim), lim);
        const double ib = fmin(fmax(__builtin_rint(fma(-a2, SL, SP) * (inv_n * sb_k)), -lim), lim);
        const int x = g.x0 + ic[j];
        reinterpret_cast<typename AB::V*>(fd.AB)[(int64_t)y * W + x] = AB::make(ia, ib);
        // the column's sums of a, b over its aligned 8-row chunk (for stage 2's window)
        atomicAdd(&s_ch[0][ic[j]], (unsigned long long)(long long)(typename AB::E)ia);
        atomicAdd(&s_ch[1][ic[j]], (unsigned long long)(long long)(typename AB::E)ib);
      }
    }
    __syncthreads();
    // the phase's last row ends an 8-row chunk (phases start at multiples of
    // kRpi, a divisor of kChunk): store the chunk sums and start the next
    const int yl = min(yb + kRpi, g.y1) - 1;
    if ((yl & (kChunk - 1)) == kChunk - 1 || yl == H - 1) {
      for (int c = tid; c < SWc; c += 256) {
        const int x = g.x0 + c;
        if (x < W) fd.S8ab[(yl / kChunk) * W + x] = make_longlong2((long long)s_ch[0][c], (long long)s_ch[1][c]);
        s_ch[0][c] = 0ull;
        s_ch[1][c] = 0ull;
      }
    }
  }
}

// Colour-balance sums that do not depend on the tiling: J_gamma in fixed
// point (2^-23 steps; exact for J_gamma >= 1), summed in u64 per block and
// merged with integer atomics.  The consumer forms the gray-world gains.
__device__ __forceinline__ uint32_t cb_fixed(float jg) { return (uint32_t)__builtin_rintf(jg * 8388608.0f); }

__device__ __forceinline__ void cb_accumulate(const FrameDev& fd, int tile, const unsigned long long acc[3],
                                              unsigned long long* s_tmp) {
  const unsigned long long s0 = block_sum(acc[0], s_tmp), s1 = block_sum(acc[1], s_tmp),
                           s2 = block_sum(acc[2], s_tmp);
  if (threadIdx.x == 0) {
    unsigned long long* slot = fd.st->cb[tile % kCbSlots];
    atomicAdd(&slot[0], s0);
    atomicAdd(&slot[1], s1);
    atomicAdd(&slot[2], s2);
  }
}

// Gray-world gains g_c = mean(mu) / mu_c (1 when mu_c = 0) from the slot
// sums: wave 0 reduces the 64 slots (one per lane), then one barrier.
__device__ __forceinline__ void cb_gains(const FrameDev& fd, float g[3], unsigned long long* s_tmp) {
  static_assert(kCbSlots == 64, "one slot per lane of wave 0");
  const int t = threadIdx.x;
  if (t < 64) {
    unsigned long long v0 = fd.st->cb[t][0], v1 = fd.st->cb[t][1], v2 = fd.st->cb[t][2];
    v0 = wave_sum(v0);
    v1 = wave_sum(v1);
    v2 = wave_sum(v2);
    if (t == 0) {
      s_tmp[0] = v0;
      s_tmp[1] = v1;
      s_tmp[2] = v2;
    }
  }
  __syncthreads();
  const double k = 1.0 / (8388608.0 * (double)fd.W * (double)fd.H);
  double mu[3];
  for (int c = 0; c < 3; ++c) mu[c] = (double)s_tmp[c] * k;
  const double mbar = (mu[0] + mu[1] + mu[2]) / 3.0;
  for (int c = 0; c < 3; ++c) g[c] = (float)(mu[c] > 0.0 ? mbar / mu[c] : 1.0);
}

// Percentile ("simple") white balance, the second balance of Sec. IV-E.  The
// sums pass histograms the codes RNE(J_gamma^c) the unbalanced output would
// have (per block in LDS, merged into the frame's slots with integer
// atomics); the output pass reads the black point lo (the (k+1)-th smallest
// code) and the white point hi (the (k+1)-th largest) of each channel off the
// merged histograms and stretches the channel: clamp((J_gamma - lo) 255 /
// (hi - lo), 0, 255), or leaves it when hi <= lo.  Every block derives the
// same points from the same integers.
constexpr int kWbBins = 3 * 256;

__device__ __forceinline__ void wb_hist_zero(uint32_t* s_wbh) {
  for (int i = threadIdx.x; i < kWbBins; i += 256) s_wbh[i] = 0u;
}

__device__ __forceinline__ void wb_hist_add(uint32_t* s_wbh, const float Jg[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) atomicAdd(&s_wbh[c * 256 + rne_u8(Jg[c])], 1u);
}

__device__ __forceinline__ void wb_hist_merge(const FrameDev& fd, int tile, const uint32_t* s_wbh) {
  __syncthreads();
  uint32_t* slot = &fd.st->wbh[tile % kHistSlots][0][0];
  for (int i = threadIdx.x; i < kWbBins; i += 256) {
    const uint32_t v = s_wbh[i];
    if (v) atomicAdd(&slot[i], v);
  }
}

struct WbConsts {
  float lo[3], sc[3];
  bool on[3];
};

// Black and white points of the three channels (256-thread blocks: thread t
// holds bin t; an inclusive scan gives #{q <= t}).  lo is the bin where the
// count first exceeds k; hi is the last bin with more than k codes at or
// above it, i.e. the bin where #{q < t} < N - k <= #{q <= t}.
__device__ __forceinline__ WbConsts wb_points(const FrameDev& fd, uint32_t* s_tmp, int* s_pts) {
  const int t = threadIdx.x;
  uint32_t h[3] = {0u, 0u, 0u};
#pragma unroll
  for (int sl = 0; sl < kHistSlots; ++sl)
#pragma unroll
    for (int c = 0; c < 3; ++c) h[c] += fd.st->wbh[sl][c][t];
  const uint32_t N = (uint32_t)fd.W * (uint32_t)fd.H, k = (uint32_t)fd.wb_k;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    uint32_t tot;
    const uint32_t incl = block_scan_total<4>(h[c], s_tmp, tot), excl = incl - h[c];
    if (incl > k && excl <= k) s_pts[2 * c] = t;
    if (excl < N - k && incl >= N - k) s_pts[2 * c + 1] = t;
  }
  __syncthreads();
  WbConsts w;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int lo = s_pts[2 * c], hi = s_pts[2 * c + 1];
    w.on[c] = hi > lo;
    w.lo[c] = (float)lo;
    w.sc[c] = w.on[c] ? 255.0f / (float)(hi - lo) : 1.0f;
  }
  return w;
}

__device__ __forceinline__ float wb_apply(const WbConsts& w, int c, float jg) {
  return w.on[c] ? __builtin_amdgcn_fmed3f((jg - w.lo[c]) * w.sc[c], 0.0f, 255.0f) : jg;
}

// Adaptive gamma (the abstract's "gamma-adaptive" correction, with the rule
// gamma = ln(mu) / ln(tau)): mu is the mean BT.601 luma of J / 255 from exact
// fixed-point sums, floored at 2^-20, and gamma is clamped to [1/2, 2].
// Every block of a launch derives the same value from the same integers.
__device__ __forceinline__ uint32_t luma_fixed(const float J[3]) {
  const float y = fmaf(0.114f, J[2], fmaf(0.587f, J[1], 0.299f * J[0]));   // <= 255
  return (uint32_t)__builtin_rintf(y * 65536.0f);
}

__device__ __forceinline__ void luma_accumulate(const FrameDev& fd, int tile, unsigned long long acc,
                                                unsigned long long* s_tmp) {
  const unsigned long long v = block_sum(acc, s_tmp);
  if (threadIdx.x == 0) atomicAdd(&fd.st->luma[tile % kCbSlots], v);
}

__device__ __forceinline__ void adaptive_gamma(const FrameDev& fd, ReconConsts& rc, unsigned long long* s_g) {
  static_assert(kCbSlots == 64, "one slot per lane of wave 0");
  const int t = threadIdx.x;
  if (t < 64) {
    const unsigned long long v = wave_sum(fd.st->luma[t]);
    if (t == 0) *s_g = v;
  }
  __syncthreads();
  const double mu = (double)(*s_g) / (65536.0 * 255.0 * (double)fd.W * (double)fd.H);
  double g = log(fmax(mu, 0x1p-20)) / log((double)fd.gamma_target);
  g = fmin(fmax(g, 0.5), 2.0);
  rc.inv_gamma = (float)(1.0 / g);
  rc.bias = (float)(log2(255.0) * (1.0 - 1.0 / g));
  rc.gamma_is_one = g == 1.0;
}

// ------------------------------------------------------------------- k_gf_q
// Eq. (6), stage 2: box means of a and b (exact i64 sums of the fixed-point
// values, same strip scheme, kRpi rows per barrier phase), q = mean(a) G +
// mean(b), clamped to [t0, 1].  PHASE 0: fuse Eqs. (7)-(8) and write the
// output.  PHASE 1: store the refined t and the colour-balance sums.  PHASE 2:
// store the refined t and the luma sums of J (adaptive gamma).  AUX: some
// frame of the launch asks for its t or J maps.
template <int NI, int PHASE, bool FP16, bool AUX, bool AB64>
__global__ __launch_bounds__(256) void k_gf_q(Batch b) {
  using ABV = typename AbStore<AB64>::V;
  // two buffers, alternating by phase: a phase's scan and output read one
  // while the next phase's column sums go to the other, so a phase needs only
  // the barrier after its column sums (a buffer is rewritten two phases
  // later, after every wave has passed the next phase's barrier and so
  // finished this output; each wave scans and reads only its own row)
  __shared__ long long s_q[2][kRpi][2][kGfCols];
  __shared__ double2 s_rows[kGfRowsMax];
  __shared__ unsigned long long s_red[4];
  __shared__ uint32_t s_wbh[PHASE == 1 ? kWbBins : 1];
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int f = frame_of(b, blk);
  const FrameDev& fd = b.f[f];
  const int tile = blk - b.tile0[f];
  const GfTile g = gf_tile(fd, tile);
  const int W = g.W, H = g.H, r = g.r;
  const int tid = threadIdx.x, wv = tid >> 6;
  // this thread's column; threads outside the frame read the nearest edge
  // column, whose sums land in prefix entries no in-frame box uses
  const ABV* col = reinterpret_cast<const ABV*>(fd.AB) + min(max(g.xl, 0), W - 1);
  gf_row_table(g, s_rows);
  const ReconConsts rc = recon_consts(fd);
  const bool wb = PHASE == 1 && (fd.flags & kFdWbPercentile);   // block-uniform
  if (wb) wb_hist_zero(s_wbh);   // ordered before its first use by the row loop's first barrier

  long long sa = 0, sb = 0;
  if (g.colin) {  // the initial window from head rows, 8-row chunk sums and tail rows
    const WindowSplit w = split_window(max(0, g.y0 - r), min(H - 1, g.y0 + r), H);
    const int nhead = w.head_end - w.ya, nedge = nhead + (w.yb + 1 - w.tail_beg);
    // the chunk sums (all of a window's, with int32 a, b) and the first
    // kEdgeBatch edge rows in one round trip
    constexpr int kQC = AB64 ? 8 : 2 * kGroupChunks;
    longlong2 cs[kQC];
#pragma unroll
    for (int i = 0; i < kQC; ++i)
      cs[i] = (i < w.nch) ? fd.S8ab[(int64_t)(w.c0 + i) * W + g.xl] : make_longlong2(0ll, 0ll);
    for (int e0 = 0; e0 < nedge; e0 += kEdgeBatch) {
      ABV ev[kEdgeBatch];
#pragma unroll
      for (int i = 0; i < kEdgeBatch; ++i) {
        const int e = e0 + i;
        const int yr = e < nhead ? w.ya + e : w.tail_beg + (e - nhead);
        ev[i] = (e < nedge) ? col[(int64_t)yr * W] : ABV{0, 0};
      }
#pragma unroll
      for (int i = 0; i < kEdgeBatch; ++i) {
        sa += ev[i].x;
        sb += ev[i].y;
      }
    }
#pragma unroll
    for (int i = 0; i < kQC; ++i) {
      sa += cs[i].x;
      sb += cs[i].y;
    }
    for (int c = kQC; c < w.nch; c += kQC) {
#pragma unroll
      for (int i = 0; i < kQC; ++i)
        cs[i] = (c + i < w.nch) ? fd.S8ab[(int64_t)(w.c0 + c + i) * W + g.xl] : make_longlong2(0ll, 0ll);
#pragma unroll
      for (int i = 0; i < kQC; ++i) {
        sa += cs[i].x;
        sb += cs[i].y;
      }
    }
  }
  // unconditional loads (rows and columns clamped into the frame): the number
  // of loads in flight is static, so a prefetch is waited for only at its use
  auto fetch = [&](int yn, ABV& vin, ABV& vout) {
    vin = col[min(yn + r, H - 1) * W];  // offsets < W*H < 2^31
    vout = col[min(max(yn - r - 1, 0), H - 1) * W];
  };
  auto enters = [&](int yn) { return yn > g.y0 && yn < g.y1 && yn + r < H; };
  auto leaves = [&](int yn) { return yn > g.y0 && yn < g.y1 && yn - r - 1 >= 0; };
  // output items of this thread in a phase: wave w owns row w of the phase,
  // lane l its columns l + 64 j (SW = 64 NI); a wave's items read only the
  // scans it made itself
  const int lane = tid & 63;
  int ic[NI], iclo[NI], ichi[NI], ixc[NI];
  double icw_s[NI];
  bool iok[NI];
  const double inv_s = 1.0 / (double)fd.ab_scale;   // exact: the scale is a power of two
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    ic[j] = lane + 64 * j;
    const int x = g.x0 + ic[j];
    iok[j] = x < W;
    ixc[j] = min(x, W - 1);
    const int lo = max(x - r, 0), hi = min(x + r, W - 1);
    iclo[j] = lo - (g.x0 - r);
    ichi[j] = hi - (g.x0 - r);
    icw_s[j] = inv_s * rcp_nr((double)(hi - lo + 1));
  }
  // an output pixel's colour (R, G in one 16-bit load, B), loaded one phase
  // ahead (row clamped into the frame: unconditional loads); its guide value
  // L = 299 R + 587 G + 114 B is formed from the same bytes, as k_gf_prep does
  auto fetch_px = [&](int yn, int xc, uint32_t& rg, uint32_t& bl) {
    const int yc = min(yn, H - 1);
    const uint8_t* p = fd.src + (int64_t)yc * fd.src_pitch + 3 * xc;
    uint16_t v;
    __builtin_memcpy(&v, p, 2);
    rg = v;
    bl = p[2];
  };
  ABV pin[kRpi], pout[kRpi];
  uint32_t pRG[NI], pB[NI];
#pragma unroll
  for (int u = 0; u < kRpi; ++u) fetch(g.y0 + u, pin[u], pout[u]);
#pragma unroll
  for (int j = 0; j < NI; ++j) fetch_px(g.y0 + wv, ixc[j], pRG[j], pB[j]);

  const double t0 = (double)fd.t0;
  unsigned long long acc[3] = {0ull, 0ull, 0ull};
  for (int yb = g.y0, buf = 0; yb < g.y1; yb += kRpi, buf ^= 1) {
    long long(&q)[kRpi][2][kGfCols] = s_q[buf];
    uint32_t curRG[NI], curB[NI];
#pragma unroll
    for (int u = 0; u < kRpi; ++u) {
      if (enters(yb + u)) {
        sa += pin[u].x;
        sb += pin[u].y;
      }
      if (leaves(yb + u)) {
        sa -= pout[u].x;
        sb -= pout[u].y;
      }
      fetch(yb + kRpi + u, pin[u], pout[u]);
      q[u][0][qsw(tid)] = sa;
      q[u][1][qsw(tid)] = sb;
    }
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      curRG[j] = pRG[j];
      curB[j] = pB[j];
      fetch_px(yb + kRpi + wv, ixc[j], pRG[j], pB[j]);
    }
    __syncthreads();
    // wave wv prefix-sums the two quantities of row wv
    wave_prefix256_rows<long long, 2>(&q[wv][0][0], kGfCols);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int u = wv, y = yb + u;
      if (iok[j] && y < g.y1) {
        const int clo = iclo[j], chi = qsw(ichi[j]), cl = qsw(max(clo - 1, 0)), x = g.x0 + ic[j];
        const double qa = i64_to_f64(q[u][0][chi] - (clo > 0 ? q[u][0][cl] : 0ll));
        const double qb = i64_to_f64(q[u][1][chi] - (clo > 0 ? q[u][1][cl] : 0ll));
        const double in = icw_s[j] * s_rows[y - g.y0].y;
        const uint32_t L = 299u * (curRG[j] & 0xFFu) + 587u * (curRG[j] >> 8) + 114u * curB[j];
        const double G = (double)L * (1.0 / 255000.0);
        const double qt = fma(qa * in, G, qb * in);
        float t = (float)fmin(fmax(qt, t0), 1.0);
        // FP16 applies to the stored t map (PHASE 1, 2): the sums here use the same
        // binary16 value that the later passes read back.  The fused output
        // (PHASE 0) keeps binary32 t, as it never leaves registers.
        if (FP16 && PHASE != 0) t = round_half(t);
        const int64_t pi = (int64_t)y * W + x;
        if (AUX && fd.t_out) fd.t_out[pi] = t;
        const uint32_t c = curRG[j] | (curB[j] << 16);
        float I[3] = {(float)(c & 0xFFu), (float)((c >> 8) & 0xFFu), (float)((c >> 16) & 0xFFu)};
        float J[3], Jg[3];
        recon_pixel(rc, I, t, J, Jg);
        if (AUX && fd.J_out) {
          fd.J_out[3 * pi] = J[0]; fd.J_out[3 * pi + 1] = J[1]; fd.J_out[3 * pi + 2] = J[2];
        }
        if (PHASE == 0) {
          uint8_t* o = fd.dst + (int64_t)y * fd.dst_pitch + 3 * x;
          // v_cvt_pk_u8_f32: clamp, round half to even, as rne_u8
          o[0] = (uint8_t)__builtin_amdgcn_cvt_pk_u8_f32(Jg[0], 0u, 0u);
          o[1] = (uint8_t)__builtin_amdgcn_cvt_pk_u8_f32(Jg[1], 0u, 0u);
          o[2] = (uint8_t)__builtin_amdgcn_cvt_pk_u8_f32(Jg[2], 0u, 0u);
        } else {
          if (FP16) reinterpret_cast<__half*>(fd.tmap)[pi] = __float2half_rn(t);
          else reinterpret_cast<float*>(fd.tmap)[pi] = t;
          if (PHASE == 1) {
            if (wb) {
              wb_hist_add(s_wbh, Jg);
            } else {
              acc[0] += cb_fixed(Jg[0]); acc[1] += cb_fixed(Jg[1]); acc[2] += cb_fixed(Jg[2]);
            }
          } else {
            acc[0] += luma_fixed(J);
          }
        }
      }
    }
  }
  if (PHASE == 1) {
    if (wb) wb_hist_merge(fd, tile, s_wbh);
    else cb_accumulate(fd, tile, acc, s_red);
  }
  if (PHASE == 2) luma_accumulate(fd, tile, acc[0], s_red);
}

// ------------------------------------------------------------------ k_recon
// Pointwise Eqs. (4)-(5) (or the refined t), Eq. (7), Eq. (8) and the colour
// balance.  A block covers kReconPx pixels of one row: each thread takes two
// groups of 4 pixels, kReconPx / 2 apart, and issues the loads of both groups
// before any arithmetic.  PHASE 0: write the output.  PHASE 1: colour-balance
// sums only.  PHASE 2: form the gray-world gains from the sums, apply them and
// write.  PHASE 3: luma sums of J only (adaptive gamma; the later phases of a
// frame with adaptive gamma take its gamma from them).  AUX: some frame of
// the launch asks for its t or J maps.
__device__ __forceinline__ void load_rgb12(const uint8_t* p, int nx, bool aligned, uint32_t w[3]) {
  if (aligned && nx == 4) {
    const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
    w[0] = q[0]; w[1] = q[1]; w[2] = q[2];
  } else {
    uint8_t tmp[12] = {0};
    for (int i = 0; i < 3 * nx; ++i) tmp[i] = p[i];
    w[0] = tmp[0] | (tmp[1] << 8) | (tmp[2] << 16) | ((uint32_t)tmp[3] << 24);
    w[1] = tmp[4] | (tmp[5] << 8) | (tmp[6] << 16) | ((uint32_t)tmp[7] << 24);
    w[2] = tmp[8] | (tmp[9] << 8) | (tmp[10] << 16) | ((uint32_t)tmp[11] << 24);
  }
}

template <int TSRC, int PHASE, bool FP16, bool AUX>
__global__ __launch_bounds__(256) void k_recon(Batch b) {
  static_assert(kReconPx == 2 * 4 * 256, "two groups of 4 pixels per thread");
  constexpr bool OUT = PHASE == 0 || PHASE == 2;   // this phase writes the output
  __shared__ unsigned long long s_red[4];
  __shared__ unsigned long long s_gam[1];
  __shared__ uint32_t s_wbh[PHASE == 1 ? kWbBins : 1];
  __shared__ uint32_t s_wtmp[4];
  __shared__ int s_wpts[6];
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int f = frame_of(b, blk);
  const FrameDev& fd = b.f[f];
  const int tile = blk - b.tile0[f];
  const int W = fd.W;
  const int per_row = (W + kReconPx - 1) / kReconPx;
  const int y = tile / per_row;
  const int xb = (tile - y * per_row) * kReconPx + 4 * (int)threadIdx.x;
  // the pixels' loads go out first: the frame-wide constants below (gains,
  // points, adaptive gamma) take a round trip and a barrier of their own
  constexpr int NG = 2;
  int x0[NG], nx[NG];
  uint32_t iw[NG][3], ew[NG][3];
  float tm[NG][4];
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    x0[q] = xb + q * (kReconPx / 2);
    nx[q] = max(0, min(4, W - x0[q]));
    iw[q][0] = iw[q][1] = iw[q][2] = 0u;
    ew[q][0] = ew[q][1] = ew[q][2] = 0u;
    tm[q][0] = tm[q][1] = tm[q][2] = tm[q][3] = 1.0f;
    if (nx[q] > 0) {
      load_rgb12(fd.src + (int64_t)y * fd.src_pitch + 3 * x0[q], nx[q], (fd.flags & kFdAligned), iw[q]);
      if (TSRC == TSRC_HE) load_rgb12(fd.E + (int64_t)y * fd.E_pitch + 3 * x0[q], nx[q], true, ew[q]);
      if (TSRC == TSRC_TMAP) {
        const int64_t pi = (int64_t)y * W + x0[q];
        if (nx[q] == 4 && (pi & 3) == 0) {  // one 16- (8-) byte load
          if (FP16) {
            const uint2 h = *reinterpret_cast<const uint2*>(reinterpret_cast<const __half*>(fd.tmap) + pi);
            tm[q][0] = __half2float(__ushort_as_half((unsigned short)(h.x & 0xFFFFu)));
            tm[q][1] = __half2float(__ushort_as_half((unsigned short)(h.x >> 16)));
            tm[q][2] = __half2float(__ushort_as_half((unsigned short)(h.y & 0xFFFFu)));
            tm[q][3] = __half2float(__ushort_as_half((unsigned short)(h.y >> 16)));
          } else {
            const float4 v = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(fd.tmap) + pi);
            tm[q][0] = v.x; tm[q][1] = v.y; tm[q][2] = v.z; tm[q][3] = v.w;
          }
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (i < nx[q])
              tm[q][i] = FP16 ? __half2float(reinterpret_cast<const __half*>(fd.tmap)[pi + i])
                              : reinterpret_cast<const float*>(fd.tmap)[pi + i];
        }
      }
    }
  }

  const TxConsts k = tx_consts(fd);
  ReconConsts rc = recon_consts(fd);
  if (PHASE != 3 && (fd.flags & kFdGammaAdaptive)) adaptive_gamma(fd, rc, s_gam);   // uniform per block
  const bool wb = (PHASE == 1 || PHASE == 2) && (fd.flags & kFdWbPercentile);   // block-uniform
  float gain[3] = {1.f, 1.f, 1.f};
  WbConsts wbc;
  if (PHASE == 2) {
    if (wb) wbc = wb_points(fd, s_wtmp, s_wpts);
    else cb_gains(fd, gain, s_red);
  }
  if (PHASE == 1 && wb) {
    wb_hist_zero(s_wbh);
    __syncthreads();
  }
  unsigned long long acc[3] = {0ull, 0ull, 0ull};

#pragma unroll
  for (int q = 0; q < NG; ++q) {
    if (nx[q] == 0) continue;
    uint32_t ow[3] = {0, 0, 0};
    auto px = [&](int i) {
      float I[3], J[3], Jg[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int byte = 3 * i + c;
        I[c] = (float)((iw[q][byte >> 2] >> (8 * (byte & 3))) & 0xFFu);
      }
      float t;
      if (TSRC == TSRC_HE) {
        float e[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int byte = 3 * i + c;
          e[c] = (float)((ew[q][byte >> 2] >> (8 * (byte & 3))) & 0xFFu);
        }
        t = tx_he(k, e[0], e[1], e[2]);
      } else if (TSRC == TSRC_PAPER) {
        t = tx_paper(k, fminf(fminf(I[0], I[1]), I[2]));
      } else {
        t = tm[q][i];  // binary16 maps hold values exactly representable in binary32
      }
      recon_pixel(rc, I, t, J, Jg);
      if (PHASE == 3) {
        acc[0] += luma_fixed(J);
      } else if (PHASE == 1) {
        if (wb) {
          wb_hist_add(s_wbh, Jg);
        } else {
          acc[0] += cb_fixed(Jg[0]); acc[1] += cb_fixed(Jg[1]); acc[2] += cb_fixed(Jg[2]);
        }
      } else {
        const int64_t pi = (int64_t)y * W + x0[q] + i;
        if (AUX && fd.t_out) fd.t_out[pi] = t;
        if (AUX && fd.J_out) {
          fd.J_out[3 * pi] = J[0]; fd.J_out[3 * pi + 1] = J[1]; fd.J_out[3 * pi + 2] = J[2];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float v = (PHASE == 2) ? (wb ? wb_apply(wbc, c, Jg[c]) : fminf(255.0f, gain[c] * Jg[c])) : Jg[c];
          const int byte = 3 * i + c;
          // one v_cvt_pk_u8_f32 per byte: clamp to [0, 255], round half to even and
          // insert, bit-identical to rne_u8 (checked on the GPU over a sweep of
          // floats with every half-way case and values out of range)
          ow[byte >> 2] = __builtin_amdgcn_cvt_pk_u8_f32(v, (uint32_t)(byte & 3), ow[byte >> 2]);
        }
      }
    };
    if (nx[q] == 4) {  // no per-pixel branches: the four pixels' chains interleave
#pragma unroll
      for (int i = 0; i < 4; ++i) px(i);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (i < nx[q]) px(i);
    }
    if (OUT) {
      uint8_t* Op = fd.dst + (int64_t)y * fd.dst_pitch + 3 * x0[q];
      if ((fd.flags & kFdAligned) && nx[q] == 4) {
        uint32_t* o = reinterpret_cast<uint32_t*>(Op);
        o[0] = ow[0]; o[1] = ow[1]; o[2] = ow[2];
      } else {
        for (int i = 0; i < 3 * nx[q]; ++i) Op[i] = (uint8_t)(ow[i >> 2] >> (8 * (i & 3)));
      }
    }
  }
  if (PHASE == 1) {
    if (wb) wb_hist_merge(fd, tile, s_wbh);
    else cb_accumulate(fd, tile, acc, s_red);
  }
  if (PHASE == 3) luma_accumulate(fd, tile, acc[0], s_red);
}

// ----------------------------------------------------------------- launches
namespace {

template <typename B, typename Fn>
int fill_tiles(B& b, Fn blocks_of) {
  int acc = 0;
  for (int i = 0; i < b.n; ++i) {
    b.tile0[i] = acc;
    acc += blocks_of(b.f[i]);
  }
  b.tile0[b.n] = acc;
  return acc;
}

template <int HP>
hipError_t dark_hp(const Batch& b, int nblk, bool write_E, hipStream_t s) {
  if (b.f[0].flags & kFdFresh) nblk += b.n;   // the leading blocks that zero the frames' state
  if (write_E) hipLaunchKernelGGL((k_dark<HP, true>), dim3(nblk), dim3(256), 0, s, b);
  else hipLaunchKernelGGL((k_dark<HP, false>), dim3(nblk), dim3(256), 0, s, b);
  return hipGetLastError();
}

// Whether any frame of the launch wants its t or J map (the kernels then keep
// the per-pixel branches for those stores).
bool any_aux_maps(const Batch& b) {
  for (int i = 0; i < b.n; ++i)
    if (b.f[i].t_out || b.f[i].J_out) return true;
  return false;
}

template <int NI, int PHASE, bool AB64>
hipError_t gf_q_n(const Batch& b, int nblk, bool fp16, bool aux, hipStream_t s) {
  if (fp16) {
    if (aux) hipLaunchKernelGGL((k_gf_q<NI, PHASE, true, true, AB64>), dim3(nblk), dim3(256), 0, s, b);
    else hipLaunchKernelGGL((k_gf_q<NI, PHASE, true, false, AB64>), dim3(nblk), dim3(256), 0, s, b);
  } else {
    if (aux) hipLaunchKernelGGL((k_gf_q<NI, PHASE, false, true, AB64>), dim3(nblk), dim3(256), 0, s, b);
    else hipLaunchKernelGGL((k_gf_q<NI, PHASE, false, false, AB64>), dim3(nblk), dim3(256), 0, s, b);
  }
  return hipGetLastError();
}

template <int PHASE>
hipError_t gf_q_p(const Batch& b, int nblk, int radius, bool fp16, bool aux, bool ab64, hipStream_t s) {
  if (ab64) {
    if (gf_strip(radius) == 192) return gf_q_n<3, PHASE, true>(b, nblk, fp16, aux, s);
    return gf_q_n<2, PHASE, true>(b, nblk, fp16, aux, s);
  }
  if (gf_strip(radius) == 192) return gf_q_n<3, PHASE, false>(b, nblk, fp16, aux, s);
  return gf_q_n<2, PHASE, false>(b, nblk, fp16, aux, s);
}

}  // namespace

hipError_t launch_resize(ResizeBatch r, hipStream_t s) {
  const int nblk = fill_tiles(r, [](const ResizeDev& f) { return ((f.Ho + 3) / 4) * ((f.Wo + 255) / 256); });
  hipLaunchKernelGGL(k_resize, dim3(nblk), dim3(256), 0, s, r);
  return hipGetLastError();
}

hipError_t launch_init(Batch b, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(b.n), dim3(256), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_dark(Batch b, const GroupKey& g, bool write_E, hipStream_t s) {
  const int nblk = fill_tiles(b, [](const FrameDev& f) {
    return ((f.W + kDarkTW - 1) / kDarkTW) * ((f.H + kDarkTH - 1) / kDarkTH);
  });
  switch (g.half_patch) {
    case 0: return dark_hp<0>(b, nblk, write_E, s);
    case 1: return dark_hp<1>(b, nblk, write_E, s);
    case 2: return dark_hp<2>(b, nblk, write_E, s);
    case 3: return dark_hp<3>(b, nblk, write_E, s);
    case 4: return dark_hp<4>(b, nblk, write_E, s);
    case 5: return dark_hp<5>(b, nblk, write_E, s);
    case 6: return dark_hp<6>(b, nblk, write_E, s);
    case 7: return dark_hp<7>(b, nblk, write_E, s);
    case 8: return dark_hp<8>(b, nblk, write_E, s);
    case 9: return dark_hp<9>(b, nblk, write_E, s);
    case 10: return dark_hp<10>(b, nblk, write_E, s);
    case 11: return dark_hp<11>(b, nblk, write_E, s);
    case 12: return dark_hp<12>(b, nblk, write_E, s);
    case 13: return dark_hp<13>(b, nblk, write_E, s);
    case 14: return dark_hp<14>(b, nblk, write_E, s);
    case 15: return dark_hp<15>(b, nblk, write_E, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_select_one(Batch b, hipStream_t s) {
  for (int i = 0; i < b.n; ++i)
    if (!select_one_fits(b.f[i].W, b.f[i].H)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_select_one<kOneVecMax>), dim3(b.n), dim3(kOneT), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_select(Batch b, hipStream_t s) {
  const int rows = b.n == 1 ? 8 : 4;   // rows (waves) per block
  const int nblk = fill_tiles(b, [rows](const FrameDev& f) { return (f.H + rows - 1) / rows; });
  if (rows == 8) hipLaunchKernelGGL(k_select_rows<512>, dim3(nblk), dim3(512), 0, s, b);
  else hipLaunchKernelGGL(k_select_rows<256>, dim3(nblk), dim3(256), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_gf_prep(Batch b, const GroupKey& g, hipStream_t s) {
  const int nblk = fill_tiles(b, [](const FrameDev& f) {
    const int nch = (f.H + kChunk - 1) / kChunk;
    return ((f.W + 63) / 64) * ((nch + kGroupChunks - 1) / kGroupChunks);
  });
  constexpr int nt = 64 * kGroupChunks;
  if (g.tx == HZD_TX_HE) hipLaunchKernelGGL((k_gf_prep<TSRC_HE>), dim3(nblk), dim3(nt), 0, s, b);
  else hipLaunchKernelGGL((k_gf_prep<TSRC_PAPER>), dim3(nblk), dim3(nt), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_gf_ab(Batch b, const GroupKey& g, hipStream_t s) {
  const int nblk = fill_tiles(b, [](const FrameDev& f) { return gf_blocks(f.W, f.H, f.radius, f.gf_rows); });
  if (g.ab64) {
    if (gf_strip(g.radius) == 192) hipLaunchKernelGGL((k_gf_ab<3, true>), dim3(nblk), dim3(256), 0, s, b);
    else hipLaunchKernelGGL((k_gf_ab<2, true>), dim3(nblk), dim3(256), 0, s, b);
  } else {
    if (gf_strip(g.radius) == 192) hipLaunchKernelGGL((k_gf_ab<3, false>), dim3(nblk), dim3(256), 0, s, b);
    else hipLaunchKernelGGL((k_gf_ab<2, false>), dim3(nblk), dim3(256), 0, s, b);
  }
  return hipGetLastError();
}

hipError_t launch_gf_q(Batch b, const GroupKey& g, hipStream_t s) {
  const int nblk = fill_tiles(b, [](const FrameDev& f) { return gf_blocks(f.W, f.H, f.radius, f.gf_rows); });
  const bool aux = any_aux_maps(b);
  if (g.gadapt) return gf_q_p<2>(b, nblk, g.radius, g.fp16, aux, g.ab64, s);
  if (g.cb) return gf_q_p<1>(b, nblk, g.radius, g.fp16, aux, g.ab64, s);
  return gf_q_p<0>(b, nblk, g.radius, g.fp16, aux, g.ab64, s);
}

namespace {
template <int TSRC, int PHASE>
hipError_t recon_tp(const Batch& b, int nblk, bool fp16, bool aux, hipStream_t s) {
  if (fp16) {
    if (aux) hipLaunchKernelGGL((k_recon<TSRC, PHASE, true, true>), dim3(nblk), dim3(256), 0, s, b);
    else hipLaunchKernelGGL((k_recon<TSRC, PHASE, true, false>), dim3(nblk), dim3(256), 0, s, b);
  } else {
    if (aux) hipLaunchKernelGGL((k_recon<TSRC, PHASE, false, true>), dim3(nblk), dim3(256), 0, s, b);
    else hipLaunchKernelGGL((k_recon<TSRC, PHASE, false, false>), dim3(nblk), dim3(256), 0, s, b);
  }
  return hipGetLastError();
}
template <int TSRC>
hipError_t recon_t(const Batch& b, int nblk, int phase, bool fp16, bool aux, hipStream_t s) {
  switch (phase) {
    case 0: return recon_tp<TSRC, 0>(b, nblk, fp16, aux, s);
    case 1: return recon_tp<TSRC, 1>(b, nblk, fp16, false, s);   // sums only: no maps written
    case 2: return recon_tp<TSRC, 2>(b, nblk, fp16, aux, s);
    case 3: return recon_tp<TSRC, 3>(b, nblk, fp16, false, s);   // luma sums only
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

hipError_t launch_recon(Batch b, const GroupKey& g, int tsrc, int phase, hipStream_t s) {
  const int nblk = fill_tiles(b, [](const FrameDev& f) { return recon_blocks(f.W, f.H); });
  const bool aux = any_aux_maps(b);
  switch (tsrc) {
    case TSRC_HE: return recon_t<TSRC_HE>(b, nblk, phase, g.fp16, aux, s);
    case TSRC_PAPER: return recon_t<TSRC_PAPER>(b, nblk, phase, g.fp16, aux, s);
    case TSRC_TMAP: return recon_t<TSRC_TMAP>(b, nblk, phase, g.fp16, aux, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hzd
