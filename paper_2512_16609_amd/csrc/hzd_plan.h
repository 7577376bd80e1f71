// Host-side planning helpers shared by the frame/batch entry points and the
// server (hzd_api.cpp, hzd_server.cpp).
#pragma once

#include <stddef.h>

#include <vector>

#include "hzd.h"
#include "hzd_internal.h"

namespace hzd {

int fail(int status, const char* fmt, ...);
void clear_error();
int validate_params(const hzd_params* p);
// Output (working) size of a frame of input size W x H.
void output_size(const hzd_params& p, int W, int H, int* Wo, int* Ho);
int validate_size(const hzd_params& p, int W, int H, int idx);
int validate_frame(const hzd_frame* f, const hzd_params& p, int idx);
GroupKey group_key(const hzd_params& p);
bool operator<(const GroupKey& a, const GroupKey& b);
size_t frame_ws_bytes(const hzd_params& p, int W, int H);
FrameDev make_frame_dev(const hzd_params& p, const hzd_frame& fr, const hzd_frame_aux* aux, uint8_t* ws,
                        ResizeDev* rz);
hzd_tile_config tile_config_for(int W, int H, bool* from_table = nullptr);
void fit_gf_rows(Batch& b);
// fresh: kFreshYes when the launches run directly and once (not recorded into
// a graph), so the frames' state is zeroed by leading blocks of k_dark instead of
// by the init kernel (Batch.epoch is set here); kFreshNo when they may be
// replayed; kFreshAsk: whether s is being captured decides, asked only when
// the init kernel would otherwise run
enum { kFreshNo = 0, kFreshYes = 1, kFreshAsk = 2 };
int run_group(const GroupKey& g, const Batch& b, const ResizeBatch* rz, hipStream_t s, bool prof, int fresh);
// Whether work enqueued on s is being recorded into a graph (true when unknown).
bool stream_capturing(hipStream_t s);
// rz: the resampling descriptors of a group with g.resize (else unused, may be NULL)
int launch_group(const GroupKey& g, const Batch& b, const ResizeBatch* rz, hipStream_t s);
int check(hipError_t e, const char* what);
// Validation shared by the frame/batch entry points (parameters, frames,
// airlight states); fills the per-frame parameters, workspace offsets and the
// total workspace bytes.  No device work.
int validate_call(const hzd_params* params, const hzd_frame* frames, int32_t n,
                  std::vector<const hzd_params*>& ps, std::vector<size_t>& offs, size_t* need);
// One validated frame, launched directly on s: no graph cache, no timing
// events, no helper streams (nothing is created or allocated).
int run_frame_direct(const hzd_params* p, const hzd_frame& fr, const hzd_frame_aux* aux, void* ws,
                     hipStream_t s);

}  // namespace hzd
