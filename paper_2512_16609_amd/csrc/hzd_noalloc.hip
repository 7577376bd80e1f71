// hzd_dehaze_frame_noalloc: the frame path with its workspace in a static
// device array, for callers that cannot allocate device memory.
//
// The array is a file-scope __device__ object of this translation unit, so
// the loader places one copy in each device's memory when the code object is
// loaded there.  Its name in host code is only a host-side handle: the
// device address of each copy is looked up once per device with
// hipGetSymbolAddress (with that device current) and used everywhere the
// host passes the memory on (the kernels take it as their workspace).
#include <hip/hip_runtime.h>

#include <mutex>

#include "hzd.h"
#include "hzd_internal.h"
#include "hzd_plan.h"

namespace hzd {
namespace {

__device__ __align__(256) uint8_t scratch[HZD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];   // device address of `scratch` on each device (null = not looked up)

// The device address of this device's copy of the array; looked up on the
// first call on the device, with the device current.
int scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(HZD_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  e != hipSuccess ? hipGetErrorString(e) : "null address");
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HZD_OK;
}

}  // namespace
}  // namespace hzd

using namespace hzd;

extern "C" int hzd_dehaze_frame_noalloc(const hzd_params* params, const hzd_frame* frame,
                                        const hzd_frame_aux* aux, void* hip_stream) {
  if (!frame) return fail(HZD_E_INVAL, "frame is NULL");
  std::vector<const hzd_params*> ps;
  std::vector<size_t> offs;
  size_t need = 0;
  int rc = validate_call(params, frame, 1, ps, offs, &need);
  if (rc) return rc;
  if (need > HZD_NOALLOC_SCRATCH_BYTES)
    return fail(HZD_E_NOMEM, "frame %dx%d needs %zu bytes of workspace; the static scratch holds %zu",
                frame->width, frame->height, need, (size_t)HZD_NOALLOC_SCRATCH_BYTES);
  int dev = -1;
  if ((rc = check(hipGetDevice(&dev), "hipGetDevice")) != HZD_OK) return rc;
  if (dev < 0 || dev >= kMaxDevices) return fail(HZD_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  if (s != nullptr) {
    int sdev = -1;
    if ((rc = check(hipStreamGetDevice(s, &sdev), "hipStreamGetDevice")) != HZD_OK) return rc;
    if (sdev != dev) return fail(HZD_E_INVAL, "hip_stream belongs to device %d, the current device is %d", sdev, dev);
  }
  void* ws = nullptr;
  if ((rc = scratch_address(dev, &ws)) != HZD_OK) return rc;
  rc = run_frame_direct(ps[0], *frame, aux, ws, s);
  if (rc == HZD_OK) clear_error();
  return rc;
}
