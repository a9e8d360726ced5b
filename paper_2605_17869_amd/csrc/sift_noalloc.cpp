// Extraction into a library-owned device scratch array, for callers that
// cannot allocate device memory (code under HIP graph capture, fixed serving
// loops, harnesses that forbid hipMalloc).
//
// The array lives in the code object: every GPU the library runs on holds its
// own copy, at its own address, from module load until the process ends.  In
// host code the array's name is only a host-side stand-in, so its device
// address is looked up once per device with hipGetSymbolAddress and only that
// address is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/sift.h"

namespace sift {
void set_last_error(const std::string& msg);
}

namespace {

constexpr size_t kScratchBytes = SIFT_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device

sift_status fail_msg(sift_status st, const std::string& msg) {
  sift::set_last_error(msg);
  return st;
}

// Device address of the current device's scratch array (looked up on the
// first call on that device, with the device current).
sift_status scratch_ptr(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return fail_msg(SIFT_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return fail_msg(SIFT_ERR_NOT_SUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail_msg(SIFT_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                        hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return SIFT_OK;
}

}  // namespace

extern "C" {

sift_status sift_extract_noalloc(sift_handle* h, const float* d_image, int32_t height,
                                 int32_t width, int64_t pitch, const sift_output* out,
                                 void* stream) {
  if (!h || !d_image || !out) return fail_msg(SIFT_ERR_INVALID_ARG, "null argument");
  size_t need = 0;
  sift_status st = sift_workspace_size(h, height, width, &need);
  if (st != SIFT_OK) return st;
  if (need > kScratchBytes)
    return fail_msg(SIFT_ERR_WORKSPACE_TOO_SMALL,
                    "a " + std::to_string(height) + "x" + std::to_string(width) +
                        " image needs " + std::to_string(need) +
                        " bytes of workspace; the static scratch holds " +
                        std::to_string(kScratchBytes) + " (use sift_extract)");
  void* ws = nullptr;
  if ((st = scratch_ptr(&ws)) != SIFT_OK) return st;
  return sift_extract(h, d_image, height, width, pitch, ws, kScratchBytes, out, stream);
}

size_t sift_noalloc_scratch_bytes(void) { return kScratchBytes; }

}  // extern "C"
