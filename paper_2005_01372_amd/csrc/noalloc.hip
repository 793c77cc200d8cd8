// lsop_apply_noalloc: the LS operator application of lsop_apply with its FFT
// intermediate in a fixed device array of the library instead of the
// operator's own buffer, for callers that cannot allocate device memory.
#include <mutex>

#include "internal.hpp"

namespace lsop {
namespace {

// The FFT intermediate of lsop_apply_noalloc: [chunk][nx][2 lz] vectors of the operator's widest dtype, as many
// whole vectors as fit.  Each GPU the library runs on holds its own copy until the process ends.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` per device, looked up once per device with that device current (the array's
// name in host code is a host-side stand-in, not a device address).
constexpr int kMaxDevices = 64;
void* g_scratch_dev[kMaxDevices] = {};
std::once_flag g_scratch_once[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices] = {};

int scratch_address(void** out) {
  int dev = -1;
  LSOP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(LSOP_EUNSUPPORTED, "device index beyond the static scratch table");
  std::call_once(g_scratch_once[dev], [dev] {
    void* p = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_dev[dev] = p;
  });
  if (g_scratch_err[dev] != hipSuccess || !g_scratch_dev[dev])
    return fail(LSOP_EHIP, std::string("hipGetSymbolAddress of the static scratch array failed: ") +
                               hipGetErrorString(g_scratch_err[dev]));
  *out = g_scratch_dev[dev];
  return LSOP_OK;
}

}  // namespace
}  // namespace lsop

using namespace lsop;

extern "C" {

int lsop_apply_noalloc(lsop_op* op, int mode, const void* x_dev, void* y_dev, int nvec, void* stream) {
  if (!op) return fail(LSOP_EINVAL, "null operator handle");
  const size_t per = apply_tmp_bytes_per_vec(op);
  if (per > kScratchBytes)
    return fail(LSOP_EINVAL, "lsop_apply_noalloc: one vector's FFT intermediate (" + std::to_string(per) +
                                 " bytes) exceeds the static scratch of " + std::to_string(kScratchBytes) + " bytes");
  void* tmp = nullptr;
  int st = scratch_address(&tmp);
  if (st) return st;
  return apply_into(op, mode, x_dev, y_dev, nvec, tmp, (int)(kScratchBytes / per),
                    reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
