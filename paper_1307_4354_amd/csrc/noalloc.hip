// Operator application without any device allocation: the variant of cpm_apply for callers
// that cannot allocate (code under HIP graph capture, tight serving loops).  Its work vector
// (the neighbour sum f + N u of every stencil node) lives in a file-scope device array that
// each GPU holds for the life of the process.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "capi_internal.h"

namespace cpm {
namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB: 4 Mi doubles / 8 Mi floats

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch`, looked up once per device with the device
// current (the array's name is a host-side stand-in, not a device address).
cpm_status scratch_ptr(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_error("cpm_apply_static: no current device");
    return CPM_E_HIP;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("cpm_apply_static: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
      return CPM_E_HIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CPM_OK;
}

}  // namespace
}  // namespace cpm

using namespace cpm;

extern "C" {

cpm_status cpm_apply_static(cpm_band band, int level, int dtype, double c, const void* u, void* Au, void* stream) {
  if (!band || level < 0 || level >= band->L || !u || !Au || !(c > 0.0) ||
      (dtype != CPM_DTYPE_F64 && dtype != CPM_DTYPE_F32)) {
    set_error("cpm_apply_static: invalid argument");
    return CPM_E_INVALID;
  }
  const size_t elem = dtype == CPM_DTYPE_F64 ? sizeof(double) : sizeof(float);
  const size_t need = (size_t)band->dev[(size_t)level].n * elem;
  if (need > kScratchBytes) {
    set_error("cpm_apply_static: level " + std::to_string(level) + " needs " + std::to_string(need) +
              " bytes of work space; the static scratch holds " + std::to_string(kScratchBytes) +
              " (use cpm_apply with a workspace)");
    return CPM_E_WORKSPACE;
  }
  void* work = nullptr;
  const cpm_status st = scratch_ptr(&work);
  if (st != CPM_OK) return st;
  return cpm_apply(band, level, dtype, c, u, Au, work, stream);
}

}  // extern "C"
