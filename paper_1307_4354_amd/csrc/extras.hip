// Tile-size autotuner of the single-problem kernels.
#include <hip/hip_runtime.h>

#include "capi_internal.h"

using namespace cpm;

extern "C" {

cpm_status cpm_autotune(cpm_band band, void* stream) {
  (void)band;
  (void)stream;
  set_error("not available");
  return CPM_E_INVALID;
}

}  // extern "C"
