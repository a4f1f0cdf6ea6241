// Batched solves, autotuner and learned smoother entry points.
#include <hip/hip_runtime.h>

#include <cstring>

#include "capi_internal.h"

namespace cpm {

template <typename T>
void learned_sweep(const cpm_band b, int l, T* u, const T* f, const T* rhsA, T* g, double c, hipStream_t s) {
  (void)b; (void)l; (void)u; (void)f; (void)rhsA; (void)g; (void)c; (void)s;
}
template void learned_sweep<double>(const cpm_band, int, double*, const double*, const double*, double*, double,
                                    hipStream_t);
template void learned_sweep<float>(const cpm_band, int, float*, const float*, const float*, float*, double,
                                   hipStream_t);

}  // namespace cpm

using namespace cpm;

extern "C" {

cpm_status cpm_workspace_size_batched(int nprob, const cpm_band* bands, const cpm_params* params, size_t* bytes) {
  (void)nprob; (void)bands; (void)params; (void)bytes;
  set_error("not available");
  return CPM_E_INVALID;
}

cpm_status cpm_solve_batched(int nprob, const cpm_band* bands, const cpm_params* params, const double* const* f,
                             double* const* u, void* work, size_t work_bytes, double rtol, int max_cycles,
                             cpm_stats* stats, void* stream) {
  (void)nprob; (void)bands; (void)params; (void)f; (void)u; (void)work; (void)work_bytes; (void)rtol;
  (void)max_cycles; (void)stats; (void)stream;
  set_error("not available");
  return CPM_E_INVALID;
}

cpm_status cpm_autotune(cpm_band band, void* stream) {
  (void)band; (void)stream;
  set_error("not available");
  return CPM_E_INVALID;
}

cpm_status cpm_set_smoother_weights(cpm_band band, const uint16_t* w_bf16, double rho_plain) {
  (void)band; (void)w_bf16; (void)rho_plain;
  set_error("not available");
  return CPM_E_INVALID;
}

cpm_status cpm_mlp_forward(int64_t m, const uint16_t* X, const uint16_t* W, float* Y, float* H, void* stream) {
  (void)m; (void)X; (void)W; (void)Y; (void)H; (void)stream;
  set_error("not available");
  return CPM_E_INVALID;
}

cpm_status cpm_mlp_backward(int64_t m, const uint16_t* X, const uint16_t* W, const float* H, const float* Y,
                            const float* T, float* G, void* stream) {
  (void)m; (void)X; (void)W; (void)H; (void)Y; (void)T; (void)G; (void)stream;
  set_error("not available");
  return CPM_E_INVALID;
}

cpm_status cpm_smoother_features(cpm_band band, int level, double c, const double* f, const double* u, uint16_t* X,
                                 float* s, void* work, void* stream) {
  (void)band; (void)level; (void)c; (void)f; (void)u; (void)X; (void)s; (void)work; (void)stream;
  set_error("not available");
  return CPM_E_INVALID;
}

}  // extern "C"
