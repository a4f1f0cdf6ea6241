// Band handle and solver internals shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "cpm_internal.h"
#include "kernels.h"

namespace cpm {

constexpr int kMaxLevels = 12;
constexpr int kMaxCoarse = 12000;  // largest coarsest level for the dense direct solve

// A registered device allocator (cpm_set_allocator); null functions: hipMalloc / hipFree.
struct DeviceAllocator {
  void* (*alloc)(void* ctx, size_t bytes) = nullptr;
  void (*free)(void* ctx, void* p) = nullptr;
  void* ctx = nullptr;
};

template <typename T>
struct LevelBufs {
  T* u = nullptr;  // iterate (correction on coarse levels)
  T* f = nullptr;  // right-hand side
  T* g = nullptr;  // f + N u
  T* r = nullptr;  // residual
  T* t = nullptr;  // second iterate of the fused sweep (it reads u while writing)
  T* p = nullptr;  // level 0, FP64: previous iterate (increment of the standard relaxation)
};

}  // namespace cpm

struct cpm_band_s {
  cpm_surface surf{};
  cpm::DeviceAllocator allocator;  // the one registered when the band was built
  cpm_grid grid{};
  int dim = 0;
  int L = 0;
  std::vector<cpm::HostLevel> host;
  std::vector<cpm::DevLevel> dev;
  // `stream`: where the current call enqueues its work (the caller's stream between enter()
  // and leave(), the private stream otherwise); `own`: the private stream, which also
  // captures the cycle graphs (the legacy default stream cannot be captured)
  hipStream_t stream = nullptr;
  hipStream_t own = nullptr;
  // coarsest level: [A_c | Z] after Gauss-Jordan, Z = A_c^{-1} E_c at column offset n; with
  // coarse_cols > 0 the left half of each row also holds Z's B_interp columns (list order)
  double coarse_c = 0.0 / 0.0;
  double* coarseM = nullptr;
  int coarse_cols = 0;
  // standard relaxation: [A_c | A_c^{-1}] for coarse_std_c, per-level omega / diag(A) for (std_c, std_omega)
  double* coarseS = nullptr;
  double coarse_std_c = 0.0 / 0.0;
  double std_c = 0.0 / 0.0, std_omega = 0.0 / 0.0;
  bool std_rb = false;  // the red-black half-sweep factors are current too
  int std_el = 3;       // degree of the E in front of L the factors are for
  // Remark 3.2's operator: [A_c | A_c^{-1}] for coarse_std1_c
  double* coarseS1 = nullptr;
  double coarse_std1_c = 0.0 / 0.0;
  // variable diffusion coefficient: set on every level (vc_active), diagonals valid for vc_c
  bool vc_active = false;
  double vc_c = 0.0 / 0.0;
  double* gj_col = nullptr;
  int* gj_info = nullptr;
  // device scalars: [0] residual norm bits, [1] ||E f|| bits; relres history + counter
  unsigned long long* dscal = nullptr;
  int* dcounter = nullptr;
  double* dhist = nullptr;
  unsigned long long* hpinned = nullptr;
  cpm::LaunchCfg lc[3];
  // learned smoother
  uint16_t* mlpW = nullptr;
  double rho_plain = 1.0;
  bool learned_active = false;
  uint16_t* featX = nullptr;  // scratch for the learned sweep (n0 x 64 bf16)
  float* featS = nullptr;
  double* feat_r64 = nullptr;
  float* feat_r32 = nullptr;
  int64_t feat_cap = 0;
  std::map<std::string, hipGraphExec_t> graphs;
};

namespace cpm {
// Restores a band's private stream when an entry point returns, on every path (enter() makes
// the caller's stream current; a later call that takes no stream must not find it there).
struct StreamScope {
  cpm_band b;
  explicit StreamScope(cpm_band band) : b(band) {}
  ~StreamScope() {
    if (b) b->stream = b->own;
  }
  StreamScope(const StreamScope&) = delete;
  StreamScope& operator=(const StreamScope&) = delete;
};
}  // namespace cpm

namespace cpm {

LaunchCfg band_cfg(const cpm_band b, int64_t n);
// device memory of a band through its allocator
void* dev_alloc(const cpm_band b, size_t bytes);
void dev_free(const cpm_band b, void* p);
LaunchCfg level_cfg(const DevLevel& D);
LaunchCfg ext_cfg(const DevLevel& D);
LaunchCfg sweep_cfg(const DevLevel& D);
ExtAddr ext_addr(const DevLevel& D);
NsumAddr nsum_addr(const DevLevel& D);
SweepAddr sweep_addr(const DevLevel& D);
TileAddr tile_addr(const DevLevel& D);
// Whole-cycle choice of every level's sweep form (second stage of cpm_autotune).
cpm_status tune_sweep_forms(cpm_band b);
double level_delta(const cpm_band b, int l, double c);
cpm_status enter(cpm_band b, void* user);
cpm_status leave(cpm_band b, void* user);
cpm_status check_launch(const char* what);
cpm_status ensure_coarse(cpm_band b, double c);
// the coarsest solve on Z's B_interp columns (csrc/coarse.hip)
void launch_compact_cols(int n, int m, int64_t ld, double* M, const int32_t* col, hipStream_t s);
template <typename T>
void launch_coarse_gemv_cols(int n, int m, const double* Z, int64_t ld, const int32_t* col, const T* x, T* y,
                             hipStream_t s);
size_t layout_bytes(const cpm_band b, int precision);
size_t workspace_bytes(const cpm_band b, const cpm_params& p);
template <typename T>
void carve_levels(const cpm_band b, void* work, LevelBufs<T>* B, double** g64);
template <typename T>
void vcycle_level(const cpm_band b, int l, LevelBufs<T>* B, const T* rhsA, const cpm_params& p, hipStream_t s,
                  bool u_zero, const T* r_first = nullptr);
void enqueue_cycle(const cpm_band b, const cpm_params& p, const double* f, double* u, void* work, hipStream_t s,
                   bool r_ready = false);
void enqueue_prologue(const cpm_band b, const cpm_params& p, const double* f, const double* u, void* work,
                      hipStream_t s);
cpm_status read_scalars(cpm_band b, double* r0, double* r1);
cpm_status validate_params(const cpm_band b, const cpm_params* p);

// fused learned update u += (s / delta) y on level l from the residual r (weights set, patch
// tables present); launch_learned_r takes the residual in another precision (float32 under a
// float64 iterate, as the learned sweep stores it)
template <typename T>
void launch_learned(const cpm_band b, int l, const T* r, T* u, double c, hipStream_t s);
template <typename T, typename R>
void launch_learned_r(const cpm_band b, int l, const R* r, T* u, double c, hipStream_t s);
// learned smoother sweep on level l (< 2): given g = f + N u already computed into g,
// evaluate the residual, the features, the network and update u.
template <typename T>
void learned_sweep(const cpm_band b, int l, T* u, const T* f, const T* rhsA, T* g, T* r, double c, hipStream_t s);

}  // namespace cpm
