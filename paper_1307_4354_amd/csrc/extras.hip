// Autotuner of the single-problem kernels: for every level it times the candidate launch
// configurations of the two passes of a smoothing sweep on the band's own addressing and
// keeps the fastest (the extension: gathers through the vector caches with workgroups of
// 128 / 256 / 512 lanes, or LDS-staged; the neighbour sum: 128 / 256 / 512 lanes), then
// times the fused one-pass sweep (128 / 256 / 512 lanes) against that pair and keeps the
// faster form for the level.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "capi_internal.h"

using namespace cpm;

namespace {

// Average launch time of fn over reps back-to-back calls, the minimum of three trials after
// a warm-up: small levels run a few microseconds per launch, where one short trial is
// easily off by more than the difference between two candidates.
template <typename Fn>
float time_us(hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps, Fn fn) {
  for (int r = 0; r < 3; ++r) fn();  // warm-up
  float best = 1e30f;
  for (int trial = 0; trial < 3; ++trial) {
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r) fn();
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    best = std::min(best, 1000.f * ms / reps);
  }
  return best;
}

}  // namespace

extern "C" {

cpm_status cpm_autotune(cpm_band band, void* stream) {
  if (!band) {
    set_error("cpm_autotune: null band");
    return CPM_E_INVALID;
  }
  cpm_status st = enter(band, stream);
  if (st != CPM_OK) return st;
  hipStream_t s = band->stream;
  const int64_t n0 = band->dev[0].n;
  double *g = nullptr, *u = nullptr;
  if (hipMalloc((void**)&g, n0 * sizeof(double)) != hipSuccess || hipMalloc((void**)&u, n0 * sizeof(double)) != hipSuccess) {
    if (g) (void)hipFree(g);
    set_error("cpm_autotune: allocation failed");
    return CPM_E_NOMEM;
  }
  launch_fill<double>(n0, g, 1.0, s);
  launch_fill<double>(n0, u, 0.5, s);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int blocks[3] = {128, 256, 512};
  for (int l = 0; l < band->L; ++l) {
    DevLevel& D = band->dev[(size_t)l];
    const int reps = D.n > (1 << 20) ? 10 : 50;
    const double delta = level_delta(band, l, 1.0);
    const double inv_h2 = 1.0 / (D.h * D.h);
    float best = 1e30f;
    bool best_lds = D.use_lds;
    int best_blk = D.ext_block;
    for (int cand = 0; cand < 4; ++cand) {
      const bool lds = cand == 3;
      if (lds && !D.lds) continue;
      D.use_lds = lds;
      D.ext_block = lds ? 256 : blocks[cand];
      const ExtAddr a = ext_addr(D);
      const LaunchCfg lc = ext_cfg(D);
      const float t = time_us(s, e0, e1, reps, [&] {
        launch_ext<double, double>(band->dim, EXT_SMOOTH, D.n, g, a, D.band_order ? D.fracE : D.fracK, nullptr, u,
                                   (double*)nullptr, delta, 0.5 / delta, nullptr, lc, s);
      });
      if (t < best) {
        best = t;
        best_lds = lds;
        best_blk = D.ext_block;
      }
    }
    D.use_lds = best_lds;
    D.ext_block = best_blk;
    best = 1e30f;
    int best_n = D.nsum_block;
    for (int bi = 0; bi < 3; ++bi) {
      LaunchCfg lc;
      lc.block = blocks[bi];
      const float t = time_us(s, e0, e1, reps, [&] {
        launch_nsum<double>(band->dim, D.m, D.ilist, D.nbrI, u, u, inv_h2, g, nullptr, lc, s);
      });
      if (t < best) {
        best = t;
        best_n = blocks[bi];
      }
    }
    D.nsum_block = best_n;
    if (!D.fusedOK) continue;
    // split sweep (both passes, tuned) against the fused pass
    const float t_split = time_us(s, e0, e1, reps, [&] {
      launch_nsum<double>(band->dim, D.m, D.ilist, D.nbrI, u, u, inv_h2, g, nullptr, level_cfg(D), s);
      launch_ext<double, double>(band->dim, EXT_SMOOTH, D.n, g, ext_addr(D), D.band_order ? D.fracE : D.fracK,
                                 nullptr, u, (double*)nullptr, delta, 0.5 / delta, nullptr, ext_cfg(D), s);
    });
    const SweepAddr sa{D.perm, D.packed, D.origin, D.originX};
    float t_fused = 1e30f;
    int best_s = D.sweep_block;
    for (int bi = 0; bi < 3; ++bi) {
      LaunchCfg lc;
      lc.block = blocks[bi];
      // u -> g and g -> u alternately, like the solver's ping-pong
      int flip = 0;
      const float t = time_us(s, e0, e1, reps, [&] {
        const double* src = flip ? g : u;
        double* dst = flip ? u : g;
        flip ^= 1;
        launch_sweep<double>(band->dim, EXT_SMOOTH, D.n, src, dst, src, nullptr, sa, D.fracK, inv_h2, delta,
                             0.5 / delta, lc, s);
      });
      if (t < t_fused) {
        t_fused = t;
        best_s = blocks[bi];
      }
    }
    D.sweep_block = best_s;
    if (!D.sweep_forced) D.fused = t_fused < t_split;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  (void)hipFree(g);
  (void)hipFree(u);
  // captured graphs hold the old launch configurations
  for (auto& kv : band->graphs) (void)hipGraphExecDestroy(kv.second);
  band->graphs.clear();
  if ((st = check_launch("cpm_autotune")) != CPM_OK) return st;
  return leave(band, stream);
}

cpm_status cpm_band_tuning(cpm_band band, int level, int* use_lds, int* ext_block, int* nsum_block, int* fused,
                           int* sweep_block) {
  if (!band || level < 0 || level >= band->L) {
    set_error("cpm_band_tuning: invalid argument");
    return CPM_E_INVALID;
  }
  const DevLevel& D = band->dev[(size_t)level];
  if (use_lds) *use_lds = D.lds && D.use_lds ? 1 : 0;
  if (ext_block) *ext_block = D.use_lds ? kExtBlock : D.ext_block;
  if (nsum_block) *nsum_block = D.nsum_block;
  if (fused) *fused = D.fused && D.fusedOK ? 1 : 0;
  if (sweep_block) *sweep_block = D.sweep_block;
  return CPM_OK;
}

}  // extern "C"
