// Autotuner of the single-problem kernels: for every level it times the candidate launch
// configurations of the two passes of a smoothing sweep on the band's own addressing and
// keeps the fastest (the extension: gathers through the vector caches with workgroups of
// 128 / 256 / 512 lanes, or LDS-staged; the neighbour sum: 128 / 256 / 512 lanes), then
// times the fused one-pass sweep (gathers with 128 / 256 / 512 lanes, or LDS-staged) against
// that pair.  Back-to-back launches of one kernel run on warm caches, which flatters the
// two-pass form on mid-sized levels, so a second stage settles each level's form (two
// passes, fused with gathers, fused from LDS) by timing whole V-cycles.
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
  StreamScope stream_scope(band);
  cpm_status st = enter(band, stream);
  if (st != CPM_OK) return st;
  hipStream_t s = band->stream;
  const int64_t n0 = band->dev[0].n;
  double* g = (double*)dev_alloc(band, n0 * sizeof(double));
  double* u = (double*)dev_alloc(band, n0 * sizeof(double));
  if (!g || !u) {
    dev_free(band, g);
    dev_free(band, u);
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
    bool best_pf = D.ext_prefetch;
    for (int cand = 0; cand < 5; ++cand) {
      const bool lds = cand >= 3;  // 3: LDS-staged, 4: LDS-staged with the node's data loaded first
      if (lds && !D.lds) continue;
      if (cand == 4 && D.prefetch_forced) continue;
      D.use_lds = lds;
      D.ext_block = lds ? 256 : blocks[cand];
      if (!D.prefetch_forced) D.ext_prefetch = cand == 4;
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
        best_pf = D.ext_prefetch;
      }
    }
    D.use_lds = best_lds;
    D.ext_block = best_blk;
    D.ext_prefetch = best_pf;
    best = 1e30f;
    int best_n = D.nsum_block;
    for (int bi = 0; bi < 3; ++bi) {
      LaunchCfg lc;
      lc.block = blocks[bi];
      const float t = time_us(s, e0, e1, reps, [&] {
        launch_nsum<double>(band->dim, nsum_addr(D), u, u, inv_h2, g, nullptr, lc, s);
      });
      if (t < best) {
        best = t;
        best_n = blocks[bi];
      }
    }
    D.nsum_block = best_n;
    if (!D.fusedOK && D.ntiles <= 0) continue;
    // split sweep (both passes, tuned) against the fused pass and the tiled pass
    const float t_split = time_us(s, e0, e1, reps, [&] {
      launch_nsum<double>(band->dim, nsum_addr(D), u, u, inv_h2, g, nullptr, level_cfg(D), s);
      launch_ext<double, double>(band->dim, EXT_SMOOTH, D.n, g, ext_addr(D), D.band_order ? D.fracE : D.fracK,
                                 nullptr, u, (double*)nullptr, delta, 0.5 / delta, nullptr, ext_cfg(D), s);
    });
    float t_fused = 1e30f, t_gather = 1e30f;
    int best_g = D.sweep_block;
    bool best_slds = D.use_sweep_lds;
    for (int cand = 0; cand < 4 && D.fusedOK; ++cand) {
      const bool slds = cand == 3;  // LDS-staged (fixed workgroup), else gathers
      if (slds && !D.sweep_lds) continue;
      D.use_sweep_lds = slds;
      const SweepAddr sa = sweep_addr(D);
      LaunchCfg lc;
      lc.block = slds ? kExtBlock : blocks[cand];
      // u -> g and g -> u alternately, like the solver's ping-pong
      int flip = 0;
      const float t = time_us(s, e0, e1, reps, [&] {
        const double* src = flip ? g : u;
        double* dst = flip ? u : g;
        flip ^= 1;
        launch_sweep<double>(band->dim, EXT_SMOOTH, D.n, src, dst, src, nullptr, sa, D.fracK, inv_h2, delta,
                             0.5 / delta, lc, s);
      });
      if (!slds && t < t_gather) {
        t_gather = t;
        best_g = lc.block;
      }
      if (t < t_fused) {
        t_fused = t;
        best_slds = slds;
      }
    }
    D.sweep_block = best_g;  // the gather form's workgroup (the LDS form's is fixed)
    D.use_sweep_lds = best_slds;
    if (!D.sweep_forced) D.fused = D.fusedOK && t_fused < t_split;
    if (D.ntiles > 0) {
      int flip = 0;
      const TileAddr ta = tile_addr(D);
      const float t_tile = time_us(s, e0, e1, reps, [&] {
        const double* src = flip ? g : u;
        double* dst = flip ? u : g;
        flip ^= 1;
        launch_tile<double, double>(EXT_SMOOTH, D.n, ta, D.fracT, src, src, nullptr, dst, inv_h2, delta, 0.5 / delta,
                                    nullptr, s);
      });
      if (!D.sweep_forced) {
        D.use_tile = t_tile < std::min(t_split, D.fused ? t_fused : 1e30f);
        if (D.use_tile) D.fused = false;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  dev_free(band, g);
  dev_free(band, u);
  // captured graphs hold the old launch configurations
  for (auto& kv : band->graphs) (void)hipGraphExecDestroy(kv.second);
  band->graphs.clear();
  if ((st = check_launch("cpm_autotune")) != CPM_OK) return st;
  // second stage: each level's sweep form decided on whole cycles
  if ((st = tune_sweep_forms(band)) != CPM_OK) return st;
  return leave(band, stream);
}

cpm_status cpm_band_tuning(cpm_band band, int level, int* use_lds, int* ext_block, int* nsum_block, int* fused,
                           int* sweep_block, int* sweep_lds, int* tiled, int* ext_prefetch, int* ext_slots) {
  if (!band || level < 0 || level >= band->L) {
    set_error("cpm_band_tuning: invalid argument");
    return CPM_E_INVALID;
  }
  const DevLevel& D = band->dev[(size_t)level];
  if (use_lds) *use_lds = D.lds && D.use_lds ? 1 : 0;
  if (ext_block) *ext_block = D.use_lds ? kExtBlock : D.ext_block;
  if (nsum_block) *nsum_block = D.nsum_block;
  if (fused) *fused = D.fused && D.fusedOK ? 1 : 0;
  const bool slds = D.sweep_lds && D.use_sweep_lds;
  if (sweep_block) *sweep_block = slds ? kExtBlock : D.sweep_block;
  if (sweep_lds) *sweep_lds = slds ? 1 : 0;
  if (tiled) *tiled = D.use_tile && D.ntiles > 0 ? 1 : 0;
  if (ext_prefetch) *ext_prefetch = D.lds && D.use_lds && D.ext_prefetch ? 1 : 0;
  if (ext_slots) *ext_slots = D.lds ? kExtBlock * D.ext_npt : 0;
  return CPM_OK;
}

cpm_status cpm_set_band_tuning(cpm_band band, int level, int use_lds, int ext_block, int nsum_block, int fused,
                               int sweep_block, int sweep_lds, int tiled, int ext_prefetch) {
  if (!band || level < 0 || level >= band->L) {
    set_error("cpm_set_band_tuning: invalid argument");
    return CPM_E_INVALID;
  }
  DevLevel& D = band->dev[(size_t)level];
  auto blk_ok = [](int b) { return b == 128 || b == 256 || b == 512; };
  if ((use_lds && !D.lds) || (ext_prefetch && !use_lds) || (fused && !D.fusedOK) || (sweep_lds && !D.sweep_lds) ||
      (tiled && D.ntiles <= 0) ||
      (tiled && fused) || !blk_ok(ext_block) || !blk_ok(nsum_block) || !blk_ok(sweep_block)) {
    set_error("cpm_set_band_tuning: configuration not supported on this level");
    return CPM_E_INVALID;
  }
  D.use_lds = use_lds != 0;
  D.ext_block = ext_block;
  D.nsum_block = nsum_block;
  D.fused = fused != 0;
  D.sweep_block = sweep_block;
  D.use_sweep_lds = sweep_lds != 0;
  D.use_tile = tiled != 0;
  D.ext_prefetch = ext_prefetch != 0;
  // captured graphs hold the old launch configurations
  for (auto& kv : band->graphs) (void)hipGraphExecDestroy(kv.second);
  band->graphs.clear();
  return CPM_OK;
}

}  // extern "C"
