// Batched mixed-precision solves of many independent CPM problems.
//
// The levels of all problems are aligned by their distance from each problem's coarsest
// level, so one V-cycle of the batch is a fixed sequence of phases (pre-smoothing,
// residual, restriction on the way down; coarsest solve; prolongation and post-smoothing
// on the way up; the float64 outer residual and refinement update at the end).  Every
// phase is ONE launch over the tiles of all problems taking part in it: each workgroup
// walks the tile list with a grid stride and finds the owning problem by binary search in
// the phase's tile prefix table, so problems of very different sizes share the machine
// without per-problem launches.  Problems that reached the tolerance are skipped through a
// device-side flag, so each problem performs exactly the cycles its own solve would.  One
// batched cycle is one captured HIP graph.  The per-node work is the same device code as
// the single-problem kernels, so every problem's iterates equal its unbatched solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "capi_internal.h"
#include "kernels_dev.h"

namespace cpm {
namespace {

struct LvItem {  // one (problem, level) of a smoothing / residual phase, float32 vectors
  int64_t n, m;
  const int32_t* perm;
  const int32_t* packed;
  const int32_t* origin;
  const int32_t* ilist;
  const int32_t* nbrI;
  const float* frac;
  float* u;
  float* f;
  float* g;
  float* r;
  const float* rhsA;  // A-space right-hand side on the problem's finest level, else null
  float delta, inv_h2, wod;
  int prob;
  // LDS staging of the extension (packedL null: gathers), neighbour-sum segments (segOff null:
  // per-node lists)
  const int32_t* packedL;
  const int32_t* blkE;
  const int32_t* gidx;
  const int32_t* blkG;
  const int32_t* lorg;
  int32_t lo_off;
  const int32_t* seg;
  const int32_t* chunkSeg;
  const uint8_t* segOff;
  // the residual before restriction over the restriction's fine nodes (rs_packedL null: the
  // whole level)
  int64_t rs_n;
  const int32_t* rs_perm;
  const int32_t* rs_packedL;
  const int32_t* rs_blkE;
  const int32_t* rs_gidx;
  const int32_t* rs_blkG;
  const int32_t* rs_lorg;
  const float* rs_frac;
  int32_t rs_lo_off;
};

struct TrItem {  // restriction into / prolongation into a level with n nodes
  int64_t n;
  const int32_t* runs;
  const float* frac;
  const float* src;
  float* dst;
  float* zero;  // restriction: coarse iterate to clear
  int prob;
};

struct CoItem {  // coarsest level: u = Z f
  int64_t n, ld;
  const double* Z;
  const float* f;
  float* u;
  int prob;
};

struct TopItem {  // finest level, float64 outer quantities
  int64_t n, m;
  const int32_t* perm;
  const int32_t* packed;
  const int32_t* origin;
  const int32_t* ilist;
  const int32_t* nbrI;
  const double* frac;
  const double* f;
  double* u;
  double* g;
  float* b32;
  float* e32;
  double delta, inv_h2;
  int prob;
  const int32_t* packedL;  // as in LvItem
  const int32_t* blkE;
  const int32_t* gidx;
  const int32_t* blkG;
  const int32_t* lorg;
  int32_t lo_off;
  const int32_t* seg;
  const int32_t* chunkSeg;
  const uint8_t* segOff;
};

__device__ __forceinline__ int find_item(const int64_t* __restrict__ pre, int ni, int64_t t) {
  int lo = 0, hi = ni - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <int D>
__global__ __launch_bounds__(kMaxBlock) void kb_nsum(const LvItem* __restrict__ it, const int64_t* __restrict__ pre,
                                                     int ni, const int* __restrict__ done) {
  const int64_t total = pre[ni];
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int q = find_item(pre, ni, t);
    const LvItem& B = it[q];
    if (done[B.prob]) continue;
    const int64_t k = (t - pre[q]) * blockDim.x + threadIdx.x;
    if (k >= B.m) continue;
    if (B.segOff)
      nsum_seg_node<D, float>(k, B.seg, B.chunkSeg, B.segOff, B.u, B.rhsA ? nullptr : B.f, B.inv_h2, B.g);
    else
      nsum_node<D, float>(k, B.m, B.ilist, B.nbrI, B.u, B.rhsA ? nullptr : B.f, B.inv_h2, B.g);
  }
}

// One tile of an extension pass over an item: LDS-staged (the tile is the item's staging
// workgroup; needs 256 lanes) when the item has the tables, else through gathers.  The
// staging synchronizes the workgroup, and the workgroup's next tile reuses the LDS, hence
// the closing barrier; both branches are uniform over the workgroup.
template <int D, typename T, typename TO, int MODE, typename Item>
__device__ __forceinline__ unsigned long long kb_ext_tile(const Item& B, int64_t lb, const T* g, const T* frac,
                                                          const T* b, T* u, TO* out, T delta, T wod, char* smem) {
  constexpr int S = D == 2 ? 4 : 16;
  unsigned long long nv = 0ull;
  if (B.packedL && blockDim.x == kExtBlock) {
    T* gl = (T*)smem;
    int32_t* lo = (int32_t*)(smem + B.lo_off);
    ext_stage<T>(lb, g, B.blkE, B.gidx, B.blkG, B.lorg, S, gl, lo);
    const int64_t k = lb * kExtBlock + threadIdx.x;
    if (k < B.n) nv = ext_node_lds<D, T, TO, MODE>(k, B.n, gl, lo, B.perm, B.packedL, frac, b, u, out, delta, wod);
    __syncthreads();
  } else {
    const int64_t k = lb * blockDim.x + threadIdx.x;
    if (k < B.n) nv = ext_node<D, T, TO, MODE>(k, B.n, g, B.perm, B.packed, B.origin, frac, b, u, out, delta, wod);
  }
  return nv;
}

template <int D, int MODE>
__global__ __launch_bounds__(kMaxBlock) void kb_ext(const LvItem* __restrict__ it, const int64_t* __restrict__ pre,
                                                    int ni, const int* __restrict__ done) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int64_t total = pre[ni];
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int q = find_item(pre, ni, t);
    const LvItem& B = it[q];
    if (done[B.prob]) continue;
    (void)kb_ext_tile<D, float, float, MODE>(B, t - pre[q], B.g, B.frac, B.rhsA, B.u, B.r, B.delta, B.wod, smem);
  }
}

// Residual before restriction: over the restriction's fine nodes (LDS-staged, 256 lanes)
// where the item has that subset's tables, else over the whole level as kb_ext does.
template <int D>
__global__ __launch_bounds__(kMaxBlock) void kb_resid(const LvItem* __restrict__ it, const int64_t* __restrict__ pre,
                                                      int ni, const int* __restrict__ done) {
  constexpr int S = D == 2 ? 4 : 16;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int64_t total = pre[ni];
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int q = find_item(pre, ni, t);
    const LvItem& B = it[q];
    if (done[B.prob]) continue;
    const int64_t lb = t - pre[q];
    if (B.rs_packedL && blockDim.x == kExtBlock) {
      float* gl = (float*)smem;
      int32_t* lo = (int32_t*)(smem + B.rs_lo_off);
      ext_stage<float>(lb, B.g, B.rs_blkE, B.rs_gidx, B.rs_blkG, B.rs_lorg, S, gl, lo);
      const int64_t k = lb * kExtBlock + threadIdx.x;
      if (k < B.rs_n)
        (void)ext_node_lds<D, float, float, EXT_RESID>(k, B.rs_n, gl, lo, B.rs_perm, B.rs_packedL, B.rs_frac, B.rhsA,
                                                       B.u, B.r, B.delta, B.wod);
      __syncthreads();
    } else {
      (void)kb_ext_tile<D, float, float, EXT_RESID>(B, lb, B.g, B.frac, B.rhsA, B.u, B.r, B.delta, B.wod, smem);
    }
  }
}

// First pre-smoothing sweep of a level from u = 0 (every level starts a cycle there): on a
// problem's finest level, with its A-space right-hand side b, the sweep is u = wod b; on a
// coarser level g = f + N 0 = f, so the sweep extends f itself and skips the neighbour sum.
// Bit for bit the two-pass sweep from zero.
template <int D>
__global__ __launch_bounds__(kMaxBlock) void kb_first(const LvItem* __restrict__ it, const int64_t* __restrict__ pre,
                                                      int ni, const int* __restrict__ done) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int64_t total = pre[ni];
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int q = find_item(pre, ni, t);
    const LvItem& B = it[q];
    if (done[B.prob]) continue;
    if (B.rhsA) {
      const int64_t k = (t - pre[q]) * blockDim.x + threadIdx.x;
      if (k < B.n) B.u[k] = B.wod * B.rhsA[k];
    } else {
      (void)kb_ext_tile<D, float, float, EXT_SMOOTH>(B, t - pre[q], B.f, B.frac, (const float*)nullptr, B.u, B.r,
                                                    B.delta, B.wod, smem);
    }
  }
}

template <int D, int RESTRICT>
__global__ __launch_bounds__(kMaxBlock) void kb_transfer(const TrItem* __restrict__ it,
                                                         const int64_t* __restrict__ pre, int ni,
                                                         const int* __restrict__ done) {
  const int64_t total = pre[ni];
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int q = find_item(pre, ni, t);
    const TrItem& T = it[q];
    if (done[T.prob]) continue;
    const int64_t j = (t - pre[q]) * blockDim.x + threadIdx.x;
    if (j < T.n) {
      const float v = linear_node<D, float>(j, T.n, T.src, T.runs, T.frac);
      if (RESTRICT) {
        T.dst[j] = v;
        T.zero[j] = 0.0f;
      } else {
        T.dst[j] += v;
      }
    }
  }
}

// coarsest: one workgroup (256 lanes) per row, the same reduction order as k_gemv
__global__ __launch_bounds__(256) void kb_coarse(const CoItem* __restrict__ it, const int64_t* __restrict__ pre,
                                                 int ni, const int* __restrict__ done) {
  const int64_t total = pre[ni];
  __shared__ double part[4];
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int q = find_item(pre, ni, t);
    const CoItem& C = it[q];
    if (done[C.prob]) continue;
    const int64_t row = t - pre[q];
    const double* zr = C.Z + row * C.ld;
    double s = 0.0;
    int64_t j = threadIdx.x;
    for (; j + 7 * 256 < C.n; j += 8 * 256) {
      double z[8], xv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        z[q] = zr[j + q * 256];
        xv[q] = (double)C.f[j + q * 256];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) s += z[q] * xv[q];
    }
    for (; j < C.n; j += 256) s += zr[j] * (double)C.f[j];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) C.u[row] = (float)(((part[0] + part[1]) + part[2]) + part[3]);
    __syncthreads();
  }
}

// finest level, float64: 0 = g = f + N u (over B_interp); 1 = residual r = E g - delta u
// -> b32 and the per-problem norm; 2 = e = 0; 3 = u += e; 4 = ||E f|| -> bnorm
template <int D, int OP>
__global__ __launch_bounds__(kMaxBlock) void kb_top(const TopItem* __restrict__ it, const int64_t* __restrict__ pre,
                                                    int ni, const int* __restrict__ done,
                                                    unsigned long long* __restrict__ slots) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int64_t total = pre[ni];
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int q = find_item(pre, ni, t);
    const TopItem& B = it[q];
    if (done[B.prob]) continue;
    const int64_t k = (t - pre[q]) * blockDim.x + threadIdx.x;
    if (OP == 0) {
      if (k < B.m) {
        if (B.segOff)
          nsum_seg_node<D, double>(k, B.seg, B.chunkSeg, B.segOff, B.u, B.f, B.inv_h2, B.g);
        else
          nsum_node<D, double>(k, B.m, B.ilist, B.nbrI, B.u, B.f, B.inv_h2, B.g);
      }
    } else if (OP == 1 || OP == 4) {
      unsigned long long nv;
      if (OP == 1)
        nv = kb_ext_tile<D, double, float, EXT_RESID>(B, t - pre[q], B.g, B.frac, (const double*)nullptr, B.u, B.b32,
                                                      B.delta, 0.0, smem);
      else
        nv = kb_ext_tile<D, double, double, EXT_PLAIN>(B, t - pre[q], B.f, B.frac, (const double*)nullptr,
                                                       (double*)nullptr, (double*)nullptr, 0.0, 0.0, smem);
      block_max_atomic(nv, slots + 2 * B.prob + (OP == 4 ? 1 : 0));
    } else if (OP == 2) {
      if (k < B.n) B.e32[k] = 0.0f;
    } else {
      if (k < B.n) B.u[k] += (double)B.e32[k];
    }
  }
}

// per problem: relres = nrm / bnorm, history, stopping decision, clear nrm for the next cycle.
// done[p]: 1 converged (or E f = 0), 2 diverged, 3 stopped at max_cycles.
__global__ void kb_finalize(int nprob, unsigned long long* __restrict__ slots, int* __restrict__ done,
                            int* __restrict__ cycles, double* __restrict__ hist, int hcap, int count, double rtol,
                            int max_cycles, int* __restrict__ ndone) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprob || done[p]) return;
  const double num = __longlong_as_double((long long)slots[2 * p]);
  const double den = __longlong_as_double((long long)slots[2 * p + 1]);
  const double rel = den > 0.0 ? num / den : 0.0;
  int c = cycles[p];
  if (count) {
    c += 1;
    cycles[p] = c;
    if (c - 1 < hcap) hist[(int64_t)p * hcap + c - 1] = rel;
  }
  slots[2 * p] = 0ull;
  const bool bad = !(rel == rel) || rel > 1e300;
  if (rel < rtol || bad || c >= max_cycles) {
    done[p] = bad ? 2 : (rel < rtol ? 1 : 3);
    atomicAdd(ndone, 1);
  }
}

// E f = 0: the problem's solution is u = 0 (its prologue marked it done with relres 0)
template <int D>
__global__ __launch_bounds__(kMaxBlock) void kb_zero_trivial(const TopItem* __restrict__ it,
                                                             const int64_t* __restrict__ pre, int ni,
                                                             const unsigned long long* __restrict__ slots) {
  const int64_t total = pre[ni];
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int q = find_item(pre, ni, t);
    const TopItem& B = it[q];
    if (slots[2 * B.prob + 1] != 0ull) continue;
    const int64_t k = (t - pre[q]) * blockDim.x + threadIdx.x;
    if (k < B.n) B.u[k] = 0.0;
  }
}

inline int64_t tiles(int64_t n, int per) { return (n + per - 1) / per; }

// batched cycles captured in one graph (one host synchronization per graph launch)
constexpr int kBatchCycles = 8;

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// Host-side plan: items and tile prefixes of every phase for one block size.
struct Plan {
  int A = 0;  // number of absolute levels (max over problems)
  std::vector<LvItem> lv[kMaxLevels];
  std::vector<TrItem> rs[kMaxLevels];  // restriction into absolute level a (from a + 1)
  std::vector<TrItem> pr[kMaxLevels];  // prolongation into absolute level a (from a - 1)
  std::vector<CoItem> co;
  std::vector<TopItem> top;
};

struct DevPhase {
  const void* items = nullptr;
  const int64_t* pre = nullptr;
  int ni = 0;
  int64_t total = 0;
};

struct Layout {
  size_t vec_bytes = 0;    // per-problem vectors
  size_t table_bytes = 0;  // item tables + prefixes
  size_t scal_bytes = 0;   // slots, flags, cycles, history
  size_t total = 0;
};

// vector bytes of one problem (float32 u, f, g, r per level + float64 g on the finest)
size_t problem_vec_bytes(const cpm_band b) {
  size_t s = 0;
  for (int l = 0; l < b->L; ++l) s += 4 * al((size_t)b->dev[(size_t)l].n * 4);
  return s + al((size_t)b->dev[0].n * 8);
}

Layout layout(int nprob, const cpm_band* bands) {
  Layout L;
  for (int p = 0; p < nprob; ++p) L.vec_bytes += problem_vec_bytes(bands[p]);
  // worst case: every problem in every phase, three block sizes of prefixes
  const size_t items = (size_t)nprob * (3 * kMaxLevels + 2);
  const size_t isz = std::max(std::max(sizeof(LvItem), sizeof(TrItem)), std::max(sizeof(CoItem), sizeof(TopItem)));
  const size_t arrays = 3 * kMaxLevels + 2;    // item arrays, each padded to 256 bytes
  const size_t prefixes = 5 * kMaxLevels + 3;  // prefix arrays per block-size candidate
  L.table_bytes = al(items * isz) + arrays * 256 + 3 * prefixes * (al((size_t)(nprob + 1) * sizeof(int64_t)) + 256);
  L.scal_bytes = al((size_t)nprob * 2 * 8) + al((size_t)nprob * 4) * 2 + al((size_t)nprob * CPM_MAX_HISTORY * 8) + 256;
  L.total = L.vec_bytes + L.table_bytes + L.scal_bytes + 1024;
  return L;
}

// Workgroup-size choices of earlier batched solves, keyed by the device, the batch's bands
// (handle and per-level sizes) and the smoothing counts: a repeated solve of the same batch
// reuses the timed choice instead of timing the candidates again.  A stale entry (a band freed
// and another built at the same address with the same sizes) only costs speed.
constexpr size_t kTuneCacheMax = 64;
std::mutex g_tune_mu;
std::map<std::vector<int64_t>, std::pair<int, int>> g_tune_cache;

std::vector<int64_t> tune_key(int nprob, const cpm_band* bands, const cpm_params& P, int device) {
  std::vector<int64_t> k{device, nprob, P.nu1, P.nu2};
  for (int p = 0; p < nprob; ++p) {
    k.push_back((int64_t)(uintptr_t)bands[p]);
    k.push_back(bands[p]->L);
    for (int l = 0; l < bands[p]->L; ++l) k.push_back(bands[p]->dev[(size_t)l].n);
  }
  return k;
}

// LDS bytes one staging workgroup of a level takes for values of vsize bytes (the layout of
// launch_ext), 0 when the level has no staging tables for workgroups of kExtBlock slots
size_t stage_bytes(const DevLevel& D, int dim, size_t vsize) {
  if (!D.lds || D.ext_npt != 1) return 0;
  const size_t lo = ((size_t)D.maxE * vsize + 15) & ~(size_t)15;
  return lo + (size_t)D.maxG * (dim == 2 ? 4 : 16) * sizeof(int32_t);
}

// LDS bytes of the residual subset's staging workgroup (float values), 0 without its tables
size_t rs_stage_bytes(const DevLevel& D, int dim) {
  if (D.rs_n <= 0 || !D.lds || D.rs_npt != 1 || !D.rs_frac32) return 0;
  const size_t lo = ((size_t)D.rs_maxE * sizeof(float) + 15) & ~(size_t)15;
  return lo + (size_t)D.rs_maxG * (dim == 2 ? 4 : 16) * sizeof(int32_t);
}

void set_rs_tables(LvItem& it, const DevLevel& D, int dim) {
  it.rs_packedL = nullptr;
  it.rs_n = 0;
  const size_t bytes = rs_stage_bytes(D, dim);
  if (bytes == 0 || bytes > (size_t)kMaxDynLds) return;
  it.rs_n = D.rs_n;
  it.rs_perm = D.rs_perm;
  it.rs_packedL = D.rs_packedL;
  it.rs_blkE = D.rs_blkE;
  it.rs_gidx = D.rs_gidx;
  it.rs_blkG = D.rs_blkG;
  it.rs_lorg = D.rs_lorg;
  it.rs_frac = D.rs_frac32;
  it.rs_lo_off = (int32_t)(((size_t)D.rs_maxE * sizeof(float) + 15) & ~(size_t)15);
}

template <typename Item>
void set_tables(Item& it, const DevLevel& D, size_t vsize, int dim) {
  it.packedL = nullptr;
  const size_t bytes = stage_bytes(D, dim, vsize);
  if (bytes > 0 && bytes <= (size_t)kMaxDynLds) {
    it.packedL = D.packedL;
    it.blkE = D.blkE;
    it.gidx = D.gidx;
    it.blkG = D.blkG;
    it.lorg = D.lorg;
    it.lo_off = (int32_t)(((size_t)D.maxE * vsize + 15) & ~(size_t)15);
  }
  it.seg = D.nsSeg;
  it.chunkSeg = D.nsChunkSeg;
  it.segOff = D.nsSegOff;
}

}  // namespace
}  // namespace cpm

using namespace cpm;

extern "C" {

cpm_status cpm_workspace_size_batched(int nprob, const cpm_band* bands, const cpm_params* params, size_t* bytes) {
  if (nprob < 1 || !bands || !params || !bytes) {
    set_error("cpm_workspace_size_batched: invalid argument");
    return CPM_E_INVALID;
  }
  for (int p = 0; p < nprob; ++p)
    if (!bands[p]) {
      set_error("null band in batch");
      return CPM_E_INVALID;
    }
  *bytes = layout(nprob, bands).total;
  return CPM_OK;
}

cpm_status cpm_solve_batched(int nprob, const cpm_band* bands, const cpm_params* params, const double* const* f,
                             double* const* u, void* work, size_t work_bytes, double rtol, int max_cycles,
                             cpm_stats* stats, void* stream) {
  if (nprob < 1 || !bands || !params || !f || !u || !work || max_cycles < 0) {
    set_error("cpm_solve_batched: invalid argument");
    return CPM_E_INVALID;
  }
  const int dim = bands[0]->dim;
  for (int p = 0; p < nprob; ++p) {
    if (!bands[p] || !f[p] || !u[p]) {
      set_error("cpm_solve_batched: null band or vector");
      return CPM_E_INVALID;
    }
    if (bands[p]->dim != dim) {
      set_error("cpm_solve_batched: all problems must have the same dimension");
      return CPM_E_INVALID;
    }
    if (bands[p]->L < 2) {
      set_error("cpm_solve_batched: every problem needs at least two levels");
      return CPM_E_INVALID;
    }
    cpm_status st = validate_params(bands[p], params);
    if (st != CPM_OK) return st;
  }
  if (params->gamma > 1 || params->fmg) {
    set_error("cpm_solve_batched runs V-cycles from the given iterates (gamma <= 1, no fmg)");
    return CPM_E_INVALID;
  }
  if (params->precision != CPM_MIXED || params->smoother != CPM_SMOOTH_JACOBI) {
    set_error("cpm_solve_batched runs mixed precision with the Jacobi smoother");
    return CPM_E_INVALID;
  }
  const Layout LY = layout(nprob, bands);
  if (work_bytes < LY.total) {
    set_error("workspace too small");
    return CPM_E_WORKSPACE;
  }
  auto t_start = std::chrono::steady_clock::now();
  const cpm_params P = *params;
  cpm_band b0 = bands[0];
  StreamScope stream_scope(b0);
  cpm_status st = enter(b0, stream);
  if (st != CPM_OK) return st;
  hipStream_t s = b0->stream;
  // coarsest-level inverses (each band's on its own stream, synchronously)
  for (int p = 0; p < nprob; ++p) {
    if ((st = ensure_coarse(bands[p], P.c)) != CPM_OK) return st;
  }
  // ---- carve the workspace
  char* base = (char*)(((uintptr_t)work + 255) & ~(uintptr_t)255);
  char* vec = base;
  char* tab = base + LY.vec_bytes;
  char* sca = tab + LY.table_bytes;
  unsigned long long* slots = (unsigned long long*)sca;
  int* done = (int*)(sca + al((size_t)nprob * 16));
  int* cyc = (int*)((char*)done + al((size_t)nprob * 4));
  double* hist = (double*)((char*)cyc + al((size_t)nprob * 4));
  int* ndone = (int*)((char*)hist + al((size_t)nprob * CPM_MAX_HISTORY * 8));
  // ---- build the plan
  Plan plan;
  size_t shm_lv = 0, shm_top = 0, shm_rs = 0;  // dynamic LDS of the staged extension launches
  struct PV {
    float *u, *f, *g, *r;
  };
  std::vector<std::vector<PV>> pv((size_t)nprob);
  std::vector<double*> g64((size_t)nprob);
  char* vp = vec;
  for (int p = 0; p < nprob; ++p) {
    cpm_band b = bands[p];
    pv[(size_t)p].resize((size_t)b->L);
    for (int l = 0; l < b->L; ++l) {
      const size_t n = (size_t)b->dev[(size_t)l].n;
      PV& v = pv[(size_t)p][(size_t)l];
      v.u = (float*)vp;
      vp += al(n * 4);
      v.f = (float*)vp;
      vp += al(n * 4);
      v.g = (float*)vp;
      vp += al(n * 4);
      v.r = (float*)vp;
      vp += al(n * 4);
    }
    g64[(size_t)p] = (double*)vp;
    vp += al((size_t)b->dev[0].n * 8);
    plan.A = std::max(plan.A, b->L);
  }
  for (int p = 0; p < nprob; ++p) {
    cpm_band b = bands[p];
    const int L = b->L;
    for (int l = 0; l < L; ++l) {
      const int a = L - 1 - l;  // distance from the coarsest level
      const DevLevel& D = b->dev[(size_t)l];
      PV& v = pv[(size_t)p][(size_t)l];
      const double delta = level_delta(b, l, P.c);
      if (l < L - 1) {
        LvItem it{};
        it.n = D.n;
        it.m = D.m;
        it.perm = D.perm;
        it.packed = D.packed;
        it.origin = D.origin;
        it.ilist = D.ilist;
        it.nbrI = D.nbrI;
        it.frac = D.fracK32;
        it.u = v.u;
        it.f = v.f;
        it.g = v.g;
        it.r = v.r;
        it.rhsA = l == 0 ? v.f : nullptr;  // finest: f holds the float32 outer residual
        it.delta = (float)delta;
        it.inv_h2 = (float)(1.0 / (D.h * D.h));
        it.wod = (float)(P.omega / delta);
        it.prob = p;
        set_tables(it, D, sizeof(float), b->dim);
        if (it.packedL) shm_lv = std::max(shm_lv, stage_bytes(D, b->dim, sizeof(float)));
        set_rs_tables(it, D, b->dim);
        if (it.rs_packedL) shm_rs = std::max(shm_rs, rs_stage_bytes(D, b->dim));
        plan.lv[a].push_back(it);
        // restriction from this level into the next coarser one (absolute a - 1)
        const DevLevel& C = b->dev[(size_t)(l + 1)];
        PV& vc = pv[(size_t)p][(size_t)(l + 1)];
        TrItem r{};
        r.n = C.n;
        r.runs = C.runR;
        r.frac = C.fracR32;
        r.src = v.r;
        r.dst = vc.f;
        r.zero = vc.u;
        r.prob = p;
        plan.rs[a - 1].push_back(r);
        TrItem q{};
        q.n = D.n;
        q.runs = D.runP;
        q.frac = D.fracP32;
        q.src = vc.u;
        q.dst = v.u;
        q.zero = nullptr;
        q.prob = p;
        plan.pr[a].push_back(q);
      } else {
        CoItem c{};
        c.n = D.n;
        c.ld = 2 * D.n;
        c.Z = b->coarseM + D.n;
        c.f = v.f;
        c.u = v.u;
        c.prob = p;
        plan.co.push_back(c);
      }
    }
    const DevLevel& D0 = b->dev[0];
    TopItem t{};
    t.n = D0.n;
    t.m = D0.m;
    t.perm = D0.perm;
    t.packed = D0.packed;
    t.origin = D0.origin;
    t.ilist = D0.ilist;
    t.nbrI = D0.nbrI;
    t.frac = D0.fracK;
    t.f = f[p];
    t.u = u[p];
    t.g = g64[(size_t)p];
    t.b32 = pv[(size_t)p][0].f;
    t.e32 = pv[(size_t)p][0].u;
    t.delta = level_delta(b, 0, P.c);
    t.inv_h2 = 1.0 / (D0.h * D0.h);
    t.prob = p;
    set_tables(t, D0, sizeof(double), b->dim);
    if (t.packedL) shm_top = std::max(shm_top, stage_bytes(D0, b->dim, sizeof(double)));
    plan.top.push_back(t);
  }
  // ---- upload item tables; prefixes per block size candidate
  const int cand_block[3] = {128, 256, 512};
  std::vector<char> htab(LY.table_bytes, 0);
  size_t off = 0;
  bool overflow = false;
  auto put_items = [&](const void* src, size_t bytes) -> const void* {
    const size_t o = off;
    if (o + al(bytes) > htab.size()) {
      overflow = true;
      return nullptr;
    }
    std::memcpy(&htab[o], src, bytes);
    off += al(bytes);
    return (const void*)(tab + o);
  };
  struct PhaseSet {
    DevPhase nsum[kMaxLevels], ext[kMaxLevels], rsx[kMaxLevels], rs[kMaxLevels], pr[kMaxLevels], co, top_n, top_m;
  };
  std::vector<PhaseSet> sets(3);
  const void* lv_items[kMaxLevels];
  const void* rs_items[kMaxLevels];
  const void* pr_items[kMaxLevels];
  for (int a = 0; a < plan.A; ++a) {
    lv_items[a] = plan.lv[a].empty() ? nullptr : put_items(plan.lv[a].data(), plan.lv[a].size() * sizeof(LvItem));
    rs_items[a] = plan.rs[a].empty() ? nullptr : put_items(plan.rs[a].data(), plan.rs[a].size() * sizeof(TrItem));
    pr_items[a] = plan.pr[a].empty() ? nullptr : put_items(plan.pr[a].data(), plan.pr[a].size() * sizeof(TrItem));
  }
  const void* co_items = put_items(plan.co.data(), plan.co.size() * sizeof(CoItem));
  const void* top_items = put_items(plan.top.data(), plan.top.size() * sizeof(TopItem));
  auto put_prefix = [&](const std::vector<int64_t>& counts, DevPhase& ph, const void* items) {
    std::vector<int64_t> pre(counts.size() + 1, 0);
    for (size_t i = 0; i < counts.size(); ++i) pre[i + 1] = pre[i] + counts[i];
    const size_t o = off;
    if (o + al(pre.size() * sizeof(int64_t)) > htab.size()) {
      overflow = true;
      return;
    }
    std::memcpy(&htab[o], pre.data(), pre.size() * sizeof(int64_t));
    off += al(pre.size() * sizeof(int64_t));
    ph.items = items;
    ph.pre = (const int64_t*)(tab + o);
    ph.ni = (int)counts.size();
    ph.total = pre.back();
  };
  for (int ci = 0; ci < 3; ++ci) {
    const int bs = cand_block[ci];
    PhaseSet& S = sets[(size_t)ci];
    for (int a = 0; a < plan.A; ++a) {
      std::vector<int64_t> cn, cm, cx, cr, cp;
      for (auto& it : plan.lv[a]) {
        cn.push_back(tiles(it.n, bs));
        cm.push_back(tiles(it.m, bs));
        cx.push_back(it.rs_packedL && bs == kExtBlock ? tiles(it.rs_n, bs) : tiles(it.n, bs));
      }
      for (auto& it : plan.rs[a]) cr.push_back(tiles(it.n, bs));
      for (auto& it : plan.pr[a]) cp.push_back(tiles(it.n, bs));
      if (!cn.empty()) {
        put_prefix(cn, S.ext[a], lv_items[a]);
        put_prefix(cm, S.nsum[a], lv_items[a]);
        put_prefix(cx, S.rsx[a], lv_items[a]);
      }
      if (!cr.empty()) put_prefix(cr, S.rs[a], rs_items[a]);
      if (!cp.empty()) put_prefix(cp, S.pr[a], pr_items[a]);
    }
    std::vector<int64_t> cc, tn, tm;
    for (auto& it : plan.co) cc.push_back(it.n);  // one row per tile
    for (auto& it : plan.top) {
      tn.push_back(tiles(it.n, bs));
      tm.push_back(tiles(it.m, bs));
    }
    put_prefix(cc, S.co, co_items);
    put_prefix(tn, S.top_n, top_items);
    put_prefix(tm, S.top_m, top_items);
  }
  if (overflow || off > LY.table_bytes) {
    set_error("internal: batch table overflow");
    return CPM_E_INVALID;
  }
  if (hipMemcpyAsync(tab, htab.data(), off, hipMemcpyHostToDevice, s) != hipSuccess) {
    set_error("batch table upload failed");
    return CPM_E_HIP;
  }
  // clear vectors and scalars
  launch_fill<float>((int64_t)(LY.vec_bytes / 4), (float*)vec, 0.0f, s);
  launch_fill<int>((int64_t)(LY.scal_bytes / 4), (int*)sca, 0, s);

  int num_cu = 256;
  {
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
      hipDeviceProp_t prop;
      if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
        num_cu = prop.multiProcessorCount;
    }
  }
  auto grid = [&](int64_t total, int gm) -> unsigned {
    int64_t g = std::min<int64_t>(total, (int64_t)num_cu * gm);
    return (unsigned)std::max<int64_t>(g, 1);
  };
  int sel = 1, gmult = 8;
  auto enqueue_sweep = [&](const PhaseSet& S, int bs, int gm, int a, hipStream_t st2) {
    const DevPhase& pn = S.nsum[a];
    const DevPhase& pe = S.ext[a];
    if (!pn.ni) return;
    if (dim == 2) {
      kb_nsum<2><<<grid(pn.total, gm), bs, 0, st2>>>((const LvItem*)pn.items, pn.pre, pn.ni, done);
      kb_ext<2, EXT_SMOOTH><<<grid(pe.total, gm), bs, shm_lv, st2>>>((const LvItem*)pe.items, pe.pre, pe.ni, done);
    } else {
      kb_nsum<3><<<grid(pn.total, gm), bs, 0, st2>>>((const LvItem*)pn.items, pn.pre, pn.ni, done);
      kb_ext<3, EXT_SMOOTH><<<grid(pe.total, gm), bs, shm_lv, st2>>>((const LvItem*)pe.items, pe.pre, pe.ni, done);
    }
  };
  auto enqueue_first = [&](const PhaseSet& S, int bs, int gm, int a, hipStream_t st2) {
    const DevPhase& pe = S.ext[a];
    if (!pe.ni) return;
    if (dim == 2)
      kb_first<2><<<grid(pe.total, gm), bs, shm_lv, st2>>>((const LvItem*)pe.items, pe.pre, pe.ni, done);
    else
      kb_first<3><<<grid(pe.total, gm), bs, shm_lv, st2>>>((const LvItem*)pe.items, pe.pre, pe.ni, done);
  };
  // ---- tile-size autotuning: time one smoothing sweep of the largest phase per candidate;
  // CPM_BATCH_BLOCK = 128 | 256 | 512 fixes the workgroup size instead
  int forced = -1;
  if (const char* e = std::getenv("CPM_BATCH_BLOCK")) {
    const int v = std::atoi(e);
    for (int ci = 0; ci < 3; ++ci)
      if (cand_block[ci] == v) forced = ci;
  }
  int dev_id = 0;
  (void)hipGetDevice(&dev_id);
  const std::vector<int64_t> tkey = tune_key(nprob, bands, P, dev_id);
  bool cached = false;
  if (forced < 0) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto itc = g_tune_cache.find(tkey);
    if (itc != g_tune_cache.end()) {
      sel = itc->second.first;
      gmult = itc->second.second;
      cached = true;
    }
  }
  if (forced >= 0) {
    sel = forced;
  } else if (!cached) {
    int abig = 0;
    int64_t nbig = -1;
    for (int a = 1; a < plan.A; ++a) {
      int64_t nn = 0;
      for (auto& it : plan.lv[a]) nn += it.n;
      if (nn > nbig) {
        nbig = nn;
        abig = a;
      }
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best = 1e30f;
    const int gms[3] = {4, 8, 16};
    for (int ci = 0; ci < 3; ++ci)
      for (int gi = 0; gi < 3; ++gi) {
        enqueue_sweep(sets[(size_t)ci], cand_block[ci], gms[gi], abig, s);  // warm-up
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < 3; ++r) enqueue_sweep(sets[(size_t)ci], cand_block[ci], gms[gi], abig, s);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
          best = ms;
          sel = ci;
          gmult = gms[gi];
        }
      }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_tune_cache.size() >= kTuneCacheMax) g_tune_cache.clear();  // bounded: many distinct batches
    g_tune_cache[tkey] = {sel, gmult};
  }
  launch_fill<float>((int64_t)(LY.vec_bytes / 4), (float*)vec, 0.0f, s);
  const PhaseSet& S = sets[(size_t)sel];
  const int bs = cand_block[sel];
  const int gm = gmult;
  auto top = [&](int op, hipStream_t st2) {
    const DevPhase& ph = op == 0 ? S.top_m : S.top_n;
    const TopItem* it = (const TopItem*)ph.items;
    const unsigned gr = grid(ph.total, gm);
    if (dim == 2) {
      switch (op) {
        case 0: kb_top<2, 0><<<gr, bs, 0, st2>>>(it, ph.pre, ph.ni, done, slots); break;
        case 1: kb_top<2, 1><<<gr, bs, shm_top, st2>>>(it, ph.pre, ph.ni, done, slots); break;
        case 2: kb_top<2, 2><<<gr, bs, 0, st2>>>(it, ph.pre, ph.ni, done, slots); break;
        case 3: kb_top<2, 3><<<gr, bs, 0, st2>>>(it, ph.pre, ph.ni, done, slots); break;
        default: kb_top<2, 4><<<gr, bs, shm_top, st2>>>(it, ph.pre, ph.ni, done, slots); break;
      }
    } else {
      switch (op) {
        case 0: kb_top<3, 0><<<gr, bs, 0, st2>>>(it, ph.pre, ph.ni, done, slots); break;
        case 1: kb_top<3, 1><<<gr, bs, shm_top, st2>>>(it, ph.pre, ph.ni, done, slots); break;
        case 2: kb_top<3, 2><<<gr, bs, 0, st2>>>(it, ph.pre, ph.ni, done, slots); break;
        case 3: kb_top<3, 3><<<gr, bs, 0, st2>>>(it, ph.pre, ph.ni, done, slots); break;
        default: kb_top<3, 4><<<gr, bs, shm_top, st2>>>(it, ph.pre, ph.ni, done, slots); break;
      }
    }
  };
  auto finalize = [&](int count, hipStream_t st2) {
    kb_finalize<<<(nprob + 255) / 256, 256, 0, st2>>>(nprob, slots, done, cyc, hist, CPM_MAX_HISTORY, count, rtol,
                                                     max_cycles, ndone);
  };
  auto transfer = [&](const DevPhase& ph, int restrict_, hipStream_t st2) {
    if (!ph.ni) return;
    const TrItem* it = (const TrItem*)ph.items;
    const unsigned gr = grid(ph.total, gm);
    if (dim == 2) {
      if (restrict_)
        kb_transfer<2, 1><<<gr, bs, 0, st2>>>(it, ph.pre, ph.ni, done);
      else
        kb_transfer<2, 0><<<gr, bs, 0, st2>>>(it, ph.pre, ph.ni, done);
    } else {
      if (restrict_)
        kb_transfer<3, 1><<<gr, bs, 0, st2>>>(it, ph.pre, ph.ni, done);
      else
        kb_transfer<3, 0><<<gr, bs, 0, st2>>>(it, ph.pre, ph.ni, done);
    }
  };
  auto cycle = [&](hipStream_t st2) {
    top(2, st2);  // e = 0 on every finest level
    for (int a = plan.A - 1; a >= 1; --a) {
      // every level enters from u = 0 (finest: cleared above; coarser: by the restriction)
      for (int k = 0; k < P.nu1; ++k) {
        if (k == 0)
          enqueue_first(S, bs, gm, a, st2);
        else
          enqueue_sweep(S, bs, gm, a, st2);
      }
      const DevPhase& pn = S.nsum[a];
      const DevPhase& px = S.rsx[a];
      const size_t shm_x = std::max(shm_lv, shm_rs);
      if (pn.ni) {
        if (dim == 2) {
          kb_nsum<2><<<grid(pn.total, gm), bs, 0, st2>>>((const LvItem*)pn.items, pn.pre, pn.ni, done);
          kb_resid<2><<<grid(px.total, gm), bs, shm_x, st2>>>((const LvItem*)px.items, px.pre, px.ni, done);
        } else {
          kb_nsum<3><<<grid(pn.total, gm), bs, 0, st2>>>((const LvItem*)pn.items, pn.pre, pn.ni, done);
          kb_resid<3><<<grid(px.total, gm), bs, shm_x, st2>>>((const LvItem*)px.items, px.pre, px.ni, done);
        }
      }
      transfer(S.rs[a - 1], 1, st2);
    }
    kb_coarse<<<grid(S.co.total, gm), 256, 0, st2>>>((const CoItem*)S.co.items, S.co.pre, S.co.ni, done);
    for (int a = 1; a < plan.A; ++a) {
      transfer(S.pr[a], 0, st2);
      for (int k = 0; k < P.nu2; ++k) enqueue_sweep(S, bs, gm, a, st2);
    }
    top(3, st2);  // u += e
    top(0, st2);  // g = f + N u
    top(1, st2);  // r -> b32, norms
    finalize(1, st2);
  };
  // ---- prologue: ||E f|| and the first residual per problem; u = 0 where E f = 0
  top(4, s);
  top(0, s);
  top(1, s);
  finalize(0, s);
  {
    const TopItem* it = (const TopItem*)S.top_n.items;
    if (dim == 2)
      kb_zero_trivial<2><<<grid(S.top_n.total, gm), bs, 0, s>>>(it, S.top_n.pre, S.top_n.ni, slots);
    else
      kb_zero_trivial<3><<<grid(S.top_n.total, gm), bs, 0, s>>>(it, S.top_n.pre, S.top_n.ni, slots);
  }
  if ((st = check_launch("cpm_solve_batched prologue")) != CPM_OK) return st;
  // ---- capture kBatchCycles batched cycles in one graph: problems that converge (or reach
  // max_cycles) inside it are skipped by every later kernel through their done flag, so the
  // host reads the count of finished problems once per graph launch
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // captured on the private stream (the caller's may be the legacy default stream),
  // launched on the caller's
  if (hipStreamBeginCapture(b0->own, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    set_error("hipStreamBeginCapture failed");
    return CPM_E_HIP;
  }
  for (int j = 0; j < kBatchCycles; ++j) cycle(b0->own);
  if (hipStreamEndCapture(b0->own, &graph) != hipSuccess || !graph ||
      hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    set_error("batched graph capture failed");
    return CPM_E_HIP;
  }
  (void)hipGraphDestroy(graph);
  int* hnd = (int*)b0->hpinned;
  int launches = 0, syncs = 0;
  st = CPM_OK;
  while (true) {
    if (hipMemcpyAsync(hnd, ndone, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      st = CPM_E_HIP;
      set_error("batched solve: synchronization failed");
      break;
    }
    ++syncs;
    // every launch advances each unfinished problem by kBatchCycles cycles, and finalize stops
    // a problem at max_cycles, so the loop ends after at most ceil(max_cycles / kBatchCycles)
    if (*hnd >= nprob || (int64_t)launches * kBatchCycles >= max_cycles) break;
    if (hipGraphLaunch(exec, s) != hipSuccess) {
      st = CPM_E_HIP;
      set_error("batched solve: graph launch failed");
      break;
    }
    ++launches;
  }
  (void)hipGraphExecDestroy(exec);
  if (st != CPM_OK) return st;
  // ---- statistics
  std::vector<int> hdone((size_t)nprob), hcyc((size_t)nprob);
  std::vector<double> hh((size_t)nprob * CPM_MAX_HISTORY);
  if (hipMemcpy(hdone.data(), done, nprob * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(hcyc.data(), cyc, nprob * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(hh.data(), hist, hh.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
    set_error("batched solve: statistics copy failed");
    return CPM_E_HIP;
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  st = CPM_OK;
  for (int p = 0; p < nprob; ++p) {
    if (hdone[(size_t)p] != 1) st = (hdone[(size_t)p] == 2 || st == CPM_E_DIVERGED) ? CPM_E_DIVERGED : CPM_E_NOCONV;
    if (stats) {
      cpm_stats& S2 = stats[p];
      std::memset(&S2, 0, sizeof(cpm_stats));
      S2.cycles = hcyc[(size_t)p];
      const int nh = std::min(S2.cycles, CPM_MAX_HISTORY);
      for (int j = 0; j < nh; ++j) S2.relres_history[j] = hh[(size_t)p * CPM_MAX_HISTORY + j];
      S2.relres = nh > 0 ? S2.relres_history[nh - 1] : 0.0;
      S2.fallback_cycle = -1;
      S2.seconds = secs;
      S2.tile_block = bs;
      S2.tile_blocks_per_cu = gm;
      S2.host_syncs = syncs;
      S2.cycles_per_launch = kBatchCycles;
    }
  }
  if (st == CPM_E_NOCONV) set_error("some problems did not reach the tolerance");
  if (st == CPM_E_DIVERGED) set_error("some problems diverged");
  cpm_status ls = leave(b0, stream);
  return st != CPM_OK ? st : ls;
}

}  // extern "C"
