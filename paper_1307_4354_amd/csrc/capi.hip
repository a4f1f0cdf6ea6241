// C ABI of libcpm: band handles, matrix-free operator application, the CPM V-cycle
// (Algorithm 4.1) in double precision and as float32 inner cycles of a float64 iterative
// refinement, solve loops (eager or as captured HIP graphs).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <map>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "capi_internal.h"

namespace cpm {

thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace cpm

using namespace cpm;

// ------------------------------------------------------------------------------------
// helpers
// ------------------------------------------------------------------------------------

namespace cpm {

LaunchCfg band_cfg(const cpm_band b, int64_t n) {
  int cls = n < (1 << 16) ? 0 : (n < (1 << 20) ? 1 : 2);
  return b->lc[cls];
}

LaunchCfg level_cfg(const DevLevel& D) {
  LaunchCfg c;
  c.block = D.nsum_block;
  return c;
}

LaunchCfg ext_cfg(const DevLevel& D) {
  LaunchCfg c;
  c.block = D.ext_block;
  c.prefetch = D.ext_prefetch ? 1 : 0;
  return c;
}

LaunchCfg sweep_cfg(const DevLevel& D) {
  LaunchCfg c;
  c.block = D.sweep_block;
  return c;
}

// Device allocations of a band go through the allocator registered when it was built
// (cpm_set_allocator; hipMalloc / hipFree by default).
static cpm::DeviceAllocator g_allocator{};

void* dev_alloc(const cpm_band b, size_t bytes) {
  if (bytes == 0) return nullptr;
  if (b->allocator.alloc) return b->allocator.alloc(b->allocator.ctx, bytes);
  void* p = nullptr;
  return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}

void dev_free(const cpm_band b, void* p) {
  if (!p) return;
  if (b->allocator.free)
    b->allocator.free(b->allocator.ctx, p);
  else
    (void)hipFree(p);
}

template <typename T>
static T* dalloc(const cpm_band b, size_t count, cpm_status* st) {
  if (count == 0) return nullptr;
  void* p = dev_alloc(b, count * sizeof(T));
  if (!p) {
    *st = CPM_E_NOMEM;
    return nullptr;
  }
  return (T*)p;
}

template <typename T>
static cpm_status upload(const cpm_band b, T** dst, const std::vector<T>& src) {
  if (src.empty()) {
    *dst = nullptr;
    return CPM_OK;
  }
  cpm_status st = CPM_OK;
  *dst = dalloc<T>(b, src.size(), &st);
  if (st != CPM_OK) return st;
  if (hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return CPM_E_HIP;
  return CPM_OK;
}

static cpm_status upload_f32(const cpm_band b, float** dst, const std::vector<double>& src) {
  std::vector<float> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) tmp[i] = (float)src[i];
  return upload(b, dst, tmp);
}

static void free_dev(cpm_band b) {
  for (auto& D : b->dev) {
    void* ps[] = {D.runE,  D.nbr,   D.fracE,  D.fracE32, D.runP,    D.fracP,  D.fracP32, D.runR,
                  D.fracR, D.fracR32, D.perm, D.packed, D.origin, D.fracK, D.fracK32, D.ilist, D.nbrI, D.nsSeg, D.nsChunkSeg, D.nsSegOff, D.rs_perm, D.rs_packedL, D.rs_blkE, D.rs_gidx, D.rs_blkG, D.rs_lorg, D.rs_frac, D.rs_frac32,
                  D.patchRow, D.patchPk, D.patchMask, D.packedB, D.packedL, D.blkE, D.gidx, D.blkG, D.lorg, D.originX,
                  D.qdiag, D.wd, D.acoef, D.vcD, D.runP3, D.fracP3, D.blkE2, D.gidx2, D.lorg2,
                  D.tileSlot, D.tileRow, D.tperm, D.tloc, D.fracT, D.fracT32, D.parity, D.wdR, D.wdB, D.q1diag, D.wd1};
    for (void* p : ps) dev_free(b, p);
  }
  b->dev.clear();
  void* ps[] = {b->coarseM, b->coarseS, b->coarseS1, b->gj_col, b->gj_info, b->dscal, b->dcounter, b->dhist, b->mlpW};
  b->mlpW = nullptr;
  for (void* p : ps) dev_free(b, p);
  b->coarseM = nullptr;
  b->coarseS = nullptr;
  b->coarseS1 = nullptr;
  if (b->hpinned) (void)hipHostFree(b->hpinned);
  b->hpinned = nullptr;
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

double level_delta(const cpm_band b, int l, double c) {
  const double h = b->dev[(size_t)l].h;
  return c + 2.0 * b->dim / (h * h);
}

// A call enqueues its work on the caller's stream itself, so that it is ordered with the
// caller's work without events.  (Handing the results back through an event that the
// caller's stream waits on while the private stream still holds a long queue of cycle
// launches slowed those launches by a sixth on MI355X.)  Only graph capture uses the
// private stream.
cpm_status enter(cpm_band b, void* user) {
  b->stream = (hipStream_t)user;
  return CPM_OK;
}

cpm_status leave(cpm_band b, void* user) {
  (void)user;
  b->stream = b->own;
  return CPM_OK;
}

cpm_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return CPM_E_HIP;
  }
  return CPM_OK;
}

// Coarsest level: Z = A_c^{-1} E_c with A_c = delta I - E_c N_c, by Gauss-Jordan with
// partial pivoting on [A_c | E_c] on the device.  Cached per value of c.
// Dense inverse on the coarsest level: Gauss-Jordan on [A_c | E_c] (-> A_c^{-1} E_c, the
// Ruuth-Merriman cycles) or on [A_c | I] (-> A_c^{-1}, the standard relaxation).
static cpm_status ensure_vc_diag(cpm_band b, double c);

// kind: 0 [A_c | E_c] (Ruuth-Merriman cycles), 1 [A_c | I] (standard relaxation), 2 [A_c | I]
// for Remark 3.2's operator (linear interpolation in front of L)
static cpm_status coarse_inverse(cpm_band b, double c, int kind, double** M, double* cached_c) {
  const bool identity_rhs = kind != 0;
  if (*M && *cached_c == c) return CPM_OK;
  const int l = b->L - 1;
  const DevLevel& D = b->dev[(size_t)l];
  const int n = (int)D.n;
  if (n > kMaxCoarse) {
    std::ostringstream os;
    os << "coarsest level has " << n << " nodes; the dense direct solve allows at most " << kMaxCoarse
       << " (use more levels)";
    set_error(os.str());
    return CPM_E_INVALID;
  }
  cpm_status st = CPM_OK;
  if (!*M) *M = dalloc<double>(b, (size_t)2 * n * n, &st);
  if (!b->gj_col) b->gj_col = dalloc<double>(b, (size_t)n, &st);
  if (!b->gj_info) b->gj_info = dalloc<int>(b, 1, &st);
  if (st != CPM_OK) {
    set_error("device allocation of the coarse matrix failed");
    return st;
  }
  hipStream_t s = b->stream;
  const double h = D.h;
  if (kind == 2) {
    launch_assemble_coarse_p1(b->dim, n, D.runE, D.fracE, D.nbr, level_delta(b, l, c), 2.0 * b->dim / (h * h),
                              1.0 / (h * h), *M, s);
  } else if (b->vc_active && !identity_rhs) {
    // variable coefficient: [I - E D^{-1} N~ | E D^{-1}]
    if ((st = ensure_vc_diag(b, c)) != CPM_OK) return st;
    launch_assemble_coarse_vc(b->dim, n, D.runE, D.fracE, D.nbr, D.acoef, D.vcD, 1.0 / (h * h), *M, s);
  } else {
    launch_assemble_coarse(b->dim, n, D.runE, D.fracE, D.nbr, level_delta(b, l, c), 1.0 / (h * h), *M, s,
                           identity_rhs);
  }
  launch_fill<int>(1, b->gj_info, 0, s);
  for (int k = 0; k < n; ++k) launch_gj_step(n, k, *M, b->gj_col, b->gj_info, s);
  if ((st = check_launch("coarse factorization")) != CPM_OK) return st;
  int info = 0;
  if (hipMemcpyAsync(&info, b->gj_info, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    set_error("coarse factorization: synchronization failed");
    return CPM_E_HIP;
  }
  if (info != 0) {
    set_error("coarsest-level matrix is singular");
    *cached_c = NAN;
    return CPM_E_INVALID;
  }
  *cached_c = c;
  return CPM_OK;
}

cpm_status ensure_coarse(cpm_band b, double c) {
  if (b->coarseM && b->coarse_c == c) return CPM_OK;
  b->coarse_cols = 0;
  cpm_status st = coarse_inverse(b, c, 0, &b->coarseM, &b->coarse_c);
  if (st != CPM_OK) return st;
  // Z = A_c^{-1} E_c is zero outside the B_interp columns: keep those in the left half
  const DevLevel& D = b->dev[(size_t)(b->L - 1)];
  if (D.ilist && D.m > 0 && D.m < D.n) {
    launch_compact_cols((int)D.n, (int)D.m, 2 * D.n, b->coarseM, D.ilist, b->stream);
    if ((st = check_launch("coarse column compaction")) != CPM_OK) return st;
    b->coarse_cols = (int)D.m;
  }
  return CPM_OK;
}

// Variable coefficient: D = c + sigma on every level for this c.
static cpm_status ensure_vc_diag(cpm_band b, double c) {
  if (b->vc_c == c) return CPM_OK;
  cpm_status st = CPM_OK;
  for (int l = 0; l < b->L; ++l) {
    DevLevel& D = b->dev[(size_t)l];
    if (!D.vcD && !(D.vcD = dalloc<double>(b, (size_t)D.n, &st))) {
      set_error("device allocation of the variable-coefficient diagonal failed");
      return st != CPM_OK ? st : CPM_E_NOMEM;
    }
    launch_vc_diag(b->dim, D.n, D.nbr, D.acoef, c, 1.0 / (D.h * D.h), D.vcD, b->stream);
  }
  if ((st = check_launch("variable-coefficient diagonal")) != CPM_OK) return st;
  b->vc_c = c;
  return CPM_OK;
}

// Standard relaxation: A_c^{-1} and omega / diag(A) on every level for (c, omega); for the
// red-black sweeps also the two half-sweeps' factors (omega / diag(A) on one colour, 0 on the
// other; colours by the parity of the grid index sum).
static cpm_status ensure_std(cpm_band b, const cpm_params& p) {
  const double c = p.c, omega = p.omega;
  const bool rb = p.smoother == CPM_SMOOTH_STANDARD_RB;
  const int el = p.el_degree == 1 ? 1 : 3;
  cpm_status st = el == 1 ? coarse_inverse(b, c, 2, &b->coarseS1, &b->coarse_std1_c)
                          : coarse_inverse(b, c, 1, &b->coarseS, &b->coarse_std_c);
  if (st != CPM_OK) return st;
  if (b->std_c == c && b->std_omega == omega && b->std_el == el && (!rb || b->std_rb)) return CPM_OK;
  for (int l = 0; l < b->L; ++l) {
    DevLevel& D = b->dev[(size_t)l];
    if (!D.wd && !(D.wd = dalloc<double>(b, (size_t)D.n, &st))) {
      set_error("device allocation of the relaxation weights failed");
      return st != CPM_OK ? st : CPM_E_NOMEM;
    }
    launch_std_scale(D.n, el == 1 ? D.q1diag : D.qdiag, level_delta(b, l, c), omega, D.wd, b->stream);
    if (!rb) continue;
    if (!D.parity) {
      const HostLevel& H = b->host[(size_t)l];
      std::vector<uint8_t> par((size_t)D.n);
      for (int64_t i = 0; i < D.n; ++i) {
        int64_t sum = 0;
        for (int a = 0; a < b->dim; ++a) sum += H.idx[(size_t)(i * b->dim + a)];
        par[(size_t)i] = (uint8_t)(sum & 1);
      }
      if ((st = upload(b, &D.parity, par)) != CPM_OK) return st;
    }
    if ((!D.wdR && !(D.wdR = dalloc<double>(b, (size_t)D.n, &st))) ||
        (!D.wdB && !(D.wdB = dalloc<double>(b, (size_t)D.n, &st)))) {
      set_error("device allocation of the relaxation weights failed");
      return st != CPM_OK ? st : CPM_E_NOMEM;
    }
    launch_split_colours(D.n, D.wd, D.parity, D.wdR, D.wdB, b->stream);
  }
  if ((st = check_launch("relaxation weights")) != CPM_OK) return st;
  b->std_c = c;
  b->std_omega = omega;
  b->std_rb = rb;  // the half-sweep factors match (c, omega) only when just recomputed
  b->std_el = el;
  return CPM_OK;
}

// Verbatim residual (Algorithm 4.1 step 2 as printed): A_c^{-1} on the coarsest level and
// every level's full neighbour table.
static cpm_status ensure_verbatim(cpm_band b, double c) {
  cpm_status st = coarse_inverse(b, c, 1, &b->coarseS, &b->coarse_std_c);
  if (st != CPM_OK) return st;
  for (int l = 0; l + 1 < b->L; ++l) {
    DevLevel& D = b->dev[(size_t)l];
    if (!D.nbr && (st = upload(b, &D.nbr, b->host[(size_t)l].nbr)) != CPM_OK) {
      set_error("upload of the neighbour table failed");
      return st;
    }
  }
  return CPM_OK;
}

// ---- workspace layout ---------------------------------------------------------------

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

template <typename T>
static T* carve(char*& p, size_t count) {
  T* r = (T*)p;
  p += align_up(count * sizeof(T));
  return r;
}

size_t layout_bytes(const cpm_band b, int precision) {
  size_t tot = 0;
  for (int l = 0; l < b->L; ++l) {
    const size_t n = (size_t)b->dev[(size_t)l].n;
    if (precision == CPM_F64) {
      tot += align_up(n * 8) * (l == 0 ? 4 : 5);
    } else {
      tot += align_up(n * 4) * 5;
      if (l == 0) tot += align_up(n * 8);
    }
  }
  return tot + 256;
}

// The caller's workspace: the level vectors of its precision; a mixed-precision solve with
// the full-multigrid start first runs that start in the float64 layout of the same buffer.
size_t workspace_bytes(const cpm_band b, const cpm_params& p) {
  size_t s = layout_bytes(b, p.precision);
  if (p.fmg && p.precision != CPM_F64) s = std::max(s, layout_bytes(b, CPM_F64));
  return s;
}

template <typename T>
void carve_levels(const cpm_band b, void* work, LevelBufs<T>* B, double** g64) {
  char* p = (char*)(((uintptr_t)work + 255) & ~(uintptr_t)255);
  for (int l = 0; l < b->L; ++l) {
    const size_t n = (size_t)b->dev[(size_t)l].n;
    if (sizeof(T) == 8) {
      if (l == 0) {
        B[l].u = nullptr;
        B[l].f = nullptr;
      } else {
        B[l].u = carve<T>(p, n);
        B[l].f = carve<T>(p, n);
      }
      B[l].g = carve<T>(p, n);
      B[l].r = carve<T>(p, n);
      B[l].t = carve<T>(p, n);
      if (l == 0) B[l].p = carve<T>(p, n);
    } else {
      B[l].u = carve<T>(p, n);
      B[l].f = carve<T>(p, n);
      B[l].g = carve<T>(p, n);
      B[l].r = carve<T>(p, n);
      B[l].t = carve<T>(p, n);
      if (l == 0 && g64) *g64 = carve<double>(p, n);
    }
  }
}

// ---- one V-cycle (Algorithm 4.1) ------------------------------------------------------

template <typename T>
static const T* fracE_of(const DevLevel& D);
template <>
const double* fracE_of<double>(const DevLevel& D) { return D.fracE; }
template <>
const float* fracE_of<float>(const DevLevel& D) { return D.fracE32; }
// Extension over the restriction's fine nodes (HostLevel::rsN): LDS-staged only; valid when
// D.rs_n > 0 and the level runs the LDS-staged extension.
static ExtAddr ext_addr_rs(const DevLevel& D) {
  ExtAddr a{D.rs_perm, nullptr, nullptr};
  a.packedL = D.rs_packedL;
  a.blkE = D.rs_blkE;
  a.gidx = D.rs_gidx;
  a.blkG = D.rs_blkG;
  a.lorg = D.rs_lorg;
  a.maxE = D.rs_maxE;
  a.maxG = D.rs_maxG;
  a.npt = D.rs_npt;
  return a;
}
template <typename T>
static const T* rs_frac_of(const DevLevel& D);
template <>
const double* rs_frac_of<double>(const DevLevel& D) { return D.rs_frac; }
template <>
const float* rs_frac_of<float>(const DevLevel& D) { return D.rs_frac32; }
static bool resid_subset(const DevLevel& D) { return D.rs_n > 0 && D.lds && D.use_lds && !D.band_order; }

NsumAddr nsum_addr(const DevLevel& D) {
  NsumAddr a{D.m, D.ilist, D.nbrI};
  a.seg = D.nsSeg;
  a.chunkSeg = D.nsChunkSeg;
  a.segOff = D.nsSegOff;
  return a;
}
ExtAddr ext_addr(const DevLevel& D) {
  if (D.band_order) return ExtAddr{nullptr, D.packedB, D.origin};
  ExtAddr a{D.perm, D.packed, D.origin};
  if (D.lds && D.use_lds) {
    a.packedL = D.packedL;
    a.blkE = D.blkE;
    a.gidx = D.gidx;
    a.blkG = D.blkG;
    a.lorg = D.lorg;
    a.maxE = D.maxE;
    a.maxG = D.maxG;
    a.npt = D.ext_npt;
  }
  return a;
}
SweepAddr sweep_addr(const DevLevel& D) {
  SweepAddr a{D.perm, D.packed, D.origin, D.originX};
  if (D.sweep_lds && D.use_sweep_lds) {
    a.packedL = D.packedL;
    a.blkE = D.blkE2;
    a.gidx = D.gidx2;
    a.blkG = D.blkG;
    a.lorg = D.lorg2;
    a.maxE = D.maxE2;
    a.maxG = D.maxG;
  }
  return a;
}
TileAddr tile_addr(const DevLevel& D) { return TileAddr{D.tileSlot, D.tileRow, D.tperm, D.tloc, D.ntiles}; }
template <typename T>
static const T* fracT_of(const DevLevel& D);
template <>
const double* fracT_of<double>(const DevLevel& D) { return D.fracT; }
template <>
const float* fracT_of<float>(const DevLevel& D) { return D.fracT32; }
static bool tiled(const DevLevel& D) { return D.use_tile && D.ntiles > 0; }
// the standard relaxation (Sec. 4.5), with Jacobi or red-black Gauss-Seidel sweeps
static bool standard(const cpm_params& p) {
  return p.smoother == CPM_SMOOTH_STANDARD || p.smoother == CPM_SMOOTH_STANDARD_RB;
}

template <typename T>
static const T* fracK_of(const DevLevel& D);
template <>
const double* fracK_of<double>(const DevLevel& D) { return D.band_order ? D.fracE : D.fracK; }
template <>
const float* fracK_of<float>(const DevLevel& D) { return D.band_order ? D.fracE32 : D.fracK32; }
template <typename T>
static const T* fracP_of(const DevLevel& D);
template <>
const double* fracP_of<double>(const DevLevel& D) { return D.fracP; }
template <>
const float* fracP_of<float>(const DevLevel& D) { return D.fracP32; }
template <typename T>
static const T* fracR_of(const DevLevel& D);
template <>
const double* fracR_of<double>(const DevLevel& D) { return D.fracR; }
template <>
const float* fracR_of<float>(const DevLevel& D) { return D.fracR32; }

// stencil-order fractions (the fused sweep always visits nodes in stencil order)
template <typename T>
static const T* fracS_of(const DevLevel& D);
template <>
const double* fracS_of<double>(const DevLevel& D) { return D.fracK; }
template <>
const float* fracS_of<float>(const DevLevel& D) { return D.fracK32; }

// Damped Ruuth-Merriman Jacobi sweep: g = f + N u, u <- u + (w/delta)(b + E g - delta u).
// u_zero: u is known to be 0 (first sweep after restriction), so g = f and the neighbour
// sum is skipped.
template <typename T>
void smooth_sweep(const cpm_band b, int l, T* u, const T* f, const T* rhsA, T* g, T* r, double c, double omega,
                  unsigned long long* nrm, hipStream_t s, bool u_zero = false) {
  const DevLevel& D = b->dev[(size_t)l];
  const LaunchCfg lc = level_cfg(D);
  const double delta = level_delta(b, l, c);
  if constexpr (sizeof(T) == 8) {
    if (b->vc_active) {
      // variable coefficient: g = (f + N~ u) / D, u <- u + omega (E g - u)
      launch_nsum_var(b->dim, D.m, D.ilist, D.nbrI, u_zero ? nullptr : u, f, D.acoef, D.vcD, 1.0 / (D.h * D.h), g,
                      lc, s);
      launch_ext<T, T>(b->dim, EXT_SMOOTH, D.n, g, ext_addr(D), fracK_of<T>(D), rhsA, u, (T*)nullptr, (T)1.0,
                       (T)omega, nrm, ext_cfg(D), s);
      return;
    }
  }
  const T* gg = g;
  if (u_zero && f)
    gg = f;
  else
    launch_nsum<T>(b->dim, nsum_addr(D), u, f, (T)(1.0 / (D.h * D.h)), g, nullptr, lc, s);
  if (b->learned_active && l < 2 && b->mlpW && D.patchRow) {
    learned_sweep<T>(b, l, u, f, rhsA, const_cast<T*>(gg), r, c, s);
    return;
  }
  launch_ext<T, T>(b->dim, EXT_SMOOTH, D.n, gg, ext_addr(D), fracK_of<T>(D), rhsA, u, (T*)nullptr, (T)delta,
                   (T)(omega / delta), nrm, ext_cfg(D), s);
}

// The level's smoothing and residual as fused passes (E f once per visit, then one pass per
// sweep, alternating between u and t).  Returns the vector holding the iterate.
template <typename T>
static T* fused_pre(const cpm_band b, int l, LevelBufs<T>* B, const T* f, const T* rhsA, const cpm_params& p,
                    int nu, bool u_zero, hipStream_t s) {
  const DevLevel& D = b->dev[(size_t)l];
  const double delta = level_delta(b, l, p.c);
  const T wod = (T)(p.omega / delta), inv_h2 = (T)(1.0 / (D.h * D.h));
  const SweepAddr sa = sweep_addr(D);
  T* Ef = nullptr;
  T* cur = B[l].u;
  T* oth = B[l].t;
  int k0 = 0;
  if (f) {
    Ef = B[l].g;
    if (u_zero && nu > 0) {
      // first sweep from u = 0: u = (omega/delta)(b + E f), keeping E f
      launch_ext<T, T>(b->dim, EXT_SMOOTH, D.n, f, ext_addr(D), fracK_of<T>(D), rhsA, cur, Ef, (T)delta, wod,
                       nullptr, ext_cfg(D), s);
      k0 = 1;
    } else {
      launch_ext<T, T>(b->dim, EXT_PLAIN, D.n, f, ext_addr(D), fracK_of<T>(D), nullptr, nullptr, Ef, (T)0, (T)0,
                       nullptr, ext_cfg(D), s);
    }
  } else if (u_zero && rhsA && nu > 0) {
    launch_scale_add<T>(D.n, rhsA, wod, cur, false, s);
    k0 = 1;
  }
  for (int k = k0; k < nu; ++k) {
    launch_sweep<T>(b->dim, EXT_SMOOTH, D.n, cur, oth, Ef, rhsA, sa, fracS_of<T>(D), inv_h2, (T)delta, wod,
                    sweep_cfg(D), s);
    std::swap(cur, oth);
  }
  launch_sweep<T>(b->dim, EXT_RESID, D.n, cur, B[l].r, Ef, rhsA, sa, fracS_of<T>(D), inv_h2, (T)delta, (T)0,
                  sweep_cfg(D), s);
  return cur;
}

template <typename T>
static void fused_post(const cpm_band b, int l, LevelBufs<T>* B, T* cur, const T* rhsA, const cpm_params& p, int nu,
                       hipStream_t s) {
  const DevLevel& D = b->dev[(size_t)l];
  const double delta = level_delta(b, l, p.c);
  const T wod = (T)(p.omega / delta), inv_h2 = (T)(1.0 / (D.h * D.h));
  const SweepAddr sa = sweep_addr(D);
  const T* Ef = rhsA ? nullptr : B[l].g;
  T* oth = cur == B[l].u ? B[l].t : B[l].u;
  for (int k = 0; k < nu; ++k) {
    launch_sweep<T>(b->dim, EXT_SMOOTH, D.n, cur, oth, Ef, rhsA, sa, fracS_of<T>(D), inv_h2, (T)delta, wod,
                    sweep_cfg(D), s);
    std::swap(cur, oth);
  }
  if (cur != B[l].u) launch_copy<T>(D.n, cur, B[l].u, s);
}

// The level's smoothing and residual with the tiled pass (f + N u formed in LDS per tile, then
// the extension, one launch per sweep), alternating between u and t.  r_first: the first
// sweep is u += (omega/delta) r_first (the residual of the entering u, bit for bit what the
// tiled residual pass computes); u_zero with an A-space right-hand side: u = (omega/delta) b.
// Returns the vector holding the iterate; the residual is left in B[l].r.
template <typename T>
static T* tile_pre(const cpm_band b, int l, LevelBufs<T>* B, const T* f, const T* rhsA, const cpm_params& p, int nu,
                   bool u_zero, const T* r_first, hipStream_t s) {
  const DevLevel& D = b->dev[(size_t)l];
  const double delta = level_delta(b, l, p.c);
  const T wod = (T)(p.omega / delta), inv_h2 = (T)(1.0 / (D.h * D.h));
  const TileAddr ta = tile_addr(D);
  T* cur = B[l].u;
  T* oth = B[l].t;
  int k0 = 0;
  if (nu > 0 && r_first) {
    launch_scale_add<T>(D.n, r_first, wod, cur, true, s);
    k0 = 1;
  } else if (nu > 0 && u_zero && rhsA && !f) {
    launch_scale_add<T>(D.n, rhsA, wod, cur, false, s);
    k0 = 1;
  }
  for (int k = k0; k < nu; ++k) {
    launch_tile<T, T>(EXT_SMOOTH, D.n, ta, fracT_of<T>(D), cur, f, rhsA, oth, inv_h2, (T)delta, wod, nullptr, s);
    std::swap(cur, oth);
  }
  launch_tile<T, T>(EXT_RESID, D.n, ta, fracT_of<T>(D), cur, f, rhsA, B[l].r, inv_h2, (T)delta, (T)0, nullptr, s);
  return cur;
}

template <typename T>
static void tile_post(const cpm_band b, int l, LevelBufs<T>* B, T* cur, const T* f, const T* rhsA,
                      const cpm_params& p, int nu, hipStream_t s) {
  const DevLevel& D = b->dev[(size_t)l];
  const double delta = level_delta(b, l, p.c);
  const T wod = (T)(p.omega / delta), inv_h2 = (T)(1.0 / (D.h * D.h));
  const TileAddr ta = tile_addr(D);
  T* oth = cur == B[l].u ? B[l].t : B[l].u;
  for (int k = 0; k < nu; ++k) {
    launch_tile<T, T>(EXT_SMOOTH, D.n, ta, fracT_of<T>(D), cur, f, rhsA, oth, inv_h2, (T)delta, wod, nullptr, s);
    std::swap(cur, oth);
  }
  if (cur != B[l].u) launch_copy<T>(D.n, cur, B[l].u, s);
}

// r_first (finest level, split sweeps only): the residual E(f + N u) - delta u of the
// entering iterate, already computed (the stopping test's) with the same two passes as a
// sweep, so that the first pre-smoothing sweep is u += (omega/delta) r_first, or the learned
// update applied to r_first, bit for bit.
// u_zero with an A-space right-hand side rhsA: the first sweep from u = 0 is
// u = (omega/delta) rhsA, and u need not be cleared beforehand.
template <typename T>
void vcycle_level(const cpm_band b, int l, LevelBufs<T>* B, const T* rhsA, const cpm_params& p, hipStream_t s,
                  bool u_zero, const T* r_first) {
  const DevLevel& D = b->dev[(size_t)l];
  const LaunchCfg lc = level_cfg(D);
  if (l == b->L - 1) {
    // coarsest: u = A_c^{-1} E_c f  (f-space right-hand side)
    if (b->coarse_cols > 0)
      launch_coarse_gemv_cols<T>((int)D.n, b->coarse_cols, b->coarseM, 2 * D.n, D.ilist, B[l].f, B[l].u, s);
    else
      launch_coarse_gemv<T>((int)D.n, b->coarseM + D.n, 2 * D.n, B[l].f, B[l].u, s);
    return;
  }
  const T* f = rhsA ? nullptr : B[l].f;
  const double delta = level_delta(b, l, p.c);
  const bool learned_here = b->learned_active && l < 2 && b->mlpW && D.patchRow;
  const bool learned = learned_here && p.learned_sweeps > 0;
  const int nu1 = learned ? p.learned_sweeps : p.nu1;
  const int nu2 = learned ? p.learned_sweeps : p.nu2;
  // u_zero: u is 0 on entry (the first visit after the restriction cleared it)
  const DevLevel& C = b->dev[(size_t)(l + 1)];
  const int visits = l + 1 == b->L - 1 ? 1 : (p.gamma > 1 ? p.gamma : 1);  // cycle index
  if (tiled(D) && !learned_here && !b->vc_active) {
    T* cur = tile_pre<T>(b, l, B, f, rhsA, p, nu1, u_zero, r_first, s);
    launch_restrict<T>(b->dim, C.n, B[l].r, C.runR, fracR_of<T>(C), B[l + 1].f, B[l + 1].u, level_cfg(C), s);
    for (int v = 0; v < visits; ++v) vcycle_level<T>(b, l + 1, B, nullptr, p, s, v == 0);
    // the post-smoothing alternates between u and t nu2 times: the prolongation writes
    // u + P e into the buffer from which the last sweep lands in u
    T* start = nu2 % 2 == 0 ? B[l].u : B[l].t;
    launch_prolong<T>(b->dim, D.n, B[l + 1].u, D.runP, fracP_of<T>(D), start, lc, s, cur);
    tile_post<T>(b, l, B, start, f, rhsA, p, nu2, s);
    return;
  }
  if (D.fused && D.fusedOK && !learned_here && !b->vc_active) {
    T* cur = fused_pre<T>(b, l, B, f, rhsA, p, nu1, u_zero, s);
    launch_restrict<T>(b->dim, C.n, B[l].r, C.runR, fracR_of<T>(C), B[l + 1].f, B[l + 1].u, level_cfg(C), s);
    for (int v = 0; v < visits; ++v) vcycle_level<T>(b, l + 1, B, nullptr, p, s, v == 0);
    // the post-smoothing alternates between u and t nu2 times: the prolongation writes
    // u + P e into the buffer from which the last sweep lands in u
    T* start = nu2 % 2 == 0 ? B[l].u : B[l].t;
    launch_prolong<T>(b->dim, D.n, B[l + 1].u, D.runP, fracP_of<T>(D), start, lc, s, cur);
    fused_post<T>(b, l, B, start, rhsA, p, nu2, s);
    return;
  }
  for (int k = 0; k < nu1; ++k) {
    if (k == 0 && learned_here && r_first) {  // the network's update from the residual at hand
      launch_learned<T>(b, l, r_first, B[l].u, p.c, s);
      continue;
    }
    if (k == 0 && !learned_here && !b->vc_active && (r_first || (u_zero && rhsA && !f))) {
      launch_scale_add<T>(D.n, r_first ? r_first : rhsA, (T)(p.omega / delta), B[l].u, r_first != nullptr, s);
      continue;
    }
    smooth_sweep<T>(b, l, B[l].u, f, rhsA, B[l].g, B[l].r, p.c, p.omega, nullptr, s, u_zero && k == 0);
  }
  // residual r = b + E(f + N u) - delta u, restricted to the next level (where u := 0)
  bool resid_done = false;
  if constexpr (sizeof(T) == 8) {
    if (b->vc_active) {
      // variable coefficient: r = D (E g - u), g = (f + N~ u) / D
      launch_nsum_var(b->dim, D.m, D.ilist, D.nbrI, (u_zero && nu1 == 0) ? nullptr : B[l].u, f, D.acoef, D.vcD,
                      1.0 / (D.h * D.h), B[l].g, lc, s);
      launch_ext<T, T>(b->dim, EXT_RESID, D.n, B[l].g, ext_addr(D), fracK_of<T>(D), rhsA, B[l].u, B[l].r, (T)1.0,
                       (T)0, nullptr, ext_cfg(D), s, D.vcD);
      resid_done = true;
    }
  }
  // the restriction reads r only at its stencils' fine nodes: where the level has that
  // subset's tables, the residual is formed there alone (the other entries are never read)
  const bool rs = resid_subset(D);
  const int64_t rn = rs ? D.rs_n : D.n;
  const ExtAddr ra = rs ? ext_addr_rs(D) : ext_addr(D);
  const T* rfrac = rs ? rs_frac_of<T>(D) : fracK_of<T>(D);
  if (resid_done) {
  } else if (u_zero && nu1 == 0 && f) {
    launch_ext<T, T>(b->dim, EXT_RESID, rn, f, ra, rfrac, rhsA, B[l].u, B[l].r, (T)delta, (T)0, nullptr, ext_cfg(D),
                     s);
  } else {
    launch_nsum<T>(b->dim, nsum_addr(D), B[l].u, f, (T)(1.0 / (D.h * D.h)), B[l].g, nullptr, lc, s);
    launch_ext<T, T>(b->dim, EXT_RESID, rn, B[l].g, ra, rfrac, rhsA, B[l].u, B[l].r, (T)delta, (T)0, nullptr,
                     ext_cfg(D), s);
  }
  launch_restrict<T>(b->dim, C.n, B[l].r, C.runR, fracR_of<T>(C), B[l + 1].f, B[l + 1].u, level_cfg(C), s);
  for (int v = 0; v < visits; ++v) vcycle_level<T>(b, l + 1, B, nullptr, p, s, v == 0);
  launch_prolong<T>(b->dim, D.n, B[l + 1].u, D.runP, fracP_of<T>(D), B[l].u, lc, s);
  for (int k = 0; k < nu2; ++k) smooth_sweep<T>(b, l, B[l].u, f, rhsA, B[l].g, B[l].r, p.c, p.omega, nullptr, s);
}

// V-cycle with the residual of Algorithm 4.1 step 2 as printed: the Ruuth-Merriman sweeps of
// the consistent cycle (two passes), r = f + N u - delta u at every node restricted to the
// coarse grid, and A_c e = f_c solved with A_c^{-1} on the coarsest level.
static void vcycle_verbatim(const cpm_band b, int l, LevelBufs<double>* B, const cpm_params& p, hipStream_t s,
                            bool u_zero) {
  const DevLevel& D = b->dev[(size_t)l];
  if (l == b->L - 1) {
    launch_coarse_gemv<double>((int)D.n, b->coarseS + D.n, 2 * D.n, B[l].f, B[l].u, s);
    return;
  }
  const LaunchCfg lc = level_cfg(D);
  for (int k = 0; k < p.nu1; ++k)
    smooth_sweep<double>(b, l, B[l].u, B[l].f, nullptr, B[l].g, B[l].r, p.c, p.omega, nullptr, s, u_zero && k == 0);
  launch_resid_verbatim(b->dim, D.n, D.nbr, B[l].u, B[l].f, level_delta(b, l, p.c), 1.0 / (D.h * D.h), B[l].r, s);
  const DevLevel& C = b->dev[(size_t)(l + 1)];
  launch_restrict<double>(b->dim, C.n, B[l].r, C.runR, fracR_of<double>(C), B[l + 1].f, B[l + 1].u, level_cfg(C), s);
  const int visits = l + 1 == b->L - 1 ? 1 : (p.gamma > 1 ? p.gamma : 1);
  for (int v = 0; v < visits; ++v) vcycle_verbatim(b, l + 1, B, p, s, v == 0);
  launch_prolong<double>(b->dim, D.n, B[l + 1].u, D.runP, fracP_of<double>(D), B[l].u, lc, s);
  for (int k = 0; k < p.nu2; ++k)
    smooth_sweep<double>(b, l, B[l].u, B[l].f, nullptr, B[l].g, B[l].r, p.c, p.omega, nullptr, s);
}

// V-cycle with the standard relaxation (Sec. 4.5): Jacobi on A_l e = f_l in steps 1 and 4,
// u <- u + (omega / diag(A)) (f - A u) with f - A u = f + E(N u) - delta u (or its red-black
// Gauss-Seidel ordering), the residual r = f - A (E u) passed to the coarse grid (the plain
// f - A u with CPM_RESIDUAL_VERBATIM); the coarsest level is solved with A_c^{-1}.  With
// el_degree 1 the operator is Remark 3.2's A = delta I - E_1 N + gamma (E_1 - E_3), whose
// sweeps read u at the stencil nodes and so write into t first.
static void vcycle_std(const cpm_band b, int l, LevelBufs<double>* B, const cpm_params& p, hipStream_t s) {
  const DevLevel& D = b->dev[(size_t)l];
  const bool el1 = p.el_degree == 1;
  if (l == b->L - 1) {
    const double* Z = el1 ? b->coarseS1 : b->coarseS;
    launch_coarse_gemv<double>((int)D.n, Z + D.n, 2 * D.n, B[l].f, B[l].u, s);
    return;
  }
  const LaunchCfg lc = level_cfg(D);
  const double delta = level_delta(b, l, p.c), inv_h2 = 1.0 / (D.h * D.h), gamma = 2.0 * b->dim * inv_h2;
  const ExtAddr ea{D.perm, D.packed, D.origin};
  // one Jacobi sweep, or the red then the black half-sweep (the cubic-E extension pass updates
  // only the node it visits, so each half-sweep is in place; the black one reads the new reds)
  auto half = [&](const double* wd) {
    launch_nsum<double>(b->dim, nsum_addr(D), B[l].u, nullptr, inv_h2, B[l].g, nullptr, lc, s);
    if (el1) {
      launch_p1(b->dim, EXT_SMOOTH, D.n, B[l].g, B[l].u, ea, D.fracK, B[l].f, wd, B[l].t, delta, gamma, ext_cfg(D),
                s);
      launch_copy<double>(D.n, B[l].t, B[l].u, s);
    } else {
      launch_ext<double, double>(b->dim, EXT_SMOOTH, D.n, B[l].g, ext_addr(D), fracK_of<double>(D), B[l].f, B[l].u,
                                 (double*)nullptr, delta, 0.0, nullptr, ext_cfg(D), s, wd);
    }
  };
  auto sweep = [&] {
    if (p.smoother == CPM_SMOOTH_STANDARD_RB) {
      half(D.wdR);
      half(D.wdB);
    } else {
      half(D.wd);
    }
  };
  for (int k = 0; k < p.nu1; ++k) sweep();
  // r = f - A v with v = E u (into t), or v = u for the plain residual
  const double* v = B[l].u;
  if (p.residual_mode != CPM_RESIDUAL_VERBATIM) {
    launch_ext<double, double>(b->dim, EXT_PLAIN, D.n, B[l].u, ext_addr(D), fracK_of<double>(D), nullptr, nullptr,
                               B[l].t, 0.0, 0.0, nullptr, ext_cfg(D), s);
    v = B[l].t;
  }
  launch_nsum<double>(b->dim, nsum_addr(D), v, nullptr, inv_h2, B[l].g, nullptr, lc, s);
  if (el1)
    launch_p1(b->dim, EXT_RESID, D.n, B[l].g, v, ea, D.fracK, B[l].f, nullptr, B[l].r, delta, gamma, ext_cfg(D), s);
  else
    launch_ext<double, double>(b->dim, EXT_RESID, D.n, B[l].g, ext_addr(D), fracK_of<double>(D), B[l].f,
                               const_cast<double*>(v), B[l].r, delta, 0.0, nullptr, ext_cfg(D), s);
  const DevLevel& C = b->dev[(size_t)(l + 1)];
  launch_restrict<double>(b->dim, C.n, B[l].r, C.runR, fracR_of<double>(C), B[l + 1].f, B[l + 1].u, level_cfg(C), s);
  const int visits = l + 1 == b->L - 1 ? 1 : (p.gamma > 1 ? p.gamma : 1);
  for (int vv = 0; vv < visits; ++vv) vcycle_std(b, l + 1, B, p, s);
  launch_prolong<double>(b->dim, D.n, B[l + 1].u, D.runP, fracP_of<double>(D), B[l].u, lc, s);
  for (int k = 0; k < p.nu2; ++k) sweep();
}

// Full-multigrid start into u (nested iteration): f restricted down the hierarchy, the
// coarsest level solved, then on each finer level the cubic closest-point interpolation of
// the coarser solution improved by one cycle.
static void enqueue_fmg(const cpm_band b, const cpm_params& p, const double* f, double* u, void* work,
                        hipStream_t s) {
  LevelBufs<double> B[kMaxLevels];
  carve_levels<double>(b, work, B, nullptr);
  B[0].u = u;
  B[0].f = const_cast<double*>(f);
  const int L = b->L;
  for (int l = 0; l + 1 < L; ++l) {
    const DevLevel& C = b->dev[(size_t)(l + 1)];
    launch_restrict<double>(b->dim, C.n, B[l].f, C.runR, fracR_of<double>(C), B[l + 1].f, nullptr, level_cfg(C), s);
  }
  vcycle_level<double>(b, L - 1, B, nullptr, p, s, true);  // coarsest: exact
  for (int l = L - 2; l >= 0; --l) {
    const DevLevel& D = b->dev[(size_t)l];
    launch_interp3(b->dim, D.n, B[l + 1].u, D.runP3, D.fracP3, B[l].u, s);
    vcycle_level<double>(b, l, B, nullptr, p, s, false);
  }
}

static bool fmg_ok(const cpm_band b) {
  for (int l = 0; l + 1 < b->L; ++l)
    if (!b->dev[(size_t)l].runP3) return false;
  return true;
}

// ||E f||_inf into scalar slot 1 (double)
void enqueue_rhs_norm(const cpm_band b, const double* f, double* g, hipStream_t s) {
  const DevLevel& D = b->dev[0];
  launch_zero_u64(b->dscal + 1, 1, s);
  if (b->vc_active) {
    // ||D E (f / D)||_inf: g = f / D, then the residual form with delta = 0 scaled by D
    launch_nsum_var(b->dim, D.m, D.ilist, D.nbrI, nullptr, f, D.acoef, D.vcD, 1.0 / (D.h * D.h), g, level_cfg(D), s);
    launch_ext<double, double>(b->dim, EXT_RESID, D.n, g, ext_addr(D), fracK_of<double>(D), nullptr, g,
                               (double*)nullptr, 0.0, 0.0, b->dscal + 1, ext_cfg(D), s, D.vcD);
    return;
  }
  launch_ext<double, double>(b->dim, EXT_PLAIN, D.n, f, ext_addr(D), fracK_of<double>(D), nullptr, nullptr, (double*)nullptr,
                             0.0, 0.0, b->dscal + 1, ext_cfg(D), s);
}

// ||E(f + N u) - delta u||_inf into slot 0; optionally the residual as float into r32 or as
// double into r64
void enqueue_resid64(const cpm_band b, const double* f, const double* u, double* g, float* r32, double c,
                     hipStream_t s, double* r64 = nullptr) {
  const DevLevel& D = b->dev[0];
  const LaunchCfg lc = level_cfg(D);
  if (b->vc_active) {
    launch_zero_u64(b->dscal, 1, s);
    launch_nsum_var(b->dim, D.m, D.ilist, D.nbrI, u, f, D.acoef, D.vcD, 1.0 / (D.h * D.h), g, lc, s);
    launch_ext<double, float>(b->dim, EXT_RESID, D.n, g, ext_addr(D), fracK_of<double>(D), nullptr,
                              const_cast<double*>(u), r32, 1.0, 0.0, b->dscal, ext_cfg(D), s, D.vcD);
    return;
  }
  if (tiled(D)) {
    launch_zero_u64(b->dscal, 1, s);
    if (r64)
      launch_tile<double, double>(EXT_RESID, D.n, tile_addr(D), D.fracT, u, f, nullptr, r64, 1.0 / (D.h * D.h),
                                  level_delta(b, 0, c), 0.0, b->dscal, s);
    else
      launch_tile<double, float>(EXT_RESID, D.n, tile_addr(D), D.fracT, u, f, nullptr, r32, 1.0 / (D.h * D.h),
                                 level_delta(b, 0, c), 0.0, b->dscal, s);
    return;
  }
  launch_nsum<double>(b->dim, nsum_addr(D), u, f, 1.0 / (D.h * D.h), g, b->dscal, lc, s);
  if (r64)
    launch_ext<double, double>(b->dim, EXT_RESID, D.n, g, ext_addr(D), fracK_of<double>(D), nullptr,
                               const_cast<double*>(u), r64, level_delta(b, 0, c), 0.0, b->dscal, ext_cfg(D), s);
  else
    launch_ext<double, float>(b->dim, EXT_RESID, D.n, g, ext_addr(D), fracK_of<double>(D), nullptr,
                              const_cast<double*>(u), r32, level_delta(b, 0, c), 0.0, b->dscal, ext_cfg(D), s);
}

// Whether a cycle may start from the residual that the previous cycle's stopping test left
// in the finest level's r: the FP64 cycle with constant coefficients whose finest level sweeps
// in two passes (the fused pass forms the same residual in another rounding order), with the
// Ruuth-Merriman step or the learned update (which is applied to that residual).
static bool resid_reuse_ok(const cpm_band b, const cpm_params& p) {
  const DevLevel& D = b->dev[0];
  if (p.precision != CPM_F64 || b->vc_active || standard(p) ||
      p.residual_mode == CPM_RESIDUAL_VERBATIM)
    return false;
  const bool learned0 = b->learned_active && b->mlpW && D.patchRow;  // never fused
  const int nu1 = learned0 && p.learned_sweeps > 0 ? p.learned_sweeps : p.nu1;
  return nu1 > 0 && (learned0 || tiled(D) || !(D.fused && D.fusedOK));
}

// One complete cycle of the solve loop on stream s, ending with the residual
// norm of the new iterate in slot 0 (and, in FP64, the residual itself in the finest
// level's r).  r_ready: that residual is the one of the entering u (the previous cycle of the
// same solve left it), so the first smoothing sweep is taken from it.
void enqueue_cycle(const cpm_band b, const cpm_params& p, const double* f, double* u, void* work, hipStream_t s,
                   bool r_ready) {
  if (standard(p) || p.residual_mode == CPM_RESIDUAL_VERBATIM) {
    // slot 0 = ||u_new - u_old||_inf, slot 1 = ||u_new||_inf (the paper's stopping test)
    LevelBufs<double> B[kMaxLevels];
    carve_levels<double>(b, work, B, nullptr);
    B[0].u = u;
    B[0].f = const_cast<double*>(f);
    launch_copy<double>(b->dev[0].n, u, B[0].p, s);
    if (standard(p))
      vcycle_std(b, 0, B, p, s);  // verbatim: the plain residual f - A u
    else
      vcycle_verbatim(b, 0, B, p, s, false);
    launch_zero_u64(b->dscal, 2, s);
    launch_incr(b->dev[0].n, u, B[0].p, b->dscal, s);
    return;
  }
  if (p.precision == CPM_F64) {
    LevelBufs<double> B[kMaxLevels];
    carve_levels<double>(b, work, B, nullptr);
    B[0].u = u;
    B[0].f = const_cast<double*>(f);
    const bool reuse = resid_reuse_ok(b, p);
    vcycle_level<double>(b, 0, B, nullptr, p, s, false, reuse && r_ready ? B[0].r : nullptr);
    enqueue_resid64(b, f, u, B[0].g, nullptr, p.c, s, reuse ? B[0].r : nullptr);
  } else {
    LevelBufs<float> B[kMaxLevels];
    double* g64 = nullptr;
    carve_levels<float>(b, work, B, &g64);
    // B[0].f holds the float32 copy of the double residual (A-space right-hand side); the
    // correction starts from 0, and its first sweep (u = (omega/delta) B[0].f) writes all of u
    const bool zero_start = p.nu1 > 0 && !b->learned_active;
    if (!zero_start) launch_fill<float>(b->dev[0].n, B[0].u, 0.0f, s);
    vcycle_level<float>(b, 0, B, B[0].f, p, s, zero_start);
    launch_axpy_f32_to_f64(b->dev[0].n, B[0].u, u, s);
    enqueue_resid64(b, f, u, g64, B[0].f, p.c, s);
  }
}

// Prologue of a solve: ||E f|| (slot 1) and, in mixed precision, the first residual.
void enqueue_prologue(const cpm_band b, const cpm_params& p, const double* f, const double* u, void* work,
                      hipStream_t s) {
  if (standard(p) || p.residual_mode == CPM_RESIDUAL_VERBATIM) {
    // ||f||_inf into slot 1 (the system is A u = f)
    launch_zero_u64(b->dscal, 2, s);
    launch_incr(b->dev[0].n, f, nullptr, b->dscal, s);
    return;
  }
  if (p.precision == CPM_F64) {
    LevelBufs<double> B[kMaxLevels];
    carve_levels<double>(b, work, B, nullptr);
    enqueue_rhs_norm(b, f, B[0].g, s);
  } else {
    LevelBufs<float> B[kMaxLevels];
    double* g64 = nullptr;
    carve_levels<float>(b, work, B, &g64);
    enqueue_rhs_norm(b, f, g64, s);
    enqueue_resid64(b, f, u, g64, B[0].f, p.c, s);
  }
}

cpm_status read_scalars(cpm_band b, double* r0, double* r1) {
  if (hipMemcpyAsync(b->hpinned, b->dscal, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, b->stream) !=
          hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess) {
    set_error(std::string("synchronization failed: ") + hipGetErrorString(hipGetLastError()));
    return CPM_E_HIP;
  }
  double v0, v1;
  std::memcpy(&v0, &b->hpinned[0], 8);
  std::memcpy(&v1, &b->hpinned[1], 8);
  if (r0) *r0 = v0;
  if (r1) *r1 = v1;
  return CPM_OK;
}

static std::string graph_key(const char* tag, const cpm_params& p, const void* a, const void* bb, const void* c,
                             int extra) {
  std::ostringstream os;
  os << tag << '|' << p.c << '|' << p.nu1 << '|' << p.nu2 << '|' << p.omega << '|' << p.precision << '|'
     << p.smoother << '|' << p.learned_sweeps << '|' << p.gamma << '|' << p.residual_mode << '|' << p.el_degree << '|' << a << '|' << bb
     << '|' << c << '|' << extra;
  return os.str();
}

// Capture `fn` on the private stream once per key and launch the executable graph on the
// current stream.
template <typename Fn>
cpm_status graph_launch(cpm_band b, const std::string& key, Fn fn) {
  auto it = b->graphs.find(key);
  if (it == b->graphs.end()) {
    if (b->graphs.size() > 64) {
      for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
      b->graphs.clear();
    }
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      set_error("hipStreamBeginCapture failed");
      return CPM_E_HIP;
    }
    fn(b->own);
    hipError_t e = hipStreamEndCapture(b->own, &graph);
    if (e != hipSuccess || !graph) {
      set_error(std::string("graph capture failed: ") + hipGetErrorString(e));
      return CPM_E_HIP;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      set_error(std::string("graph instantiation failed: ") + hipGetErrorString(e));
      return CPM_E_HIP;
    }
    it = b->graphs.emplace(key, exec).first;
  }
  if (hipGraphLaunch(it->second, b->stream) != hipSuccess) {
    set_error("hipGraphLaunch failed");
    return CPM_E_HIP;
  }
  return CPM_OK;
}

// For every level that has the fused pass (and whose form no environment variable pins),
// time FP64 V-cycles of the paper's parameters (nu1 = nu2 = 3, omega = 2/3, c = 1) on a
// constant right-hand side with the level sweeping in two passes, fused with gathers, and
// fused from LDS, the other levels as they stand, and keep the fastest.
cpm_status tune_sweep_forms(cpm_band b) {
  if (b->vc_active) return CPM_OK;  // variable coefficients always sweep in two passes
  bool any = false;  // a level that could sweep more than one way
  for (int l = 0; l + 1 < b->L; ++l) {
    const DevLevel& D = b->dev[(size_t)l];
    any = any || ((D.fusedOK || D.ntiles > 0) && !D.sweep_forced);
  }
  // bands that cannot run cycles (coarsest level beyond the dense solve) keep the first stage
  if (!any || b->dev[(size_t)(b->L - 1)].n > kMaxCoarse) return CPM_OK;
  cpm_status st = ensure_coarse(b, 1.0);
  if (st != CPM_OK) return st;
  const int64_t n0 = b->dev[0].n;
  const size_t wb = layout_bytes(b, CPM_F64);
  double* f = (double*)dev_alloc(b, n0 * sizeof(double));
  double* u = (double*)dev_alloc(b, n0 * sizeof(double));
  void* work = dev_alloc(b, wb);
  if (!f || !u || !work) {
    dev_free(b, f);
    dev_free(b, u);
    dev_free(b, work);
    set_error("autotune: allocation failed");
    return CPM_E_NOMEM;
  }
  hipStream_t s = b->stream;
  launch_fill<double>(n0, f, 1.0, s);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  cpm_params p{};
  p.c = 1.0;
  p.nu1 = 3;
  p.nu2 = 3;
  p.omega = 2.0 / 3.0;
  p.precision = CPM_F64;
  p.smoother = CPM_SMOOTH_JACOBI;
  p.gamma = 1;
  const bool learned = b->learned_active;
  b->learned_active = false;
  // Each candidate is captured once into a graph of kCyc cycles; the candidates are then
  // timed in turn over several rounds (the minimum per candidate), so that slow drifts of
  // the clock do not favour the one measured first.
  constexpr int kCyc = 4, kReps = 4, kRounds = 4;
  auto body = [&](hipStream_t st2) {
    for (int j = 0; j < kCyc; ++j) enqueue_cycle(b, p, f, u, work, st2, j > 0);
  };
  for (int l = 0; l < b->L - 1 && st == CPM_OK; ++l) {
    DevLevel& D = b->dev[(size_t)l];
    if ((!D.fusedOK && D.ntiles <= 0) || D.sweep_forced) continue;
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
    launch_fill<double>(n0, u, 0.0, s);
    // candidates: 0 two passes, 1 fused with gathers, 2 fused from LDS, 3 tiled
    bool have[4] = {false, false, false, false};
    for (int cand = 0; cand < 4 && st == CPM_OK; ++cand) {
      if ((cand == 1 && !D.fusedOK) || (cand == 2 && !D.sweep_lds) || (cand == 3 && D.ntiles <= 0)) continue;
      D.fused = cand == 1 || cand == 2;
      D.use_sweep_lds = cand == 2;
      D.use_tile = cand == 3;
      st = graph_launch(b, "autotune" + std::to_string(cand), body);  // capture + warm-up
      have[cand] = st == CPM_OK;
    }
    float best[4] = {1e30f, 1e30f, 1e30f, 1e30f};
    for (int round = 0; round < kRounds && st == CPM_OK; ++round)
      for (int cand = 0; cand < 4 && st == CPM_OK; ++cand) {
        if (!have[cand]) continue;
        const std::string key = "autotune" + std::to_string(cand);
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < kReps && st == CPM_OK; ++r) st = graph_launch(b, key, body);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        best[cand] = std::min(best[cand], 1000.f * ms / (kCyc * kReps));
      }
    int pick = 0;
    for (int cand = 1; cand < 4; ++cand)
      if (have[cand] && best[cand] < best[pick]) pick = cand;
    D.fused = pick == 1 || pick == 2;
    D.use_sweep_lds = pick == 2;
    D.use_tile = pick == 3;
  }
  b->learned_active = learned;
  (void)hipStreamSynchronize(s);
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  dev_free(b, f);
  dev_free(b, u);
  dev_free(b, work);
  if (st != CPM_OK) return st;
  return check_launch("autotune (whole cycles)");
}

cpm_status validate_params(const cpm_band b, const cpm_params* p) {
  if (!p) {
    set_error("params is NULL");
    return CPM_E_INVALID;
  }
  if (!(p->c > 0.0) || p->nu1 < 0 || p->nu2 < 0 || p->nu1 + p->nu2 == 0 || !(p->omega > 0.0) ||
      !(p->omega <= 2.0)) {
    set_error("invalid solver parameters (need c > 0, nu1 + nu2 > 0, 0 < omega <= 2)");
    return CPM_E_INVALID;
  }
  if (p->learned_sweeps < 0) {
    set_error("learned_sweeps must be >= 0");
    return CPM_E_INVALID;
  }
  if (p->precision != CPM_F64 && p->precision != CPM_MIXED) {
    set_error("unknown precision");
    return CPM_E_INVALID;
  }
  if (p->smoother != CPM_SMOOTH_JACOBI && p->smoother != CPM_SMOOTH_LEARNED && p->smoother != CPM_SMOOTH_STANDARD &&
      p->smoother != CPM_SMOOTH_STANDARD_RB) {
    set_error("unknown smoother");
    return CPM_E_INVALID;
  }
  if (b->vc_active && (p->precision != CPM_F64 || p->smoother != CPM_SMOOTH_JACOBI)) {
    set_error("a variable diffusion coefficient runs with precision CPM_F64 and smoother CPM_SMOOTH_JACOBI only");
    return CPM_E_INVALID;
  }
  if (p->residual_mode != CPM_RESIDUAL_CONSISTENT && p->residual_mode != CPM_RESIDUAL_VERBATIM) {
    set_error("unknown residual mode");
    return CPM_E_INVALID;
  }
  if (p->residual_mode == CPM_RESIDUAL_VERBATIM &&
      (p->precision != CPM_F64 || !(p->smoother == CPM_SMOOTH_JACOBI || standard(*p)) || b->vc_active || p->fmg)) {
    set_error("the verbatim residual runs with precision CPM_F64, the Jacobi or standard-relaxation smoother, a "
              "constant coefficient and no full-multigrid start");
    return CPM_E_INVALID;
  }
  if (p->el_degree != 0 && p->el_degree != 1 && p->el_degree != 3) {
    set_error("el_degree must be 1 or 3 (0 = 3)");
    return CPM_E_INVALID;
  }
  if (p->el_degree == 1 && !standard(*p)) {
    set_error("the linear interpolation in front of L (Remark 3.2) runs with the standard relaxation");
    return CPM_E_INVALID;
  }
  if (p->gamma < 0 || p->gamma > 4) {
    set_error("cycle index gamma must be in 0..4");
    return CPM_E_INVALID;
  }
  if (p->fmg && p->smoother != CPM_SMOOTH_JACOBI) {
    set_error("the full-multigrid start runs with smoother CPM_SMOOTH_JACOBI");
    return CPM_E_INVALID;
  }
  if (p->fmg && !fmg_ok(b)) {
    set_error("no full-multigrid start on this band: a cubic interpolation stencil leaves a coarser band");
    return CPM_E_INVALID;
  }
  if (standard(*p) && p->precision != CPM_F64) {
    set_error("the standard relaxation runs in double precision only");
    return CPM_E_INVALID;
  }
  if (p->precision == CPM_MIXED && b->L < 2) {
    set_error("mixed precision needs at least two levels");
    return CPM_E_INVALID;
  }
  if (p->smoother == CPM_SMOOTH_LEARNED && !b->mlpW) {
    set_error("learned smoother selected but no weights were set");
    return CPM_E_INVALID;
  }
  if (p->smoother == CPM_SMOOTH_LEARNED)
    for (int l = 0; l < 2 && l + 1 < b->L; ++l)
      if (!b->dev[(size_t)l].patchRow) {
        set_error("learned smoother unavailable: level " + std::to_string(l) +
                  " has too many patch groups to address (more than 2^23)");
        return CPM_E_INVALID;
      }
  return CPM_OK;
}

}  // namespace cpm

// ------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------

extern "C" {

const char* cpm_status_string(int status) {
  switch (status) {
    case CPM_OK: return "ok";
    case CPM_E_INVALID: return "invalid argument";
    case CPM_E_BAND: return "stencil leaves the band";
    case CPM_E_NOMEM: return "out of memory";
    case CPM_E_HIP: return "HIP runtime error";
    case CPM_E_NOCONV: return "not converged";
    case CPM_E_DIVERGED: return "diverged (NaN or Inf residual)";
    case CPM_E_WORKSPACE: return "workspace too small";
    default: return "unknown status";
  }
}

const char* cpm_last_error(void) { return cpm::g_last_error.c_str(); }

cpm_status cpm_set_allocator(void* (*alloc)(void* ctx, size_t bytes), void (*release)(void* ctx, void* ptr),
                             void* ctx) {
  if ((alloc == nullptr) != (release == nullptr)) {
    set_error("cpm_set_allocator: give both functions or neither");
    return CPM_E_INVALID;
  }
  g_allocator = cpm::DeviceAllocator{alloc, release, ctx};
  return CPM_OK;
}

cpm_status cpm_build_band(const cpm_surface* surface, const cpm_grid* grid, void* stream, cpm_band* out) {
  if (!surface || !grid || !out) {
    set_error("null argument");
    return CPM_E_INVALID;
  }
  *out = nullptr;
  const int kind = surface->kind;
  if (kind != CPM_CIRCLE && kind != CPM_SPHERE && kind != CPM_TORUS && kind != CPM_DZIUK) {
    set_error("unknown surface kind");
    return CPM_E_INVALID;
  }
  if ((kind != CPM_DZIUK && !(surface->R > 0)) ||
      (kind == CPM_TORUS && !(surface->r > 0 && surface->r < surface->R))) {
    set_error("invalid surface radii");
    return CPM_E_INVALID;
  }
  if (!(grid->h0 > 0) || grid->levels < 1 || grid->levels > kMaxLevels) {
    set_error("invalid grid (need h0 > 0, 1 <= levels <= 12)");
    return CPM_E_INVALID;
  }
  const int dim = kind == CPM_CIRCLE ? 2 : 3;
  cpm_band b = new (std::nothrow) cpm_band_s();
  if (!b) return CPM_E_NOMEM;
  b->surf = *surface;
  b->grid = *grid;
  b->allocator = g_allocator;
  b->dim = dim;
  b->L = grid->levels;
  std::string err;
  cpm_status st = build_host_levels(*surface, *grid, dim, b->host, err);
  if (st != CPM_OK) {
    set_error(err);
    delete b;
    return st;
  }
  if (hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking) != hipSuccess) {
    set_error("stream creation failed");
    delete b;
    return CPM_E_HIP;
  }
  b->stream = b->own;
  b->dev.resize((size_t)b->L);
  // order in which the extension visits nodes: stencil order (default) or band order
  const char* ord = std::getenv("CPM_EXT_ORDER");
  const bool band_order = ord && std::strcmp(ord, "band") == 0;
  for (int l = 0; l < b->L && st == CPM_OK; ++l) {
    HostLevel& H = b->host[(size_t)l];
    DevLevel& D = b->dev[(size_t)l];
    D.n = H.n;
    D.h = H.h;
    D.m = (int64_t)H.ilist.size();
    D.ngroups = H.ngroups;
    if (st == CPM_OK) st = upload(b, &D.perm, H.perm);
    if (st == CPM_OK) st = upload(b, &D.packed, H.packed);
    if (st == CPM_OK) st = upload(b, &D.origin, H.origin);
    if (st == CPM_OK) st = upload(b, &D.fracK, H.fracK);
    if (st == CPM_OK) st = upload_f32(b, &D.fracK32, H.fracK);
    if (st == CPM_OK) st = upload(b, &D.ilist, H.ilist);
    if (st == CPM_OK) st = upload(b, &D.nbrI, H.nbrI);
    // the neighbour sum reads its segment tables unless CPM_NSUM_SEG=0
    const char* nseg_env = std::getenv("CPM_NSUM_SEG");
    if (!H.nsSegOff.empty() && !(nseg_env && std::strcmp(nseg_env, "0") == 0)) {
      if (st == CPM_OK) st = upload(b, &D.nsSeg, H.nsSeg);
      if (st == CPM_OK) st = upload(b, &D.nsChunkSeg, H.nsChunkSeg);
      if (st == CPM_OK) st = upload(b, &D.nsSegOff, H.nsSegOff);
    }
    if (H.patchOK && !H.patchBase.empty()) {
      if (st == CPM_OK) st = upload(b, &D.patchRow, H.patchBase);
      if (st == CPM_OK) st = upload(b, &D.patchPk, H.patchPk);
      if (st == CPM_OK) st = upload(b, &D.patchMask, H.patchMask);
      D.patchGroups = H.patchGroups;
    }
    std::vector<int32_t>().swap(H.patchRow);
    std::vector<int32_t>().swap(H.patchBase);
    std::vector<int32_t>().swap(H.patchPk);
    std::vector<uint32_t>().swap(H.patchMask);
    D.band_order = band_order;
    if (st == CPM_OK) st = upload(b, &D.qdiag, H.qdiag);
    if (st == CPM_OK) st = upload(b, &D.q1diag, H.q1diag);
    std::vector<double>().swap(H.qdiag);
    std::vector<double>().swap(H.q1diag);
    if (st == CPM_OK) st = upload(b, &D.originX, H.originX);
    std::vector<int32_t>().swap(H.originX);
    D.fusedOK = H.fusedOK && D.originX != nullptr;
    {
      // sweep form before autotuning: CPM_SWEEP=fused|split forces one, otherwise the fused
      // pass on levels small enough for launch latency to dominate
      const char* e = std::getenv("CPM_SWEEP");
      D.sweep_forced = e && (std::strcmp(e, "fused") == 0 || std::strcmp(e, "split") == 0);
      if (e && std::strcmp(e, "fused") == 0)
        D.fused = D.fusedOK;
      else if (e && std::strcmp(e, "split") == 0)
        D.fused = false;
      else
        D.fused = D.fusedOK && H.n <= kFusedDefaultNodes;
    }
    // LDS-staged extension unless disabled or a workgroup would stage too many values
    const char* lds_env = std::getenv("CPM_EXT_LDS");
    const size_t lds_bytes = (((size_t)H.maxE * sizeof(double) + 15) & ~(size_t)15) +
                             (size_t)H.maxG * (H.dim == 2 ? 4 : 16) * sizeof(int32_t);
    D.lds = !band_order && H.maxE <= kMaxStaged && lds_bytes <= (size_t)kMaxDynLds &&
            !(lds_env && std::strcmp(lds_env, "0") == 0);
    // defaults before autotuning: with the Morton-blocked visit order the LDS-staged form
    // is the faster one on every level measured, and loading the node's own data before the
    // staging pays on the largest levels (8.5M nodes: 150 vs 156 us per launch)
    D.use_lds = D.lds;
    D.ext_prefetch = H.n >= kExtNptMinNodes;
    if (const char* pe = std::getenv("CPM_EXT_PREFETCH")) {
      D.ext_prefetch = std::strcmp(pe, "1") == 0;
      D.prefetch_forced = true;
    }
    D.maxE = H.maxE;
    D.maxG = H.maxG;
    D.ext_npt = H.extNpt;
    if (D.lds) {
      if (st == CPM_OK) st = upload(b, &D.packedL, H.packedL);
      if (st == CPM_OK) st = upload(b, &D.blkE, H.blkE);
      if (st == CPM_OK) st = upload(b, &D.gidx, H.gidx);
      if (st == CPM_OK) st = upload(b, &D.blkG, H.blkG);
      if (st == CPM_OK) st = upload(b, &D.lorg, H.lorg);
    }
    // the residual before restriction over the restriction's fine nodes only
    if (D.lds && H.rsN > 0) {
      const size_t rs_bytes = (((size_t)H.rsMaxE * sizeof(double) + 15) & ~(size_t)15) +
                              (size_t)H.rsMaxG * (H.dim == 2 ? 4 : 16) * sizeof(int32_t);
      if (H.rsMaxE <= kMaxStaged && rs_bytes <= (size_t)kMaxDynLds) {
        if (st == CPM_OK) st = upload(b, &D.rs_perm, H.rsPerm);
        if (st == CPM_OK) st = upload(b, &D.rs_packedL, H.rsPackedL);
        if (st == CPM_OK) st = upload(b, &D.rs_blkE, H.rsBlkE);
        if (st == CPM_OK) st = upload(b, &D.rs_gidx, H.rsGidx);
        if (st == CPM_OK) st = upload(b, &D.rs_blkG, H.rsBlkG);
        if (st == CPM_OK) st = upload(b, &D.rs_lorg, H.rsLorg);
        if (st == CPM_OK) st = upload(b, &D.rs_frac, H.rsFrac);
        if (st == CPM_OK) st = upload_f32(b, &D.rs_frac32, H.rsFrac);
        D.rs_n = H.rsN;
        D.rs_maxE = H.rsMaxE;
        D.rs_maxG = H.rsMaxG;
        D.rs_npt = H.rsNpt;
      }
    }
    // LDS-staged fused sweep (on the extension's workgroups) unless disabled by
    // CPM_SWEEP_LDS=0 or a workgroup would stage too many values; it is the default form of
    // the fused pass where present
    const char* slds_env = std::getenv("CPM_SWEEP_LDS");
    D.sweep_lds = D.lds && D.fusedOK && !H.blkE2.empty() && H.maxE2 <= kMaxStaged &&
                  !(slds_env && std::strcmp(slds_env, "0") == 0);
    D.use_sweep_lds = D.sweep_lds;
    D.maxE2 = H.maxE2;
    if (D.sweep_lds) {
      if (st == CPM_OK) st = upload(b, &D.blkE2, H.blkE2);
      if (st == CPM_OK) st = upload(b, &D.gidx2, H.gidx2);
      if (st == CPM_OK) st = upload(b, &D.lorg2, H.lorg2);
    }
    // tiled sweep tables: a candidate of cpm_autotune (measured slower than the two passes on
    // the large levels it is built for), or forced with CPM_SWEEP=tile
    if (H.ntiles > 0) {
      D.ntiles = H.ntiles;
      if (st == CPM_OK) st = upload(b, &D.tileSlot, H.tileSlot);
      if (st == CPM_OK) st = upload(b, &D.tileRow, H.tileRow);
      if (st == CPM_OK) st = upload(b, &D.tperm, H.tperm);
      if (st == CPM_OK) st = upload(b, &D.tloc, H.tloc);
      if (st == CPM_OK) st = upload(b, &D.fracT, H.fracT);
      if (st == CPM_OK) st = upload_f32(b, &D.fracT32, H.fracT);
      const char* e = std::getenv("CPM_SWEEP");
      D.use_tile = e && std::strcmp(e, "tile") == 0;
      if (D.use_tile) {
        D.sweep_forced = true;
        D.fused = false;
      }
    }
    std::vector<int32_t>().swap(H.tileSlot);
    std::vector<int32_t>().swap(H.tileOrg);
    std::vector<int32_t>().swap(H.tileRow);
    std::vector<int32_t>().swap(H.tperm);
    std::vector<int32_t>().swap(H.tloc);
    std::vector<double>().swap(H.fracT);
    std::vector<int32_t>().swap(H.blkE2);
    std::vector<int32_t>().swap(H.gidx2);
    std::vector<int32_t>().swap(H.lorg2);
    std::vector<int32_t>().swap(H.packedL);
    std::vector<int32_t>().swap(H.blkE);
    std::vector<int32_t>().swap(H.gidx);
    std::vector<int32_t>().swap(H.blkG);
    std::vector<int32_t>().swap(H.lorg);
    // band-order fractions: band-order extension, the learned smoother's weights features,
    // and the coarsest level's matrix assembly
    const bool learned_level = D.patchRow != nullptr;
    if (band_order && st == CPM_OK) st = upload(b, &D.packedB, H.packedB);
    if ((band_order || learned_level) && st == CPM_OK) st = upload_f32(b, &D.fracE32, H.fracE);
    if ((band_order || learned_level || l == b->L - 1) && st == CPM_OK) st = upload(b, &D.fracE, H.fracE);
    if (l == b->L - 1) {
      // band-order addressing of the coarsest level, used to assemble its dense matrix
      if (st == CPM_OK) st = upload(b, &D.runE, H.runE);
      if (st == CPM_OK) st = upload(b, &D.nbr, H.nbr);
    }
    if (st == CPM_OK) st = upload(b, &D.runP, H.runP);
    if (st == CPM_OK) st = upload(b, &D.fracP, H.fracP);
    if (st == CPM_OK && !H.fracP.empty()) st = upload_f32(b, &D.fracP32, H.fracP);
    if (st == CPM_OK) st = upload(b, &D.runP3, H.runP3);
    if (st == CPM_OK) st = upload(b, &D.fracP3, H.fracP3);
    std::vector<int32_t>().swap(H.runP3);
    std::vector<double>().swap(H.fracP3);
    if (st == CPM_OK) st = upload(b, &D.runR, H.runR);
    if (st == CPM_OK) st = upload(b, &D.fracR, H.fracR);
    if (st == CPM_OK && !H.fracR.empty()) st = upload_f32(b, &D.fracR32, H.fracR);
    // keep only what export needs on the host
    std::vector<double>().swap(H.fracE);
    std::vector<double>().swap(H.fracP);
    std::vector<double>().swap(H.fracR);
    std::vector<int32_t>().swap(H.runE);
    std::vector<int32_t>().swap(H.runP);
    std::vector<int32_t>().swap(H.runR);
    // H.nbr stays on the host: cpm_set_diffusion uploads it for levels that get a coefficient
    std::vector<int32_t>().swap(H.perm);
    std::vector<int32_t>().swap(H.packed);
    std::vector<int32_t>().swap(H.packedB);
    std::vector<int32_t>().swap(H.origin);
    std::vector<double>().swap(H.fracK);
    std::vector<int32_t>().swap(H.ilist);
    std::vector<int32_t>().swap(H.nbrI);
  }
  if (st == CPM_OK) {
    b->dscal = dalloc<unsigned long long>(b, 8, &st);
    b->dcounter = dalloc<int>(b, 4, &st);
    b->dhist = dalloc<double>(b, CPM_MAX_HISTORY, &st);
    if (st == CPM_OK && hipHostMalloc((void**)&b->hpinned, 8 * sizeof(unsigned long long), 0) != hipSuccess)
      st = CPM_E_NOMEM;
  }
  if (st != CPM_OK) {
    set_error(st == CPM_E_NOMEM ? "device allocation failed" : "host to device copy failed");
    free_dev(b);
    delete b;
    return st;
  }
  (void)stream;
  *out = b;
  return CPM_OK;
}

cpm_status cpm_build_bands(int count, const cpm_surface* surfaces, const cpm_grid* grids, void* stream,
                           cpm_band* out) {
  if (count < 0 || (count > 0 && (!surfaces || !grids || !out))) {
    set_error("cpm_build_bands: invalid argument");
    return CPM_E_INVALID;
  }
  for (int k = 0; k < count; ++k) out[k] = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_error("cpm_build_bands: no current device");
    return CPM_E_HIP;
  }
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int nthr = (int)std::min<unsigned>(hw, (unsigned)std::max(count, 1));
  std::atomic<int> next{0};
  std::vector<cpm_status> sts((size_t)count, CPM_OK);
  std::vector<std::string> errs((size_t)count);
  auto worker = [&]() {
    (void)hipSetDevice(dev);
    set_host_build_threads(1);  // parallel over bands, not inside one
    for (int k = next++; k < count; k = next++) {
      sts[(size_t)k] = cpm_build_band(&surfaces[k], &grids[k], stream, &out[k]);
      if (sts[(size_t)k] != CPM_OK) errs[(size_t)k] = g_last_error;
    }
  };
  std::vector<std::thread> pool;
  for (int t = 0; t < nthr; ++t) pool.emplace_back(worker);
  for (auto& th : pool) th.join();
  for (int k = 0; k < count; ++k)
    if (sts[(size_t)k] != CPM_OK) {
      set_error("band " + std::to_string(k) + ": " + errs[(size_t)k]);
      const cpm_status st = sts[(size_t)k];
      for (int j = 0; j < count; ++j) {
        (void)cpm_band_free(out[j]);
        out[j] = nullptr;
      }
      return st;
    }
  return CPM_OK;
}

cpm_status cpm_band_free(cpm_band band) {
  if (!band) return CPM_OK;
  (void)hipDeviceSynchronize();  // work of earlier calls runs on the callers' streams
  free_dev(band);
  if (band->own) (void)hipStreamDestroy(band->own);
  delete band;
  return CPM_OK;
}

cpm_status cpm_band_levels(cpm_band band, int* levels, int* dim) {
  if (!band) {
    set_error("null band");
    return CPM_E_INVALID;
  }
  if (levels) *levels = band->L;
  if (dim) *dim = band->dim;
  return CPM_OK;
}

cpm_status cpm_band_info(cpm_band band, int level, int64_t* n, double* h, int* flags) {
  if (!band || level < 0 || level >= band->L) {
    set_error("null band or level out of range");
    return CPM_E_INVALID;
  }
  const DevLevel& D = band->dev[(size_t)level];
  if (n) *n = D.n;
  if (h) *h = D.h;
  if (flags) {
    const double lam2 = band->grid.lam2 > 0 ? band->grid.lam2 : (band->dim == 2 ? 13.0 : 17.0);
    *flags = std::sqrt(lam2) * D.h >= surface_reach(band->surf) ? CPM_BAND_BEYOND_REACH : 0;
    if (resid_subset(D)) *flags |= CPM_BAND_RESID_SUBSET;
  }
  return CPM_OK;
}

cpm_status cpm_band_export(cpm_band band, int level, int32_t* idx_host, double* cp_host) {
  if (!band || level < 0 || level >= band->L) {
    set_error("null band or level out of range");
    return CPM_E_INVALID;
  }
  const HostLevel& H = band->host[(size_t)level];
  if (idx_host) std::memcpy(idx_host, H.idx.data(), H.idx.size() * sizeof(int32_t));
  if (cp_host) std::memcpy(cp_host, H.cp.data(), H.cp.size() * sizeof(double));
  return CPM_OK;
}

static cpm_status copy_rows(int32_t* dst, const int32_t* src, int64_t n, int cols) {
  // device slot-major (cols x n) -> host row-major (n x cols)
  std::vector<int32_t> tmp((size_t)(n * cols));
  if (hipMemcpy(tmp.data(), src, tmp.size() * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) {
    set_error("device to host copy failed");
    return CPM_E_HIP;
  }
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < cols; ++c) dst[i * cols + c] = tmp[(size_t)(c * n + i)];
  return CPM_OK;
}

cpm_status cpm_band_export_stencils(cpm_band band, int level, int32_t* runE, int32_t* nbr, int32_t* runP,
                                    int32_t* runR) {
  if (!band || level < 0 || level >= band->L) {
    set_error("null band or level out of range");
    return CPM_E_INVALID;
  }
  const DevLevel& D = band->dev[(size_t)level];
  const int d = band->dim;
  const int S = d == 2 ? 4 : 16;
  const int64_t n = D.n;
  cpm_status st = CPM_OK;
  auto fetch = [&](std::vector<int32_t>& v, const int32_t* src, size_t count) -> cpm_status {
    v.resize(count);
    if (count && hipMemcpy(v.data(), src, count * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) {
      set_error("device to host copy failed");
      return CPM_E_HIP;
    }
    return CPM_OK;
  };
  if (runE) {
    // reconstruct per-node x-run starts from the stencil-ordered groups
    std::vector<int32_t> perm, packed, origin;
    if ((st = fetch(perm, D.perm, (size_t)n)) != CPM_OK) return st;
    if ((st = fetch(packed, D.packed, (size_t)n)) != CPM_OK) return st;
    if ((st = fetch(origin, D.origin, (size_t)(D.ngroups * S))) != CPM_OK) return st;
    for (int64_t k = 0; k < n; ++k) {
      const int32_t i = perm[(size_t)k];
      const int32_t gid = packed[(size_t)k] >> kXoffBits, xo = packed[(size_t)k] & ((1 << kXoffBits) - 1);
      for (int s2 = 0; s2 < S; ++s2) runE[(int64_t)i * S + s2] = origin[(size_t)gid * S + s2] + xo;
    }
  }
  if (nbr) {
    // neighbours are stored for B_interp nodes only; other rows read -2
    std::vector<int32_t> il, nb;
    if ((st = fetch(il, D.ilist, (size_t)D.m)) != CPM_OK) return st;
    if ((st = fetch(nb, D.nbrI, (size_t)(D.m * (2 * d - 2)))) != CPM_OK) return st;
    for (int64_t i = 0; i < n * 2 * d; ++i) nbr[i] = -2;
    for (int64_t k = 0; k < D.m; ++k) {
      const int32_t j = il[(size_t)k];
      nbr[(int64_t)j * 2 * d + 0] = j - 1;
      nbr[(int64_t)j * 2 * d + 1] = j + 1;
      for (int q = 0; q < 2 * d - 2; ++q) nbr[(int64_t)j * 2 * d + 2 + q] = nb[(size_t)(q * D.m + k)];
    }
  }
  if (runP && D.runP && (st = copy_rows(runP, D.runP, D.n, d == 2 ? 2 : 4)) != CPM_OK) return st;
  if (runR && D.runR && (st = copy_rows(runR, D.runR, D.n, d == 2 ? 2 : 4)) != CPM_OK) return st;
  return CPM_OK;
}

cpm_status cpm_workspace_size(cpm_band band, const cpm_params* params, size_t* bytes) {
  if (!band || !params || !bytes) {
    set_error("null argument");
    return CPM_E_INVALID;
  }
  *bytes = workspace_bytes(band, *params);
  return CPM_OK;
}

cpm_status cpm_apply(cpm_band band, int level, int dtype, double c, const void* u, void* Au, void* work,
                     void* stream) {
  if (!band || level < 0 || level >= band->L || !u || !Au || !work || !(c > 0.0) ||
      (dtype != CPM_DTYPE_F64 && dtype != CPM_DTYPE_F32)) {
    set_error("cpm_apply: invalid argument");
    return CPM_E_INVALID;
  }
  const DevLevel& D = band->dev[(size_t)level];
  StreamScope stream_scope(band);
  cpm_status st = enter(band, stream);
  if (st != CPM_OK) return st;
  const LaunchCfg lc = level_cfg(D);
  if (dtype == CPM_DTYPE_F64) {
    launch_nsum<double>(band->dim, nsum_addr(D), (const double*)u, nullptr, 1.0 / (D.h * D.h), (double*)work,
                        nullptr, lc, band->stream);
    launch_ext<double, double>(band->dim, EXT_APPLY, D.n, (const double*)work, ext_addr(D), fracK_of<double>(D),
                               nullptr, (double*)u, (double*)Au, level_delta(band, level, c), 0.0, nullptr, ext_cfg(D),
                               band->stream);
  } else {
    launch_nsum<float>(band->dim, nsum_addr(D), (const float*)u, nullptr, (float)(1.0 / (D.h * D.h)),
                       (float*)work, nullptr, lc, band->stream);
    launch_ext<float, float>(band->dim, EXT_APPLY, D.n, (const float*)work, ext_addr(D), fracK_of<float>(D), nullptr,
                             (float*)u, (float*)Au, (float)level_delta(band, level, c), 0.0f, nullptr, ext_cfg(D),
                             band->stream);
  }
  if ((st = check_launch("cpm_apply")) != CPM_OK) return st;
  return leave(band, stream);
}

cpm_status cpm_apply_pq(cpm_band band, int level, int p, double c, const double* u, double* Au, double* work,
                        void* stream) {
  if (p == 3) return cpm_apply(band, level, CPM_DTYPE_F64, c, u, Au, work, stream);
  if (!band || level < 0 || level >= band->L || !u || !Au || !work || !(c > 0.0) || p != 1) {
    set_error("cpm_apply_pq: invalid argument (p must be 1 or 3)");
    return CPM_E_INVALID;
  }
  const DevLevel& D = band->dev[(size_t)level];
  StreamScope stream_scope(band);
  cpm_status st = enter(band, stream);
  if (st != CPM_OK) return st;
  const double inv_h2 = 1.0 / (D.h * D.h);
  launch_nsum<double>(band->dim, nsum_addr(D), u, nullptr, inv_h2, work, nullptr, level_cfg(D), band->stream);
  launch_p1(band->dim, EXT_APPLY, D.n, work, u, ExtAddr{D.perm, D.packed, D.origin}, D.fracK, nullptr, nullptr, Au,
            level_delta(band, level, c), 2.0 * band->dim * inv_h2, ext_cfg(D), band->stream);
  if ((st = check_launch("cpm_apply_pq")) != CPM_OK) return st;
  return leave(band, stream);
}

cpm_status cpm_extend(cpm_band band, int level, const double* g, double* out, void* stream) {
  if (!band || level < 0 || level >= band->L || !g || !out) {
    set_error("cpm_extend: invalid argument");
    return CPM_E_INVALID;
  }
  const DevLevel& D = band->dev[(size_t)level];
  StreamScope stream_scope(band);
  cpm_status st = enter(band, stream);
  if (st != CPM_OK) return st;
  launch_ext<double, double>(band->dim, EXT_PLAIN, D.n, g, ext_addr(D), fracK_of<double>(D), nullptr, nullptr, out, 0.0, 0.0,
                             nullptr, ext_cfg(D), band->stream);
  if ((st = check_launch("cpm_extend")) != CPM_OK) return st;
  return leave(band, stream);
}

cpm_status cpm_set_diffusion(cpm_band band, int level, const double* a) {
  if (!band || level < 0 || level >= band->L) {
    set_error("cpm_set_diffusion: invalid argument");
    return CPM_E_INVALID;
  }
  if (hipStreamSynchronize(band->stream) != hipSuccess) {
    set_error("cpm_set_diffusion: synchronization failed");
    return CPM_E_HIP;
  }
  band->vc_c = NAN;
  band->coarse_c = NAN;  // the coarsest inverse changes form
  for (auto& kv : band->graphs) (void)hipGraphExecDestroy(kv.second);
  band->graphs.clear();
  if (!a) {
    for (auto& D : band->dev) {
      dev_free(band, D.acoef);
      D.acoef = nullptr;
    }
    band->vc_active = false;
    return CPM_OK;
  }
  DevLevel& D = band->dev[(size_t)level];
  const HostLevel& H = band->host[(size_t)level];
  for (int64_t i = 0; i < D.n; ++i)
    if (!(a[i] > 0.0) || !std::isfinite(a[i])) {
      set_error("cpm_set_diffusion: the coefficient must be positive and finite");
      return CPM_E_INVALID;
    }
  cpm_status st = CPM_OK;
  if (!D.acoef && !(D.acoef = dalloc<double>(band, (size_t)D.n, &st))) return st != CPM_OK ? st : CPM_E_NOMEM;
  if (hipMemcpy(D.acoef, a, (size_t)D.n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("cpm_set_diffusion: copy failed");
    return CPM_E_HIP;
  }
  if (!D.nbr && (st = upload(band, &D.nbr, H.nbr)) != CPM_OK) return st;
  bool all = true;
  for (auto& Dl : band->dev) all = all && Dl.acoef != nullptr;
  band->vc_active = all;
  return CPM_OK;
}

cpm_status cpm_vcycle(cpm_band band, const cpm_params* params, const double* f, double* u, void* work,
                      size_t work_bytes, double* relres_out, void* stream) {
  if (!band || !f || !u || !work) {
    set_error("cpm_vcycle: null argument");
    return CPM_E_INVALID;
  }
  cpm_status st = validate_params(band, params);
  if (st != CPM_OK) return st;
  if (params->precision != CPM_F64 || params->smoother == CPM_SMOOTH_LEARNED) {
    set_error("cpm_vcycle runs the double-precision cycles (Jacobi or standard relaxation) only");
    return CPM_E_INVALID;
  }
  if (work_bytes < workspace_bytes(band, *params)) {
    set_error("workspace too small");
    return CPM_E_WORKSPACE;
  }
  StreamScope stream_scope(band);
  if ((st = enter(band, stream)) != CPM_OK) return st;
  if ((st = ensure_coarse(band, params->c)) != CPM_OK) return st;
  if (standard(*params) && (st = ensure_std(band, *params)) != CPM_OK)
    return st;
  if (params->residual_mode == CPM_RESIDUAL_VERBATIM && !standard(*params) &&
      (st = ensure_verbatim(band, params->c)) != CPM_OK)
    return st;
  band->learned_active = false;
  if (relres_out) enqueue_prologue(band, *params, f, u, work, band->stream);
  enqueue_cycle(band, *params, f, u, work, band->stream);
  if ((st = check_launch("cpm_vcycle")) != CPM_OK) return st;
  if (relres_out) {
    double r0, r1;
    if ((st = read_scalars(band, &r0, &r1)) != CPM_OK) return st;
    *relres_out = r1 > 0 ? r0 / r1 : 0.0;
  }
  return leave(band, stream);
}

cpm_status cpm_solve(cpm_band band, const cpm_params* params, const double* f, double* u, void* work,
                     size_t work_bytes, double rtol, int max_cycles, cpm_stats* stats, void* stream) {
  if (!band || !f || !u || !work || max_cycles < 0) {
    set_error("cpm_solve: invalid argument");
    return CPM_E_INVALID;
  }
  cpm_status st = validate_params(band, params);
  if (st != CPM_OK) return st;
  if (work_bytes < workspace_bytes(band, *params)) {
    set_error("workspace too small");
    return CPM_E_WORKSPACE;
  }
  cpm_stats local;
  cpm_stats* S = stats ? stats : &local;
  std::memset(S, 0, sizeof(cpm_stats));
  S->fallback_cycle = -1;
  auto t0 = std::chrono::steady_clock::now();
  StreamScope stream_scope(band);
  if ((st = enter(band, stream)) != CPM_OK) return st;
  if ((st = ensure_coarse(band, params->c)) != CPM_OK) return st;
  if (standard(*params) && (st = ensure_std(band, *params)) != CPM_OK)
    return st;
  if (params->residual_mode == CPM_RESIDUAL_VERBATIM && !standard(*params) &&
      (st = ensure_verbatim(band, params->c)) != CPM_OK)
    return st;
  const cpm_params p = *params;
  band->learned_active = p.smoother == CPM_SMOOTH_LEARNED;
  enqueue_prologue(band, p, f, u, work, band->stream);
  double r0 = 0, bn = 0;
  if ((st = read_scalars(band, &r0, &bn)) != CPM_OK) return st;
  if (!std::isfinite(bn) || !std::isfinite(r0)) {
    set_error("right-hand side or initial residual is not finite");
    (void)leave(band, stream);
    return CPM_E_DIVERGED;
  }
  if (!(bn > 0)) {
    // E f = 0: the solution is u = 0
    launch_fill<double>(band->dev[0].n, u, 0.0, band->stream);
    S->relres = 0.0;
    (void)hipStreamSynchronize(band->stream);
    return leave(band, stream);
  }
  if (p.fmg) {
    enqueue_fmg(band, p, f, u, work, band->stream);
    if (p.precision != CPM_F64) {
      // the start used the workspace in its double-precision layout: the mixed cycle's
      // first residual (float32 copy in the finest level's f) is that of the start
      LevelBufs<float> B[kMaxLevels];
      double* g64 = nullptr;
      carve_levels<float>(band, work, B, &g64);
      enqueue_resid64(band, f, u, g64, B[0].f, p.c, band->stream);
    }
    if ((st = check_launch("full-multigrid start")) != CPM_OK) return st;
  }
  double prev = p.precision == CPM_F64 || p.fmg ? NAN : r0 / bn;
  st = CPM_E_NOCONV;
  // stagnation: the stopping quantity has not dropped below 0.99 of its best value for
  // kStallCycles cycles (it has reached the rounding floor of its own evaluation)
  constexpr int kStallCycles = 8;
  double best = INFINITY;
  int best_k = -1;
  bool stalled = false;
  for (int k = 0; k < max_cycles; ++k) {
    // cycles after the first start from the residual the previous one left
    const bool r_ready = k > 0;
    const std::string key = graph_key(r_ready ? "cycle_r" : "cycle", p, f, u, work, band->learned_active ? 1 : 0);
    cpm_status gs =
        graph_launch(band, key, [&](hipStream_t s) { enqueue_cycle(band, p, f, u, work, s, r_ready); });
    if (gs != CPM_OK) return gs;
    double rn = 0, un = 0;
    if ((gs = read_scalars(band, &rn, &un)) != CPM_OK) return gs;
    // standard relaxation: the relative increment ||u_k - u_{k-1}|| / ||u_k|| (Sec. 4.6)
    const bool incr = standard(p) || p.residual_mode == CPM_RESIDUAL_VERBATIM;
    const double rel = incr ? (un > 0 ? rn / un : 0.0) : rn / bn;
    if (k < CPM_MAX_HISTORY) S->relres_history[k] = rel;
    S->cycles = k + 1;
    S->relres = rel;
    if (!std::isfinite(rel)) {
      st = CPM_E_DIVERGED;
      set_error("residual is not finite");
      break;
    }
    // learned smoother: fall back to Jacobi when a cycle contracts worse than the plain method
    if (band->learned_active && std::isfinite(prev) && prev > 0 && rel / prev > band->rho_plain) {
      band->learned_active = false;
      S->fallback_cycle = k;
      best = INFINITY;  // the plain cycle starts its own record
    }
    prev = rel;
    if (rel < rtol) {
      st = CPM_OK;
      break;
    }
    if (rel < 0.99 * best) {
      best = rel;
      best_k = k;
    } else if (k - best_k >= kStallCycles) {
      stalled = true;
      break;
    }
  }
  band->learned_active = false;
  S->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st == CPM_E_NOCONV) {
    if (stalled) {
      std::ostringstream os;
      os << "stagnated: the stopping quantity has not dropped below 0.99 of its best value " << best
         << " for " << kStallCycles << " cycles (last " << S->relres << ", rtol " << rtol
         << "); a steady value is the rounding floor of its evaluation at this resolution and precision";
      set_error(os.str());
    } else {
      set_error("maximum number of cycles reached");
    }
  }
  cpm_status ls = leave(band, stream);
  return st != CPM_OK ? st : ls;
}

cpm_status cpm_run_cycles(cpm_band band, const cpm_params* params, const double* f, double* u, void* work,
                          size_t work_bytes, int cycles, int cycles_per_launch, double* relres_dev, void* stream) {
  if (!band || !f || !u || !work || !relres_dev || cycles < 0 || cycles_per_launch < 1) {
    set_error("cpm_run_cycles: invalid argument");
    return CPM_E_INVALID;
  }
  cpm_status st = validate_params(band, params);
  if (st != CPM_OK) return st;
  if (work_bytes < workspace_bytes(band, *params)) {
    set_error("workspace too small");
    return CPM_E_WORKSPACE;
  }
  StreamScope stream_scope(band);
  if ((st = enter(band, stream)) != CPM_OK) return st;
  if ((st = ensure_coarse(band, params->c)) != CPM_OK) return st;
  if (standard(*params) && (st = ensure_std(band, *params)) != CPM_OK)
    return st;
  if (params->residual_mode == CPM_RESIDUAL_VERBATIM && !standard(*params) &&
      (st = ensure_verbatim(band, params->c)) != CPM_OK)
    return st;
  const cpm_params p = *params;
  band->learned_active = p.smoother == CPM_SMOOTH_LEARNED;
  launch_fill<int>(1, band->dcounter, 0, band->stream);
  enqueue_prologue(band, p, f, u, work, band->stream);
  int done = 0;
  while (done < cycles) {
    const int k = std::min(cycles_per_launch, cycles - done);
    // every cycle but the run's first starts from the residual the previous one left
    const bool first = done == 0;
    const std::string key = graph_key(first ? "run0" : "run", p, f, u, work, k * 4 + (band->learned_active ? 1 : 0)) +
                            std::to_string((uintptr_t)relres_dev);
    st = graph_launch(band, key, [&](hipStream_t s) {
      for (int j = 0; j < k; ++j) {
        enqueue_cycle(band, p, f, u, work, s, !(first && j == 0));
        launch_record_relres(band->dscal, band->dscal + 1, relres_dev, band->dcounter, s);
      }
    });
    if (st != CPM_OK) return st;
    done += k;
  }
  band->learned_active = false;
  if ((st = check_launch("cpm_run_cycles")) != CPM_OK) return st;
  return leave(band, stream);
}

cpm_status cpm_time_kernel(cpm_band band, const cpm_params* params, int which, int level, int reps,
                           const double* f, double* u, void* work, size_t work_bytes, double* avg_us,
                           void* stream) {
  if (!band || !f || !u || !work || !avg_us || reps < 1 || level < 0 || level >= band->L || which < 0 ||
      which > 6) {
    set_error("cpm_time_kernel: invalid argument");
    return CPM_E_INVALID;
  }
  cpm_status st = validate_params(band, params);
  if (st != CPM_OK) return st;
  if (work_bytes < workspace_bytes(band, *params)) {
    set_error("workspace too small");
    return CPM_E_WORKSPACE;
  }
  if ((which == 2 && level == 0) || (which == 3 && level == band->L - 1)) {
    set_error("cpm_time_kernel: no such transfer on this level");
    return CPM_E_INVALID;
  }
  if (which == 4 && (level > 1 || !band->mlpW || !band->dev[(size_t)level].patchRow)) {
    set_error("cpm_time_kernel: no learned smoother on this level (weights unset or level >= 2)");
    return CPM_E_INVALID;
  }
  if (which == 5 && !band->dev[(size_t)level].fusedOK) {
    set_error("cpm_time_kernel: no fused-sweep addressing on this level");
    return CPM_E_INVALID;
  }
  if (which == 6 && band->dev[(size_t)level].ntiles <= 0) {
    set_error("cpm_time_kernel: no tiled-sweep tables on this level");
    return CPM_E_INVALID;
  }
  StreamScope stream_scope(band);
  if ((st = enter(band, stream)) != CPM_OK) return st;
  hipStream_t s = band->stream;
  const DevLevel& D = band->dev[(size_t)level];
  const LaunchCfg lc = level_cfg(D);
  const double delta = level_delta(band, level, params->c);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return CPM_E_HIP;
  auto run = [&](auto tag) {
    using T = decltype(tag);
    LevelBufs<T> B[kMaxLevels];
    double* g64 = nullptr;
    carve_levels<T>(band, work, B, &g64);
    T* uu = (sizeof(T) == 8 && level == 0) ? (T*)u : B[level].u;
    const T* ff = (sizeof(T) == 8 && level == 0) ? (const T*)f : B[level].f;
    if (!(sizeof(T) == 8 && level == 0)) {
      launch_fill<T>(D.n, B[level].u, (T)0.25, s);
      launch_fill<T>(D.n, B[level].f, (T)1.0, s);
    }
    launch_nsum<T>(band->dim, nsum_addr(D), uu, ff, (T)(1.0 / (D.h * D.h)), B[level].g, nullptr, lc, s);
    if (which == 4)  // residual of the current iterate (float32, as the learned sweep keeps it)
      launch_ext<T, float>(band->dim, EXT_RESID, D.n, B[level].g, ext_addr(D), fracK_of<T>(D), (const T*)nullptr,
                           uu, reinterpret_cast<float*>(B[level].r), (T)delta, (T)0, nullptr, ext_cfg(D), s);
    for (int pass = 0; pass < 2; ++pass) {  // pass 0 warms up
      const int k = pass == 0 ? 1 : reps;
      if (pass == 1) (void)hipEventRecord(e0, s);
      for (int r = 0; r < k; ++r) {
        if (which == 0) {
          launch_ext<T, T>(band->dim, EXT_SMOOTH, D.n, B[level].g, ext_addr(D), fracK_of<T>(D), nullptr, uu, (T*)nullptr,
                           (T)delta, (T)(params->omega / delta), nullptr, ext_cfg(D), s);
        } else if (which == 1) {
          launch_nsum<T>(band->dim, nsum_addr(D), uu, ff, (T)(1.0 / (D.h * D.h)), B[level].g, nullptr, lc, s);
        } else if (which == 2) {
          const DevLevel& F = band->dev[(size_t)(level - 1)];
          (void)F;
          launch_restrict<T>(band->dim, D.n, B[level - 1].g, D.runR, fracR_of<T>(D), B[level].r, nullptr, lc, s);
        } else if (which == 3) {
          launch_prolong<T>(band->dim, D.n, B[level + 1].g, D.runP, fracP_of<T>(D), B[level].r, lc, s);
        } else if (which == 6) {
          // u -> t and back, with the right-hand side f
          const bool odd = r & 1;
          launch_tile<T, T>(EXT_SMOOTH, D.n, tile_addr(D), fracT_of<T>(D), odd ? B[level].t : uu, ff, nullptr,
                            odd ? uu : B[level].t, (T)(1.0 / (D.h * D.h)), (T)delta, (T)(params->omega / delta),
                            nullptr, s);
        } else if (which == 5) {
          // u -> t and back, reading E f from g
          const bool odd = r & 1;
          launch_sweep<T>(band->dim, EXT_SMOOTH, D.n, odd ? B[level].t : uu, odd ? uu : B[level].t, B[level].g,
                          (const T*)nullptr, sweep_addr(D), fracS_of<T>(D),
                          (T)(1.0 / (D.h * D.h)), (T)delta, (T)(params->omega / delta), sweep_cfg(D), s);
        } else {
          // the update as the learned sweep runs it: residual in float32
          launch_learned_r<T, float>(band, level, reinterpret_cast<const float*>(B[level].r), uu, params->c, s);
        }
      }
      if (pass == 1) (void)hipEventRecord(e1, s);
    }
  };
  if (params->precision == CPM_F64)
    run(double(0));
  else
    run(float(0));
  if ((st = check_launch("cpm_time_kernel")) != CPM_OK) return st;
  float ms = 0.f;
  if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
    set_error("event timing failed");
    return CPM_E_HIP;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_us = 1000.0 * ms / reps;
  return leave(band, stream);
}

}  // extern "C"

namespace cpm {
template void vcycle_level<double>(const cpm_band, int, LevelBufs<double>*, const double*, const cpm_params&,
                                   hipStream_t, bool, const double*);
template void vcycle_level<float>(const cpm_band, int, LevelBufs<float>*, const float*, const cpm_params&,
                                  hipStream_t, bool, const float*);
}  // namespace cpm
