// Launchers of the gfx950 kernels (kernels.hip).  All launches are asynchronous on the
// given stream; sizes are validated by the caller.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cpm {

// Modes of the extension pass (t = E g at every node of a level).
enum ExtMode {
  EXT_SMOOTH = 0,  // u <- u + (omega/delta) r,  r = b + t - delta u   (in place on u; out = t if not null)
  EXT_RESID = 1,   // out = r = b + t - delta u
  EXT_APPLY = 2,   // out = delta u - t
  EXT_PLAIN = 3,   // out = t
};

// Launch geometry of the node-parallel kernels (set by the autotuner).
struct LaunchCfg {
  int block = 256;      // neighbour sum, transfers, gather extension
  int xcd_remap = 1;    // map consecutive tiles to the same XCD (shared L2)
  int prefetch = 0;     // LDS-staged extension: load the node's own data before the staging
};

// Stencil-ordered extension addressing of one level (see HostLevel).
struct ExtAddr {
  const int32_t* perm;
  const int32_t* packed;
  const int32_t* origin;
  // LDS staging (used when packedL is not null; stencil order only)
  const int32_t* packedL = nullptr;
  const int32_t* blkE = nullptr;
  const int32_t* gidx = nullptr;
  const int32_t* blkG = nullptr;
  const int32_t* lorg = nullptr;
  int32_t maxE = 0;
  int32_t maxG = 0;
  int32_t npt = 1;  // workgroup = kExtBlock * npt stencil slots
};

// Fused sweep addressing (stencil order): ExtAddr's perm, packed, origin plus the cross-row
// origins of the widened stencil; with packedL set, the LDS staging tables of the fused
// sweep instead (blkE, gidx, lorg of the widened rows; blkG, packedL of the extension).
struct SweepAddr {
  const int32_t* perm;
  const int32_t* packed;
  const int32_t* origin;
  const int32_t* originX;
  const int32_t* packedL = nullptr;
  const int32_t* blkE = nullptr;
  const int32_t* gidx = nullptr;
  const int32_t* blkG = nullptr;
  const int32_t* lorg = nullptr;
  int32_t maxE = 0;
  int32_t maxG = 0;
};

// Tiled sweep addressing (3-D levels with HostLevel::tileSlot ...).
struct TileAddr {
  const int32_t* slot;
  const int32_t* row;
  const int32_t* perm;
  const int32_t* loc;
  int64_t ntiles;
};

// One tiled Ruuth-Merriman pass over a level: mode EXT_SMOOTH out = u + wod r, EXT_RESID
// out = r (and ||r||_inf into nrm if not null), r = b + E(f + N u) - delta u; f, b may be
// null; frac in slot order; out must not overlap u.
template <typename T, typename TO>
void launch_tile(int mode, int64_t n, const TileAddr& a, const T* frac, const T* u, const T* f, const T* b, TO* out,
                 T inv_h2, T delta, T wod, unsigned long long* nrm, hipStream_t s);

// mode EXT_SMOOTH: uo = u + (omega/delta)(b + E f + (E N) u - delta u); EXT_RESID: uo = that
// residual.  Ef and b may be null; uo must not overlap u.
template <typename T>
void launch_sweep(int dim, int mode, int64_t n, const T* u, T* uo, const T* Ef, const T* b, const SweepAddr& a,
                  const T* frac, T inv_h2, T delta, T wod, const LaunchCfg& lc, hipStream_t s);

// g = f + N u on the m nodes of B_interp (ilist), f may be null.
// Neighbour-sum addressing: the B_interp list with its +-y, +-z neighbours, and (segOff set)
// the same list as segments of consecutive entries (see HostLevel::nsSeg), which the kernel
// reads instead of the two per-node index arrays.
struct NsumAddr {
  int64_t m;
  const int32_t* ilist;
  const int32_t* nbrI;
  const int32_t* seg = nullptr;
  const int32_t* chunkSeg = nullptr;
  const uint8_t* segOff = nullptr;
};

template <typename T>
void launch_nsum(int dim, const NsumAddr& a, const T* u, const T* f, T inv_h2, T* g, unsigned long long* zero_slot,
                 const LaunchCfg& lc, hipStream_t s);

// out/u types: the output of EXT_RESID may be float while T is double (mixed precision).
// frac: fractions in stencil order.
template <typename T, typename TO>
void launch_ext(int dim, int mode, int64_t n, const T* g, const ExtAddr& a, const T* frac, const T* b, T* u,
                TO* out, T delta, T w_over_delta, unsigned long long* nrm, const LaunchCfg& lc, hipStream_t s,
                const T* wd = nullptr);  // wd: per-node factor: EXT_SMOOTH uses it in place of
                                         // w_over_delta, EXT_RESID multiplies the residual by it

template <typename T>
void launch_restrict(int dim, int64_t nc, const T* rf, const int32_t* runR, const T* fracR, T* fc,
                     T* uc, const LaunchCfg& lc, hipStream_t s);

// uf = src + P ec (src = nullptr: in place, uf += P ec)
template <typename T>
void launch_prolong(int dim, int64_t nf, const T* ec, const int32_t* runP, const T* fracP, T* uf,
                    const LaunchCfg& lc, hipStream_t s, const T* src = nullptr);

// y = Z x with Z (n x n, leading dimension ld, double), x, y of type T.
template <typename T>
void launch_coarse_gemv(int n, const double* Z, int64_t ld, const T* x, T* y, hipStream_t s);

// Remark 3.2's operator A u = delta u - E_1 (N u) + gamma (E_1 u - E_3 u) over the extension's
// stencil-order addressing (a.perm, a.packed, a.origin), g = N u: mode EXT_APPLY out = A u,
// EXT_RESID out = b - A u, EXT_SMOOTH out = u + wd (b - A u); out must not overlap u.
void launch_p1(int dim, int mode, int64_t n, const double* g, const double* u, const ExtAddr& a, const double* frac,
               const double* b, const double* wd, double* out, double delta, double gamma, const LaunchCfg& lc,
               hipStream_t s);
// [A_c | I] for that operator on the coarsest level (n x 2n, row-major)
void launch_assemble_coarse_p1(int dim, int n, const int32_t* runE, const double* fracE, const int32_t* nbr,
                               double delta, double gamma, double inv_h2, double* M, hipStream_t s);
// red-black half-sweeps: wdR = wd on red nodes (even grid index sum), 0 elsewhere; wdB the rest
void launch_split_colours(int64_t n, const double* wd, const uint8_t* parity, double* wdR, double* wdB,
                          hipStream_t s);
// standard relaxation: wd = omega / (delta - q) per node
void launch_std_scale(int64_t n, const double* q, double delta, double omega, double* wd, hipStream_t s);
// slot[0] = max |u - p| (0 when p is null), slot[1] = max |u|, as bit patterns (atomicMax;
// the slots must be cleared first)
void launch_incr(int64_t n, const double* u, const double* p, unsigned long long* slot, hipStream_t s);
// Algorithm 4.1's printed residual r = f + N u - delta u at every node (nbr: 2d x n, -1 absent)
void launch_resid_verbatim(int dim, int64_t n, const int32_t* nbr, const double* u, const double* f, double delta,
                           double inv_h2, double* r, hipStream_t s);

// Variable diffusion coefficient (flux form): g = (f + N~ u) / D on B_interp (u, f may be
// null); D_i = c + sigma_i on every node; the coarsest level's [I - E D^{-1} N~ | E D^{-1}].
void launch_nsum_var(int dim, int64_t m, const int32_t* ilist, const int32_t* nbrI, const double* u,
                     const double* f, const double* a, const double* Dd, double inv_h2, double* g,
                     const LaunchCfg& lc, hipStream_t s);
void launch_vc_diag(int dim, int64_t n, const int32_t* nbr, const double* a, double c, double inv_h2, double* Dd,
                    hipStream_t s);
void launch_assemble_coarse_vc(int dim, int n, const int32_t* runE, const double* fracE, const int32_t* nbr,
                               const double* a, const double* Dd, double inv_h2, double* M, hipStream_t s);

// out = cubic closest-point interpolation of the coarse vector v at the n fine nodes
void launch_interp3(int dim, int64_t n, const double* v, const int32_t* runs, const double* frac, double* out,
                    hipStream_t s);

// dst = src (n elements)
template <typename T>
void launch_copy(int64_t n, const T* src, T* dst, hipStream_t s);

template <typename T>
void launch_fill(int64_t n, T* p, T v, hipStream_t s);

void launch_axpy_f32_to_f64(int64_t n, const float* e, double* u, hipStream_t s);
// y = a x, or y += a x with accumulate
template <typename T>
void launch_scale_add(int64_t n, const T* x, T a, T* y, bool accumulate, hipStream_t s);
void launch_cast_f64_to_f32(int64_t n, const double* a, float* b, hipStream_t s);
void launch_zero_u64(unsigned long long* p, int count, hipStream_t s);

// relres: hist[*counter] = nrm / bnorm, ++*counter (device-side bookkeeping for graphs)
void launch_record_relres(const unsigned long long* nrm, const unsigned long long* bnrm, double* hist,
                          int* counter, hipStream_t s);

// Dense coarse operator: M (n x 2n, row-major, ld = 2n) = [delta I - E N | E]
void launch_assemble_coarse(int dim, int n, const int32_t* runE, const double* fracE, const int32_t* nbr,
                            double delta, double inv_h2, double* M, hipStream_t s, bool identity_rhs = false);
// One Gauss-Jordan step with partial pivoting on column k of M (n x 2n).
void launch_gj_step(int n, int k, double* M, double* col, int* info, hipStream_t s);

// learned smoother
void launch_features(int dim, int64_t n, const double* r, const int32_t* nbr, const double* fracE,
                     uint16_t* X, float* scale, hipStream_t s);
template <typename T>
void launch_learned_update(int dim, int64_t n, const uint16_t* X, const float* scale, const uint16_t* W,
                           T inv_delta, T* u, hipStream_t s);
void launch_mlp_forward(int64_t m, const uint16_t* X, const uint16_t* W, float* Y, float* H, hipStream_t s);
void launch_mlp_backward(int64_t m, const uint16_t* X, const uint16_t* W, const float* H, const float* Y,
                         const float* T, float* G, hipStream_t s);

}  // namespace cpm
