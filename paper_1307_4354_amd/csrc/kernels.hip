// gfx950 kernels of the CPM V-cycle: neighbour sum, closest-point extension (cubic
// tensor-product gather) fused with Jacobi smoothing / residual / operator application and
// an exact infinity-norm reduction, closest-point restriction and prolongation, and the
// dense coarsest-level solve.
//
// All kernels are node-parallel gathers over sorted band-index lists: one lane per band
// node, no atomics on values (the only atomic is an integer max on the bit pattern of a
// non-negative double, which makes the infinity norm exact and order independent).
#include <hip/hip_runtime.h>

#include "kernels_dev.h"

namespace cpm {
namespace {

template <int D, typename T>
__global__ __launch_bounds__(kMaxBlock) void k_nsum(int64_t m, const int32_t* __restrict__ ilist,
                                                    const int32_t* __restrict__ nbrI,
                                                    const T* __restrict__ u, const T* __restrict__ f,
                                                    T inv_h2, T* __restrict__ g,
                                                    unsigned long long* __restrict__ zero_slot,
                                                    int remap) {
  if (zero_slot && blockIdx.x == 0 && threadIdx.x == 0) *zero_slot = 0ull;
  const int64_t k = tile_of_block(remap) * blockDim.x + threadIdx.x;
  if (k < m) nsum_node<D, T>(k, m, ilist, nbrI, u, f, inv_h2, g);
}

// The neighbour sum from the segment tables (nsum_seg_node).
template <int D, typename T>
__global__ __launch_bounds__(kMaxBlock) void k_nsum_seg(int64_t m, const int32_t* __restrict__ seg,
                                                        const int32_t* __restrict__ chunkSeg,
                                                        const uint8_t* __restrict__ segOff,
                                                        const T* __restrict__ u, const T* __restrict__ f,
                                                        T inv_h2, T* __restrict__ g,
                                                        unsigned long long* __restrict__ zero_slot, int remap) {
  if (zero_slot && blockIdx.x == 0 && threadIdx.x == 0) *zero_slot = 0ull;
  const int64_t k = tile_of_block(remap) * blockDim.x + threadIdx.x;
  if (k < m) nsum_seg_node<D, T>(k, seg, chunkSeg, segOff, u, f, inv_h2, g);
}

template <int D, typename T, typename TO, int MODE>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_ext(
    int64_t n, const T* __restrict__ g,
                                                   const int32_t* __restrict__ perm,
                                                   const int32_t* __restrict__ packed,
                                                   const int32_t* __restrict__ origin,
                                                   const T* __restrict__ frac,
                                                   const T* __restrict__ b, T* __restrict__ u,
                                                   TO* __restrict__ out, T delta, T wod,
                                                   unsigned long long* __restrict__ nrm, int remap,
                                                   const T* __restrict__ wd) {
  const int64_t k = tile_of_block(remap) * blockDim.x + threadIdx.x;
  unsigned long long nv = 0ull;
  if (k < n) nv = ext_node<D, T, TO, MODE>(k, n, g, perm, packed, origin, frac, b, u, out, delta, wod, wd);
  if (MODE != EXT_APPLY && nrm) block_max_atomic(nv, nrm);
}

// Fused sweep: one pass per Jacobi sweep (E f + (E N) u), stencil order, u read only.
template <int D, typename T, int MODE>
__global__ __launch_bounds__(kMaxBlock) void k_sweep(int64_t n, const T* __restrict__ u, T* __restrict__ uo,
                                                     const T* __restrict__ Ef, const T* __restrict__ b,
                                                     const int32_t* __restrict__ perm,
                                                     const int32_t* __restrict__ packed,
                                                     const int32_t* __restrict__ origin,
                                                     const int32_t* __restrict__ originX, const T* __restrict__ frac,
                                                     T inv_h2, T delta, T wod, int remap) {
  const int64_t k = tile_of_block(remap) * blockDim.x + threadIdx.x;
  if (k < n) sweep_node<D, T, MODE>(k, n, u, uo, Ef, b, perm, packed, origin, originX, frac, inv_h2, delta, wod);
}

// Fused sweep, LDS-staged: the workgroup of kExtBlock stencil slots copies the u values its
// widened stencils read into LDS, then sweeps from there.
template <int D, typename T, int MODE>
__global__ __launch_bounds__(kExtBlock) void k_sweep_lds(int64_t n, const T* __restrict__ u, T* __restrict__ uo,
                                                         const T* __restrict__ Ef, const T* __restrict__ b,
                                                         const int32_t* __restrict__ perm,
                                                         const int32_t* __restrict__ packedL,
                                                         const int32_t* __restrict__ blkE,
                                                         const int32_t* __restrict__ gidx,
                                                         const int32_t* __restrict__ blkG,
                                                         const int32_t* __restrict__ lorg, const T* __restrict__ frac,
                                                         T inv_h2, T delta, T wod, int remap, int lo_offset) {
  constexpr int SR = D == 2 ? 4 + 2 : 16 + 16;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  T* gl = (T*)smem;
  int32_t* lo = (int32_t*)(smem + lo_offset);
  const int64_t blk = tile_of_block(remap);
  ext_stage<T>(blk, u, blkE, gidx, blkG, lorg, SR, gl, lo);
  const int64_t k = blk * kExtBlock + threadIdx.x;
  if (k < n) sweep_node_lds<D, T, MODE>(k, n, gl, lo, u, uo, Ef, b, perm, packedL, frac, inv_h2, delta, wod);
}

// NPT consecutive runs of kExtBlock stencil slots per workgroup (the staging tables are built
// for workgroups of kExtBlock * NPT slots): on large levels a bigger workgroup stages fewer
// values per node, since the stencils of neighbouring nodes overlap.
template <int D, typename T, typename TO, int MODE, int NPT>
__global__ __launch_bounds__(kExtBlock) void k_ext_lds(int64_t n, const T* __restrict__ g,
                                                       const int32_t* __restrict__ perm,
                                                       const int32_t* __restrict__ packedL,
                                                       const int32_t* __restrict__ blkE,
                                                       const int32_t* __restrict__ gidx,
                                                       const int32_t* __restrict__ blkG,
                                                       const int32_t* __restrict__ lorg,
                                                       const T* __restrict__ frac, const T* __restrict__ b,
                                                       T* __restrict__ u, TO* __restrict__ out, T delta, T wod,
                                                       unsigned long long* __restrict__ nrm, int remap,
                                                       int lo_offset, const T* __restrict__ wd) {
  constexpr int S = D == 2 ? 4 : 16;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  T* gl = (T*)smem;
  int32_t* lo = (int32_t*)(smem + lo_offset);
  const int64_t blk = tile_of_block(remap);
  ext_stage<T>(blk, g, blkE, gidx, blkG, lorg, S, gl, lo);
  unsigned long long nv = 0ull;
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int64_t k = (blk * NPT + j) * kExtBlock + threadIdx.x;
    if (k < n) {
      const unsigned long long v = ext_node_lds<D, T, TO, MODE>(k, n, gl, lo, perm, packedL, frac, b, u, out, delta,
                                                                wod, wd);
      nv = v > nv ? v : nv;
    }
  }
  if (MODE != EXT_APPLY && nrm) block_max_atomic(nv, nrm);
}

// Tiled Ruuth-Merriman sweep (3-D): one workgroup per tile of kTileX x kTileY x kTileZ
// stencil bases.  The workgroup stages u over the tile's box (the stencils of its nodes
// widened by one cell on each side) and f over the stencils' box in LDS, row by row from the
// tile's row table (each box row's in-band nodes are consecutive band entries, so a row is
// one coalesced read), forms g = f + N u at every stencil node in LDS (the neighbour sum in
// the order of the two-pass sweep's neighbour-sum pass), then every node interpolates g at
// its closest point from LDS (the extension pass's order) and takes the Jacobi step:
//   MODE EXT_SMOOTH: out = u + (omega/delta) r,  EXT_RESID: out = r,  r = b + E g - delta u.
// out must not overlap u (other workgroups stage u while this one writes).  A node whose own
// grid cell lies inside the box reads its u from LDS.
constexpr int kTileStageU = (kBoxCells + kTileBlock - 1) / kTileBlock;
constexpr int kTileStageF = (kGCells + kTileBlock - 1) / kTileBlock;

template <typename T, typename TO, int MODE>
__global__ __launch_bounds__(kTileBlock) void k_tile(int64_t n, const int32_t* __restrict__ tileSlot,
                                                     const int32_t* __restrict__ tileRow,
                                                     const int32_t* __restrict__ tperm,
                                                     const int32_t* __restrict__ tloc, const T* __restrict__ frac,
                                                     const T* __restrict__ u, const T* __restrict__ f,
                                                     const T* __restrict__ b, TO* __restrict__ out, T inv_h2,
                                                     T delta, T wod, unsigned long long* __restrict__ nrm,
                                                     int remap) {
  __shared__ T U[kBoxCells];
  __shared__ T G[kGCells];
  __shared__ int2 rows[kBoxRows];
  const int64_t t = tile_of_block(remap);
  const int tid = (int)threadIdx.x;
  const int32_t s0 = tileSlot[t], s1 = tileSlot[t + 1];
  const int2* __restrict__ rt = (const int2*)tileRow + t * kBoxRows;
  for (int r = tid; r < kBoxRows; r += kTileBlock) rows[r] = rt[r];
  __syncthreads();
  // stage: every load issued before any LDS store (one memory round trip per thread)
  T uv[kTileStageU], fv[kTileStageF];
#pragma unroll
  for (int j = 0; j < kTileStageU; ++j) {
    const int e = tid + j * kTileBlock;
    uv[j] = T(0);
    if (e < kBoxCells) {
      const int2 rr = rows[e / kBoxX];
      const uint32_t below = (uint32_t)rr.y & ((1u << (e % kBoxX)) - 1u);
      if (((uint32_t)rr.y >> (e % kBoxX)) & 1u) uv[j] = u[rr.x + __popc(below)];
    }
  }
#pragma unroll
  for (int j = 0; j < kTileStageF; ++j) {
    const int g = tid + j * kTileBlock;
    fv[j] = T(0);
    if (f && g < kGCells) {
      const int x = g % kGX + 1, q = g / kGX;
      const int2 rr = rows[(q / kGY + 1) * kBoxY + q % kGY + 1];
      const uint32_t below = (uint32_t)rr.y & ((1u << x) - 1u);
      if (((uint32_t)rr.y >> x) & 1u) fv[j] = f[rr.x + __popc(below)];
    }
  }
#pragma unroll
  for (int j = 0; j < kTileStageU; ++j) {
    const int e = tid + j * kTileBlock;
    if (e < kBoxCells) U[e] = uv[j];
  }
#pragma unroll
  for (int j = 0; j < kTileStageF; ++j) {
    const int g = tid + j * kTileBlock;
    if (g < kGCells) G[g] = fv[j];
  }
  __syncthreads();
  // g = f + N u at the stencils' box cells (zeros outside the band, never read); each thread
  // updates the cells it staged
#pragma unroll
  for (int j = 0; j < kTileStageF; ++j) {
    const int g = tid + j * kTileBlock;
    if (g < kGCells) {
      const int gx = g % kGX, q = g / kGX;
      const int rr = (q / kGY + 1) * kBoxY + q % kGY + 1;
      if (!(((uint32_t)rows[rr].y >> (gx + 1)) & 1u)) continue;  // not in the band: never read
      const int c = rr * kBoxX + gx + 1;
      T sum = U[c - 1] + U[c + 1];
      sum += U[c - kBoxX];
      sum += U[c + kBoxX];
      sum += U[c - kBoxX * kBoxY];
      sum += U[c + kBoxX * kBoxY];
      T gj = sum * inv_h2;
      if (f) gj += G[g];
      G[g] = gj;
    }
  }
  __syncthreads();
  unsigned long long nv = 0ull;
  for (int32_t k = s0 + tid; k < s1; k += kTileBlock) {
    const int32_t i = tperm[k];
    const int32_t loc = tloc[k];
    T wx[4], wy[4], wz[4];
    cubic_weights<T>(frac[k], wx);
    cubic_weights<T>(frac[n + k], wy);
    cubic_weights<T>(frac[2 * n + k], wz);
    const T* gp = G + ((loc >> 10 & 31) * kGY + (loc >> 5 & 31)) * kGX + (loc & 31);
    T tv = T(0);
    // one z-plane of the stencil at a time: 16 LDS values in flight instead of 64 keeps the
    // registers at a level that lets more wavefronts share a CU
#pragma unroll 1
    for (int c = 0; c < 4; ++c) {
      T tc = T(0);
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) tc += wy[bb] * run_dot_lds(gp + (c * kGY + bb) * kGX, wx);
      tv += wz[c] * tc;
    }
    const T ui = (loc >> 30 & 1) ? U[((loc >> 25 & 31) * kBoxY + (loc >> 20 & 31)) * kBoxX + (loc >> 15 & 31)] : u[i];
    T r = tv - delta * ui;
    if (b) r += b[i];
    if (MODE == EXT_SMOOTH) {
      out[i] = (TO)(ui + wod * r);
    } else {
      if (out) out[i] = (TO)r;
      nv = nv > abs_bits((double)r) ? nv : abs_bits((double)r);
    }
  }
  if (MODE == EXT_RESID && nrm) block_max_atomic(nv, nrm);
}

// Remark 3.2's operator A u = delta u - E_1 (N u) + gamma (E_1 u - E_3 u) (linear
// interpolation in front of the Laplacian, cubic in the gamma term) at the node in stencil
// slot k: g = N u (from the neighbour-sum pass) and u are gathered through the cubic
// stencil's x-runs; the linear stencil is the inner 2^D nodes of the cubic one, with 1-D
// weights (1 - a, a) on its positions 1 and 2.  MODE EXT_APPLY: out = A u; EXT_RESID:
// out = b - A u; EXT_SMOOTH: out = u + wd (b - A u) (b may be null); out must not overlap u.
template <int D, int MODE>
__global__ __launch_bounds__(kMaxBlock) void k_p1(int64_t n, const double* __restrict__ g,
                                                  const double* __restrict__ u, const int32_t* __restrict__ perm,
                                                  const int32_t* __restrict__ packed,
                                                  const int32_t* __restrict__ origin, const double* __restrict__ frac,
                                                  const double* __restrict__ b, const double* __restrict__ wd,
                                                  double* __restrict__ out, double delta, double gamma, int remap) {
  constexpr int S = D == 2 ? 4 : 16;
  const int64_t k = tile_of_block(remap) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t i = perm[k];
  const int32_t pk = packed[k];
  const int32_t* org = origin + (int64_t)(pk >> kXoffBits) * S;
  const int32_t xo = pk & ((1 << kXoffBits) - 1);
  double wx[4], wy[4], wz[4] = {1.0, 0.0, 0.0, 0.0};
  const double ax = frac[k], ay = frac[n + k], az = D == 3 ? frac[2 * n + k] : 0.0;
  cubic_weights<double>(ax, wx);
  cubic_weights<double>(ay, wy);
  if (D == 3) cubic_weights<double>(az, wz);
  const double lx[2] = {1.0 - ax, ax}, ly[2] = {1.0 - ay, ay}, lz[2] = {1.0 - az, az};
  double t1 = 0.0, t2 = 0.0, t3 = 0.0;  // E_1 g, E_1 u, E_3 u
  constexpr int NC = D == 2 ? 1 : 4;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      const int32_t r0 = org[bb + 4 * c] + xo;
      s3 += wy[bb] * run_dot(u + r0, wx);
      if (bb == 1 || bb == 2) {
        s1 += ly[bb - 1] * (lx[0] * g[r0 + 1] + lx[1] * g[r0 + 2]);
        s2 += ly[bb - 1] * (lx[0] * u[r0 + 1] + lx[1] * u[r0 + 2]);
      }
    }
    t3 += wz[c] * s3;
    if (D == 2) {
      t1 = s1;
      t2 = s2;
    } else if (c == 1 || c == 2) {
      t1 += lz[c - 1] * s1;
      t2 += lz[c - 1] * s2;
    }
  }
  const double ui = u[i];
  const double Au = (delta * ui - t1) + gamma * (t2 - t3);
  if (MODE == EXT_APPLY) {
    out[i] = Au;
  } else {
    const double r = (b ? b[i] : 0.0) - Au;
    out[i] = MODE == EXT_RESID ? r : ui + wd[i] * r;
  }
}

// Row i of [A | I] for Remark 3.2's operator A = delta I - E_1 N + gamma (E_1 - E_3) (one lane
// per row, so no two lanes write the same row).
template <int D>
__global__ void k_assemble_coarse_p1(int n, const int32_t* __restrict__ runE, const double* __restrict__ fracE,
                                     const int32_t* __restrict__ nbr, double delta, double gamma, double inv_h2,
                                     double* __restrict__ M) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t ld = 2 * (int64_t)n;
  double* row = M + (int64_t)i * ld;
  row[i] += delta;
  row[n + i] = 1.0;
  double wx[4], wy[4], wz[4] = {1.0, 0.0, 0.0, 0.0};
  const double ax = fracE[i], ay = fracE[n + i], az = D == 3 ? fracE[2 * n + i] : 0.0;
  cubic_weights<double>(ax, wx);
  cubic_weights<double>(ay, wy);
  if (D == 3) cubic_weights<double>(az, wz);
  const double l1[3][4] = {{0.0, 1.0 - ax, ax, 0.0}, {0.0, 1.0 - ay, ay, 0.0}, {D == 3 ? 0.0 : 1.0, 1.0 - az, az, 0.0}};
  const int nruns = D == 2 ? 4 : 16;
  for (int r = 0; r < nruns; ++r) {
    const int bb = r & 3, c = r >> 2;
    const int32_t j0 = runE[(int64_t)r * n + i];
    for (int a = 0; a < 4; ++a) {
      const int32_t j = j0 + a;
      row[j] -= gamma * (wx[a] * wy[bb] * wz[c]);
      const double w1 = l1[0][a] * l1[1][bb] * (D == 3 ? l1[2][c] : 1.0);
      if (w1 == 0.0) continue;
      row[j] += gamma * w1;
      for (int q = 0; q < 2 * D; ++q) {
        const int32_t m = nbr[(int64_t)q * n + j];
        if (m >= 0) row[m] -= w1 * inv_h2;
      }
    }
  }
}

// The LDS-staged extension with the node's own data (band index, local run offsets, closest-
// point fractions, and u at the node) loaded before the barrier instead of after it: on large
// levels, where many workgroups take turns on a CU, those loads then overlap the staging's
// round trips.  With 4-byte values the staging indices go out together with the node's data
// and the staged values together with u (two dependent round trips before the barrier); with
// 8-byte values the node's data and u go first and the staging follows (measured on the
// largest level, each order is about 2 % faster for its value size).  Arithmetic as in
// k_ext_lds, term for term; NPT as there.
template <int D, typename T, typename TO, int MODE, int NPT>
__global__ __launch_bounds__(kExtBlock) void k_ext_ldsp(int64_t n, const T* __restrict__ g,
                                                        const int32_t* __restrict__ perm,
                                                        const int32_t* __restrict__ packedL,
                                                        const int32_t* __restrict__ blkE,
                                                        const int32_t* __restrict__ gidx,
                                                        const int32_t* __restrict__ blkG,
                                                        const int32_t* __restrict__ lorg,
                                                        const T* __restrict__ frac, const T* __restrict__ b,
                                                        T* __restrict__ u, TO* __restrict__ out, T delta, T wod,
                                                        unsigned long long* __restrict__ nrm, int remap,
                                                        int lo_offset, const T* __restrict__ wd) {
  constexpr int S = D == 2 ? 4 : 16;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  T* gl = (T*)smem;
  int32_t* lo = (int32_t*)(smem + lo_offset);
  const int64_t blk = tile_of_block(remap);
  int32_t i[NPT], pk[NPT];
  T fx[NPT], fy[NPT], fz[NPT], ui[NPT], bi[NPT], wdi[NPT];
  if constexpr (sizeof(T) == 4) {
    // the staging of ext_stage, split around the node's loads
    const int32_t tid = (int32_t)threadIdx.x;
    const int32_t e0 = blkE[blk], e1 = blkE[blk + 1];
    const int32_t q0 = blkG[blk] * S, q1 = blkG[blk + 1] * S;
    int32_t gi[kStageUnroll], lq[kStageUnroll];
#pragma unroll
    for (int j = 0; j < kStageUnroll; ++j) {
      const int32_t e = e0 + tid + j * kExtBlock, q = q0 + tid + j * kExtBlock;
      gi[j] = e < e1 ? gidx[e] : -1;
      lq[j] = q < q1 ? lorg[q] : 0;
    }
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
      const int64_t k = (blk * NPT + j) * kExtBlock + tid;
      i[j] = 0;
      pk[j] = 0;
      fx[j] = fy[j] = fz[j] = ui[j] = bi[j] = wdi[j] = T(0);
      if (k < n) {
        i[j] = ld_nt(perm + k);
        pk[j] = ld_nt(packedL + k);
        fx[j] = ld_nt(frac + k);
        fy[j] = ld_nt(frac + n + k);
        if (D == 3) fz[j] = ld_nt(frac + 2 * n + k);
      }
    }
    T gv[kStageUnroll];
#pragma unroll
    for (int j = 0; j < kStageUnroll; ++j) gv[j] = gi[j] >= 0 ? g[gi[j]] : T(0);
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
      const int64_t k = (blk * NPT + j) * kExtBlock + tid;
      if (k < n) {
        if (MODE != EXT_PLAIN) ui[j] = u[i[j]];
        if (b && (MODE == EXT_SMOOTH || MODE == EXT_RESID)) bi[j] = b[i[j]];
        if (wd && (MODE == EXT_SMOOTH || MODE == EXT_RESID)) wdi[j] = wd[i[j]];
      }
    }
#pragma unroll
    for (int j = 0; j < kStageUnroll; ++j) {
      const int32_t e = e0 + tid + j * kExtBlock, q = q0 + tid + j * kExtBlock;
      if (e < e1) gl[e - e0] = gv[j];
      if (q < q1) lo[q - q0] = lq[j];
    }
    for (int32_t e = e0 + tid + kStageUnroll * kExtBlock; e < e1; e += kExtBlock) gl[e - e0] = g[gidx[e]];
    for (int32_t q = q0 + tid + kStageUnroll * kExtBlock; q < q1; q += kExtBlock) lo[q - q0] = lorg[q];
    __syncthreads();
  } else {
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
      const int64_t k = (blk * NPT + j) * kExtBlock + threadIdx.x;
      i[j] = 0;
      pk[j] = 0;
      fx[j] = fy[j] = fz[j] = ui[j] = bi[j] = wdi[j] = T(0);
      if (k < n) {
        i[j] = ld_nt(perm + k);
        pk[j] = ld_nt(packedL + k);
        fx[j] = ld_nt(frac + k);
        fy[j] = ld_nt(frac + n + k);
        if (D == 3) fz[j] = ld_nt(frac + 2 * n + k);
      }
    }
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
      const int64_t k = (blk * NPT + j) * kExtBlock + threadIdx.x;
      if (k < n) {
        if (MODE != EXT_PLAIN) ui[j] = u[i[j]];
        if (b && (MODE == EXT_SMOOTH || MODE == EXT_RESID)) bi[j] = b[i[j]];
        if (wd && (MODE == EXT_SMOOTH || MODE == EXT_RESID)) wdi[j] = wd[i[j]];
      }
    }
    ext_stage<T>(blk, g, blkE, gidx, blkG, lorg, S, gl, lo);
  }
  unsigned long long nv = 0ull;
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int64_t k = (blk * NPT + j) * kExtBlock + threadIdx.x;
    if (k >= n) continue;
    const int32_t* org = lo + (pk[j] >> kXoffBits) * S;
    const T* gx = gl + (pk[j] & ((1 << kXoffBits) - 1));
    T wx[4], wy[4], wz[4];
    cubic_weights<T>(fx[j], wx);
    cubic_weights<T>(fy[j], wy);
    T t = T(0);
    if (D == 2) {
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) t += wy[bb] * run_dot_lds(gx + org[bb], wx);
    } else {
      cubic_weights<T>(fz[j], wz);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        T tc = T(0);
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) tc += wy[bb] * run_dot_lds(gx + org[bb + 4 * c], wx);
        t += wz[c] * tc;
      }
    }
    unsigned long long v = 0ull;
    if (MODE == EXT_SMOOTH) {
      T r = t - delta * ui[j];
      if (b) r += bi[j];
      u[i[j]] = ui[j] + (wd ? wdi[j] : wod) * r;
      if (out) out[i[j]] = (TO)t;
      v = abs_bits((double)r);
    } else if (MODE == EXT_RESID) {
      T r = t - delta * ui[j];
      if (b) r += bi[j];
      if (wd) r *= wdi[j];
      if (out) out[i[j]] = (TO)r;
      v = abs_bits((double)r);
    } else if (MODE == EXT_APPLY) {
      out[i[j]] = (TO)(delta * ui[j] - t);
    } else {
      if (out) out[i[j]] = (TO)t;
      v = abs_bits((double)t);
    }
    nv = v > nv ? v : nv;
  }
  if (MODE != EXT_APPLY && nrm) block_max_atomic(nv, nrm);
}

// f_c[j] = linear interpolation at cp(x_j^c) of fine-band values r_f; u_c[j] = 0
template <int D, typename T>
__global__ __launch_bounds__(kMaxBlock) void k_restrict(int64_t nc, const T* __restrict__ rf,
                                                        const int32_t* __restrict__ runR,
                                                        const T* __restrict__ fracR,
                                                        T* __restrict__ fc, T* __restrict__ uc,
                                                        int remap) {
  const int64_t j = tile_of_block(remap) * blockDim.x + threadIdx.x;
  if (j >= nc) return;
  fc[j] = linear_node<D, T>(j, nc, rf, runR, fracR);
  if (uc) uc[j] = T(0);
}

// u_f[i] += linear interpolation at cp(x_i) of coarse-band values e_c
template <int D, typename T>
__global__ __launch_bounds__(kMaxBlock) void k_prolong(int64_t nf, const T* __restrict__ ec,
                                                       const int32_t* __restrict__ runP,
                                                       const T* __restrict__ fracP, const T* src,
                                                       T* uf, int remap) {
  const int64_t i = tile_of_block(remap) * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  uf[i] = src[i] + linear_node<D, T>(i, nf, ec, runP, fracP);  // src may be uf
}

// y = Z x, one workgroup per row (coalesced row reads spread over 256 lanes), wavefront
// shuffle + LDS reduction.  Each lane issues eight row loads before it accumulates them
// (in the order j = lane, lane + 256, ...), so that the matrix streams at the memory's rate
// rather than one load latency per element.
template <typename T>
__global__ __launch_bounds__(256) void k_gemv(int n, const double* __restrict__ Z, int64_t ld,
                                              const T* __restrict__ x, T* __restrict__ y) {
  const int row = blockIdx.x;
  const double* zr = Z + (int64_t)row * ld;
  double s = 0.0;
  int j = threadIdx.x;
  for (; j + 7 * 256 < n; j += 8 * 256) {
    double z[8], xv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      z[q] = ld_nt(zr + j + q * 256);
      xv[q] = (double)x[j + q * 256];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) s += z[q] * xv[q];
  }
  for (; j < n; j += 256) s += ld_nt(zr + j) * (double)x[j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) y[row] = (T)(((part[0] + part[1]) + part[2]) + part[3]);
}

template <typename T>
__global__ void k_fill(int64_t n, T* __restrict__ p, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_axpy_f32_f64(int64_t n, const float* __restrict__ e, double* __restrict__ u) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) u[i] += (double)e[i];
}

// y = a x (ACC false) or y = y + a x (ACC true): a Jacobi step whose residual is at hand
template <typename T, bool ACC>
__global__ void k_scale_add(int64_t n, const T* __restrict__ x, T a, T* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = ACC ? y[i] + a * x[i] : a * x[i];
}

__global__ void k_cast_f64_f32(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

__global__ void k_zero_u64(unsigned long long* p, int count) {
  const int i = threadIdx.x;
  if (i < count) p[i] = 0ull;
}

__global__ void k_record_relres(const unsigned long long* nrm, const unsigned long long* bnrm,
                                double* hist, int* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double num = __longlong_as_double((long long)*nrm);
    const double den = __longlong_as_double((long long)*bnrm);
    const int k = *counter;
    hist[k] = num / den;
    *counter = k + 1;
  }
}

// Row i of [delta I - E N | E] ([delta I - E N | I] when identity_rhs; one lane per row, so no
// two lanes write the same row).
template <int D>
__global__ void k_assemble_coarse(int n, const int32_t* __restrict__ runE,
                                  const double* __restrict__ fracE, const int32_t* __restrict__ nbr,
                                  double delta, double inv_h2, double* __restrict__ M, bool identity_rhs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t ld = 2 * (int64_t)n;
  double* row = M + (int64_t)i * ld;
  row[i] += delta;
  if (identity_rhs) row[n + i] = 1.0;
  double wx[4], wy[4], wz[4] = {1.0, 0.0, 0.0, 0.0};
  cubic_weights<double>(fracE[i], wx);
  cubic_weights<double>(fracE[n + i], wy);
  if (D == 3) cubic_weights<double>(fracE[2 * n + i], wz);
  const int nruns = D == 2 ? 4 : 16;
  for (int r = 0; r < nruns; ++r) {
    const int bb = r & 3, c = r >> 2;
    const int32_t j0 = runE[(int64_t)r * n + i];
    for (int a = 0; a < 4; ++a) {
      const int32_t j = j0 + a;
      const double w = wx[a] * wy[bb] * wz[c];
      if (!identity_rhs) row[n + j] += w;
      for (int k = 0; k < 2 * D; ++k) {
        const int32_t m = nbr[(int64_t)k * n + j];
        if (m >= 0) row[m] -= w * inv_h2;
      }
    }
  }
}

// Gauss-Jordan step k, part 1 (one workgroup): partial pivot search on column k (largest
// magnitude, lowest row on ties), row swap, scaling of the pivot row, multipliers.
__global__ __launch_bounds__(1024) void k_gj_pivot(int n, int k, double* __restrict__ M,
                                                   double* __restrict__ col, int* __restrict__ info) {
  const int64_t ld = 2 * (int64_t)n;
  __shared__ double sv[1024];
  __shared__ int si[1024];
  __shared__ double piv;
  const int t = threadIdx.x, bd = blockDim.x;
  double best = -1.0;
  int bi = n;
  for (int i = k + t; i < n; i += bd) {
    const double v = fabs(M[(int64_t)i * ld + k]);
    if (v > best) {
      best = v;
      bi = i;
    }
  }
  sv[t] = best;
  si[t] = bi;
  __syncthreads();
  for (int s = bd >> 1; s > 0; s >>= 1) {
    if (t < s) {
      const double ov = sv[t + s];
      const int oi = si[t + s];
      if (ov > sv[t] || (ov == sv[t] && oi < si[t])) {
        sv[t] = ov;
        si[t] = oi;
      }
    }
    __syncthreads();
  }
  const int p = si[0];
  if (p != k && p < n) {
    for (int64_t j = t; j < ld; j += bd) {
      const double a = M[(int64_t)k * ld + j];
      M[(int64_t)k * ld + j] = M[(int64_t)p * ld + j];
      M[(int64_t)p * ld + j] = a;
    }
  }
  __syncthreads();
  if (t == 0) {
    piv = M[(int64_t)k * ld + k];
    if (piv == 0.0 && *info == 0) *info = k + 1;
  }
  __syncthreads();
  const double pv = piv;
  for (int64_t j = k + t; j < ld; j += bd) M[(int64_t)k * ld + j] = M[(int64_t)k * ld + j] / pv;
  for (int i = t; i < n; i += bd) col[i] = (i == k) ? 0.0 : M[(int64_t)i * ld + k];
}

// Gauss-Jordan step k, part 2: eliminate column k from every other row.
__global__ __launch_bounds__(256) void k_gj_elim(int n, int k, double* __restrict__ M,
                                                 const double* __restrict__ col) {
  const int64_t ld = 2 * (int64_t)n;
  const int i = blockIdx.y;
  if (i == k) return;
  const double m = col[i];
  if (m == 0.0) return;
  double* ri = M + (int64_t)i * ld;
  const double* rk = M + (int64_t)k * ld;
  for (int64_t j = k + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ld;
       j += (int64_t)gridDim.x * blockDim.x)
    ri[j] -= m * rk[j];
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

// ------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------

template <typename T>
void launch_nsum(int dim, const NsumAddr& a, const T* u, const T* f, T inv_h2, T* g, unsigned long long* zero_slot,
                 const LaunchCfg& lc, hipStream_t s) {
  const int64_t m = a.m;
  if (m <= 0) {
    if (zero_slot) k_zero_u64<<<1, 64, 0, s>>>(zero_slot, 1);
    return;
  }
  const unsigned gr = grid_for(m, lc.block);
  if (a.segOff) {
    if (dim == 2)
      k_nsum_seg<2, T><<<gr, lc.block, 0, s>>>(m, a.seg, a.chunkSeg, a.segOff, u, f, inv_h2, g, zero_slot,
                                               lc.xcd_remap);
    else
      k_nsum_seg<3, T><<<gr, lc.block, 0, s>>>(m, a.seg, a.chunkSeg, a.segOff, u, f, inv_h2, g, zero_slot,
                                               lc.xcd_remap);
    return;
  }
  if (dim == 2)
    k_nsum<2, T><<<gr, lc.block, 0, s>>>(m, a.ilist, a.nbrI, u, f, inv_h2, g, zero_slot, lc.xcd_remap);
  else
    k_nsum<3, T><<<gr, lc.block, 0, s>>>(m, a.ilist, a.nbrI, u, f, inv_h2, g, zero_slot, lc.xcd_remap);
}

template <typename T, typename TO>
void launch_ext(int dim, int mode, int64_t n, const T* g, const ExtAddr& a, const T* frac, const T* b, T* u,
                TO* out, T delta, T wod, unsigned long long* nrm, const LaunchCfg& lc, hipStream_t s, const T* wd) {
  if (n <= 0) return;
  if (a.packedL) {
    // LDS-staged path: workgroups of kExtBlock * npt stencil slots (the staging tables are
    // built for it); dynamic LDS = staged values + local-group run offsets
    const int S = dim == 2 ? 4 : 16;
    const int lo_off = (int)(((size_t)a.maxE * sizeof(T) + 15) & ~(size_t)15);
    const size_t shm = (size_t)lo_off + (size_t)a.maxG * S * sizeof(int32_t);
    const int64_t wgn = (int64_t)kExtBlock * a.npt;
    const unsigned gl = (unsigned)((n + wgn - 1) / wgn);
    const int rm = lc.xcd_remap;
#define CPM_EXTL_NPT(DD, MM, NP)                                                                           \
  if (lc.prefetch)                                                                                         \
    k_ext_ldsp<DD, T, TO, MM, NP><<<gl, kExtBlock, shm, s>>>(n, g, a.perm, a.packedL, a.blkE, a.gidx,       \
                                                             a.blkG, a.lorg, frac, b, u, out, delta, wod, nrm, \
                                                             rm, lo_off, wd);                                \
  else                                                                                                     \
    k_ext_lds<DD, T, TO, MM, NP><<<gl, kExtBlock, shm, s>>>(n, g, a.perm, a.packedL, a.blkE, a.gidx, a.blkG, \
                                                            a.lorg, frac, b, u, out, delta, wod, nrm, rm, lo_off, wd)
#define CPM_EXTL_CASE(DD, MM)      \
  if (a.npt == 4) {                \
    CPM_EXTL_NPT(DD, MM, 4);       \
  } else if (a.npt == 2) {         \
    CPM_EXTL_NPT(DD, MM, 2);       \
  } else {                         \
    CPM_EXTL_NPT(DD, MM, 1);       \
  }
    if (dim == 2) {
      switch (mode) {
        case EXT_SMOOTH: CPM_EXTL_CASE(2, EXT_SMOOTH); break;
        case EXT_RESID: CPM_EXTL_CASE(2, EXT_RESID); break;
        case EXT_APPLY: CPM_EXTL_CASE(2, EXT_APPLY); break;
        default: CPM_EXTL_CASE(2, EXT_PLAIN); break;
      }
    } else {
      switch (mode) {
        case EXT_SMOOTH: CPM_EXTL_CASE(3, EXT_SMOOTH); break;
        case EXT_RESID: CPM_EXTL_CASE(3, EXT_RESID); break;
        case EXT_APPLY: CPM_EXTL_CASE(3, EXT_APPLY); break;
        default: CPM_EXTL_CASE(3, EXT_PLAIN); break;
      }
    }
#undef CPM_EXTL_CASE
#undef CPM_EXTL_NPT
    return;
  }
  const unsigned gr = grid_for(n, lc.block);
  const int rm = lc.xcd_remap;
#define CPM_EXT_CASE(DD, MM)                                                                        \
  k_ext<DD, T, TO, MM><<<gr, lc.block, 0, s>>>(n, g, a.perm, a.packed, a.origin, frac, b, u, out, delta, wod, \
                                               nrm, rm, wd)
  if (dim == 2) {
    switch (mode) {
      case EXT_SMOOTH: CPM_EXT_CASE(2, EXT_SMOOTH); break;
      case EXT_RESID: CPM_EXT_CASE(2, EXT_RESID); break;
      case EXT_APPLY: CPM_EXT_CASE(2, EXT_APPLY); break;
      default: CPM_EXT_CASE(2, EXT_PLAIN); break;
    }
  } else {
    switch (mode) {
      case EXT_SMOOTH: CPM_EXT_CASE(3, EXT_SMOOTH); break;
      case EXT_RESID: CPM_EXT_CASE(3, EXT_RESID); break;
      case EXT_APPLY: CPM_EXT_CASE(3, EXT_APPLY); break;
      default: CPM_EXT_CASE(3, EXT_PLAIN); break;
    }
  }
#undef CPM_EXT_CASE
}

template <typename T, typename TO>
void launch_tile(int mode, int64_t n, const TileAddr& a, const T* frac, const T* u, const T* f, const T* b, TO* out,
                 T inv_h2, T delta, T wod, unsigned long long* nrm, hipStream_t s) {
  if (n <= 0 || a.ntiles <= 0) return;
  const unsigned gr = (unsigned)a.ntiles;
  if (mode == EXT_SMOOTH)
    k_tile<T, TO, EXT_SMOOTH><<<gr, kTileBlock, 0, s>>>(n, a.slot, a.row, a.perm, a.loc, frac, u, f, b, out, inv_h2,
                                                       delta, wod, nrm, 1);
  else
    k_tile<T, TO, EXT_RESID><<<gr, kTileBlock, 0, s>>>(n, a.slot, a.row, a.perm, a.loc, frac, u, f, b, out, inv_h2,
                                                      delta, wod, nrm, 1);
}

void launch_p1(int dim, int mode, int64_t n, const double* g, const double* u, const ExtAddr& a, const double* frac,
               const double* b, const double* wd, double* out, double delta, double gamma, const LaunchCfg& lc,
               hipStream_t s) {
  if (n <= 0) return;
  const unsigned gr = grid_for(n, lc.block);
#define CPM_P1_CASE(DD, MM) \
  k_p1<DD, MM><<<gr, lc.block, 0, s>>>(n, g, u, a.perm, a.packed, a.origin, frac, b, wd, out, delta, gamma, lc.xcd_remap)
  if (dim == 2) {
    if (mode == EXT_APPLY) CPM_P1_CASE(2, EXT_APPLY);
    else if (mode == EXT_RESID) CPM_P1_CASE(2, EXT_RESID);
    else CPM_P1_CASE(2, EXT_SMOOTH);
  } else {
    if (mode == EXT_APPLY) CPM_P1_CASE(3, EXT_APPLY);
    else if (mode == EXT_RESID) CPM_P1_CASE(3, EXT_RESID);
    else CPM_P1_CASE(3, EXT_SMOOTH);
  }
#undef CPM_P1_CASE
}

void launch_assemble_coarse_p1(int dim, int n, const int32_t* runE, const double* fracE, const int32_t* nbr,
                               double delta, double gamma, double inv_h2, double* M, hipStream_t s) {
  if (n <= 0) return;
  launch_fill<double>(2 * (int64_t)n * n, M, 0.0, s);
  if (dim == 2)
    k_assemble_coarse_p1<2><<<grid_for(n, 128), 128, 0, s>>>(n, runE, fracE, nbr, delta, gamma, inv_h2, M);
  else
    k_assemble_coarse_p1<3><<<grid_for(n, 128), 128, 0, s>>>(n, runE, fracE, nbr, delta, gamma, inv_h2, M);
}

template <typename T>
void launch_restrict(int dim, int64_t nc, const T* rf, const int32_t* runR, const T* fracR, T* fc,
                     T* uc, const LaunchCfg& lc, hipStream_t s) {
  if (nc <= 0) return;
  const unsigned gr = grid_for(nc, lc.block);
  if (dim == 2)
    k_restrict<2, T><<<gr, lc.block, 0, s>>>(nc, rf, runR, fracR, fc, uc, lc.xcd_remap);
  else
    k_restrict<3, T><<<gr, lc.block, 0, s>>>(nc, rf, runR, fracR, fc, uc, lc.xcd_remap);
}

template <typename T>
void launch_prolong(int dim, int64_t nf, const T* ec, const int32_t* runP, const T* fracP, T* uf,
                    const LaunchCfg& lc, hipStream_t s, const T* src) {
  if (nf <= 0) return;
  if (!src) src = uf;
  const unsigned gr = grid_for(nf, lc.block);
  if (dim == 2)
    k_prolong<2, T><<<gr, lc.block, 0, s>>>(nf, ec, runP, fracP, src, uf, lc.xcd_remap);
  else
    k_prolong<3, T><<<gr, lc.block, 0, s>>>(nf, ec, runP, fracP, src, uf, lc.xcd_remap);
}

template <typename T>
void launch_coarse_gemv(int n, const double* Z, int64_t ld, const T* x, T* y, hipStream_t s) {
  if (n <= 0) return;
  k_gemv<T><<<(unsigned)n, 256, 0, s>>>(n, Z, ld, x, y);
}

template <typename T>
__global__ void k_copy(int64_t n, const T* __restrict__ a, T* __restrict__ b) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

template <typename T>
void launch_copy(int64_t n, const T* src, T* dst, hipStream_t s) {
  if (n > 0) k_copy<T><<<grid_for(n, 256), 256, 0, s>>>(n, src, dst);
}

template <typename T>
void launch_fill(int64_t n, T* p, T v, hipStream_t s) {
  if (n <= 0) return;
  int64_t gr = (n + 255) / 256;
  if (gr > 65536) gr = 65536;
  k_fill<T><<<(unsigned)gr, 256, 0, s>>>(n, p, v);
}

template <typename T>
void launch_scale_add(int64_t n, const T* x, T a, T* y, bool accumulate, hipStream_t s) {
  if (n <= 0) return;
  if (accumulate)
    k_scale_add<T, true><<<grid_for(n, 256), 256, 0, s>>>(n, x, a, y);
  else
    k_scale_add<T, false><<<grid_for(n, 256), 256, 0, s>>>(n, x, a, y);
}

void launch_axpy_f32_to_f64(int64_t n, const float* e, double* u, hipStream_t s) {
  if (n > 0) k_axpy_f32_f64<<<grid_for(n, 256), 256, 0, s>>>(n, e, u);
}

void launch_cast_f64_to_f32(int64_t n, const double* a, float* b, hipStream_t s) {
  if (n > 0) k_cast_f64_f32<<<grid_for(n, 256), 256, 0, s>>>(n, a, b);
}

void launch_zero_u64(unsigned long long* p, int count, hipStream_t s) {
  k_zero_u64<<<1, 64, 0, s>>>(p, count);
}

void launch_record_relres(const unsigned long long* nrm, const unsigned long long* bnrm, double* hist,
                          int* counter, hipStream_t s) {
  k_record_relres<<<1, 64, 0, s>>>(nrm, bnrm, hist, counter);
}

void launch_assemble_coarse(int dim, int n, const int32_t* runE, const double* fracE, const int32_t* nbr,
                            double delta, double inv_h2, double* M, hipStream_t s, bool identity_rhs) {
  launch_fill<double>(2 * (int64_t)n * n, M, 0.0, s);
  if (dim == 2)
    k_assemble_coarse<2><<<grid_for(n, 128), 128, 0, s>>>(n, runE, fracE, nbr, delta, inv_h2, M, identity_rhs);
  else
    k_assemble_coarse<3><<<grid_for(n, 128), 128, 0, s>>>(n, runE, fracE, nbr, delta, inv_h2, M, identity_rhs);
}

void launch_gj_step(int n, int k, double* M, double* col, int* info, hipStream_t s) {
  k_gj_pivot<<<1, 1024, 0, s>>>(n, k, M, col, info);
  const int64_t cols = 2 * (int64_t)n - k;
  unsigned gx = grid_for(cols, 256);
  if (gx > 16) gx = 16;
  k_gj_elim<<<dim3(gx, (unsigned)n), 256, 0, s>>>(n, k, M, col);
}

template <typename T>
void launch_sweep(int dim, int mode, int64_t n, const T* u, T* uo, const T* Ef, const T* b, const SweepAddr& a,
                  const T* frac, T inv_h2, T delta, T wod, const LaunchCfg& lc, hipStream_t s) {
  if (n <= 0) return;
  if (a.packedL) {
    // LDS-staged: fixed workgroup of kExtBlock stencil slots; dynamic LDS = staged values +
    // the local groups' row offsets
    const int SR = dim == 2 ? 6 : 32;
    const int lo_off = (int)(((size_t)a.maxE * sizeof(T) + 15) & ~(size_t)15);
    const size_t shm = (size_t)lo_off + (size_t)a.maxG * SR * sizeof(int32_t);
    const unsigned gl = (unsigned)((n + kExtBlock - 1) / kExtBlock);
    const int rm = lc.xcd_remap;
#define CPM_SWEEPL_CASE(DD, MM)                                                                                   \
  k_sweep_lds<DD, T, MM><<<gl, kExtBlock, shm, s>>>(n, u, uo, Ef, b, a.perm, a.packedL, a.blkE, a.gidx, a.blkG, \
                                                    a.lorg, frac, inv_h2, delta, wod, rm, lo_off)
    if (dim == 2) {
      if (mode == EXT_SMOOTH) CPM_SWEEPL_CASE(2, EXT_SMOOTH); else CPM_SWEEPL_CASE(2, EXT_RESID);
    } else {
      if (mode == EXT_SMOOTH) CPM_SWEEPL_CASE(3, EXT_SMOOTH); else CPM_SWEEPL_CASE(3, EXT_RESID);
    }
#undef CPM_SWEEPL_CASE
    return;
  }
  const unsigned gr = grid_for(n, lc.block);
  const int rm = lc.xcd_remap;
#define CPM_SWEEP_CASE(DD, MM)                                                                                  \
  k_sweep<DD, T, MM><<<gr, lc.block, 0, s>>>(n, u, uo, Ef, b, a.perm, a.packed, a.origin, a.originX, frac, inv_h2, \
                                             delta, wod, rm)
  if (dim == 2) {
    if (mode == EXT_SMOOTH) CPM_SWEEP_CASE(2, EXT_SMOOTH); else CPM_SWEEP_CASE(2, EXT_RESID);
  } else {
    if (mode == EXT_SMOOTH) CPM_SWEEP_CASE(3, EXT_SMOOTH); else CPM_SWEEP_CASE(3, EXT_RESID);
  }
#undef CPM_SWEEP_CASE
}

__global__ void k_std_scale(int64_t n, const double* __restrict__ q, double dc, double omega,
                            double* __restrict__ wd) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) wd[i] = omega / (dc - q[i]);
}

void launch_std_scale(int64_t n, const double* q, double delta, double omega, double* wd, hipStream_t s) {
  if (n > 0) k_std_scale<<<grid_for(n, 256), 256, 0, s>>>(n, q, delta, omega, wd);
}

// slot[0] = max |u - p| and slot[1] = max |u| (bit patterns, atomicMax); p may be null
__global__ __launch_bounds__(256) void k_incr(int64_t n, const double* __restrict__ u, const double* __restrict__ p,
                                              unsigned long long* __restrict__ slot) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  unsigned long long d = 0ull, m = 0ull;
  if (i < n) {
    m = abs_bits(u[i]);
    if (p) d = abs_bits(u[i] - p[i]);
  }
  block_max_atomic(d, slot);
  block_max_atomic(m, slot + 1);
}

__global__ void k_split_colours(int64_t n, const double* __restrict__ wd, const uint8_t* __restrict__ parity,
                                double* __restrict__ wdR, double* __restrict__ wdB) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool red = parity[i] == 0;
  wdR[i] = red ? wd[i] : 0.0;
  wdB[i] = red ? 0.0 : wd[i];
}

void launch_split_colours(int64_t n, const double* wd, const uint8_t* parity, double* wdR, double* wdB,
                          hipStream_t s) {
  if (n > 0) k_split_colours<<<grid_for(n, 256), 256, 0, s>>>(n, wd, parity, wdR, wdB);
}

void launch_incr(int64_t n, const double* u, const double* p, unsigned long long* slot, hipStream_t s) {
  if (n > 0) k_incr<<<grid_for(n, 256), 256, 0, s>>>(n, u, p, slot);
}

// The residual of Algorithm 4.1 step 2 as printed: r = f - (cI - L) u = f + N u - delta u at
// every node, neighbours outside the band dropped.
template <int D>
__global__ __launch_bounds__(256) void k_resid_verbatim(int64_t n, const int32_t* __restrict__ nbr,
                                                        const double* __restrict__ u, const double* __restrict__ f,
                                                        double delta, double inv_h2, double* __restrict__ r) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double sum = 0.0;
#pragma unroll
  for (int q = 0; q < 2 * D; ++q) {
    const int32_t j = nbr[q * n + i];
    if (j >= 0) sum += u[j];
  }
  r[i] = (f[i] + sum * inv_h2) - delta * u[i];
}

void launch_resid_verbatim(int dim, int64_t n, const int32_t* nbr, const double* u, const double* f, double delta,
                           double inv_h2, double* r, hipStream_t s) {
  if (n <= 0) return;
  if (dim == 2)
    k_resid_verbatim<2><<<grid_for(n, 256), 256, 0, s>>>(n, nbr, u, f, delta, inv_h2, r);
  else
    k_resid_verbatim<3><<<grid_for(n, 256), 256, 0, s>>>(n, nbr, u, f, delta, inv_h2, r);
}

template <int D, typename T>
__global__ __launch_bounds__(kMaxBlock) void k_nsum_var(int64_t m, const int32_t* __restrict__ ilist,
                                                        const int32_t* __restrict__ nbrI, const T* __restrict__ u,
                                                        const T* __restrict__ f, const T* __restrict__ a,
                                                        const T* __restrict__ Dd, T inv_h2, T* __restrict__ g,
                                                        int remap) {
  const int64_t k = tile_of_block(remap) * blockDim.x + threadIdx.x;
  if (k < m) nsum_var_node<D, T>(k, m, ilist, nbrI, u, f, a, Dd, inv_h2, g);
}

void launch_nsum_var(int dim, int64_t m, const int32_t* ilist, const int32_t* nbrI, const double* u,
                     const double* f, const double* a, const double* Dd, double inv_h2, double* g,
                     const LaunchCfg& lc, hipStream_t s) {
  if (m <= 0) return;
  const unsigned gr = grid_for(m, lc.block);
  if (dim == 2)
    k_nsum_var<2, double><<<gr, lc.block, 0, s>>>(m, ilist, nbrI, u, f, a, Dd, inv_h2, g, lc.xcd_remap);
  else
    k_nsum_var<3, double><<<gr, lc.block, 0, s>>>(m, ilist, nbrI, u, f, a, Dd, inv_h2, g, lc.xcd_remap);
}

// D_i = c + sigma_i, sigma_i = sum over the 2d axis directions of (a_i + a_q) / 2 / h^2, a
// missing neighbour counting with a_i (so that a = 1 gives the 2d/h^2 of every row of L).
__global__ void k_vc_diag(int64_t n, int nq, const int32_t* __restrict__ nbr, const double* __restrict__ a,
                          double c, double inv_h2, double* __restrict__ Dd) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double ai = a[i];
  double s = 0.0;
  for (int q = 0; q < nq; ++q) {
    const int32_t j = nbr[(int64_t)q * n + i];
    s += j >= 0 ? 0.5 * (ai + a[j]) : ai;
  }
  Dd[i] = c + s * inv_h2;
}

void launch_vc_diag(int dim, int64_t n, const int32_t* nbr, const double* a, double c, double inv_h2, double* Dd,
                    hipStream_t s) {
  if (n > 0) k_vc_diag<<<grid_for(n, 256), 256, 0, s>>>(n, 2 * dim, nbr, a, c, inv_h2, Dd);
}

// Row i of [I - E D^{-1} N~ | E D^{-1}] on the coarsest level (variable coefficient): the
// fixed-point equation of its Ruuth-Merriman smoother.  One lane per row.
template <int D>
__global__ void k_assemble_coarse_vc(int n, const int32_t* __restrict__ runE, const double* __restrict__ fracE,
                                     const int32_t* __restrict__ nbr, const double* __restrict__ a,
                                     const double* __restrict__ Dd, double inv_h2, double* __restrict__ M) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t ld = 2 * (int64_t)n;
  double* row = M + (int64_t)i * ld;
  row[i] += 1.0;
  double wx[4], wy[4], wz[4] = {1.0, 0.0, 0.0, 0.0};
  cubic_weights<double>(fracE[i], wx);
  cubic_weights<double>(fracE[n + i], wy);
  if (D == 3) cubic_weights<double>(fracE[2 * n + i], wz);
  const int nruns = D == 2 ? 4 : 16;
  for (int r = 0; r < nruns; ++r) {
    const int bb = r & 3, c = r >> 2;
    const int32_t j0 = runE[(int64_t)r * n + i];
    for (int q = 0; q < 4; ++q) {
      const int32_t j = j0 + q;
      const double w = wx[q] * wy[bb] * wz[c] / Dd[j];
      row[n + j] += w;
      for (int k = 0; k < 2 * D; ++k) {
        const int32_t mm = nbr[(int64_t)k * n + j];
        if (mm >= 0) row[mm] -= w * 0.5 * (a[j] + a[mm]) * inv_h2;
      }
    }
  }
}

void launch_assemble_coarse_vc(int dim, int n, const int32_t* runE, const double* fracE, const int32_t* nbr,
                               const double* a, const double* Dd, double inv_h2, double* M, hipStream_t s) {
  launch_fill<double>(2 * (int64_t)n * n, M, 0.0, s);
  if (dim == 2)
    k_assemble_coarse_vc<2><<<grid_for(n, 128), 128, 0, s>>>(n, runE, fracE, nbr, a, Dd, inv_h2, M);
  else
    k_assemble_coarse_vc<3><<<grid_for(n, 128), 128, 0, s>>>(n, runE, fracE, nbr, a, Dd, inv_h2, M);
}

template <int D>
__global__ __launch_bounds__(256) void k_interp3(int64_t n, const double* __restrict__ v,
                                                 const int32_t* __restrict__ runs, const double* __restrict__ frac,
                                                 double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = cubic_node<D, double>(i, n, v, runs, frac);
}

void launch_interp3(int dim, int64_t n, const double* v, const int32_t* runs, const double* frac, double* out,
                    hipStream_t s) {
  if (n <= 0) return;
  if (dim == 2)
    k_interp3<2><<<grid_for(n, 256), 256, 0, s>>>(n, v, runs, frac, out);
  else
    k_interp3<3><<<grid_for(n, 256), 256, 0, s>>>(n, v, runs, frac, out);
}

// explicit instantiations
template void launch_nsum<double>(int, const NsumAddr&, const double*, const double*, double, double*,
                                  unsigned long long*, const LaunchCfg&, hipStream_t);
template void launch_nsum<float>(int, const NsumAddr&, const float*, const float*, float, float*,
                                 unsigned long long*, const LaunchCfg&, hipStream_t);
template void launch_ext<double, double>(int, int, int64_t, const double*, const ExtAddr&, const double*,
                                         const double*, double*, double*, double, double,
                                         unsigned long long*, const LaunchCfg&, hipStream_t, const double*);
template void launch_ext<double, float>(int, int, int64_t, const double*, const ExtAddr&, const double*,
                                        const double*, double*, float*, double, double,
                                        unsigned long long*, const LaunchCfg&, hipStream_t, const double*);
template void launch_ext<float, float>(int, int, int64_t, const float*, const ExtAddr&, const float*,
                                       const float*, float*, float*, float, float, unsigned long long*,
                                       const LaunchCfg&, hipStream_t, const float*);
template void launch_sweep<double>(int, int, int64_t, const double*, double*, const double*, const double*,
                                   const SweepAddr&, const double*, double, double, double, const LaunchCfg&,
                                   hipStream_t);
template void launch_sweep<float>(int, int, int64_t, const float*, float*, const float*, const float*,
                                  const SweepAddr&, const float*, float, float, float, const LaunchCfg&, hipStream_t);
template void launch_tile<double, double>(int, int64_t, const TileAddr&, const double*, const double*, const double*,
                                          const double*, double*, double, double, double, unsigned long long*,
                                          hipStream_t);
template void launch_tile<double, float>(int, int64_t, const TileAddr&, const double*, const double*, const double*,
                                         const double*, float*, double, double, double, unsigned long long*,
                                         hipStream_t);
template void launch_tile<float, float>(int, int64_t, const TileAddr&, const float*, const float*, const float*,
                                        const float*, float*, float, float, float, unsigned long long*, hipStream_t);
template void launch_restrict<double>(int, int64_t, const double*, const int32_t*, const double*, double*,
                                      double*, const LaunchCfg&, hipStream_t);
template void launch_restrict<float>(int, int64_t, const float*, const int32_t*, const float*, float*,
                                     float*, const LaunchCfg&, hipStream_t);
template void launch_prolong<double>(int, int64_t, const double*, const int32_t*, const double*, double*,
                                     const LaunchCfg&, hipStream_t, const double*);
template void launch_prolong<float>(int, int64_t, const float*, const int32_t*, const float*, float*,
                                    const LaunchCfg&, hipStream_t, const float*);
template void launch_coarse_gemv<double>(int, const double*, int64_t, const double*, double*, hipStream_t);
template void launch_coarse_gemv<float>(int, const double*, int64_t, const float*, float*, hipStream_t);
template void launch_scale_add<double>(int64_t, const double*, double, double*, bool, hipStream_t);
template void launch_scale_add<float>(int64_t, const float*, float, float*, bool, hipStream_t);
template void launch_copy<double>(int64_t, const double*, double*, hipStream_t);
template void launch_copy<float>(int64_t, const float*, float*, hipStream_t);
template void launch_fill<double>(int64_t, double*, double, hipStream_t);
template void launch_fill<float>(int64_t, float*, float, hipStream_t);
template void launch_fill<int>(int64_t, int*, int, hipStream_t);

}  // namespace cpm
