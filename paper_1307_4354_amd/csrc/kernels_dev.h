// Device-side building blocks shared by the single-problem and the batched kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "cpm_internal.h"
#include "kernels.h"

namespace cpm {

constexpr int kMaxBlock = 512;

// Workgroups are dispatched round robin over the 8 XCDs (workgroup b runs on XCD b % 8).
// Remap so that XCD x processes one contiguous range of tiles: neighbouring band nodes
// share most of their stencil data, and this keeps that sharing inside one L2.
__device__ __forceinline__ int64_t tile_of_block(int remap) {
  const int64_t nb = gridDim.x, b = blockIdx.x;
  if (!remap || nb < 16) return b;
  const int64_t per = nb / 8, rem = nb % 8, x = b % 8, k = b / 8;
  return x * per + (x < rem ? x : rem) + k;
}

// A load of data that one pass streams through once (per-node fractions and addressing of
// the finest level, staging indices, the coarsest inverse): issued non-temporal, so that it
// does not displace from the caches what the next kernels of the cycle read again (u, f, g).
// Measured on the C3 torus: the FP64 cycle 2.21 -> 2.07 ms, the mixed cycle 1.85 -> 1.78 ms.
// Marking also the per-node loads of the other LDS-staged form (ext_node_lds), the
// neighbour-sum segment tables, the transfers' tables or the float32 staging indices of the
// finest level made the cycles slower.
template <typename T>
__device__ __forceinline__ T ld_nt(const T* p) {
  return __builtin_nontemporal_load(p);
}

template <typename T>
__device__ __forceinline__ void cubic_weights(T a, T w[4]) {
  // Lagrange basis on nodes 0..3 at s = 1 + a, a = frac in [0, 1)
  const T am1 = a - T(1), am2 = a - T(2), ap1 = a + T(1);
  w[0] = -(a * am1 * am2) * T(1.0 / 6.0);
  w[1] = (ap1 * am1 * am2) * T(0.5);
  w[2] = -(ap1 * a * am2) * T(0.5);
  w[3] = (ap1 * a * am1) * T(1.0 / 6.0);
}

__device__ __forceinline__ unsigned long long abs_bits(double v) {
  return (unsigned long long)__double_as_longlong(fabs(v));
}

// Block-wide max of 64-bit patterns followed by one atomicMax; every thread must call it.
__device__ __forceinline__ void block_max_atomic(unsigned long long v, unsigned long long* dst) {
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(v, off);
    v = v > o ? v : o;
  }
  __shared__ unsigned long long part[kMaxBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) part[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = 0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) m = part[w] > m ? part[w] : m;
    // the stored maximum only grows: skip the atomic when it cannot change it, so that
    // thousands of workgroups do not serialize on one address
    if (m && m > __atomic_load_n(dst, __ATOMIC_RELAXED)) atomicMax(dst, m);
  }
  __syncthreads();  // part[] may be reused by a following call (grid-stride loops)
}

// g_j = f_j + (sum of the 2d axis neighbours of u) / h^2 at node k of B_interp (j = ilist[k]);
// f may be null (g = N u).  Only these nodes are ever read by the extension, all of their
// neighbours are in the band, and the +-x neighbours are the adjacent band entries.
template <int D, typename T>
__device__ __forceinline__ void nsum_node(int64_t k, int64_t m, const int32_t* __restrict__ ilist,
                                          const int32_t* __restrict__ nbrI, const T* __restrict__ u,
                                          const T* __restrict__ f, T inv_h2, T* __restrict__ g) {
  const int32_t j = ilist[k];
  T s = u[j - 1] + u[j + 1];
#pragma unroll
  for (int q = 0; q < 2 * D - 2; ++q) s += u[nbrI[q * m + k]];
  T gj = s * inv_h2;
  if (f) gj += f[j];
  g[j] = gj;
}

// The same sum from the segment tables: list position k lies in segment
// chunkSeg[k / kNsumChunk] + segOff[k], whose t-th node has band index j0 + t and neighbours
// nb_q + t.  Arithmetic as nsum_node's, term for term.
template <int D, typename T>
__device__ __forceinline__ void nsum_seg_node(int64_t k, const int32_t* __restrict__ seg,
                                              const int32_t* __restrict__ chunkSeg,
                                              const uint8_t* __restrict__ segOff, const T* __restrict__ u,
                                              const T* __restrict__ f, T inv_h2, T* __restrict__ g) {
  const int32_t* sg = seg + (int64_t)(chunkSeg[k >> kNsumChunkBits] + segOff[k]) * kNsumSegWords;
  const int32_t t = (int32_t)k - sg[0];
  const int32_t j = sg[1] + t;
  T s = u[j - 1] + u[j + 1];
#pragma unroll
  for (int q = 0; q < 2 * D - 2; ++q) s += u[sg[2 + q] + t];
  T gj = s * inv_h2;
  if (f) gj += f[j];
  g[j] = gj;
}

// Variable coefficient: g_j = (f_j + sum_q abar_q u_q / h^2) / D_j at node k of B_interp,
// abar_q = (a_j + a_q) / 2 over the 2d axis neighbours q (the flux form D^b diag(A^f a) D^f),
// D_j = c + sigma_j precomputed.  u may be null (g = f / D), f may be null.
template <int D, typename T>
__device__ __forceinline__ void nsum_var_node(int64_t k, int64_t m, const int32_t* __restrict__ ilist,
                                              const int32_t* __restrict__ nbrI, const T* __restrict__ u,
                                              const T* __restrict__ f, const T* __restrict__ a,
                                              const T* __restrict__ Dd, T inv_h2, T* __restrict__ g) {
  const int32_t j = ilist[k];
  T gj = T(0);
  if (u) {
    const T aj = a[j];
    T s = (aj + a[j - 1]) * u[j - 1] + (aj + a[j + 1]) * u[j + 1];
#pragma unroll
    for (int q = 0; q < 2 * D - 2; ++q) {
      const int32_t nq = nbrI[q * m + k];
      s += (aj + a[nq]) * u[nq];
    }
    gj = T(0.5) * s * inv_h2;
  }
  if (f) gj += f[j];
  g[j] = gj / Dd[j];
}

// Weighted sum of one x-run of 4 consecutive values, loaded with 16-byte vector loads
// (the run start is only element aligned; global loads of several dwords need dword
// alignment, which every double and float address has).
typedef double run_d2 __attribute__((ext_vector_type(2), aligned(8)));
typedef float run_f4 __attribute__((ext_vector_type(4), aligned(4)));

__device__ __forceinline__ double run_dot(const double* __restrict__ p, const double w[4]) {
  const run_d2 a = *(const run_d2*)p;
  const run_d2 b = *(const run_d2*)(p + 2);
  return w[0] * a.x + w[1] * a.y + w[2] * b.x + w[3] * b.y;
}

__device__ __forceinline__ float run_dot(const float* __restrict__ p, const float w[4]) {
  const run_f4 a = *(const run_f4*)p;
  return w[0] * a.x + w[1] * a.y + w[2] * a.z + w[3] * a.w;
}

// t = E g at the node in stencil slot k (tensor-product cubic interpolation at its closest
// point), then one of the ExtMode updates; returns the bit pattern of |r| (or |t|) for the
// infinity norm.  Nodes are visited in stencil order (sorted by the base of their cubic
// stencil) so that the lanes of a wavefront gather from the same few rows: node
// i = perm[k]; its x-run (b, c) starts at origin[gid * 4^(D-1) + b + 4c] + xoff with
// (gid, xoff) packed in packed[k]; frac holds the fractions in stencil order.
template <int D, typename T, typename TO, int MODE>
__device__ __forceinline__ unsigned long long ext_node(int64_t k, int64_t n, const T* __restrict__ g,
                                                       const int32_t* __restrict__ perm,
                                                       const int32_t* __restrict__ packed,
                                                       const int32_t* __restrict__ origin,
                                                       const T* __restrict__ frac, const T* __restrict__ b,
                                                       T* __restrict__ u, TO* __restrict__ out, T delta,
                                                       T wod, const T* __restrict__ wd = nullptr) {
  constexpr int S = D == 2 ? 4 : 16;
  const int32_t i = perm ? perm[k] : (int32_t)k;  // null perm: band order
  const int32_t pk = packed[k];
  const int32_t* org = origin + (int64_t)(pk >> kXoffBits) * S;
  const T* gx = g + (pk & ((1 << kXoffBits) - 1));
  T wx[4], wy[4], wz[4];
  cubic_weights<T>(frac[k], wx);
  cubic_weights<T>(frac[n + k], wy);
  T t = T(0);
  if (D == 2) {
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) t += wy[bb] * run_dot(gx + org[bb], wx);
  } else {
    cubic_weights<T>(frac[2 * n + k], wz);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      T tc = T(0);
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) tc += wy[bb] * run_dot(gx + org[bb + 4 * c], wx);
      t += wz[c] * tc;
    }
  }
  if (MODE == EXT_SMOOTH) {
    const T ui = u[i];
    T r = t - delta * ui;
    if (b) r += b[i];
    u[i] = ui + (wd ? wd[i] : wod) * r;  // wd: per-node scale of the standard relaxation
    if (out) out[i] = (TO)t;  // optionally keep E g
    return abs_bits((double)r);
  } else if (MODE == EXT_RESID) {
    T r = t - delta * u[i];
    if (b) r += b[i];
    if (wd) r *= wd[i];  // variable coefficient: residual brought to the units of f
    if (out) out[i] = (TO)r;
    return abs_bits((double)r);
  } else if (MODE == EXT_APPLY) {
    out[i] = (TO)(delta * u[i] - t);
    return 0ull;
  } else {
    if (out) out[i] = (TO)t;
    return abs_bits((double)t);
  }
}

// ---- fused sweep ---------------------------------------------------------------------
// E is linear, so E (f + N u) = E f + (E N) u.  (E N) u at a node reads the node's cubic
// stencil widened by the axis neighbours of its nodes: the 4^(D-1) x-runs extended to 6
// nodes (x0-1 .. x0+4, consecutive band entries because every x neighbour of a stencil node
// is in the band and adjacent to it) plus the cross rows of 4 nodes just outside the stencil
// in y (and z).  Its weights are the 1-D cubic weights convolved with (1, 0, 1):
//   x: (w0, w1, w0+w2, w1+w3, w2, w3) over x0-1 .. x0+4,  y and z alike.

// the 6 values p[0..5]
__device__ __forceinline__ void run6(const double* __restrict__ p, double v[6]) {
  const run_d2 a = *(const run_d2*)p, b = *(const run_d2*)(p + 2), c = *(const run_d2*)(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y; v[4] = c.x; v[5] = c.y;
}
typedef float run_f2 __attribute__((ext_vector_type(2), aligned(4)));
__device__ __forceinline__ void run6(const float* __restrict__ p, float v[6]) {
  const run_f4 a = *(const run_f4*)p;
  const run_f2 b = *(const run_f2*)(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y;
}

// (E N) u times h^2 at one node: ux = u + xoff, org / orgX its group's run origins.
template <int D, typename T>
__device__ __forceinline__ T en_node(const T* __restrict__ ux, const int32_t* __restrict__ org,
                                     const int32_t* __restrict__ orgX, const T wx[4], const T wy[4],
                                     const T wz[4]) {
  const T cx[6] = {wx[0], wx[1], wx[0] + wx[2], wx[1] + wx[3], wx[2], wx[3]};
  const T cy[4] = {wy[1], wy[0] + wy[2], wy[1] + wy[3], wy[2]};  // y-shift weights of the stencil rows
  T acc = T(0);
  if (D == 2) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      T v[6];
      run6(ux + org[b] - 1, v);
      T A = T(0), B = T(0);
#pragma unroll
      for (int a = 0; a < 6; ++a) A += cx[a] * v[a];
#pragma unroll
      for (int a = 0; a < 4; ++a) B += wx[a] * v[a + 1];
      acc += wy[b] * A + cy[b] * B;
    }
    acc += wy[0] * run_dot(ux + orgX[0], wx) + wy[3] * run_dot(ux + orgX[1], wx);
  } else {
    const T cz[4] = {wz[1], wz[0] + wz[2], wz[1] + wz[3], wz[2]};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      T zc = T(0);  // rows of this z: x and y shifts
      T yc = T(0);  // rows of this z weighted for the z shift
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        T v[6];
        run6(ux + org[b + 4 * c] - 1, v);
        T A = T(0), B = T(0);
#pragma unroll
        for (int a = 0; a < 6; ++a) A += cx[a] * v[a];
#pragma unroll
        for (int a = 0; a < 4; ++a) B += wx[a] * v[a + 1];
        zc += wy[b] * A + cy[b] * B;
        yc += wy[b] * B;
      }
      // cross rows y0-1 and y0+4 at this z
      zc += wy[0] * run_dot(ux + orgX[c], wx) + wy[3] * run_dot(ux + orgX[4 + c], wx);
      acc += wz[c] * zc + cz[c] * yc;
    }
    // cross rows z0-1 and z0+4
    T zm = T(0), zp = T(0);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      zm += wy[b] * run_dot(ux + orgX[8 + b], wx);
      zp += wy[b] * run_dot(ux + orgX[12 + b], wx);
    }
    acc += wz[0] * zm + wz[3] * zp;
  }
  return acc;
}

// One Jacobi sweep (MODE EXT_SMOOTH: uo = u + (omega/delta) r) or the residual (EXT_RESID:
// uo = r) with r = b + E f + (E N) u - delta u, at the node in stencil slot k.  Ef (E f of
// this level) and b may be null.  u is only read: uo is another vector.
template <int D, typename T, int MODE>
__device__ __forceinline__ void sweep_node(int64_t k, int64_t n, const T* __restrict__ u, T* __restrict__ uo,
                                           const T* __restrict__ Ef, const T* __restrict__ b,
                                           const int32_t* __restrict__ perm, const int32_t* __restrict__ packed,
                                           const int32_t* __restrict__ origin, const int32_t* __restrict__ originX,
                                           const T* __restrict__ frac, T inv_h2, T delta, T wod) {
  constexpr int S = D == 2 ? 4 : 16;
  constexpr int SX = D == 2 ? 2 : 16;
  const int32_t i = perm[k];
  const int32_t pk = packed[k];
  const int32_t gid = pk >> kXoffBits;
  const T* ux = u + (pk & ((1 << kXoffBits) - 1));
  T wx[4], wy[4], wz[4] = {T(0), T(0), T(0), T(0)};
  cubic_weights<T>(frac[k], wx);
  cubic_weights<T>(frac[n + k], wy);
  if (D == 3) cubic_weights<T>(frac[2 * n + k], wz);
  T t = en_node<D, T>(ux, origin + (int64_t)gid * S, originX + (int64_t)gid * SX, wx, wy, wz) * inv_h2;
  if (Ef) t += Ef[i];
  const T ui = u[i];
  T r = t - delta * ui;
  if (b) r += b[i];
  uo[i] = MODE == EXT_SMOOTH ? ui + wod * r : r;
}

// The fused sweep at slot k from LDS: gl holds the workgroup's staged u values, lo the LDS
// offsets of the local groups' rows (4^(D-1) widened rows, then the cross rows), packedL
// the node's local group and x offset.  The arithmetic is sweep_node's, term for term.
template <int D, typename T, int MODE>
__device__ __forceinline__ void sweep_node_lds(int64_t k, int64_t n, const T* gl, const int32_t* lo,
                                               const T* __restrict__ u, T* __restrict__ uo,
                                               const T* __restrict__ Ef, const T* __restrict__ b,
                                               const int32_t* __restrict__ perm,
                                               const int32_t* __restrict__ packedL, const T* __restrict__ frac,
                                               T inv_h2, T delta, T wod) {
  constexpr int S = D == 2 ? 4 : 16;
  constexpr int SX = D == 2 ? 2 : 16;
  const int32_t i = perm[k];
  const int32_t pk = packedL[k];
  const int32_t* org = lo + (pk >> kXoffBits) * (S + SX);
  const T* ux = gl + (pk & ((1 << kXoffBits) - 1));
  T wx[4], wy[4], wz[4] = {T(0), T(0), T(0), T(0)};
  cubic_weights<T>(frac[k], wx);
  cubic_weights<T>(frac[n + k], wy);
  if (D == 3) cubic_weights<T>(frac[2 * n + k], wz);
  T t = en_node<D, T>(ux, org, org + S, wx, wy, wz) * inv_h2;
  if (Ef) t += Ef[i];
  const T ui = u[i];
  T r = t - delta * ui;
  if (b) r += b[i];
  uo[i] = MODE == EXT_SMOOTH ? ui + wod * r : r;
}

// ---- LDS-staged extension ---------------------------------------------------------
// A workgroup of kExtBlock consecutive stencil slots first copies the g values its
// stencils read into LDS (a few hundred values instead of 64 gathers per node through the
// vector caches), then every lane interpolates from LDS.

template <typename T>
__device__ __forceinline__ T run_dot_lds(const T* p, const T w[4]) {
  return w[0] * p[0] + w[1] * p[1] + w[2] * p[2] + w[3] * p[3];
}

// Every thread of the workgroup must call it (it synchronizes the block).  The copies are
// unrolled by kStageUnroll so that a thread issues all of its index loads, then all of its
// value loads (two memory round trips instead of two per copy); a workgroup staging more
// than kStageUnroll * blockDim values finishes in a plain loop.
constexpr int kStageUnroll = 8;

template <typename T>
__device__ __forceinline__ void ext_stage(int64_t blk, const T* __restrict__ g, const int32_t* __restrict__ blkE,
                                          const int32_t* __restrict__ gidx, const int32_t* __restrict__ blkG,
                                          const int32_t* __restrict__ lorg, int S, T* gl, int32_t* lo) {
  const int32_t e0 = blkE[blk], e1 = blkE[blk + 1];
  const int32_t q0 = blkG[blk] * S, q1 = blkG[blk + 1] * S;
  const int32_t tid = (int32_t)threadIdx.x, bd = (int32_t)blockDim.x;
  int32_t gi[kStageUnroll], lq[kStageUnroll];
#pragma unroll
  for (int j = 0; j < kStageUnroll; ++j) {
    const int32_t e = e0 + tid + j * bd, q = q0 + tid + j * bd;
    gi[j] = e < e1 ? ld_nt(gidx + e) : -1;
    lq[j] = q < q1 ? ld_nt(lorg + q) : 0;
  }
  T gv[kStageUnroll];
#pragma unroll
  for (int j = 0; j < kStageUnroll; ++j) gv[j] = gi[j] >= 0 ? g[gi[j]] : T(0);
#pragma unroll
  for (int j = 0; j < kStageUnroll; ++j) {
    const int32_t e = e0 + tid + j * bd, q = q0 + tid + j * bd;
    if (e < e1) gl[e - e0] = gv[j];
    if (q < q1) lo[q - q0] = lq[j];
  }
  for (int32_t e = e0 + tid + kStageUnroll * bd; e < e1; e += bd) gl[e - e0] = g[gidx[e]];
  for (int32_t q = q0 + tid + kStageUnroll * bd; q < q1; q += bd) lo[q - q0] = lorg[q];
  __syncthreads();
}

template <int D, typename T, typename TO, int MODE>
__device__ __forceinline__ unsigned long long ext_node_lds(int64_t k, int64_t n, const T* gl, const int32_t* lo,
                                                           const int32_t* __restrict__ perm,
                                                           const int32_t* __restrict__ packedL,
                                                           const T* __restrict__ frac, const T* __restrict__ b,
                                                           T* __restrict__ u, TO* __restrict__ out, T delta, T wod,
                                                           const T* __restrict__ wd = nullptr) {
  constexpr int S = D == 2 ? 4 : 16;
  const int32_t i = perm[k];
  const int32_t pk = packedL[k];
  const int32_t* org = lo + (pk >> kXoffBits) * S;
  const T* gx = gl + (pk & ((1 << kXoffBits) - 1));
  T wx[4], wy[4], wz[4];
  cubic_weights<T>(frac[k], wx);
  cubic_weights<T>(frac[n + k], wy);
  T t = T(0);
  if (D == 2) {
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) t += wy[bb] * run_dot_lds(gx + org[bb], wx);
  } else {
    cubic_weights<T>(frac[2 * n + k], wz);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      T tc = T(0);
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) tc += wy[bb] * run_dot_lds(gx + org[bb + 4 * c], wx);
      t += wz[c] * tc;
    }
  }
  if (MODE == EXT_SMOOTH) {
    const T ui = u[i];
    T r = t - delta * ui;
    if (b) r += b[i];
    u[i] = ui + (wd ? wd[i] : wod) * r;  // wd: per-node scale of the standard relaxation
    if (out) out[i] = (TO)t;  // optionally keep E g
    return abs_bits((double)r);
  } else if (MODE == EXT_RESID) {
    T r = t - delta * u[i];
    if (b) r += b[i];
    if (wd) r *= wd[i];  // variable coefficient: residual brought to the units of f
    if (out) out[i] = (TO)r;
    return abs_bits((double)r);
  } else if (MODE == EXT_APPLY) {
    out[i] = (TO)(delta * u[i] - t);
    return 0ull;
  } else {
    if (out) out[i] = (TO)t;
    return abs_bits((double)t);
  }
}

// Linear interpolation at a closest point of values v through 2^(D-1) x-runs of length 2:
// runs[r * cnt + j], fractions frac[a * cnt + j].
template <int D, typename T>
__device__ __forceinline__ T linear_node(int64_t j, int64_t cnt, const T* __restrict__ v,
                                         const int32_t* __restrict__ runs, const T* __restrict__ frac) {
  const T ax = frac[j], ay = frac[cnt + j];
  const T wx0 = T(1) - ax, wy0 = T(1) - ay;
  const T* p0 = v + runs[j];
  const T* p1 = v + runs[cnt + j];
  const T z0 = wy0 * (wx0 * p0[0] + ax * p0[1]) + ay * (wx0 * p1[0] + ax * p1[1]);
  if (D == 2) return z0;
  const T az = frac[2 * cnt + j];
  const T* p2 = v + runs[2 * cnt + j];
  const T* p3 = v + runs[3 * cnt + j];
  const T z1 = wy0 * (wx0 * p2[0] + ax * p2[1]) + ay * (wx0 * p3[0] + ax * p3[1]);
  return (T(1) - az) * z0 + az * z1;
}

// Cubic closest-point interpolation of v at target node j (4^(D-1) runs of 4 consecutive
// source entries, fractions per axis; the layout of the transfer runs).
template <int D, typename T>
__device__ __forceinline__ T cubic_node(int64_t j, int64_t cnt, const T* __restrict__ v,
                                        const int32_t* __restrict__ runs, const T* __restrict__ frac) {
  T wx[4], wy[4];
  cubic_weights<T>(frac[j], wx);
  cubic_weights<T>(frac[cnt + j], wy);
  if (D == 2) {
    T t = T(0);
#pragma unroll
    for (int b = 0; b < 4; ++b) t += wy[b] * run_dot(v + runs[b * cnt + j], wx);
    return t;
  }
  T wz[4];
  cubic_weights<T>(frac[2 * cnt + j], wz);
  T t = T(0);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    T tc = T(0);
#pragma unroll
    for (int b = 0; b < 4; ++b) tc += wy[b] * run_dot(v + runs[(b + 4 * c) * cnt + j], wx);
    t += wz[c] * tc;
  }
  return t;
}

}  // namespace cpm
