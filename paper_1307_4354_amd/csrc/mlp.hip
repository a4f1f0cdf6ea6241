// Learned local smoother: a two-layer network (64 inputs, 64 hidden units, 1 output) that
// maps a node's normalised 3^d residual patch and its own 1-D cubic interpolation weights
// to an update of u, replacing the damped Jacobi step on the two finest levels.
//
// Layer 1 (the only dense contraction) runs on the matrix cores: for 64 nodes at a time a
// wavefront computes H (64 x 64) = X (64 x 64, bf16) * W1^T (64 x 64, bf16) with
// v_mfma_f32_32x32x8_bf16 in float32 accumulators (2 x 2 output tiles, 8 k-steps).
// Operand layout of that instruction (per lane l, half = l / 32, col = l % 32):
//   A (32 x 8): row col, k = 4 half .. 4 half + 3        (4 bf16 in one 64-bit register pair)
//   B (8 x 32): col col, k = 4 half .. 4 half + 3
//   D (32 x 32): register v holds row 8 (v / 4) + 4 half + v % 4, column col.
// Layer 2 (64 -> 1) and the update are float32 VALU work.  The weight gradient of layer 1,
// dW1 = dH^T X summed over nodes, uses the same instruction with the node index as k.
#include <hip/hip_runtime.h>

#include <cstring>

#include "capi_internal.h"
#include "kernels_dev.h"

namespace cpm {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kIn = CPM_MLP_IN;
constexpr int kHid = CPM_MLP_HIDDEN;
constexpr int kB1 = kHid * kIn;      // offset of b1 in the packed weights
constexpr int kW2 = kB1 + kHid;      // offset of w2
constexpr int kB2 = kW2 + kHid;      // offset of b2
constexpr int kWCount = kB2 + 1;
constexpr int kPartStride = 33;      // padded row of the layer-2 partial sums in LDS

__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t b = __float_as_uint(x);
  b += 0x7FFFu + ((b >> 16) & 1u);  // round to nearest even
  return (uint16_t)(b >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// One wavefront evaluates the network on 64 feature rows X[row * 64 + k] (bf16, generic
// pointer: global or LDS), rows >= valid read as zero.  Returns y for row = lane.  If H is
// not null the hidden activations of valid rows are stored (float, row stride 64).  part is
// this wavefront's LDS scratch (64 x kPartStride floats).  Every thread of the block must
// call it (it synchronizes the block).
__device__ float mlp_wave(const uint16_t* X, int valid, const uint16_t* __restrict__ W, float* part,
                          float* __restrict__ H) {
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5, col = lane & 31;
  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.0f;
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) {
    bf16x4 av[2], bv[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      const int row = mb * 32 + col;
      if (row < valid) {
        av[mb] = *(const bf16x4*)(X + row * kIn + ks * 8 + half * 4);
      } else {
        av[mb] = bf16x4{0, 0, 0, 0};
      }
    }
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) bv[nb] = *(const bf16x4*)(W + (nb * 32 + col) * kIn + ks * 8 + half * 4);
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av[mb], bv[nb], acc[mb][nb], 0, 0, 0);
  }
  float b1v[2], w2v[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    b1v[nb] = bf2f(W[kB1 + nb * 32 + col]);
    w2v[nb] = bf2f(W[kW2 + nb * 32 + col]);
  }
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = mb * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
      float p = 0.0f;
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const float hv = fmaxf(acc[mb][nb][v] + b1v[nb], 0.0f);
        p += hv * w2v[nb];
        if (H && row < valid) H[row * kHid + nb * 32 + col] = hv;
      }
      part[row * kPartStride + col] = p;
    }
  __syncthreads();
  float y = bf2f(W[kB2]);
  for (int c = 0; c < 32; ++c) y += part[lane * kPartStride + c];
  __syncthreads();
  return y;
}

// Features of one node: residual patch / s, then the 1-D weights, then zeros.  Writes
// NOUT bf16 into xw, two per word (slot 2j in the low half of word j); returns s.
template <int D, typename T, int NOUT = kIn, typename TF = T>
__device__ __forceinline__ float node_features(int64_t k, int64_t n, const T* __restrict__ r,
                                               const int32_t* __restrict__ prow, const int32_t* __restrict__ ppk,
                                               int64_t groups, const uint32_t* __restrict__ pmask,
                                               const TF* __restrict__ frac, uint32_t* xw) {
  constexpr int R = D == 2 ? 3 : 9;
  constexpr int P = 3 * R;
  const uint32_t mask = ld_nt(pmask + k);
  // the node's rows: its group's rows (one per group of consecutive nodes) plus its offset
  const int32_t pk = ld_nt(ppk + k);
  const int32_t* grow = prow + (pk >> kPatchBits);
  const int32_t toff = pk & (kPatchRun - 1);
  // every load is issued unconditionally (the index clamped into the array, the value of an
  // absent node discarded below), so the 3^D loads are in flight together; the addresses are
  // 32-bit byte offsets from r (a level's vector is far below 4 GiB), one register each
  T patch[P];
  const char* rb = reinterpret_cast<const char*>(r);
  const int32_t last = (int32_t)(n - 1);
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int32_t base = grow[q * groups] + toff;
    // a row with its outer nodes present and its middle one absent stores them adjacently
    const int gap = ((mask >> (3 * q)) & 7u) == 5u;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      int32_t a = base + dx - (dx == 2 ? gap : 0);
      a = a < 0 ? 0 : (a > last ? last : a);
      patch[dx + 3 * q] = *reinterpret_cast<const T*>(rb + (uint32_t)a * (uint32_t)sizeof(T));
    }
  }
  T s = T(0);
#pragma unroll
  for (int bit = 0; bit < P; ++bit) {
    patch[bit] = (mask >> bit) & 1u ? patch[bit] : T(0);
    s = fmax(s, (T)fabs((double)patch[bit]));
  }
  // patch / s to bfloat16: formed in float32 as patch * (1 / s); it differs from the
  // correctly rounded quotient by at most 2 float ulps, below the bf16 rounding step
  const float inv_s = s > T(0) ? 1.0f / (float)s : 0.0f;
#pragma unroll
  for (int j = 0; j < NOUT / 2; ++j) xw[j] = 0u;
  // each slot's bf16 goes straight into its word, so no per-slot register is kept
  auto put = [&](int q, float v) { xw[q >> 1] |= (uint32_t)f2bf(v) << (16 * (q & 1)); };
#pragma unroll
  for (int q = 0; q < P; ++q) put(q, (float)patch[q] * inv_s);
  TF w[4];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    cubic_weights<TF>(ld_nt(frac + a * n + k), w);
#pragma unroll
    for (int j = 0; j < 4; ++j) put(P + 4 * a + j, (float)w[j]);
  }
  return (float)s;
}

// Features of every node of a level, in band order (patch tables and band-order fractions).
template <int D, typename T>
__global__ __launch_bounds__(256) void k_features(int64_t n, const T* __restrict__ r, const int32_t* __restrict__ prow,
                                                  const int32_t* __restrict__ ppk, int64_t groups,
                                                  const uint32_t* __restrict__ pmask, const T* __restrict__ frac,
                                                  uint16_t* __restrict__ X, float* __restrict__ scale) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t xw[kIn / 2];
  const float s = node_features<D, T>(i, n, r, prow, ppk, groups, pmask, frac, xw);
  uint64_t* dst = (uint64_t*)(X + (int64_t)i * kIn);
#pragma unroll
  for (int q = 0; q < kIn / 4; ++q) dst[q] = (uint64_t)xw[2 * q] | ((uint64_t)xw[2 * q + 1] << 32);
  scale[i] = s;
}

// Fused learned sweep, one node per lane and 64 consecutive band nodes per wavefront (their
// patch rows overlap, so the residual gathers coalesce).
// Layer 1 is computed transposed, H^T (hidden x node) = W1 * X^T, so that after the matrix
// cores a lane holds 16 hidden units of one node and layer 2 is a per-lane sum plus one
// exchange with lane ^ 32.  The matrix cores run gfx950's double-rate
// v_mfma_f32_32x32x16_bf16 (operand layouts below).  A lane computes the whole feature row of
// its own node; the k-chunk its partner lane needs for the other node block arrives through
// xor-32 shuffles.  Only the k-steps that hold features are issued (3 of 4 in 3-D); the last
// slot of the last step, a zero of the network's input, carries a constant 1 whose A entry is
// b1, so the bias is added inside the float32 accumulation.  The used
// columns of W1 (with b1) and w2 are staged once per workgroup in LDS.  The residual may come
// in float32 (R = float) under a float64 iterate: the features take it in float32 anyway, and
// the largest float32-rounded entry is the float32-rounded largest entry, so the scale s and
// the update are the same bit for bit; the patch then holds half the registers.
template <int D, typename T, typename R = T>
__global__ __launch_bounds__(256) void k_learned(int64_t n, const R* __restrict__ r, const int32_t* __restrict__ prow,
                                                 const int32_t* __restrict__ ppk, int64_t groups,
                                                 const uint32_t* __restrict__ pmask, const T* __restrict__ frac,
                                                 const uint16_t* __restrict__ W, T inv_delta, T* __restrict__ u) {
  constexpr int NF = (D == 2 ? 9 : 27) + 4 * D;  // features in use
  constexpr int KS = (NF + 1 + 15) / 16;          // k-steps of 16, with room for the constant slot
  constexpr int KB = 16 * KS - 1;                 // slot of the constant 1 (a zero input)
  static_assert(KB >= NF && 16 * KS <= kIn, "feature layout");
  constexpr int WS = 16 * KS + 8;  // LDS row of W1 in bf16 (16-byte aligned rows, padded)
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
  __shared__ __attribute__((aligned(16))) uint16_t w1s[64 * WS];  // the 16 KS used columns of W1, b1 in column KB
  __shared__ float w2s[64];
  for (int e = threadIdx.x; e < 64 * 4 * KS; e += blockDim.x) {
    const int row = e / (4 * KS), c = 4 * (e % (4 * KS));
    bf16x4 q = *(const bf16x4*)(W + row * kIn + c);
    if (c + 3 == KB) q[3] = (short)W[kB1 + row];
    *(bf16x4*)&w1s[row * WS + c] = q;
  }
  if (threadIdx.x < 64) w2s[threadIdx.x] = bf2f(W[kW2 + threadIdx.x]);
  __syncthreads();
  const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
  const int64_t k = (blockIdx.x * 4 + (threadIdx.x >> 6)) * (int64_t)64 + lane;
  uint32_t xw[8 * KS];  // own feature row, bf16 pairs (slot 2j in the low half of word j)
  float s = 0.0f;
  if (k < n) {
    s = node_features<D, R, 16 * KS, T>(k, n, r, prow, ppk, groups, pmask, frac, xw);
  } else {
#pragma unroll
    for (int j = 0; j < 8 * KS; ++j) xw[j] = 0u;
  }
  xw[KB >> 1] |= 0x3F80u << (16 * (KB & 1));  // the constant 1.0 (a zero slot of the input)
  // v_mfma_f32_32x32x16_bf16 operands (lane l, half = l/32, col = l%32): A = W1 row (hidden
  // unit col of the block), k = 16 ks + 8 half .. + 7; B = X^T column (node col), the same k
  // range; D element v of lane l = row 8 (v/4) + 4 half + v%4, column col.  A lane's own node
  // is column col of node block half; the 8 k-slots the partner lane needs for the other node
  // block arrive through one xor-32 exchange of four words per k-step.
  uint32_t own[4 * KS], got[4 * KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t lo = xw[8 * ks + e], hi = xw[8 * ks + 4 + e];
      own[4 * ks + e] = half ? hi : lo;
      got[4 * ks + e] = __shfl_xor(half ? lo : hi, 32);
    }
  }
  // one 32x32 accumulator tile at a time (hidden block mb of node block nb)
  float y = 0.0f;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const bool mine = nb == half;  // this lane's own node is column col of node block nb
    float p = 0.0f;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      f32x16 acc;
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const u32x4 bw = {mine ? own[4 * ks] : got[4 * ks], mine ? own[4 * ks + 1] : got[4 * ks + 1],
                          mine ? own[4 * ks + 2] : got[4 * ks + 2], mine ? own[4 * ks + 3] : got[4 * ks + 3]};
        const bf16x8 bv = __builtin_bit_cast(bf16x8, bw);
        const bf16x8 av = *(const bf16x8*)&w1s[(mb * 32 + col) * WS + ks * 16 + half * 8];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) p += fmaxf(acc[v], 0.0f) * w2s[mb * 32 + 8 * (v >> 2) + 4 * half + (v & 3)];
    }
    p += __shfl_xor(p, 32);
    if (mine) y = p;
  }
  if (k < n) {
    y += bf2f(W[kB2]);
    u[k] += (T)s * inv_delta * (T)y;
  }
}

__global__ __launch_bounds__(256) void k_mlp_fwd(int64_t m, const uint16_t* __restrict__ X,
                                                 const uint16_t* __restrict__ W, float* __restrict__ Y,
                                                 float* __restrict__ H) {
  __shared__ float part[4][64 * kPartStride];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r0 = (blockIdx.x * 4 + wave) * (int64_t)64;
  const int64_t rem = m - r0;
  const int valid = rem <= 0 ? 0 : (rem >= 64 ? 64 : (int)rem);
  const uint16_t* Xw = X + (valid > 0 ? r0 * kIn : 0);
  float* Hw = (H && valid > 0) ? H + r0 * kHid : nullptr;
  const float y = mlp_wave(Xw, valid, W, part[wave], Hw);
  if (lane < valid) Y[r0 + lane] = y;
}

// Gradient of (1/m) sum (y - t)^2.  Each wavefront takes chunks of 64 nodes; per chunk the
// lanes own hidden unit j = lane for the small gradients, dH^T (bf16) and the X chunk are
// staged in LDS, and dW1 += dH^T X on the matrix cores.  Partial sums end in G by atomics.
__global__ __launch_bounds__(256) void k_mlp_bwd(int64_t m, const uint16_t* __restrict__ X,
                                                 const uint16_t* __restrict__ W, const float* __restrict__ H,
                                                 const float* __restrict__ Y, const float* __restrict__ T,
                                                 float* __restrict__ G) {
  constexpr int LS = 68;  // padded LDS row (bf16 elements)
  __shared__ uint16_t dht[4][64 * LS];
  __shared__ uint16_t xs[4][64 * LS];
  __shared__ float dys[4][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int half = lane >> 5, col = lane & 31;
  const float w2j = bf2f(W[kW2 + lane]);
  const float two_over_m = 2.0f / (float)m;
  float gw2 = 0.0f, gb1 = 0.0f, gb2 = 0.0f;
  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.0f;
  const int64_t nchunks = (m + 63) / 64;
  for (int64_t cb = blockIdx.x; cb * 4 < nchunks; cb += gridDim.x) {  // same trip count for all waves
    const int64_t c = cb * 4 + wave;
    const int64_t i0 = c * 64;
    const int64_t rem = m - i0;
    const int valid = rem <= 0 ? 0 : (rem >= 64 ? 64 : (int)rem);
    // stage X rows and dy
    for (int q = 0; q < kIn; ++q) xs[wave][lane * LS + q] = lane < valid ? X[(i0 + lane) * kIn + q] : (uint16_t)0;
    const float dy = lane < valid ? two_over_m * (Y[i0 + lane] - T[i0 + lane]) : 0.0f;
    dys[wave][lane] = dy;
    gb2 += dy;
    __syncthreads();
    // lane = hidden unit j: small gradients and dH^T
    for (int i = 0; i < 64; ++i) {
      const float hv = i < valid ? H[(i0 + i) * kHid + lane] : 0.0f;
      const float d = dys[wave][i];
      gw2 += d * hv;
      const float dh = hv > 0.0f ? d * w2j : 0.0f;
      gb1 += dh;
      dht[wave][lane * LS + i] = f2bf(dh);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      bf16x4 av[2], bv[2];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) av[mb] = *(const bf16x4*)&dht[wave][(mb * 32 + col) * LS + ks * 8 + half * 4];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const int kk = ks * 8 + half * 4;
        bf16x4 t;
        t[0] = (short)xs[wave][(kk + 0) * LS + nb * 32 + col];
        t[1] = (short)xs[wave][(kk + 1) * LS + nb * 32 + col];
        t[2] = (short)xs[wave][(kk + 2) * LS + nb * 32 + col];
        t[3] = (short)xs[wave][(kk + 3) * LS + nb * 32 + col];
        bv[nb] = t;
      }
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
          acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av[mb], bv[nb], acc[mb][nb], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int j = mb * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
        atomicAdd(&G[j * kIn + nb * 32 + col], acc[mb][nb][v]);
      }
  atomicAdd(&G[kB1 + lane], gb1);
  atomicAdd(&G[kW2 + lane], gw2);
  for (int off = 32; off > 0; off >>= 1) gb2 += __shfl_xor(gb2, off);
  if (lane == 0) atomicAdd(&G[kB2], gb2);
}

// Adam step on float32 master weights; the bf16 copy used by the kernels is refreshed.
__global__ void k_adam(int count, float* __restrict__ w, float* __restrict__ m1, float* __restrict__ m2,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2,
                       uint16_t* __restrict__ wb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.0f - b1) * gi;
  const float b = b2 * m2[i] + (1.0f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  const float wn = w[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
  w[i] = wn;
  wb[i] = f2bf(wn);
}

// Training target of the learned step at every node: the undamped Ruuth-Merriman correction
// in the network's units, t_i = r_i / s_i clipped to [-clip, clip] (0 where s_i = 0).
__global__ void k_targets(int64_t n, const double* __restrict__ r, const float* __restrict__ scale, double clip,
                          float* __restrict__ T) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float s = scale[i];
  double t = s > 0.0f ? r[i] / (double)s : 0.0;
  t = t > clip ? clip : (t < -clip ? -clip : t);
  T[i] = (float)t;
}

// loss = (1/m) sum (Y - T)^2 in double, one workgroup (fixed summation order).
__global__ __launch_bounds__(1024) void k_mse(int64_t m, const float* __restrict__ Y, const float* __restrict__ T,
                                              double* __restrict__ loss) {
  __shared__ double part[16];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
    const double d = (double)Y[i] - (double)T[i];
    acc += d * d;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += part[w];
    *loss = t / (double)m;
  }
}

// fractions in the extension's processing order, and in band order
template <typename T>
const T* frac_k(const DevLevel& D);
template <>
const double* frac_k<double>(const DevLevel& D) { return D.band_order ? D.fracE : D.fracK; }
template <>
const float* frac_k<float>(const DevLevel& D) { return D.band_order ? D.fracE32 : D.fracK32; }
template <typename T>
const T* frac_b(const DevLevel& D);
template <>
const double* frac_b<double>(const DevLevel& D) { return D.fracE; }
template <>
const float* frac_b<float>(const DevLevel& D) { return D.fracE32; }

}  // namespace

// The fused network update u += (s / delta) y on level l from the residual r.
template <typename T, typename R>
void launch_learned_r(const cpm_band b, int l, const R* r, T* u, double c, hipStream_t s) {
  const DevLevel& D = b->dev[(size_t)l];
  const double delta = level_delta(b, l, c);
  const unsigned gr = (unsigned)((D.n + 255) / 256);  // 64 nodes per wavefront, 4 per block
  if (b->dim == 2)
    k_learned<2, T, R><<<gr, 256, 0, s>>>(D.n, r, D.patchRow, D.patchPk, D.patchGroups, D.patchMask, frac_b<T>(D),
                                          b->mlpW, (T)(1.0 / delta), u);
  else
    k_learned<3, T, R><<<gr, 256, 0, s>>>(D.n, r, D.patchRow, D.patchPk, D.patchGroups, D.patchMask, frac_b<T>(D),
                                          b->mlpW, (T)(1.0 / delta), u);
}

template <typename T>
void launch_learned(const cpm_band b, int l, const T* r, T* u, double c, hipStream_t s) {
  launch_learned_r<T, T>(b, l, r, u, c, s);
}

// r = b + E g - delta u into B.r (in float32: the network reads no more of it, see k_learned),
// then the fused network update of u.
template <typename T>
void learned_sweep(const cpm_band b, int l, T* u, const T* f, const T* rhsA, T* g, T* r, double c, hipStream_t s) {
  (void)f;
  const DevLevel& D = b->dev[(size_t)l];
  const double delta = level_delta(b, l, c);
  float* r32 = reinterpret_cast<float*>(r);
  launch_ext<T, float>(b->dim, EXT_RESID, D.n, g, ext_addr(D), frac_k<T>(D), rhsA, u, r32, (T)delta, (T)0, nullptr,
                       ext_cfg(D), s);
  launch_learned_r<T, float>(b, l, r32, u, c, s);
}

template void launch_learned_r<double, float>(const cpm_band, int, const float*, double*, double, hipStream_t);
template void launch_learned<double>(const cpm_band, int, const double*, double*, double, hipStream_t);
template void launch_learned<float>(const cpm_band, int, const float*, float*, double, hipStream_t);
template void learned_sweep<double>(const cpm_band, int, double*, const double*, const double*, double*, double*,
                                    double, hipStream_t);
template void learned_sweep<float>(const cpm_band, int, float*, const float*, const float*, float*, float*, double,
                                   hipStream_t);

}  // namespace cpm

using namespace cpm;

extern "C" {

cpm_status cpm_set_smoother_weights(cpm_band band, const uint16_t* w_bf16, double rho_plain) {
  if (!band || !w_bf16 || !(rho_plain > 0.0)) {
    set_error("cpm_set_smoother_weights: invalid argument");
    return CPM_E_INVALID;
  }
  if (!band->mlpW && !(band->mlpW = (uint16_t*)dev_alloc(band, kWCount * sizeof(uint16_t)))) {
    set_error("device allocation failed");
    return CPM_E_NOMEM;
  }
  if (hipMemcpy(band->mlpW, w_bf16, kWCount * sizeof(uint16_t), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("weight upload failed");
    return CPM_E_HIP;
  }
  band->rho_plain = rho_plain;
  for (auto& kv : band->graphs) (void)hipGraphExecDestroy(kv.second);
  band->graphs.clear();
  return CPM_OK;
}

cpm_status cpm_mlp_forward(int64_t m, const uint16_t* X, const uint16_t* W, float* Y, float* H, void* stream) {
  if (m < 0 || (m > 0 && (!X || !W || !Y))) {
    set_error("cpm_mlp_forward: invalid argument");
    return CPM_E_INVALID;
  }
  if (m == 0) return CPM_OK;
  hipStream_t s = (hipStream_t)stream;
  k_mlp_fwd<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(m, X, W, Y, H);
  return check_launch("cpm_mlp_forward");
}

cpm_status cpm_mlp_backward(int64_t m, const uint16_t* X, const uint16_t* W, const float* H, const float* Y,
                            const float* T, float* G, void* stream) {
  if (m <= 0 || !X || !W || !H || !Y || !T || !G) {
    set_error("cpm_mlp_backward: invalid argument");
    return CPM_E_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  launch_fill<float>(kWCount, G, 0.0f, s);
  const int64_t chunks = (m + 63) / 64;
  int64_t blocks = (chunks + 3) / 4;
  if (blocks > 2048) blocks = 2048;
  k_mlp_bwd<<<(unsigned)blocks, 256, 0, s>>>(m, X, W, H, Y, T, G);
  return check_launch("cpm_mlp_backward");
}

cpm_status cpm_mlp_adam(int step, float lr, float* w_master, float* m1, float* m2, const float* G,
                        uint16_t* w_bf16, void* stream) {
  if (step < 1 || !(lr > 0.0f) || !w_master || !m1 || !m2 || !G || !w_bf16) {
    set_error("cpm_mlp_adam: invalid argument");
    return CPM_E_INVALID;
  }
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  k_adam<<<(kWCount + 255) / 256, 256, 0, (hipStream_t)stream>>>(kWCount, w_master, m1, m2, G, lr, b1, b2, 1e-8f, c1,
                                                                 c2, w_bf16);
  return check_launch("cpm_mlp_adam");
}

cpm_status cpm_smoother_features(cpm_band band, int level, double c, const double* f, const double* u, uint16_t* X,
                                 float* scale, void* work, void* stream) {
  if (!band || level < 0 || level >= band->L || level > 1 || !f || !u || !X || !scale || !work || !(c > 0.0)) {
    set_error("cpm_smoother_features: invalid argument (levels 0 and 1 only)");
    return CPM_E_INVALID;
  }
  const DevLevel& D = band->dev[(size_t)level];
  if (!D.patchRow) {
    set_error("cpm_smoother_features: no patch addressing on this level");
    return CPM_E_INVALID;
  }
  StreamScope stream_scope(band);
  cpm_status st = enter(band, stream);
  if (st != CPM_OK) return st;
  hipStream_t s = band->stream;
  const LaunchCfg lc = band_cfg(band, D.n);
  double* g = (double*)work;
  double* r = g + D.n;
  launch_nsum<double>(band->dim, nsum_addr(D), u, f, 1.0 / (D.h * D.h), g, nullptr, lc, s);
  launch_ext<double, double>(band->dim, EXT_RESID, D.n, g, ExtAddr{D.perm, D.packed, D.origin}, D.fracK, nullptr,
                             const_cast<double*>(u), r, level_delta(band, level, c), 0.0, nullptr, lc, s);
  const unsigned gr = (unsigned)((D.n + 255) / 256);
  if (band->dim == 2)
    k_features<2, double><<<gr, 256, 0, s>>>(D.n, r, D.patchRow, D.patchPk, D.patchGroups, D.patchMask, D.fracE, X,
                                             scale);
  else
    k_features<3, double><<<gr, 256, 0, s>>>(D.n, r, D.patchRow, D.patchPk, D.patchGroups, D.patchMask, D.fracE, X,
                                             scale);
  if ((st = check_launch("cpm_smoother_features")) != CPM_OK) return st;
  return leave(band, stream);
}

cpm_status cpm_smoother_pairs(cpm_band band, int level, double c, const double* f, const double* u, uint16_t* X,
                              float* T, float* scale, double clip, void* work, void* stream) {
  if (!T || !(clip > 0.0)) {
    set_error("cpm_smoother_pairs: invalid argument");
    return CPM_E_INVALID;
  }
  cpm_status st = cpm_smoother_features(band, level, c, f, u, X, scale, work, stream);
  if (st != CPM_OK) return st;
  const int64_t n = band->dev[(size_t)level].n;
  const double* r = (const double*)work + n;  // the residual cpm_smoother_features left there
  k_targets<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(n, r, scale, clip, T);
  return check_launch("cpm_smoother_pairs");
}

cpm_status cpm_mlp_loss(int64_t m, const float* Y, const float* T, double* loss, void* stream) {
  if (m <= 0 || !Y || !T || !loss) {
    set_error("cpm_mlp_loss: invalid argument");
    return CPM_E_INVALID;
  }
  k_mse<<<1, 1024, 0, (hipStream_t)stream>>>(m, Y, T, loss);
  return check_launch("cpm_mlp_loss");
}

}  // extern "C"
