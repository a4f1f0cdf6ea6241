// Coarsest-level solve on the nonzero columns of Z = A_c^{-1} E_c only.
//
// E_c reads a grid function only at the nodes of B_interp (the nodes of some cubic stencil,
// Sec. 3.1), so every other column of E_c is zero, and so is the same column of Z: Gauss-
// Jordan on [A_c | E_c] only combines rows, and a column of zeros stays zero.  On the torus
// at h = 1/8 B_interp holds 68 % of the nodes, so the per-cycle product reads 68 % of the
// matrix.  After the factorization, the B_interp columns of the right half are copied, in
// list order, into the (no longer needed) left half of the same rows; the right half is kept
// as it was for the batched solver, which reads it in place.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "capi_internal.h"
#include "kernels_dev.h"

namespace cpm {
namespace {

// Row `row` of [I | Z] (row stride ld): r[j] = r[n + col[j]] for j < m.  The reads (columns
// n .. 2n - 1) and the writes (columns 0 .. m - 1, m <= n) never overlap.
__global__ __launch_bounds__(256) void k_compact_cols(int n, int m, int64_t ld, double* __restrict__ M,
                                                      const int32_t* __restrict__ col) {
  double* r = M + (int64_t)blockIdx.y * ld;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) r[j] = r[n + col[j]];
}

// y[row] = sum_{j < m} Zc[row][j] x[col[j]]: one workgroup per row, as the dense product
// (eight independent loads in flight per thread, the matrix streamed non-temporal).
template <typename T>
__global__ __launch_bounds__(256) void k_gemv_cols(int m, const double* __restrict__ Z, int64_t ld,
                                                   const int32_t* __restrict__ col, const T* __restrict__ x,
                                                   T* __restrict__ y) {
  const int row = blockIdx.x;
  const double* zr = Z + (int64_t)row * ld;
  double s = 0.0;
  int j = threadIdx.x;
  for (; j + 7 * 256 < m; j += 8 * 256) {
    double z[8], xv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      z[q] = ld_nt(zr + j + q * 256);
      xv[q] = (double)x[col[j + q * 256]];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) s += z[q] * xv[q];
  }
  for (; j < m; j += 256) s += ld_nt(zr + j) * (double)x[col[j]];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) y[row] = (T)(((part[0] + part[1]) + part[2]) + part[3]);
}

}  // namespace

void launch_compact_cols(int n, int m, int64_t ld, double* M, const int32_t* col, hipStream_t s) {
  if (n <= 0 || m <= 0) return;
  const unsigned gx = (unsigned)std::min((m + 255) / 256, 64);
  k_compact_cols<<<dim3(gx, (unsigned)n), 256, 0, s>>>(n, m, ld, M, col);
}

template <typename T>
void launch_coarse_gemv_cols(int n, int m, const double* Z, int64_t ld, const int32_t* col, const T* x, T* y,
                             hipStream_t s) {
  if (n <= 0) return;
  k_gemv_cols<T><<<(unsigned)n, 256, 0, s>>>(m, Z, ld, col, x, y);
}

template void launch_coarse_gemv_cols<double>(int, int, const double*, int64_t, const int32_t*, const double*,
                                              double*, hipStream_t);
template void launch_coarse_gemv_cols<float>(int, int, const double*, int64_t, const int32_t*, const float*,
                                             float*, hipStream_t);

}  // namespace cpm
