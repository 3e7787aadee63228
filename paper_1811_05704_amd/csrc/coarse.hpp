// Dense inverse of a symmetric positive definite coarsest operator on the
// device (section 2, "AMG solve": the coarsest level is solved directly; the
// library applies the inverse as a GEMV).
//
// Blocked Gauss-Jordan elimination without pivoting, in place on the dense
// row-major n x n matrix, 64 x 64 blocks.  For each diagonal block K:
//   P = A_KK^-1                       (one workgroup, in LDS)
//   A_Kj = P A_Kj          (j != K)   (block row)
//   A_ij = A_ij - A_iK A_Kj  (i, j != K)   (trailing update, the bulk: 2 n^3
//                                      flops in all, LDS-tiled)
//   A_iK = -A_iK P         (i != K)   (block column)
//   A_KK = P
// after which A holds A^-1.  Every pivot of a symmetric positive definite
// matrix (and of its Schur complements) is positive; a pivot that is not
// raises a flag and the caller falls back to LU with partial pivoting.
// Each output is summed in a fixed order, so the result is deterministic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amg {

constexpr int kGjB = 64;   // block size
constexpr int kGjBS = 256; // threads per workgroup

// P = A_KK^-1 for the kb x kb diagonal block at k0 (in-place Gauss-Jordan in
// LDS); bad = 1 if a pivot is not positive.
static __global__ void __launch_bounds__(kGjBS) gj_diag_kernel(int n, const double* __restrict__ A, int k0, int kb,
                                                               double* __restrict__ P, int* bad) {
  __shared__ double D[kGjB][kGjB + 1];
  __shared__ double f[kGjB];
  const int tid = threadIdx.x;
  for (int e = tid; e < kGjB * kGjB; e += kGjBS) {
    const int r = e / kGjB, c = e % kGjB;
    D[r][c] = (r < kb && c < kb) ? A[static_cast<int64_t>(k0 + r) * n + k0 + c] : 0.0;
  }
  for (int k = 0; k < kb; ++k) {
    __syncthreads();
    const double p = D[k][k];
    if (tid == 0 && !(p > 0.0)) *bad = 1;
    if (tid < kb) f[tid] = D[tid][k];
    __syncthreads();
    if (tid < kb) D[k][tid] = (tid == k ? 1.0 : D[k][tid]) / p;
    __syncthreads();
    for (int e = tid; e < kb * kb; e += kGjBS) {
      const int r = e / kb, c = e % kb;
      if (r == k) continue;
      D[r][c] = (c == k ? 0.0 : D[r][c]) - f[r] * D[k][c];
    }
  }
  __syncthreads();
  for (int e = tid; e < kGjB * kGjB; e += kGjBS) P[e] = D[e / kGjB][e % kGjB];  // zero outside kb x kb
}

// A_Kj = P A_Kj for every column j outside the block (one thread per column).
static __global__ void __launch_bounds__(kGjBS) gj_row_kernel(int n, double* __restrict__ A, int k0, int kb,
                                                              const double* __restrict__ P) {
  __shared__ double Ps[kGjB * kGjB];
  for (int e = threadIdx.x; e < kGjB * kGjB; e += kGjBS) Ps[e] = P[e];
  __syncthreads();
  const int j = blockIdx.x * kGjBS + threadIdx.x;
  if (j >= n || (j >= k0 && j < k0 + kb)) return;
  double x[kGjB];
#pragma unroll
  for (int c = 0; c < kGjB; ++c) x[c] = c < kb ? A[static_cast<int64_t>(k0 + c) * n + j] : 0.0;
  for (int r = 0; r < kb; ++r) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kGjB; ++c) s += Ps[r * kGjB + c] * x[c];
    A[static_cast<int64_t>(k0 + r) * n + j] = s;
  }
}

// A_ij -= A_iK A_Kj for i, j outside the block: 64 x 64 output tiles, each
// thread 4 x 4 outputs, the tile's A_iK and A_Kj staged in LDS.
static __global__ void __launch_bounds__(kGjBS) gj_trailing_kernel(int n, double* __restrict__ A, int k0, int kb) {
  const int bi = blockIdx.y, bj = blockIdx.x;
  const int K = k0 / kGjB;
  if (bi == K || bj == K) return;
  __shared__ double L[kGjB][kGjB + 1];
  __shared__ double U[kGjB][kGjB + 1];
  const int i0 = bi * kGjB, j0 = bj * kGjB;
  const int tid = threadIdx.x;
  for (int e = tid; e < kGjB * kGjB; e += kGjBS) {
    const int r = e / kGjB, c = e % kGjB;
    L[r][c] = (i0 + r < n && c < kb) ? A[static_cast<int64_t>(i0 + r) * n + k0 + c] : 0.0;
    U[r][c] = (r < kb && j0 + c < n) ? A[static_cast<int64_t>(k0 + r) * n + j0 + c] : 0.0;
  }
  __syncthreads();
  const int ty = tid / 16, tx = tid % 16;
  double acc[4][4] = {};
  for (int c = 0; c < kb; ++c) {
    double a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[q] = L[ty * 4 + q][c];
      b[q] = U[c][tx * 4 + q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int w = 0; w < 4; ++w) acc[q][w] += a[q] * b[w];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = i0 + ty * 4 + q;
    if (i >= n) continue;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int j = j0 + tx * 4 + w;
      if (j < n) A[static_cast<int64_t>(i) * n + j] -= acc[q][w];
    }
  }
}

// A_iK = -A_iK P for every row i outside the block (one thread per row), and
// A_KK = P.
static __global__ void __launch_bounds__(kGjBS) gj_col_kernel(int n, double* __restrict__ A, int k0, int kb,
                                                              const double* __restrict__ P) {
  __shared__ double Ps[kGjB * kGjB];
  for (int e = threadIdx.x; e < kGjB * kGjB; e += kGjBS) Ps[e] = P[e];
  __syncthreads();
  const int i = blockIdx.x * kGjBS + threadIdx.x;
  if (i >= n) return;
  double* row = A + static_cast<int64_t>(i) * n + k0;
  if (i >= k0 && i < k0 + kb) {
    for (int c = 0; c < kb; ++c) row[c] = Ps[(i - k0) * kGjB + c];
    return;
  }
  double x[kGjB];
#pragma unroll
  for (int r = 0; r < kGjB; ++r) x[r] = r < kb ? row[r] : 0.0;
  for (int c = 0; c < kb; ++c) {
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < kGjB; ++r) s += x[r] * Ps[r * kGjB + c];
    row[c] = -s;
  }
}

// In-place inverse of the dense row-major n x n matrix A (device), scratch P
// of 64 x 64 doubles and the flag `bad` (cleared here).  Enqueued on s.
inline hipError_t gj_inverse_spd(int n, double* A, double* P, int* bad, hipStream_t s) {
  hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), s);
  if (e != hipSuccess) return e;
  const int nt = (n + kGjB - 1) / kGjB;
  const int lines = (n + kGjBS - 1) / kGjBS;
  for (int K = 0; K < nt; ++K) {
    const int k0 = K * kGjB, kb = (n - k0 < kGjB) ? n - k0 : kGjB;
    gj_diag_kernel<<<1, kGjBS, 0, s>>>(n, A, k0, kb, P, bad);
    gj_row_kernel<<<lines, kGjBS, 0, s>>>(n, A, k0, kb, P);
    gj_trailing_kernel<<<dim3(nt, nt), kGjBS, 0, s>>>(n, A, k0, kb);
    gj_col_kernel<<<lines, kGjBS, 0, s>>>(n, A, k0, kb, P);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace amg
