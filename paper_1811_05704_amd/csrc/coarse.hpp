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

// P = A_KK^-1 for the kb x kb diagonal block at k0 (Gauss-Jordan in place,
// one workgroup); bad = 1 if a pivot is not positive.  Thread t keeps 16
// entries of row t / 4 (columns 16 (t % 4) ..) in registers; each pivot step
// publishes the scaled pivot row and the pivot column through LDS (double
// buffered, two barriers per step).
static __global__ void __launch_bounds__(kGjBS) gj_diag_kernel(int n, const double* __restrict__ A, int k0, int kb,
                                                               double* __restrict__ P, int* bad) {
  static_assert(kGjB == 64 && kGjBS == 256, "thread layout: 64 rows x 4 column groups");
  __shared__ double prow[2][kGjB];
  __shared__ double fcol[2][kGjB];
  __shared__ double pdiag[2];
  const int t = threadIdx.x;
  const int r = t >> 2, c0 = (t & 3) * 16;
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int c = c0 + q;
    v[q] = (r < kb && c < kb) ? A[static_cast<int64_t>(k0 + r) * n + k0 + c] : 0.0;
  }
  if (t == 0) pdiag[0] = v[0];  // D[0][0]
  __syncthreads();
  for (int k = 0; k < kb; ++k) {
    const int b = k & 1;
    const double p = pdiag[b];
    if (t == 0 && !(p > 0.0)) *bad = 1;
    if (r == k) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        v[q] = (c0 + q == k ? 1.0 : v[q]) / p;
        prow[b][c0 + q] = v[q];
      }
    }
    if ((k >> 4) == (t & 3)) {
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (c0 + q == k) fcol[b][r] = v[q];
    }
    __syncthreads();
    if (r != k) {
      const double f = fcol[b][r];
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = (c0 + q == k ? 0.0 : v[q]) - f * prow[b][c0 + q];
    }
    if (r == k + 1 && ((k + 1) >> 4) == (t & 3)) {
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (c0 + q == k + 1) pdiag[1 - b] = v[q];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) P[r * kGjB + c0 + q] = (r < kb && c0 + q < kb) ? v[q] : 0.0;  // zero outside kb x kb
}

// A_Kj = P A_Kj for every column j outside the block: a workgroup takes four
// columns, stages their kb-entry segments in LDS and writes 64 x 4 outputs.
static __global__ void __launch_bounds__(kGjBS) gj_row_kernel(int n, double* __restrict__ A, int k0, int kb,
                                                              const double* __restrict__ P) {
  __shared__ double X[kGjB][4];
  const int t = threadIdx.x;
  const int r = t >> 2, jq = t & 3;
  const int j = blockIdx.x * 4 + jq;
  const bool col_ok = j < n && !(j >= k0 && j < k0 + kb);
  X[r][jq] = (col_ok && r < kb) ? A[static_cast<int64_t>(k0 + r) * n + j] : 0.0;
  __syncthreads();
  if (!col_ok || r >= kb) return;
  const double* pr = P + r * kGjB;
  double s = 0.0;
  for (int c = 0; c < kb; ++c) s += pr[c] * X[c][jq];
  A[static_cast<int64_t>(k0 + r) * n + j] = s;
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

// A_iK = -A_iK P for every row i outside the block, and A_KK = P: a
// workgroup takes four rows, stages their kb-entry segments in LDS and writes
// 4 x 64 outputs.
static __global__ void __launch_bounds__(kGjBS) gj_col_kernel(int n, double* __restrict__ A, int k0, int kb,
                                                              const double* __restrict__ P) {
  __shared__ double X[4][kGjB];
  const int t = threadIdx.x;
  const int iq = t >> 6, c = t & 63;
  const int i = blockIdx.x * 4 + iq;
  const bool row_ok = i < n;
  double* row = A + static_cast<int64_t>(i) * n + k0;
  const bool in_block = i >= k0 && i < k0 + kb;
  X[iq][c] = (row_ok && !in_block && c < kb) ? row[c] : 0.0;
  __syncthreads();
  if (!row_ok || c >= kb) return;
  if (in_block) {
    row[c] = P[(i - k0) * kGjB + c];
    return;
  }
  double s = 0.0;
  for (int q = 0; q < kb; ++q) s += X[iq][q] * P[q * kGjB + c];
  row[c] = -s;
}

// In-place inverse of the dense row-major n x n matrix A (device), scratch P
// of 64 x 64 doubles and the flag `bad` (cleared here).  Enqueued on s.
inline hipError_t gj_inverse_spd(int n, double* A, double* P, int* bad, hipStream_t s) {
  hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), s);
  if (e != hipSuccess) return e;
  const int nt = (n + kGjB - 1) / kGjB;
  const int quads = (n + 3) / 4;
  for (int K = 0; K < nt; ++K) {
    const int k0 = K * kGjB, kb = (n - k0 < kGjB) ? n - k0 : kGjB;
    gj_diag_kernel<<<1, kGjBS, 0, s>>>(n, A, k0, kb, P, bad);
    gj_row_kernel<<<quads, kGjBS, 0, s>>>(n, A, k0, kb, P);
    gj_trailing_kernel<<<dim3(nt, nt), kGjBS, 0, s>>>(n, A, k0, kb);
    gj_col_kernel<<<quads, kGjBS, 0, s>>>(n, A, k0, kb, P);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace amg
