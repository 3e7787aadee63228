// Block values on the device (section 3, "Value types": matrix entries that
// are small static 4 x 4 matrices, one per pair of coupled grid nodes).
//
// Storage is block CSR: one int32 column per block and its 16 values
// contiguous (row-major), so a block costs 128 bytes of values plus 4 of
// index in FP64 (136 against 192 for the same entries in scalar CSR).
//
// SpMV: a group of 4 SUB lanes owns one block row; lane (q, u) accumulates
// row q of the block row over the blocks u, u + SUB, ... .  The four lanes
// with the same u read one block as one contiguous 128-byte (FP64) line and
// share one 32-byte gather of x.  SUB = 1 for short block rows (each lane sums
// its scalar row in column order, as a sequential CSR product does) and 4 for
// long ones (four partial sums, then a fixed butterfly).  After the sums,
// every lane of the group holds the group's four row results, so epilogues
// can apply a 4 x 4 smoother block to them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace amg {

constexpr int kB = 4;
constexpr int kB2 = kB * kB;

template <class T>
struct BsrView {
  const int32_t* ptr;
  const int32_t* col;
  const T* val;  // 16 per block, row-major
  int32_t rows;  // block rows
};

// A scalar epilogue applied to scalar row 4 i + q.
template <class E>
struct PerRow {
  static constexpr int K = E::K;
  E e;
  template <class T>
  __device__ __forceinline__ void operator()(int i, int q, const T* s4, double* d) const {
    e(kB * i + q, s4[q], d);
  }
};

// f_c = R r and the next level's first sweep from zero, mf_c = M_c f_c.
template <class T>
struct EpiBRestrict {
  static constexpr int K = 0;
  T* f;
  T* mf;
  const T* M;
  __device__ __forceinline__ void operator()(int i, int q, const T* s4, double*) const {
    f[kB * i + q] = s4[q];
    const T* m = M + static_cast<int64_t>(i) * kB2 + q * kB;
    T v = m[0] * s4[0];
    v = v + m[1] * s4[1];
    v = v + m[2] * s4[2];
    v = v + m[3] * s4[3];
    mf[kB * i + q] = v;
  }
};

// Level 1: y = M f + P z_c (the pre-sweep from zero recomputed).
template <class T, class TF>
struct EpiBProlongMF {
  static constexpr int K = 0;
  T* y;
  const T* M;
  const TF* f;
  __device__ __forceinline__ void operator()(int i, int q, const T* s4, double*) const {
    const T* m = M + static_cast<int64_t>(i) * kB2 + q * kB;
    const TF* fi = f + kB * i;
    T v = m[0] * static_cast<T>(fi[0]);
    v = v + m[1] * static_cast<T>(fi[1]);
    v = v + m[2] * static_cast<T>(fi[2]);
    v = v + m[3] * static_cast<T>(fi[3]);
    y[kB * i + q] = v + s4[q];
  }
};

// Post-sweep z = y + M^T (f - A y), the adjoint of the pre-sweep; with DOT
// also dot += f . z in FP64 (level 1 of PCG: rho = r . z).
template <class T, class TF, class TZ, int DOT>
struct EpiBSmooth {
  static constexpr int K = DOT;
  TZ* z;
  const T* y;
  const T* M;
  const TF* f;
  __device__ __forceinline__ void operator()(int i, int q, const T* s4, double* d) const {
    const T* m = M + static_cast<int64_t>(i) * kB2 + q;  // column q of M_i = row q of M_i^T
    const TF* fi = f + kB * i;
    T v = m[0] * (static_cast<T>(fi[0]) - s4[0]);
    v = v + m[kB] * (static_cast<T>(fi[1]) - s4[1]);
    v = v + m[2 * kB] * (static_cast<T>(fi[2]) - s4[2]);
    v = v + m[3 * kB] * (static_cast<T>(fi[3]) - s4[3]);
    const TZ o = static_cast<TZ>(y[kB * i + q] + v);
    z[kB * i + q] = o;
    if constexpr (DOT) d[0] += static_cast<double>(fi[q]) * static_cast<double>(o);
  }
};

// SUB lanes per block-row component; kBS / (4 SUB) block rows per workgroup.
// Block row i = vb * rows-per-block + group; its dot partials go to
// partials[k * nparts + vb].
template <int SUB, class T, class Gth, class E>
__device__ __forceinline__ void bsr_block(const BsrView<T>& A, const Gth& gather, const E& epi, int vb,
                                          double* partials, int nparts) {
  constexpr int GS = kB * SUB;
  constexpr int RPB = kBS / GS;
  const int tid = threadIdx.x;
  const int i = vb * RPB + tid / GS;
  const int q = (tid % GS) / SUB, u = tid % SUB;
  double d[E::K > 0 ? E::K : 1] = {};
  T s = T(0);
  if (i < A.rows) {
    const int b = A.ptr[i], e = A.ptr[i + 1];
    // FP32: the blocks of U iterations are loaded and gathered before they
    // are summed (in the same order), the last block re-read past the row's
    // end; this took the FP32 block V-cycle from 625 to 571 us at 96^3 nodes
    // and made the FP64 one 1 % slower, which keeps one block at a time.
    constexpr int U = sizeof(T) == 4 ? 4 : 1;
    for (int k0 = b + u; k0 < e; k0 += U * SUB) {
      int jj[U];
      T vv[U][kB];
#pragma unroll
      for (int t = 0; t < U; ++t) {
        const int k = min(k0 + t * SUB, e - 1);
        jj[t] = kB * A.col[k];
        const T* v = A.val + static_cast<int64_t>(k) * kB2 + q * kB;
#pragma unroll
        for (int c = 0; c < kB; ++c) vv[t][c] = v[c];
      }
      T xx[U][kB];
#pragma unroll
      for (int t = 0; t < U; ++t)
#pragma unroll
        for (int c = 0; c < kB; ++c) xx[t][c] = gather(jj[t] + c);
#pragma unroll
      for (int t = 0; t < U; ++t) {
        if (k0 + t * SUB < e) {
          s = s + vv[t][0] * xx[t][0];
          s = s + vv[t][1] * xx[t][1];
          s = s + vv[t][2] * xx[t][2];
          s = s + vv[t][3] * xx[t][3];
        }
      }
    }
  }
  s = group_sum<SUB>(s);
  // the group's four row results in every lane of the group
  const int base = (tid & 63) - (tid % GS);
  T s4[kB];
#pragma unroll
  for (int t = 0; t < kB; ++t) s4[t] = __shfl(s, base + t * SUB, 64);
  if (i < A.rows && u == 0) epi(i, q, s4, d);
  if constexpr (E::K > 0) block_partials<E::K, kBS>(d, partials, nparts, vb);
}

template <int SUB, class T, class Gth, class E>
static __global__ void __launch_bounds__(kBS) bsr_kernel(BsrView<T> A, Gth gather, E epi, double* partials,
                                                        const int* skip) {
  if (skip && *skip) return;
  bsr_block<SUB>(A, gather, epi, xcd_remap(blockIdx.x, gridDim.x), partials, gridDim.x);
}

}  // namespace amg
