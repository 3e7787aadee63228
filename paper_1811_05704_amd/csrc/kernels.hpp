// gfx950 kernels of the AMG solve phase.
//
// The solve phase (section 2, "AMG solve"; section 3 names the two backend
// primitives it rests on) reduces to CSR sparse matrix-vector products with
// fused element-wise epilogues, vector updates and dot products.  Everything here is bandwidth bound (about 2
// flops per 12 bytes of matrix in FP64), so no matrix cores are used: the
// kernels are built around coalesced streaming of the CSR arrays, gathers of
// x that hit in L2, LDS-staged row sums and wave64 reductions.
//
// Two SpMV variants, chosen per matrix from its row lengths and size:
//  * stream: a workgroup takes a precomputed block of consecutive rows whose
//    entries fit in LDS (4, 8 or 16 KB of products), streams val/col of the
//    whole block with consecutive lanes on consecutive entries (perfectly
//    coalesced), stores the products in LDS, then G = 1, 4, 16 or 64 lanes
//    sum each row from LDS (every matrix of the hierarchy with mean row
//    length up to 512).  A row longer than the LDS block gets a block of its
//    own and is reduced by the whole workgroup.
//  * vector: 64 lanes per row straight from memory, strided loads within the
//    row and a butterfly reduction with lane shuffles (very long rows).
// Workgroups are remapped so that each of the 8 XCDs (each with its own L2)
// works on one contiguous range of rows, keeping x-gathers XCD-local.
//
// Reductions are deterministic: each workgroup writes one partial per dot
// product, and a one-workgroup finalize kernel sums the partials in a fixed
// order and updates the Krylov scalars on the device.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amg {

constexpr int kBS = 256;             // threads per workgroup for the sparse kernels
constexpr int kFinBS = 1024;         // finalize workgroup
constexpr int kNumXcd = 8;

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ int xcd_remap(int b, int nb) {
  // Blocks are dispatched round-robin over the XCDs; give XCD x the x-th
  // contiguous slice of the virtual block range.
  const int x = b % kNumXcd, local = b / kNumXcd;
  const int per = nb / kNumXcd, rem = nb % kNumXcd;
  return x < rem ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int G, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

// Sum K per-thread values over the workgroup; thread 0 writes them to
// partials[k * nparts + slot].
template <int K, int BS>
__device__ __forceinline__ void block_partials(const double* v, double* partials, int nparts,
                                               int slot) {
  if constexpr (K > 0) {
    __shared__ double sh[K][BS / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = wave_sum(v[k]);
      if (lane == 0) sh[k][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int w = 0; w < BS / 64; ++w) s += sh[k][w];
        partials[k * nparts + slot] = s;
      }
    }
  }
}

// ---------------------------------------------------------------- CSR views

template <class T>
struct CsrView {
  const int32_t* ptr;
  const int32_t* col;
  const T* val;
  const int32_t* blk;  // stream variant: first row of each block, nblocks + 1
  int32_t rows;
  int32_t nblocks;
  // Stream variant, optional: column of entry e = cbase[block] + col16[e]
  // for every block that fits in one LDS pass (NULL: read col).
  const uint16_t* col16;
  const int32_t* cbase;
};

// x-gathers ---------------------------------------------------------------

template <class T, class TX>
struct GatherX {
  const TX* x;
  __device__ __forceinline__ T operator()(int j) const { return static_cast<T>(x[j]); }
};

// x_j = m_j f_j: the first relaxation sweep from a zero guess, recomputed on
// the fly instead of stored.
template <class T, class TF>
struct GatherMF {
  const T* m;
  const TF* f;
  __device__ __forceinline__ T operator()(int j) const { return m[j] * static_cast<T>(f[j]); }
};

// Epilogues: called once per row with the row sum s = (A x)_i; may add to K
// dot-product partials.  ------------------------------------------------------

template <class T, class TY>
struct EpiStore {  // y = A x
  static constexpr int K = 0;
  TY* y;
  __device__ __forceinline__ void operator()(int i, T s, double*) const { y[i] = static_cast<TY>(s); }
};

struct EpiStoreDot {  // y = A x, dot += w . y   (FP64 Krylov)
  static constexpr int K = 1;
  double* y;
  const double* w;
  __device__ __forceinline__ void operator()(int i, double s, double* d) const {
    y[i] = s;
    d[0] += w[i] * s;
  }
};

struct EpiStoreDot2 {  // y = A x, dots += (w . y, y . y)
  static constexpr int K = 2;
  double* y;
  const double* w;
  __device__ __forceinline__ void operator()(int i, double s, double* d) const {
    y[i] = s;
    d[0] += w[i] * s;
    d[1] += s * s;
  }
};

// f_c = R r, plus m_c .* f_c: the next level's first relaxation sweep from a
// zero guess, gathered by its fused pre-sweep + residual kernel.
template <class T>
struct EpiRestrict {
  static constexpr int K = 0;
  T* f;
  T* mf;
  const T* m;
  __device__ __forceinline__ void operator()(int i, T s, double*) const {
    f[i] = s;
    mf[i] = m[i] * s;
  }
};

// r = b - A x, with ||r||^2 and ||b||^2 (FP64 Krylov initial / true residual)
struct EpiResidNorms {
  static constexpr int K = 2;
  double* r;
  const double* b;
  __device__ __forceinline__ void operator()(int i, double s, double* d) const {
    const double bi = b[i];
    const double ri = bi - s;
    r[i] = ri;
    d[0] += ri * ri;
    d[1] += bi * bi;
  }
};

// r = f - A x in the V-cycle's value type (f may be wider: level 1, mixed).
template <class T, class TF>
struct EpiResid {
  static constexpr int K = 0;
  T* r;
  const TF* f;
  __device__ __forceinline__ void operator()(int i, T s, double*) const {
    r[i] = static_cast<T>(f[i]) - s;
  }
};

// y = base + P z_c, base = m.*f (one pre-sweep), a stored vector, or zero.
template <class T, class TF, int BASE>  // BASE: 0 none, 1 m.*f, 2 stored
struct EpiProlong {
  static constexpr int K = 0;
  T* y;
  const T* m;
  const TF* f;
  const T* base;
  __device__ __forceinline__ void operator()(int i, T s, double*) const {
    if constexpr (BASE == 1) {
      y[i] = m[i] * static_cast<T>(f[i]) + s;
    } else if constexpr (BASE == 2) {
      y[i] = base[i] + s;
    } else {
      y[i] = s;
    }
  }
};

// One relaxation sweep z_out = z + m.*(f - A z); optionally dot += f . z_out
// in FP64 (level 1 of PCG: rho = r . z).
template <class T, class TF, class TZ, int DOT>
struct EpiSmooth {
  static constexpr int K = DOT;
  TZ* zout;
  const T* z;
  const T* m;
  const TF* f;
  __device__ __forceinline__ void operator()(int i, T s, double* d) const {
    const T v = z[i] + m[i] * (static_cast<T>(f[i]) - s);
    const TZ o = static_cast<TZ>(v);
    zout[i] = o;
    if constexpr (DOT) d[0] += static_cast<double>(f[i]) * static_cast<double>(o);
  }
};

// ---------------------------------------------------------------- SpMV kernels

// Products staged in LDS per stream block: AMG_STREAM_BYTES (16 KB: 2048
// FP64 or 4096 FP32 values, 8 or 16 per thread) for large matrices, and
// kStreamSmallBytes (4 KB) for matrices below kStreamSmallMatrix bytes of
// values, where the larger blocks would leave too few workgroups to hide
// memory latency (measured on the level matrices of the 150^3 hierarchy:
// 15-40% faster below 32 MB).  Larger matrices take the smallest block that
// holds one reduction pass (the schedule puts at most kBS / G rows in a
// block), kStreamMidBytes (8 KB; G = 1, 4, 16) or AMG_STREAM_BYTES.
#ifndef AMG_STREAM_BYTES
#define AMG_STREAM_BYTES 16384
#endif
constexpr int kStreamSmallBytes = 4096;
constexpr int kStreamMidBytes = 8192;
constexpr int64_t kStreamSmallMatrix = int64_t(32) << 20;

template <class T, int NB = AMG_STREAM_BYTES>
constexpr int stream_nnz() {
  return NB / static_cast<int>(sizeof(T));
}

constexpr int kStreamMaxRows = 1024;  // rows per stream block

// Stream variant.  Block vb covers rows [blk[vb], blk[vb+1]): either at most
// kStreamMaxRows rows with at most stream_nnz<T, NB>() entries, or a single
// longer row.  Phase 1: every lane loads its share of the block's val/col (all loads
// issued before any use; streamed with non-temporal hints so that L2 keeps x),
// gathers x and stores the products in LDS.  Phase 2: G lanes per row sum the
// row's products (strided, then a butterfly) and apply the epilogue.  The
// block's dot-product partials go to partials[k * nparts + vb].  `prod` is the
// caller's LDS buffer of at least stream_nnz<T, NB>() + kBS entries.
// C16: the matrix's 2-byte column offsets are read (the caller checked that
// A.col16 is set); -1: either, decided at run time.
template <int G, int NB, class T, class Gth, class E, int C16 = -1>
__device__ __forceinline__ void stream_block(const CsrView<T>& A, const Gth& gather, const E& epi, int vb,
                                             double* partials, int nparts, T* prod) {
  constexpr int NNZ = stream_nnz<T, NB>();
  constexpr int PER = NNZ / kBS;
  static_assert(PER * kBS == NNZ, "block entries must be a multiple of the workgroup size");
  const int r0 = A.blk[vb], r1 = A.blk[vb + 1];
  const int e0 = A.ptr[r0], e1 = A.ptr[r1];
  const int cnt = e1 - e0;
  const int tid = threadIdx.x;
  double d[E::K > 0 ? E::K : 1] = {};
  if (cnt <= NNZ) {
    if (cnt > 0) {
      // All loads of a lane are issued before any is used, and nothing is
      // predicated: surplus lanes re-read the block's last entry and park
      // their product in the spare slots.
      int c[PER];
      T v[PER];
      if (C16 == 1 || (C16 < 0 && A.col16)) {  // 2-byte offsets from the block's smallest column
        const int base = A.cbase[vb];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
          const int e = min(e0 + k * kBS + tid, e1 - 1);
          c[k] = base + static_cast<int>(__builtin_nontemporal_load(A.col16 + e));
          v[k] = __builtin_nontemporal_load(A.val + e);
        }
      } else {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
          const int e = min(e0 + k * kBS + tid, e1 - 1);
          c[k] = __builtin_nontemporal_load(A.col + e);
          v[k] = __builtin_nontemporal_load(A.val + e);
        }
      }
      T x[PER];
#pragma unroll
      for (int k = 0; k < PER; ++k) x[k] = gather(c[k]);
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int slot = k * kBS + tid;
        prod[slot < cnt ? slot : NNZ + tid] = v[k] * x[k];
      }
    }
    __syncthreads();
    const int lane = tid % G;
    for (int i = r0 + tid / G; i < r1; i += kBS / G) {
      const int b = A.ptr[i] - e0, e = A.ptr[i + 1] - e0;
      T s = T(0);
      for (int k = b + lane; k < e; k += G) s += prod[k];
      s = group_sum<G>(s);
      if (lane == 0) epi(i, s, d);
    }
  } else {
    // one long row: strided over the workgroup, then a fixed-order tree
    T s = T(0);
    for (int e = e0 + tid; e < e1; e += kBS) s += A.val[e] * gather(A.col[e]);
    s = group_sum<64>(s);
    if ((tid & 63) == 0) prod[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) {
      T t = T(0);
      for (int w = 0; w < kBS / 64; ++w) t += prod[w];
      epi(r0, t, d);
    }
  }
  if constexpr (E::K > 0) block_partials<E::K, kBS>(d, partials, nparts, vb);
}

// Column offsets of the stream schedule's blocks: cbase[vb] = the smallest
// column of block vb and col16[e] = col[e] - cbase[vb] for blocks of at
// most cap entries (longer single rows keep reading col; cbase 0); *bad = 1
// if a block spans more than 65536 columns.  One workgroup per block.
static __global__ void __launch_bounds__(kBS) compact_cols_kernel(const int32_t* ptr, const int32_t* col,
                                                                  const int32_t* blk, int cap, int32_t* cbase,
                                                                  uint16_t* col16, int32_t* bad) {
  __shared__ int wlo[kBS / 64], whi[kBS / 64];
  const int vb = blockIdx.x, tid = threadIdx.x;
  const int e0 = ptr[blk[vb]], e1 = ptr[blk[vb + 1]];
  if (e1 - e0 > cap || e1 == e0) {
    if (tid == 0) cbase[vb] = 0;
    return;
  }
  int lo = 0x7fffffff, hi = -1;
  for (int e = e0 + tid; e < e1; e += kBS) {
    lo = min(lo, col[e]);
    hi = max(hi, col[e]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = min(lo, __shfl_xor(lo, off, 64));
    hi = max(hi, __shfl_xor(hi, off, 64));
  }
  if ((tid & 63) == 0) {
    wlo[tid >> 6] = lo;
    whi[tid >> 6] = hi;
  }
  __syncthreads();
  lo = wlo[0];
  hi = whi[0];
#pragma unroll
  for (int w = 1; w < kBS / 64; ++w) {
    lo = min(lo, wlo[w]);
    hi = max(hi, whi[w]);
  }
  if (hi - lo > 65535) {
    if (tid == 0) *bad = 1;
    return;
  }
  if (tid == 0) cbase[vb] = lo;
  for (int e = e0 + tid; e < e1; e += kBS) col16[e] = static_cast<uint16_t>(col[e] - lo);
}

template <int G, int NB, class T, class Gth, class E, int C16>
static __global__ void __launch_bounds__(kBS) csr_stream_kernel(CsrView<T> A, Gth gather, E epi,
                                                         double* partials, const int* skip) {
  if (skip && *skip) return;
  __shared__ T prod[stream_nnz<T, NB>() + kBS];  // the last kBS slots take surplus lanes' products
  stream_block<G, NB, T, Gth, E, C16>(A, gather, epi, xcd_remap(blockIdx.x, gridDim.x), partials, gridDim.x,
                                      prod);
}

// Vector variant: L lanes per row, kBS / L rows per workgroup.  Block vb
// covers rows [vb * kBS / L, (vb + 1) * kBS / L); its dot-product partials go
// to partials[k * nparts + vb].
template <int L, class T, class G, class E>
__device__ __forceinline__ void vector_block(const CsrView<T>& A, const G& gather, const E& epi, int vb,
                                             double* partials, int nparts) {
  constexpr int RPB = kBS / L;
  const int i = vb * RPB + threadIdx.x / L;
  const int lane = threadIdx.x % L;
  double d[E::K > 0 ? E::K : 1] = {};
  T s = T(0);
  if (i < A.rows) {
    const int b = A.ptr[i], e = A.ptr[i + 1];
    for (int k = b + lane; k < e; k += L) s += A.val[k] * gather(A.col[k]);
  }
  s = group_sum<L>(s);
  if (i < A.rows && lane == 0) epi(i, s, d);
  if constexpr (E::K > 0) block_partials<E::K, kBS>(d, partials, nparts, vb);
}

template <int L, class T, class G, class E>
static __global__ void __launch_bounds__(kBS) csr_vector_kernel(CsrView<T> A, G gather, E epi,
                                                         double* partials, const int* skip) {
  if (skip && *skip) return;
  vector_block<L>(A, gather, epi, xcd_remap(blockIdx.x, gridDim.x), partials, gridDim.x);
}

// ---------------------------------------------------------------- Krylov scalars

// Device-resident Krylov state; the host reads it only to poll convergence.
enum : int32_t {
  kRunning = 0,
  kConverged = 1,
  kMaxIter = 2,
  kBreakdown = 3,
  kNonFinite = 4,
  kZeroRhs = 5,
  kHalfStep = 6,  // BiCGStab met tol after the first half step
};

struct KState {
  double rho, rho1, alpha, beta, omega;
  double ff, tol2, rr, true_rr;
  double tol;
  int32_t iters, done, max_iter, first;
};

// Finalize operations (one workgroup): sums of the partials are in s[].
enum FinOp : int {
  kFinInit = 0,       // s = (r.r, f.f) of r = f - A x0
  kFinTrue = 1,       // s = (r.r, f.f) of the true residual at exit
  kFinAlpha = 2,      // PCG: s = p.q -> alpha = rho / p.q
  kFinPcgRR = 3,      // PCG: s = r.r -> iteration done, test convergence
  kFinPcgRho = 4,     // PCG: s = r.z -> beta, rho
  kFinBiAlpha = 5,    // BiCGStab: s = rt.v -> alpha
  kFinBiS = 6,        // BiCGStab: s = s.s -> iteration counted, half-step test
  kFinBiOmega = 7,    // BiCGStab: s = (t.s, t.t) -> omega
  kFinBiR = 8,        // BiCGStab: s = (r.r, rt.r) -> convergence, rho, beta
  kFinBiHalfDone = 9, // BiCGStab: half-step exit completed
};

template <int K>
__device__ __forceinline__ void finalize_body(const double* partials, int nparts, KState* st, int op) {
  const bool always = (op == kFinInit || op == kFinTrue || op == kFinBiHalfDone);
  if (!always && st->done != kRunning) return;
  if (op == kFinBiHalfDone) {
    if (threadIdx.x == 0 && st->done == kHalfStep) st->done = kConverged;
    return;
  }
  __shared__ double sh[K][kFinBS / 64];
  double s[2] = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double* p = partials + k * nparts;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int b = threadIdx.x;
    for (; b + 3 * kFinBS < nparts; b += 4 * kFinBS) {
      a0 += p[b];
      a1 += p[b + kFinBS];
      a2 += p[b + 2 * kFinBS];
      a3 += p[b + 3 * kFinBS];
    }
    for (; b < nparts; b += kFinBS) a0 += p[b];
    double a = wave_sum((a0 + a1) + (a2 + a3));
    if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = a;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double a = 0.0;
    for (int w = 0; w < kFinBS / 64; ++w) a += sh[k][w];
    s[k] = a;
  }
  auto bad = [](double v) { return !isfinite(v); };
  switch (op) {
    case kFinInit: {
      st->rr = s[0];
      st->ff = s[1];
      st->tol2 = st->tol * st->tol * s[1];
      if (s[1] == 0.0) st->done = kZeroRhs;
      else if (bad(s[0]) || bad(s[1])) st->done = kNonFinite;
      else if (s[0] <= st->tol2) st->done = kConverged;
      else st->done = kRunning;
      st->first = 1;
      st->rho = s[0];  // BiCGStab: rt = r, so rt . r = r . r
      st->rho1 = st->alpha = st->omega = 1.0;
      break;
    }
    case kFinTrue:
      st->true_rr = s[0];
      break;
    case kFinAlpha:
      if (bad(s[0]) || s[0] == 0.0) { st->done = bad(s[0]) ? kNonFinite : kBreakdown; break; }
      st->alpha = st->rho / s[0];
      st->first = 0;
      break;
    case kFinPcgRR:
      st->rr = s[0];
      st->iters += 1;
      if (bad(s[0])) st->done = kNonFinite;
      else if (s[0] <= st->tol2) st->done = kConverged;
      else if (st->iters >= st->max_iter) st->done = kMaxIter;
      break;
    case kFinPcgRho:
      if (bad(s[0])) { st->done = kNonFinite; break; }
      st->beta = st->first ? 0.0 : s[0] / st->rho;
      st->rho = s[0];
      break;
    case kFinBiAlpha:
      if (bad(s[0]) || s[0] == 0.0) { st->done = bad(s[0]) ? kNonFinite : kBreakdown; break; }
      st->alpha = st->rho / s[0];
      break;
    case kFinBiS:
      st->iters += 1;
      st->rr = s[0];
      if (bad(s[0])) st->done = kNonFinite;
      else if (s[0] <= st->tol2) st->done = kHalfStep;
      break;
    case kFinBiOmega:
      if (bad(s[0]) || bad(s[1]) || s[1] == 0.0) { st->done = kBreakdown; break; }
      st->omega = s[0] / s[1];
      break;
    case kFinBiR: {
      st->rr = s[0];
      if (bad(s[0]) || bad(s[1])) { st->done = kNonFinite; break; }
      if (s[0] <= st->tol2) { st->done = kConverged; break; }
      if (st->omega == 0.0) { st->done = kBreakdown; break; }
      if (st->iters >= st->max_iter) { st->done = kMaxIter; break; }
      st->rho1 = st->rho;
      st->rho = s[1];
      if (s[1] == 0.0) { st->done = kBreakdown; break; }
      st->beta = (st->rho / st->rho1) * (st->alpha / st->omega);
      st->first = 0;
      break;
    }
    default:
      break;
  }
}

template <int K>
static __global__ void __launch_bounds__(kFinBS) finalize_kernel(const double* partials, int nparts,
                                                               KState* st, int op) {
  finalize_body<K>(partials, nparts, st, op);
}

// ---------------------------------------------------------------- vector kernels (FP64)

constexpr int kVecBS = 256;

__device__ __forceinline__ int vec_grid_start() {
  return xcd_remap(blockIdx.x, gridDim.x) * kVecBS + threadIdx.x;
}

// x += alpha p; r -= alpha q; partial r.r.  Block vb of nb handles indices
// vb*kVecBS + tid + k*nb*kVecBS and writes partial slot vb.
__device__ __forceinline__ void pcg_update_block(int n, double* x, double* r, const double* p, const double* q,
                                                 const KState* st, double* partials, int vb, int nb) {
  const double alpha = st->alpha;
  double d[1] = {0.0};
  const int stride = nb * kVecBS;
  for (int i = vb * kVecBS + threadIdx.x; i < n; i += stride) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    d[0] += ri * ri;
  }
  block_partials<1, kVecBS>(d, partials, nb, vb);
}

static __global__ void __launch_bounds__(kVecBS) pcg_update_kernel(int n, double* x, double* r,
                                                                   const double* p, const double* q,
                                                                   const KState* st, double* partials) {
  if (st->done != kRunning) return;
  pcg_update_block(n, x, r, p, q, st, partials, xcd_remap(blockIdx.x, gridDim.x), gridDim.x);
}

// p = z + beta p  (p = z on the first iteration)
__device__ __forceinline__ void pcg_dir_block(int n, double* p, const double* z, const KState* st, int vb,
                                              int nb) {
  const double beta = st->beta;
  const bool first = st->first;
  const int stride = nb * kVecBS;
  for (int i = vb * kVecBS + threadIdx.x; i < n; i += stride) p[i] = first ? z[i] : z[i] + beta * p[i];
}

static __global__ void __launch_bounds__(kVecBS) pcg_dir_kernel(int n, double* p, const double* z,
                                                                const KState* st) {
  if (st->done != kRunning) return;
  pcg_dir_block(n, p, z, st, xcd_remap(blockIdx.x, gridDim.x), gridDim.x);
}

// BiCGStab: p = r (first) or p = r + beta (p - omega v)
static __global__ void __launch_bounds__(kVecBS) bicg_p_kernel(int n, double* p, const double* r,
                                                        const double* v, const KState* st) {
  if (st->done != kRunning) return;
  const double beta = st->beta, omega = st->omega;
  const bool first = st->first;
  const int stride = gridDim.x * kVecBS;
  for (int i = vec_grid_start(); i < n; i += stride)
    p[i] = first ? r[i] : r[i] + beta * (p[i] - omega * v[i]);
}

// BiCGStab: s = r - alpha v; partial s.s
static __global__ void __launch_bounds__(kVecBS) bicg_s_kernel(int n, double* s, const double* r,
                                                        const double* v, const KState* st,
                                                        double* partials) {
  if (st->done != kRunning) return;
  const double alpha = st->alpha;
  double d[1] = {0.0};
  const int stride = gridDim.x * kVecBS;
  for (int i = vec_grid_start(); i < n; i += stride) {
    const double si = r[i] - alpha * v[i];
    s[i] = si;
    d[0] += si * si;
  }
  block_partials<1, kVecBS>(d, partials, gridDim.x, xcd_remap(blockIdx.x, gridDim.x));
}

// BiCGStab half-step exit: x += alpha p_hat (only when the s-test passed)
static __global__ void __launch_bounds__(kVecBS) bicg_half_kernel(int n, double* x, const double* phat,
                                                           const KState* st) {
  if (st->done != kHalfStep) return;
  const double alpha = st->alpha;
  const int stride = gridDim.x * kVecBS;
  for (int i = vec_grid_start(); i < n; i += stride) x[i] += alpha * phat[i];
}

// BiCGStab: x += alpha p_hat + omega s_hat; r = s - omega t; partials r.r, rt.r
static __global__ void __launch_bounds__(kVecBS) bicg_xr_kernel(int n, double* x, double* r,
                                                         const double* phat, const double* shat,
                                                         const double* s, const double* t,
                                                         const double* rt, const KState* st,
                                                         double* partials) {
  if (st->done != kRunning) return;
  const double alpha = st->alpha, omega = st->omega;
  double d[2] = {0.0, 0.0};
  const int stride = gridDim.x * kVecBS;
  for (int i = vec_grid_start(); i < n; i += stride) {
    x[i] += alpha * phat[i] + omega * shat[i];
    const double ri = s[i] - omega * t[i];
    r[i] = ri;
    d[0] += ri * ri;
    d[1] += rt[i] * ri;
  }
  block_partials<2, kVecBS>(d, partials, gridDim.x, xcd_remap(blockIdx.x, gridDim.x));
}

template <class TD, class TS>
static __global__ void __launch_bounds__(kVecBS) copy_kernel(int n, TD* dst, const TS* src) {
  const int stride = gridDim.x * kVecBS;
  for (int i = blockIdx.x * kVecBS + threadIdx.x; i < n; i += stride)
    dst[i] = static_cast<TD>(src[i]);
}

template <class T>
static __global__ void __launch_bounds__(kVecBS) fill_kernel(int n, T* dst, T v) {
  const int stride = gridDim.x * kVecBS;
  for (int i = blockIdx.x * kVecBS + threadIdx.x; i < n; i += stride) dst[i] = v;
}

// z = m .* f   (first pre-sweep from zero, materialised when npre > 1)
template <class T, class TF>
static __global__ void __launch_bounds__(kVecBS) scale_kernel(int n, T* z, const T* m, const TF* f,
                                                       const int* skip) {
  if (skip && *skip) return;
  const int stride = gridDim.x * kVecBS;
  for (int i = blockIdx.x * kVecBS + threadIdx.x; i < n; i += stride)
    z[i] = m[i] * static_cast<T>(f[i]);
}

// ---------------------------------------------------------------- coarse solve

// z = Ainv f with the dense inverse of the coarsest operator (FP64, row-major),
// one workgroup per row, FP64 accumulation; f and z in the V-cycle's types.
template <class TF, class TZ>
__device__ __forceinline__ void coarse_row(int n, const double* __restrict__ Ainv, const TF* __restrict__ f,
                                           TZ* __restrict__ z, int row) {
  const double* a = Ainv + static_cast<int64_t>(row) * n;
  double s0 = 0.0, s1 = 0.0;
  int j = threadIdx.x;
  for (; j + kBS < n; j += 2 * kBS) {
    s0 += a[j] * static_cast<double>(f[j]);
    s1 += a[j + kBS] * static_cast<double>(f[j + kBS]);
  }
  if (j < n) s0 += a[j] * static_cast<double>(f[j]);
  double s = wave_sum(s0 + s1);
  __shared__ double sh[kBS / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBS / 64; ++w) t += sh[w];
    z[row] = static_cast<TZ>(t);
  }
}

template <class TF, class TZ>
__global__ void __launch_bounds__(kBS) coarse_gemv_kernel(int n, const double* __restrict__ Ainv,
                                                          const TF* __restrict__ f, TZ* __restrict__ z,
                                                          const int* skip) {
  if (skip && *skip) return;
  coarse_row<TF, TZ>(n, Ainv, f, z, blockIdx.x);
}

// partials of a . b (FP64)
static __global__ void __launch_bounds__(kVecBS) dot_kernel(int n, const double* a, const double* b,
                                                     double* partials, const int* skip) {
  if (skip && *skip) return;
  double d[1] = {0.0};
  const int stride = gridDim.x * kVecBS;
  for (int i = vec_grid_start(); i < n; i += stride) d[0] += a[i] * b[i];
  block_partials<1, kVecBS>(d, partials, gridDim.x, xcd_remap(blockIdx.x, gridDim.x));
}

// zout = y (no post-sweep); optionally partials of f . zout
template <class T, class TF, class TZ, int DOT>
static __global__ void __launch_bounds__(kVecBS) copy_dot_kernel(int n, TZ* zout, const T* y, const TF* f,
                                                          double* partials, const int* skip) {
  if (skip && *skip) return;
  double d[1] = {0.0};
  const int stride = gridDim.x * kVecBS;
  for (int i = vec_grid_start(); i < n; i += stride) {
    const TZ o = static_cast<TZ>(y[i]);
    zout[i] = o;
    if constexpr (DOT) d[0] += static_cast<double>(f[i]) * static_cast<double>(o);
  }
  if constexpr (DOT) block_partials<1, kVecBS>(d, partials, gridDim.x, xcd_remap(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------- batched kernels (serving)
//
// One launch runs the same step of many independent solves.  A batch lists,
// per live solve, its operands and its number of work blocks; the fixed grid
// strides over the concatenated blocks.  Each block does exactly what the
// corresponding block of the single-solve kernel does (same rows, same
// partial slot, same summation order), so every solve's result is bitwise the
// same alone and in any mix.

constexpr int kMaxSlots = 64;

template <class Item>
struct Batch {
  int n;                     // live items
  int total;                 // total work blocks
  int off[kMaxSlots + 1];    // first work block of each item
  Item it[kMaxSlots];
};

__device__ __forceinline__ int batch_item(const int* off, int n, int w) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= w) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <class T, class Gth, class E>
struct SpmvItem {
  CsrView<T> A;
  Gth g;
  E e;
  double* partials;
  const int* skip;
  int kind;    // 0 stream (block table A.blk), 1 vector (64 lanes per row)
  int lanes;
  int bclass;  // stream block size class: 0 = 16 KB, 1 = 4 KB, 2 = 8 KB
};

// (lanes, block class) pairs of the stream schedule that the batched kernel
// dispatches; the host checks every item against it before a launch.
__host__ __device__ constexpr bool stream_dispatchable(int lanes, int bclass) {
  return (lanes == 1 || lanes == 4 || lanes == 16) ? (bclass >= 0 && bclass <= 2)
         : (lanes == 64)                            ? (bclass == 0 || bclass == 1)
                                                    : false;
}

template <class T, class Gth, class E>
__global__ void __launch_bounds__(kBS) batched_spmv_kernel(const Batch<SpmvItem<T, Gth, E>>* B) {
  __shared__ T prod[stream_nnz<T>() + kBS];
  const int n = B->n, total = B->total;
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int i = batch_item(B->off, n, w);
    const SpmvItem<T, Gth, E> it = B->it[i];
    if (!*it.skip) {
      const int vb = w - B->off[i], nb = B->off[i + 1] - B->off[i];
      constexpr int NS = kStreamSmallBytes, NM = kStreamMidBytes, NL = AMG_STREAM_BYTES;
      if (it.kind == 1) vector_block<64>(it.A, it.g, it.e, vb, it.partials, nb);
      else switch (it.lanes * 4 + it.bclass) {
        case 4: stream_block<1, NL, T, Gth, E, 0>(it.A, it.g, it.e, vb, it.partials, nb, prod); break;
        case 5: stream_block<1, NS, T, Gth, E, 0>(it.A, it.g, it.e, vb, it.partials, nb, prod); break;
        case 6: stream_block<1, NM, T, Gth, E, 0>(it.A, it.g, it.e, vb, it.partials, nb, prod); break;
        case 16: stream_block<4, NL, T, Gth, E, 0>(it.A, it.g, it.e, vb, it.partials, nb, prod); break;
        case 17: stream_block<4, NS, T, Gth, E, 0>(it.A, it.g, it.e, vb, it.partials, nb, prod); break;
        case 18: stream_block<4, NM, T, Gth, E, 0>(it.A, it.g, it.e, vb, it.partials, nb, prod); break;
        case 64: stream_block<16, NL, T, Gth, E, 0>(it.A, it.g, it.e, vb, it.partials, nb, prod); break;
        case 65: stream_block<16, NS, T, Gth, E, 0>(it.A, it.g, it.e, vb, it.partials, nb, prod); break;
        case 66: stream_block<16, NM, T, Gth, E, 0>(it.A, it.g, it.e, vb, it.partials, nb, prod); break;
        case 256: stream_block<64, NL, T, Gth, E, 0>(it.A, it.g, it.e, vb, it.partials, nb, prod); break;
        default: stream_block<64, NS, T, Gth, E, 0>(it.A, it.g, it.e, vb, it.partials, nb, prod); break;
      }
    }
    __syncthreads();
  }
}

struct UpdItem {
  int n;
  double* x;
  double* r;
  const double* p;
  const double* q;
  const KState* st;
  double* partials;
};

static __global__ void __launch_bounds__(kVecBS) batched_update_kernel(const Batch<UpdItem>* B) {
  const int n = B->n, total = B->total;
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int i = batch_item(B->off, n, w);
    const UpdItem it = B->it[i];
    if (it.st->done == kRunning)
      pcg_update_block(it.n, it.x, it.r, it.p, it.q, it.st, it.partials, w - B->off[i], B->off[i + 1] - B->off[i]);
    __syncthreads();
  }
}

struct DirItem {
  int n;
  double* p;
  const double* z;
  const KState* st;
};

static __global__ void __launch_bounds__(kVecBS) batched_dir_kernel(const Batch<DirItem>* B) {
  const int n = B->n, total = B->total;
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int i = batch_item(B->off, n, w);
    const DirItem it = B->it[i];
    if (it.st->done == kRunning) pcg_dir_block(it.n, it.p, it.z, it.st, w - B->off[i], B->off[i + 1] - B->off[i]);
  }
}

struct FinItem {
  const double* partials;
  int nparts;
  KState* st;
};

template <int K>
__global__ void __launch_bounds__(kFinBS) batched_finalize_kernel(const Batch<FinItem>* B, int op) {
  for (int w = blockIdx.x; w < B->n; w += gridDim.x) {
    const FinItem it = B->it[w];
    finalize_body<K>(it.partials, it.nparts, it.st, op);
    __syncthreads();
  }
}

template <class T>
struct GemvItem {
  int n;
  const double* Ainv;
  const T* f;
  T* z;
  const int* skip;
};

template <class T>
__global__ void __launch_bounds__(kBS) batched_gemv_kernel(const Batch<GemvItem<T>>* B) {
  const int n = B->n, total = B->total;
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int i = batch_item(B->off, n, w);
    const GemvItem<T> it = B->it[i];
    if (!*it.skip) coarse_row<T, T>(it.n, it.Ainv, it.f, it.z, w - B->off[i]);
    __syncthreads();
  }
}

}  // namespace amg
