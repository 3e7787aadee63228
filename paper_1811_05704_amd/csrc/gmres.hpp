#pragma once
// Flexible restarted GMRES(m) on the device: GMRES is one of the iterative
// solvers of section 3; the flexible form (Saad 1993; Saad 2003, Alg. 9.6)
// keeps z_j = M v_j so that x += Z_k y is exact also for the FP32 V-cycle.
// Arnoldi orthogonalisation is classical Gram-Schmidt applied twice (Giraud,
// Langou and Rozloznik 2005): each pass is one batched dot-product kernel
// (all j+1 products against the same w), one fixed-order summation kernel and
// one fused subtract kernel.  The Hessenberg column, the Givens rotations and
// the least-squares residual are updated by one thread on the device, so the
// host only polls a stop flag.
//
// Per Arnoldi step j (every kernel returns at once when GState::stop is set):
//   z_j = M v_j (V-cycle); w = A z_j;
//   twice: c_i = v_i . w (i <= j), w -= sum_i c_i v_i, h += c;
//   ||w|| fused into the second subtract; rotations; v_{j+1} = w / ||w||.
// End of a cycle (k steps): y = R_k^-1 g_k; x += sum_i y_i z_i; r = f - A x;
// the next cycle starts from r, and its norm decides convergence.

#include "kernels.hpp"

namespace amg {

constexpr int kMaxGmresM = 64;
constexpr int kGmDotBlocks = 1024;  // most workgroups of a dot / subtract pass

// Device-resident GMRES state.  H is column-major with leading dimension
// kMaxGmresM + 1.
struct GState {
  int32_t k;     // Arnoldi steps done in the current cycle
  int32_t stop;  // the current cycle has ended (or the solve has)
  double hn;     // ||w|| of the last step
  double H[(kMaxGmresM + 1) * kMaxGmresM];
  double cs[kMaxGmresM], sn[kMaxGmresM];
  double g[kMaxGmresM + 1], y[kMaxGmresM];
  double h[kMaxGmresM + 1];   // coefficients of the current column (both passes)
  double hp[kMaxGmresM + 1];  // coefficients of the current pass
};

// Sum of p[0 .. np) by one workgroup of kFinBS threads in a fixed order:
// strided per-thread sums, wavefront butterflies, then the waves in order.
// The total is returned in thread 0.
// Safe to call repeatedly in one kernel (the staging array is reused only
// after every thread has passed the barrier of the previous call).
__device__ __forceinline__ double gm_block_total(const double* p, int np) {
  __shared__ double sh[kFinBS / 64];
  double a = 0.0;
  for (int b = threadIdx.x; b < np; b += kFinBS) a += p[b];
  a = wave_sum(a);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kFinBS / 64; ++w) t += sh[w];
  return t;
}

// Partials of v_i . w for i = blockIdx.y (grid: nb x (j + 1)).
static __global__ void __launch_bounds__(kVecBS) gm_dots_kernel(int n, const double* V, int64_t ldv,
                                                                const double* w, double* partials,
                                                                const GState* G) {
  if (G->stop) return;
  const int i = blockIdx.y, nb = gridDim.x, b = blockIdx.x;
  const double* v = V + static_cast<int64_t>(i) * ldv;
  double d[1] = {0.0};
  for (int idx = b * kVecBS + threadIdx.x; idx < n; idx += nb * kVecBS) d[0] += v[idx] * w[idx];
  block_partials<1, kVecBS>(d, partials + static_cast<int64_t>(i) * nb, nb, b);
}

// c_i = sum of the partials of row i (one workgroup per i); pass 0 sets
// h = c, pass 1 adds c to h.
static __global__ void __launch_bounds__(kFinBS) gm_sum_kernel(const double* partials, int nb, GState* G,
                                                               int pass) {
  if (G->stop) return;
  const int i = blockIdx.x;
  const double t = gm_block_total(partials + static_cast<int64_t>(i) * nb, nb);
  if (threadIdx.x == 0) {
    G->hp[i] = t;
    G->h[i] = pass ? G->h[i] + t : t;
  }
}

// w -= sum_{i < k} c_i v_i (i in order); NORM: partials of ||w||^2.
template <int NORM>
static __global__ void __launch_bounds__(kVecBS) gm_subtract_kernel(int n, int k, const double* V, int64_t ldv,
                                                                    double* w, double* partials, const GState* G) {
  if (G->stop) return;
  const int nb = gridDim.x, b = blockIdx.x;
  double d[1] = {0.0};
  for (int idx = b * kVecBS + threadIdx.x; idx < n; idx += nb * kVecBS) {
    double wi = w[idx];
    for (int i = 0; i < k; ++i) wi = wi - G->hp[i] * V[static_cast<int64_t>(i) * ldv + idx];
    w[idx] = wi;
    if constexpr (NORM) d[0] += wi * wi;
  }
  if constexpr (NORM) block_partials<1, kVecBS>(d, partials, nb, b);
}

// Column j of the Hessenberg matrix from h and ||w||, the earlier rotations
// applied, a new rotation, the least-squares residual |g_{j+1}|; stop the
// cycle on convergence, ||w|| = 0, the iteration limit or j = m - 1.
static __global__ void __launch_bounds__(kFinBS) gm_givens_kernel(const double* partials, int nb, GState* G,
                                                                  KState* st, int j, int m) {
  if (G->stop) return;
  const double ww = gm_block_total(partials, nb);
  if (threadIdx.x != 0) return;
  constexpr int ld = kMaxGmresM + 1;
  double* Hj = G->H + static_cast<int64_t>(j) * ld;
  const double hn = sqrt(ww);
  for (int i = 0; i <= j; ++i) Hj[i] = G->h[i];
  Hj[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double a = Hj[i], b = Hj[i + 1];
    Hj[i] = G->cs[i] * a + G->sn[i] * b;
    Hj[i + 1] = -G->sn[i] * a + G->cs[i] * b;
  }
  const double a = Hj[j], b = Hj[j + 1];
  const double d = sqrt(a * a + b * b);
  G->cs[j] = a / d;
  G->sn[j] = b / d;
  Hj[j] = d;
  Hj[j + 1] = 0.0;
  G->g[j + 1] = -G->sn[j] * G->g[j];
  G->g[j] = G->cs[j] * G->g[j];
  G->hn = hn;
  G->k = j + 1;
  st->iters += 1;
  const double rr = G->g[j + 1] * G->g[j + 1];
  st->rr = rr;
  if (!isfinite(rr) || !isfinite(d) || d == 0.0) {
    st->done = kNonFinite;
    G->stop = 1;
  } else if (rr <= st->tol2 || hn == 0.0 || st->iters >= st->max_iter || j == m - 1) {
    G->stop = 1;
  }
}

// v_{j+1} = w / ||w||
static __global__ void __launch_bounds__(kVecBS) gm_scale_kernel(int n, double* v, const double* w,
                                                                 const GState* G) {
  if (G->stop) return;
  const double hn = G->hn;
  const int stride = gridDim.x * kVecBS;
  for (int i = vec_grid_start(); i < n; i += stride) v[i] = w[i] / hn;
}

// y = R_k^-1 g_k by back substitution (one thread; k <= 64).
static __global__ void gm_solve_kernel(GState* G, const KState* st) {
  if (st->done != kRunning || threadIdx.x != 0) return;
  constexpr int ld = kMaxGmresM + 1;
  const int k = G->k;
  for (int i = k - 1; i >= 0; --i) {
    double s = G->g[i];
    for (int c = i + 1; c < k; ++c) s = s - G->H[static_cast<int64_t>(c) * ld + i] * G->y[c];
    G->y[i] = s / G->H[static_cast<int64_t>(i) * ld + i];
  }
}

// x += sum_{i < k} y_i z_i (i in order)
static __global__ void __launch_bounds__(kVecBS) gm_update_kernel(int n, double* x, const double* Z, int64_t ldz,
                                                                  const GState* G, const KState* st) {
  if (st->done != kRunning) return;
  const int k = G->k;
  const int stride = gridDim.x * kVecBS;
  for (int idx = vec_grid_start(); idx < n; idx += stride) {
    double xi = x[idx];
    for (int i = 0; i < k; ++i) xi = xi + G->y[i] * Z[static_cast<int64_t>(i) * ldz + idx];
    x[idx] = xi;
  }
}

// Start of a cycle from r = f - A x, with s = (r.r, f.f) summed from the
// residual kernel's partials.  FIRST: the initial residual (sets ||f||, the
// target, zero right-hand side); otherwise a restart (skipped once the solve
// has ended).  Convergence of the true residual, the iteration limit and
// non-finite values end the solve; otherwise the cycle is opened.
static __global__ void __launch_bounds__(kFinBS) gm_start_state_kernel(const double* partials, int nb, KState* st,
                                                                       GState* G, int first) {
  if (!first && st->done != kRunning) return;
  const double rr = gm_block_total(partials, nb);
  const double ff = gm_block_total(partials + nb, nb);
  if (threadIdx.x != 0) return;
  if (first) {
    st->ff = ff;
    st->tol2 = st->tol * st->tol * ff;
    st->done = kRunning;
    if (ff == 0.0) st->done = kZeroRhs;
  }
  st->rr = rr;
  st->true_rr = rr;
  if (st->done == kRunning) {
    if (!isfinite(rr) || !isfinite(ff)) st->done = kNonFinite;
    else if (rr <= st->tol2) st->done = kConverged;
    else if (st->iters >= st->max_iter) st->done = kMaxIter;
  }
  G->k = 0;
  G->stop = (st->done != kRunning);
  G->g[0] = sqrt(rr);
}

// v_0 = r / ||r|| when a cycle opens.
static __global__ void __launch_bounds__(kVecBS) gm_first_vector_kernel(int n, double* v, const double* r,
                                                                        const GState* G) {
  if (G->stop) return;
  const double beta = G->g[0];
  const int stride = gridDim.x * kVecBS;
  for (int i = vec_grid_start(); i < n; i += stride) v[i] = r[i] / beta;
}

}  // namespace amg
