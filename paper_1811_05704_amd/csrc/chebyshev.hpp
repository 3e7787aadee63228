#pragma once
// Chebyshev relaxation inside the V-cycle: the diagonally scaled Chebyshev
// iteration (Saad 2003, Alg. 12.1, with D = diag(A_l) as preconditioner), one
// of the relaxation choices listed in section 3.  For a spectrum of D^-1 A
// inside [lo, hi]: theta = (hi + lo) / 2, delta = (hi - lo) / 2,
// sigma = theta / delta, rho_0 = 1 / sigma.  From x with r = f - A x:
//   d = D^-1 r / theta;  then per step j = 0 .. k-1:
//   x += d;  r -= A d;  rho_{j+1} = 1 / (2 sigma - rho_j);
//   d = (rho_{j+1} rho_j) d + (2 rho_{j+1} / delta) D^-1 r.
// Every step is one SpMV with d gathered; the elementwise updates of x, r and
// the next d are fused into its epilogue (d ping-pongs between two buffers,
// x and r are updated in place, row by row).  The last update of x needs no
// product: unless the sweep's residual is wanted (the last pre-sweep, whose
// residual is restricted), it is folded into the step before it.

#include "kernels.hpp"

namespace amg {

constexpr int kMaxChebDegree = 16;

// Coefficients of one level's sweep, in the V-cycle's value type.
template <class T>
struct ChebCoef {
  int degree = 0;
  T theta = 0;
  T c1[kMaxChebDegree] = {};  // rho_{j+1} rho_j
  T c2[kMaxChebDegree] = {};  // 2 rho_{j+1} / delta
};

// Host-side coefficients from the spectrum bound hi and hi / lo = ratio;
// computed in FP64, then rounded to T.
template <class T>
inline ChebCoef<T> cheb_coefficients(double hi, double ratio, int degree) {
  ChebCoef<T> c;
  const double lo = hi / ratio;
  const double theta = 0.5 * (hi + lo);
  const double delta = 0.5 * (hi - lo);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  c.degree = degree;
  c.theta = static_cast<T>(theta);
  for (int j = 0; j + 1 < degree; ++j) {
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    c.c1[j] = static_cast<T>(rho_new * rho);
    c.c2[j] = static_cast<T>(2.0 * rho_new / delta);
    rho = rho_new;
  }
  return c;
}

// d_j = (m_j f_j) / theta: the first direction of a sweep from a zero guess,
// recomputed on the fly (level 1, whose right-hand side is the caller's).
template <class T, class TF>
struct GatherMFc {
  const T* m;
  const TF* f;
  T theta;
  __device__ __forceinline__ T operator()(int j) const { return (m[j] * static_cast<T>(f[j])) / theta; }
};

// f_c = R r, plus the next level's first direction (m_c .* f_c) / theta_c.
template <class T>
struct EpiRestrictCheb {
  static constexpr int K = 0;
  T* f;
  T* d0;
  const T* m;
  T theta;
  __device__ __forceinline__ void operator()(int i, T s, double*) const {
    f[i] = s;
    d0[i] = (m[i] * s) / theta;
  }
};

// Residual of a sweep that starts from x (s = (A x)_i): r = f - s,
// d = m .* r / theta.  FUSED (one-step sweep whose residual is not wanted):
// out = x + d instead, with dot += f . out when DOT.
template <class T, class TF, class TZ, int FUSED, int DOT>
struct EpiChebInit {
  static constexpr int K = DOT;
  const T* x;
  T* r;
  T* d;
  const T* m;
  const TF* f;
  T theta;
  TZ* out;
  __device__ __forceinline__ void operator()(int i, T s, double* acc) const {
    const T ri = static_cast<T>(f[i]) - s;
    const T di = (m[i] * ri) / theta;
    if constexpr (FUSED) {
      const TZ o = static_cast<TZ>(x[i] + di);
      out[i] = o;
      if constexpr (DOT) acc[0] += static_cast<double>(f[i]) * static_cast<double>(o);
    } else {
      r[i] = ri;
      d[i] = di;
    }
  }
};

// Step modes: kChebMid writes x, r and the next d; kChebLast writes x and r
// (the last step of a sweep whose residual is wanted); kChebFused forms the
// next d and writes out = (x + d) + d_next, the sweep's result.
enum ChebMode { kChebMid = 0, kChebLast = 1, kChebFused = 2 };

// One step with s = (A d)_i.  FROM_ZERO: first step of a sweep from a zero
// guess (x = 0, r = f; d is d0[i] when D0, else (m_i f_i) / theta).
template <class T, class TF, class TZ, int FROM_ZERO, int D0, int MODE, int DOT>
struct EpiChebStep {
  static constexpr int K = DOT;
  T* x;
  T* r;
  const T* d;   // current direction (FROM_ZERO && D0: the stored d0)
  T* dn;        // next direction
  const T* m;
  const TF* f;
  T theta, c1, c2;
  TZ* out;
  __device__ __forceinline__ void operator()(int i, T s, double* acc) const {
    T di, xi, ri;
    if constexpr (FROM_ZERO) {
      if constexpr (D0) di = d[i];
      else di = (m[i] * static_cast<T>(f[i])) / theta;
      xi = di;
      ri = static_cast<T>(f[i]) - s;
    } else {
      di = d[i];
      xi = x[i] + di;
      ri = r[i] - s;
    }
    if constexpr (MODE == kChebLast) {
      x[i] = xi;
      r[i] = ri;
    } else {
      const T dni = c1 * di + c2 * (m[i] * ri);
      if constexpr (MODE == kChebMid) {
        x[i] = xi;
        r[i] = ri;
        dn[i] = dni;
      } else {
        const TZ o = static_cast<TZ>(xi + dni);
        out[i] = o;
        if constexpr (DOT) acc[0] += static_cast<double>(f[i]) * static_cast<double>(o);
      }
    }
  }
};

// out = d0: a one-step sweep from a zero guess whose residual is not wanted
// (no product needed).  d0 stored (D0) or (m .* f) / theta.
template <class T, class TF, class TZ, int D0>
static __global__ void __launch_bounds__(kVecBS) cheb_first_kernel(int n, TZ* out, const T* d0, const T* m,
                                                                   const TF* f, T theta, const int* skip) {
  if (skip && *skip) return;
  const int stride = gridDim.x * kVecBS;
  for (int i = blockIdx.x * kVecBS + threadIdx.x; i < n; i += stride) {
    if constexpr (D0) out[i] = static_cast<TZ>(d0[i]);
    else out[i] = static_cast<TZ>((m[i] * static_cast<T>(f[i])) / theta);
  }
}

}  // namespace amg
