#pragma once
// Schur-complement pressure-correction preconditioner on the device (section
// 3, "Extensibility"; the Navier-Stokes runs of section 4).  For the system
// [[K, G], [D, S]] (velocity unknowns first) it applies to r = (r_u, r_p)
//   r_p' = r_p - (D diag(M_u)) r_u           SpMV, pressure rows
//   p    = V(S_hat; r_p')                    one V-cycle of the pressure
//                                            Schur complement's hierarchy
//   z_u  = M_u .* (r_u - G p)                SpMV, velocity rows
// with M_u the SPAI-0 diagonal of K.  The first step is u* = M_u r_u and
// r_p - D u* with M_u folded into D's values; the last is u* - M_u G p.
// The V-cycle runs in its own value type (FP32 in the mixed form); the two
// products and the vectors around them stay FP64.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "vcycle.hpp"

namespace amg {

// z_u = m .* (f - G p): the velocity back-substitution.
struct EpiSchurVelocity {
  static constexpr int K = 0;
  double* z;
  const double* m;
  const double* f;
  __device__ __forceinline__ void operator()(int i, double s, double*) const { z[i] = m[i] * (f[i] - s); }
};

// dst[j] = src[idx[j]] and dst[idx[j]] = src[j]: vectors between the
// caller's order and the velocity-first order (idx a permutation).
static __global__ void __launch_bounds__(kVecBS) gather_kernel(int n, double* dst, const double* src,
                                                               const int32_t* idx) {
  const int stride = gridDim.x * kVecBS;
  for (int j = blockIdx.x * kVecBS + threadIdx.x; j < n; j += stride) dst[j] = src[idx[j]];
}

static __global__ void __launch_bounds__(kVecBS) scatter_kernel(int n, double* dst, const double* src,
                                                                const int32_t* idx) {
  const int stride = gridDim.x * kVecBS;
  for (int j = blockIdx.x * kVecBS + threadIdx.x; j < n; j += stride) dst[idx[j]] = src[j];
}

struct SchurOps {
  const DevCsr<double>* Dm = nullptr;  // D diag(M_u): pressure rows, velocity columns
  const DevCsr<double>* G = nullptr;   // velocity rows, pressure columns
  const double* mu = nullptr;          // M_u
  double* rp = nullptr;                // r_p', the V-cycle's right-hand side
  int64_t n_u = 0;
};

template <class T>
class SchurPrecond {
 public:
  SchurPrecond(Vcycle<T> v, const SchurOps& o) : v_(v), o_(o) {}

  // z = M r over the whole system (r, z double[n]).  DOT (r . z, for CG)
  // is refused: the split is not symmetric.
  template <int DOT>
  int run(const double* r, double* z, double* partials, const int* skip, hipStream_t s) {
    if (DOT) throw DevError{AMG_ERR_INVALID_ARG, "the field split is not symmetric: CG is not available"};
    launch_spmv(*o_.Dm, GatherX<double, double>{r}, EpiResid<double, double>{o_.rp, r + o_.n_u}, nullptr, skip,
                s);
    v_.template run<0>(o_.rp, z + o_.n_u, partials, skip, s);
    launch_spmv(*o_.G, GatherX<double, double>{z + o_.n_u}, EpiSchurVelocity{z, o_.mu, r}, nullptr, skip, s);
    return 0;
  }

 private:
  Vcycle<T> v_;
  SchurOps o_;
};

}  // namespace amg
