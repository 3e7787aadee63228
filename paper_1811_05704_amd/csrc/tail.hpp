// The coarse end of the V-cycle as one persistent launch.
//
// Below some size a level's kernels are too short to fill the chip: each of
// the four sparse products of a level (pre-sweep + residual, restriction,
// prolongation + correction, post-sweep) and the coarse solve (section 2,
// "AMG solve") costs a launch, a ramp-up and a drain for a few microseconds
// of work.  Here every level from `first` down to the coarsest runs inside one
// launch of G workgroups that are all resident at once: each step is a phase
// over the same stream blocks, rows and epilogues as the one-kernel-per-step
// path, and a grid-wide barrier separates consecutive phases.  Each block is
// computed exactly as by the standalone kernel (same rows, same summation
// order), so the result is bitwise the same whichever path runs.
//
// The barrier waits a bounded time: a wait that runs out sets an error flag,
// every workgroup then leaves, and the host reports the error; no launch can
// hang on it.  Its counters return to zero when the last workgroup leaves,
// so consecutive launches (and graph replays) reuse them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace amg {

constexpr int kTailMaxLevels = 6;

struct TailSync {
  unsigned int arrive;  // barrier arrivals in the running launch
  unsigned int leave;   // workgroups that left the running launch
  int error;            // a barrier wait ran out of time
  int pad;
};

// A level matrix with its SpMV schedule.
template <class T>
struct TailMat {
  CsrView<T> A;
  int kind, lanes, bclass;
};

template <class T>
struct TailLevel {
  TailMat<T> A, P, R;
  T* f;         // right-hand side (written by the restriction above)
  T* mf;        // m .* f (written with it)
  const T* m;   // smoother diagonal
  T* r;         // residual
  T* y;         // prolongated correction
  T* z;         // output
  T* fnext;     // next level's f (or the coarsest right-hand side)
  T* mfnext;    // next level's m .* f (NULL when the next level is the coarsest)
  const T* mnext;
};

template <class T>
struct TailPlan {
  int nlev;  // levels first .. first + nlev - 1; the next one is the coarsest
  TailLevel<T> lev[kTailMaxLevels];
  const double* Ainv;  // dense inverse of the coarsest operator, row-major
  int nL;
  T* fL;
  T* zL;
  TailSync* sync;
  uint64_t limit;  // longest barrier wait, in wall-clock ticks
};

// Grid-wide barrier number `k` (0-based) of a launch of G workgroups.  Every
// thread makes its own stores visible device-wide first; one thread per
// workgroup counts in and waits for the count to reach (k + 1) G.  Returns
// false if this wait, or another workgroup's, ran out of time.
__device__ __forceinline__ bool tail_barrier(TailSync* sy, unsigned int target, uint64_t limit) {
  __shared__ int ok;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    int good = 1;
    if (__hip_atomic_load(&sy->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      good = 0;
    } else {
      __hip_atomic_fetch_add(&sy->arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint64_t t0 = wall_clock64();
      while (__hip_atomic_load(&sy->arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(&sy->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          good = 0;
          break;
        }
        if (wall_clock64() - t0 > limit) {
          __hip_atomic_store(&sy->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          good = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __threadfence();  // what the other workgroups wrote before arriving is visible now
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

// Called once by every workgroup at the end of a launch (also after a
// failed wait).  The last one to leave resets the counters: by then every
// workgroup has passed its last barrier, so nobody reads them again.
__device__ __forceinline__ void tail_leave(TailSync* sy) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int prev = __hip_atomic_fetch_add(&sy->leave, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == gridDim.x - 1) {
      __hip_atomic_store(&sy->arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&sy->leave, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// One sparse product of a phase: the matrix's blocks split into eight
// contiguous ranges, one per XCD (workgroups are dispatched round-robin over
// the XCDs), each range strided over that XCD's workgroups.
template <class T, class Gth, class E>
__device__ __forceinline__ void tail_spmv(const TailMat<T>& M, const Gth& g, const E& e, T* prod) {
  const int nb = M.A.nblocks;
  const int G = gridDim.x;
  const int x = blockIdx.x % kNumXcd, j = blockIdx.x / kNumXcd;
  const int gx = G / kNumXcd + (x < G % kNumXcd ? 1 : 0);
  const int per = nb / kNumXcd, rem = nb % kNumXcd;
  const int b0 = x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per;
  const int b1 = b0 + per + (x < rem ? 1 : 0);
  constexpr int NS = kStreamSmallBytes, NM = kStreamMidBytes, NL = AMG_STREAM_BYTES;
  for (int vb = b0 + j; vb < b1; vb += gx) {
    if (M.kind == 1) vector_block<64>(M.A, g, e, vb, nullptr, 0);
    else switch (M.lanes * 4 + M.bclass) {
      case 4: stream_block<1, NL>(M.A, g, e, vb, nullptr, 0, prod); break;
      case 5: stream_block<1, NS>(M.A, g, e, vb, nullptr, 0, prod); break;
      case 6: stream_block<1, NM>(M.A, g, e, vb, nullptr, 0, prod); break;
      case 16: stream_block<4, NL>(M.A, g, e, vb, nullptr, 0, prod); break;
      case 17: stream_block<4, NS>(M.A, g, e, vb, nullptr, 0, prod); break;
      case 18: stream_block<4, NM>(M.A, g, e, vb, nullptr, 0, prod); break;
      case 64: stream_block<16, NL>(M.A, g, e, vb, nullptr, 0, prod); break;
      case 65: stream_block<16, NS>(M.A, g, e, vb, nullptr, 0, prod); break;
      case 66: stream_block<16, NM>(M.A, g, e, vb, nullptr, 0, prod); break;
      case 256: stream_block<64, NL>(M.A, g, e, vb, nullptr, 0, prod); break;
      default: stream_block<64, NS>(M.A, g, e, vb, nullptr, 0, prod); break;
    }
    __syncthreads();  // prod is reused by the next block
  }
}

// The tail of one V-cycle with one pre- and one post-sweep per level (zero
// initial guess, so the pre-sweep is m .* f, which the restriction above
// already wrote).  Per level, down: r = f - A (m .* f); f_next = R r (and
// m_next .* f_next).  Coarsest: z_L = A_L^-1 f_L.  Per level, up:
// y = m .* f + P z_next; z = y + m .* (f - A y).
template <class T>
__global__ void __launch_bounds__(kBS) vcycle_tail_kernel(TailPlan<T> P, const int* skip) {
  if (skip && *skip) return;
  __shared__ T prod[stream_nnz<T>() + kBS];
  TailSync* sy = P.sync;
  const unsigned int G = gridDim.x;
  unsigned int k = 0;  // barriers passed
  bool ok = true;
  for (int l = 0; l < P.nlev && ok; ++l) {
    const TailLevel<T>& L = P.lev[l];
    tail_spmv(L.A, GatherX<T, T>{L.mf}, EpiResid<T, T>{L.r, L.f}, prod);
    ok = tail_barrier(sy, ++k * G, P.limit);
    if (!ok) break;
    if (L.mfnext)
      tail_spmv(L.R, GatherX<T, T>{L.r}, EpiRestrict<T>{L.fnext, L.mfnext, L.mnext}, prod);
    else
      tail_spmv(L.R, GatherX<T, T>{L.r}, EpiStore<T, T>{L.fnext}, prod);
    ok = tail_barrier(sy, ++k * G, P.limit);
  }
  if (ok) {
    for (int row = blockIdx.x; row < P.nL; row += G) {
      coarse_row<T, T>(P.nL, P.Ainv, P.fL, P.zL, row);
      __syncthreads();
    }
    ok = tail_barrier(sy, ++k * G, P.limit);
  }
  for (int l = P.nlev - 1; l >= 0 && ok; --l) {
    const TailLevel<T>& L = P.lev[l];
    const T* zc = (l + 1 < P.nlev) ? P.lev[l + 1].z : P.zL;
    tail_spmv(L.P, GatherX<T, T>{zc}, EpiProlong<T, T, 2>{L.y, L.m, L.f, L.mf}, prod);
    ok = tail_barrier(sy, ++k * G, P.limit);
    if (!ok) break;
    tail_spmv(L.A, GatherX<T, T>{L.y}, EpiSmooth<T, T, T, 0>{L.z, L.y, L.m, L.f}, prod);
    if (l > 0) ok = tail_barrier(sy, ++k * G, P.limit);
  }
  tail_leave(sy);
}

// Clears a tail's error flag and counters (after a reported failure).
static __global__ void tail_reset_kernel(TailSync* sy) {
  if (threadIdx.x == 0) {
    sy->arrive = 0;
    sy->leave = 0;
    sy->error = 0;
  }
}

}  // namespace amg
