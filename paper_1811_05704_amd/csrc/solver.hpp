#pragma once
// Solve phase on the device: Krylov drivers, solver object, device setup.
//
// Section 2 ("AMG solve") and its closing remark: one V-cycle (vcycle.hpp) is
// one preconditioning step of a Krylov method.  Section 3: the hierarchy is set
// up once (its data-parallel steps on the device, the rest on the CPU) and
// reused for every right-hand side; smoothers and Krylov methods are
// expressed with the backend's primitives (here: fused HIP kernels on gfx950).
//
// The Krylov loop (PCG, BiCGStab or flexible GMRES) is FP64; its scalars
// (alpha, beta, omega, convergence flag) live on the device.  For PCG and
// BiCGStab one iteration is a fixed sequence of kernels that is captured once
// into a hipGraph and replayed; the host polls the flag every few iterations.
// Kernels early-exit once the flag is set, so replays past convergence are
// no-ops and the iteration count stays exact.  GMRES launches its kernels
// directly and polls a per-cycle stop flag (gmres.hpp).

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "chebyshev.hpp"
#include "device.hpp"
#include "block_device.hpp"
#include "coarse.hpp"
#include "field_split.hpp"
#include "galerkin.hpp"
#include "gmres.hpp"
#include "schur.hpp"
#include "tail.hpp"
#include "vcycle.hpp"

namespace amg {

inline thread_local std::string g_last_error;

inline amg_status set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return static_cast<amg_status>(code);
}

inline double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ solver object

}  // namespace amg

struct amg_solver {
  amg_params prm{};
  amg::HostHierarchy host;
  double setup_s = 0.0;
  bool on_device = false;
  int device = 0;

  std::unique_ptr<amg::DevArena> arena;
  hipStream_t cap_stream = nullptr;

  amg::DevCsr<double> A0;  // FP64 fine operator for the Krylov loop
  amg::DevHierarchy<double> h64;
  amg::DevHierarchy<float> h32;

  // Block values (4 x 4 per node): host hierarchy, FP64 fine operator and
  // the device hierarchies; the scalar members above stay empty.
  bool block = false;
  amg::BlockHierarchy bhost;
  amg::DevBsr<double> B0;
  amg::DevBlockHierarchy<double> bh64;
  amg::DevBlockHierarchy<float> bh32;
  double* Ainv = nullptr;
  int32_t nL = 0;
  int64_t n = 0;

  // Schur-complement field split: the hierarchy above (host, A0, h64/h32)
  // is that of the approximate pressure Schur complement; the Krylov loop
  // runs on the whole system Afull (n unknowns, velocity first).
  bool schur = false;
  amg::FieldSplit split;  // host copies: whole system, D diag(M_u), G, M_u
  amg::DevCsr<double> Afull, Dm, Gs;
  double* mu = nullptr;
  double* rp = nullptr;
  int32_t* perm = nullptr;  // caller's index of each velocity-first unknown (NULL: same order)

  amg::KState* st = nullptr;
  amg::KState* st_host = nullptr;  // pinned mirror for polling
  double* partials = nullptr;
  // Krylov vectors
  double *f = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *tmp = nullptr;
  double *rt = nullptr, *v = nullptr, *phat = nullptr, *s = nullptr, *shat = nullptr, *t = nullptr;

  // flexible GMRES: bases V ((m+1) x ld) and Z (m x ld), state, partials
  double *gmV = nullptr, *gmZ = nullptr, *gm_partials = nullptr;
  amg::GState* gm = nullptr;
  int32_t* gm_host = nullptr;  // pinned mirror of GState::k, GState::stop
  int64_t gm_ld = 0;
  int gm_nb = 0;

  hipGraphExec_t iter_exec = nullptr;
  hipGraph_t iter_graph = nullptr;
  // GMRES: one graph per group of check_every Arnoldi steps of a cycle, and
  // one for the end of a cycle (with the next cycle's start)
  std::vector<hipGraphExec_t> gm_execs;
  std::vector<hipGraph_t> gm_graphs;

  ~amg_solver() {
    if (iter_exec) (void)hipGraphExecDestroy(iter_exec);
    if (iter_graph) (void)hipGraphDestroy(iter_graph);
    for (auto e : gm_execs) (void)hipGraphExecDestroy(e);
    for (auto g : gm_graphs) (void)hipGraphDestroy(g);
    if (st_host) (void)hipHostFree(st_host);
    if (gm_host) (void)hipHostFree(gm_host);
    arena.reset();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

namespace amg {

inline SetupParams setup_params(const amg_params& p) {
  SetupParams s;
  s.relax = p.relax;
  s.eps_strong = p.eps_strong;
  s.jacobi_omega = p.jacobi_omega;
  s.coarse_enough = p.coarse_enough;
  s.max_levels = p.max_levels;
  return s;
}

inline void check_params(const amg_params& p) {
  if (p.solver != AMG_CG && p.solver != AMG_BICGSTAB && p.solver != AMG_GMRES)
    throw SetupError{-1, "solver must be AMG_CG, AMG_BICGSTAB or AMG_GMRES"};
  if (p.solver == AMG_GMRES && (p.gmres_m < 1 || p.gmres_m > kMaxGmresM))
    throw SetupError{-1, "gmres_m must be in [1, 64]"};
  if (p.relax != AMG_SPAI0 && p.relax != AMG_JACOBI && p.relax != AMG_CHEBYSHEV)
    throw SetupError{-1, "relax must be AMG_SPAI0, AMG_JACOBI or AMG_CHEBYSHEV"};
  if (p.relax == AMG_CHEBYSHEV) {
    if (p.cheb_degree < 1 || p.cheb_degree > kMaxChebDegree) throw SetupError{-1, "cheb_degree must be in [1, 16]"};
    if (!(p.cheb_ratio > 1.0)) throw SetupError{-1, "cheb_ratio must be > 1"};
  }
  if (p.precision != AMG_FP64 && p.precision != AMG_MIXED) throw SetupError{-1, "precision must be AMG_FP64 or AMG_MIXED"};
  if (p.npre < 0 || p.npost < 0 || p.npre > 16 || p.npost > 16) throw SetupError{-1, "npre/npost must be in [0, 16]"};
  if (p.coarse_enough < 1 || p.max_levels < 1 || p.max_iter < 1) throw SetupError{-1, "coarse_enough, max_levels, max_iter must be >= 1"};
  if (!(p.tol >= 0.0) || !(p.eps_strong >= 0.0)) throw SetupError{-1, "tol and eps_strong must be >= 0"};
  if (p.check_every < 1 || p.check_every > 64) throw SetupError{-1, "check_every must be in [1, 64]"};
  if (p.fuse_coarse != 0 && p.fuse_coarse != 1) throw SetupError{-1, "fuse_coarse must be 0 or 1"};
}

// Settings the block path implements: CG or BiCGStab, SPAI-0 or Jacobi
// blocks, 0 .. 16 pre- and post-sweeps (checked with the scalar settings).
inline void check_block_params(const amg_params& p) {
  if (p.solver != AMG_CG && p.solver != AMG_BICGSTAB && p.solver != AMG_GMRES)
    throw SetupError{-1, "block values: solver must be AMG_CG, AMG_BICGSTAB or AMG_GMRES"};
  if (p.relax != AMG_SPAI0 && p.relax != AMG_JACOBI)
    throw SetupError{-1, "block values: relax must be AMG_SPAI0 or AMG_JACOBI"};
}

inline Csr to_csr(int64_t n, const int64_t* ptr, const int32_t* col, const double* val) {
  Csr A;
  A.rows = A.cols = n;
  A.ptr.resize(n + 1);
  A.col.resize(ptr[n]);
  A.val.resize(ptr[n]);
  copy_parallel(A.ptr.data(), ptr, sizeof(int64_t) * (n + 1));
  copy_parallel(A.col.data(), col, sizeof(int32_t) * ptr[n]);
  copy_parallel(A.val.data(), val, sizeof(double) * ptr[n]);
  return A;
}

// M = I (n x n, dense)
static __global__ void __launch_bounds__(kVecBS) identity_kernel(int n, double* M) {
  const int64_t total = static_cast<int64_t>(n) * n;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kVecBS;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * kVecBS + threadIdx.x; k < total; k += stride)
    M[k] = (k / n == k % n) ? 1.0 : 0.0;
}

// Row i of the dense row-major n x n matrix M from row i of a CSR matrix:
// zeros, then the stored entries (one workgroup per row; columns unique).
static __global__ void __launch_bounds__(kVecBS) dense_rows_kernel(int n, const int32_t* ptr, const int32_t* col,
                                                                   const double* val, double* M) {
  const int i = blockIdx.x;
  double* row = M + static_cast<int64_t>(i) * n;
  for (int j = threadIdx.x; j < n; j += kVecBS) row[j] = 0.0;
  __syncthreads();
  for (int e = ptr[i] + threadIdx.x; e < ptr[i + 1]; e += kVecBS) row[col[e]] = val[e];
}

// Symmetry up to rounding of a CSR matrix with ascending columns:
// |a_ij - a_ji| <= 1e-12 sqrt(|a_ii a_jj|) for every stored entry (a missing
// a_ji counts as 0).  A Galerkin product R A P of a symmetric A with R = P^T
// is symmetric in exact arithmetic; its two triangles differ only by the
// order in which their sums were rounded.
inline bool symmetric_to_rounding(const Csr& M) {
  std::vector<double> d(M.rows, 0.0);
  for (int64_t i = 0; i < M.rows; ++i)
    for (int64_t e = M.ptr[i]; e < M.ptr[i + 1]; ++e)
      if (M.col[e] == i) d[i] = std::fabs(M.val[e]);
  for (int64_t i = 0; i < M.rows; ++i)
    for (int64_t e = M.ptr[i]; e < M.ptr[i + 1]; ++e) {
      const int32_t j = M.col[e];
      if (j == i) continue;
      const auto b = M.col.begin() + M.ptr[j], en = M.col.begin() + M.ptr[j + 1];
      const auto it = std::lower_bound(b, en, static_cast<int32_t>(i));
      const double aji = (it != en && *it == i) ? M.val[it - M.col.begin()] : 0.0;
      if (!(std::fabs(M.val[e] - aji) <= 1e-12 * std::sqrt(d[i] * d[j]))) return false;
    }
  return true;
}

// rocBLAS and rocSOLVER are entered by one thread at a time.  The serving
// workers set up requests side by side, each with its own handle; entered
// from two workers at once, rocBLAS's kernel-library initialisation has
// failed and aborted the process.  Every call into either library (handle
// creation and destruction included) holds this lock, so its lazy
// initialisation also runs under it.  The device work those calls enqueue
// still runs asynchronously on each caller's stream.
inline std::unique_lock<std::mutex> blas_lock() {
  static std::mutex mu;
  return std::unique_lock<std::mutex>(mu);
}

// Dense inverse of the coarsest operator on the device (FP64), in two steps:
// an LU factorisation, then n triangular solves against I (rocsolver getrs).
// A matrix symmetric to rounding is first factored without pivoting
// (getrf_npvt, about 3 times faster than getrf at orders 1,000-3,000); that
// factorisation is kept only if every pivot is positive, which for a
// symmetric matrix says it is positive definite, where elimination without
// pivoting is backward stable.  Otherwise, and for every nonsymmetric
// matrix, a fresh copy is factored with partial pivoting (getrf).  The dense
// copy is expanded on the device from the CSR matrix (the host never holds
// the n^2 array); its row-major layout read as column-major is A^T, and
// inv(A^T) read back as row-major is inv(A).  rocsolver's in-place getri is
// not used: on the ROCm 7.2 / gfx950 stack it returns a wrong inverse for
// some orders (for example 255, 511, 895, 1023; getrf and getrs are correct
// there), so the inverse is also checked once: Ainv (A v) must reproduce a
// known vector v.  Cholesky (potrf) is not used: run from several threads at
// once (the serving workers) it does not reproduce its own results.
inline void coarse_inverse(amg_solver& S, const Csr& AL, hipStream_t stream, const amg_allocator* alloc,
                           rocblas_handle shared = nullptr) {
  const int32_t n = static_cast<int32_t>(AL.rows);
  S.Ainv = S.arena->get<double>(static_cast<size_t>(n) * n);
  DevArena tmp(alloc, stream);  // CSR copy, LU factors, pivots, check vectors: freed on return
  const std::vector<int32_t> p32(AL.ptr.begin(), AL.ptr.end());
  const int32_t* dptr = tmp.upload(p32.data(), p32.size());
  const int32_t* dcol = tmp.upload(AL.col.data(), AL.col.size());
  const double* dval = tmp.upload(AL.val.data(), AL.val.size());
  auto expand_into = [&](double* M) {
    dense_rows_kernel<<<n, kVecBS, 0, stream>>>(n, dptr, dcol, dval, M);
    AMG_LAUNCHED();
  };
  // the check vectors: w = A v on the host, z = Ainv w on the device
  std::vector<double> v(n), w(n, 0.0), z(n);
  for (int32_t i = 0; i < n; ++i) v[i] = 1.0 + (i % 7) / 8.0;
  for (int32_t i = 0; i < n; ++i)
    for (int64_t e = AL.ptr[i]; e < AL.ptr[i + 1]; ++e) w[i] += AL.val[e] * v[AL.col[e]];
  double* wd = tmp.upload(w.data(), w.size());
  double* zd = tmp.get<double>(n);
  // largest relative error of z against v (a wrong inverse is off by O(1);
  // ill-conditioning up to about 1e12 stays below 1e-3)
  auto check_error = [&]() {
    coarse_gemv_kernel<double, double><<<n, kBS, 0, stream>>>(n, S.Ainv, wd, zd, nullptr);
    AMG_LAUNCHED();
    AMG_HIP(hipMemcpyAsync(z.data(), zd, sizeof(double) * n, hipMemcpyDeviceToHost, stream));
    AMG_HIP(hipStreamSynchronize(stream));
    double err = 0.0;
    for (int32_t i = 0; i < n; ++i) err = std::max(err, std::fabs(z[i] - v[i]) / v[i]);
    return err;
  };
  if (symmetric_to_rounding(AL)) {
    expand_into(S.Ainv);
    double* P = tmp.get<double>(kGjB * kGjB);
    int* bad = tmp.get<int>(1);
    AMG_HIP(gj_inverse_spd(n, S.Ainv, P, bad, stream));
    int hbad = 0;
    AMG_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, stream));
    AMG_HIP(hipStreamSynchronize(stream));
    if (!hbad && check_error() <= 1e-3) return;
    // not positive definite (or not accurate enough): LU with pivoting below
  }
  double* lu = tmp.get<double>(static_cast<size_t>(n) * n);
  expand_into(lu);
  identity_kernel<<<std::min<int64_t>((static_cast<int64_t>(n) * n + kVecBS - 1) / kVecBS, 65536), kVecBS, 0,
                    stream>>>(n, S.Ainv);
  AMG_LAUNCHED();
  rocblas_int* ipiv = tmp.get<rocblas_int>(n);
  rocblas_int* dinfo = tmp.get<rocblas_int>(1);
  struct Handle {  // the caller's rocBLAS handle, or one of our own
    rocblas_handle h = nullptr;
    bool own = false;
    ~Handle() {
      if (own) {
        auto lk = blas_lock();
        rocblas_destroy_handle(h);
      }
    }
  } hb;
  hb.h = shared;
  {
    auto lk = blas_lock();
    if (!hb.h) {
      if (rocblas_create_handle(&hb.h) != rocblas_status_success) throw DevError{-6, "rocblas_create_handle failed"};
      hb.own = true;
    }
    rocblas_set_stream(hb.h, stream);
  }
  rocblas_int info = 0;
  rocblas_status st1;
  {
    auto lk = blas_lock();
    st1 = rocsolver_dgetrf(hb.h, n, n, lu, n, ipiv, dinfo);
  }
  const hipError_t e1 = hipMemcpyAsync(&info, dinfo, sizeof(info), hipMemcpyDeviceToHost, stream);
  const hipError_t e2 = hipStreamSynchronize(stream);
  if (st1 != rocblas_status_success || e1 != hipSuccess || e2 != hipSuccess)
    throw DevError{-6, "coarse LU factorisation failed"};
  if (info != 0)
    throw DevError{-4, "zero pivot " + std::to_string(info) + " in the coarsest LU (n = " + std::to_string(n) + ")"};
  // the solves against I with pivots ipiv
  rocblas_status st2;
  {
    auto lk = blas_lock();
    st2 = rocsolver_dgetrs(hb.h, rocblas_operation_none, n, n, lu, n, ipiv, S.Ainv, n);
  }
  if (st2 != rocblas_status_success || hipStreamSynchronize(stream) != hipSuccess)
    throw DevError{-6, "coarse triangular solves failed"};
  const double err = check_error();
  if (!(err <= 1e-3))
    throw DevError{-4, "coarse inverse check failed (max error " + std::to_string(err) + ", n = " + std::to_string(n) + ")"};
}

// out_k = a_k m_{col_k} rounded to T: the values of A diag(m)
template <class T>
static __global__ void __launch_bounds__(kVecBS) scaled_values_kernel(int nnz, const int32_t* col,
                                                                      const double* val, const double* m, T* out) {
  const int stride = gridDim.x * kVecBS;
  for (int k = blockIdx.x * kVecBS + threadIdx.x; k < nnz; k += stride)
    out[k] = static_cast<T>(val[k] * m[col[k]]);
}

// A device copy in value type T of an FP64 device matrix (int32 row pointers
// and columns, same matrix as the host copy M, whose row pointers give the
// SpMV schedule); FP32 values are rounded to nearest, as on the host.
template <class T>
DevCsr<T> device_copy_csr(DevArena& ar, const DeviceCsrRef& src, const Csr& M) {
  const hipStream_t s = ar.stream();
  DevCsr<T> d;
  d.rows = src.rows;
  d.cols = src.cols;
  d.nnz = src.nnz;
  d.ptr = ar.get<int32_t>(static_cast<size_t>(src.rows) + 1);
  d.col = ar.get<int32_t>(std::max<int64_t>(src.nnz, 1));
  d.val = ar.get<T>(std::max<int64_t>(src.nnz, 1));
  AMG_HIP(hipMemcpyAsync(d.ptr, src.ptr, sizeof(int32_t) * (static_cast<size_t>(src.rows) + 1),
                         hipMemcpyDeviceToDevice, s));
  if (src.nnz) {
    AMG_HIP(hipMemcpyAsync(d.col, src.col, sizeof(int32_t) * src.nnz, hipMemcpyDeviceToDevice, s));
    if constexpr (std::is_same<T, double>::value) {
      AMG_HIP(hipMemcpyAsync(d.val, src.val, sizeof(double) * src.nnz, hipMemcpyDeviceToDevice, s));
    } else {
      copy_kernel<T, double><<<vec_blocks(src.nnz), kVecBS, 0, s>>>(static_cast<int>(src.nnz), d.val, src.val);
      AMG_LAUNCHED();
    }
  }
  Schedule sc = make_schedule<T>(M, -1);
  d.kind = sc.kind;
  d.lanes = sc.lanes;
  d.bclass = sc.bclass;
  d.nblocks = sc.nblocks;
  if (sc.kind == 0) d.blk = ar.upload(sc.blk.data(), sc.blk.size());
  attach_compact_cols(ar, d);
  return d;
}

// Level storage on the device in value type T.  Matrices and smoother
// diagonals the setup steps left on the device (`accel`, FP64, equal to the
// host hierarchy) are copied or rounded there; the rest is uploaded from the
// host hierarchy.
template <class T>
inline void upload_levels(amg_solver& S, DevHierarchy<T>& H, const SetupAccel* accel = nullptr) {
  DevArena& ar = *S.arena;
  const hipStream_t s = ar.stream();
  const int L = static_cast<int>(S.host.levels.size());
  const int npre = S.prm.npre;
  const bool cheb = S.prm.relax == AMG_CHEBYSHEV;
  for (int l = 0; l < L - 1; ++l) {
    const HostLevel& hl = S.host.levels[l];
    DeviceLevelRefs ref;
    const bool dev = accel && device_level_refs(accel, l, &ref);
    DevLevel<T> d;
    d.n = static_cast<int32_t>(hl.A.rows);
    d.nc = static_cast<int32_t>(hl.P.cols);
    if (l == 0) {
      DeviceCsrRef a0;  // the solver's FP64 fine operator
      a0.rows = S.A0.rows;
      a0.cols = S.A0.cols;
      a0.nnz = S.A0.nnz;
      a0.ptr = S.A0.ptr;
      a0.col = S.A0.col;
      a0.val = S.A0.val;
      if constexpr (std::is_same<T, double>::value) {
        d.A = S.A0;
      } else {
        // level 1 shares its pattern with the FP64 fine operator
        d.A.rows = S.A0.rows;
        d.A.cols = S.A0.cols;
        d.A.nnz = S.A0.nnz;
        d.A.ptr = S.A0.ptr;
        d.A.col = S.A0.col;
        d.A.val = ar.get<T>(std::max<int64_t>(a0.nnz, 1));
        if (a0.nnz) {
          copy_kernel<T, double><<<vec_blocks(a0.nnz), kVecBS, 0, s>>>(static_cast<int>(a0.nnz), d.A.val, a0.val);
          AMG_LAUNCHED();
        }
        Schedule sc = make_schedule<T>(hl.A, -1);
        d.A.kind = sc.kind;
        d.A.lanes = sc.lanes;
        d.A.bclass = sc.bclass;
        d.A.nblocks = sc.nblocks;
        d.A.blk = sc.kind == 0 ? ar.upload(sc.blk.data(), sc.blk.size()) : nullptr;
        attach_compact_cols(ar, d.A);
      }
    } else {
      d.A = (dev && ref.A.val) ? device_copy_csr<T>(ar, ref.A, hl.A) : upload_csr<T>(ar, hl.A);
    }
    d.P = (dev && ref.P.val) ? device_copy_csr<T>(ar, ref.P, hl.P) : upload_csr<T>(ar, hl.P);
    d.R = (dev && ref.R.val) ? device_copy_csr<T>(ar, ref.R, hl.R) : upload_csr<T>(ar, hl.R);
    const double* m64 = (dev && ref.m) ? ref.m : nullptr;
    if (m64) {
      d.m = ar.get<T>(std::max<int32_t>(d.n, 1));
      copy_kernel<T, double><<<vec_blocks(d.n), kVecBS, 0, s>>>(d.n, d.m, m64);
      AMG_LAUNCHED();
    } else {
      std::vector<T> m(hl.m.begin(), hl.m.end());
      d.m = ar.upload(m.data(), m.size());
    }
    if (l == 0 && npre == 1 && !cheb) {
      // the first pre-sweep from zero reads A (m .* f) = (A diag(m)) f
      if (!m64) m64 = ar.upload(hl.m.data(), hl.m.size());
      d.As = d.A;
      d.As.val = ar.get<T>(std::max<int64_t>(S.A0.nnz, 1));
      if (S.A0.nnz) {
        scaled_values_kernel<T><<<vec_blocks(S.A0.nnz), kVecBS, 0, s>>>(static_cast<int>(S.A0.nnz), S.A0.col,
                                                                       S.A0.val, m64, d.As.val);
        AMG_LAUNCHED();
      }
    }
    AMG_HIP(hipStreamSynchronize(ar.stream()));
    if (l > 0) {
      d.f = ar.get<T>(d.n);
      d.z = ar.get<T>(d.n);
      if (npre == 1 || (cheb && npre > 0)) d.mf = ar.get<T>(d.n);
    }
    d.r = ar.get<T>(d.n);
    d.y = ar.get<T>(d.n);
    d.t = ar.get<T>(d.n);
    if (npre > 1 || cheb) {
      d.zp[0] = ar.get<T>(d.n);
      d.zp[1] = ar.get<T>(d.n);
    }
    if (cheb) {
      d.dc[0] = ar.get<T>(d.n);
      d.dc[1] = ar.get<T>(d.n);
      d.cheb = cheb_coefficients<T>(hl.cheb_hi, S.prm.cheb_ratio, S.prm.cheb_degree);
    }
    H.lev.push_back(d);
  }
  if (L > 1) {
    if (S.nL != static_cast<int32_t>(S.host.levels.back().A.rows))
      throw DevError{-6, "coarsest level size not set before the level upload"};
    H.fL = ar.get<T>(S.nL);
    H.zL = ar.get<T>(S.nL);
  }
}

// Fused coarse tail (tail.hpp): the levels below level 1 whose operator
// holds at most kTailMaxBytes of values join the launch, up to
// kTailMaxLevels of them; kTailPerCu workgroups per compute unit (fewer if
// fewer fit), so that every workgroup of the launch is resident at once.
constexpr int64_t kTailMaxBytes = int64_t(32) << 20;
constexpr int kTailPerCu = 2;
constexpr double kTailWaitSeconds = 0.25;

template <class T>
inline void plan_tail(amg_solver& S, DevHierarchy<T>& H, hipStream_t s) {
  if (!S.prm.fuse_coarse || S.prm.relax == AMG_CHEBYSHEV || S.prm.npre != 1 || S.prm.npost != 1) return;
  const int nl = static_cast<int>(H.lev.size());
  int first = nl;
  while (first - 1 >= 1 && nl - (first - 1) <= kTailMaxLevels &&
         H.lev[first - 1].A.nnz * static_cast<int64_t>(sizeof(T)) <= kTailMaxBytes)
    --first;
  if (first >= nl) return;
  int occ = 0, cus = 0, khz = 0;
  AMG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, vcycle_tail_kernel<T>, kBS, 0));
  AMG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, S.device));
  AMG_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, S.device));
  if (occ < 1 || cus < 1 || khz < 1) return;
  H.tail_grid = std::min(occ, kTailPerCu) * cus;
  H.tail_sync = S.arena->get<TailSync>(1);
  AMG_HIP(hipMemsetAsync(H.tail_sync, 0, sizeof(TailSync), s));
  AMG_HIP(hipStreamSynchronize(s));
  H.tail_limit = static_cast<uint64_t>(kTailWaitSeconds * 1000.0 * khz);
  H.tail_first = first;
}

// Raises if a fused tail launch reported a barrier wait that ran out of
// time (its results are then invalid); clears the flag for the next call.
template <class T>
inline void check_tail(DevHierarchy<T>& H, hipStream_t s) {
  if (!H.tail_sync) return;
  int err = 0;
  AMG_HIP(hipMemcpyAsync(&err, &H.tail_sync->error, sizeof(int), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  if (err) {
    tail_reset_kernel<<<1, 64, 0, s>>>(H.tail_sync);
    AMG_LAUNCHED();
    AMG_HIP(hipStreamSynchronize(s));
    throw DevError{-6, "fused coarse levels: a grid barrier wait ran out of time; the result is invalid"};
  }
}

inline int64_t max_parts(const amg_solver& S) {
  int64_t m = vec_blocks(S.n);
  m = std::max<int64_t>(m, S.A0.nblocks);
  m = std::max<int64_t>(m, S.Afull.nblocks);
  if (S.block) {
    m = std::max<int64_t>(m, S.B0.blocks());
    for (const auto& lv : S.bh64.lev) m = std::max<int64_t>(m, lv.A.blocks());
    for (const auto& lv : S.bh32.lev) m = std::max<int64_t>(m, lv.A.blocks());
  }
  auto scan = [&](const auto& H) {
    for (const auto& lv : H.lev) {
      m = std::max<int64_t>(m, lv.A.nblocks);
      m = std::max<int64_t>(m, vec_blocks(lv.n));
    }
  };
  scan(S.h64);
  scan(S.h32);
  return m;
}

template <class F>
inline auto with_vcycle(amg_solver& S, F fn) {
  VcycleOpts o{S.prm.npre, S.prm.npost, S.prm.relax};
  if (S.schur) {
    const SchurOps so{&S.Dm, &S.Gs, S.mu, S.rp, S.split.n_u};
    if (S.prm.precision == AMG_MIXED) {
      SchurPrecond<float> P(Vcycle<float>(&S.h32, S.Ainv, S.nL, o), so);
      return fn(P);
    }
    SchurPrecond<double> P(Vcycle<double>(&S.h64, S.Ainv, S.nL, o), so);
    return fn(P);
  }
  if (S.block) {
    if (S.prm.precision == AMG_MIXED) {
      BlockVcycle<float> V(&S.bh32, S.Ainv, S.nL, S.prm.npre, S.prm.npost);
      return fn(V);
    }
    BlockVcycle<double> V(&S.bh64, S.Ainv, S.nL, S.prm.npre, S.prm.npost);
    return fn(V);
  }
  if (S.prm.precision == AMG_MIXED) {
    Vcycle<float> V(&S.h32, S.Ainv, S.nL, o);
    return fn(V);
  }
  Vcycle<double> V(&S.h64, S.Ainv, S.nL, o);
  return fn(V);
}

// ------------------------------------------------------------------ Krylov

inline void fin(amg_solver& S, int K, int nparts, int op, hipStream_t s) {
  if (K == 1) finalize_kernel<1><<<1, kFinBS, 0, s>>>(S.partials, nparts, S.st, op);
  else finalize_kernel<2><<<1, kFinBS, 0, s>>>(S.partials, nparts, S.st, op);
  AMG_LAUNCHED();
}

inline const int* skip_of(amg_solver& S) { return &S.st->done; }

// The Krylov loop's scalar FP64 operator: the fine level, or the whole
// system of a field split.
inline const DevCsr<double>& krylov_op(const amg_solver& S) { return S.schur ? S.Afull : S.A0; }

// Product with the FP64 operator of the Krylov loop (scalar CSR, or block
// CSR with the scalar epilogue applied row by row).
template <class G, class E>
inline int outer_spmv(amg_solver& S, G g, E e, double* partials, const int* skip, hipStream_t s) {
  if (S.block) return launch_bsr(S.B0, g, PerRow<E>{e}, partials, skip, s);
  return launch_spmv(krylov_op(S), g, e, partials, skip, s);
}

// r = f - A x with (r.r, f.f) and the init scalar update.
inline void enqueue_init(amg_solver& S, hipStream_t s) {
  int nb = outer_spmv(S, GatherX<double, double>{S.x}, EpiResidNorms{S.r, S.f}, S.partials, nullptr, s);
  fin(S, 2, nb, kFinInit, s);
}

inline void enqueue_pcg_start(amg_solver& S, hipStream_t s) {
  enqueue_init(S, s);
  int nb = with_vcycle(S, [&](auto& V) { return V.template run<1>(S.r, S.z, S.partials, skip_of(S), s); });
  fin(S, 1, nb, kFinPcgRho, s);
  pcg_dir_kernel<<<vec_blocks(S.n), kVecBS, 0, s>>>(static_cast<int>(S.n), S.p, S.z, S.st);
  AMG_LAUNCHED();
}

inline void enqueue_pcg_iteration(amg_solver& S, hipStream_t s) {
  const int n = static_cast<int>(S.n);
  const int vb = vec_blocks(n);
  int nb = outer_spmv(S, GatherX<double, double>{S.p}, EpiStoreDot{S.q, S.p}, S.partials, skip_of(S), s);
  fin(S, 1, nb, kFinAlpha, s);
  pcg_update_kernel<<<vb, kVecBS, 0, s>>>(n, S.x, S.r, S.p, S.q, S.st, S.partials);
  AMG_LAUNCHED();
  fin(S, 1, vb, kFinPcgRR, s);
  nb = with_vcycle(S, [&](auto& V) { return V.template run<1>(S.r, S.z, S.partials, skip_of(S), s); });
  fin(S, 1, nb, kFinPcgRho, s);
  pcg_dir_kernel<<<vb, kVecBS, 0, s>>>(n, S.p, S.z, S.st);
  AMG_LAUNCHED();
}

inline void enqueue_bicg_start(amg_solver& S, hipStream_t s) {
  enqueue_init(S, s);
  copy_kernel<double, double><<<vec_blocks(S.n), kVecBS, 0, s>>>(static_cast<int>(S.n), S.rt, S.r);
  AMG_LAUNCHED();
}

inline void enqueue_bicg_iteration(amg_solver& S, hipStream_t s) {
  const int n = static_cast<int>(S.n);
  const int vb = vec_blocks(n);
  bicg_p_kernel<<<vb, kVecBS, 0, s>>>(n, S.p, S.r, S.v, S.st);
  AMG_LAUNCHED();
  with_vcycle(S, [&](auto& V) { return V.template run<0>(S.p, S.phat, S.partials, skip_of(S), s); });
  int nb = outer_spmv(S, GatherX<double, double>{S.phat}, EpiStoreDot{S.v, S.rt}, S.partials, skip_of(S), s);
  fin(S, 1, nb, kFinBiAlpha, s);
  bicg_s_kernel<<<vb, kVecBS, 0, s>>>(n, S.s, S.r, S.v, S.st, S.partials);
  AMG_LAUNCHED();
  fin(S, 1, vb, kFinBiS, s);
  bicg_half_kernel<<<vb, kVecBS, 0, s>>>(n, S.x, S.phat, S.st);
  AMG_LAUNCHED();
  fin(S, 1, 0, kFinBiHalfDone, s);
  with_vcycle(S, [&](auto& V) { return V.template run<0>(S.s, S.shat, S.partials, skip_of(S), s); });
  nb = outer_spmv(S, GatherX<double, double>{S.shat}, EpiStoreDot2{S.t, S.s}, S.partials, skip_of(S), s);
  fin(S, 2, nb, kFinBiOmega, s);
  bicg_xr_kernel<<<vb, kVecBS, 0, s>>>(n, S.x, S.r, S.phat, S.shat, S.s, S.t, S.rt, S.st, S.partials);
  AMG_LAUNCHED();
  fin(S, 2, vb, kFinBiR, s);
}

inline void enqueue_iteration(amg_solver& S, hipStream_t s) {
  if (S.prm.solver == AMG_CG) enqueue_pcg_iteration(S, s);
  else enqueue_bicg_iteration(S, s);
}

inline void build_graph(amg_solver& S) {
  if (S.iter_exec) return;
  AMG_HIP(hipStreamBeginCapture(S.cap_stream, hipStreamCaptureModeThreadLocal));
  try {
    for (int it = 0; it < S.prm.check_every; ++it) enqueue_iteration(S, S.cap_stream);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(S.cap_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  AMG_HIP(hipStreamEndCapture(S.cap_stream, &S.iter_graph));
  AMG_HIP(hipGraphInstantiate(&S.iter_exec, S.iter_graph, nullptr, nullptr, 0));
}

inline KState poll(amg_solver& S, hipStream_t s) {
  AMG_HIP(hipMemcpyAsync(S.st_host, S.st, sizeof(KState), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  return *S.st_host;
}

// ------------------------------------------------------------------ GMRES

// r = f - A x and the opening of a cycle (first: the initial residual).
inline void enqueue_gm_cycle_start(amg_solver& S, bool first, hipStream_t s) {
  const int n = static_cast<int>(S.n);
  int nb = outer_spmv(S, GatherX<double, double>{S.x}, EpiResidNorms{S.r, S.f}, S.partials,
                      first ? nullptr : skip_of(S), s);
  gm_start_state_kernel<<<1, kFinBS, 0, s>>>(S.partials, nb, S.st, S.gm, first ? 1 : 0);
  AMG_LAUNCHED();
  gm_first_vector_kernel<<<vec_blocks(n), kVecBS, 0, s>>>(n, S.gmV, S.r, S.gm);
  AMG_LAUNCHED();
}

// Arnoldi step j: z_j = M v_j, w = A z_j, two Gram-Schmidt passes, rotation,
// v_{j+1} = w / ||w||.  Every kernel returns at once once the cycle stopped.
inline void enqueue_gm_step(amg_solver& S, int j, hipStream_t s) {
  const int n = static_cast<int>(S.n);
  const int64_t ld = S.gm_ld;
  double* vj = S.gmV + j * ld;
  double* zj = S.gmZ + j * ld;
  double* w = S.q;
  const int* stop = &S.gm->stop;
  with_vcycle(S, [&](auto& V) { return V.template run<0>(vj, zj, S.partials, stop, s); });
  outer_spmv(S, GatherX<double, double>{zj}, EpiStore<double, double>{w}, nullptr, stop, s);
  const int nb = S.gm_nb;
  for (int pass = 0; pass < 2; ++pass) {
    gm_dots_kernel<<<dim3(nb, j + 1), kVecBS, 0, s>>>(n, S.gmV, ld, w, S.gm_partials, S.gm);
    AMG_LAUNCHED();
    gm_sum_kernel<<<j + 1, kFinBS, 0, s>>>(S.gm_partials, nb, S.gm, pass);
    AMG_LAUNCHED();
    if (pass == 0)
      gm_subtract_kernel<0><<<nb, kVecBS, 0, s>>>(n, j + 1, S.gmV, ld, w, nullptr, S.gm);
    else
      gm_subtract_kernel<1><<<nb, kVecBS, 0, s>>>(n, j + 1, S.gmV, ld, w, S.gm_partials, S.gm);
    AMG_LAUNCHED();
  }
  gm_givens_kernel<<<1, kFinBS, 0, s>>>(S.gm_partials, nb, S.gm, S.st, j, S.prm.gmres_m);
  AMG_LAUNCHED();
  gm_scale_kernel<<<vec_blocks(n), kVecBS, 0, s>>>(n, S.gmV + (j + 1) * ld, w, S.gm);
  AMG_LAUNCHED();
}

// End of a cycle: y = R^-1 g, x += Z y, then the next cycle's start.
inline void enqueue_gm_cycle_end(amg_solver& S, hipStream_t s) {
  const int n = static_cast<int>(S.n);
  gm_solve_kernel<<<1, 64, 0, s>>>(S.gm, S.st);
  AMG_LAUNCHED();
  gm_update_kernel<<<vec_blocks(n), kVecBS, 0, s>>>(n, S.x, S.gmZ, S.gm_ld, S.gm, S.st);
  AMG_LAUNCHED();
  enqueue_gm_cycle_start(S, false, s);
}

// Krylov state and the cycle's stop flag, read after the stream drains.
inline KState gm_poll(amg_solver& S, hipStream_t s, int32_t* stop) {
  AMG_HIP(hipMemcpyAsync(S.st_host, S.st, sizeof(KState), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipMemcpyAsync(S.gm_host, &S.gm->k, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  *stop = S.gm_host[1];
  return *S.st_host;
}

// Captures the GMRES graphs: group g holds Arnoldi steps [g ce, min(m, (g +
// 1) ce)), the last graph the end of a cycle and the next one's start.
inline void build_gm_graphs(amg_solver& S) {
  if (!S.gm_execs.empty()) return;
  const int m = S.prm.gmres_m, ce = S.prm.check_every;
  const int groups = (m + ce - 1) / ce;
  // built into local lists and kept only when every graph was made
  std::vector<hipGraph_t> graphs;
  std::vector<hipGraphExec_t> execs;
  auto drop = [&] {
    for (auto e : execs) (void)hipGraphExecDestroy(e);
    for (auto g : graphs) (void)hipGraphDestroy(g);
  };
  try {
    for (int g = 0; g <= groups; ++g) {
      AMG_HIP(hipStreamBeginCapture(S.cap_stream, hipStreamCaptureModeThreadLocal));
      try {
        if (g < groups) {
          for (int j = g * ce; j < std::min(m, (g + 1) * ce); ++j) enqueue_gm_step(S, j, S.cap_stream);
        } else {
          enqueue_gm_cycle_end(S, S.cap_stream);
        }
      } catch (...) {
        hipGraph_t gr = nullptr;
        (void)hipStreamEndCapture(S.cap_stream, &gr);
        if (gr) (void)hipGraphDestroy(gr);
        throw;
      }
      hipGraph_t gr = nullptr;
      AMG_HIP(hipStreamEndCapture(S.cap_stream, &gr));
      graphs.push_back(gr);
      hipGraphExec_t ex = nullptr;
      AMG_HIP(hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
      execs.push_back(ex);
    }
  } catch (...) {
    drop();
    throw;
  }
  S.gm_graphs = std::move(graphs);
  S.gm_execs = std::move(execs);
}

// The whole GMRES solve; the host polls every check_every Arnoldi steps and
// at the end of each cycle.  With use_graph each group of steps between
// polls, and the end of a cycle, is one graph launch (the same kernels in
// the same order as the direct launches).  Returns the final state and the
// number of cycles run.
inline KState run_gmres(amg_solver& S, hipStream_t s, int* cycles) {
  int32_t stop = 0;
  enqueue_gm_cycle_start(S, true, s);
  KState k = gm_poll(S, s, &stop);
  *cycles = 0;
  const int m = S.prm.gmres_m, ce = S.prm.check_every;
  const int groups = (m + ce - 1) / ce;
  if (S.prm.use_graph) build_gm_graphs(S);
  while (k.done == kRunning) {
    ++*cycles;
    for (int g = 0; g < groups; ++g) {
      if (S.prm.use_graph) {
        AMG_HIP(hipGraphLaunch(S.gm_execs[g], s));
      } else {
        for (int j = g * ce; j < std::min(m, (g + 1) * ce); ++j) enqueue_gm_step(S, j, s);
      }
      k = gm_poll(S, s, &stop);
      if (stop) break;
    }
    if (S.prm.use_graph) AMG_HIP(hipGraphLaunch(S.gm_execs[groups], s));
    else enqueue_gm_cycle_end(S, s);
    k = gm_poll(S, s, &stop);
  }
  return k;
}

inline amg_status run_solve(amg_solver& S, const double* f_dev, double* u_dev, hipStream_t s, amg_info* info) {
  const double t0 = now_s();
  const int n = static_cast<int>(S.n);
  const size_t bytes = sizeof(double) * S.n;
  if (S.perm) {  // the caller's order -> velocity first
    gather_kernel<<<vec_blocks(n), kVecBS, 0, s>>>(n, S.f, f_dev, S.perm);
    AMG_LAUNCHED();
    gather_kernel<<<vec_blocks(n), kVecBS, 0, s>>>(n, S.x, u_dev, S.perm);
    AMG_LAUNCHED();
  } else {
    AMG_HIP(hipMemcpyAsync(S.f, f_dev, bytes, hipMemcpyDeviceToDevice, s));
    AMG_HIP(hipMemcpyAsync(S.x, u_dev, bytes, hipMemcpyDeviceToDevice, s));
  }
  KState init{};
  init.tol = S.prm.tol;
  init.max_iter = S.prm.max_iter;
  init.first = 1;
  *S.st_host = init;
  AMG_HIP(hipMemcpyAsync(S.st, S.st_host, sizeof(KState), hipMemcpyHostToDevice, s));
  if (S.prm.use_graph && S.prm.solver != AMG_GMRES) build_graph(S);

  int restarts = 0;
  KState k{};
  if (S.prm.solver == AMG_GMRES) {
    int cycles = 0;
    k = run_gmres(S, s, &cycles);
    restarts = std::max(cycles - 1, 0);
    if (k.done != kZeroRhs) {
      int nb = outer_spmv(S, GatherX<double, double>{S.x}, EpiResidNorms{S.tmp, S.f}, S.partials, nullptr, s);
      fin(S, 2, nb, kFinTrue, s);
      k = poll(S, s);
    }
  }
  for (; S.prm.solver != AMG_GMRES;) {
    if (S.prm.solver == AMG_CG) enqueue_pcg_start(S, s);
    else enqueue_bicg_start(S, s);
    k = poll(S, s);
    while (k.done == kRunning) {
      if (S.prm.use_graph) {
        AMG_HIP(hipGraphLaunch(S.iter_exec, s));  // check_every iterations
      } else {
        for (int it = 0; it < S.prm.check_every; ++it) enqueue_iteration(S, s);
      }
      k = poll(S, s);
    }
    if (k.done == kZeroRhs) break;
    // true residual of the current iterate
    int nb = outer_spmv(S, GatherX<double, double>{S.x}, EpiResidNorms{S.tmp, S.f}, S.partials, nullptr, s);
    fin(S, 2, nb, kFinTrue, s);
    k = poll(S, s);
    if (k.done == kConverged && k.true_rr > k.tol2 && restarts == 0) {
      ++restarts;  // restart once from the current iterate; the count continues
      continue;
    }
    break;
  }
  if (k.done == kZeroRhs) {
    fill_kernel<double><<<vec_blocks(n), kVecBS, 0, s>>>(n, S.x, 0.0);
    AMG_LAUNCHED();
  }
  if (S.perm) {
    scatter_kernel<<<vec_blocks(n), kVecBS, 0, s>>>(n, u_dev, S.x, S.perm);
    AMG_LAUNCHED();
  } else {
    AMG_HIP(hipMemcpyAsync(u_dev, S.x, bytes, hipMemcpyDeviceToDevice, s));
  }
  AMG_HIP(hipStreamSynchronize(s));
  check_tail(S.h64, s);
  check_tail(S.h32, s);

  amg_status status = AMG_OK;
  switch (k.done) {
    case kConverged:
      status = (k.true_rr <= k.tol2) ? AMG_OK : AMG_NOT_CONVERGED;
      break;
    case kZeroRhs: status = AMG_OK; break;
    case kMaxIter: status = AMG_NOT_CONVERGED; break;
    case kBreakdown: status = AMG_ERR_BREAKDOWN; break;
    default: status = AMG_ERR_NAN; break;
  }
  if (info) {
    info->iters = k.iters;
    info->levels = static_cast<int32_t>(S.block ? S.bhost.levels.size() : S.host.levels.size());
    info->restarts = restarts;
    info->status = status;
    const bool zero = (k.done == kZeroRhs);
    info->rel_resid = zero ? 0.0 : std::sqrt(k.rr / k.ff);
    info->true_rel_resid = zero ? 0.0 : std::sqrt(k.true_rr / k.ff);
    info->setup_s = S.setup_s;
    info->solve_s = now_s() - t0;
    double nnz = 0;
    if (S.block) {
      for (auto& lv : S.bhost.levels) nnz += double(lv.A.nnzb());
      info->op_complexity = nnz / double(S.bhost.levels[0].A.nnzb());
    } else {
      for (auto& lv : S.host.levels) nnz += double(lv.A.nnz());
      info->op_complexity = nnz / double(S.host.levels[0].A.nnz());
    }
  }
  if (status == AMG_NOT_CONVERGED) g_last_error = "iteration limit or tolerance not reached";
  if (status == AMG_ERR_BREAKDOWN) g_last_error = "Krylov breakdown (zero inner product)";
  if (status == AMG_ERR_NAN) g_last_error = "non-finite value in the iteration";
  return status;
}

// Options of device_setup for solves owned by a server: no graph-capture
// stream or pinned state mirror of their own, a shared rocBLAS handle, and
// the Krylov state in the server's slot table (assigned at admission).
struct DeviceSetupOpts {
  bool standalone = true;
  rocblas_handle blas = nullptr;
};

// Releases the device storage of a setup that failed part-way (out of
// memory) so that device_setup can run again from the host hierarchy: every
// member that points into the arena is cleared with it (device_setup keeps
// a fine operator it finds already uploaded, so a stale one would be read
// after its memory went back to the pool).
inline void drop_device_state(amg_solver& S) {
  S.arena.reset();
  S.A0 = DevCsr<double>{};
  S.B0 = DevBsr<double>{};
  S.h64 = DevHierarchy<double>{};
  S.h32 = DevHierarchy<float>{};
  S.bh64 = DevBlockHierarchy<double>{};
  S.bh32 = DevBlockHierarchy<float>{};
  S.Ainv = nullptr;
  S.partials = nullptr;
  S.f = S.x = S.r = S.z = S.p = S.q = S.tmp = nullptr;
  S.rt = S.v = S.phat = S.s = S.shat = S.t = nullptr;
  S.gmV = S.gmZ = S.gm_partials = nullptr;
  S.gm = nullptr;
  S.Afull = S.Dm = S.Gs = DevCsr<double>{};
  S.mu = S.rp = nullptr;
  S.perm = nullptr;
  // captured graphs hold pointers into the released memory
  if (S.iter_exec) (void)hipGraphExecDestroy(S.iter_exec);
  if (S.iter_graph) (void)hipGraphDestroy(S.iter_graph);
  S.iter_exec = nullptr;
  S.iter_graph = nullptr;
  for (auto e : S.gm_execs) (void)hipGraphExecDestroy(e);
  for (auto g : S.gm_graphs) (void)hipGraphDestroy(g);
  S.gm_execs.clear();
  S.gm_graphs.clear();
}

// `accel`: the setup steps' accelerator, whose device copies of the levels
// (if it kept them) replace uploads from the host hierarchy.
inline void device_setup(amg_solver& S, const amg_allocator* alloc, hipStream_t s,
                         const DeviceSetupOpts& opts = DeviceSetupOpts{}, const SetupAccel* accel = nullptr) {
  AMG_HIP(hipGetDevice(&S.device));
  if (!S.arena) S.arena = std::make_unique<DevArena>(alloc, s);
  if (opts.standalone) AMG_HIP(hipStreamCreateWithFlags(&S.cap_stream, hipStreamNonBlocking));
  DevArena& ar = *S.arena;
  // served solves keep int32 columns (their footprint is planned before placement)
  ar.compact_cols = opts.standalone;
  // the coarsest operator in scalar form; upload_levels sizes f_L, z_L by nL
  const Csr AL = S.block ? bsr_to_csr(S.bhost.levels.back().A) : S.host.levels.back().A;
  S.nL = static_cast<int32_t>(AL.rows);
  PhaseClock clk(S.host.phase_s);
  clk.enter(kPhUpload);
  if (S.block) {
    const Bsr& fine = S.bhost.levels[0].A;
    S.n = int64_t(kB) * fine.rows;
    S.B0 = upload_bsr<double>(ar, fine);
    if (S.prm.precision == AMG_MIXED) upload_block_levels<float>(ar, S.bhost, S.B0, S.bh32, S.prm.npre, S.prm.npost);
    else upload_block_levels<double>(ar, S.bhost, S.B0, S.bh64, S.prm.npre, S.prm.npost);
  } else {
    const HostLevel& fine = S.host.levels[0];
    S.n = fine.A.rows;
    if (!S.A0.val) S.A0 = upload_csr<double>(ar, fine.A);  // unless uploaded before the setup steps
    else if (!S.A0.col16) attach_compact_cols(ar, S.A0);
    if (S.prm.precision == AMG_MIXED) upload_levels<float>(S, S.h32, accel);
    else upload_levels<double>(S, S.h64, accel);
    if (S.schur) {
      S.n = S.split.A.rows;
      S.Afull = upload_csr<double>(ar, S.split.A);
      S.Dm = upload_csr<double>(ar, S.split.Dm);
      S.Gs = upload_csr<double>(ar, S.split.G);
      S.mu = ar.upload(S.split.mu.data(), S.split.mu.size());
      S.rp = ar.get<double>(S.split.A.rows - S.split.n_u);
      if (!S.split.old_of_new.empty()) S.perm = ar.upload(S.split.old_of_new.data(), S.split.old_of_new.size());
    }
  }
  clk.enter(kPhCoarse);
  coarse_inverse(S, AL, s, alloc, opts.blas);
  clk.enter(kPhOther);
  if (opts.standalone && !S.block) {
    if (S.prm.precision == AMG_MIXED) plan_tail<float>(S, S.h32, s);
    else plan_tail<double>(S, S.h64, s);
  }
  if (opts.standalone) {
    S.st = ar.get<KState>(1);
    if (!S.st_host)
      AMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&S.st_host), sizeof(KState), hipHostMallocDefault));
  }
  S.partials = ar.get<double>(2 * max_parts(S));
  const int64_t n = S.n;
  S.f = ar.get<double>(n);
  S.x = ar.get<double>(n);
  S.r = ar.get<double>(n);
  S.z = ar.get<double>(n);
  S.p = ar.get<double>(n);
  S.q = ar.get<double>(n);
  S.tmp = ar.get<double>(n);
  if (S.prm.solver == AMG_GMRES) {
    const int m = S.prm.gmres_m;
    S.gm_ld = (n + 31) & ~int64_t(31);  // 256-byte aligned basis vectors
    S.gmV = ar.get<double>(static_cast<size_t>(m + 1) * S.gm_ld);
    S.gmZ = ar.get<double>(static_cast<size_t>(m) * S.gm_ld);
    S.gm = ar.get<GState>(1);
    S.gm_nb = static_cast<int>(std::min<int64_t>(vec_blocks(n), kGmDotBlocks));
    S.gm_partials = ar.get<double>(static_cast<size_t>(m + 1) * S.gm_nb);
    if (opts.standalone && !S.gm_host)
      AMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&S.gm_host), 2 * sizeof(int32_t), hipHostMallocDefault));
  }
  if (S.prm.solver == AMG_BICGSTAB) {
    S.rt = ar.get<double>(n);
    S.v = ar.get<double>(n);
    S.phat = ar.get<double>(n);
    S.s = ar.get<double>(n);
    S.shat = ar.get<double>(n);
    S.t = ar.get<double>(n);
  }
  AMG_HIP(hipStreamSynchronize(s));
  clk.stop();
  S.on_device = true;
}



// --------------------------------------------------------------- C ABI helpers

template <class F>
inline amg_status guarded(F fn) {
  try {
    return fn();
  } catch (const SetupError& e) {
    return set_error(e.code, e.msg);
  } catch (const DevError& e) {
    return set_error(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return set_error(AMG_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return set_error(AMG_ERR_INVALID_ARG, e.what());
  } catch (...) {
    return set_error(AMG_ERR_INVALID_ARG, "unknown error");
  }
}

}  // namespace amg
