// C ABI of the solver (include/amg.h): setup, solve, queries, measurement.

#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>

#include "galerkin.hpp"
#include "solver.hpp"

using namespace amg;

extern "C" {

void amg_params_default(amg_params* p) {
  if (!p) return;
  p->solver = AMG_CG;
  p->relax = AMG_SPAI0;
  p->precision = AMG_FP64;
  p->npre = 1;
  p->npost = 1;
  p->coarse_enough = 3000;
  p->max_levels = 30;
  p->max_iter = 500;
  p->eps_strong = 0.08;
  p->jacobi_omega = 0.72;
  p->tol = 1e-8;
  p->use_graph = 1;
  p->check_every = 4;
  p->cheb_degree = 3;
  p->cheb_ratio = 30.0;
  p->gmres_m = 30;
  p->fuse_coarse = 0;
}

const char* amg_last_error(void) { return g_last_error.c_str(); }

// n_u > 0: a Schur-complement field split with n_u velocity unknowns; the
// hierarchy is built for the approximate pressure Schur complement.
// pmask (with n_u = -1): the field split with the pressure unknowns marked,
// in any order; the system is renumbered velocity first.
static amg_status do_setup(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                           const amg_params* p, bool device, const amg_allocator* alloc, void* stream,
                           amg_handle* out, int64_t n_u = 0, const uint8_t* pmask = nullptr) {
  if (out) *out = nullptr;
  return guarded([&]() -> amg_status {
    if (!out) throw SetupError{-1, "out must not be NULL"};
    TraceRange range("amg setup");
    const double t0 = now_s();
    double pre[kPhCount] = {};  // input and fine upload, before the hierarchy exists
    PhaseClock clk(pre);
    clk.enter(kPhInput);
    auto S = std::make_unique<amg_solver>();
    if (p) S->prm = *p;
    else amg_params_default(&S->prm);
    check_params(S->prm);
    if (n_u && S->prm.solver != AMG_BICGSTAB && S->prm.solver != AMG_GMRES)
      throw SetupError{-1, "the field split is not symmetric: solver must be AMG_BICGSTAB or AMG_GMRES"};
    // The runtime loads a code object on the first use of one of its kernels
    // (tens of ms for the solve's several hundred).  The setup kernels' is
    // loaded on a side thread while the input is checked and copied, the
    // solve's while the host aggregates the first level (loading it blocks
    // kernel launches of other threads, so not while the device steps run).
    std::thread preload;
    std::mutex pre_mu;
    std::condition_variable pre_cv;
    bool pre_go = false;
    if (device) {
      int dev = 0;
      AMG_HIP(hipGetDevice(&dev));
      preload = std::thread([dev, &pre_mu, &pre_cv, &pre_go] {
        if (hipSetDevice(dev) != hipSuccess) return;
        preload_setup_kernels();
        {
          std::unique_lock<std::mutex> lk(pre_mu);
          pre_cv.wait(lk, [&] { return pre_go; });
        }
        hipFuncAttributes a;
        (void)hipFuncGetAttributes(&a, reinterpret_cast<const void*>(&copy_kernel<double, double>));
        (void)hipGetLastError();
      });
    }
    auto release_preload = [&pre_mu, &pre_cv, &pre_go] {
      {
        std::lock_guard<std::mutex> lk(pre_mu);
        pre_go = true;
      }
      pre_cv.notify_all();
    };
    struct Join {
      std::thread& t;
      std::function<void()> release;
      ~Join() {
        if (t.joinable()) {
          release();
          t.join();
        }
      }
    } join_preload{preload, release_preload};
    validate_csr(n, row_ptr, col, val, /*require_diag=*/n_u == 0);
    Csr A = to_csr(n, row_ptr, col, val);
    if (n_u) {
      std::vector<int32_t> order;
      if (pmask) {
        n_u = field_order(n, pmask, &order);
        A = permute_symmetric(A, order);
      }
      A = split_fields(std::move(A), n_u, &S->split);
      S->split.old_of_new = std::move(order);
      S->schur = true;
    }
    // Data-parallel setup steps on the device (bit-identical to the host's);
    // a step that does not fit the device path stays on the host.  The fine
    // operator goes to the device once: the solver's copy also serves them.
    std::unique_ptr<SetupAccel> accel;
    if (device) {
      clk.enter(kPhUpload);
      S->arena = std::make_unique<DevArena>(alloc, static_cast<hipStream_t>(stream));
      // (its column offsets are added in device_setup: the kernel that forms
      // them would load the solve's code object here, before the side
      // thread does so during aggregation)
      S->A0 = upload_csr<double>(*S->arena, A);
      DeviceCsrRef fine;
      fine.rows = S->A0.rows;
      fine.cols = S->A0.cols;
      fine.nnz = S->A0.nnz;
      fine.ptr = S->A0.ptr;
      fine.col = S->A0.col;
      fine.val = S->A0.val;
      accel = make_device_setup_accel(alloc, static_cast<hipStream_t>(stream), &fine, /*keep_levels=*/true,
                                      release_preload);
    }
    clk.stop();
    S->host = build_hierarchy(std::move(A), setup_params(S->prm), accel.get());
    for (int k = 0; k < kPhCount; ++k) S->host.phase_s[k] += pre[k];
    if (preload.joinable()) {
      PhaseClock wait(S->host.phase_s);
      wait.enter(kPhOther);
      release_preload();  // a one-level hierarchy never aggregates
      preload.join();
    }
    if (device) {
      try {
        device_setup(*S, alloc, static_cast<hipStream_t>(stream), DeviceSetupOpts{}, accel.get());
      } catch (const DevError& e) {
        if (e.code != AMG_ERR_OOM || !accel) throw;
        // Out of device memory with the setup's own level copies still held:
        // let them go and build the solver's storage from the host hierarchy.
        accel.reset();
        drop_device_state(*S);
        if (S->cap_stream) {
          (void)hipStreamDestroy(S->cap_stream);
          S->cap_stream = nullptr;
        }
        device_setup(*S, alloc, static_cast<hipStream_t>(stream), DeviceSetupOpts{}, nullptr);
      }
    }
    {
      PhaseClock other(S->host.phase_s);
      other.enter(kPhOther);
      accel.reset();
    }
    S->setup_s = now_s() - t0;
    *out = S.release();
    g_last_error.clear();
    return AMG_OK;
  });
}

static amg_status do_setup_block(int64_t nb, int32_t bs, const int64_t* ptr, const int32_t* col,
                                 const double* val, const amg_params* p, bool device, const amg_allocator* alloc,
                                 void* stream, amg_handle* out) {
  if (out) *out = nullptr;
  return guarded([&]() -> amg_status {
    if (!out) throw SetupError{-1, "out must not be NULL"};
    if (bs != kBlock) throw SetupError{-1, "block_size must be 4"};
    TraceRange range("amg setup");
    const double t0 = now_s();
    double pre[kPhCount] = {};
    PhaseClock clk(pre);
    clk.enter(kPhInput);
    auto S = std::make_unique<amg_solver>();
    if (p) S->prm = *p;
    else amg_params_default(&S->prm);
    check_params(S->prm);
    check_block_params(S->prm);
    validate_bsr(nb, ptr, col, val);
    Bsr A;
    A.rows = A.cols = nb;
    A.ptr.resize(nb + 1);
    A.col.resize(ptr[nb]);
    A.val.resize(static_cast<size_t>(ptr[nb]) * kBB);
    copy_parallel(A.ptr.data(), ptr, sizeof(int64_t) * (nb + 1));
    copy_parallel(A.col.data(), col, sizeof(int32_t) * ptr[nb]);
    copy_parallel(A.val.data(), val, sizeof(double) * ptr[nb] * kBB);
    clk.stop();
    S->block = true;
    S->bhost = build_block_hierarchy(std::move(A), setup_params(S->prm));
    for (int k = 0; k < kPhCount; ++k) S->host.phase_s[k] = S->bhost.phase_s[k] + pre[k];
    if (device) device_setup(*S, alloc, static_cast<hipStream_t>(stream));
    S->setup_s = now_s() - t0;
    *out = S.release();
    g_last_error.clear();
    return AMG_OK;
  });
}

amg_status amg_setup_block(int64_t nb, int32_t block_size, const int64_t* block_row_ptr, const int32_t* block_col,
                           const double* block_val, const amg_params* p, const amg_allocator* alloc,
                           void* hip_stream, amg_handle* out) {
  return do_setup_block(nb, block_size, block_row_ptr, block_col, block_val, p, true, alloc, hip_stream, out);
}

amg_status amg_setup_block_host(int64_t nb, int32_t block_size, const int64_t* block_row_ptr,
                                const int32_t* block_col, const double* block_val, const amg_params* p,
                                amg_handle* out) {
  return do_setup_block(nb, block_size, block_row_ptr, block_col, block_val, p, false, nullptr, nullptr, out);
}

amg_status amg_setup(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                     const amg_params* p, const amg_allocator* alloc, void* hip_stream, amg_handle* out) {
  return do_setup(n, row_ptr, col, val, p, true, alloc, hip_stream, out);
}

amg_status amg_setup_host(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                          const amg_params* p, amg_handle* out) {
  return do_setup(n, row_ptr, col, val, p, false, nullptr, nullptr, out);
}

amg_status amg_setup_schur(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val, int64_t n_u,
                           const amg_params* p, const amg_allocator* alloc, void* hip_stream, amg_handle* out) {
  if (n_u <= 0 || n_u >= n) {
    if (out) *out = nullptr;
    return set_error(AMG_ERR_INVALID_ARG, "velocity unknowns n_u must satisfy 0 < n_u < n");
  }
  return do_setup(n, row_ptr, col, val, p, true, alloc, hip_stream, out, n_u);
}

amg_status amg_setup_schur_masked(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                                  const uint8_t* pmask, const amg_params* p, const amg_allocator* alloc,
                                  void* hip_stream, amg_handle* out) {
  if (out) *out = nullptr;
  if (n <= 0 || !pmask) return set_error(AMG_ERR_INVALID_ARG, "null pmask or non-positive size");
  return guarded([&]() -> amg_status {
    std::vector<int32_t> order;
    (void)field_order(n, pmask, &order);  // the mask's errors before any device work
    return do_setup(n, row_ptr, col, val, p, true, alloc, hip_stream, out, -1, pmask);
  });
}

amg_status amg_setup_schur_host(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                                int64_t n_u, const amg_params* p, amg_handle* out) {
  if (n_u <= 0 || n_u >= n) {
    if (out) *out = nullptr;
    return set_error(AMG_ERR_INVALID_ARG, "velocity unknowns n_u must satisfy 0 < n_u < n");
  }
  return do_setup(n, row_ptr, col, val, p, false, nullptr, nullptr, out, n_u);
}

amg_status amg_solve(amg_handle h, const double* f_dev, double* u_dev, void* hip_stream, amg_info* info) {
  return guarded([&]() -> amg_status {
    if (!h || !f_dev || !u_dev) throw SetupError{-1, "NULL handle or vector"};
    if (!h->on_device) throw SetupError{-1, "handle was built by amg_setup_host: no device data"};
    TraceRange range("amg solve");
    return run_solve(*h, f_dev, u_dev, static_cast<hipStream_t>(hip_stream), info);
  });
}

void amg_release(amg_handle h) { delete h; }

amg_status amg_vcycle(amg_handle h, const double* r_dev, double* z_dev, void* hip_stream) {
  return guarded([&]() -> amg_status {
    if (!h || !r_dev || !z_dev) throw SetupError{-1, "NULL handle or vector"};
    if (!h->on_device) throw SetupError{-1, "handle was built by amg_setup_host: no device data"};
    if (static_cast<const void*>(r_dev) == static_cast<const void*>(z_dev))
      throw SetupError{-1, "r and z must not alias"};
    TraceRange range("amg V-cycle");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (h->perm) {  // the caller's order -> velocity first and back, through two work vectors
      const int n = static_cast<int>(h->n);
      gather_kernel<<<vec_blocks(n), kVecBS, 0, s>>>(n, h->tmp, r_dev, h->perm);
      AMG_LAUNCHED();
      with_vcycle(*h, [&](auto& V) { return V.template run<0>(h->tmp, h->q, h->partials, nullptr, s); });
      scatter_kernel<<<vec_blocks(n), kVecBS, 0, s>>>(n, z_dev, h->q, h->perm);
      AMG_LAUNCHED();
    } else {
      with_vcycle(*h, [&](auto& V) { return V.template run<0>(r_dev, z_dev, h->partials, nullptr, s); });
    }
    AMG_HIP(hipStreamSynchronize(s));
    check_tail(h->h64, s);
    check_tail(h->h32, s);
    return AMG_OK;
  });
}

static_assert(kPhCount == AMG_SETUP_PHASES, "setup phases of the C ABI");

amg_status amg_setup_profile(amg_handle h, double* seconds) {
  return guarded([&]() -> amg_status {
    if (!h || !seconds) throw SetupError{-1, "NULL argument"};
    for (int k = 0; k < kPhCount; ++k) seconds[k] = h->host.phase_s[k];
    return AMG_OK;
  });
}

amg_status amg_tail_info(amg_handle h, int32_t* first_level, int32_t* grid) {
  return guarded([&]() -> amg_status {
    if (!h) throw SetupError{-1, "NULL handle"};
    const bool mixed = h->prm.precision == AMG_MIXED;
    const int first = mixed ? h->h32.tail_first : h->h64.tail_first;
    if (first_level) *first_level = first >= 1 ? first : -1;
    if (grid) *grid = first >= 1 ? (mixed ? h->h32.tail_grid : h->h64.tail_grid) : 0;
    return AMG_OK;
  });
}

amg_status amg_tail_set_wait(amg_handle h, double seconds) {
  return guarded([&]() -> amg_status {
    if (!h || !(seconds >= 0.0) || seconds > 60.0) throw SetupError{-1, "bad argument"};
    int khz = 0;
    AMG_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device));
    const uint64_t ticks = static_cast<uint64_t>(seconds * 1000.0 * khz);
    h->h64.tail_limit = ticks;
    h->h32.tail_limit = ticks;
    return AMG_OK;
  });
}

}  // extern "C"

namespace amg {
namespace {

// Algorithmic bytes of one V-cycle with Chebyshev relaxation, one pre- and
// one post-sweep of k steps: k passes over A_l for each sweep, one over P_l
// and R_l, and each vector read or written once per kernel (level 1: f and z
// FP64); dense coarse inverse + f, z.
// Algorithmic bytes of one pass over a CSR matrix's entries: its values and
// int32 column indices (row pointers are counted by the callers).  A stream
// matrix may be read through 2-byte column offsets instead, which lowers the
// traffic of the launch, not this count of the product's bytes.
template <class T>
double csr_entry_bytes(const DevCsr<T>& M) {
  return double(M.nnz) * (sizeof(T) + 4.0);
}

template <class T>
double cheb_vcycle_bytes(const amg_solver& S, const DevHierarchy<T>& H) {
  const double sz = sizeof(T);
  double b = 0.0;
  const size_t nlev = H.lev.size();
  for (size_t l = 0; l < nlev; ++l) {
    const DevLevel<T>& L = H.lev[l];
    const int k = L.cheb.degree;
    const double n = L.n, nc = L.nc;
    const double szf = (l == 0) ? 8.0 : sz;
    const double passA = csr_entry_bytes(L.A) + 4.0 * (n + 1);
    b += 2.0 * k * passA;                                          // pre and post sweeps
    b += csr_entry_bytes(L.P) + csr_entry_bytes(L.R) + 4.0 * (n + 1) + 4.0 * (nc + 1);  // P and R
    // pre-sweep from zero, residual kept
    if (l == 0) b += n * (sz + szf);                               // m, f
    else b += n * sz * ((k == 1) ? 2.0 : 3.0);                     // d0, f (, m)
    b += n * sz * ((k == 1) ? 2.0 : 3.0);                          // x, r (, d')
    if (k >= 2) b += 7.0 * sz * n * (k - 2) + 5.0 * sz * n;        // middle steps, last step
    // restriction: r in; f_c (and d0_c from m_c) out
    b += sz * n + ((l + 1 < nlev) ? 3.0 * sz * nc : sz * nc);
    // prolongation: z_c, x_pre in; y out
    b += sz * nc + 2.0 * sz * n;
    // post-sweep from y
    if (k == 1) {
      b += n * (2.0 * sz + szf) + n * szf;                         // y, f, m in; z out
    } else {
      b += n * (2.0 * sz + szf) + 2.0 * sz * n;                    // init: y, f, m in; r, d out
      b += 7.0 * sz * n * (k - 2);                                 // middle steps
      b += 4.0 * sz * n + szf * n;                                 // fused last: d, x, r, m in; z out
    }
  }
  b += 8.0 * double(S.nL) * double(S.nL) + 2.0 * double(S.nL) * sz;
  return b;
}

// Algorithmic bytes of one V-cycle with npre = npost = 1: per level
// 2 passes over A_l, one over P_l and R_l each, 11 vector passes of n_l
// and 2 of n_{l+1}, by step: pre-sweep + residual reads f and m, writes
// r; restriction reads r (writes f_c); prolongation reads z_c, m, f,
// writes y; post-sweep reads y (gathered), m, f, writes z.  On level 1 f
// and z are the Krylov loop's FP64 vectors: 3 reads of f and the write of
// z at 8 bytes, the other 7 passes at the hierarchy's value size.
// Dense coarse inverse + f_L, z_L.
template <class T>
double vcycle_bytes(const amg_solver& S, const DevHierarchy<T>& H) {
  if (S.prm.relax == AMG_CHEBYSHEV) return cheb_vcycle_bytes(S, H);
  const double sz = sizeof(T);
  double b = 0.0;
  for (size_t l = 0; l < H.lev.size(); ++l) {
    const DevLevel<T>& L = H.lev[l];
    const double nl = L.n, ncl = L.nc;
    b += csr_entry_bytes(L.A) + csr_entry_bytes(l == 0 && L.As.val ? L.As : L.A) + csr_entry_bytes(L.P) +
         csr_entry_bytes(L.R);
    b += 12.0 * (nl + 1) + 4.0 * (ncl + 1) + 2.0 * ncl * sz;
    b += (l == 0) ? nl * (4.0 * 8.0 + 7.0 * sz) : 11.0 * nl * sz;
  }
  b += 8.0 * double(S.nL) * double(S.nL) + 2.0 * double(S.nL) * sz;
  return b;
}

template <class T>
double time_level0_kernel(amg_solver& S, DevHierarchy<T>& H, int which, int reps, hipStream_t s,
                          double* bytes) {
  if (H.lev.empty()) throw SetupError{-1, "single-level hierarchy: no level-1 kernels to time"};
  DevLevel<T>& lv = H.lev[0];
  const double n = lv.n, nc = lv.nc;
  const double sz = sizeof(T);
  T* fnext = H.lev.size() > 1 ? H.lev[1].f : H.fL;
  const T* zc = H.lev.size() > 1 ? H.lev[1].z : H.zL;
  const int nb = vec_blocks(S.n);
  fill_kernel<double><<<nb, kVecBS, 0, s>>>(static_cast<int>(S.n), S.r, 1.0);
  fill_kernel<double><<<nb, kVecBS, 0, s>>>(static_cast<int>(S.n), S.p, 1.0);
  fill_kernel<T><<<vec_blocks(lv.n), kVecBS, 0, s>>>(lv.n, lv.y, T(1));
  fill_kernel<T><<<vec_blocks(lv.nc), kVecBS, 0, s>>>(lv.nc, const_cast<T*>(zc), T(1));
  AMG_LAUNCHED();
  auto launch = [&](hipStream_t st) {
    switch (which) {
      case 0:
        launch_spmv(S.A0, GatherX<double, double>{S.p}, EpiStoreDot{S.q, S.p}, S.partials, nullptr, st);
        break;
      case 1:
        if (lv.As.val)
          launch_spmv(lv.As, GatherX<T, double>{S.r}, EpiResid<T, double>{lv.r, S.r}, nullptr, nullptr, st);
        else
          launch_spmv(lv.A, GatherMF<T, double>{lv.m, S.r}, EpiResid<T, double>{lv.r, S.r}, nullptr, nullptr, st);
        break;
      case 2:
        launch_spmv(lv.A, GatherX<T, T>{lv.y}, EpiSmooth<T, double, double, 1>{S.z, lv.y, lv.m, S.r}, S.partials,
                    nullptr, st);
        break;
      case 3:
        launch_spmv(lv.R, GatherX<T, T>{lv.r}, EpiStore<T, T>{fnext}, nullptr, nullptr, st);
        break;
      case 4:
        launch_spmv(lv.P, GatherX<T, T>{zc}, EpiProlong<T, double, 1>{lv.y, lv.m, S.r, nullptr}, nullptr, nullptr,
                    st);
        break;
      case 6:
        launch_spmv(S.Afull, GatherX<double, double>{S.p}, EpiStoreDot{S.q, S.p}, S.partials, nullptr, st);
        break;
      case 7: {
        VcycleOpts o{S.prm.npre, S.prm.npost, S.prm.relax};
        const SchurOps so{&S.Dm, &S.Gs, S.mu, S.rp, S.split.n_u};
        SchurPrecond<T> P(Vcycle<T>(&H, S.Ainv, S.nL, o), so);
        P.template run<0>(S.r, S.z, S.partials, nullptr, st);
        break;
      }
      default: {
        VcycleOpts o{S.prm.npre, S.prm.npost, S.prm.relax};
        Vcycle<T> V(&H, S.Ainv, S.nL, o);
        V.template run<0>(S.r, S.z, S.partials, nullptr, st);
        break;
      }
    }
  };
  // The timed launches are captured into one graph so that the measured
  // interval holds only device work (no host launch gaps).
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  AMG_HIP(hipStreamBeginCapture(S.cap_stream, hipStreamCaptureModeThreadLocal));
  try {
    for (int k = 0; k < reps; ++k) launch(S.cap_stream);
  } catch (...) {
    (void)hipStreamEndCapture(S.cap_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  AMG_HIP(hipStreamEndCapture(S.cap_stream, &g));
  AMG_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
  hipEvent_t e0, e1;
  AMG_HIP(hipEventCreate(&e0));
  AMG_HIP(hipEventCreate(&e1));
  AMG_HIP(hipGraphLaunch(ge, s));  // warm-up
  AMG_HIP(hipEventRecord(e0, s));
  AMG_HIP(hipGraphLaunch(ge, s));
  AMG_HIP(hipEventRecord(e1, s));
  AMG_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  AMG_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipGraphExecDestroy(ge);
  (void)hipGraphDestroy(g);
  check_tail(H, s);
  if (which == 5) {
    *bytes = vcycle_bytes(S, H);
    return 1000.0 * ms / reps;
  }
  if (which == 6) {
    // the whole system: p in, q out (p also the dot's second operand)
    const double na = double(S.Afull.rows);
    *bytes = csr_entry_bytes(S.Afull) + 4.0 * (na + 1) + 16.0 * na;
    return 1000.0 * ms / reps;
  }
  if (which == 7) {
    // r_p' = r_p - (D diag(M_u)) r_u: D's arrays, r_u gathered, r_p in, r_p' out;
    // the pressure V-cycle; z_u = M_u (r_u - G z_p): G's arrays, z_p
    // gathered, M_u and r_u in, z_u out.
    const double nu = double(S.split.n_u), np = double(S.Dm.rows);
    double b = csr_entry_bytes(S.Dm) + 4.0 * (np + 1) + 8.0 * nu + 16.0 * np;
    b += vcycle_bytes(S, H);
    b += csr_entry_bytes(S.Gs) + 4.0 * (nu + 1) + 8.0 * np + 24.0 * nu;
    *bytes = b;
    return 1000.0 * ms / reps;
  }
  const double idx = 4.0;
  switch (which) {
    case 0: *bytes = csr_entry_bytes(S.A0) + idx * (n + 1) + 16 * n; break;  // p in, q out
    case 1:  // f, m (folded into A diag(m)) in; r out
      *bytes = csr_entry_bytes(lv.As.val ? lv.As : lv.A) + idx * (n + 1) + n * 8 + 2 * n * sz;
      break;
    case 2: *bytes = csr_entry_bytes(lv.A) + idx * (n + 1) + n * sz * 2 + n * 8 * 2; break;  // y, m, f in; z out
    case 3: *bytes = csr_entry_bytes(lv.R) + idx * (nc + 1) + n * sz + nc * sz; break;       // r in; f_c out
    default:  // z_c, f, m in; y out
      *bytes = csr_entry_bytes(lv.P) + idx * (n + 1) + nc * sz + n * 8 + 2 * n * sz;
      break;
  }
  return 1000.0 * ms / reps;
}

// Back-to-back block V-cycles captured in one graph, between HIP events.
// Algorithmic bytes per level l < L (one pre- and one post-sweep): two
// passes over A_l (level 1: A M for the pre-sweep) and one over P_l and
// R_l, each 16 values + 4 index bytes per block and 4 bytes per block row
// pointer; vectors of 4 n_l values: pre-sweep f (gathered and read) and r,
// restriction r in, f_c and m_c f_c out (M_c read, 16 per node), or the
// coarsest f_L; prolongation z_c in, M f (level 1: M and f) or the stored
// M f in, y out; post-sweep y (gathered and read), M, f in, z out (level 1:
// f and z FP64).  Coarsest: dense inverse + f_L, z_L.
template <class T>
double time_block_vcycle(amg_solver& S, DevBlockHierarchy<T>& H, int reps, hipStream_t s, double* bytes) {
  const int nb = vec_blocks(S.n);
  fill_kernel<double><<<nb, kVecBS, 0, s>>>(static_cast<int>(S.n), S.r, 1.0);
  AMG_LAUNCHED();
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  AMG_HIP(hipStreamBeginCapture(S.cap_stream, hipStreamCaptureModeThreadLocal));
  try {
    BlockVcycle<T> V(&H, S.Ainv, S.nL, S.prm.npre, S.prm.npost);
    for (int k = 0; k < reps; ++k) V.template run<0>(S.r, S.z, S.partials, nullptr, S.cap_stream);
  } catch (...) {
    (void)hipStreamEndCapture(S.cap_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  AMG_HIP(hipStreamEndCapture(S.cap_stream, &g));
  AMG_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
  hipEvent_t e0, e1;
  AMG_HIP(hipEventCreate(&e0));
  AMG_HIP(hipEventCreate(&e1));
  AMG_HIP(hipGraphLaunch(ge, s));  // warm-up
  AMG_HIP(hipEventRecord(e0, s));
  AMG_HIP(hipGraphLaunch(ge, s));
  AMG_HIP(hipEventRecord(e1, s));
  AMG_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  AMG_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipGraphExecDestroy(ge);
  (void)hipGraphDestroy(g);
  const double sz = sizeof(T);
  double b = 0.0;
  const size_t nlev = H.lev.size();
  for (size_t l = 0; l < nlev; ++l) {
    const DevBlockLevel<T>& L = H.lev[l];
    const double n = double(kB) * L.nb, nbr = L.nb, ncb = L.R.rows, nc = double(kB) * ncb;
    const double sf = (l == 0) ? 8.0 : sz;  // level 1: f and z are the Krylov loop's FP64 vectors
    auto pass = [&](const DevBsr<T>& M) { return double(M.nnzb) * (16.0 * sz + 4.0) + 4.0 * (M.rows + 1); };
    b += 2.0 * pass(L.A) + pass(L.P) + pass(L.R);
    b += (l == 0) ? n * sf * 2.0 + n * sz : n * sz * 3.0;                          // pre-sweep: f (or m f), f in; r out
    b += n * sz + ((l + 1 < nlev) ? 2.0 * nc * sz + 16.0 * ncb * sz : nc * sz);     // restriction
    b += nc * sz + ((l == 0) ? 16.0 * nbr * sz + n * sf : n * sz) + n * sz;         // prolongation
    b += 2.0 * n * sz + 16.0 * nbr * sz + n * sf + n * sf;                          // post-sweep
  }
  b += 8.0 * double(S.nL) * double(S.nL) + 2.0 * double(S.nL) * sz;
  *bytes = b;
  return 1000.0 * ms / reps;
}

}  // namespace
}  // namespace amg

extern "C" {

amg_status amg_time_kernel(amg_handle h, int32_t which, int32_t reps, void* hip_stream, double* avg_us,
                           double* bytes) {
  return guarded([&]() -> amg_status {
    if (!h || !avg_us || !bytes || reps < 1 || which < 0 || which > 7) throw SetupError{-1, "bad argument"};
    if (!h->on_device) throw SetupError{-1, "handle was built by amg_setup_host: no device data"};
    if (which >= 6 && !h->schur) throw SetupError{-1, "which = 6, 7 need a field-split handle"};
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (h->block) {
      if (which != 5) throw SetupError{-1, "block-value handles time the whole V-cycle only (which = 5)"};
      if (h->prm.npre != 1 || h->prm.npost != 1)
        throw SetupError{-1, "block V-cycle timing counts bytes for npre = npost = 1 only"};
      if (h->prm.precision == AMG_MIXED) *avg_us = time_block_vcycle<float>(*h, h->bh32, reps, s, bytes);
      else *avg_us = time_block_vcycle<double>(*h, h->bh64, reps, s, bytes);
      return AMG_OK;
    }
    if (h->prm.precision == AMG_MIXED) *avg_us = time_level0_kernel<float>(*h, h->h32, which, reps, s, bytes);
    else *avg_us = time_level0_kernel<double>(*h, h->h64, which, reps, s, bytes);
    return AMG_OK;
  });
}

int32_t amg_num_levels(amg_handle h) {
  if (!h) return 0;
  return static_cast<int32_t>(h->block ? h->bhost.levels.size() : h->host.levels.size());
}

static const HostLevel& level_of(amg_handle h, int32_t level) {
  if (!h) throw SetupError{-1, "NULL handle"};
  if (h->block) throw SetupError{-1, "block-value handle: use the block queries"};
  if (level < 0 || level >= static_cast<int32_t>(h->host.levels.size())) throw SetupError{-1, "level out of range"};
  return h->host.levels[level];
}

static const BlockLevel& block_level_of(amg_handle h, int32_t level) {
  if (!h) throw SetupError{-1, "NULL handle"};
  if (!h->block) throw SetupError{-1, "not a block-value handle"};
  if (level < 0 || level >= static_cast<int32_t>(h->bhost.levels.size())) throw SetupError{-1, "level out of range"};
  return h->bhost.levels[level];
}

amg_status amg_level_info(amg_handle h, int32_t level, int64_t* n, int64_t* nnz_A, int64_t* nnz_P) {
  return guarded([&]() -> amg_status {
    if (h && h->block) {
      const BlockLevel& L = block_level_of(h, level);
      if (n) *n = L.A.rows;
      if (nnz_A) *nnz_A = L.A.nnzb();
      if (nnz_P) *nnz_P = L.P.nnzb();
      return AMG_OK;
    }
    const HostLevel& L = level_of(h, level);
    if (n) *n = L.A.rows;
    if (nnz_A) *nnz_A = L.A.nnz();
    if (nnz_P) *nnz_P = L.P.nnz();
    return AMG_OK;
  });
}

amg_status amg_get_aggregates(amg_handle h, int32_t level, int32_t* agg_host) {
  return guarded([&]() -> amg_status {
    const std::vector<int32_t>& agg = (h && h->block) ? block_level_of(h, level).agg : level_of(h, level).agg;
    if (!agg_host) throw SetupError{-1, "NULL output"};
    if (agg.empty()) throw SetupError{-1, "the coarsest level has no aggregates"};
    std::memcpy(agg_host, agg.data(), agg.size() * sizeof(int32_t));
    return AMG_OK;
  });
}

amg_status amg_get_level_bsr(amg_handle h, int32_t level, int32_t which, int64_t* block_row_ptr,
                             int32_t* block_col, double* block_val) {
  return guarded([&]() -> amg_status {
    const BlockLevel& L = block_level_of(h, level);
    if (!block_row_ptr || !block_col || !block_val) throw SetupError{-1, "NULL output"};
    const Bsr* M = which == 0 ? &L.A : which == 1 ? &L.P : which == 2 ? &L.R : nullptr;
    if (!M) throw SetupError{-1, "which must be 0 (A), 1 (P) or 2 (R)"};
    if (M->ptr.empty()) throw SetupError{-1, "matrix not present on this level"};
    std::memcpy(block_row_ptr, M->ptr.data(), M->ptr.size() * sizeof(int64_t));
    std::memcpy(block_col, M->col.data(), M->col.size() * sizeof(int32_t));
    std::memcpy(block_val, M->val.data(), M->val.size() * sizeof(double));
    return AMG_OK;
  });
}

amg_status amg_get_smoother_blocks(amg_handle h, int32_t level, double* blocks, double* omega) {
  return guarded([&]() -> amg_status {
    const BlockLevel& L = block_level_of(h, level);
    if (L.M.empty()) throw SetupError{-1, "the coarsest level has no smoother"};
    if (blocks) std::memcpy(blocks, L.M.data(), L.M.size() * sizeof(double));
    if (omega) *omega = L.omega;
    return AMG_OK;
  });
}

amg_status amg_get_level_csr(amg_handle h, int32_t level, int32_t which, int64_t* row_ptr, int32_t* col,
                             double* val) {
  return guarded([&]() -> amg_status {
    const HostLevel& L = level_of(h, level);
    if (!row_ptr || !col || !val) throw SetupError{-1, "NULL output"};
    const Csr* M = which == 0 ? &L.A : which == 1 ? &L.P : which == 2 ? &L.R : nullptr;
    if (!M) throw SetupError{-1, "which must be 0 (A), 1 (P) or 2 (R)"};
    if (M->ptr.empty()) throw SetupError{-1, "matrix not present on this level"};
    std::memcpy(row_ptr, M->ptr.data(), M->ptr.size() * sizeof(int64_t));
    std::memcpy(col, M->col.data(), M->col.size() * sizeof(int32_t));
    std::memcpy(val, M->val.data(), M->val.size() * sizeof(double));
    return AMG_OK;
  });
}

amg_status amg_get_smoother(amg_handle h, int32_t level, double* m_host, double* omega, double* cheb_hi) {
  return guarded([&]() -> amg_status {
    const HostLevel& L = level_of(h, level);
    if (L.m.empty()) throw SetupError{-1, "the coarsest level has no smoother"};
    if (m_host) std::memcpy(m_host, L.m.data(), L.m.size() * sizeof(double));
    if (omega) *omega = L.omega;
    if (cheb_hi) *cheb_hi = L.cheb_hi;
    return AMG_OK;
  });
}

amg_status amg_level_kernel_info(amg_handle h, int32_t level, int32_t which, int32_t precision, int32_t* kind,
                                 int32_t* lanes, int32_t* blocks, int32_t* block_bytes) {
  return guarded([&]() -> amg_status {
    const HostLevel& L = level_of(h, level);
    const Csr* M = which == 0 ? &L.A : which == 1 ? &L.P : which == 2 ? &L.R : nullptr;
    if (!M) throw SetupError{-1, "which must be 0 (A), 1 (P) or 2 (R)"};
    if (M->ptr.empty()) throw SetupError{-1, "matrix not present on this level"};
    if (precision != AMG_FP64 && precision != AMG_MIXED) throw SetupError{-1, "bad precision"};
    const Schedule sc = precision == AMG_FP64 ? make_schedule<double>(*M) : make_schedule<float>(*M);
    if (kind) *kind = sc.kind;
    if (lanes) *lanes = sc.lanes;
    if (blocks) *blocks = sc.nblocks;
    if (block_bytes)
      *block_bytes = sc.kind != 0 ? 0 : sc.bclass == 1 ? kStreamSmallBytes : sc.bclass == 2 ? kStreamMidBytes
                                                                                           : AMG_STREAM_BYTES;
    return AMG_OK;
  });
}

}  // extern "C"

// --------------------------------------------------------------- standalone SpMV

struct amg_matrix_s {
  std::unique_ptr<DevArena> arena;
  int precision = AMG_FP64;
  DevCsr<double> d64;
  DevCsr<float> d32;
};

extern "C" {

amg_status amg_csr_upload(int64_t rows, int64_t cols, const int64_t* row_ptr, const int32_t* col,
                          const double* val, int32_t precision, void* hip_stream, amg_matrix* out) {
  if (out) *out = nullptr;
  return guarded([&]() -> amg_status {
    if (!out || !row_ptr || !col || !val) throw SetupError{-1, "NULL argument"};
    if (rows < 0 || cols < 0 || rows >= (int64_t(1) << 31) || cols >= (int64_t(1) << 31))
      throw SetupError{-1, "bad matrix shape"};
    if (precision != AMG_FP64 && precision != AMG_MIXED) throw SetupError{-1, "bad precision"};
    if (row_ptr[0] != 0) throw SetupError{-2, "row_ptr[0] must be 0"};
    for (int64_t i = 0; i < rows; ++i)
      if (row_ptr[i + 1] < row_ptr[i]) throw SetupError{-2, "row_ptr must be non-decreasing"};
    if (row_ptr[rows] >= (int64_t(1) << 31)) throw SetupError{-8, "nnz must be below 2^31"};
    for (int64_t e = 0; e < row_ptr[rows]; ++e)
      if (col[e] < 0 || col[e] >= cols) throw SetupError{-2, "column index out of range"};
    Csr M;
    M.rows = rows;
    M.cols = cols;
    M.ptr.assign(row_ptr, row_ptr + rows + 1);
    M.col.assign(col, col + row_ptr[rows]);
    M.val.assign(val, val + row_ptr[rows]);
    auto m = std::make_unique<amg_matrix_s>();
    m->arena = std::make_unique<DevArena>(nullptr, static_cast<hipStream_t>(hip_stream));
    m->arena->compact_cols = true;
    m->precision = precision;
    if (precision == AMG_FP64) m->d64 = upload_csr<double>(*m->arena, M);
    else m->d32 = upload_csr<float>(*m->arena, M);
    *out = m.release();
    return AMG_OK;
  });
}

amg_status amg_csr_spmv(amg_matrix m, const void* x_dev, void* y_dev, void* hip_stream) {
  return guarded([&]() -> amg_status {
    if (!m || !x_dev || !y_dev) throw SetupError{-1, "NULL argument"};
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (m->precision == AMG_FP64)
      launch_spmv(m->d64, GatherX<double, double>{static_cast<const double*>(x_dev)},
                  EpiStore<double, double>{static_cast<double*>(y_dev)}, nullptr, nullptr, s);
    else
      launch_spmv(m->d32, GatherX<float, float>{static_cast<const float*>(x_dev)},
                  EpiStore<float, float>{static_cast<float*>(y_dev)}, nullptr, nullptr, s);
    AMG_HIP(hipStreamSynchronize(s));
    return AMG_OK;
  });
}

amg_status amg_csr_kernel_info(amg_matrix m, int32_t* kind, int32_t* lanes, int32_t* blocks, int32_t* block_bytes) {
  return guarded([&]() -> amg_status {
    if (!m) throw SetupError{-1, "NULL matrix"};
    const bool f64 = m->precision == AMG_FP64;
    if (kind) *kind = f64 ? m->d64.kind : m->d32.kind;
    if (lanes) *lanes = f64 ? m->d64.lanes : m->d32.lanes;
    if (blocks) *blocks = f64 ? m->d64.nblocks : m->d32.nblocks;
    if (block_bytes) {
      const int k = f64 ? m->d64.kind : m->d32.kind;
      const int bc = f64 ? m->d64.bclass : m->d32.bclass;
      *block_bytes = k != 0 ? 0 : bc == 1 ? kStreamSmallBytes : bc == 2 ? kStreamMidBytes : AMG_STREAM_BYTES;
    }
    return AMG_OK;
  });
}

amg_status amg_csr_column_bytes(amg_matrix m, int32_t* bytes) {
  return guarded([&]() -> amg_status {
    if (!m || !bytes) throw SetupError{-1, "NULL argument"};
    const bool c16 = m->precision == AMG_FP64 ? m->d64.col16 != nullptr : m->d32.col16 != nullptr;
    *bytes = c16 ? 2 : 4;
    return AMG_OK;
  });
}

void amg_csr_release(amg_matrix m) { delete m; }

}  // extern "C"
