// Host-side smoothed-aggregation setup (section 2, "AMG setup"; section 3,
// "Coarsening strategies": smoothed aggregation after Vanek, Mandel and
// Brezina 1996).  Builds A_l, P_l, R_l = P_l^T and the smoother diagonals on
// the CPU; the device layer uploads the result.
#pragma once

#include <cstdint>
#include <functional>
#include <memory>
#include <new>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

namespace amg {

// Allocator of the large host arrays of a hierarchy (column indices, values,
// the strong graph): value-initialisation of elements is skipped, so resize()
// leaves new elements unset.  The memory is then first touched where it is
// filled, by the parallel loops and multi-threaded copies of the setup,
// instead of by one thread writing zeros (a page fault per 4 KB page: about
// 20 ms per 100 MB on one core).  Every resize of such an array is followed
// by writes to all of its new elements.
template <class T>
struct FillLater : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = FillLater<U>;
  };
  FillLater() = default;
  template <class U>
  FillLater(const FillLater<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept(std::is_nothrow_default_constructible<U>::value) {
    ::new (static_cast<void*>(p)) U;
  }
  template <class U, class... A>
  void construct(U* p, A&&... a) {
    ::new (static_cast<void*>(p)) U(std::forward<A>(a)...);
  }
};
template <class T>
using hvec = std::vector<T, FillLater<T>>;

struct Csr {
  int64_t rows = 0, cols = 0;
  std::vector<int64_t> ptr;  // rows + 1
  hvec<int32_t> col;         // ascending within each row
  hvec<double> val;
  int64_t nnz() const { return ptr.empty() ? 0 : ptr.back(); }
};

struct SetupParams {
  int relax = 0;  // 0 SPAI-0, 1 damped Jacobi, 2 Chebyshev
  double eps_strong = 0.08;
  double jacobi_omega = 0.72;
  int coarse_enough = 3000;
  int max_levels = 30;
  int max_coarse = 20000;
};

struct HostLevel {
  Csr A, P, R;                // P, R empty on the coarsest level
  std::vector<int32_t> agg;   // aggregate per node, -1 isolated
  std::vector<double> m;      // smoother diagonal
  double omega = 0.0;         // prolongator damping
  double cheb_hi = 0.0;       // Chebyshev: Gershgorin bound of D^-1 A
  double eps = 0.0;           // strength threshold used on this level
};

// Wall time of the setup by step (seconds, summed over the levels); the
// order is the one amg_setup_profile documents.
enum SetupPhase : int {
  kPhInput = 0,      // copy and validation of the caller's CSR
  kPhStrength,       // strength graph
  kPhAggregate,      // aggregation
  kPhProlong,        // filtered matrix, omega and the smoothed prolongator
  kPhTranspose,      // R = P^T
  kPhSmoother,       // smoother diagonals (and Chebyshev bounds)
  kPhGalerkin,       // A_{l+1} = R (A P)
  kPhUpload,         // level matrices, vectors and SpMV schedules to the device
  kPhCoarse,         // dense inverse of the coarsest operator
  kPhOther,          // everything else (Krylov vectors, fused-launch plan)
  kPhCount
};

struct HostHierarchy {
  std::vector<HostLevel> levels;  // the last one is the coarsest (A only)
  double phase_s[kPhCount] = {};
};

// Seconds of a monotonic clock.
double setup_clock();

// A named roctx range on the calling thread for the object's lifetime (shown
// by rocprofv3 --marker-trace; a no-op when no profiler is attached).
class TraceRange {
 public:
  explicit TraceRange(const char* name);
  ~TraceRange();
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

// Wall time of the setup by step: enter(p) ends the running step, adds its
// seconds to acc[step] and starts step p; each step is also a roctx range
// "amg setup: <step>".  The destructor ends the running step.
class PhaseClock {
 public:
  explicit PhaseClock(double* acc) : acc_(acc) {}
  ~PhaseClock() { stop(); }
  PhaseClock(const PhaseClock&) = delete;
  PhaseClock& operator=(const PhaseClock&) = delete;
  void enter(int phase);
  void stop();

 private:
  double* acc_;
  int cur_ = -1;
  double t0_ = 0.0;
};

// Error raised by the setup; code is an amg_status value.
struct SetupError {
  int code;
  std::string msg;
};

// Validate a CSR input as the C ABI requires; throws SetupError.  With
// require_diag false a row's diagonal may be missing or of any sign (the
// whole system of a field split, whose pressure block may be zero).
void validate_csr(int64_t n, const int64_t* ptr, const int32_t* col, const double* val, bool require_diag = true);

// Limit the worker threads the setup of the calling thread uses (0 = default).
void set_setup_threads(int n);
// Worker threads the setup of the calling thread may use (at least 1).
int setup_threads();

// Sets the calling thread's setup thread limit for a scope.
class ScopedSetupThreads {
 public:
  explicit ScopedSetupThreads(int n);
  ~ScopedSetupThreads();
  ScopedSetupThreads(const ScopedSetupThreads&) = delete;
  ScopedSetupThreads& operator=(const ScopedSetupThreads&) = delete;

 private:
  int saved_;
};

// memcpy split over the setup's worker threads (large copies only).
void copy_parallel(void* dst, const void* src, size_t bytes);

// Runs fn(begin, end) over [0, n) in contiguous chunks on the calling
// thread's setup worker threads (one chunk when n is small); fn must not throw.
void for_row_ranges(int64_t n, const std::function<void(int64_t, int64_t)>& fn);

struct Graph;

// Optional accelerator for the data-parallel steps of one level (the device).
// Every step must give exactly what the host step gives, or return false to
// leave that step to the host.  The steps of a level are called in order:
// begin_level, strength, prolongator, transpose, smoother, galerkin;
// `from_galerkin` tells that A is the product the accelerator returned for the
// previous level.
//
// A step may return with the column indices and values of its output matrix
// (P, R = P^T, the next level's A) and the smoother diagonal still being
// copied into the given objects; row pointers and sizes are final.  Those
// objects must stay where they are and must not be read until
// finish_host_copies() returns; a step that returns false has finished them.
class SetupAccel {
 public:
  virtual ~SetupAccel() = default;
  virtual void finish_host_copies() = 0;
  virtual void begin_level(const Csr& A, bool from_galerkin) = 0;
  virtual bool strength(const Csr& A, double eps, Graph& S) = 0;
  virtual bool prolongator(const Csr& A, const Graph& S, const std::vector<int32_t>& agg, int32_t nc, Csr& P,
                           double* omega) = 0;
  virtual bool transpose(const Csr& P, Csr& R) = 0;
  virtual bool smoother(const Csr& A, const SetupParams& prm, std::vector<double>& m) = 0;
  virtual bool galerkin(const Csr& R, const Csr& A, const Csr& P, Csr& Ac) = 0;
  // The host is about to aggregate (the device is idle meanwhile).
  virtual void host_work_begins() {}
};

// Full hierarchy; throws SetupError.  `accel` (optional) runs the
// data-parallel steps elsewhere (on the device).
HostHierarchy build_hierarchy(Csr A, const SetupParams& prm, SetupAccel* accel = nullptr);

// Steps, exposed for tests of the host logic.
struct Graph {
  std::vector<int64_t> ptr;
  hvec<int32_t> idx;
};
Graph strength_graph(const Csr& A, double eps);
std::vector<int32_t> aggregate(const Graph& S, int32_t* count);
Csr transpose(const Csr& M);
Csr spgemm(const Csr& A, const Csr& B);

}  // namespace amg
