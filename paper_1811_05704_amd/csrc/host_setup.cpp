// Host-side smoothed-aggregation setup.
//
// Section 2 ("AMG setup"): starting from A_1 = A, while A_l is larger than a
// direct solver should take, build a prolongator P_l and restriction
// R_l = P_l^T and form the Galerkin operator A_{l+1} = R_l A_l P_l.  The
// transfer operators come from smoothed aggregation (section 3, "Coarsening
// strategies"; Vanek, Mandel and Brezina 1996):
//   1. strength graph: j != i is strong for i when a_ij^2 > eps^2 |a_ii a_jj|,
//      made symmetric by union; eps halves on every coarser level;
//   2. greedy aggregation in natural order (root nodes whose whole strong
//      neighbourhood is free; leftovers join the aggregate of their
//      lowest-index neighbour aggregated in the first pass; anything still
//      left starts its own aggregate);
//   3. piecewise-constant tentative prolongator (entries 1);
//   4. filtered matrix: weak entries are lumped into the diagonal;
//   5. P = P_hat - omega D_F^-1 A_F P_hat with omega = (4/3) / rho, rho the
//      Gershgorin bound of D_F^-1 A_F.
// No entry is ever dropped by value: every structurally generated entry of
// P and of A_{l+1} is kept.  Arithmetic is done in FP64 in the natural order
// of each definition (rows in column order), without fused multiply-adds.
//
// The smoother diagonal for each level (section 3, "Relaxation methods"):
// SPAI-0, m_i = a_ii / sum_j a_ij^2 (Broeker and Grote 2002), damped Jacobi,
// m_i = omega_J / a_ii, or for Chebyshev m_i = 1 / a_ii together with the
// Gershgorin bound of the spectrum of D^-1 A.

#include "host_setup.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>

#include <rocprofiler-sdk-roctx/roctx.h>

namespace amg {

namespace {

constexpr int32_t kUnagg = -2;
constexpr int32_t kIsolated = -1;

thread_local int tl_max_threads = 0;  // 0: use the hardware concurrency (at most 16)

int num_threads() {
  if (tl_max_threads > 0) return tl_max_threads;
  unsigned h = std::thread::hardware_concurrency();
  if (h == 0) h = 1;
  return static_cast<int>(std::min(h, 16u));
}

// Run fn(begin, end) over [0, n) split in contiguous chunks on worker threads.
template <class F>
void parallel_rows(int64_t n, F fn) {
  int nt = num_threads();
  if (n < 65536 || nt == 1) {
    fn(int64_t(0), n);
    return;
  }
  std::vector<std::thread> th;
  int64_t chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    int64_t b = t * chunk, e = std::min(n, b + chunk);
    if (b >= e) break;
    th.emplace_back([=] { fn(b, e); });
  }
  for (auto& x : th) x.join();
}

[[noreturn]] void fail(int code, const std::string& msg) { throw SetupError{code, msg}; }

std::vector<double> diagonal(const Csr& A) {
  std::vector<double> d(A.rows, 0.0);
  for (int64_t i = 0; i < A.rows; ++i)
    for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e)
      if (A.col[e] == i) d[i] = A.val[e];
  return d;
}

}  // namespace

void set_setup_threads(int n) { tl_max_threads = n; }

int setup_threads() { return num_threads(); }

ScopedSetupThreads::ScopedSetupThreads(int n) : saved_(tl_max_threads) { tl_max_threads = n; }
ScopedSetupThreads::~ScopedSetupThreads() { tl_max_threads = saved_; }

void for_row_ranges(int64_t n, const std::function<void(int64_t, int64_t)>& fn) { parallel_rows(n, fn); }

void copy_parallel(void* dst, const void* src, size_t bytes) {
  constexpr size_t kChunk = size_t(8) << 20;
  const int nt = num_threads();
  if (bytes < 4 * kChunk || nt == 1) {
    if (bytes) std::memcpy(dst, src, bytes);
    return;
  }
  const size_t per = (bytes + nt - 1) / nt;
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) {
    const size_t b = t * per, e = std::min(bytes, b + per);
    if (b >= e) break;
    th.emplace_back([=] { std::memcpy(static_cast<char*>(dst) + b, static_cast<const char*>(src) + b, e - b); });
  }
  for (auto& x : th) x.join();
}

void validate_csr(int64_t n, const int64_t* ptr, const int32_t* col, const double* val, bool require_diag) {
  if (n <= 0 || !ptr || !col || !val) fail(-1, "null array or non-positive size");
  // int32 indices everywhere on the device; grid-stride loops step past the
  // last index by up to 2^25 before they stop, so that much headroom is kept
  constexpr int64_t kIndexLimit = (int64_t(1) << 31) - (int64_t(1) << 25);
  if (n >= kIndexLimit) fail(-8, "n must be below 2^31 - 2^25");
  if (ptr[0] != 0) fail(-2, "row_ptr[0] must be 0");
  for (int64_t i = 0; i < n; ++i)
    if (ptr[i + 1] < ptr[i]) fail(-2, "row_ptr must be non-decreasing");
  if (ptr[n] >= kIndexLimit) fail(-8, "nnz must be below 2^31 - 2^25");
  // Rows are checked in parallel chunks; the lowest failing row is reported.
  struct Bad {
    int64_t row = -1;
    int code = 0;
    const char* what = nullptr;
  };
  auto check = [&](int64_t b, int64_t e) -> Bad {
    for (int64_t i = b; i < e; ++i) {
      bool has_diag = false;
      for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
        const int32_t c = col[k];
        if (c < 0 || c >= n) return {i, -2, "column index out of range in row "};
        if (k > ptr[i] && col[k - 1] >= c) return {i, -2, "columns not strictly ascending in row "};
        if (!std::isfinite(val[k])) return {i, -9, "non-finite matrix value in row "};
        if (c == i) {
          has_diag = true;
          if (require_diag && !(val[k] > 0.0)) return {i, -3, "non-positive diagonal in row "};
        }
      }
      if (require_diag && !has_diag) return {i, -3, "missing diagonal in row "};
    }
    return {};
  };
  const int nt = (n < 65536) ? 1 : num_threads();
  std::vector<Bad> bad(nt);
  const int64_t chunk = (n + nt - 1) / nt;
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) {
    const int64_t b = t * chunk, e = std::min(n, b + chunk);
    if (b >= e) break;
    if (nt == 1) bad[t] = check(b, e);
    else th.emplace_back([&, t, b, e] { bad[t] = check(b, e); });
  }
  for (auto& x : th) x.join();
  for (const Bad& x : bad)
    if (x.row >= 0) fail(x.code, std::string(x.what) + std::to_string(x.row));
}

Graph strength_graph(const Csr& A, double eps) {
  const int64_t n = A.rows;
  const std::vector<double> d = diagonal(A);
  const double eps2 = eps * eps;
  // Directed test per stored entry.
  std::vector<uint8_t> strong(A.nnz(), 0);
  std::vector<int64_t> cnt_t(n + 1, 0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
      int32_t j = A.col[e];
      if (j == i) continue;
      double v = A.val[e];
      if (v * v > eps2 * std::fabs(d[i] * d[j])) {
        strong[e] = 1;
        cnt_t[j + 1]++;
      }
    }
  // Transposed directed graph: rows filled in increasing source order (sorted).
  for (int64_t i = 0; i < n; ++i) cnt_t[i + 1] += cnt_t[i];
  std::vector<int32_t> idx_t(cnt_t[n]);
  {
    std::vector<int64_t> pos(cnt_t.begin(), cnt_t.end() - 1);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e)
        if (strong[e]) idx_t[pos[A.col[e]]++] = static_cast<int32_t>(i);
  }
  // Union of the two sorted lists per row.
  Graph S;
  S.ptr.assign(n + 1, 0);
  auto merge_row = [&](int64_t i, int32_t* out) -> int64_t {
    int64_t a = A.ptr[i], ae = A.ptr[i + 1], b = cnt_t[i], be = cnt_t[i + 1];
    int64_t k = 0;
    while (true) {
      while (a < ae && !strong[a]) ++a;
      bool ha = a < ae, hb = b < be;
      if (!ha && !hb) break;
      int32_t ca = ha ? A.col[a] : INT32_MAX;
      int32_t cb = hb ? idx_t[b] : INT32_MAX;
      int32_t c = std::min(ca, cb);
      if (out) out[k] = c;
      ++k;
      if (ca == c) ++a;
      if (cb == c) ++b;
    }
    return k;
  };
  for (int64_t i = 0; i < n; ++i) S.ptr[i + 1] = S.ptr[i] + merge_row(i, nullptr);
  S.idx.resize(S.ptr[n]);
  parallel_rows(n, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) merge_row(i, S.idx.data() + S.ptr[i]);
  });
  return S;
}

std::vector<int32_t> aggregate(const Graph& S, int32_t* count) {
  const int64_t n = static_cast<int64_t>(S.ptr.size()) - 1;
  std::vector<int32_t> agg(n, kUnagg);
  int32_t c = 0;
  parallel_rows(n, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i)
      if (S.ptr[i] == S.ptr[i + 1]) agg[i] = kIsolated;
  });
  // Pass 1: a free node whose strong neighbours are all free becomes a root.
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] != kUnagg) continue;
    bool free_nbhd = true;
    for (int64_t e = S.ptr[i]; e < S.ptr[i + 1]; ++e)
      if (agg[S.idx[e]] != kUnagg) {
        free_nbhd = false;
        break;
      }
    if (!free_nbhd) continue;
    agg[i] = c;
    for (int64_t e = S.ptr[i]; e < S.ptr[i + 1]; ++e) agg[S.idx[e]] = c;
    ++c;
  }
  // Pass 2: leftovers join the pass-1 aggregate of their lowest-index strong
  // neighbour (neighbour lists are ascending; pass-1 membership is frozen).
  // (each node reads only the frozen copy: the nodes are independent)
  std::vector<int32_t> frozen(n);
  copy_parallel(frozen.data(), agg.data(), sizeof(int32_t) * n);
  parallel_rows(n, [&](int64_t b, int64_t end) {
    for (int64_t i = b; i < end; ++i) {
      if (agg[i] != kUnagg) continue;
      for (int64_t e = S.ptr[i]; e < S.ptr[i + 1]; ++e) {
        int32_t a = frozen[S.idx[e]];
        if (a >= 0) {
          agg[i] = a;
          break;
        }
      }
    }
  });
  // Pass 3: whatever is left starts a new aggregate with its free neighbours.
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] != kUnagg) continue;
    agg[i] = c;
    for (int64_t e = S.ptr[i]; e < S.ptr[i + 1]; ++e)
      if (agg[S.idx[e]] == kUnagg) agg[S.idx[e]] = c;
    ++c;
  }
  *count = c;
  return agg;
}

// T = M^T.  Each thread takes a contiguous range of M's rows; within a row
// of T the entries of thread t follow those of threads < t, each in row
// order, so T's rows come out in ascending column order whatever the thread
// count (the sequential transpose's result).
Csr transpose(const Csr& M) {
  Csr T;
  T.rows = M.cols;
  T.cols = M.rows;
  T.ptr.assign(T.rows + 1, 0);
  T.col.resize(M.nnz());
  T.val.resize(M.nnz());
  const int64_t nr = M.rows, nc = T.rows;
  int nt = (nr < 65536 || nc == 0) ? 1 : num_threads();
  // per-thread column counts are nt * nc int64: keep them within ~256 MB
  nt = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(nt, (int64_t(32) << 20) / std::max<int64_t>(nc, 1))));
  const int64_t chunk = (nr + nt - 1) / nt;
  std::vector<int64_t> cnt(static_cast<size_t>(nt) * nc, 0);  // cnt[t * nc + c]
  auto run = [&](auto body) {
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) {
      const int64_t b = t * chunk, e = std::min(nr, b + chunk);
      if (b >= e) break;
      if (nt == 1) body(t, b, e);
      else th.emplace_back([=] { body(t, b, e); });
    }
    for (auto& x : th) x.join();
  };
  run([&](int t, int64_t b, int64_t e) {
    int64_t* c = &cnt[static_cast<size_t>(t) * nc];
    for (int64_t k = M.ptr[b]; k < M.ptr[e]; ++k) c[M.col[k]]++;
  });
  // row pointers of T, and each thread's first slot in every row of T
  for (int64_t c = 0; c < nc; ++c) {
    int64_t s = T.ptr[c];
    for (int t = 0; t < nt; ++t) {
      const int64_t k = cnt[static_cast<size_t>(t) * nc + c];
      cnt[static_cast<size_t>(t) * nc + c] = s;
      s += k;
    }
    T.ptr[c + 1] = s;
  }
  run([&](int t, int64_t b, int64_t e) {
    int64_t* pos = &cnt[static_cast<size_t>(t) * nc];
    for (int64_t i = b; i < e; ++i)
      for (int64_t k = M.ptr[i]; k < M.ptr[i + 1]; ++k) {
        const int64_t p = pos[M.col[k]]++;
        T.col[p] = static_cast<int32_t>(i);
        T.val[p] = M.val[k];
      }
  });
  return T;
}

// C = A B (Gustavson, row by row).  For each output entry the products are
// accumulated in the order A's row is stored, then B's rows in stored order;
// output columns are sorted; structural zeros are kept.
Csr spgemm(const Csr& A, const Csr& B) {
  Csr C;
  C.rows = A.rows;
  C.cols = B.cols;
  C.ptr.assign(A.rows + 1, 0);
  const int nt = num_threads();
  // Symbolic: distinct columns per row.
  parallel_rows(A.rows, [&](int64_t b, int64_t e) {
    std::vector<int64_t> mark(B.cols, -1);
    for (int64_t i = b; i < e; ++i) {
      int64_t k = 0;
      for (int64_t ea = A.ptr[i]; ea < A.ptr[i + 1]; ++ea) {
        int32_t j = A.col[ea];
        for (int64_t eb = B.ptr[j]; eb < B.ptr[j + 1]; ++eb) {
          int32_t c = B.col[eb];
          if (mark[c] != i) {
            mark[c] = i;
            ++k;
          }
        }
      }
      C.ptr[i + 1] = k;
    }
  });
  (void)nt;
  for (int64_t i = 0; i < A.rows; ++i) C.ptr[i + 1] += C.ptr[i];
  C.col.resize(C.ptr[A.rows]);
  C.val.resize(C.ptr[A.rows]);
  // Numeric.
  parallel_rows(A.rows, [&](int64_t b, int64_t e) {
    std::vector<int64_t> mark(B.cols, -1);
    std::vector<double> acc(B.cols, 0.0);
    std::vector<int32_t> cols;
    for (int64_t i = b; i < e; ++i) {
      cols.clear();
      for (int64_t ea = A.ptr[i]; ea < A.ptr[i + 1]; ++ea) {
        int32_t j = A.col[ea];
        double a = A.val[ea];
        for (int64_t eb = B.ptr[j]; eb < B.ptr[j + 1]; ++eb) {
          int32_t c = B.col[eb];
          double prod = a * B.val[eb];
          if (mark[c] != i) {
            mark[c] = i;
            acc[c] = 0.0;
            cols.push_back(c);
          }
          acc[c] += prod;
        }
      }
      std::sort(cols.begin(), cols.end());
      int64_t p = C.ptr[i];
      for (int32_t c : cols) {
        C.col[p] = c;
        C.val[p] = acc[c];
        ++p;
      }
    }
  });
  return C;
}

namespace {

// Smoothed prolongator of one level from A, its strong graph and aggregates.
Csr smoothed_prolongator(const Csr& A, const Graph& S, const std::vector<int32_t>& agg,
                         int32_t nc, double* omega_out) {
  const int64_t n = A.rows;
  std::vector<double> dF(n);
  std::vector<uint8_t> kept(A.nnz(), 0);  // entry belongs to A_F (diagonal included)
  std::vector<double> ratio(n, 0.0);
  // Filtered matrix: strong entries kept, weak ones lumped into the diagonal.
  parallel_rows(n, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      double aii = 0.0, lumped = 0.0;
      int64_t s = S.ptr[i];
      const int64_t se = S.ptr[i + 1];
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        int32_t j = A.col[k];
        if (j == i) {
          aii = A.val[k];
          kept[k] = 1;
          continue;
        }
        while (s < se && S.idx[s] < j) ++s;
        if (s < se && S.idx[s] == j) {
          kept[k] = 1;
        } else {
          lumped += A.val[k];
        }
      }
      double d = aii + lumped;
      const bool isolated = S.ptr[i] == se;
      if (!isolated && d <= 0.0) d = aii;
      dF[i] = d;
      // Gershgorin row sum of |A_F| in column order (diagonal = d).
      double row = 0.0;
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        if (!kept[k]) continue;
        row += (A.col[k] == i) ? std::fabs(d) : std::fabs(A.val[k]);
      }
      ratio[i] = isolated ? 0.0 : row / std::fabs(d);
    }
  });
  double rho = 0.0;
  bool any = false;
  for (int64_t i = 0; i < n; ++i)
    if (S.ptr[i] != S.ptr[i + 1]) {
      rho = any ? std::max(rho, ratio[i]) : ratio[i];
      any = true;
    }
  if (!any) rho = 1.0;
  const double omega = (4.0 / 3.0) / rho;
  *omega_out = omega;

  // P = P_hat - omega D_F^-1 (A_F P_hat): row i collects, for every kept
  // entry in column order, a_F(i,j) into the column agg(j).
  Csr P;
  P.rows = n;
  P.cols = nc;
  P.ptr.assign(n + 1, 0);
  auto row_cols = [&](int64_t i, int32_t* cbuf, double* sbuf) -> int {
    int k = 0;
    for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
      if (!kept[e]) continue;
      int32_t j = A.col[e];
      int32_t c = agg[j];
      if (c < 0) continue;
      double a = (j == i) ? dF[i] : A.val[e];
      int q = 0;
      while (q < k && cbuf[q] != c) ++q;
      if (q == k) {
        cbuf[k] = c;
        sbuf[k] = 0.0;
        ++k;
      }
      sbuf[q] += a * 1.0;
    }
    return k;
  };
  int64_t maxrow = 0;
  for (int64_t i = 0; i < n; ++i) maxrow = std::max(maxrow, A.ptr[i + 1] - A.ptr[i]);
  parallel_rows(n, [&](int64_t b, int64_t e) {
    std::vector<int32_t> cb(maxrow + 1);
    std::vector<double> sb(maxrow + 1);
    for (int64_t i = b; i < e; ++i) P.ptr[i + 1] = row_cols(i, cb.data(), sb.data());
  });
  for (int64_t i = 0; i < n; ++i) P.ptr[i + 1] += P.ptr[i];
  P.col.resize(P.ptr[n]);
  P.val.resize(P.ptr[n]);
  parallel_rows(n, [&](int64_t b, int64_t e) {
    std::vector<int32_t> cb(maxrow + 1);
    std::vector<double> sb(maxrow + 1);
    std::vector<int> order(maxrow + 1);
    for (int64_t i = b; i < e; ++i) {
      int k = row_cols(i, cb.data(), sb.data());
      for (int q = 0; q < k; ++q) order[q] = q;
      std::sort(order.begin(), order.begin() + k, [&](int x, int y) { return cb[x] < cb[y]; });
      const double inv_d = 1.0 / dF[i];
      int64_t p = P.ptr[i];
      for (int q = 0; q < k; ++q) {
        int32_t c = cb[order[q]];
        double smoothed = omega * (inv_d * sb[order[q]]);
        P.col[p] = c;
        P.val[p] = (c == agg[i] ? 1.0 : 0.0) - smoothed;
        ++p;
      }
    }
  });
  return P;
}

// Gershgorin bound of the spectrum of D^-1 A: max_i (sum_j |a_ij|) / |a_ii|,
// each row summed in column order.
double gershgorin_dinv(const Csr& A) {
  double hi = 0.0;
  for (int64_t i = 0; i < A.rows; ++i) {
    double row = 0.0, aii = 0.0;
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      row += std::fabs(A.val[k]);
      if (A.col[k] == i) aii = A.val[k];
    }
    hi = std::max(hi, row / std::fabs(aii));
  }
  return hi;
}

std::vector<double> smoother_diagonal(const Csr& A, const SetupParams& prm) {
  std::vector<double> m(A.rows);
  parallel_rows(A.rows, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      double aii = 0.0, sq = 0.0;
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        double v = A.val[k];
        sq += v * v;
        if (A.col[k] == i) aii = v;
      }
      m[i] = (prm.relax == 0) ? aii / sq : (prm.relax == 1) ? prm.jacobi_omega / aii : 1.0 / aii;
    }
  });
  return m;
}

}  // namespace

double setup_clock() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

TraceRange::TraceRange(const char* name) { roctxRangePushA(name); }
TraceRange::~TraceRange() { roctxRangePop(); }

namespace {
const char* const kPhaseRange[kPhCount] = {
    "amg setup: input",       "amg setup: strength", "amg setup: aggregate", "amg setup: prolongator",
    "amg setup: transpose",   "amg setup: smoother", "amg setup: galerkin",  "amg setup: upload",
    "amg setup: coarse inverse", "amg setup: other",
};
}  // namespace

void PhaseClock::enter(int phase) {
  stop();
  cur_ = phase;
  roctxRangePushA(kPhaseRange[phase]);
  t0_ = setup_clock();
}

void PhaseClock::stop() {
  if (cur_ < 0) return;
  acc_[cur_] += setup_clock() - t0_;
  roctxRangePop();
  cur_ = -1;
}

HostHierarchy build_hierarchy(Csr A0, const SetupParams& prm, SetupAccel* accel) {
  HostHierarchy H;
  // Levels are built in place and never move (the capacity is reserved), so
  // an accelerator may still be filling a level's arrays while the next
  // level is set up (SetupAccel::finish_host_copies).
  H.levels.reserve(static_cast<size_t>(std::max(prm.max_levels, 1)) + 1);
  H.levels.emplace_back();
  H.levels[0].A = std::move(A0);
  bool from_galerkin = false;
  PhaseClock clk(H.phase_s);
  // copies into H may be in flight: they must land before H can go
  struct Settle {
    SetupAccel* a;
    bool armed = true;
    ~Settle() {
      if (armed && a) {
        try {
          a->finish_host_copies();
        } catch (...) {
        }
      }
    }
  } settle{accel};
  for (size_t l = 0;; ++l) {
    HostLevel& L = H.levels[l];
    const Csr& A = L.A;
    const int64_t n = A.rows;
    const int lvl_no = static_cast<int>(l) + 1;  // 1-based
    if (n <= prm.coarse_enough || lvl_no >= prm.max_levels) break;
    const double eps = prm.eps_strong * std::ldexp(1.0, -(lvl_no - 1));
    clk.enter(kPhUpload);
    if (accel) accel->begin_level(A, from_galerkin);
    clk.enter(kPhStrength);
    Graph S;
    if (!accel || !accel->strength(A, eps, S)) S = strength_graph(A, eps);
    clk.enter(kPhAggregate);
    if (accel) accel->host_work_begins();
    int32_t nc = 0;
    std::vector<int32_t> agg = aggregate(S, &nc);
    if (nc == 0 || nc >= n) break;  // this level is the coarsest
    L.eps = eps;
    clk.enter(kPhProlong);
    if (!accel || !accel->prolongator(A, S, agg, nc, L.P, &L.omega))
      L.P = smoothed_prolongator(A, S, agg, nc, &L.omega);
    clk.enter(kPhTranspose);
    if (!accel || !accel->transpose(L.P, L.R)) L.R = transpose(L.P);
    clk.enter(kPhSmoother);
    if (!accel || !accel->smoother(A, prm, L.m)) L.m = smoother_diagonal(A, prm);
    if (prm.relax == 2) {
      if (accel) accel->finish_host_copies();  // the bound reads A's values
      L.cheb_hi = gershgorin_dinv(A);
    }
    clk.enter(kPhGalerkin);
    L.agg = std::move(agg);
    H.levels.emplace_back();  // within the reserved capacity: L stays put
    Csr& Ac = H.levels[l + 1].A;
    from_galerkin = accel && accel->galerkin(L.R, A, L.P, Ac);
    if (!from_galerkin) Ac = spgemm(L.R, spgemm(A, L.P));
  }
  if (accel) accel->finish_host_copies();
  settle.armed = false;
  clk.stop();
  const Csr& AL = H.levels.back().A;
  if (AL.rows > prm.max_coarse)
    fail(-8, "coarsest level has " + std::to_string(AL.rows) + " rows (limit " +
                 std::to_string(prm.max_coarse) + ")");
  return H;
}

}  // namespace amg
