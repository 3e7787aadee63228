// Host-side smoothed aggregation for block values.
//
// Section 3, "Value types": the value type of a matrix may be a small static
// matrix; with kBlock x kBlock blocks the unknowns of a grid node move
// together through the hierarchy.  Each step of section 2's "AMG setup"
// (smoothed aggregation after Vanek, Mandel and Brezina 1996) is taken
// blockwise:
//   1. strength: node j != i is strong for i when s_ij^2 > eps^4 s_ii s_jj,
//      s_ij = ||A_ij||_F^2; symmetrised by union; eps halves per level;
//   2. the greedy aggregation of the scalar setup, over nodes;
//   3. tentative prolongator: an identity block for node i in aggregate c;
//   4. filtered matrix: weak blocks summed into the diagonal block (kept as
//      A_ii for a non-isolated node whose lumped block's symmetric part is
//      not positive definite);
//   5. P = P_hat - omega D_F^-1 A_F P_hat, omega = (4/3) / rho, rho the
//      Gershgorin bound of D_F^-1 A_F (largest row sum of its magnitudes);
//   6. R = P^T (blocks transposed), A_{l+1} = R (A P);
//   7. smoother blocks: block SPAI-0, M_i = A_ii^T (sum_j A_ij A_ij^T)^-1
//      (the block-diagonal M minimising ||I - M A||_F), or block Jacobi,
//      M_i = omega A_ii^-1.
// The arithmetic order is fixed so that the result can be reproduced: a
// block product sums over the inner index in order; a sparse block product
// accumulates C_ij from zero over k in X's row order; a block inverse is
// Gauss-Jordan elimination with partial pivoting (largest magnitude, lowest
// row on ties); a squared Frobenius norm adds the squares row-major.

#include "block_setup.hpp"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <thread>

namespace amg {

namespace {

[[noreturn]] void bfail(int code, const std::string& msg) { throw SetupError{code, msg}; }

// T = X Y (kBlock x kBlock, row-major), summed over c in order.
inline void bprod(const double* X, const double* Y, double* T) {
  for (int r = 0; r < kBlock; ++r)
    for (int s = 0; s < kBlock; ++s) {
      double t = X[r * kBlock] * Y[s];
      for (int c = 1; c < kBlock; ++c) t = t + X[r * kBlock + c] * Y[c * kBlock + s];
      T[r * kBlock + s] = t;
    }
}

inline void btranspose(const double* X, double* T) {
  for (int r = 0; r < kBlock; ++r)
    for (int s = 0; s < kBlock; ++s) T[s * kBlock + r] = X[r * kBlock + s];
}

inline double frob_sq(const double* B) {
  double s = 0.0;
  for (int k = 0; k < kBB; ++k) s = s + B[k] * B[k];
  return s;
}

// Symmetric part positive definite (Cholesky of (B + B^T) / 2 succeeds).
bool sym_part_pos_def(const double* B) {
  double H[kBB];
  for (int r = 0; r < kBlock; ++r)
    for (int s = 0; s < kBlock; ++s) H[r * kBlock + s] = 0.5 * (B[r * kBlock + s] + B[s * kBlock + r]);
  for (int j = 0; j < kBlock; ++j) {
    double d = H[j * kBlock + j];
    for (int k = 0; k < j; ++k) d -= H[j * kBlock + k] * H[j * kBlock + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    H[j * kBlock + j] = d;
    for (int i = j + 1; i < kBlock; ++i) {
      double v = H[i * kBlock + j];
      for (int k = 0; k < j; ++k) v -= H[i * kBlock + k] * H[j * kBlock + k];
      H[i * kBlock + j] = v / d;
    }
  }
  return true;
}

std::vector<double> diagonal_blocks(const Bsr& A) {
  std::vector<double> D(static_cast<size_t>(A.rows) * kBB, 0.0);
  for_row_ranges(A.rows, [&](int64_t b, int64_t end) {
    for (int64_t i = b; i < end; ++i)
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e)
        if (A.col[e] == i) std::copy(&A.val[e * kBB], &A.val[e * kBB] + kBB, &D[i * kBB]);
  });
  return D;
}

// Filtered matrix (strong off-diagonal blocks and the lumped diagonal block)
// and its diagonal blocks.
Bsr filtered_matrix(const Bsr& A, const Graph& S, std::vector<double>& DF, std::vector<uint8_t>& isolated) {
  const int64_t n = A.rows;
  const std::vector<double> D = diagonal_blocks(A);
  std::vector<double> lumped(static_cast<size_t>(n) * kBB, 0.0);
  isolated.assign(n, 0);
  Bsr F;
  F.rows = F.cols = n;
  F.ptr.assign(n + 1, 0);
  std::vector<uint8_t> keep(A.nnzb(), 0);
  // rows are independent: kept blocks, lumped weak blocks and the kept count
  for_row_ranges(n, [&](int64_t b, int64_t end) {
    for (int64_t i = b; i < end; ++i) {
      isolated[i] = S.ptr[i] == S.ptr[i + 1];
      int64_t s = S.ptr[i];
      int64_t kept = 0;
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
        const int32_t j = A.col[e];
        if (j == i) {
          keep[e] = 1;
          ++kept;
          continue;
        }
        while (s < S.ptr[i + 1] && S.idx[s] < j) ++s;
        const bool strong = s < S.ptr[i + 1] && S.idx[s] == j;
        if (strong) {
          keep[e] = 1;
          ++kept;
        } else {
          for (int k = 0; k < kBB; ++k) lumped[i * kBB + k] = lumped[i * kBB + k] + A.val[e * kBB + k];
        }
      }
      F.ptr[i + 1] = kept;
    }
  });
  for (int64_t i = 0; i < n; ++i) F.ptr[i + 1] += F.ptr[i];
  DF.assign(static_cast<size_t>(n) * kBB, 0.0);
  F.col.resize(F.ptr[n]);
  F.val.resize(static_cast<size_t>(F.ptr[n]) * kBB);
  for_row_ranges(n, [&](int64_t b, int64_t end) {
    for (int64_t i = b; i < end; ++i) {
      double* d = &DF[i * kBB];
      for (int k = 0; k < kBB; ++k) d[k] = D[i * kBB + k] + lumped[i * kBB + k];
      if (!isolated[i] && !sym_part_pos_def(d)) std::copy(&D[i * kBB], &D[i * kBB] + kBB, d);
      int64_t p = F.ptr[i];
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
        if (!keep[e]) continue;
        F.col[p] = A.col[e];
        const double* src = (A.col[e] == i) ? d : &A.val[e * kBB];
        std::copy(src, src + kBB, &F.val[p * kBB]);
        ++p;
      }
    }
  });
  return F;
}

double prolongator_damping(const Bsr& AF, const std::vector<double>& Dinv, const std::vector<uint8_t>& isolated) {
  // the maximum over the rows: exact whatever the order, so taken per range
  std::mutex mu;
  double rho = -1.0;
  bool any = false;
  for_row_ranges(AF.rows, [&](int64_t b, int64_t end) {
    double local = -1.0;
    bool local_any = false;
    double T[kBB];
    for (int64_t i = b; i < end; ++i) {
      if (isolated[i]) continue;
      double absrow[kBlock] = {};
      for (int64_t e = AF.ptr[i]; e < AF.ptr[i + 1]; ++e) {
        bprod(&Dinv[i * kBB], &AF.val[e * kBB], T);
        for (int r = 0; r < kBlock; ++r) {
          double t = std::fabs(T[r * kBlock]);
          for (int c = 1; c < kBlock; ++c) t = t + std::fabs(T[r * kBlock + c]);
          absrow[r] = absrow[r] + t;
        }
      }
      for (int r = 0; r < kBlock; ++r) {
        local = local_any ? std::max(local, absrow[r]) : absrow[r];
        local_any = true;
      }
    }
    if (!local_any) return;
    std::lock_guard<std::mutex> lk(mu);
    rho = any ? std::max(rho, local) : local;
    any = true;
  });
  if (!any) rho = 1.0;
  return (4.0 / 3.0) / rho;
}

Bsr tentative(const std::vector<int32_t>& agg, int32_t nc) {
  Bsr P;
  P.rows = static_cast<int64_t>(agg.size());
  P.cols = nc;
  P.ptr.assign(P.rows + 1, 0);
  for (int64_t i = 0; i < P.rows; ++i) {
    P.ptr[i + 1] = P.ptr[i] + (agg[i] >= 0 ? 1 : 0);
    if (agg[i] >= 0) {
      P.col.push_back(agg[i]);
      for (int r = 0; r < kBlock; ++r)
        for (int s = 0; s < kBlock; ++s) P.val.push_back(r == s ? 1.0 : 0.0);
    }
  }
  return P;
}

Bsr smoothed_prolongator(const Bsr& AF, const std::vector<double>& Dinv, const Bsr& Phat, double omega) {
  Bsr Y = block_spgemm(AF, Phat);
  for_row_ranges(Y.rows, [&](int64_t b, int64_t end) {
    double X[kBB];
    for (int64_t i = b; i < end; ++i) {
      // the tentative block of row i (at most one) sits inside Y's pattern
      const int32_t c_hat = (Phat.ptr[i + 1] > Phat.ptr[i]) ? Phat.col[Phat.ptr[i]] : -1;
      for (int64_t e = Y.ptr[i]; e < Y.ptr[i + 1]; ++e) {
        bprod(&Dinv[i * kBB], &Y.val[e * kBB], X);
        const bool on = Y.col[e] == c_hat;
        for (int r = 0; r < kBlock; ++r)
          for (int s = 0; s < kBlock; ++s) {
            const double hat = (on && r == s) ? 1.0 : 0.0;
            Y.val[e * kBB + r * kBlock + s] = hat - omega * X[r * kBlock + s];
          }
      }
    }
  });
  return Y;
}

std::vector<double> smoother_blocks(const Bsr& A, const SetupParams& prm) {
  const int64_t n = A.rows;
  std::vector<double> M(static_cast<size_t>(n) * kBB);
  const std::vector<double> D = diagonal_blocks(A);
  for_row_ranges(n, [&](int64_t b, int64_t end) {
    double G[kBB], acc[kBB], inv[kBB], Dt[kBB], At[kBB];
    for (int64_t i = b; i < end; ++i) {
      if (prm.relax == 1) {
        block_inverse(&D[i * kBB], inv);
        for (int k = 0; k < kBB; ++k) M[i * kBB + k] = prm.jacobi_omega * inv[k];
        continue;
      }
      for (int k = 0; k < kBB; ++k) acc[k] = 0.0;
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
        btranspose(&A.val[e * kBB], At);
        bprod(&A.val[e * kBB], At, G);
        for (int k = 0; k < kBB; ++k) acc[k] = acc[k] + G[k];
      }
      block_inverse(acc, inv);
      btranspose(&D[i * kBB], Dt);
      bprod(Dt, inv, &M[i * kBB]);
    }
  });
  for (double v : M)
    if (!std::isfinite(v)) bfail(-3, "singular diagonal block: the block smoother is not defined");
  return M;
}

}  // namespace

void block_inverse(const double* B, double* inv) {
  double W[kBlock][2 * kBlock];
  for (int r = 0; r < kBlock; ++r)
    for (int s = 0; s < kBlock; ++s) {
      W[r][s] = B[r * kBlock + s];
      W[r][kBlock + s] = (r == s) ? 1.0 : 0.0;
    }
  for (int c = 0; c < kBlock; ++c) {
    int p = c;
    for (int r = c + 1; r < kBlock; ++r)
      if (std::fabs(W[r][c]) > std::fabs(W[p][c])) p = r;
    if (p != c)
      for (int k = 0; k < 2 * kBlock; ++k) std::swap(W[c][k], W[p][k]);
    const double piv = W[c][c];
    for (int k = 0; k < 2 * kBlock; ++k) W[c][k] = W[c][k] / piv;
    for (int r = 0; r < kBlock; ++r) {
      if (r == c) continue;
      const double f = W[r][c];
      for (int k = 0; k < 2 * kBlock; ++k) W[r][k] = W[r][k] - f * W[c][k];
    }
  }
  for (int r = 0; r < kBlock; ++r)
    for (int s = 0; s < kBlock; ++s) inv[r * kBlock + s] = W[r][kBlock + s];
}

void validate_bsr(int64_t nb, const int64_t* ptr, const int32_t* col, const double* val) {
  if (nb <= 0 || !ptr || !col || !val) bfail(-1, "null array or non-positive size");
  constexpr int64_t kIndexLimit = (int64_t(1) << 31) - (int64_t(1) << 25);
  if (nb * kBlock >= kIndexLimit) bfail(-8, "unknowns must be below 2^31 - 2^25");
  if (ptr[0] != 0) bfail(-2, "block_row_ptr[0] must be 0");
  for (int64_t i = 0; i < nb; ++i)
    if (ptr[i + 1] < ptr[i]) bfail(-2, "block_row_ptr must be non-decreasing");
  if (ptr[nb] * kBB >= kIndexLimit) bfail(-8, "stored values must be below 2^31 - 2^25");
  for (int64_t i = 0; i < nb; ++i) {
    bool has_diag = false;
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
      const int32_t c = col[e];
      if (c < 0 || c >= nb) bfail(-2, "block column out of range in block row " + std::to_string(i));
      if (e > ptr[i] && col[e - 1] >= c)
        bfail(-2, "block columns not strictly ascending in block row " + std::to_string(i));
      for (int k = 0; k < kBB; ++k)
        if (!std::isfinite(val[e * kBB + k])) bfail(-9, "non-finite value in block row " + std::to_string(i));
      if (c == i) has_diag = true;
    }
    if (!has_diag) bfail(-3, "missing diagonal block in block row " + std::to_string(i));
  }
}

Graph block_strength_graph(const Bsr& A, double eps) {
  const int64_t n = A.rows;
  std::vector<double> sd(n, 0.0);
  std::vector<double> s(A.nnzb());
  for_row_ranges(n, [&](int64_t b, int64_t end) {
    for (int64_t i = b; i < end; ++i)
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
        s[e] = frob_sq(&A.val[e * kBB]);
        if (A.col[e] == i) sd[i] = s[e];
      }
  });
  const double e4 = (eps * eps) * (eps * eps);
  std::vector<uint8_t> strong(A.nnzb(), 0);
  for_row_ranges(n, [&](int64_t b, int64_t end) {
    for (int64_t i = b; i < end; ++i)
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
        const int32_t j = A.col[e];
        strong[e] = (j != i && s[e] * s[e] > e4 * (sd[i] * sd[j])) ? 1 : 0;
      }
  });
  // The union with the transposed strong entries: row j of T lists the rows
  // i < ... with a strong entry (i, j), in ascending order (contiguous row
  // ranges, one count array each, as in the transpose).
  int nt = (n < 65536) ? 1 : setup_threads();
  nt = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(nt, (int64_t(32) << 20) / std::max<int64_t>(n, 1))));
  const int64_t chunk = (n + nt - 1) / nt;
  auto each_range = [&](auto body) {
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) {
      const int64_t b = t * chunk, e = std::min(n, b + chunk);
      if (b >= e) break;
      if (nt == 1) body(t, b, e);
      else th.emplace_back([=] { body(t, b, e); });
    }
    for (auto& x : th) x.join();
  };
  std::vector<int64_t> cnt(static_cast<size_t>(nt) * n, 0);
  each_range([&](int t, int64_t b, int64_t e) {
    int64_t* c = &cnt[static_cast<size_t>(t) * n];
    for (int64_t i = b; i < e; ++i)
      for (int64_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q)
        if (strong[q]) c[A.col[q]]++;
  });
  std::vector<int64_t> Tp(n + 1, 0);
  for (int64_t j = 0; j < n; ++j) {
    int64_t acc = Tp[j];
    for (int t = 0; t < nt; ++t) {
      const int64_t k = cnt[t * n + j];
      cnt[t * n + j] = acc;
      acc += k;
    }
    Tp[j + 1] = acc;
  }
  std::vector<int32_t> Ti(Tp[n]);
  each_range([&](int t, int64_t b, int64_t e) {
    int64_t* pos = &cnt[static_cast<size_t>(t) * n];
    for (int64_t i = b; i < e; ++i)
      for (int64_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q)
        if (strong[q]) Ti[pos[A.col[q]]++] = static_cast<int32_t>(i);
  });
  // row i of S: the sorted union of its strong columns and of T's row i
  auto merge_row = [&](int64_t i, int32_t* out) -> int64_t {
    int64_t a = A.ptr[i], ae = A.ptr[i + 1], t = Tp[i], te = Tp[i + 1], k = 0;
    while (true) {
      while (a < ae && !strong[a]) ++a;
      if (a >= ae && t >= te) break;
      int32_t c;
      if (t >= te || (a < ae && A.col[a] <= Ti[t])) {
        c = A.col[a];
        if (t < te && Ti[t] == c) ++t;
        ++a;
      } else {
        c = Ti[t++];
      }
      if (out) out[k] = c;
      ++k;
    }
    return k;
  };
  Graph S;
  S.ptr.assign(n + 1, 0);
  for_row_ranges(n, [&](int64_t b, int64_t end) {
    for (int64_t i = b; i < end; ++i) S.ptr[i + 1] = merge_row(i, nullptr);
  });
  for (int64_t i = 0; i < n; ++i) S.ptr[i + 1] += S.ptr[i];
  S.idx.resize(S.ptr[n]);
  for_row_ranges(n, [&](int64_t b, int64_t end) {
    for (int64_t i = b; i < end; ++i) merge_row(i, S.idx.data() + S.ptr[i]);
  });
  return S;
}

Bsr block_spgemm(const Bsr& X, const Bsr& Y) {
  Bsr C;
  C.rows = X.rows;
  C.cols = Y.cols;
  C.ptr.assign(X.rows + 1, 0);
  // symbolic: distinct block columns per row (rows are independent)
  for_row_ranges(X.rows, [&](int64_t b, int64_t end) {
    std::vector<int64_t> mark(Y.cols, -1);
    for (int64_t i = b; i < end; ++i) {
      int64_t k = 0;
      for (int64_t e = X.ptr[i]; e < X.ptr[i + 1]; ++e) {
        const int32_t kk = X.col[e];
        for (int64_t f = Y.ptr[kk]; f < Y.ptr[kk + 1]; ++f) {
          const int32_t j = Y.col[f];
          if (mark[j] != i) {
            mark[j] = i;
            ++k;
          }
        }
      }
      C.ptr[i + 1] = k;
    }
  });
  for (int64_t i = 0; i < X.rows; ++i) C.ptr[i + 1] += C.ptr[i];
  C.col.resize(C.ptr[X.rows]);
  C.val.resize(static_cast<size_t>(C.ptr[X.rows]) * kBB);
  // numeric: each row summed in its own order (X's row in order, each Y row
  // in order, from zero), then written in column order
  for_row_ranges(X.rows, [&](int64_t b, int64_t end) {
    std::vector<int64_t> slot(Y.cols, -1);
    std::vector<int32_t> cols;
    std::vector<double> acc;  // kBB per column in `cols` order of first touch
    double T[kBB];
    for (int64_t i = b; i < end; ++i) {
      cols.clear();
      acc.clear();
      for (int64_t e = X.ptr[i]; e < X.ptr[i + 1]; ++e) {
        const int32_t k = X.col[e];
        for (int64_t f = Y.ptr[k]; f < Y.ptr[k + 1]; ++f) {
          const int32_t j = Y.col[f];
          if (slot[j] < 0) {
            slot[j] = static_cast<int64_t>(cols.size());
            cols.push_back(j);
            acc.resize(acc.size() + kBB, 0.0);
          }
          bprod(&X.val[e * kBB], &Y.val[f * kBB], T);
          double* a = &acc[slot[j] * kBB];
          for (int q = 0; q < kBB; ++q) a[q] = a[q] + T[q];
        }
      }
      std::vector<int32_t> sorted(cols);
      std::sort(sorted.begin(), sorted.end());
      int64_t p = C.ptr[i];
      for (int32_t j : sorted) {
        C.col[p] = j;
        const double* a = &acc[slot[j] * kBB];
        std::copy(a, a + kBB, &C.val[p * kBB]);
        ++p;
      }
      for (int32_t j : cols) slot[j] = -1;
    }
  });
  return C;
}

Bsr block_transpose(const Bsr& P) {
  Bsr R;
  R.rows = P.cols;
  R.cols = P.rows;
  R.ptr.assign(R.rows + 1, 0);
  const int64_t nr = P.rows, nc = P.cols;
  // contiguous ranges of P's rows, each with its own column counts, so that
  // every row of R lists its blocks in ascending column order
  int nt = (nr < 65536 || nc == 0) ? 1 : setup_threads();
  nt = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(nt, (int64_t(32) << 20) / std::max<int64_t>(nc, 1))));
  const int64_t chunk = (nr + nt - 1) / nt;
  std::vector<int64_t> cnt(static_cast<size_t>(nt) * nc, 0);
  auto each_range = [&](auto body) {  // body(t, first row, end row), one thread per range
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) {
      const int64_t b = t * chunk, e = std::min(nr, b + chunk);
      if (b >= e) break;
      if (nt == 1) body(t, b, e);
      else th.emplace_back([=] { body(t, b, e); });
    }
    for (auto& x : th) x.join();
  };
  each_range([&](int t, int64_t b, int64_t e) {
    int64_t* c = &cnt[static_cast<size_t>(t) * nc];
    for (int64_t i = b; i < e; ++i)
      for (int64_t q = P.ptr[i]; q < P.ptr[i + 1]; ++q) c[P.col[q]]++;
  });
  for (int64_t j = 0; j < nc; ++j) {
    int64_t s = R.ptr[j];
    for (int t = 0; t < nt; ++t) {
      const int64_t k = cnt[t * nc + j];
      cnt[t * nc + j] = s;  // first slot of range t in row j
      s += k;
    }
    R.ptr[j + 1] = s;
  }
  R.col.resize(P.nnzb());
  R.val.resize(static_cast<size_t>(P.nnzb()) * kBB);
  each_range([&](int t, int64_t b, int64_t e) {
    int64_t* pos = &cnt[static_cast<size_t>(t) * nc];
    for (int64_t i = b; i < e; ++i)
      for (int64_t q = P.ptr[i]; q < P.ptr[i + 1]; ++q) {
        const int64_t p = pos[P.col[q]]++;
        R.col[p] = static_cast<int32_t>(i);
        btranspose(&P.val[q * kBB], &R.val[p * kBB]);
      }
  });
  return R;
}

Csr bsr_to_csr(const Bsr& A) {
  Csr C;
  C.rows = A.rows * kBlock;
  C.cols = A.cols * kBlock;
  C.ptr.assign(C.rows + 1, 0);
  C.col.reserve(static_cast<size_t>(A.nnzb()) * kBB);
  C.val.reserve(static_cast<size_t>(A.nnzb()) * kBB);
  for (int64_t i = 0; i < A.rows; ++i)
    for (int r = 0; r < kBlock; ++r) {
      for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e)
        for (int c = 0; c < kBlock; ++c) {
          C.col.push_back(A.col[e] * kBlock + c);
          C.val.push_back(A.val[e * kBB + r * kBlock + c]);
        }
      C.ptr[i * kBlock + r + 1] = static_cast<int64_t>(C.col.size());
    }
  return C;
}

BlockHierarchy build_block_hierarchy(Bsr A, const SetupParams& prm) {
  if (prm.relax != 0 && prm.relax != 1) bfail(-1, "block values take the SPAI-0 or Jacobi smoother");
  BlockHierarchy H;
  PhaseClock clk(H.phase_s);
  while (true) {
    const int64_t n = A.rows;
    const int lvl_no = static_cast<int>(H.levels.size()) + 1;
    if (n * kBlock <= prm.coarse_enough || lvl_no >= prm.max_levels) break;
    const double eps = prm.eps_strong * std::ldexp(1.0, -(lvl_no - 1));
    clk.enter(kPhStrength);
    Graph S = block_strength_graph(A, eps);
    clk.enter(kPhAggregate);
    int32_t nc = 0;
    std::vector<int32_t> agg = aggregate(S, &nc);
    if (nc == 0 || nc >= n) break;
    BlockLevel L;
    L.eps = eps;
    clk.enter(kPhProlong);
    std::vector<double> DF;
    std::vector<uint8_t> isolated;
    const Bsr AF = filtered_matrix(A, S, DF, isolated);
    std::vector<double> Dinv(DF.size());
    for (int64_t i = 0; i < n; ++i) block_inverse(&DF[i * kBB], &Dinv[i * kBB]);
    L.omega = prolongator_damping(AF, Dinv, isolated);
    L.P = smoothed_prolongator(AF, Dinv, tentative(agg, nc), L.omega);
    clk.enter(kPhTranspose);
    L.R = block_transpose(L.P);
    clk.enter(kPhSmoother);
    L.M = smoother_blocks(A, prm);
    clk.enter(kPhGalerkin);
    Bsr Ac = block_spgemm(L.R, block_spgemm(A, L.P));
    L.agg = std::move(agg);
    L.A = std::move(A);
    H.levels.push_back(std::move(L));
    A = std::move(Ac);
  }
  clk.stop();
  if (A.rows * kBlock > prm.max_coarse)
    bfail(-8, "coarsest level has " + std::to_string(A.rows * kBlock) + " unknowns (limit " +
                  std::to_string(prm.max_coarse) + ")");
  BlockLevel C;
  C.A = std::move(A);
  H.levels.push_back(std::move(C));
  return H;
}

}  // namespace amg
