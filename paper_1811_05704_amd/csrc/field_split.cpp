// Host part of the Schur-complement field split: block extraction, SPAI-0 of
// the velocity block and the approximate Schur complement (field_split.hpp).
#include "field_split.hpp"

#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace amg {

namespace {

// First entry of row i whose column is >= c (columns ascending).
int64_t first_at_or_after(const Csr& A, int64_t i, int64_t c) {
  const int32_t* b = A.col.data() + A.ptr[i];
  const int32_t* e = A.col.data() + A.ptr[i + 1];
  return A.ptr[i] + (std::lower_bound(b, e, static_cast<int32_t>(c)) - b);
}

// Rows [r0, r1) of A restricted to columns [c0, c1), columns shifted by -c0
// and values scaled by scale[col] when scale is given.
Csr extract(const Csr& A, int64_t r0, int64_t r1, int64_t c0, int64_t c1, const double* scale) {
  Csr B;
  B.rows = r1 - r0;
  B.cols = c1 - c0;
  B.ptr.assign(B.rows + 1, 0);
  for_row_ranges(B.rows, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i)
      B.ptr[i + 1] = first_at_or_after(A, r0 + i, c1) - first_at_or_after(A, r0 + i, c0);
  });
  for (int64_t i = 0; i < B.rows; ++i) B.ptr[i + 1] += B.ptr[i];
  B.col.resize(B.nnz());
  B.val.resize(B.nnz());
  for_row_ranges(B.rows, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      int64_t o = B.ptr[i];
      for (int64_t k = first_at_or_after(A, r0 + i, c0); k < first_at_or_after(A, r0 + i, c1); ++k, ++o) {
        const int32_t j = A.col[k];
        B.col[o] = static_cast<int32_t>(j - c0);
        B.val[o] = scale ? A.val[k] * scale[j] : A.val[k];
      }
    }
  });
  return B;
}

}  // namespace

int64_t field_order(int64_t n, const uint8_t* pmask, std::vector<int32_t>* old_of_new) {
  if (!pmask) throw SetupError{-1, "pmask must not be NULL"};
  int64_t n_u = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (pmask[i] > 1) throw SetupError{-1, "pmask entries must be 0 (velocity) or 1 (pressure)"};
    n_u += pmask[i] == 0;
  }
  if (n_u == 0 || n_u == n) throw SetupError{-1, "pmask must mark some but not all unknowns as pressure"};
  old_of_new->resize(n);
  int64_t u = 0, p = n_u;
  for (int64_t i = 0; i < n; ++i) (*old_of_new)[pmask[i] ? p++ : u++] = static_cast<int32_t>(i);
  return n_u;
}

Csr permute_symmetric(const Csr& A, const std::vector<int32_t>& old_of_new) {
  const int64_t n = A.rows;
  std::vector<int32_t> new_of_old(n);
  for (int64_t j = 0; j < n; ++j) new_of_old[old_of_new[j]] = static_cast<int32_t>(j);
  Csr B;
  B.rows = B.cols = n;
  B.ptr.assign(n + 1, 0);
  for (int64_t j = 0; j < n; ++j) B.ptr[j + 1] = B.ptr[j] + (A.ptr[old_of_new[j] + 1] - A.ptr[old_of_new[j]]);
  B.col.resize(B.nnz());
  B.val.resize(B.nnz());
  for_row_ranges(n, [&](int64_t b, int64_t e) {
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t j = b; j < e; ++j) {
      const int64_t i = old_of_new[j];
      row.clear();
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) row.emplace_back(new_of_old[A.col[k]], A.val[k]);
      std::sort(row.begin(), row.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
      int64_t o = B.ptr[j];
      for (const auto& c : row) {
        B.col[o] = c.first;
        B.val[o] = c.second;
        ++o;
      }
    }
  });
  return B;
}

Csr split_fields(Csr A, int64_t n_u, FieldSplit* out) {
  const int64_t n = A.rows;
  if (n_u <= 0 || n_u >= n) throw SetupError{-1, "velocity unknowns n_u must satisfy 0 < n_u < n"};
  const int64_t np = n - n_u;

  // velocity diagonal, its reciprocal, and SPAI-0 over K's columns
  hvec<double> kinv(n_u);
  out->mu.resize(n_u);
  std::atomic<int64_t> bad{-1};
  for_row_ranges(n_u, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      double d = 0.0, ss = 0.0;
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1] && A.col[k] < n_u; ++k) {
        const double v = A.val[k];
        ss += v * v;
        if (A.col[k] == i) d = v;
      }
      if (d == 0.0) {
        int64_t cur = bad.load();
        while ((cur < 0 || i < cur) && !bad.compare_exchange_weak(cur, i)) {
        }
        kinv[i] = 0.0;
        out->mu[i] = 0.0;
        continue;
      }
      kinv[i] = 1.0 / d;
      out->mu[i] = d / ss;
    }
  });
  if (bad.load() >= 0)
    throw SetupError{-3, "velocity row " + std::to_string(bad.load()) + " has a zero or missing diagonal"};

  out->n_u = n_u;
  out->G = extract(A, 0, n_u, n_u, n, nullptr);
  out->Dm = extract(A, n_u, n, 0, n_u, out->mu.data());
  const Csr Dk = extract(A, n_u, n, 0, n_u, kinv.data());  // D diag(K)^-1
  const Csr& G = out->G;

  // S_hat row i = S row i - (D diag(K)^-1 G) row i.  Each chunk of rows is
  // computed once into the chunk's own arrays (dense accumulators over the
  // pressure columns, left unset until a row first touches a column), then
  // the chunks are copied into place after the row counts are summed.
  Csr Sh;
  Sh.rows = Sh.cols = np;
  Sh.ptr.assign(np + 1, 0);
  struct Chunk {
    int64_t b = 0;
    hvec<int32_t> col;
    hvec<double> val;
  };
  std::mutex mu;
  std::vector<Chunk> chunks;
  for_row_ranges(np, [&](int64_t b, int64_t e) {
    Chunk c;
    c.b = b;
    hvec<double> acc(np), sv(np);
    std::vector<int32_t> mark(np, -1);
    std::vector<int32_t> cols;
    for (int64_t i = b; i < e; ++i) {
      const int32_t stamp = static_cast<int32_t>(i);
      cols.clear();
      for (int64_t k = Dk.ptr[i]; k < Dk.ptr[i + 1]; ++k) {
        const int32_t v = Dk.col[k];
        const double w = Dk.val[k];
        for (int64_t q = G.ptr[v]; q < G.ptr[v + 1]; ++q) {
          const int32_t j = G.col[q];
          if (mark[j] != stamp) {
            mark[j] = stamp;
            acc[j] = 0.0;
            sv[j] = 0.0;
            cols.push_back(j);
          }
          acc[j] += w * G.val[q];
        }
      }
      for (int64_t k = first_at_or_after(A, n_u + i, n_u); k < A.ptr[n_u + i + 1]; ++k) {
        const int32_t j = static_cast<int32_t>(A.col[k] - n_u);
        if (mark[j] != stamp) {
          mark[j] = stamp;
          acc[j] = 0.0;
          cols.push_back(j);
        }
        sv[j] = A.val[k];
      }
      std::sort(cols.begin(), cols.end());
      int64_t cnt = 0;
      for (int32_t j : cols) {
        const double t = sv[j] - acc[j];
        if (t == 0.0) continue;
        c.col.push_back(j);
        c.val.push_back(t);
        ++cnt;
      }
      Sh.ptr[i + 1] = cnt;
    }
    std::lock_guard<std::mutex> lk(mu);
    chunks.push_back(std::move(c));
  });
  for (int64_t i = 0; i < np; ++i) Sh.ptr[i + 1] += Sh.ptr[i];
  Sh.col.resize(Sh.nnz());
  Sh.val.resize(Sh.nnz());
  std::vector<std::thread> copiers;
  for (const Chunk& c : chunks)
    copiers.emplace_back([&Sh, &c] {
      std::copy(c.col.begin(), c.col.end(), Sh.col.begin() + Sh.ptr[c.b]);
      std::copy(c.val.begin(), c.val.end(), Sh.val.begin() + Sh.ptr[c.b]);
    });
  for (auto& t : copiers) t.join();

  // the hierarchy is built for S_hat: every row needs a positive diagonal
  std::atomic<int64_t> bad_p{-1};
  for_row_ranges(np, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      bool ok = false;
      for (int64_t k = Sh.ptr[i]; k < Sh.ptr[i + 1]; ++k)
        if (Sh.col[k] == i) ok = Sh.val[k] > 0.0;
      if (!ok) {
        int64_t cur = bad_p.load();
        while ((cur < 0 || i < cur) && !bad_p.compare_exchange_weak(cur, i)) {
        }
      }
    }
  });
  if (bad_p.load() >= 0)
    throw SetupError{-3, "pressure Schur complement row " + std::to_string(bad_p.load()) +
                             " has a missing or non-positive diagonal"};
  out->A = std::move(A);
  return Sh;
}

}  // namespace amg
