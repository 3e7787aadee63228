// Setup steps on the device (section 2, "AMG setup"): the Galerkin products
// A_{l+1} = R_l A_l P_l, the smoothed prolongator and the strength graph.
//
// C = A B by expansion and sort, one workgroup per block of consecutive rows
// of A holding at most kGCap products:
//   1. the products a_ik b_kj of the block are generated in the host's order
//      (A's rows in order, each row's entries in stored order, each B row in
//      stored order) and keyed by (row in block, column);
//   2. a stable LDS radix sort (rocPRIM) orders them by key, keeping the
//      generation order among equal keys;
//   3. every run of equal keys is summed by one thread, first to last, which
//      is the host's accumulation order, so C is bit-identical to the host
//      product.
// A symbolic pass counts the distinct columns of every row (C's row
// pointers); the numeric pass writes C in place.
//
// The same product forms the smoothed prolongator: P = P_hat - omega D_F^-1
// (A_F P_hat), where A_F P_hat sums, in column order, the filtered entries of
// a row by aggregate, which is what the host does.  The strength graph and the
// smoother diagonal are per-row formulas; R = P^T scatters the entries by
// column and then orders each row of R by column, which fixes the order the
// host's transpose gives.  Only the greedy aggregation (sequential by its
// definition) stays on the host.

#include <rocprim/block/block_radix_sort.hpp>
#include <rocprim/block/block_scan.hpp>
#include <rocprim/device/device_scan.hpp>

#include <condition_variable>
#include <deque>
#include <exception>
#include <functional>
#include <mutex>
#include <thread>

#include "device.hpp"
#include "galerkin.hpp"

namespace amg {
namespace {

constexpr int kGBS = 512;                      // threads per workgroup
constexpr int kGItems = 16;                    // products per thread
constexpr int kGCap = kGBS * kGItems;          // products per workgroup
constexpr int kGMaxEntries = 8192;             // A entries per workgroup
constexpr int kGEntriesPerThread = kGMaxEntries / kGBS;
constexpr int kGRowBits = 10;
constexpr int kGMaxRows = 1 << kGRowBits;      // rows per workgroup
constexpr int kGMaxColBits = 32 - kGRowBits;   // key = row << colbits | column

struct DMat {
  int32_t rows = 0, cols = 0;
  int64_t nnz = 0;
  int32_t* ptr = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
};

// Products of each row of A B: the lengths of the B rows A's row selects.
__global__ void __launch_bounds__(256) row_products_kernel(DMat A, const int32_t* Bp, int64_t* L) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < A.rows; i += gridDim.x * 256) {
    int64_t s = 0;
    for (int e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
      const int j = A.col[e];
      s += Bp[j + 1] - Bp[j];
    }
    L[i] = s;
  }
}

using PairSort = rocprim::block_radix_sort<uint32_t, kGBS, kGItems, double>;
using BlockScan = rocprim::block_scan<int32_t, kGBS>;

struct GShared {
  union {
    typename PairSort::storage_type sort;
    struct {
      uint32_t key[kGCap];
      double val[kGCap];
    } run;
  } u;
  typename BlockScan::storage_type scan;
  int32_t eoff[kGMaxEntries + 1];  // first product of each A entry of the block
  int32_t rstart[kGMaxRows + 1];   // first A entry of each row of the block
  int32_t rowcnt[kGMaxRows];       // distinct columns per row
  int32_t rowfirst[kGMaxRows];     // index of the row's first run in the block
};

// NUMERIC = 0: count the distinct columns of each row into cnt.
// NUMERIC = 1: write C's columns and values at the row pointers Cp.
template <int NUMERIC>
__global__ void __launch_bounds__(kGBS) spgemm_block_kernel(DMat A, DMat B, const int32_t* blk, int colbits,
                                                            int32_t* cnt, const int32_t* Cp, int32_t* Cc,
                                                            double* Cv) {
  __shared__ GShared sh;
  const int tid = threadIdx.x;
  const int r0 = blk[blockIdx.x], r1 = blk[blockIdx.x + 1];
  const int nr = r1 - r0;
  const int ea0 = A.ptr[r0];
  const int ne = A.ptr[r1] - ea0;
  for (int r = tid; r <= nr; r += kGBS) sh.rstart[r] = A.ptr[r0 + r] - ea0;
  for (int r = tid; r < nr; r += kGBS) sh.rowcnt[r] = 0;

  // product offsets of the block's A entries (exclusive scan of B row lengths)
  int lens[kGEntriesPerThread];
  int tsum = 0;
#pragma unroll
  for (int k = 0; k < kGEntriesPerThread; ++k) {
    const int e = tid * kGEntriesPerThread + k;
    int len = 0;
    if (e < ne) {
      const int j = A.col[ea0 + e];
      len = B.ptr[j + 1] - B.ptr[j];
    }
    lens[k] = len;
    tsum += len;
  }
  int run = 0;
  BlockScan().exclusive_scan(tsum, run, 0, sh.scan);
#pragma unroll
  for (int k = 0; k < kGEntriesPerThread; ++k) {
    const int e = tid * kGEntriesPerThread + k;
    if (e < ne) sh.eoff[e] = run;
    run += lens[k];
  }
  if (tid == kGBS - 1) sh.eoff[ne] = run;
  __syncthreads();
  const int total = sh.eoff[ne];

  // product p = tid * kGItems + k (blocked arrangement, generation order)
  uint32_t key[kGItems];
  double val[kGItems];
#pragma unroll
  for (int k = 0; k < kGItems; ++k) {
    const int p = tid * kGItems + k;
    key[k] = 0xFFFFFFFFu;
    val[k] = 0.0;
    if (p < total) {
      int lo = 0, hi = ne - 1;  // last entry whose first product is <= p
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sh.eoff[mid] <= p) lo = mid;
        else hi = mid - 1;
      }
      int rl = 0, rh = nr - 1;  // last row whose first entry is <= lo
      while (rl < rh) {
        const int mid = (rl + rh + 1) >> 1;
        if (sh.rstart[mid] <= lo) rl = mid;
        else rh = mid - 1;
      }
      const int j = A.col[ea0 + lo];
      const int eb = B.ptr[j] + (p - sh.eoff[lo]);
      key[k] = (static_cast<uint32_t>(rl) << colbits) | static_cast<uint32_t>(B.col[eb]);
      val[k] = A.val[ea0 + lo] * B.val[eb];
    }
  }
  __syncthreads();
  PairSort().sort(key, val, sh.u.sort, 0, colbits + kGRowBits);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kGItems; ++k) {
    sh.u.run.key[tid * kGItems + k] = key[k];
    sh.u.run.val[tid * kGItems + k] = val[k];
  }
  __syncthreads();

  // runs of equal keys: count per thread, then their block-wide index
  int starts = 0;
#pragma unroll
  for (int k = 0; k < kGItems; ++k) {
    const int q = tid * kGItems + k;
    if (q < total && (q == 0 || sh.u.run.key[q] != sh.u.run.key[q - 1])) ++starts;
  }
  int rix = 0;
  BlockScan().exclusive_scan(starts, rix, 0, sh.scan);
  const int rix0 = rix;
#pragma unroll
  for (int k = 0; k < kGItems; ++k) {
    const int q = tid * kGItems + k;
    if (q < total && (q == 0 || sh.u.run.key[q] != sh.u.run.key[q - 1])) {
      const int rl = static_cast<int>(sh.u.run.key[q] >> colbits);
      if (q == 0 || static_cast<int>(sh.u.run.key[q - 1] >> colbits) != rl) sh.rowfirst[rl] = rix;
      atomicAdd(&sh.rowcnt[rl], 1);
      ++rix;
    }
  }
  __syncthreads();
  if constexpr (!NUMERIC) {
    for (int r = tid; r < nr; r += kGBS) cnt[r0 + r] = sh.rowcnt[r];
  } else {
    const uint32_t colmask = (colbits >= 32) ? 0xFFFFFFFFu : ((1u << colbits) - 1u);
    rix = rix0;
#pragma unroll
    for (int k = 0; k < kGItems; ++k) {
      const int q = tid * kGItems + k;
      if (q < total && (q == 0 || sh.u.run.key[q] != sh.u.run.key[q - 1])) {
        const uint32_t kq = sh.u.run.key[q];
        const int rl = static_cast<int>(kq >> colbits);
        double s = 0.0 + sh.u.run.val[q];
        for (int q2 = q + 1; q2 < total && sh.u.run.key[q2] == kq; ++q2) s += sh.u.run.val[q2];
        const int64_t out = static_cast<int64_t>(Cp[r0 + rl]) + (rix - sh.rowfirst[rl]);
        Cc[out] = static_cast<int32_t>(kq & colmask);
        Cv[out] = s;
        ++rix;
      }
    }
  }
}

int bits_for(int64_t n) {
  int b = 1;
  while ((int64_t(1) << b) < n) ++b;
  return b;
}

DMat upload_mat(DevArena& ar, const Csr& M, hipStream_t s) {
  DMat d;
  d.rows = static_cast<int32_t>(M.rows);
  d.cols = static_cast<int32_t>(M.cols);
  d.nnz = M.nnz();
  std::vector<int32_t> p32(M.ptr.begin(), M.ptr.end());
  d.ptr = ar.upload(p32.data(), p32.size());
  d.col = ar.get<int32_t>(std::max<int64_t>(d.nnz, 1));
  d.val = ar.get<double>(std::max<int64_t>(d.nnz, 1));
  if (d.nnz) {
    staged_h2d(d.col, M.col.data(), sizeof(int32_t) * d.nnz, s);
    staged_h2d(d.val, M.val.data(), sizeof(double) * d.nnz, s);
  }
  return d;
}

// Row lengths of A on the host: ptr[i + 1] - ptr[i] + extra.
struct HostRows {
  const int64_t* ptr;
  int64_t extra;
};

// C = A B with A's row lengths on the host (for the block schedule); C's row
// pointers are returned on the host too.  False: a row does not fit a block.
bool spgemm_dev(DevArena& ar, DevArena& out, HostRows arows, const DMat& A, const DMat& B, DMat& C,
                std::vector<int64_t>& Cptr, hipStream_t s) {
  const int colbits = bits_for(B.cols);
  if (colbits > kGMaxColBits) return false;
  const int m = A.rows;
  C.rows = m;
  C.cols = B.cols;
  Cptr.assign(m + 1, 0);
  std::vector<int64_t> L(m);
  if (m > 0) {
    int64_t* Ld = ar.get<int64_t>(m);
    row_products_kernel<<<static_cast<int>(std::min<int64_t>((m + 255) / 256, 4096)), 256, 0, s>>>(A, B.ptr, Ld);
    AMG_LAUNCHED();
    AMG_HIP(hipMemcpyAsync(L.data(), Ld, sizeof(int64_t) * m, hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
  }
  // blocks of whole rows: at most kGCap products, kGMaxEntries entries, kGMaxRows rows
  std::vector<int32_t> blk{0};
  int64_t prods = 0, ents = 0;
  for (int i = 0; i < m; ++i) {
    const int64_t len = arows.ptr[i + 1] - arows.ptr[i] + arows.extra;
    if (L[i] > kGCap || len > kGMaxEntries) return false;
    if (prods + L[i] > kGCap || ents + len > kGMaxEntries || i - blk.back() >= kGMaxRows) {
      blk.push_back(i);
      prods = ents = 0;
    }
    prods += L[i];
    ents += len;
  }
  if (blk.back() != m) blk.push_back(m);
  const int nb = static_cast<int>(blk.size()) - 1;
  if (nb <= 0) {
    C.nnz = 0;
    C.ptr = out.get<int32_t>(m + 1);
    C.col = out.get<int32_t>(1);
    C.val = out.get<double>(1);
    std::vector<int32_t> z(m + 1, 0);
    AMG_HIP(hipMemcpyAsync(C.ptr, z.data(), sizeof(int32_t) * (m + 1), hipMemcpyHostToDevice, s));
    AMG_HIP(hipStreamSynchronize(s));
    return true;
  }
  int32_t* blk_d = ar.upload(blk.data(), blk.size());
  int32_t* cnt = ar.get<int32_t>(m);
  spgemm_block_kernel<0><<<nb, kGBS, 0, s>>>(A, B, blk_d, colbits, cnt, nullptr, nullptr, nullptr);
  AMG_LAUNCHED();
  std::vector<int32_t> ch(m);
  AMG_HIP(hipMemcpyAsync(ch.data(), cnt, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < m; ++i) Cptr[i + 1] = Cptr[i] + ch[i];
  if (Cptr[m] >= (int64_t(1) << 31)) return false;
  C.nnz = Cptr[m];
  std::vector<int32_t> p32(Cptr.begin(), Cptr.end());
  C.ptr = out.upload(p32.data(), p32.size());
  C.col = out.get<int32_t>(std::max<int64_t>(C.nnz, 1));
  C.val = out.get<double>(std::max<int64_t>(C.nnz, 1));
  spgemm_block_kernel<1><<<nb, kGBS, 0, s>>>(A, B, blk_d, colbits, nullptr, C.ptr, C.col, C.val);
  AMG_LAUNCHED();
  AMG_HIP(hipStreamSynchronize(s));  // p32 and blk are pageable temporaries
  return true;
}

// ------------------------------------------------------------------ strength, prolongator

// d_i = a_ii (0 when not stored)
__global__ void __launch_bounds__(256) diag_kernel(DMat A, double* d) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < A.rows; i += gridDim.x * 256) {
    double v = 0.0;
    for (int e = A.ptr[i]; e < A.ptr[i + 1]; ++e)
      if (A.col[e] == i) v = A.val[e];
    d[i] = v;
  }
}

// Strength test of every stored entry, made symmetric by union: entry (i, j)
// is strong when a_ij^2 > eps^2 |a_ii a_jj| or a_ji^2 > eps^2 |a_jj a_ii|
// (the reverse entry found by binary search in row j).  A missing reverse
// entry (structurally nonsymmetric A) or a row without a stored diagonal
// raises *unsupported: the union would then hold entries A does not store,
// and the filtered matrix's layout assumes the diagonal.
__global__ void __launch_bounds__(256) strength_kernel(DMat A, const double* d, double eps2, uint8_t* strong,
                                                       int32_t* cnt, int32_t* unsupported) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < A.rows; i += gridDim.x * 256) {
    int c = 0;
    bool diag = false;
    for (int e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
      const int j = A.col[e];
      if (j == i) {
        strong[e] = 0;
        diag = true;
        continue;
      }
      const double v = A.val[e];
      bool st = v * v > eps2 * fabs(d[i] * d[j]);
      int lo = A.ptr[j], hi = A.ptr[j + 1] - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (A.col[mid] < i) lo = mid + 1;
        else hi = mid;
      }
      if (lo <= hi && A.col[lo] == i) {
        const double w = A.val[lo];
        st = st || (w * w > eps2 * fabs(d[j] * d[i]));
      } else {
        *unsupported = 1;
      }
      strong[e] = st ? 1 : 0;
      c += st ? 1 : 0;
    }
    if (!diag) *unsupported = 1;
    cnt[i] = c;
  }
}

// Columns of the strong entries of each row, in column order.
__global__ void __launch_bounds__(256) strong_fill_kernel(DMat A, const uint8_t* strong, const int32_t* Sp,
                                                          int32_t* Si) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < A.rows; i += gridDim.x * 256) {
    int p = Sp[i];
    for (int e = A.ptr[i]; e < A.ptr[i + 1]; ++e)
      if (strong[e]) Si[p++] = A.col[e];
  }
}

// Filtered matrix A_F (strong entries kept, weak ones lumped into the
// diagonal, in column order; a non-isolated row whose lumped diagonal is not
// positive keeps a_ii), written with the diagonal in place: row i of A_F has
// the diagonal and the strong entries, starting at AFp[i] = Sp[i] + i.  Also
// dF and the Gershgorin ratio sum_j |a^F_ij| / |a^F_ii| (0 for isolated rows).
__global__ void __launch_bounds__(256) filtered_kernel(DMat A, const uint8_t* strong, const int32_t* Sp,
                                                       double* dF, double* ratio, uint8_t* iso, int32_t* AFc,
                                                       double* AFv) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < A.rows; i += gridDim.x * 256) {
    double aii = 0.0, lumped = 0.0;
    for (int e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
      if (A.col[e] == i) aii = A.val[e];
      else if (!strong[e]) lumped += A.val[e];
    }
    const bool isolated = Sp[i] == Sp[i + 1];
    double dd = aii + lumped;
    if (!isolated && dd <= 0.0) dd = aii;
    double row = 0.0;
    int p = Sp[i] + i;
    for (int e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
      const int j = A.col[e];
      if (j == i) {
        row += fabs(dd);
        AFc[p] = i;
        AFv[p] = dd;
        ++p;
      } else if (strong[e]) {
        row += fabs(A.val[e]);
        AFc[p] = j;
        AFv[p] = A.val[e];
        ++p;
      }
    }
    dF[i] = dd;
    ratio[i] = isolated ? 0.0 : row / fabs(dd);
    iso[i] = isolated ? 1 : 0;
  }
}

// Per-workgroup maximum of the ratio over non-isolated rows (-1: none).
__global__ void __launch_bounds__(256) ratio_max_kernel(int n, const double* ratio, const uint8_t* iso,
                                                        double* partial) {
  __shared__ double sh[256];
  double m = -1.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
    if (!iso[i]) m = fmax(m, ratio[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// P = P_hat - omega D_F^-1 (A_F P_hat), in place on the product's values.
__global__ void __launch_bounds__(256) prolongator_finish_kernel(DMat C, const int32_t* agg, const double* dF,
                                                                 double omega) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < C.rows; i += gridDim.x * 256) {
    const double inv_d = 1.0 / dF[i];
    for (int e = C.ptr[i]; e < C.ptr[i + 1]; ++e) {
      const double smoothed = omega * (inv_d * C.val[e]);
      C.val[e] = (C.col[e] == agg[i] ? 1.0 : 0.0) - smoothed;
    }
  }
}

// ------------------------------------------------------------------ transpose, smoother

// Entries per column of M (the row lengths of M^T).
__global__ void __launch_bounds__(256) col_count_kernel(DMat M, int32_t* cnt) {
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < M.nnz; e += static_cast<int64_t>(gridDim.x) * 256)
    atomicAdd(&cnt[M.col[e]], 1);
}

// Entry (i, j) of M goes to row j of T at the slot it takes from pos[j]; the
// slots of a row are filled in no fixed order (rank_rows_kernel fixes it).
__global__ void __launch_bounds__(256) transpose_scatter_kernel(DMat M, int32_t* pos, int32_t* Tc, double* Tv) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < M.rows; i += gridDim.x * 256)
    for (int e = M.ptr[i]; e < M.ptr[i + 1]; ++e) {
      const int p = atomicAdd(&pos[M.col[e]], 1);
      Tc[p] = i;
      Tv[p] = M.val[e];
    }
}

// Row j of T in ascending column order from its slots in (Uc, Uv), filled in
// no fixed order: each entry goes to its rank among the row's columns (the
// columns of a row are distinct), one thread per entry.
__global__ void __launch_bounds__(256) rank_rows_kernel(int rows, int64_t nnz, const int32_t* Tp, const int32_t* Uc,
                                                        const double* Uv, int32_t* Tc, double* Tv) {
  for (int64_t q = blockIdx.x * 256 + threadIdx.x; q < nnz; q += static_cast<int64_t>(gridDim.x) * 256) {
    int lo = 0, hi = rows - 1;  // the row holding slot q: last j with Tp[j] <= q
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (Tp[mid] <= q) lo = mid;
      else hi = mid - 1;
    }
    const int b = Tp[lo], e = Tp[lo + 1];
    const int c = Uc[q];
    int rank = 0;
    for (int k = b; k < e; ++k) rank += Uc[k] < c ? 1 : 0;
    Tc[b + rank] = c;
    Tv[b + rank] = Uv[q];
  }
}

// Row pointers of the filtered matrix: row i holds the diagonal and the
// strong entries, AFp[i] = Sp[i] + i.
__global__ void __launch_bounds__(256) af_ptr_kernel(int n, const int32_t* Sp, int32_t* AFp) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i <= n; i += gridDim.x * 256) AFp[i] = Sp[i] + i;
}

// flag[i] = 1 when node i belongs to an aggregate (its row of P_hat holds one entry).
__global__ void __launch_bounds__(256) aggregated_kernel(int n, const int32_t* agg, int32_t* flag) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) flag[i] = agg[i] >= 0 ? 1 : 0;
}

// Tentative prolongator P_hat: entry 1 at (i, agg_i) for every aggregated node.
__global__ void __launch_bounds__(256) tentative_kernel(int n, const int32_t* agg, const int32_t* php, int32_t* phc,
                                                        double* phv) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
    if (agg[i] >= 0) {
      phc[php[i]] = agg[i];
      phv[php[i]] = 1.0;
    }
}

// Smoother diagonal, the host's formula and summation order: SPAI-0
// m_i = a_ii / sum_j a_ij^2 (relax 0), damped Jacobi omega / a_ii (relax 1),
// 1 / a_ii for the Chebyshev scaling (relax 2).
__global__ void __launch_bounds__(256) smoother_kernel(DMat A, int relax, double omega, double* m) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < A.rows; i += gridDim.x * 256) {
    double aii = 0.0, sq = 0.0;
    for (int e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
      const double v = A.val[e];
      sq += v * v;
      if (A.col[e] == i) aii = v;
    }
    m[i] = (relax == 0) ? aii / sq : (relax == 1) ? omega / aii : 1.0 / aii;
  }
}

int grid_for(int64_t n) { return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096))); }

// Waits for the copy: h may be a local of a step that a later allocation
// failure unwinds, and a copy still pending would then write freed memory.
template <class V>
void download(V& h, const typename V::value_type* d, size_t n, hipStream_t s) {
  h.resize(n);
  if (n) staged_d2h(h.data(), d, sizeof(typename V::value_type) * n, s);
}

class DeviceSetupAccel final : public SetupAccel {
 public:
  DeviceSetupAccel(const amg_allocator* alloc, hipStream_t s, const DeviceCsrRef* fine, bool keep)
      : stream_(s), keep_(keep) {
    if (alloc) {
      alloc_ = *alloc;
      has_alloc_ = true;
    }
    if (fine) {
      fine_ = *fine;
      has_fine_ = true;
    }
  }

  ~DeviceSetupAccel() override {
    try {
      finish_host_copies();
    } catch (...) {
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : copiers_)
      if (t.joinable()) t.join();
  }

  void begin_level(const Csr& A, bool from_galerkin) override {
    s_ok_ = p_ok_ = r_ok_ = have_A_ = false;
    cur_ = level_++;
    if (lv_.size() < static_cast<size_t>(cur_ + 1)) lv_.resize(cur_ + 1);
    if (!keep_ && cur_ > 0) lv_[cur_ - 1] = Level{};  // only this level's A is still needed
    work_ = arena();
    Level& L = lv_[cur_];
    try {
      if (from_galerkin && L.A.val) {
        // the previous level's product, already in L's storage
      } else if (cur_ == 0 && has_fine_ && fine_.rows == A.rows && fine_.nnz == A.nnz()) {
        // the caller's device copy of level 1 (read only by the steps)
        L.A.rows = fine_.rows;
        L.A.cols = fine_.cols;
        L.A.nnz = fine_.nnz;
        L.A.ptr = const_cast<int32_t*>(fine_.ptr);
        L.A.col = const_cast<int32_t*>(fine_.col);
        L.A.val = const_cast<double*>(fine_.val);
      } else {
        finish_host_copies();  // A's values come from the host
        L = Level{};
        L.ar = arena();
        L.A = upload_mat(*L.ar, A, stream_);
      }
      if (!L.ar) L.ar = arena();
      have_A_ = true;
    } catch (const DevError& e) {
      if (e.code != AMG_ERR_OOM) throw;
      L = Level{};
    }
  }

  bool strength(const Csr& A, double eps, Graph& S) override {
    if (!have_A_) return host_step();
    const DMat& dA = lv_[cur_].A;
    return guard([&] {
      const int n = dA.rows;
      d_ = work_->get<double>(n);
      strong_ = work_->get<uint8_t>(std::max<int64_t>(dA.nnz, 1));
      int32_t* cnt = work_->get<int32_t>(n);
      int32_t* unsupported = work_->get<int32_t>(1);
      AMG_HIP(hipMemsetAsync(unsupported, 0, sizeof(int32_t), stream_));
      diag_kernel<<<grid_for(n), 256, 0, stream_>>>(dA, d_);
      AMG_LAUNCHED();
      strength_kernel<<<grid_for(n), 256, 0, stream_>>>(dA, d_, eps * eps, strong_, cnt, unsupported);
      AMG_LAUNCHED();
      std::vector<int32_t> ch, ah;
      download(ch, cnt, n, stream_);
      download(ah, unsupported, 1, stream_);
      AMG_HIP(hipStreamSynchronize(stream_));
      if (ah[0]) return false;
      S.ptr.assign(n + 1, 0);
      for (int i = 0; i < n; ++i) S.ptr[i + 1] = S.ptr[i] + ch[i];
      std::vector<int32_t> p32(S.ptr.begin(), S.ptr.end());
      Sp_ = work_->upload(p32.data(), p32.size());
      int32_t* Si = work_->get<int32_t>(std::max<int64_t>(S.ptr[n], 1));
      strong_fill_kernel<<<grid_for(n), 256, 0, stream_>>>(dA, strong_, Sp_, Si);
      AMG_LAUNCHED();
      download(S.idx, Si, S.ptr[n], stream_);
      AMG_HIP(hipStreamSynchronize(stream_));  // p32 is a pageable temporary
      (void)A;
      s_ok_ = true;
      return true;
    });
  }

  bool prolongator(const Csr& A, const Graph& S, const std::vector<int32_t>& agg, int32_t nc, Csr& P,
                   double* omega) override {
    if (!s_ok_) return host_step();
    Level& L = lv_[cur_];
    const DMat& dA = L.A;
    return guard([&] {
      const int n = dA.rows;
      // A_F on the device (row i: the diagonal and the strong entries), dF,
      // ratio, isolated flags
      DMat AF;
      AF.rows = n;
      AF.cols = n;
      AF.nnz = S.ptr[n] + n;
      AF.ptr = work_->get<int32_t>(n + 1);
      AF.col = work_->get<int32_t>(std::max<int64_t>(AF.nnz, 1));
      AF.val = work_->get<double>(std::max<int64_t>(AF.nnz, 1));
      af_ptr_kernel<<<grid_for(n + 1), 256, 0, stream_>>>(n, Sp_, AF.ptr);
      AMG_LAUNCHED();
      dF_ = work_->get<double>(n);
      double* ratio = work_->get<double>(n);
      uint8_t* iso = work_->get<uint8_t>(n);
      filtered_kernel<<<grid_for(n), 256, 0, stream_>>>(dA, strong_, Sp_, dF_, ratio, iso, AF.col, AF.val);
      AMG_LAUNCHED();
      const int nbm = grid_for(n);
      double* part = work_->get<double>(nbm);
      ratio_max_kernel<<<nbm, 256, 0, stream_>>>(n, ratio, iso, part);
      AMG_LAUNCHED();
      // P_hat: one entry 1 per aggregated row (row pointers by a scan of the flags)
      int32_t* agg_d = work_->upload(agg.data(), agg.size());
      DMat Ph;
      Ph.rows = n;
      Ph.cols = nc;
      Ph.nnz = n;  // at most
      Ph.ptr = work_->get<int32_t>(n + 1);
      Ph.col = work_->get<int32_t>(std::max(n, 1));
      Ph.val = work_->get<double>(std::max(n, 1));
      int32_t* flag = work_->get<int32_t>(std::max(n, 1));
      aggregated_kernel<<<grid_for(n), 256, 0, stream_>>>(n, agg_d, flag);
      AMG_LAUNCHED();
      AMG_HIP(hipMemsetAsync(Ph.ptr, 0, sizeof(int32_t), stream_));
      size_t scan_bytes = 0;
      AMG_HIP(rocprim::inclusive_scan(nullptr, scan_bytes, flag, Ph.ptr + 1, static_cast<size_t>(n),
                                      rocprim::plus<int32_t>(), stream_));
      void* scan_tmp = work_->raw(scan_bytes);
      AMG_HIP(rocprim::inclusive_scan(scan_tmp, scan_bytes, flag, Ph.ptr + 1, static_cast<size_t>(n),
                                      rocprim::plus<int32_t>(), stream_));
      tentative_kernel<<<grid_for(n), 256, 0, stream_>>>(n, agg_d, Ph.ptr, Ph.col, Ph.val);
      AMG_LAUNCHED();
      std::vector<double> ph;
      download(ph, part, nbm, stream_);
      double rho = -1.0;
      for (double v : ph) rho = std::max(rho, v);
      if (rho < 0.0) rho = 1.0;  // no non-isolated row
      const double om = (4.0 / 3.0) / rho;
      std::vector<int64_t> Pptr;
      DMat dP;
      if (!spgemm_dev(*work_, *L.ar, HostRows{S.ptr.data(), 1}, AF, Ph, dP, Pptr, stream_)) return false;
      prolongator_finish_kernel<<<grid_for(n), 256, 0, stream_>>>(dP, agg_d, dF_, om);
      AMG_LAUNCHED();
      P = Csr{};
      P.rows = n;
      P.cols = nc;
      P.ptr = std::move(Pptr);
      to_host(P.col, dP.col, dP.nnz);
      to_host(P.val, dP.val, dP.nnz);
      (void)A;
      *omega = om;
      L.P = dP;
      p_ok_ = true;
      return true;
    });
  }

  bool transpose(const Csr& P, Csr& R) override {
    // Only worth it when the levels stay on the device: R is then made there
    // anyway and the solve uses that copy.
    if (!p_ok_ || !keep_) return host_step();
    Level& L = lv_[cur_];
    return guard([&] {
      const DMat& dP = L.P;
      const int nc = dP.cols;
      int32_t* cnt = work_->get<int32_t>(std::max(nc, 1));
      AMG_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * std::max(nc, 1), stream_));
      if (dP.nnz) {
        col_count_kernel<<<grid_for(dP.nnz), 256, 0, stream_>>>(dP, cnt);
        AMG_LAUNCHED();
      }
      std::vector<int32_t> ch;
      download(ch, cnt, nc, stream_);
      R = Csr{};
      R.rows = nc;
      R.cols = dP.rows;
      R.ptr.assign(nc + 1, 0);
      for (int j = 0; j < nc; ++j) R.ptr[j + 1] = R.ptr[j] + ch[j];
      std::vector<int32_t> p32(R.ptr.begin(), R.ptr.end());
      DMat dR;
      dR.rows = nc;
      dR.cols = dP.rows;
      dR.nnz = dP.nnz;
      dR.ptr = L.ar->upload(p32.data(), p32.size());
      dR.col = L.ar->get<int32_t>(std::max<int64_t>(dR.nnz, 1));
      dR.val = L.ar->get<double>(std::max<int64_t>(dR.nnz, 1));
      if (dP.nnz) {
        int32_t* pos = work_->get<int32_t>(std::max(nc, 1));
        int32_t* Uc = work_->get<int32_t>(dP.nnz);
        double* Uv = work_->get<double>(dP.nnz);
        AMG_HIP(hipMemcpyAsync(pos, dR.ptr, sizeof(int32_t) * nc, hipMemcpyDeviceToDevice, stream_));
        transpose_scatter_kernel<<<grid_for(dP.rows), 256, 0, stream_>>>(dP, pos, Uc, Uv);
        AMG_LAUNCHED();
        rank_rows_kernel<<<grid_for(dP.nnz), 256, 0, stream_>>>(nc, dP.nnz, dR.ptr, Uc, Uv, dR.col, dR.val);
        AMG_LAUNCHED();
      }
      to_host(R.col, dR.col, dR.nnz);
      to_host(R.val, dR.val, dR.nnz);
      (void)P;
      L.R = dR;
      r_ok_ = true;
      return true;
    });
  }

  bool smoother(const Csr& A, const SetupParams& prm, std::vector<double>& m) override {
    if (!have_A_ || !keep_ || prm.relax < 0 || prm.relax > 2) return host_step();
    Level& L = lv_[cur_];
    return guard([&] {
      const int n = L.A.rows;
      double* dm = L.ar->get<double>(std::max(n, 1));
      smoother_kernel<<<grid_for(n), 256, 0, stream_>>>(L.A, prm.relax, prm.jacobi_omega, dm);
      AMG_LAUNCHED();
      to_host(m, static_cast<const double*>(dm), n);
      (void)A;
      L.m = dm;
      return true;
    });
  }

  bool galerkin(const Csr& R, const Csr& A, const Csr& P, Csr& Ac) override {
    if (!have_A_) return host_step();
    return guard([&] {
      {
        Level& L = lv_[cur_];
        if (!p_ok_ || !r_ok_) finish_host_copies();  // P or R come from the host
        if (!p_ok_) L.P = upload_mat(*L.ar, P, stream_);
        if (!r_ok_) L.R = upload_mat(*L.ar, R, stream_);
      }
      DMat AP;
      std::vector<int64_t> APptr, Cptr;
      if (!spgemm_dev(*work_, *work_, HostRows{A.ptr.data(), 0}, lv_[cur_].A, lv_[cur_].P, AP, APptr, stream_))
        return false;
      if (lv_.size() < static_cast<size_t>(cur_ + 2)) lv_.resize(cur_ + 2);
      Level& N = lv_[cur_ + 1];
      N = Level{};
      N.ar = arena();
      DMat dAc;
      if (!spgemm_dev(*work_, *N.ar, HostRows{R.ptr.data(), 0}, lv_[cur_].R, AP, dAc, Cptr, stream_)) {
        N = Level{};
        return false;
      }
      N.A = dAc;
      Ac = Csr{};
      Ac.rows = dAc.rows;
      Ac.cols = dAc.cols;
      Ac.ptr = std::move(Cptr);
      to_host(Ac.col, dAc.col, dAc.nnz);
      to_host(Ac.val, dAc.val, dAc.nnz);
      return true;
    });
  }

  void host_work_begins() override {
    if (on_host_work) {
      std::function<void()> f = std::move(on_host_work);
      on_host_work = nullptr;
      f();
    }
  }

  std::function<void()> on_host_work;

  // Waits for the copies to_host started; rethrows the first error of one.
  void finish_host_copies() override {
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.wait(lk, [&] { return q_.empty() && busy_ == 0; });
    if (err_) {
      std::exception_ptr e = err_;
      err_ = nullptr;
      std::rethrow_exception(e);
    }
  }

  bool level_refs(int l, DeviceLevelRefs* out) const {
    if (!keep_ || l < 0 || static_cast<size_t>(l) >= lv_.size()) return false;
    const Level& L = lv_[l];
    *out = DeviceLevelRefs{};
    out->A = ref(L.A);
    out->P = ref(L.P);
    out->R = ref(L.R);
    out->m = L.m;
    return true;
  }

 private:
  // Device copies of one level (FP64): A (the caller's for level 1), P, R =
  // P^T and the smoother diagonal, in the level's own arena.
  struct Level {
    std::unique_ptr<DevArena> ar;
    DMat A, P, R;
    double* m = nullptr;
  };

  static DeviceCsrRef ref(const DMat& M) {
    DeviceCsrRef r;
    if (!M.val) return r;
    r.rows = M.rows;
    r.cols = M.cols;
    r.nnz = M.nnz;
    r.ptr = M.ptr;
    r.col = M.col;
    r.val = M.val;
    return r;
  }

  std::unique_ptr<DevArena> arena() { return std::make_unique<DevArena>(has_alloc_ ? &alloc_ : nullptr, stream_); }

  // Host copy of n device elements into h.  With kept levels the copy runs on
  // one of a few threads, each with a stream of its own, after the work
  // enqueued so far on the setup stream, and overlaps the following steps
  // (the device memory lives until the accelerator goes; the threads also
  // spread the page faults of the new host arrays); otherwise it completes
  // before returning.
  template <class V>
  void to_host(V& h, const typename V::value_type* d, int64_t n) {
    if (!keep_) {
      download(h, d, static_cast<size_t>(n), stream_);
      return;
    }
    hipEvent_t ev = nullptr;
    AMG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    const hipError_t e = hipEventRecord(ev, stream_);
    if (e != hipSuccess) {
      (void)hipEventDestroy(ev);
      AMG_HIP(e);
    }
    V* dst = &h;
    enqueue([dst, d, n, ev](hipStream_t cs) {
      struct Ev {
        hipEvent_t e;
        ~Ev() { (void)hipEventDestroy(e); }
      } guard_ev{ev};
      AMG_HIP(hipStreamWaitEvent(cs, ev, 0));
      download(*dst, d, static_cast<size_t>(n), cs);
    });
  }

  static constexpr int kCopyThreads = 3;

  void enqueue(std::function<void(hipStream_t)> job) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      q_.push_back(std::move(job));
      if (copiers_.empty())
        for (int t = 0; t < kCopyThreads; ++t) copiers_.emplace_back([this] { copy_loop(); });
    }
    cv_.notify_one();
  }

  void copy_loop() {
    hipStream_t cs = nullptr;
    std::exception_ptr init_err;
    try {
      AMG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    } catch (...) {
      init_err = std::current_exception();
    }
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_.wait(lk, [&] { return stop_ || !q_.empty(); });
      if (q_.empty()) break;  // stopping
      std::function<void(hipStream_t)> job = std::move(q_.front());
      q_.pop_front();
      ++busy_;
      lk.unlock();
      std::exception_ptr e = init_err;
      if (!e) {
        try {
          job(cs);
        } catch (...) {
          e = std::current_exception();
        }
      }
      lk.lock();
      --busy_;
      if (e && !err_) err_ = e;
      if (q_.empty() && busy_ == 0) cv_done_.notify_all();
    }
    lk.unlock();
    if (cs) (void)hipStreamDestroy(cs);
  }

  // A step left to the host reads the host copies of its inputs.
  bool host_step() {
    finish_host_copies();
    return false;
  }

  // Runs a step; a false result (a row that does not fit the device kernels,
  // an allocation failure) leaves the step to the host.
  template <class F>
  bool guard(F fn) {
    bool ok = false;
    try {
      ok = fn();
    } catch (const DevError& e) {
      if (e.code != AMG_ERR_OOM) throw;
      ok = false;
    }
    return ok ? true : host_step();
  }

  hipStream_t stream_;
  bool keep_;
  amg_allocator alloc_{};
  bool has_alloc_ = false;
  std::vector<Level> lv_;
  std::unique_ptr<DevArena> work_;  // scratch of the current level
  int cur_ = -1;
  double* d_ = nullptr;
  double* dF_ = nullptr;
  uint8_t* strong_ = nullptr;
  int32_t* Sp_ = nullptr;
  bool have_A_ = false, s_ok_ = false, p_ok_ = false, r_ok_ = false;
  DeviceCsrRef fine_;
  bool has_fine_ = false;
  int level_ = 0;
  // host copies in flight (kept levels only)
  std::vector<std::thread> copiers_;
  std::mutex mu_;
  std::condition_variable cv_, cv_done_;
  std::deque<std::function<void(hipStream_t)>> q_;
  int busy_ = 0;
  bool stop_ = false;
  std::exception_ptr err_;
};

}  // namespace

std::unique_ptr<SetupAccel> make_device_setup_accel(const amg_allocator* alloc, hipStream_t stream,
                                                    const DeviceCsrRef* fine, bool keep_levels,
                                                    std::function<void()> on_host_work) {
  auto a = std::make_unique<DeviceSetupAccel>(alloc, stream, fine, keep_levels);
  a->on_host_work = std::move(on_host_work);
  return a;
}

void preload_setup_kernels() {
  hipFuncAttributes a;
  (void)hipFuncGetAttributes(&a, reinterpret_cast<const void*>(&diag_kernel));
  (void)hipGetLastError();
}

bool device_level_refs(const SetupAccel* accel, int level, DeviceLevelRefs* out) {
  const auto* d = dynamic_cast<const DeviceSetupAccel*>(accel);
  return d && d->level_refs(level, out);
}

}  // namespace amg
