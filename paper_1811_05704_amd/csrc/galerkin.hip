// Galerkin products on the device (section 2, "AMG setup": A_{l+1} = R_l A_l P_l).
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

#include <rocprim/block/block_radix_sort.hpp>
#include <rocprim/block/block_scan.hpp>

#include <climits>

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
    AMG_HIP(hipMemcpyAsync(d.col, M.col.data(), sizeof(int32_t) * d.nnz, hipMemcpyHostToDevice, s));
    AMG_HIP(hipMemcpyAsync(d.val, M.val.data(), sizeof(double) * d.nnz, hipMemcpyHostToDevice, s));
  }
  AMG_HIP(hipStreamSynchronize(s));  // p32 is a pageable temporary
  return d;
}

// C = A B with A's host row pointers (Ahost) for the block schedule; C's row
// pointers are returned on the host too.  False: a row does not fit a block.
bool spgemm_dev(DevArena& ar, const std::vector<int64_t>& Aptr_host, const DMat& A, const DMat& B, DMat& C,
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
    const int64_t len = Aptr_host[i + 1] - Aptr_host[i];
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
    C.ptr = ar.get<int32_t>(m + 1);
    C.col = ar.get<int32_t>(1);
    C.val = ar.get<double>(1);
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
  C.ptr = ar.upload(p32.data(), p32.size());
  C.col = ar.get<int32_t>(std::max<int64_t>(C.nnz, 1));
  C.val = ar.get<double>(std::max<int64_t>(C.nnz, 1));
  spgemm_block_kernel<1><<<nb, kGBS, 0, s>>>(A, B, blk_d, colbits, nullptr, C.ptr, C.col, C.val);
  AMG_LAUNCHED();
  AMG_HIP(hipStreamSynchronize(s));  // p32 and blk are pageable temporaries
  return true;
}

}  // namespace

bool device_galerkin(const Csr& R, const Csr& A, const Csr& P, Csr& Ac, const amg_allocator* alloc,
                     hipStream_t stream) {
  DevArena ar(alloc, stream);
  const DMat dA = upload_mat(ar, A, stream);
  const DMat dP = upload_mat(ar, P, stream);
  const DMat dR = upload_mat(ar, R, stream);
  DMat AP, C;
  std::vector<int64_t> APptr, Cptr;
  if (!spgemm_dev(ar, A.ptr, dA, dP, AP, APptr, stream)) return false;
  if (!spgemm_dev(ar, R.ptr, dR, AP, C, Cptr, stream)) return false;
  Csr out;
  out.rows = C.rows;
  out.cols = C.cols;
  out.ptr = std::move(Cptr);
  out.col.resize(C.nnz);
  out.val.resize(C.nnz);
  if (C.nnz) {
    AMG_HIP(hipMemcpyAsync(out.col.data(), C.col, sizeof(int32_t) * C.nnz, hipMemcpyDeviceToHost, stream));
    AMG_HIP(hipMemcpyAsync(out.val.data(), C.val, sizeof(double) * C.nnz, hipMemcpyDeviceToHost, stream));
  }
  AMG_HIP(hipStreamSynchronize(stream));
  Ac = std::move(out);
  return true;
}

}  // namespace amg
