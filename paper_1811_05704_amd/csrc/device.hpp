// Device-side data of the solver: level matrices and vectors in HBM, the
// per-matrix SpMV schedule (variant chosen by row length), and launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/amg.h"
#include "host_setup.hpp"
#include "kernels.hpp"

namespace amg {

struct DevError {
  int code;
  std::string msg;
};

#define AMG_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::amg::DevError{-6, std::string(#call) + ": " + hipGetErrorString(e_)};     \
  } while (0)

#define AMG_LAUNCHED()                                                                  \
  do {                                                                                  \
    hipError_t e_ = hipGetLastError();                                                  \
    if (e_ != hipSuccess)                                                               \
      throw ::amg::DevError{-6, std::string("kernel launch: ") + hipGetErrorString(e_)}; \
  } while (0)

// Copies between pageable host memory and the device that return when done;
// large ones are staged through pinned buffers (staging.hip).
void staged_h2d(void* dst, const void* src, size_t bytes, hipStream_t s);
void staged_d2h(void* dst, const void* src, size_t bytes, hipStream_t s);

// Device memory from the caller's allocator (or hipMalloc), freed together.
class DevArena {
 public:
  DevArena(const amg_allocator* a, hipStream_t s) : stream_(s) {
    if (a && a->alloc && a->free) {
      alloc_ = *a;
      custom_ = true;
    }
  }
  ~DevArena() { release(); }
  DevArena(const DevArena&) = delete;
  DevArena& operator=(const DevArena&) = delete;

  void* raw(size_t bytes) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~size_t(255);
    void* p = nullptr;
    if (custom_) {
      p = alloc_.alloc(bytes, stream_, alloc_.ctx);
      if (!p) throw DevError{-5, "device allocator returned NULL for " + std::to_string(bytes) + " bytes"};
    } else {
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        throw DevError{-5, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
      }
    }
    blocks_.push_back(p);
    bytes_ += bytes;
    return p;
  }
  template <class T>
  T* get(size_t count) {
    return static_cast<T*>(raw(count * sizeof(T)));
  }
  // Copies count elements from host memory and waits for the copy: the source
  // is usually a pageable temporary of the caller, which an exception from a
  // later allocation (out of memory) would free while the copy still reads it.
  template <class T>
  T* upload(const T* host, size_t count) {
    T* d = get<T>(count);
    if (count) staged_h2d(d, host, count * sizeof(T), stream_);
    return d;
  }
  size_t bytes() const { return bytes_; }
  hipStream_t stream() const { return stream_; }
  // Stream matrices uploaded here also get 2-byte column offsets (attach_compact_cols).
  bool compact_cols = false;
  // Stream that release() synchronises before freeing (the owner's compute stream).
  void set_stream(hipStream_t s) { stream_ = s; }
  void release() {
    if (!blocks_.empty()) (void)hipStreamSynchronize(stream_);
    for (void* p : blocks_) {
      if (custom_) alloc_.free(p, stream_, alloc_.ctx);
      else (void)hipFree(p);
    }
    blocks_.clear();
    bytes_ = 0;
  }

 private:
  amg_allocator alloc_{};
  bool custom_ = false;
  hipStream_t stream_;
  std::vector<void*> blocks_;
  size_t bytes_ = 0;
};

// SpMV schedule selection by row length: the LDS-staged stream kernel with
// G = 1, 4, 16 or 64 lanes reducing each row, or (very long rows) G = 64 lanes
// per row reading straight from memory.
constexpr double kVectorMinMean = 512.0;

template <class T>
struct DevCsr {
  int32_t rows = 0, cols = 0;
  int64_t nnz = 0;
  int32_t* ptr = nullptr;
  int32_t* col = nullptr;
  T* val = nullptr;
  int kind = 0;   // 0 stream, 1 vector
  int lanes = 1;  // lanes per row (stream: in the LDS reduction phase)
  int bclass = 0;  // stream block size class: 0 = 16 KB, 1 = 4 KB, 2 = 8 KB
  int32_t nblocks = 0;
  int32_t* blk = nullptr;
  uint16_t* col16 = nullptr;  // stream: 2-byte column offsets per block (NULL: col)
  int32_t* cbase = nullptr;
  CsrView<T> view() const { return CsrView<T>{ptr, col, val, blk, rows, nblocks, col16, cbase}; }
};

struct Schedule {
  int kind = 0, lanes = 1, bclass = 0;
  std::vector<int32_t> blk;
  int32_t nblocks = 0;
};

inline int stream_lanes(double mean) {
  if (mean <= 12.0) return 1;
  if (mean <= 48.0) return 4;
  if (mean <= 192.0) return 16;
  return 64;
}

template <class T>
Schedule make_schedule(const Csr& M, int force_kind = -1) {
  Schedule s;
  const int64_t rows = M.rows;
  const double mean = rows ? double(M.nnz()) / double(rows) : 0.0;
  s.kind = force_kind >= 0 ? force_kind : (mean <= kVectorMinMean ? 0 : 1);
  if (s.kind == 0) {
    s.lanes = stream_lanes(mean);
    // Block size: 4 KB for small matrices; otherwise the smallest of 4, 8 and
    // 16 KB that holds the rows of the reduction phase (kBS / G rows of mean
    // length per pass; one pass, two for G = 16), so few of the unrolled
    // loads re-read the last entry (8 KB exists for G = 1, 4 and 16; FP64
    // one-lane rows keep 8 KB, measured best).  With one pass of 16 rows the
    // 60-entry rows of a pressure Schur complement filled half of a 16 KB
    // FP64 block; two passes of 16 fill it and were 2-6 % faster than one
    // pass in 8 KB blocks.
    const int npass = s.lanes == 16 ? 2 : 1;
    const double pass = double(npass * kBS / s.lanes) * mean;
    if (M.nnz() * static_cast<int64_t>(sizeof(T)) < kStreamSmallMatrix) s.bclass = 1;
    else if (s.lanes == 1 && sizeof(T) == 8) s.bclass = 2;
    else if (pass <= stream_nnz<T, kStreamSmallBytes>()) s.bclass = 1;
    else if (s.lanes <= 16 && pass <= stream_nnz<T, kStreamMidBytes>()) s.bclass = 2;
    const int64_t cap = s.bclass == 1   ? stream_nnz<T, kStreamSmallBytes>()
                        : s.bclass == 2 ? stream_nnz<T, kStreamMidBytes>()
                                        : stream_nnz<T>();
    // rows per block: at most npass reduction passes of the workgroup
    const int64_t max_rows = std::min<int64_t>(kStreamMaxRows, npass * kBS / s.lanes);
    s.blk.push_back(0);
    int64_t r = 0;
    while (r < rows) {
      const int64_t start = r;
      if (M.ptr[r + 1] - M.ptr[r] > cap) {
        ++r;
      } else {
        int64_t nnz = 0;
        while (r < rows && r - start < max_rows) {
          const int64_t len = M.ptr[r + 1] - M.ptr[r];
          if (nnz + len > cap) break;
          nnz += len;
          ++r;
        }
      }
      s.blk.push_back(static_cast<int32_t>(r));
    }
    s.nblocks = static_cast<int32_t>(s.blk.size()) - 1;
  } else {
    s.lanes = 64;
    const int rpb = kBS / s.lanes;
    s.nblocks = static_cast<int32_t>((rows + rpb - 1) / rpb);
  }
  return s;
}

// Entries per stream block of the matrix's block size class.
template <class T>
int stream_block_entries(int bclass) {
  return bclass == 1 ? stream_nnz<T, kStreamSmallBytes>() : bclass == 2 ? stream_nnz<T, kStreamMidBytes>()
                                                                         : stream_nnz<T>();
}

// With ar.compact_cols, gives a stream matrix 2-byte column offsets from each
// block's smallest column (2 bytes per entry and 4 per block read instead
// of 4 per entry) when every block of at most one LDS pass spans at most
// 65536 columns; otherwise the matrix keeps reading its int32 columns.  The
// same columns either way, so results do not change.  Waits for the check.
template <class T>
void attach_compact_cols(DevArena& ar, DevCsr<T>& d) {
  if (!ar.compact_cols || d.kind != 0 || d.nnz == 0 || d.nblocks == 0) return;
  const hipStream_t s = ar.stream();
  int32_t* cbase = ar.get<int32_t>(d.nblocks);
  uint16_t* c16 = ar.get<uint16_t>(d.nnz);
  int32_t* bad = ar.get<int32_t>(1);
  fill_kernel<int32_t><<<1, kVecBS, 0, s>>>(1, bad, 0);
  AMG_LAUNCHED();
  compact_cols_kernel<<<d.nblocks, kBS, 0, s>>>(d.ptr, d.col, d.blk, stream_block_entries<T>(d.bclass), cbase, c16,
                                                bad);
  AMG_LAUNCHED();
  int32_t h = 1;
  AMG_HIP(hipMemcpyAsync(&h, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  if (h == 0) {
    d.col16 = c16;
    d.cbase = cbase;
  }
}

template <class T>
DevCsr<T> upload_csr(DevArena& ar, const Csr& M, int force_kind = -1) {
  DevCsr<T> d;
  d.rows = static_cast<int32_t>(M.rows);
  d.cols = static_cast<int32_t>(M.cols);
  d.nnz = M.nnz();
  std::vector<int32_t> p32(M.ptr.begin(), M.ptr.end());
  if (p32.empty()) p32.assign(1, 0);
  d.ptr = ar.upload(p32.data(), p32.size());
  const size_t nz = M.col.size();
  d.col = ar.upload(M.col.data(), nz);  // an empty matrix still gets (unread) storage
  if constexpr (std::is_same<T, double>::value) {
    d.val = ar.upload(M.val.data(), nz);
  } else {
    std::vector<T> v(nz);
    for (size_t k = 0; k < nz; ++k) v[k] = static_cast<T>(M.val[k]);  // FP32: round to nearest
    d.val = ar.upload(v.data(), nz);
  }
  Schedule s = make_schedule<T>(M, force_kind);
  d.kind = s.kind;
  d.lanes = s.lanes;
  d.bclass = s.bclass;
  d.nblocks = s.nblocks;
  if (s.kind == 0) d.blk = ar.upload(s.blk.data(), s.blk.size());
  // upload uses pageable host buffers: finish before they go out of scope
  AMG_HIP(hipStreamSynchronize(ar.stream()));
  attach_compact_cols(ar, d);
  return d;
}

// Launch y-epilogue SpMV with the matrix's schedule; returns the grid size
// (= number of partials written when E::K > 0).
template <class T, class G, class E>
int launch_spmv(const DevCsr<T>& M, G g, E e, double* partials, const int* skip, hipStream_t s) {
  if (M.rows == 0) return 0;
  if (M.kind == 0) {
    constexpr int NS = kStreamSmallBytes, NM = kStreamMidBytes, NL = AMG_STREAM_BYTES;
    const CsrView<T> A = M.view();
    const int n = M.nblocks;
    auto go = [&](auto c16) {
      constexpr int C = decltype(c16)::value;
      switch (M.lanes * 4 + M.bclass) {
        case 4: csr_stream_kernel<1, NL, T, G, E, C><<<n, kBS, 0, s>>>(A, g, e, partials, skip); break;
        case 5: csr_stream_kernel<1, NS, T, G, E, C><<<n, kBS, 0, s>>>(A, g, e, partials, skip); break;
        case 6: csr_stream_kernel<1, NM, T, G, E, C><<<n, kBS, 0, s>>>(A, g, e, partials, skip); break;
        case 16: csr_stream_kernel<4, NL, T, G, E, C><<<n, kBS, 0, s>>>(A, g, e, partials, skip); break;
        case 17: csr_stream_kernel<4, NS, T, G, E, C><<<n, kBS, 0, s>>>(A, g, e, partials, skip); break;
        case 18: csr_stream_kernel<4, NM, T, G, E, C><<<n, kBS, 0, s>>>(A, g, e, partials, skip); break;
        case 64: csr_stream_kernel<16, NL, T, G, E, C><<<n, kBS, 0, s>>>(A, g, e, partials, skip); break;
        case 65: csr_stream_kernel<16, NS, T, G, E, C><<<n, kBS, 0, s>>>(A, g, e, partials, skip); break;
        case 66: csr_stream_kernel<16, NM, T, G, E, C><<<n, kBS, 0, s>>>(A, g, e, partials, skip); break;
        case 256: csr_stream_kernel<64, NL, T, G, E, C><<<n, kBS, 0, s>>>(A, g, e, partials, skip); break;
        default: csr_stream_kernel<64, NS, T, G, E, C><<<n, kBS, 0, s>>>(A, g, e, partials, skip); break;
      }
    };
    if (M.col16) go(std::integral_constant<int, 1>{});
    else go(std::integral_constant<int, 0>{});
  } else {
    csr_vector_kernel<64, T, G, E><<<M.nblocks, kBS, 0, s>>>(M.view(), g, e, partials, skip);
  }
  AMG_LAUNCHED();
  return M.nblocks;
}

inline int vec_blocks(int64_t n) {
  int64_t b = (n + kVecBS - 1) / kVecBS;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(b, 65536)));
}

}  // namespace amg
