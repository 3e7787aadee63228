// Large copies between pageable host memory and the device, staged through
// pinned buffers.
//
// hipMemcpyAsync from pageable memory moves 13-28 GB/s host to device and
// 17 GB/s device to host on MI355X; a DMA from pinned memory runs at the
// link's ~51 GB/s.  Each copy is split into 16 MB chunks: while one pinned
// buffer is in flight the next chunk is copied into the other by up to four
// host threads (the calling thread's setup thread limit; one memcpy thread
// caps the staged rate near 14 GB/s host to device, so a single-threaded
// caller copies host to device directly, and 27 GB/s device to host, still
// above the direct 17 GB/s).
// The staging pairs are kept in a process-wide pool and reused; a thread
// that finds none free allocates another (one per concurrent caller, each
// 32 MB of pinned memory, held until the process ends).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "device.hpp"

namespace amg {

namespace {

constexpr size_t kStageChunk = size_t(16) << 20;
constexpr size_t kStageMin = size_t(4) << 20;  // smaller copies go straight through hipMemcpyAsync
constexpr int kStageThreads = 4;

struct StagePair {
  void* buf[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
};

std::mutex g_stage_mu;
std::vector<StagePair*> g_stage_free;

StagePair* take_pair() {
  {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    if (!g_stage_free.empty()) {
      StagePair* p = g_stage_free.back();
      g_stage_free.pop_back();
      return p;
    }
  }
  auto* p = new StagePair;
  for (int k = 0; k < 2; ++k) {
    if (hipHostMalloc(&p->buf[k], kStageChunk, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev[k], hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      for (int j = 0; j < 2; ++j) {
        if (p->buf[j]) (void)hipHostFree(p->buf[j]);
        if (p->ev[j]) (void)hipEventDestroy(p->ev[j]);
      }
      delete p;
      return nullptr;
    }
  }
  return p;
}

void give_pair(StagePair* p) {
  std::lock_guard<std::mutex> lk(g_stage_mu);
  g_stage_free.push_back(p);
}

void host_copy(void* dst, const void* src, size_t bytes) {
  const int nt = std::max(1, std::min(kStageThreads, setup_threads()));
  const size_t per = (bytes + nt - 1) / nt;
  std::thread th[kStageThreads - 1];
  for (int t = 1; t < nt; ++t) {
    const size_t b = t * per, e = std::min(bytes, b + per);
    if (b < e)
      th[t - 1] = std::thread([=] { std::memcpy(static_cast<char*>(dst) + b, static_cast<const char*>(src) + b, e - b); });
  }
  std::memcpy(dst, src, std::min(bytes, per));
  for (auto& x : th)
    if (x.joinable()) x.join();
}

}  // namespace

void staged_h2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  StagePair* p = (bytes >= kStageMin && setup_threads() > 1) ? take_pair() : nullptr;
  if (!p) {
    AMG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    AMG_HIP(hipStreamSynchronize(s));
    return;
  }
  struct Back {
    StagePair* p;
    hipStream_t s;
    ~Back() {
      (void)hipStreamSynchronize(s);
      give_pair(p);
    }
  } back{p, s};
  bool pending[2] = {false, false};
  size_t c = 0;
  for (size_t off = 0; off < bytes; off += kStageChunk, ++c) {
    const int k = static_cast<int>(c & 1);
    const size_t len = std::min(kStageChunk, bytes - off);
    if (pending[k]) AMG_HIP(hipEventSynchronize(p->ev[k]));
    host_copy(p->buf[k], static_cast<const char*>(src) + off, len);
    AMG_HIP(hipMemcpyAsync(static_cast<char*>(dst) + off, p->buf[k], len, hipMemcpyHostToDevice, s));
    AMG_HIP(hipEventRecord(p->ev[k], s));
    pending[k] = true;
  }
  AMG_HIP(hipStreamSynchronize(s));
}

void staged_d2h(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  StagePair* p = bytes >= kStageMin ? take_pair() : nullptr;
  if (!p) {
    AMG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    return;
  }
  struct Back {
    StagePair* p;
    hipStream_t s;
    ~Back() {
      (void)hipStreamSynchronize(s);
      give_pair(p);
    }
  } back{p, s};
  // chunk c is copied out of its buffer while chunk c + 1 is in flight
  size_t prev_off = 0, prev_len = 0;
  int prev = -1;
  size_t c = 0;
  for (size_t off = 0; off < bytes; off += kStageChunk, ++c) {
    const int k = static_cast<int>(c & 1);
    const size_t len = std::min(kStageChunk, bytes - off);
    AMG_HIP(hipMemcpyAsync(p->buf[k], static_cast<const char*>(src) + off, len, hipMemcpyDeviceToHost, s));
    AMG_HIP(hipEventRecord(p->ev[k], s));
    if (prev >= 0) {
      AMG_HIP(hipEventSynchronize(p->ev[prev]));
      host_copy(static_cast<char*>(dst) + prev_off, p->buf[prev], prev_len);
    }
    prev = k;
    prev_off = off;
    prev_len = len;
  }
  AMG_HIP(hipEventSynchronize(p->ev[prev]));
  host_copy(static_cast<char*>(dst) + prev_off, p->buf[prev], prev_len);
}

}  // namespace amg
