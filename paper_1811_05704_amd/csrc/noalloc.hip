// amg_vcycle_noalloc: one V-cycle (section 2, "AMG solve") whose work
// vectors live in a fixed device array of this library instead of the
// handle's allocations, for callers that cannot allocate device memory
// (code under stream capture, tight serving loops).
//
// The per-level work vectors of the V-cycle (right-hand sides, m .* f,
// residuals, prolongated corrections, outputs, sweep buffers) are carved out
// of `scratch`, a file-scope device array of kNoAllocScratchBytes that every
// GPU the library runs on holds until the process ends.  Host code never
// uses the array's name as an address: the device address is looked up once
// per device with hipGetSymbolAddress and kept.  The call enqueues the same
// kernels as amg_vcycle (one launch per step; the fused coarse launch is not
// used, so no barrier state is involved) and returns without waiting.  Every
// vector is written before it is read within one V-cycle, so nothing needs
// clearing between calls.  All calls on one GPU share the array: calls that
// overlap on one GPU (other streams, threads or handles) race.

#include <mutex>

#include "solver.hpp"

using namespace amg;

namespace {

constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// Device address of `scratch` per device, looked up with that device current.
unsigned char* scratch_on_device(int device) {
  static std::mutex mu;
  static unsigned char* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) throw SetupError{-1, "device ordinal out of range"};
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {
    int cur = 0;
    AMG_HIP(hipGetDevice(&cur));
    if (cur != device) AMG_HIP(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      throw DevError{-6, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    addr[device] = static_cast<unsigned char*>(p);
  }
  return addr[device];
}

// Bump allocation inside the scratch array (256-byte aligned pieces).
struct Carve {
  unsigned char* base;
  size_t used = 0;
  template <class T>
  T* take(int64_t count) {
    const size_t bytes = (static_cast<size_t>(count) * sizeof(T) + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + used);
    used += bytes;
    return p;
  }
};

// Points the hierarchy's work vectors into the scratch array for one call
// and puts the handle's own back afterwards (also on an exception).  Needs
// no allocation: the levels are re-pointed in place.
template <class T>
class ScratchVectors {
 public:
  ScratchVectors(DevHierarchy<T>& H, int64_t nL, unsigned char* base, bool dry) : H_(H) {
    Carve c{base};
    saved_tail_ = H.tail_first;
    for (size_t l = 0; l < H.lev.size(); ++l) {
      DevLevel<T>& v = H.lev[l];
      DevLevel<T> w = v;  // only the pointer members below change
      auto repoint = [&](T*& dst, const T* own) {
        if (own) dst = c.take<T>(v.n);
      };
      repoint(w.f, v.f);
      repoint(w.r, v.r);
      repoint(w.y, v.y);
      repoint(w.t, v.t);
      repoint(w.zp[0], v.zp[0]);
      repoint(w.zp[1], v.zp[1]);
      repoint(w.z, v.z);
      repoint(w.mf, v.mf);
      repoint(w.dc[0], v.dc[0]);
      repoint(w.dc[1], v.dc[1]);
      if (!dry) {
        saved_[l] = v;
        have_[l] = true;
        v = w;
      }
    }
    T* fL = H.fL ? c.take<T>(nL) : nullptr;
    T* zL = H.zL ? c.take<T>(nL) : nullptr;
    bytes_ = c.used;
    if (!dry) {
      saved_fL_ = H.fL;
      saved_zL_ = H.zL;
      H.fL = fL;
      H.zL = zL;
      H.tail_first = 0;
      active_ = true;
    }
  }
  ~ScratchVectors() {
    if (!active_) return;
    for (size_t l = 0; l < H_.lev.size() && l < kMaxLevels; ++l)
      if (have_[l]) H_.lev[l] = saved_[l];
    H_.fL = saved_fL_;
    H_.zL = saved_zL_;
    H_.tail_first = saved_tail_;
  }
  size_t bytes() const { return bytes_; }

  static constexpr size_t kMaxLevels = 32;

 private:
  DevHierarchy<T>& H_;
  DevLevel<T> saved_[kMaxLevels];
  bool have_[kMaxLevels] = {};
  T* saved_fL_ = nullptr;
  T* saved_zL_ = nullptr;
  int saved_tail_ = 0;
  size_t bytes_ = 0;
  bool active_ = false;
};

template <class T>
amg_status vcycle_noalloc(amg_solver& S, DevHierarchy<T>& H, const double* r, double* z, hipStream_t s) {
  if (H.lev.size() > ScratchVectors<T>::kMaxLevels) throw SetupError{-8, "hierarchy too deep for the scratch layout"};
  unsigned char* base = scratch_on_device(S.device);
  {
    ScratchVectors<T> probe(H, S.nL, base, true);
    if (probe.bytes() > kNoAllocScratchBytes)
      throw SetupError{-8, "V-cycle work vectors need " + std::to_string(probe.bytes()) +
                               " bytes; the fixed scratch array holds " + std::to_string(kNoAllocScratchBytes)};
  }
  ScratchVectors<T> use(H, S.nL, base, false);
  VcycleOpts o{S.prm.npre, S.prm.npost, S.prm.relax};
  Vcycle<T> V(&H, S.Ainv, S.nL, o);
  V.template run<0>(r, z, nullptr, nullptr, s);
  return AMG_OK;
}

}  // namespace

extern "C" amg_status amg_vcycle_noalloc(amg_handle h, const double* r_dev, double* z_dev, void* hip_stream) {
  return guarded([&]() -> amg_status {
    if (!h || !r_dev || !z_dev) throw SetupError{-1, "NULL handle or vector"};
    if (!h->on_device) throw SetupError{-1, "handle was built by amg_setup_host: no device data"};
    if (h->block) throw SetupError{-1, "block-value handles are not supported here"};
    if (h->schur) throw SetupError{-1, "field-split handles are not supported here"};
    if (static_cast<const void*>(r_dev) == static_cast<const void*>(z_dev))
      throw SetupError{-1, "r and z must not alias"};
    int cur = 0;
    AMG_HIP(hipGetDevice(&cur));
    if (cur != h->device) throw SetupError{-1, "the handle's device is not the current device"};
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (h->prm.precision == AMG_MIXED) return vcycle_noalloc<float>(*h, h->h32, r_dev, z_dev, s);
    return vcycle_noalloc<double>(*h, h->h64, r_dev, z_dev, s);
  });
}
