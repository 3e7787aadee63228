#pragma once
// Setup steps on the device (section 2, "AMG setup": strength graph, smoothed
// prolongator, A_{l+1} = R_l A_l P_l).
//
// The sparse products run on the GPU with the host's arithmetic: every entry
// of C = A B is the sum of its products a_ik b_kj taken in the order the host
// takes them (A's row in stored order, then B's row in stored order), so the
// coarse operators are bit-identical to the host setup's.

#include <hip/hip_runtime.h>

#include <functional>
#include <memory>

#include "../../include/amg.h"
#include "host_setup.hpp"

namespace amg {

// Accelerator of the setup's data-parallel steps on the device: strength
// graph, smoothed prolongator and Galerkin products, each bit-identical to
// the host step; the coarse operator a level produces stays on the device
// for the next level.  Device memory comes from `alloc` (NULL: hipMalloc);
// a step whose allocation fails, whose rows do not fit the sort blocks, or
// (strength graph) whose matrix is structurally nonsymmetric is left to the
// host.  Other HIP errors throw DevError.
//
// `fine` (optional) is a device copy of the level-1 matrix the caller already
// holds (int32 row pointers and columns, FP64 values, valid while the
// accelerator lives); level 1 then uses it instead of uploading A again.
// With `keep_levels` the accelerator keeps every level's device matrices
// (A, P, R = P^T, smoother diagonal) until it is destroyed, for
// device_level_refs; otherwise a level's storage goes when the next begins.
struct DeviceCsrRef {
  int32_t rows = 0, cols = 0;
  int64_t nnz = 0;
  const int32_t* ptr = nullptr;
  const int32_t* col = nullptr;
  const double* val = nullptr;  // NULL: not on the device
};
// `on_host_work` (optional) runs once, on the calling thread, when the host
// first starts aggregating (the device has nothing queued then).
std::unique_ptr<SetupAccel> make_device_setup_accel(const amg_allocator* alloc, hipStream_t stream,
                                                    const DeviceCsrRef* fine = nullptr, bool keep_levels = false,
                                                    std::function<void()> on_host_work = nullptr);

// Has the runtime load the code object of the setup kernels on the calling
// thread (it is loaded on first use otherwise).
void preload_setup_kernels();

// FP64 device copies the accelerator made for level `level` (0-based), equal
// to the host hierarchy's; a member with val == NULL (m == NULL) was made on
// the host.  False when the accelerator keeps no levels or has no such level.
struct DeviceLevelRefs {
  DeviceCsrRef A, P, R;
  const double* m = nullptr;
};
bool device_level_refs(const SetupAccel* accel, int level, DeviceLevelRefs* out);

}  // namespace amg
