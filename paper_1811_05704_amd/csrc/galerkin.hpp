#pragma once
// Galerkin products on the device (section 2, "AMG setup": A_{l+1} = R_l A_l P_l).
//
// The sparse products run on the GPU with the host's arithmetic: every entry
// of C = A B is the sum of its products a_ik b_kj taken in the order the host
// takes them (A's row in stored order, then B's row in stored order), so the
// coarse operators are bit-identical to the host setup's.

#include <hip/hip_runtime.h>

#include "../../include/amg.h"
#include "host_setup.hpp"

namespace amg {

// Ac = R (A P) with both products on the device (the intermediate A P stays
// there); device memory comes from `alloc` (NULL: hipMalloc) and is released
// before returning.  Returns false, leaving Ac untouched, when a row has more
// products than one workgroup sorts or the column count does not fit the
// sort keys; the caller then forms the product on the host.  Throws DevError
// on HIP errors or when the allocator fails.
bool device_galerkin(const Csr& R, const Csr& A, const Csr& P, Csr& Ac, const amg_allocator* alloc,
                     hipStream_t stream);

}  // namespace amg
