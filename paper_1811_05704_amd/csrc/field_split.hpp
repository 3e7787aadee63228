// Schur-complement pressure-correction field split (section 3,
// "Extensibility"; the Navier-Stokes runs of section 4), host part of the
// setup.  The system A = [[K, G], [D, S]] holds the velocity unknowns first
// (rows and columns 0 .. n_u-1) and the pressure unknowns after them.  The
// preconditioner applies, to r = (r_u, r_p),
//   u* = M_u r_u,   p = V(S_hat; r_p - D u*),   u = M_u (r_u - G p),
// with M_u the SPAI-0 diagonal of K, S_hat = S - D diag(K)^-1 G and V one
// smoothed-aggregation V-cycle of S_hat.
#pragma once

#include <cstdint>
#include <vector>

#include "host_setup.hpp"

namespace amg {

struct FieldSplit {
  int64_t n_u = 0;  // velocity unknowns
  Csr A;            // the whole system (the Krylov loop's operator)
  Csr Dm;           // D diag(M_u): pressure rows, velocity columns
  Csr G;            // velocity rows, pressure columns numbered from 0
  hvec<double> mu;  // SPAI-0 diagonal of K: k_ii / sum_j k_ij^2 over K's columns
  // The caller's index of each unknown of the velocity-first order (empty:
  // the caller's order is velocity first).
  std::vector<int32_t> old_of_new;
};

// Velocity-first order of a system whose pressure unknowns are marked by
// pmask[i] = 1 (velocity 0; the fields in any order): old_of_new[j] is the
// caller's index of unknown j of the new order (the velocity unknowns, then
// the pressure unknowns, each in the caller's order).  Returns n_u; throws
// SetupError unless every entry is 0 or 1 and both fields are present.
int64_t field_order(int64_t n, const uint8_t* pmask, std::vector<int32_t>* old_of_new);

// B = Q A Q^T with Q the permutation of old_of_new (row j of B is row
// old_of_new[j] of A, columns renumbered and ascending).
Csr permute_symmetric(const Csr& A, const std::vector<int32_t>& old_of_new);

// Takes the whole system A (columns ascending within each row), fills *out
// with it and the preconditioner's operators, and returns S_hat (columns
// ascending, entries that sum to exactly zero dropped).  S_hat's entries are
// s_ij - sum_k (d_ik / k_kk) g_kj, the products summed in ascending k
// (with d_ik / k_kk formed as d_ik * (1 / k_kk)).  Throws SetupError if not
// 0 < n_u < n, if a velocity row has a zero or missing diagonal, or if a row
// of S_hat has no positive diagonal.
Csr split_fields(Csr A, int64_t n_u, FieldSplit* out);

}  // namespace amg
