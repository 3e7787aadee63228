// Host-side smoothed-aggregation setup for block values (section 3, "Value
// types": the entries of the matrix are small dense b x b blocks, one per
// pair of coupled grid nodes; the paper's Navier-Stokes runs use 4 x 4).
// The method of section 2 ("AMG setup") taken blockwise: the b unknowns of a
// node move together through the hierarchy.
#pragma once

#include <cstdint>
#include <vector>

#include "host_setup.hpp"

namespace amg {

constexpr int kBlock = 4;  // the block size the library is built for
constexpr int kBB = kBlock * kBlock;

// Block sparse matrix: rows x cols blocks of kBlock x kBlock, each stored
// row-major (kBB values); block columns ascending within a block row.
struct Bsr {
  int64_t rows = 0, cols = 0;
  std::vector<int64_t> ptr;
  hvec<int32_t> col;  // block columns, ascending within each block row
  hvec<double> val;   // 16 values per block, row-major
  int64_t nnzb() const { return ptr.empty() ? 0 : ptr.back(); }
};

struct BlockLevel {
  Bsr A, P, R;                // P, R empty on the coarsest level
  std::vector<int32_t> agg;   // aggregate per node, -1 isolated
  std::vector<double> M;      // smoother block per node (kBB values)
  double omega = 0.0;         // prolongator damping
  double eps = 0.0;           // strength threshold used on this level
};

struct BlockHierarchy {
  std::vector<BlockLevel> levels;  // the last one is the coarsest (A only)
  double phase_s[kPhCount] = {};
};

// Validates a block CSR input (block row pointers from 0, non-decreasing,
// block columns in range and strictly ascending, a stored diagonal block,
// finite values, nnzb * kBB < 2^31); throws SetupError.
void validate_bsr(int64_t nb, const int64_t* ptr, const int32_t* col, const double* val);

// Full block hierarchy (relax 0 = block SPAI-0, 1 = block Jacobi); throws
// SetupError.  A level with b * rows <= coarse_enough unknowns is the coarsest.
BlockHierarchy build_block_hierarchy(Bsr A, const SetupParams& prm);

// Scalar CSR form (kBlock rows per block row), every stored block entry kept.
Csr bsr_to_csr(const Bsr& A);

// Steps, exposed for the tests of the host logic.
void block_inverse(const double* B, double* inv);  // Gauss-Jordan, partial pivoting
Graph block_strength_graph(const Bsr& A, double eps);
Bsr block_spgemm(const Bsr& X, const Bsr& Y);
Bsr block_transpose(const Bsr& P);

}  // namespace amg
