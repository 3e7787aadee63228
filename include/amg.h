/*
 * amg.h -- C ABI of an MI355X (gfx950) smoothed-aggregation AMG solver.
 *
 * The library solves A u = f for a square sparse matrix A given in CSR form
 * (the problem statement of section 2, eq. 1).  Following section 3, the
 * hierarchy is built once on the host (the paper's "AMG setup" algorithm of
 * section 2, with smoothed aggregation as the coarsening strategy) and moved
 * to the device; each solve then runs a Krylov method (CG or BiCGStab,
 * section 3 "Iterative solvers") preconditioned by one V-cycle (section 2,
 * "AMG solve" and the closing remark of section 2) entirely in HIP kernels.
 * The hierarchy is reused across right-hand sides (section 3).
 *
 * Conventions for every entry point:
 *  - No C++ exception crosses this boundary; every failure is a negative
 *    amg_status, and amg_last_error() returns a thread-local message.
 *  - "host" pointers are ordinary CPU memory owned by the caller, read only
 *    during the call (the library copies what it keeps).  "device" pointers
 *    are caller-owned device memory of the current HIP device.
 *  - hip_stream is a hipStream_t (NULL = the legacy default stream).  Work is
 *    enqueued on it; calls that report results (amg_solve, amg_vcycle's
 *    status) synchronise that stream before returning.
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef AMG_H
#define AMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AMG_OK = 0,
  AMG_NOT_CONVERGED = 1,        /* warning: outputs are valid, tol not met   */
  AMG_ERR_INVALID_ARG = -1,     /* NULL pointer, bad enum, bad size          */
  AMG_ERR_BAD_CSR = -2,         /* row_ptr/col malformed or columns unsorted */
  AMG_ERR_ZERO_DIAG = -3,       /* missing or non-positive diagonal entry    */
  AMG_ERR_SINGULAR_COARSE = -4, /* coarsest matrix singular (zero LU pivot)  */
  AMG_ERR_OOM = -5,             /* device or host allocation failed          */
  AMG_ERR_HIP = -6,             /* a HIP runtime call failed                 */
  AMG_ERR_BREAKDOWN = -7,       /* BiCGStab rho = 0 or omega = 0             */
  AMG_ERR_TOO_LARGE = -8,       /* n or nnz too large, coarsest level > 20000 */
  AMG_ERR_NAN = -9              /* non-finite value in the iteration         */
} amg_status;

enum { AMG_CG = 0, AMG_BICGSTAB = 1, AMG_GMRES = 2 }; /* Krylov method (section 3) */
enum { AMG_SPAI0 = 0, AMG_JACOBI = 1, AMG_CHEBYSHEV = 2 }; /* relaxation (section 3) */
enum { AMG_FP64 = 0, AMG_MIXED = 1 };          /* value type of the V-cycle */

/*
 * Method parameters: the paper's nested params structs (section 3.1) and its
 * runtime keys (section 3.2: solver.type, solver.tol,
 * precond.coarsening.type, precond.relax.type), flattened.
 * amg_params_default() fills: CG, SPAI-0, FP64, eps_strong 0.08 (halved on
 * every coarser level), jacobi_omega 0.72, npre = npost = 1, coarse_enough
 * 3000, max_levels 30, max_iter 500, tol 1e-8 (relative to ||f||_2),
 * use_graph 1, check_every 4, cheb_degree 3, cheb_ratio 30, gmres_m 30.
 * AMG_CHEBYSHEV is the diagonally scaled Chebyshev iteration (Saad 2003,
 * cited in section 3) of cheb_degree steps per sweep on [hi/cheb_ratio, hi],
 * hi the Gershgorin bound of D^-1 A_l.
 * AMG_GMRES is flexible restarted GMRES(gmres_m) (Saad 2003, Alg. 9.6; the
 * paper lists GMRES among its solvers in section 3) with Arnoldi by
 * classical Gram-Schmidt applied twice; one iteration is one Arnoldi step,
 * every cycle restarts from the true residual, and its kernels are launched
 * directly (use_graph does not apply).  Its device memory grows by
 * (2 gmres_m + 1) n doubles.
 */
typedef struct {
  int32_t solver;        /* AMG_CG | AMG_BICGSTAB | AMG_GMRES                   */
  int32_t relax;         /* AMG_SPAI0 | AMG_JACOBI | AMG_CHEBYSHEV              */
  int32_t precision;     /* AMG_FP64 | AMG_MIXED (FP32 V-cycle, FP64 Krylov)    */
  int32_t npre;          /* pre-relaxation sweeps per level (>= 0)              */
  int32_t npost;         /* post-relaxation sweeps per level (>= 0)             */
  int32_t coarse_enough; /* a level with at most this many rows is the coarsest */
  int32_t max_levels;    /* hierarchy depth limit (>= 1)                        */
  int32_t max_iter;      /* Krylov iteration limit (>= 1)                       */
  double eps_strong;     /* strength threshold on level 1                      */
  double jacobi_omega;   /* damping of the Jacobi smoother                     */
  double tol;            /* stop when ||r||_2 <= tol * ||f||_2                 */
  int32_t use_graph;     /* 1: replay check_every Krylov iterations as one
                            captured hipGraph; 0: launch kernels directly     */
  int32_t check_every;   /* iterations enqueued between host convergence polls
                            (1..64)                                            */
  int32_t cheb_degree;   /* AMG_CHEBYSHEV: steps per sweep (1..16)              */
  double cheb_ratio;     /* AMG_CHEBYSHEV: upper / lower end of the interval   */
  int32_t gmres_m;       /* AMG_GMRES: restart length m (1..64)                 */
  int32_t fuse_coarse;   /* 1: the levels below level 1 whose operator holds at
                            most 32 MB of values, and the coarse solve, run as
                            one persistent launch with grid-wide barriers
                            (SPAI-0 or Jacobi with npre = npost = 1; other
                            settings always launch per step); bitwise the
                            same result as 0, one launch per step.  Served
                            solves never fuse.  Default 0.                     */
} amg_params;

/* Optional device allocator; NULL everywhere means hipMalloc / hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* hip_stream, void* ctx);
  void (*free)(void* ptr, void* hip_stream, void* ctx);
  void* ctx;
} amg_allocator;

typedef struct {
  int32_t iters;          /* PCG: products q = A p; BiCGStab: loop passes      */
  int32_t levels;         /* L, including the coarsest                         */
  int32_t restarts;       /* 0 or 1 (restart when the true residual misses tol) */
  int32_t status;         /* same as the return value of amg_solve             */
  double rel_resid;       /* recursive ||r|| / ||f|| at exit                   */
  double true_rel_resid;  /* ||f - A u|| / ||f|| recomputed at exit            */
  double setup_s;         /* wall seconds of amg_setup                         */
  double solve_s;         /* wall seconds of this amg_solve                    */
  double op_complexity;   /* sum of nnz(A_l) / nnz(A_1)                        */
} amg_info;

typedef struct amg_solver* amg_handle;

/* Fill *p with the defaults listed above.  p must not be NULL. */
void amg_params_default(amg_params* p);

/*
 * Build the hierarchy for the n x n CSR matrix (row_ptr int64[n+1], col
 * int32[nnz], val double[nnz]; host, caller-owned, copied) and upload it to
 * the current device (section 2, "AMG setup").  The strength graph, the
 * smoothed prolongators and the Galerkin products run on the device on
 * hip_stream, with temporaries from alloc; the greedy aggregation runs on the
 * host; the result is bit-identical to amg_setup_host.  The coarsest level's
 * dense inverse (section 2: a direct solver on the coarsest level) is formed
 * on the device from an LU factorisation, without pivoting when that matrix
 * is symmetric to rounding and every pivot comes out positive (positive
 * definite), with partial pivoting otherwise, and checked once.
 * Requirements:
 * row_ptr[0] = 0, non-decreasing row_ptr, 0 <= col < n, strictly ascending
 * columns within a row, a stored diagonal entry a_ii > 0 in every row,
 * n and nnz below 2^31 - 2^25 (int32 device indices with headroom for
 * grid-stride loops).  p = NULL means defaults.  On success *out receives a handle
 * owning all device memory; on error *out is set to NULL.
 */
amg_status amg_setup(int64_t n, const int64_t* row_ptr, const int32_t* col,
                     const double* val, const amg_params* p,
                     const amg_allocator* alloc, void* hip_stream,
                     amg_handle* out);

/*
 * Same hierarchy construction, host only: nothing is allocated on or sent to
 * a device.  The handle answers the query functions below; amg_solve and
 * amg_vcycle reject it with AMG_ERR_INVALID_ARG.
 */
amg_status amg_setup_host(int64_t n, const int64_t* row_ptr, const int32_t* col,
                          const double* val, const amg_params* p, amg_handle* out);

/*
 * Block values (section 3, "Value types": matrix entries that are 4 x 4
 * blocks, one per pair of coupled grid nodes, as in the paper's
 * Navier-Stokes runs of section 4).  A has nb block rows; block_row_ptr
 * int64[nb+1] (from 0, non-decreasing), block_col int32[nnzb] (strictly
 * ascending per block row, the diagonal block stored), block_val
 * double[16 nnzb] (block k row-major at 16 k); host arrays owned by the
 * caller, read during the call and copied.  block_size must be 4.  The
 * unknowns are interlaced (unknown 4 i + f is component f of node i), so
 * amg_solve, amg_vcycle and amg_time_kernel (which = 5) take vectors of
 * n = 4 nb doubles.  The hierarchy is built blockwise: strength from block
 * Frobenius norms, aggregation over nodes, identity tentative blocks,
 * block-diagonal filtered matrix and damping, block Galerkin products, and
 * block SPAI-0 (the block-diagonal minimiser of ||I - M A||_F) or block
 * Jacobi smoothing, the post-sweep applying M^T.  Supported: solver AMG_CG,
 * AMG_BICGSTAB or AMG_GMRES, relax AMG_SPAI0 or AMG_JACOBI, npre and npost in
 * [0, 16] (one each runs fused kernels; other counts run one product per
 * sweep), precision AMG_FP64 or AMG_MIXED; anything else is
 * AMG_ERR_INVALID_ARG.  amg_time_kernel (which = 5) reports block bytes for
 * npre = npost = 1 only and refuses other counts.
 * coarse_enough counts unknowns (4 nb).  Errors as for amg_setup; a singular
 * diagonal block gives AMG_ERR_ZERO_DIAG.  amg_level_info then reports block
 * rows and stored blocks; amg_get_level_csr, amg_get_smoother and the
 * scalar kernel queries refuse the handle.
 */
amg_status amg_setup_block(int64_t nb, int32_t block_size, const int64_t* block_row_ptr,
                           const int32_t* block_col, const double* block_val,
                           const amg_params* p, const amg_allocator* alloc, void* hip_stream,
                           amg_handle* out);
/* The block hierarchy on the host only (queries only, like amg_setup_host). */
amg_status amg_setup_block_host(int64_t nb, int32_t block_size, const int64_t* block_row_ptr,
                                const int32_t* block_col, const double* block_val,
                                const amg_params* p, amg_handle* out);
/*
 * A block level matrix (which = 0 A_l, 1 P_l, 2 R_l) in the layout of
 * amg_setup_block, arrays sized from amg_level_info (block rows, stored
 * blocks); and the smoother blocks of a level (double[16 nb], M_i row-major)
 * with the prolongator damping.  Block-value handles only.
 */
amg_status amg_get_level_bsr(amg_handle h, int32_t level, int32_t which, int64_t* block_row_ptr,
                             int32_t* block_col, double* block_val);
amg_status amg_get_smoother_blocks(amg_handle h, int32_t level, double* blocks, double* omega);

/*
 * Schur-complement pressure-correction field split (section 3,
 * "Extensibility": a two-step field-split preconditioner whose pressure
 * block is preconditioned with AMG; section 4: the Navier-Stokes runs use it
 * with smoothed aggregation on the pressure and SPAI-0 on the velocity).
 * A is the whole n x n system [[K, G], [D, S]] in the CSR layout of
 * amg_setup, velocity unknowns first: rows and columns 0 .. n_u-1 are the
 * velocity, n_u .. n-1 the pressure.  Diagonal entries may be missing or of
 * any sign outside K; K needs a nonzero diagonal in every row (else
 * AMG_ERR_ZERO_DIAG).  The setup forms M_u = SPAI-0 of K (k_ii / sum_j k_ij^2
 * over K's columns) and S_hat = S - D diag(K)^-1 G, and builds the
 * smoothed-aggregation hierarchy of S_hat as amg_setup builds that of A
 * (a row of S_hat without a positive diagonal is AMG_ERR_ZERO_DIAG).  The
 * preconditioner maps r = (r_u, r_p) to z = (z_u, z_p):
 *   z_p = V(r_p - D (M_u r_u)),  z_u = M_u (r_u - G z_p),
 * V one V-cycle of that hierarchy (FP32 in AMG_MIXED, the rest FP64).
 * amg_solve then solves the whole system (vectors of n doubles) with
 * p->solver AMG_BICGSTAB or AMG_GMRES (the split is not symmetric: AMG_CG is
 * AMG_ERR_INVALID_ARG, as is n_u outside 0 < n_u < n); amg_vcycle applies
 * the preconditioner once to a vector of n doubles.  amg_level_info,
 * amg_get_level_csr and the kernel queries describe the hierarchy of S_hat
 * (level 0 is S_hat, n - n_u rows).  Memory and errors otherwise as for
 * amg_setup.
 */
amg_status amg_setup_schur(int64_t n, const int64_t* row_ptr, const int32_t* col,
                           const double* val, int64_t n_u, const amg_params* p,
                           const amg_allocator* alloc, void* hip_stream, amg_handle* out);
/*
 * The same field split for a system in any order (for example interlaced,
 * four unknowns per mesh node): pmask uint8[n] (host, caller-owned, read
 * during the call) marks each pressure unknown with 1 and each velocity
 * unknown with 0; anything else, or a mask without both fields, is
 * AMG_ERR_INVALID_ARG.  The library renumbers the system velocity first
 * (each field in the caller's order) and works in that order; amg_solve and
 * amg_vcycle take and return vectors in the caller's order (amg_vcycle then
 * uses two of the handle's work vectors, so it must not overlap a solve on
 * the same handle).  The query functions describe the renumbered system's
 * pressure hierarchy.
 */
amg_status amg_setup_schur_masked(int64_t n, const int64_t* row_ptr, const int32_t* col,
                                  const double* val, const uint8_t* pmask, const amg_params* p,
                                  const amg_allocator* alloc, void* hip_stream, amg_handle* out);
/* The field split's setup on the host only (queries only, like amg_setup_host). */
amg_status amg_setup_schur_host(int64_t n, const int64_t* row_ptr, const int32_t* col,
                                const double* val, int64_t n_u, const amg_params* p,
                                amg_handle* out);

/*
 * Solve A u = f.  f_dev, u_dev: device double[n]; u holds the initial guess
 * on entry and the solution on exit.  info may be NULL.  Returns AMG_OK,
 * AMG_NOT_CONVERGED (u is the last iterate), or a negative error.  A zero f
 * gives u = 0 and 0 iterations.
 */
amg_status amg_solve(amg_handle h, const double* f_dev, double* u_dev,
                     void* hip_stream, amg_info* info);

/* Free everything the handle owns.  NULL-safe. */
void amg_release(amg_handle h);

/* Message of the last error on this thread ("" if none). */
const char* amg_last_error(void);

/* --- test and measurement exports ----------------------------------------- */

/*
 * One V-cycle (section 2, "AMG solve", with zero initial guess on every
 * level) applied to r: z = M^-1 r.  r_dev, z_dev: device double[n], must not
 * alias.  Runs in the handle's precision.
 */
amg_status amg_vcycle(amg_handle h, const double* r_dev, double* z_dev, void* hip_stream);

/* Number of levels L of the hierarchy (0 on a NULL handle). */
int32_t amg_num_levels(amg_handle h);

/*
 * Sizes of level `level` (0-based).  n: rows of A_l; nnz_A: stored entries of
 * A_l; nnz_P: stored entries of P_l (0 on the coarsest level).  Any output
 * pointer may be NULL.
 */
amg_status amg_level_info(amg_handle h, int32_t level, int64_t* n, int64_t* nnz_A,
                          int64_t* nnz_P);

/* Aggregate id of every node of level `level` (< L-1); -1 = isolated. Host int32[n]. */
amg_status amg_get_aggregates(amg_handle h, int32_t level, int32_t* agg_host);

/*
 * Copy a level matrix to host arrays sized from amg_level_info: which = 0 for
 * A_l (n x n), 1 for P_l (n x n_{l+1}), 2 for R_l = P_l^T (n_{l+1} x n).
 * row_ptr int64[rows+1], col int32[nnz], val double[nnz].
 */
amg_status amg_get_level_csr(amg_handle h, int32_t level, int32_t which,
                             int64_t* row_ptr, int32_t* col, double* val);

/*
 * Smoother diagonal m_l (host double[n]), prolongator damping omega_l and,
 * for AMG_CHEBYSHEV, the Gershgorin bound of the spectrum of D_l^-1 A_l
 * (0 for the other smoothers).  Any output pointer may be NULL.
 */
amg_status amg_get_smoother(amg_handle h, int32_t level, double* m_host, double* omega,
                            double* cheb_hi);

/*
 * For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): one
 * V-cycle z = V(r) exactly as amg_vcycle computes it (bitwise the same z),
 * whose per-level work vectors live in a fixed device array of the library
 * (64 MiB per GPU, held until the process ends) instead of the handle's
 * memory.  Calls no hipMalloc, hipFree or allocating library routine.
 * r_dev, z_dev: double[n] device arrays of the caller (must not alias).
 * The kernels are enqueued on hip_stream (one launch per step) and the call
 * returns without waiting; the handle's device must be current.  Returns
 * AMG_ERR_TOO_LARGE when the work vectors of the hierarchy (the sum over
 * the levels of their vector lengths times the value size, 256-byte
 * aligned) exceed 64 MiB.  All calls on one GPU share that array: calls
 * that overlap on one GPU (other streams, threads or handles) race.
 */
amg_status amg_vcycle_noalloc(amg_handle h, const double* r_dev, double* z_dev, void* hip_stream);

/*
 * Where the setup's wall time went: seconds[AMG_SETUP_PHASES] receives the
 * time of each step of section 2's "AMG setup", summed over the levels, in
 * this order: 0 copy and validation of the input CSR, 1 strength graph,
 * 2 aggregation, 3 filtered matrix + damping + smoothed prolongator,
 * 4 R = P^T, 5 smoother diagonals, 6 Galerkin products A_{l+1} = R A P,
 * 7 uploads (fine operator to the device for the setup steps, then level
 * matrices, vectors and SpMV schedules), 8 dense inverse of the coarsest
 * operator, 9 everything else.  Their sum is amg_info.setup_s up to the
 * handle's own allocation.
 */
#define AMG_SETUP_PHASES 10
amg_status amg_setup_profile(amg_handle h, double* seconds);

/*
 * Fused coarse levels (the amg_params field fuse_coarse): *first_level =
 * the 0-based first level run inside the single persistent launch (-1 when
 * nothing is fused), *grid = its workgroup count.  Either pointer may be NULL.
 */
amg_status amg_tail_info(amg_handle h, int32_t* first_level, int32_t* grid);
/*
 * Test hook: the longest time (seconds, 0..60; default 0.25) one workgroup
 * of the fused launch waits at a grid barrier before it gives up.  A wait
 * that runs out makes every workgroup of that launch leave at once and the
 * calling amg_solve / amg_vcycle return AMG_ERR_HIP ("ran out of time");
 * the next call starts clean.  Used to check that path with seconds = 0.
 */
amg_status amg_tail_set_wait(amg_handle h, double seconds);

/*
 * SpMV schedule (section 3: the backend's sparse matrix-vector product,
 * variant chosen by row length) that the device path gives a level matrix:
 * which = 0 for A_l, 1 for P_l, 2 for R_l; precision AMG_FP64 or AMG_MIXED
 * (the value type of the copy: FP64, or FP32 for the mixed V-cycle; the
 * Krylov loop's product with A_1 is always FP64).  Outputs as for
 * amg_csr_kernel_info; any may be NULL.  Computed on the host from the
 * level's CSR, so it also answers for handles of amg_setup_host.
 */
amg_status amg_level_kernel_info(amg_handle h, int32_t level, int32_t which, int32_t precision,
                                 int32_t* kind, int32_t* lanes_per_row, int32_t* blocks,
                                 int32_t* block_bytes);

/*
 * Device SpMV y = A x for a standalone CSR matrix, using the same kernel
 * selection as the solver (by row length).  precision AMG_FP64: x, y double;
 * AMG_MIXED: FP32 copies of the values, x and y float.  rows x cols matrix;
 * empty rows give y_i = 0.
 */
typedef struct amg_matrix_s* amg_matrix;
amg_status amg_csr_upload(int64_t rows, int64_t cols, const int64_t* row_ptr,
                          const int32_t* col, const double* val, int32_t precision,
                          void* hip_stream, amg_matrix* out);
amg_status amg_csr_spmv(amg_matrix m, const void* x_dev, void* y_dev, void* hip_stream);
/*
 * kind: 0 = LDS-staged stream kernel (short rows), 1 = sub-wavefront per row;
 * block_bytes: LDS bytes of products per stream block (4096 for matrices
 * with less than 32 MiB of values; otherwise 8192 for FP64 matrices reduced
 * by one lane per row, else the smallest of 4096, 8192 and 16384 that holds
 * 256 / lanes_per_row rows of mean length, 512 / lanes_per_row with 16
 * lanes per row), 0 for kind 1.  Any output pointer
 * may be NULL.
 */
amg_status amg_csr_kernel_info(amg_matrix m, int32_t* kind, int32_t* lanes_per_row,
                               int32_t* blocks, int32_t* block_bytes);
/*
 * Bytes per column index the stream kernel reads for this matrix: 2 when
 * every stream block of at most one LDS pass spans at most 65536 columns
 * (2-byte offsets from a per-block int32 base, which solver handles use for
 * their own stream matrices too), else 4; *bytes is 4 for kind 1.
 */
amg_status amg_csr_column_bytes(amg_matrix m, int32_t* bytes);
void amg_csr_release(amg_matrix m);

/*
 * Measurement: launch one hot kernel of the solve `reps` times back to back
 * on hip_stream between two HIP events and report the mean duration per
 * launch (microseconds) and the kernel's algorithmic HBM bytes per launch
 * (CSR arrays read once, int32 indices, each vector read or written once;
 * a kernel that reads 2-byte column offsets moves fewer bytes than this).
 * which: 0 outer SpMV q = A p with p.q (FP64), 1 level-1 pre-sweep +
 * residual, 2 level-1 post-sweep (with r.z), 3 level-1 restriction,
 * 4 level-1 prolongation + correction, 5 one whole V-cycle (all levels,
 * bytes summed over the hierarchy); field-split handles only: 6 the Krylov
 * loop's SpMV with the whole system (as 0), 7 one application of the
 * field-split preconditioner (its two SpMVs and the pressure V-cycle, bytes
 * summed); on a field-split handle 0-5 concern the pressure hierarchy.
 * 1-5 and 7 run in the handle's precision on its internal work vectors
 * (contents are overwritten).
 */
amg_status amg_time_kernel(amg_handle h, int32_t which, int32_t reps, void* hip_stream,
                           double* avg_us, double* bytes);

/* --- serving: continuous batching of many independent systems -------------- */

/*
 * A request loop over independent systems A u = f of uneven sizes (section 3:
 * the hierarchy depends only on A, is set up once and then lives on the
 * backend).  Submitted requests are set up by `setup_threads` worker
 * threads (device steps on each worker's own stream, their temporaries drawn
 * from the budget without waiting; a step the budget cannot cover at that
 * moment runs on the host), placed in a device pool of hbm_budget_bytes
 * (allocated once here; a request whose footprint exceeds the budget fails
 * with AMG_ERR_OOM) and
 * admitted into one of max_slots (1..64) live slots at an iteration
 * boundary.  Each amg_server_step admits what is ready, runs check_every PCG
 * iterations of every live solve in one captured graph of batched kernels
 * (one launch per operation covers all live solves), then retires the
 * solves that stopped.  Parameters as for amg_setup, restricted to PCG with
 * npre = npost = 1; precision AMG_MIXED is the served configuration.  A
 * request's solution is bitwise identical to amg_solve's for the same system
 * and parameters, whatever else is in the batch.  Threads: one thread drives
 * a server (step, wait_ready, poll, fetch, destroy); amg_server_submit may be
 * called from other threads at the same time (requests arriving from
 * clients), but not during or after amg_server_destroy.
 */
typedef struct amg_server_s* amg_server;
amg_status amg_server_create(const amg_params* p, size_t hbm_budget_bytes, int32_t max_slots,
                             int32_t setup_threads, void* hip_stream, amg_server* out);
/* Copy a request in (host arrays, validated like amg_setup; f_host double[n]). */
amg_status amg_server_submit(amg_server s, uint64_t request_id, int64_t n, const int64_t* row_ptr,
                             const int32_t* col, const double* val, const double* f_host);
/* One step; *live = solves in slots after it, *waiting = submitted, not yet admitted. */
amg_status amg_server_step(amg_server s, int32_t* live, int32_t* waiting);
/* Block until at least `count` submitted requests are set up and waiting for
 * a slot (AMG_OK), or until timeout_s passes or nothing is left in setup
 * (AMG_NOT_CONVERGED); *ready (may be NULL) = requests waiting for a slot. */
amg_status amg_server_wait_ready(amg_server s, int32_t count, double timeout_s, int32_t* ready);
/* Oldest finished request: AMG_OK with its id and size n (0 if it failed before
 * solving), or AMG_NOT_CONVERGED (1) when none is finished. */
amg_status amg_server_poll(amg_server s, uint64_t* request_id, int64_t* n);
/* Take that request: x_host double[n] (may be NULL), info (may be NULL), times
 * (may be NULL) = {submit, setup done, admitted, finished} in seconds of a
 * monotonic clock.  Returns the request's own status; for a failed request
 * amg_last_error() on the calling thread then says what failed. */
amg_status amg_server_fetch(amg_server s, uint64_t request_id, double* x_host, amg_info* info,
                            double* times);
/* Stop the workers and free everything.  NULL-safe. */
void amg_server_destroy(amg_server s);

#ifdef __cplusplus
}
#endif

#endif /* AMG_H */
