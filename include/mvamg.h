/*
 * mvamg.h -- C ABI of the MI355X (gfx950) solve phase of the single-hierarchy
 * multiple-vector aggregation-based AMG (D'Ambra & Vassilevski, "Improving
 * Solve Time of Aggregation-based Adaptive AMG").
 *
 * The library solves A x = b, A sparse symmetric positive definite (Section 1),
 * by conjugate gradients preconditioned with one V-cycle of a hierarchy whose
 * prolongators P^k = blockdiag(U_a) are block diagonal over composite
 * aggregates, each block an orthonormal basis of the smooth vectors restricted
 * to the aggregate, with Galerkin coarse matrices A^k = (P^k)^T A^{k-1} P^k
 * (Section 4).  The cycle uses forward Gauss-Seidel pre-smoothing, backward
 * Gauss-Seidel post-smoothing and an exact coarsest solve (Section 5).
 *
 * Conventions shared by every entry point:
 *   - Device pointers are HIP device memory owned by the caller (for example
 *     torch tensors); the library never frees them.  Host pointers are plain
 *     host memory.  Vectors are float64 of length n (the order of the rows of
 *     the hierarchy file's level 0) unless stated otherwise.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *     device work of a call is enqueued on it; calls that return results to
 *     the host synchronise it.
 *   - Every call returns an mvamg_status.  On failure mvamg_last_error()
 *     returns a message (thread-local, valid until the next call on that
 *     thread).  No C++ exception crosses the ABI.  Arguments are validated on
 *     the host before any kernel is launched.
 *   - A handle is bound to the device that was current at mvamg_upload;
 *     calls on it must run with that device current.  Calls on one handle must
 *     not overlap (the handle owns its work vectors).
 */
#ifndef MVAMG_H
#define MVAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MVAMG_OK = 0,
  MVAMG_NOT_CONVERGED = 1,  /* maxit reached; x holds the last iterate, info is filled */
  MVAMG_ERR_ARG = -1,       /* invalid argument (null pointer, size, unsupported option) */
  MVAMG_ERR_FILE = -2,      /* hierarchy file missing, truncated or inconsistent */
  MVAMG_ERR_NOT_SPD = -3,   /* coarsest Cholesky pivot <= 0, or a non-positive diagonal */
  MVAMG_ERR_NONFINITE = -4, /* NaN or Inf in the right-hand side or initial guess */
  MVAMG_ERR_BREAKDOWN = -5, /* p^T A p <= 0 in CG (matrix not s.p.d.) */
  MVAMG_ERR_HIP = -6        /* a HIP runtime call failed */
} mvamg_status;

/* Parsed hierarchy file in host memory, owned by the library. */
typedef struct mvamg_hier_host mvamg_hier_host;
/* Hierarchy resident on one GPU, owned by the library (device memory
   allocated at upload, released by mvamg_free). */
typedef struct mvamg_hier mvamg_hier;

enum { MVAMG_SMOOTH_GS = 0, MVAMG_SMOOTH_L1JACOBI = 1 };
/* The preconditioner CG applies: one V-cycle, or one K-cycle -- the V-cycle's
   smoothing and transfers, with the coarse correction on every level that is
   neither the finest nor the coarsest taken as two flexible-CG iterations on
   that level, each preconditioned by the K-cycle of that level (Section 5:
   the bootstrap applies its AMG components as K-cycles, nonlinear AMLI
   cycles, with two inner flexible-CG iterations per level but the
   coarsest). */
enum { MVAMG_CYCLE_V = 0, MVAMG_CYCLE_K = 1 };

typedef struct {
  int precision;     /* 64: whole cycle in binary64; 32: cycle (smoother, level
                        residuals, transfers) in binary32, coarsest solve, CG
                        recurrences and inner products in binary64, flexible CG */
  int smoother;      /* MVAMG_SMOOTH_GS (multicolour Gauss-Seidel, Section 5) or
                        MVAMG_SMOOTH_L1JACOBI (one l1-Jacobi sweep pre and post) */
  double rtol;       /* stop when ||r_k||_2 <= rtol * ||b - A x_0||_2 (Section 5) */
  int maxit;         /* iteration cap (the paper uses 1000) */
  int max_restarts;  /* precision 32: restarts from x when the recomputed true
                        residual misses rtol (iterative refinement); ignored for 64 */
  double* history;   /* host, optional (NULL): receives ||r_k|| / ||r_0|| for
                        k = 0..iterations; capacity maxit + 1 */
  int cycle;         /* MVAMG_CYCLE_V, or MVAMG_CYCLE_K (precision 64 only; the
                        K-cycle is not a linear operator, so CG then takes the
                        flexible beta); block and batch solves take V only */
} mvamg_solve_params;

typedef struct {
  int iterations;      /* CG iterations (A p products) performed */
  int converged;       /* 1 if rtol was met */
  int restarts;        /* true-residual restarts taken (precision 32) */
  double rel_res;      /* last recursive ||r_k|| / ||r_0|| */
  double rel_res_true; /* ||b - A x|| / ||r_0|| recomputed in binary64 at exit */
} mvamg_info;

/* ---------------------------------------------------------------- setup */

/* Reads a hierarchy file written by the host setup (levels A^k in CSR, the
   smoother order of every non-coarsest level, the blocks U_a of every P^k).
   *out must be released with mvamg_hier_host_free.  Errors: MVAMG_ERR_FILE. */
mvamg_status mvamg_hier_read(const char* path, mvamg_hier_host** out);
void mvamg_hier_host_free(mvamg_hier_host* h);

/* Level count, fine size n and fine nonzeros of a parsed file. */
mvamg_status mvamg_hier_host_info(const mvamg_hier_host* h, int* nlevels, int* n, int64_t* nnz);

/* Device memory of a handle.  The caller owns all of it: one arena (a
   device buffer, 256-byte aligned, e.g. a torch uint8 tensor) per handle,
   passed to mvamg_upload and borrowed by the handle until mvamg_free; it
   must not be freed or reused before.  The library keeps only host
   structures (the parsed layout, mapped host memory for the per-iteration
   scalars, captured graphs).

   *bytes receives the arena size mvamg_upload needs for h: the level
   layouts in binary64 and binary32, the transfers, the coarsest inverse, the
   CG and cycle work vectors, and the temporaries of the coarsest
   factorisation (released inside the arena and reused).  nrhs > 1 (at most
   MVAMG_BLOCK_MAX) adds the work space of the block calls for several
   right-hand sides.  Host only, nothing touches the device.
   Errors: MVAMG_ERR_ARG. */
mvamg_status mvamg_arena_bytes(const mvamg_hier_host* h, int nrhs, size_t* bytes);

/* Copies the hierarchy into the caller's arena (arena_bytes bytes at
   arena_dev) in the library's layout (rows permuted into smoother order,
   off-group entries in sliced-ELL or grouped CSR, per-aggregate U blocks),
   keeps binary32 copies for the mixed cycle, and factors the coarsest matrix
   with a dense Cholesky on the device (Section 5 uses a direct coarsest
   solve).  Allocates no device memory.  The host object may be freed
   afterwards.  Errors: MVAMG_ERR_ARG (null or unaligned arena, an arena
   smaller than mvamg_arena_bytes reports -- also raised by the first block
   call when the arena was sized with nrhs = 1), MVAMG_ERR_NOT_SPD,
   MVAMG_ERR_HIP. */
mvamg_status mvamg_upload(const mvamg_hier_host* h, void* arena_dev, size_t arena_bytes, void* stream,
                          mvamg_hier** out);
/* Releases the handle's host structures; the arena goes back to the caller. */
void mvamg_free(mvamg_hier* h);

/* Level count and sizes of an uploaded hierarchy: n[l], nnz[l] for
   l < nlevels (arrays of capacity 32, may be NULL), stages[l] = number of
   smoother stages (0 on the coarsest). */
mvamg_status mvamg_levels(const mvamg_hier* h, int* nlevels, int* n, int64_t* nnz, int* stages);

/* Sizes of the transfers P^l of an uploaded hierarchy, l < nlevels - 1:
   nagg[l] aggregates and nu[l] = sum over aggregates of n_a k_a stored
   entries of the blocks U_a (arrays of capacity 32, may be NULL). */
mvamg_status mvamg_transfers(const mvamg_hier* h, int* nagg, int64_t* nu);

/* Replaces the values of the finest matrix by val_dev (device, float64,
   nnz entries in the CSR order of the file's level 0): a near-by matrix with
   the same pattern (Section 1).  The fine-level products and smoothing use
   the new values, coarser levels keep the stored Galerkin matrices.  The
   1-byte value codes a sliced-ELL fine level may use describe the uploaded
   values only: from this call on the kernels read the stored values, and the
   captured iteration graphs are rebuilt on the next solve.  Ordered on
   `stream` like the solves; errors: MVAMG_ERR_ARG, MVAMG_ERR_HIP. */
mvamg_status mvamg_set_fine_values(mvamg_hier* h, const double* val_dev, void* stream);

/* ---------------------------------------------------------------- solve */

/* y = A x with the current finest matrix (device vectors, file order). */
mvamg_status mvamg_spmv(mvamg_hier* h, const double* x_dev, double* y_dev, void* stream);

/* z = B r: one V-cycle from a zero initial guess (Section 5).
   precision 64 or 32 (binary32 inside the cycle), smoother as in
   mvamg_solve_params.  r_dev and z_dev must not alias. */
mvamg_status mvamg_cycle_apply(mvamg_hier* h, const double* r_dev, double* z_dev, int precision,
                               int smoother, void* stream);

/* z = K r: one K-cycle (MVAMG_CYCLE_K) from a zero initial guess, binary64,
   smoother as in mvamg_solve_params.  On a two-level hierarchy it equals
   mvamg_cycle_apply.  r_dev and z_dev must not alias. */
mvamg_status mvamg_kcycle_apply(mvamg_hier* h, const double* r_dev, double* z_dev, int smoother, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, serving loops, harnesses that forbid hipMalloc): z = B r exactly
   as mvamg_cycle_apply (same kernels, same results bit for bit), but every
   work vector of the cycle -- the level-0 input and output in smoother
   order, r, x and s of every level in the cycle's precision, the coarsest
   solve's vectors and product slots -- lives in one static device array of
   MVAMG_NOALLOC_SCRATCH_BYTES per device instead of the handle's work space.
   The call allocates nothing: no hipMalloc, hipFree or allocating library
   routine.  The array is set up on the first call on a device (its address
   is taken once and kept) and held until the process ends.  Every call on a
   device shares that device's array and leaves its contents behind; nothing
   in it needs to start at zero.  Calls that overlap on one device (two
   streams, two threads) race on the array and must not be issued.
   MVAMG_ERR_ARG if the cycle's work space exceeds the array (about 1.3 M
   fine rows in binary64, 2.5 M in binary32, with the usual coarse levels) or
   while measurement (mvamg_profile) is on. */
#define MVAMG_NOALLOC_SCRATCH_BYTES (32u << 20)
mvamg_status mvamg_cycle_apply_noalloc(mvamg_hier* h, const double* r_dev, double* z_dev, int precision,
                                       int smoother, void* stream);

/* Preconditioned CG (Section 5) on A x = b with B = one V-cycle.  A is the
   finest-level matrix in the file's CSR form (device arrays: rowptr int32
   [n+1], col int32 [nnz], val float64 [nnz]).  It must have the hierarchy's
   pattern; its values may differ from the hierarchy's A_0 (a near-by matrix,
   Section 1): the fine-level products and smoothing then use them, coarser
   levels keep the stored Galerkin matrices.  rowptr and col are compared
   with the stored pattern (MVAMG_ERR_ARG if they differ); both may be NULL to
   skip that check.  val is compared with the values in use and, if any
   entry differs, replaces them as mvamg_set_fine_values does; NULL keeps
   the values in use.  x_dev holds
   x_0 on entry (zero for the paper's setting) and the solution on exit.
   Returns MVAMG_OK, MVAMG_NOT_CONVERGED, or an error.  Each iteration's
   scalars (||r_k||^2 for the stopping test, the breakdown flag) are written
   by the last kernel of the iteration straight into mapped host memory that
   the handle owns (two slots, alternating); the host reads them once the
   iteration has ended.  The first solve of each precision and smoother
   captures one iteration as a HIP graph and replays it, with the next
   iteration queued before the host reads the current one's scalars; an
   iteration queued past the stopping one only applies the last step's
   pending x update.  The runtime's executable graph holds about 2 MiB of
   device memory of its own until mvamg_free (the environment variable
   MVAMG_NO_GRAPH=1, read at upload, runs plain launches, one iteration at a
   time, instead). */
mvamg_status mvamg_pcg_solve(mvamg_hier* h, const int* rowptr_dev, const int* col_dev, const double* val_dev,
                             const double* b_dev, double* x_dev, const mvamg_solve_params* prm, mvamg_info* info,
                             void* stream);

/* Adjoint solve for a loss L(x): A^T lambda = dL/dx.  A is symmetric, so
   this is the same preconditioned CG with right-hand side dLdx_dev (the
   hierarchy is reused as is).  rowptr_dev, col_dev, val_dev: A, as for
   mvamg_pcg_solve.  lambda_dev receives the solution (initial guess zero). */
mvamg_status mvamg_adjoint_solve(mvamg_hier* h, const int* rowptr_dev, const int* col_dev, const double* val_dev,
                                 const double* dLdx_dev, double* lambda_dev, const mvamg_solve_params* prm,
                                 mvamg_info* info, void* stream);

/* Gradient of L with respect to the stored finest-matrix values:
   dval[k] = -lambda_i x_j for the k-th stored entry (i, j) of the file's
   level-0 CSR pattern.  (dL/db = lambda.) */
mvamg_status mvamg_grad_coeffs(mvamg_hier* h, const double* lambda_dev, const double* x_dev,
                               double* dval_dev, void* stream);

/* ------------------------------------------- several right-hand sides */

/* Up to MVAMG_BLOCK_MAX right-hand sides through one hierarchy (the same
   method applied to each column; the paper motivates amortising one
   hierarchy over many solves, Sections 1 and 6).  Blocks are device arrays
   of n x m binary64 values, row-major (row i holds the m values of row i of
   every column, file order of the rows).  The library stages them in n x 32
   blocks so that one load of a matrix entry serves every column; columns
   m..31 are carried as zero.  The first block call on a handle takes
   about (7 x 8 + 3 x 4) x 32 bytes per fine row of work space from the
   arena, kept until mvamg_free: size the arena with nrhs > 1
   (mvamg_arena_bytes).  Not available on batch handles. */
#define MVAMG_BLOCK_MAX 32

/* Y = A X for m columns (1 <= m <= 32). */
mvamg_status mvamg_spmv_block(mvamg_hier* h, const double* X_dev, double* Y_dev, int m, void* stream);

/* Z = B R: one V-cycle per column (as mvamg_cycle_apply). */
mvamg_status mvamg_cycle_apply_block(mvamg_hier* h, const double* R_dev, double* Z_dev, int m, int precision,
                                     int smoother, void* stream);

/* Preconditioned CG on the m systems A X[:, c] = B[:, c] at once.  Every
   column has its own alpha, beta, stopping test, iteration count and (binary32
   cycle) restarts; a column that met rtol keeps its iterate while the others
   go on.  info: m entries (may be NULL).  prm->history, if not NULL, holds
   m x (maxit + 1) values, column c's history at c * (maxit + 1).  Returns
   MVAMG_OK if every column converged, MVAMG_NOT_CONVERGED otherwise; a
   breakdown or non-finite value in any column is an error for the call. */
mvamg_status mvamg_pcg_solve_block(mvamg_hier* h, const double* B_dev, double* X_dev, int m,
                                   const mvamg_solve_params* prm, mvamg_info* info, void* stream);

/* ------------------------------------------------ batch of problems */

/* Uploads nprob independent hierarchies (each parsed by mvamg_hier_read) as
   one batch.  Vectors of a batch are the problems' vectors one after another
   (problem p at rows offsets[p] .. offsets[p+1]-1 of mvamg_batch_problems).
   The problems are split between two paths:
   - the small-problem path: every problem with at most mini_rows rows, and
     every problem whose level count differs from the most common one among
     the others, is solved by one persistent launch in which one workgroup
     runs the whole CG and V-cycle of a problem over its own hierarchy (any
     depth from 2 to 16 levels, coarsest at most 2048 rows), using only
     workgroup barriers; the workgroups stride over the problems;
   - the lockstep path: the other problems form one block-diagonal hierarchy
     (level l holds level l of every such problem, smoother stage c holds
     stage c of every problem, every problem keeps its own coarsest inverse),
     and each launch of a level kernel covers the same step of all of them.
   mini_rows = 0 puts everything on the lockstep path unless the level counts
   differ.  The handle is released with mvamg_free; mvamg_spmv,
   mvamg_cycle_apply (block diagonal) and mvamg_set_fine_values accept it
   when no problem is on the small path; mvamg_pcg_solve does not.  The
   caller owns the device memory, as for mvamg_upload: *bytes of
   mvamg_batch_arena_bytes (host only) is the arena mvamg_batch_upload needs.
   Errors: MVAMG_ERR_ARG (too large, arena too small), as mvamg_upload. */
mvamg_status mvamg_batch_arena_bytes(const mvamg_hier_host* const* hs, int nprob, int mini_rows, size_t* bytes);
mvamg_status mvamg_batch_upload(const mvamg_hier_host* const* hs, int nprob, int mini_rows, void* arena_dev,
                                size_t arena_bytes, void* stream, mvamg_hier** out);

/* flags[p] (nprob entries) = 1 if problem p is on the small-problem path. */
mvamg_status mvamg_batch_small_path(const mvamg_hier* h, int* flags);

/* Problem count (0 for a single-problem handle) and row offsets
   (nprob + 1 entries, may be NULL). */
mvamg_status mvamg_batch_problems(const mvamg_hier* h, int* nprob, int* offsets);

/* Preconditioned CG on every problem of a batch, each with its own
   recurrence, stopping test and restarts (as mvamg_pcg_solve_block with
   problems in place of columns; info and history have nprob entries /
   rows).  With problems on the small-problem path: precision 64 only and
   maxit at most 1000; that path's launch runs on a second stream of the
   handle while the lockstep path runs on `stream`, and the call returns when
   both are done. */
mvamg_status mvamg_batch_pcg_solve(mvamg_hier* h, const double* b_dev, double* x_dev,
                                   const mvamg_solve_params* prm, mvamg_info* info, void* stream);

/* ------------------------------------------ composite (bootstrap) AMG */

/* The bootstrap's own solver (eq. 1.1 and Algorithm 1; Section 5 item (i)):
   the symmetrized multiplicative composite of r hierarchies B_1..B_r built on
   one fine matrix A (the files the host setup writes for every bootstrap
   stage), whose error propagator is
     I - B A = (I - B_1 A)..(I - B_r A)(I - B_r A)..(I - B_1 A),
   applied factor by factor, rightmost first.  hs holds r single-problem
   handles whose finest matrices agree in size, pattern and values (checked
   on the device; MVAMG_ERR_ARG otherwise); products with A use hs[0]'s.
   cycle: every component a V-cycle or a K-cycle (the paper's bootstrap
   default), binary64.  Vectors are device arrays in the file's row order.
   The calls take a caller-owned device work space (256-byte aligned) of at
   least *bytes from mvamg_composite_work_bytes(n); calls sharing a work space
   or a handle must not overlap.  The handles' own level vectors are used as
   scratch by every factor. */
mvamg_status mvamg_composite_work_bytes(int n, size_t* bytes);

/* z = B res, from z = 0: every factor k takes z += B_k (res - A z). */
mvamg_status mvamg_composite_apply(mvamg_hier* const* hs, int r, int cycle, int smoother, const double* res_dev,
                                   double* z_dev, void* work_dev, size_t work_bytes, void* stream);

/* The testing phase of Algorithm 1 with the symmetrized product: x <- E x,
   nu times (every factor x <- x - B_k A x), from x_dev's content.  *rho
   receives ||x^nu||_A / ||x^{nu-1}||_A and x_dev the new smooth vector
   x^nu / ||x^nu||_A (x^nu if its A-norm is zero). */
mvamg_status mvamg_composite_test(mvamg_hier* const* hs, int r, int cycle, int smoother, int nu, double* x_dev,
                                  double* rho, void* work_dev, size_t work_bytes, void* stream);

/* CG preconditioned by the composite (the paper's original bootstrap AMG),
   with the flexible beta (K-cycle components are not linear); prm as for
   mvamg_pcg_solve (precision 64; max_restarts ignored).  x_dev holds x_0 on
   entry and the solution on exit; each iteration reads its inner products
   on the host. */
mvamg_status mvamg_composite_pcg_solve(mvamg_hier* const* hs, int r, const double* b_dev, double* x_dev,
                                       const mvamg_solve_params* prm, mvamg_info* info, void* work_dev,
                                       size_t work_bytes, void* stream);

/* ------------------------------------------ numeric setup of a level */

/* One multiple-vector level's numeric setup on the device (Section 4):
   the local bases (eq. 4.3), the Galerkin coarse matrix A_c = P^T A P with
   P = blockdiag(U_a), and the smooth vectors on the coarse level (Section
   4.1).  The aggregates come from the host setup (matching and composition,
   Sections 3 and 4).  Arrays are device arrays unless stated; the caller
   owns all of them.  Aggregate a has the members arows[aptr[a] ..
   aptr[a+1]) (rows of the level, 0-based).

   Bases: W (n_level x m, row-major, 1 <= m <= 16) holds the smooth vectors on
   the level.  For every aggregate, the singular value decomposition of its
   n_a x m block (one-sided Jacobi) gives the left singular vectors whose
   singular values exceed TOL_a = tol * n_a / n_level, at least one and at
   most min(n_a, m) (Section 5: TOL = 0.1), each with its entry of largest
   magnitude (lowest row on ties) positive.  Outputs: k[a] (nagg) the number
   kept; U (n_level x m, row-major, laid out like the members: row
   aptr[a] + i holds member i's entries of u_0 .. u_{k_a - 1}, then zeros);
   dropped[a] the sum of the squared singular values not kept; flag: one int
   of scratch.  max_na bounds every n_a (max_na * m <= 8192).
   MVAMG_ERR_ARG for sizes out of range or an aggregate whose smooth vectors
   are all zero. */
mvamg_status mvamg_setup_bases(int n_level, int m, int nagg, int max_na, const int* aptr_dev,
                               const int* arows_dev, const double* W_dev, double tol, int* k_dev, double* U_dev,
                               double* dropped_dev, int* flag_dev, void* stream);

/* Coarse pattern of P^T A P, on the host (host arrays): A's pattern (rowptr,
   col), the aggregates and the widths k.  Fills agg (n: aggregate of each
   row), loc (n: the row's place among its aggregate's members), coff
   (nagg + 1: first coarse dof of each aggregate), cagg (nc = coff[nagg]:
   aggregate of each coarse dof), and *nnz (coarse nonzeros); when crp and
   ccol are not NULL, also crp (nc + 1) and ccol (*nnz, sorted rows).  The
   rows of aggregate a couple to every dof of every aggregate that A couples
   a's rows to.  MVAMG_ERR_ARG if the aggregates do not partition the rows. */
mvamg_status mvamg_setup_pattern(int n, const int* rowptr, const int* col, int nagg, const int* aptr,
                                 const int* arows, const int* k, int* agg, int* loc, int* coff, int* cagg,
                                 int* crp, int* ccol, int64_t* nnz);

/* Values of A_c = P^T A P on the pattern of mvamg_setup_pattern (all arrays
   on the device, as that call and mvamg_setup_bases produced them): each
   entry sums U_a[i][l] a_ij U_b[j][mm] over the fine entries between the two
   aggregates in a fixed order, and (A_c + A_c^T) / 2 is stored, so cval is
   exactly symmetric.  work: nnz doubles of scratch; flag: one int. */
mvamg_status mvamg_setup_galerkin(int m, int nagg, int nc, const int* aptr_dev, const int* arows_dev,
                                  const int* coff_dev, const int* agg_dev, const int* loc_dev, const int* cagg_dev,
                                  const int* rowptr_dev, const int* col_dev, const double* val_dev,
                                  const double* U_dev, const int* crp_dev, const int* ccol_dev, double* cval_dev,
                                  double* work_dev, int* flag_dev, void* stream);

/* The smooth vectors on the coarse level: Wc = P^T W (nc x m, row-major). */
mvamg_status mvamg_setup_restrict(int m, int nagg, const int* aptr_dev, const int* arows_dev, const int* coff_dev,
                                  const double* U_dev, const double* W_dev, double* Wc_dev, void* stream);

/* --------------------------------------------------------- autotuning */

enum {
  MVAMG_TUNE_GROUP_LANES = 1,   /* grouped levels: 64 / G lanes per row, G from the
                                   largest group (power of two) up to 8 */
  MVAMG_TUNE_BLOCK_COARSE = 2,  /* block path: coarsest product on vector FMA or on
                                   MFMA (wave count, inner-dimension split); allocates
                                   the block work space */
  MVAMG_TUNE_BATCH_CHUNKS = 4,  /* batch: chunks per problem of its reductions */
  MVAMG_TUNE_ALL = 7
};

/* Times the kernel variants selected by `what` on this hierarchy's own data
   (a few launches each on `stream`, which is synchronised) and keeps the
   fastest for later calls on the handle.  report (may be NULL) receives the
   measured times and the choice, truncated to cap bytes.  A different choice
   changes rounding only; results with a fixed choice repeat bitwise. */
mvamg_status mvamg_autotune(mvamg_hier* h, int what, char* report, size_t cap, void* stream);

/* The handle's current choices as text ("G1=8;gemm=4;..."), NUL-terminated;
   MVAMG_ERR_ARG if cap is too small. */
mvamg_status mvamg_tune_get(const mvamg_hier* h, char* buf, size_t cap);

/* Restores choices written by mvamg_tune_get (every value is checked before
   any is applied).  Waits for the device to be idle. */
mvamg_status mvamg_tune_set(mvamg_hier* h, const char* text);

/* Device and hierarchy signature (GPU architecture and CU count, problem
   count, level sizes and nonzeros) for keying a cache of tuning choices. */
mvamg_status mvamg_signature(const mvamg_hier* h, char* buf, size_t cap);

/* ---------------------------------------------------------- measurement */

/* Kernel classes for mvamg_kernel_stats. */
enum {
  MVAMG_KC_SMOOTH_FINE = 0,   /* smoother stages of the finest level */
  MVAMG_KC_SMOOTH_COARSE = 1, /* smoother stages of coarser levels */
  MVAMG_KC_SPMV = 2,          /* q = A p of CG (finest level) */
  MVAMG_KC_RESIDUAL = 3,      /* s = r - A x inside the cycle (all smoothed levels) */
  MVAMG_KC_RESTRICT = 4,      /* r_c = P^T s */
  MVAMG_KC_PROLONG = 5,       /* x += P x_c */
  MVAMG_KC_COARSE = 6,        /* coarsest solve (dense product with A_L^{-1}) */
  MVAMG_KC_COUNT = 7
};

/* Measurement switch (not needed for solving).  enable 1 or 2: every later
   launch of the classes above carries start/stop HIP events on its stream
   (graph replay is off meanwhile) and its algorithmic HBM bytes are booked
   to its class, each vector element touched once and each row's pointer 4
   bytes, with the matrix data counted as
     2: the plain model -- every stored entry a value (8 bytes, 4 in the
        binary32 cycle) and a 4-byte index, the coarsest inverse whole;
     1: the compact forms the kernels read -- 1-byte value codes and 2-byte
        column deltas on sliced-ELL levels, one index per shared column-list
        entry on grouped levels, the lower triangle of the coarsest inverse.
   enable 0 turns measurement off.  Calling it resets the totals.
   Errors: MVAMG_ERR_ARG for another enable. */
mvamg_status mvamg_profile(mvamg_hier* h, int enable);

/* Launch count, summed kernel time (ms) and summed algorithmic bytes of one
   kernel class since the last mvamg_profile call. */
mvamg_status mvamg_kernel_stats(mvamg_hier* h, int kclass, int64_t* launches, double* ms, double* bytes);

/* Message of the last failed call on this thread ("" if none). */
const char* mvamg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MVAMG_H */
