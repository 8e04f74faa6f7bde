/*
 * nfield.h - C ABI of the MI355X (gfx950) n-field block solver.
 *
 * The library solves the N x N block-sparse linear system of a monolithic
 * coupled problem,
 *
 *     [A_11 ... A_1N] [x_1]   [b_1]
 *     [ ...  ...  ...] [...] = [...]        (paper: Sec. 4, the blocked system;
 *     [A_N1 ... A_NN] [x_N]   [b_N]         some blocks may be zero)
 *
 * with restarted GMRES preconditioned from the right (Sec. 3.2: solve
 * (A P) y = b, then x = P y), where the preconditioner P ~ A^-1 is one of the
 * paper's block methods (Sec. 4) or a nesting of them (Sec. 5):
 *
 *   "BGS(AMG)"              block Gauss-Seidel (Sec. 4.1) with one
 *                           smoothed-aggregation AMG V-cycle (Sec. 3.3,
 *                           Algorithm 1) per diagonal block;
 *   "SIMPLE(AMG)"           SIMPLE / SIMPLEC (Sec. 4.2);
 *   "SIMPLE(BGS(AMG);AMG)"  n-field SIMPLE with merged predictor fields
 *                           (Sec. 4.2, block merging) and an AMG on the
 *                           approximate Schur complement;
 *   "AMG(BGS)", "AMG(SIMPLE)"  monolithic AMG (Sec. 4.3): block-diagonal
 *                           transfers, coarse blocks R_i A_ij P_j, BGS or
 *                           SIMPLE level smoothers (SIMPLE: the last field is
 *                           the Schur field and is not coarsened, P = I; its
 *                           S~ on every level is inverted densely up to
 *                           schur_direct_max, else smoothed by Chebyshev);
 *   "LU"                    dense direct solve (Gauss-Jordan inverse with
 *                           partial pivoting, up to 12000 unknowns; a
 *                           symmetric definite matrix is inverted without
 *                           row exchanges).
 * Optional per-method parameters: "BGS[sweeps=2,order=bwd](AMG)" (sweeps and
 * order of one BGS / SIMPLE node), "AMG[degree=1]" (Chebyshev smoother degree
 * of one hierarchy; degree 1 is damped Jacobi), "AMG[smoother=sgs,omega=0.69,
 * steps=1]" (symmetric multicolour Gauss-Seidel with damping omega instead of
 * Chebyshev, in the spirit of the damped Gauss-Seidel smoothers of Sec. 7;
 * "half=1": pre-smoothing sweeps the colours forward only, post-smoothing
 * backward only, instead of both sweeping forward then backward;
 * "cheb_from=L", L >= 1: levels L and coarser use the Chebyshev smoother of
 * the hierarchy's degree instead, Gauss-Seidel stays on the finer levels),
 * "AMG[smoother=ddgs,omega=0.79]" (the paper's DD(GS) smoother of Sec. 7:
 * Gauss-Seidel inside subdomains coupled additively; the subdomains are the
 * level's aggregates, relaxed in colour order, one workgroup each),
 * "AMG[pg=1]" (Petrov-Galerkin transfers for nonsymmetric fields, the
 * paper's fluid AMG of Sec. 7 after Sala and Tuminaro: P = P_tent -
 * D^-1 A P_tent diag(omega) with column dampings minimising ||A P e_j||_2,
 * R from the same construction on A^T, coarse blocks R_i A_ij P_j).  A
 * single-level block solve: "DDGS[omega=0.79,steps=1]" (DD(GS) sweeps from
 * a zero guess, the paper's BGS(DD(GS)) comparison).
 *
 * All device work runs in the library's own HIP kernels for gfx950, enqueued
 * on the caller's stream (setup and rebuild may also use streams of the
 * library's own for independent parts, ordered after the caller's stream and
 * before its later work; see parallel_setup).  Every vector argument named *_dev is a device
 * pointer owned by the caller (for instance a torch tensor), FP64, holding
 * nrhs columns of length n = sum_i ndof_i one after the other (column-major
 * n x nrhs), each column in global field order [x_1; ...; x_N].
 *
 * Return codes: 0 = OK; NFIELD_NOT_CONVERGED (> 0) is soft (x holds the last
 * iterate and stats are valid); negative values are hard errors (outputs
 * undefined; a context being created is not returned).  nfield_last_error()
 * gives a message for the last error of the calling thread.  A context is not
 * thread-safe; distinct contexts are independent.
 */
#ifndef NFIELD_H
#define NFIELD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NFIELD_OK = 0,
  NFIELD_NOT_CONVERGED = 1,
  NFIELD_EINVAL = -1,      /* malformed input: CSR not sorted/unique/in range, sizes, spec */
  NFIELD_ENOMEM = -2,      /* device allocation failed or a size limit was exceeded */
  NFIELD_ESINGULAR = -3,   /* zero diagonal block / entry where a method needs one, zero LU pivot */
  NFIELD_EBREAKDOWN = -4,  /* Krylov breakdown that is not a converged solution */
  NFIELD_ENAN = -5,        /* non-finite value in the right-hand side or the iteration */
  NFIELD_EHIP = -6         /* a HIP runtime call failed */
} nfield_status;

typedef struct nfield_ctx nfield_ctx;   /* opaque; owns all device state of one system */

/* One block A_ij in CSR form, host memory, FP64.  Column indices must be
 * strictly increasing within each row.  nnz == 0 or val == NULL marks a zero
 * block.  Copied by nfield_setup; the caller may free it on return. */
typedef struct {
  int32_t nrows, ncols;
  int64_t nnz;
  const int64_t *rowptr;   /* nrows + 1 */
  const int32_t *colind;   /* nnz */
  const double *val;       /* nnz */
} nfield_csr;

/* One physical field.  Its dofs are grouped in nodes of block_size
 * consecutive dofs (ndof % block_size == 0).  nullspace holds nns
 * near-nullspace vectors (rigid-body modes, constants, unit vectors) as
 * nns rows of ndof values (ndof x nns column-major), host memory, copied. */
typedef struct {
  int32_t ndof, block_size, nns;
  const double *nullspace;
} nfield_field;

/* Setup options.  Zero-initialise and call nfield_default_opts() first. */
typedef struct {
  int32_t sweeps;          /* BGS sweeps k_max (Sec. 4.1); default 1 */
  int32_t order;           /* BGS order: 0 forward, 1 backward, 2 symmetric; default 1 */
  int32_t coarse_max;      /* stop coarsening at <= this many dofs; dense LU there; 200 */
  int32_t max_levels;      /* AMG level limit; 10 */
  int32_t cheb_degree;     /* Chebyshev polynomial degree of the smoother; 2 */
  int32_t power_its;       /* power iterations for lambda_max(D^-1 A); 10 */
  double cheb_ratio;       /* smoothing interval [lambda/ratio, boost*lambda]; 30 */
  double cheb_boost;       /* 1.1 */
  int32_t simplec_mode;    /* SIMPLE diagonal: 0 sum_j|a_ij|, 1 |sum_j a_ij|, 2 a_ii; 0 */
  const int32_t *split;    /* field -> SIMPLE group (0 predictor, 1 Schur); NULL: last field */
  int32_t schur_direct_max;/* Schur complements up to this size are inverted densely; 5000 */
  int32_t hier_fp32;       /* 1: store and run the AMG hierarchies in FP32 (precision form).
                              The FP32 tree keeps FP32 copies of the input blocks it reads;
                              the input blocks' FP64 values are then released (the merged
                              FP64 operator of GMRES holds the same values) and gathered
                              back from it at each rebuild, so a rebuild briefly holds
                              them again. */
  uint64_t seed;           /* MIS-2 keys and power-iteration start vectors */
  int32_t graphs;          /* 1: the preconditioner's kernels are captured once (per column
                              count, after every rebuild) into a HIP graph and replayed;
                              0 (default): launched one by one.  Same bits either way; on
                              gfx950 / ROCm 7.2 replay did not shorten the solve. */
  int32_t block_products;  /* 1 (default): Galerkin products of node-blocked fields are
                              formed block by block (one hash insert per block pair);
                              0: entry by entry.  Same pattern and bits either way. */
  int32_t parallel_setup;  /* 1 (default): independent parts of the preconditioner (the
                              fields of BGS, the predictor and Schur parts of SIMPLE)
                              are set up concurrently, each on a host thread and HIP
                              stream of the library's own that first waits for the
                              caller's stream (which then waits for them); 0: one after
                              another on the caller's stream.  Same bits either way. */
  int32_t max_rhs;         /* right-hand sides one launch sequence handles (1..8; default 8):
                              the preconditioner's temporaries and the Krylov workspace
                              hold this many columns; calls with more columns run in
                              batches of max_rhs.  1 for single right-hand-side use keeps
                              the context small. */
} nfield_opts;

typedef struct {
  int32_t restart;         /* GMRES restart length m; 50 */
  int32_t maxit;           /* total Arnoldi steps allowed; 1000 */
  int32_t flexible;        /* 1: flexible GMRES (stores Z = M V); required with hier_fp32 */
  double rtol;             /* stop when ||b - A x||_2 / ||b - A x0||_2 < rtol; 1e-8 */
} nfield_solve_opts;

typedef struct {
  int32_t iters, restarts, status;
  double relres;           /* final true relative residual */
  double setup_s, solve_s; /* wall seconds of the last setup / rebuild and of this solve */
  double bytes;            /* algorithmic HBM bytes of the solve's launches (every operand
                              once per launch: matrix entries and indices, the vectors read
                              and written; a Gauss-Seidel sweep's operand once per sweep).
                              The columns of one batch of up to 8 share their launches: each
                              column reports the batch's bytes. */
  double gbps;             /* bytes / solve_s, in GB/s (1e9 bytes per second) */
} nfield_stats;

void nfield_default_opts(nfield_opts *opts);
void nfield_default_solve_opts(nfield_solve_opts *sopts);

/* Build the preconditioner for the system: upload every block, parse spec,
 * build the AMG hierarchies (node graph, MIS-2 aggregation, tentative and
 * smoothed prolongators, Galerkin products, smoothers, coarse LU) on the
 * device.  hip_stream may be NULL (default stream).  Returns after the device
 * work has finished.  Errors: EINVAL for
 * malformed CSR, block shapes that disagree with fields[i].ndof, or a bad
 * spec; ESINGULAR for BGS / AMG on a zero diagonal block or entry, or a
 * zero coarse pivot; ENOMEM; EHIP. */
nfield_status nfield_setup(int32_t nfields, const nfield_field *fields,
                           const nfield_csr *blocks /* nfields*nfields, row-major (i,j) */,
                           const char *spec, const nfield_opts *opts, void *hip_stream,
                           nfield_ctx **out);

/* z = P r for nrhs columns (the preconditioner as an operator, Sec. 3.2).
 * r_dev and z_dev must not overlap. */
nfield_status nfield_precond_apply(nfield_ctx *ctx, const double *r_dev, double *z_dev,
                                   int32_t nrhs, void *hip_stream);

/* y = A x for nrhs columns (every nonzero block). */
nfield_status nfield_matvec(nfield_ctx *ctx, const double *x_dev, double *y_dev, int32_t nrhs,
                            void *hip_stream);

/* Solve A x = b with right-preconditioned (or flexible) GMRES(m) per column.
 * x_dev holds the initial guess on entry and the solution on return.  stats
 * (nrhs entries, may be NULL) receives per-column results.  The call returns
 * after the solve has finished on the device.  Per column: OK when the true
 * relative residual is below rtol; NOT_CONVERGED at maxit; EBREAKDOWN when
 * the Arnoldi process broke down (||w|| <= 1e-300 after orthogonalisation:
 * an invariant Krylov space) and the true residual still fails the test,
 * where a restart would rebuild the same space (x holds the last iterate);
 * ENAN for a non-finite right-hand side or iterate.  The return value is
 * the worst column status (any negative one first). */
nfield_status nfield_gmres_solve(nfield_ctx *ctx, const double *b_dev, double *x_dev,
                                 int32_t nrhs, const nfield_solve_opts *sopts,
                                 nfield_stats *stats, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as nfield_gmres_solve (same kernels in the same order, so the same
 * results bit for bit), with its Krylov workspace (basis V, flexible basis
 * Z, Hessenberg and rotation arrays, reduction partials, the FP32 staging of
 * the precision form) in a static device array of 256 MiB per device
 * instead of buffers of the context, and its host staging in the call's own
 * pageable arrays.  It calls no hipMalloc / hipFree / hipHostMalloc and no
 * allocating routine; the preconditioner is launched directly (no graph
 * replay).  The workspace takes about 8 n ((m + 1) + m (flexible) + 4)
 * min(nrhs, 8) bytes (+ 4 n min(nrhs, 8) with hier_fp32); a call whose
 * workspace exceeds 256 MiB returns NFIELD_ENOMEM before any device work.
 * Every call on one device shares that device's array, which keeps the last
 * call's contents: calls that overlap on one device (from several threads
 * or streams) race and must be serialised by the caller. */
nfield_status nfield_gmres_solve_noalloc(nfield_ctx *ctx, const double *b_dev, double *x_dev,
                                         int32_t nrhs, const nfield_solve_opts *sopts,
                                         nfield_stats *stats, void *hip_stream);

/* ---- slot batches: iteration-level continuous batching of GMRES columns.
 * A batch holds `slots` columns (1 <= slots <= the context's max_rhs), each
 * running the restarted GMRES of nfield_gmres_solve (Sec. 3.2) on its own
 * right-hand side: the same kernels act on each column, so a column's
 * solution and statistics are those of nfield_gmres_solve of that column
 * alone, bit for bit.  nfield_batch_step advances every running column by
 * one Arnoldi step in shared launches; between steps the caller submits new
 * right-hand sides into free slots and takes finished ones out, so columns
 * join and leave a running batch at its Arnoldi step boundaries.  A
 * column's Krylov cycle ends as in nfield_gmres_solve (estimate below rtol,
 * breakdown, maxit or m steps); the step after, its solution is updated and
 * its true residual tested, and it finishes (stats as nfield_gmres_solve's,
 * with solve_s the wall time from submission, bytes and gbps 0) or starts
 * the next cycle in the same step.  The batch owns about 8 n slots
 * ((m + 1) + 6 + (m if flexible, else 1)) bytes of device memory, taken
 * from its context's cache (and counted in nfield_footprint_bytes);
 * it uses the context's preconditioner and must be destroyed before it.
 * Calls on one batch, and solves on its context, must not overlap (one
 * stream or host thread at a time); every call is enqueued on hip_stream. */
typedef struct nfield_batch nfield_batch;   /* opaque */

/* Create a batch of `slots` free slots with the solve options sopts (NULL:
 * defaults).  EINVAL for slots outside [1, max_rhs] or bad options. */
nfield_status nfield_batch_create(nfield_ctx *ctx, int32_t slots, const nfield_solve_opts *sopts,
                                  nfield_batch **out);
/* Put a right-hand side (device, n doubles, copied) into a free slot, with
 * the initial guess x0_dev (device, n doubles, copied; NULL: zero).  The
 * column joins at the next step.  EINVAL if the slot is not free. */
nfield_status nfield_batch_submit(nfield_batch *batch, int32_t slot, const double *b_dev,
                                  const double *x0_dev, void *hip_stream);
/* One step: cycle ends, true-residual tests and cycle starts of the columns
 * that need them, then one Arnoldi step of every running column.  The
 * slots that finished in this step are written to done (up to `slots`
 * entries, may be NULL) and counted in *ndone; *nactive receives the
 * number of slots still working.  Returns after the step has finished on
 * the device. */
nfield_status nfield_batch_step(nfield_batch *batch, int32_t *done, int32_t *ndone,
                                int32_t *nactive, void *hip_stream);
/* Copy a finished slot's solution to x_dev (device, n doubles, may be
 * NULL), its statistics to *stats (may be NULL), and free the slot.  EINVAL
 * if the slot has not finished. */
nfield_status nfield_batch_take(nfield_batch *batch, int32_t slot, double *x_dev,
                                nfield_stats *stats, void *hip_stream);
/* 0 free, 1 waiting for its true residual, 2 in an Arnoldi cycle, 3 cycle
 * ended, 4 finished (take it); -1 for a bad argument. */
int32_t nfield_batch_state(const nfield_batch *batch, int32_t slot);
/* Device bytes the batch holds. */
size_t nfield_batch_bytes(const nfield_batch *batch);
void nfield_batch_destroy(nfield_batch *batch);

/* Replace the values of the nonzero block (i, j), keeping its pattern (the
 * next Newton step of the paper's monolithic scheme, Sec. 2).  val holds the
 * block's nnz values in its CSR order, in device memory (on_device = 1,
 * enqueued on hip_stream) or host memory (copied before return).  The
 * preconditioner keeps using the old values until nfield_rebuild. */
nfield_status nfield_update_values(nfield_ctx *ctx, int32_t i, int32_t j, const double *val,
                                   int32_t on_device, void *hip_stream);

/* Rebuild the whole preconditioner (hierarchies, smoothers, Schur
 * complements, coarse inverses) from the device-resident blocks. */
nfield_status nfield_rebuild(nfield_ctx *ctx, void *hip_stream);

/* Launch timing of the SpMV kernels (HIP events on the launch stream).
 * nfield_prof_enable(1) clears and starts recording, 0 stops.  prof_read
 * returns the number of kernel variants and fills up to max entries: key =
 * ((16*lanes_per_row + rows_per_node_group)*100 + kind)*10 + (1 if FP32),
 * kind 0-5 = SpMV epilogue (store, residual, add, subtract, Chebyshev step,
 * diagonal scaling); Gauss-Seidel sweeps (timed per sweep): 6 = a launch per
 * colour, one lane group per node; 7 = every colour in one single-workgroup
 * launch (tiny levels with many colours); 8 = a launch per colour, one
 * workgroup per node (long rows); 9 = the whole symmetric sweep of a small
 * many-colour level as one dense affine map x <- S x + Q b; 10 = a DD(GS)
 * sweep (one workgroup per subdomain); 11 = a launch per colour from the
 * block copy of a level made of dense 2 x 2 or 3 x 3 node blocks.  For
 * kinds 0-3 and 11 from a block copy, rows_per_node_group is the block
 * size.  Launches, total milliseconds, total
 * algorithmic bytes (matrix once, operand once, epilogue streams). */
void nfield_prof_enable(int32_t on);
int32_t nfield_prof_read(int32_t max, int32_t *key, int64_t *count, double *ms, double *bytes);

/* Device bytes the context holds: its buffers plus the blocks it keeps
 * cached for reuse by later calls (temporaries of a rebuild return there
 * instead of being freed). */
size_t nfield_footprint_bytes(const nfield_ctx *ctx);
/* Device bytes the preconditioner itself holds after the last setup or
 * rebuild: hierarchies (coarse blocks, transfers), smoother data, Schur
 * approximations, coarse inverses, FP32 copies of the input blocks that an
 * FP32 solver reads (precision form) and the preconditioner's temporaries;
 * not the input blocks (nor the FP64 input values the precision form
 * releases), the Krylov workspace or the cache. */
size_t nfield_precond_bytes(const nfield_ctx *ctx);
int64_t nfield_size(const nfield_ctx *ctx);             /* n = sum of field sizes */
void nfield_destroy(nfield_ctx *ctx);
const char *nfield_strerror(nfield_status s);
const char *nfield_last_error(void);

/* ---- inspection of the AMG hierarchies a context built (build order) ----
 * Copies to host; for tests and reports.  h indexes the hierarchies, l the
 * level, f / i / j the field(s) of a (monolithic) hierarchy. */
int32_t nfield_hier_count(const nfield_ctx *ctx);
int32_t nfield_hier_nlevels(const nfield_ctx *ctx, int32_t h);
int32_t nfield_hier_nfields(const nfield_ctx *ctx, int32_t h);
int32_t nfield_hier_size(const nfield_ctx *ctx, int32_t h, int32_t l, int32_t f);
double nfield_hier_lambda(const nfield_ctx *ctx, int32_t h, int32_t l, int32_t f);
/* which: 0 = A_ij, 1 = P_i, 2 = R_i.  Returns nnz, or -1 if absent; the
 * arrays (host, may be NULL) receive the CSR. */
int64_t nfield_hier_matrix(const nfield_ctx *ctx, int32_t h, int32_t l, int32_t which, int32_t i,
                           int32_t j, int64_t *rowptr, int32_t *colind, double *val,
                           int32_t *nrows, int32_t *ncols);
/* aggregate number of every node of field f on level l; returns the node count or -1 */
int32_t nfield_hier_aggregates(const nfield_ctx *ctx, int32_t h, int32_t l, int32_t f,
                               int32_t *agg);
/* stored entries of every block of level l of hierarchy h (-1 if absent) */
int64_t nfield_hier_nnz(const nfield_ctx *ctx, int32_t h, int32_t l);
/* operator complexity sum_l nnz(A^l) / nnz(A^0) and grid complexity
 * sum_l n^l / n^0 of hierarchy h (0 if absent) */
double nfield_hier_op_complexity(const nfield_ctx *ctx, int32_t h);
double nfield_hier_grid_complexity(const nfield_ctx *ctx, int32_t h);

/* Residual history of the last nfield_gmres_solve call, column col: the
 * relative residual estimate |g_{j+1}| / ||r_0|| after every Arnoldi step
 * (host copies).  Returns the number of steps (filling at most max values of
 * out, which may be NULL), or -1 for a column the last call did not have. */
int32_t nfield_residual_history(const nfield_ctx *ctx, int32_t col, double *out, int32_t max);

#ifdef __cplusplus
}
#endif
#endif /* NFIELD_H */
