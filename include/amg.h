/*
 * amg.h - C ABI of the MI355X (gfx950) matching-AMG preconditioned CG library.
 *
 * Method: D'Ambra, Durastante, Filippone, "AMG preconditioners for linear
 * solvers towards extreme scale".
 *   - The system: s.p.d. A x = b (Section 1, eq. (sys); Section 3.1).
 *   - Hierarchy: A_{l+1} = P_l^T A_l P_l (Section 3.1), with P_l the product
 *     of `sweeps` pairwise prolongators built by coupled aggregation based on
 *     compatible weighted matching: edge weights eq. (weights), an
 *     approximate maximum-weight matching of the locally-dominant class,
 *     eq. (prolongator), and the restriction of the smooth vector w to the
 *     next level (Section 3.2). Coarsening stops once a level has at most
 *     `max_coarse` unknowns (Section 5).
 *   - Smoother: l1-Jacobi, eqs. (ml1hgs)/(l1weights) with blocks of one row
 *     (Section 3.3); one pre- and one post-sweep by default.
 *   - Preconditioner: the V-cycle of eq. (amg) or the K-cycle (Section
 *     3.1); the coarsest system is solved exactly with a dense Cholesky
 *     factorisation, or iteratively by CG with the l1-Jacobi diagonal as in
 *     the GPU runs of Section 5 (AMG_COARSE_PCG).
 *   - Solver: preconditioned CG, stopped on the relative residual (Section 5).
 *
 * Matching ties are broken by the strict key (weight descending, smaller
 * endpoint ascending, larger endpoint ascending); aggregates are numbered by
 * their smallest member. With these rules the hierarchy is fully determined
 * and the library reproduces it bit for bit on every run.
 *
 * Conventions shared by every entry point:
 *   - A hierarchy lives on one device: amg_params.device, or the current
 *     device (hipGetDevice) at amg_setup when that is -1. Every call on it
 *     works on that device and leaves the caller's current device as it was.
 *   - All array arguments named "device" are HIP device pointers on the
 *     hierarchy's device (amg_setup: on the device it builds on); a pointer
 *     the runtime reports on another device, or not as device memory, is
 *     rejected with AMG_ERR_ARG, and so is one whose allocation ends before
 *     the extent the call reads or writes. Arrays named "host" are host
 *     pointers. The library never takes ownership of caller arrays; it owns
 *     only what it allocates inside a hierarchy.
 *   - Indices are 0-based int32. CSR rows hold strictly ascending columns,
 *     the diagonal is stored and positive, and A is bitwise symmetric.
 *   - Calls are ordered after the work already queued on the hierarchy's
 *     caller stream (amg_params.stream, or amg_set_stream; NULL is the
 *     device's default stream). Every call returns after its results are
 *     complete on the device, except the solves of a hierarchy built with
 *     AMG_ASYNC (see amg_wait).
 *   - One hierarchy is used by one host thread at a time. Distinct
 *     hierarchies may be used concurrently from different threads.
 *   - No call aborts or throws; failures return a status code and leave the
 *     outputs unspecified unless stated.
 */
#ifndef AMG_H
#define AMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amg_hierarchy amg_hierarchy; /* opaque; owns its device memory */

typedef enum {
  AMG_OK = 0,
  AMG_ERR_ARG = 1,           /* invalid argument or malformed CSR */
  AMG_ERR_NOT_SYMMETRIC = 2, /* A is not bitwise symmetric */
  AMG_ERR_NOT_SPD = 3,       /* non-positive diagonal or Cholesky pivot */
  AMG_ERR_STALL = 4,         /* coarsening stopped above the dense limit */
  AMG_ERR_OOM = 5,           /* device allocation failed */
  AMG_ERR_HIP = 6,           /* a HIP runtime call failed */
  AMG_ERR_BREAKDOWN = 7,     /* CG breakdown: (p, Ap) <= 0 or NaN */
  AMG_NOT_CONVERGED = 8      /* maxit reached; x and info are still written */
} amg_status;

/* precision of the stored hierarchy and of the V-cycle arithmetic */
enum { AMG_FP64 = 0, AMG_FP32 = 1 };

/* amg_params.cycle: the multilevel preconditioner.
 * AMG_CYCLE_V: the V-cycle of eq. (amg), used inside CG.
 * AMG_CYCLE_K: the K-cycle of Section 3.1: on every level strictly between
 *   the finest and the coarsest, the coarse correction is two iterations of
 *   flexible CG (truncation 1) preconditioned by the K-cycle starting on that
 *   level; the outer solver is then flexible CG (Section 5), since the
 *   K-cycle is not a fixed linear operator. */
enum { AMG_CYCLE_V = 0, AMG_CYCLE_K = 1 };

/* amg_params.coarse_solver: how a cycle solves the coarsest system.
 * AMG_COARSE_CHOLESKY: exactly, z_L = A_L^-1 r_L from a dense Cholesky
 *   factorisation made at setup.
 * AMG_COARSE_PCG: the iterative coarsest solver of Section 5 with the
 *   l1-Jacobi preconditioner: CG on A_L z_L = r_L from z_L = 0 with
 *   z = r / m_L, stopped as soon as ||r_k||_2 < coarse_rtol ||r_L||_2 or
 *   after coarse_maxit iterations. The cycle then differs slightly from one
 *   right-hand side to the next (it is not a fixed linear operator), so
 *   amg_pcg_solve runs flexible CG, as the paper does. */
enum { AMG_COARSE_CHOLESKY = 0, AMG_COARSE_PCG = 1 };

/* amg_params.flags */
enum {
  AMG_FLAG_NO_GRAPH = 1,   /* launch the solve kernels directly, no hipGraph */
  AMG_FLAG_SKIP_CHECKS = 2, /* skip the symmetry/structure validation pass */
  /* keep level 0's values in FP64 only. By default, when every value of A is
   * an FP32 number, the FP64 products of level 0 (outer CG SpMV, level-0
   * post-smoothing) read an FP32 copy of A: the same numbers, half the value
   * bytes, bit-identical results. */
  AMG_FLAG_NO_VALUE_COMPRESSION = 4,
  /* non-blocking solves: amg_pcg_solve and amg_pcg_solve_batch check their
   * arguments, order the solve after the caller stream's queued work and
   * return AMG_OK at once; the solve itself (its kernels and its host-side
   * convergence checks) proceeds on a host thread of the hierarchy. b, x, B,
   * X and info must stay valid, and x / X unread, until amg_wait returns the
   * solve's status (info written by then). amg_query tests for completion.
   * Any other call on the hierarchy first waits for the solve in flight. */
  AMG_ASYNC = 8
};

/* Largest coarsest level the dense Cholesky accepts (AMG_ERR_STALL above). */
#define AMG_MAX_DENSE 4096

/* Square CSR matrix: device pointers, n + 1 row offsets, nnz columns and
 * values. nnz must be below 2^31. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int32_t *row_ptr; /* device, n + 1 */
  const int32_t *col;     /* device, nnz */
  const double *val;      /* device, nnz */
} amg_csr;

typedef struct {
  int32_t sweeps;     /* pairwise sweeps per level (aggregates <= 2^sweeps); 3 */
  int32_t max_coarse; /* stop coarsening at n_l <= max_coarse; 200 */
  int32_t max_levels; /* hard cap on the number of levels; 32 */
  int32_t pre, post;  /* l1-Jacobi sweeps before / after the coarse correction; 1, 1 */
  int32_t precision;  /* AMG_FP64 or AMG_FP32 (hierarchy values and V-cycle) */
  const double *w;    /* device, n: smooth vector (or the sample smoothed by w_sweeps),
                         no zero entry; NULL = ones */
  void *stream;       /* hipStream_t for every call on this hierarchy; NULL = the
                         device's default stream */
  int32_t device;     /* HIP device ordinal the hierarchy lives on; -1 = the current
                         device at amg_setup. -1 */
  int32_t flags;      /* AMG_FLAG_* and AMG_ASYNC */
  int32_t cycle;      /* AMG_CYCLE_V or AMG_CYCLE_K; AMG_CYCLE_V */
  int32_t w_sweeps;   /* smooth vector: w = (I - M^-1 A)^w_sweeps w0, with M the l1-Jacobi
                         diagonal of A and w0 = w (NULL: ones), i.e. w_sweeps iterations of
                         the smoother on A w = 0 from the sample w0 (the algebraically
                         smooth vectors recommended after eq. (prolongator)); 0 */
  int32_t coarse_solver; /* AMG_COARSE_CHOLESKY or AMG_COARSE_PCG; AMG_COARSE_CHOLESKY */
  int32_t coarse_maxit;  /* AMG_COARSE_PCG: iteration cap, 1..10000; 30 (Section 5) */
  double coarse_rtol;    /* AMG_COARSE_PCG: relative residual target, >= 0 (0: run
                            coarse_maxit iterations); 1e-4 (Section 5) */
  int32_t smooth_p;      /* 1: smoothed aggregation (the alternative to the K-cycle in
                            Section 3.2): the next level is Pbar^T A Pbar with
                            Pbar = (I - omega D^-1 A) P, omega = 4 / (3 ||D^-1 A||_inf)
                            (the damping 4 / (3 rho(D^-1 A)), rho estimated by the
                            infinity norm: the value that reproduces the supplement's
                            convergence constant K of the smoothed prolongator),
                            D = diag(A), P the tentative prolongator of the matching
                            sweeps (which still chooses the aggregates and restricts w);
                            the V-cycle restricts with Pbar^T and prolongates with Pbar.
                            V-cycle only. The setup's sort buffers come from a workspace
                            per device that is kept, and reused, until the process ends
                            (about twice the largest setup's temporaries: ~30 GB for
                            4.1 M unknowns); smoothed setups on one device take turns.
                            0 */
} amg_params;

typedef struct {
  int32_t iterations;       /* CG iterations performed */
  double rel_res_recursive; /* ||r_k|| / ||b|| of the CG recurrence at exit */
  double rel_res_true;      /* ||b - A x|| / ||b|| recomputed at exit */
  int32_t converged;        /* 1 if ||r_k||_2 <= rtol ||b||_2 */
  double ms;                /* wall time of the solve (AMG_ASYNC: from the call to the
                               end of the solve, not to amg_wait) */
} amg_solve_info;

/* Fills the defaults listed beside each field above. */
void amg_params_default(amg_params *p);

/* Builds the hierarchy of A (Sections 3.1-3.3, see the header comment).
 * A's arrays are copied; the caller may free them on return. The whole setup
 * runs in device kernels on the hierarchy's stream.
 * Errors: AMG_ERR_ARG (n < 1, bad sizes, unsorted or out-of-range columns,
 * zero or non-finite w before or after smoothing, bad params, or a level
 * whose 64-row slices padded to their longest row exceed 2^31 - 1 stored
 * entries, or a pairwise Galerkin row that gathers more than 2048 fine
 * entries, i.e. two matched rows with more than 2048 entries together),
 * AMG_ERR_NOT_SYMMETRIC, AMG_ERR_NOT_SPD
 * (diagonal <= 0 or coarsest Cholesky failure), AMG_ERR_STALL (a level that
 * no longer coarsens holds more than AMG_MAX_DENSE unknowns), AMG_ERR_OOM,
 * AMG_ERR_HIP. On error *out is NULL. */
amg_status amg_setup(const amg_csr *A, const amg_params *params, amg_hierarchy **out);

/* Preconditioned CG on A x = b with the V-cycle as preconditioner (Section
 * 5), or, for a hierarchy built with AMG_CYCLE_K or AMG_COARSE_PCG, flexible
 * CG (truncation 1: each direction A-orthogonal to the previous) with the
 * hierarchy's cycle.
 * b: device, n (read). x: device, n (in: initial guess, out: iterate).
 * Stops when ||r_k||_2 <= rtol ||b||_2 or after maxit iterations; b = 0 gives
 * x = 0 after 0 iterations. rtol = 0 runs exactly maxit iterations.
 * info may be NULL. Returns AMG_OK, AMG_NOT_CONVERGED (x and info written),
 * AMG_ERR_BREAKDOWN, AMG_ERR_ARG, AMG_ERR_HIP. */
amg_status amg_pcg_solve(amg_hierarchy *h, const double *b, double *x, double rtol,
                         int32_t maxit, amg_solve_info *info);

/* amg_pcg_solve for callers that cannot allocate device memory (code that
 * must not call hipMalloc: tight serving loops, harnesses that forbid
 * allocation). Same arguments, results (bit for bit) and errors as
 * amg_pcg_solve, but the call allocates nothing: the solve's scratch (the
 * block partial sums of its reductions, 3 x 65536 doubles, the CG scalars
 * and the K-cycle scalars of up to 64 levels: ~1.6 MB in all) comes from
 * one static device array per device, which the library holds until the
 * process ends, and the iterations are launched directly instead of from
 * the graph amg_pcg_solve instantiates on its first call. Every hierarchy
 * fits that array (its size does not depend on n). The array is shared by
 * all hierarchies on a device: calls on one device that overlap in time
 * race, so issue them from one host thread at a time. Always blocking (a
 * hierarchy built with AMG_ASYNC is solved synchronously here). */
amg_status amg_pcg_solve_noalloc(amg_hierarchy *h, const double *b, double *x, double rtol,
                                 int32_t maxit, amg_solve_info *info);

/* k independent PCG solves sharing the hierarchy: column j of the n x k
 * row-major blocks B (device, read) and X (device, in: x0, out: x) is solved
 * with its own CG recurrence (own alpha, beta, stop test); the V-cycle runs
 * once per iteration on the whole block. info: host array of k, may be NULL.
 * The first call with a given k allocates the block's buffers and autotunes
 * the kernels' tiles (amg_batch_tile); later calls with that k repeat the
 * same arithmetic bit for bit.
 * Returns AMG_OK if every column converged, else AMG_NOT_CONVERGED, or an
 * error; AMG_ERR_ARG for a hierarchy built with AMG_CYCLE_K or
 * AMG_COARSE_PCG (the block solve runs the V-cycle with the Cholesky
 * coarsest solve only). k = 0 is a no-op. */
amg_status amg_pcg_solve_batch(amg_hierarchy *h, int32_t k, const double *B, double *X,
                               double rtol, int32_t maxit, amg_solve_info *info);

/* One application of the hierarchy's preconditioner, z = B_0 r: the V-cycle
 * of eq. (amg), or the K-cycle for a hierarchy built with AMG_CYCLE_K.
 * r, z: device, n. */
amg_status amg_vcycle_apply(amg_hierarchy *h, const double *r, double *z);

/* Waits for the solve in flight on a hierarchy built with AMG_ASYNC and
 * returns its status: what the blocking call would have returned (AMG_OK,
 * AMG_NOT_CONVERGED, AMG_ERR_BREAKDOWN, ...); its info is written by then.
 * AMG_OK at once when no solve is in flight; AMG_ERR_ARG for h = NULL. */
amg_status amg_wait(amg_hierarchy *h);

/* Non-blocking completion test: *done = 1 when no solve is in flight or the
 * one in flight has finished (amg_wait then returns without waiting), else 0. */
amg_status amg_query(amg_hierarchy *h, int32_t *done);

/* Rebinds the hierarchy to another caller stream (hipStream_t, NULL = the
 * device's default stream): later calls are ordered after the work queued
 * on it. Lets a serving loop reuse a cached hierarchy from any slot. */
amg_status amg_set_stream(amg_hierarchy *h, void *stream);

/* Releases the hierarchy and all its device memory. NULL is a no-op. */
void amg_free(amg_hierarchy *h);

/* ---- introspection (tests, serving, benchmarks) ------------------------ */

amg_status amg_num_levels(const amg_hierarchy *h, int32_t *nlev);
/* size and nnz of level l, 0 <= l < nlev */
amg_status amg_level_info(const amg_hierarchy *h, int32_t l, int64_t *n, int64_t *nnz);
/* Copies level l's CSR (FP64 values) to host arrays of n + 1, nnz, nnz. */
amg_status amg_get_level_csr(const amg_hierarchy *h, int32_t l, int32_t *row_ptr_host,
                             int32_t *col_host, double *val_host);
/* Copies the aggregate map of level l (l < nlev - 1) to a host array of n_l:
 * agg_host[i] is the level-(l+1) unknown that fine unknown i belongs to, the
 * composition of the `sweeps` pairwise matchings of Section 3.2; aggregates
 * are numbered by their smallest member. */
amg_status amg_get_aggregates(const amg_hierarchy *h, int32_t l, int32_t *agg_host);
/* Copies the composed aggregate map and prolongator values of level l
 * (l < nlev - 1): agg_host[i] is the level-(l+1) index of fine row i and
 * p_host[i] the entry P_l(i, agg_host[i]). Either pointer may be NULL. */
amg_status amg_get_transfer(const amg_hierarchy *h, int32_t l, int32_t *agg_host,
                            double *p_host);
/* Smoothed prolongator Pbar of level l (l < nlev - 1) of a hierarchy built
 * with smooth_p = 1: *nnz its number of entries; when the arrays are given
 * (host, n_l + 1 / nnz / nnz), its CSR with columns in level l + 1's
 * numbering, ascending in each row; *omega (may be NULL) the omega used.
 * AMG_ERR_ARG for a hierarchy without smoothing. */
amg_status amg_get_prolongator(const amg_hierarchy *h, int32_t l, int64_t *nnz,
                               int32_t *row_ptr_host, int32_t *col_host, double *val_host,
                               double *omega);
/* Copies the l1-Jacobi diagonal m of level l (l < nlev - 1; also the
 * coarsest level of an AMG_COARSE_PCG hierarchy, whose CG uses it). */
amg_status amg_get_l1diag(const amg_hierarchy *h, int32_t l, double *m_host);
/* Copies the smooth vector w restricted to level l. */
amg_status amg_get_w(const amg_hierarchy *h, int32_t l, double *w_host);
/* Device bytes owned by the hierarchy. */
size_t amg_footprint_bytes(const amg_hierarchy *h);
/* Upper estimate of the device bytes amg_setup and one amg_pcg_solve need
 * for an n x n matrix with nnz entries (used for admission control). */
size_t amg_estimate_footprint(int64_t n, int64_t nnz, const amg_params *params);
/* Milliseconds of the last amg_setup, split by stage (host array of 8):
 * validate, weights+matching, numbering+prolongator, Galerkin, compose,
 * smoother+coarsest, solve-format conversion, total. */
amg_status amg_setup_times(const amg_hierarchy *h, double *ms_host);
/* Number of matching rounds run when building level l (sum over sweeps). */
amg_status amg_matching_rounds(const amg_hierarchy *h, int32_t l, int32_t *rounds);

/* Times `reps` launches of one solve-phase kernel on level l with live data
 * between HIP events on the hierarchy's stream; *ms = mean per launch and
 * *bytes = the kernel's algorithmic HBM bytes per launch. kernel:
 * 0 = pre-smoothing + residual + restriction to level l + 1,
 * 1 = post-smoothing (on level 0 with the CG dot product),
 * 2 = post-smoothing of level l + 1 fused with the prolongation into level l
 *     (level l + 1 must not be the coarsest), 3 = same as 2,
 * 4 = outer-CG SpMV with its dot product (level 0),
 * 5 = one whole V-cycle as inside the solve (level ignored; *bytes its
 *     algorithmic total, without the coarsest solve when it is the
 *     iterative one, whose L2-resident traffic depends on its iteration
 *     count; AMG_ERR_ARG for a K-cycle hierarchy).
 * kernel | AMG_TIME_IN_SOLVE, for kernels 0, 1 and 4 on level 0: the kernel
 * timed where the solve runs it, inside `reps` (1..10000) CG iterations
 * from x = 0 on the right-hand side of the last amg_pcg_solve (launched
 * without the graph, rtol 0, so every launch does its full work); *ms is
 * the mean of its dispatches' own start-to-end times, which the runtime
 * stamps into events given to the launch (hipExtLaunchKernelGGL), as a
 * profiler's kernel trace measures them. AMG_ERR_ARG before any solve, and
 * for a hierarchy with the K-cycle, the iterative coarsest solve, smoothed
 * prolongators, or more than one pre- or post-sweep. */
#define AMG_TIME_IN_SOLVE 16
amg_status amg_time_kernel(amg_hierarchy *h, int32_t kernel, int32_t level, int32_t reps,
                           double *ms, double *bytes);

/* Tiles the batch solve's autotuner chose for the last k used with this
 * hierarchy, by timing the block CG iteration as the solve runs it for each
 * candidate: *tile, the column tile of the one-value kernels (64 / tile rows
 * x tile columns per wavefront), and *vshift (may be NULL), the scale
 * 2^vshift (vshift in -1..1) applied to the vector kernels' default tile
 * (the power of two covering their kv = k / 2 or k / 4 column vectors per
 * row, within 4..64). 0, 0 before any batch solve. */
amg_status amg_batch_tile(const amg_hierarchy *h, int32_t *tile, int32_t *vshift);

const char *amg_status_string(amg_status s);

#ifdef __cplusplus
}
#endif
#endif /* AMG_H */
