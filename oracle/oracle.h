/*
 * Plain FP64 CPU oracle for matching-based AMG-preconditioned CG.
 *
 * TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library. The GPU library never calls
 * it and shares no code with it.
 *
 * Method: D'Ambra, Durastante, Filippone, "AMG preconditioners for linear
 * solvers towards extreme scale":
 *   Section 3.1        Galerkin hierarchy and the V-cycle, eq. (amg)
 *   Section 3.2        coarsening by compatible weighted matching:
 *                      eq. (weights), eq. (prolongator), multi-sweep
 *                      composition, restriction of the smooth vector w
 *   Section 3.3        l1-Jacobi smoother, eqs. (ml1hgs)/(l1weights), nb = 1
 *   Section 5          CG-type outer solver, relative residual stop,
 *                      coarsest-size stop rule
 * The coarsest level is solved by a dense Cholesky factorisation.
 *
 * Every function is pinned by tests against values the paper prints, closed
 * forms, dense or library computations or brute force. One printed figure is
 * not reproduced: the operator complexity of the smoothed-prolongator
 * hierarchy in Section 5 (80^3); for that figure parity is unpinned, while
 * the smoothed hierarchy itself is pinned (dense products and the
 * supplement's convergence constant for the smoothed prolongator).
 *
 * Arithmetic: IEEE binary64, round to nearest, compiled with
 * -ffp-contract=off; every sum runs left to right starting from its first
 * term, in the order each function states.
 */
#ifndef AMG_ORACLE_H
#define AMG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes (same meanings as the GPU library's) */
enum {
  ORC_OK = 0,
  ORC_ERR_ARG = 1,
  ORC_ERR_NOT_SYMMETRIC = 2,
  ORC_ERR_NOT_SPD = 3,
  ORC_ERR_STALL = 4,
  ORC_ERR_OOM = 5,
  ORC_ERR_BREAKDOWN = 7,
  ORC_NOT_CONVERGED = 8
};

/* 0-based CSR, columns strictly ascending in each row, diagonal stored. */
typedef struct {
  int32_t n;
  int64_t nnz;
  int32_t *rp;  /* n + 1 */
  int32_t *ci;  /* nnz */
  double *val;  /* nnz */
} orc_csr;

/* ---- single steps (exposed for tests) ---------------------------------- */

/* y = A x, each row summed over ascending columns. */
void orc_spmv(const orc_csr *A, const double *x, double *y);

/* Checks the structural preconditions: ascending columns in range, diagonal
 * present and positive, A bitwise symmetric. Returns a status code. */
int orc_check(const orc_csr *A);

/* Number of undirected edges = stored entries with column > row. */
int64_t orc_num_edges(const orc_csr *A);

/* eq. (weights): for every stored entry (lo, hi) with lo < hi, taken from
 * row lo, c = 1 - num/den with num = ((2 a) w_lo) w_hi and
 * den = (a_lolo w_lo) w_lo + (a_hihi w_hi) w_hi. Edges are emitted in row
 * order of lo, then ascending hi. */
void orc_edge_weights(const orc_csr *A, const double *w,
                      int32_t *lo, int32_t *hi, double *c);

/* Greedy matching under the strict order (c descending, lo ascending,
 * hi ascending): scan edges in that order, take an edge whose ends are both
 * free. mate[v] = partner or -1. Returns the number of matched edges. */
int64_t orc_greedy_matching(int32_t n, int64_t ne, const int32_t *lo,
                            const int32_t *hi, const double *c, int32_t *mate);

/* Aggregate numbering: scan v = 0..n-1; a v not yet numbered gets the next
 * id and so does its mate. Returns n_c. */
int32_t orc_number_aggregates(int32_t n, const int32_t *mate, int32_t *agg);

/* eq. (prolongator) for one pairwise sweep: pair {i<j}:
 * p_v = w_v / sqrt(w_i w_i + w_j w_j); singleton: p_s = w_s / |w_s|. */
void orc_pairwise_prolongator(int32_t n, const int32_t *mate, const double *w,
                              double *p);

/* vc = P^T v for P with one entry p[i] in row i, column agg[i]: each vc[I]
 * sums p[i] v[i] over members i of I in ascending i. */
void orc_restrict(int32_t n, int32_t nc, const int32_t *agg, const double *p,
                  const double *v, double *vc);

/* Galerkin product Ac = P^T A P for a pairwise P (aggregates of <= 2).
 * Entry (I, J) sums the terms (p_lo a_lo,hi) p_hi over stored fine entries
 * (i in I, j in J), each mapped to (lo, hi) = (min, max), a read from row lo,
 * terms sorted by (lo, hi). Every structural entry is kept. Ac's arrays are
 * allocated here (free with orc_csr_free). */
int orc_galerkin_pairwise(const orc_csr *A, int32_t nc, const int32_t *agg,
                          const double *p, orc_csr *Ac);

void orc_csr_free(orc_csr *A);

/* Smoothed aggregation (the alternative to the K-cycle in Section 3.2):
 * omega = 4 / (3 ||D^-1 A||_inf) with D = diag(A) (the damping that reproduces
 * the supplement's smoothed-prolongator convergence constant); the smoothed prolongator
 * Pbar = (I - omega D^-1 A) P of the tentative P given as (agg, p), with nc
 * columns (row order and sums as stated in oracle.c); and the Galerkin
 * product A_c = Pbar^T A Pbar (lower triangle mirrored from the upper). */
double orc_smoothing_omega(const orc_csr *A);
int orc_smooth_prolongator(const orc_csr *A, int32_t nc, const int32_t *agg, const double *p,
                           double omega, orc_csr *Pb);
int orc_galerkin_general(const orc_csr *A, const orc_csr *Pb, int32_t nc, orc_csr *Ac);

/* l1-Jacobi diagonal, eq. (l1weights) with nb = 1:
 * m_i = a_ii + (sum over j != i, ascending, of |a_ij|). */
void orc_l1_diag(const orc_csr *A, double *m);

/* nu l1-Jacobi iterations on A w = 0 from the sample w (in place): an
 * algebraically smooth vector for the matching weights. */
void orc_smooth_w(const orc_csr *A, int32_t nu, double *w);
/* Dense Cholesky A = L L^T of a row-major n x n s.p.d. matrix, in place
 * (lower triangle holds L, upper is zeroed). Returns ORC_ERR_NOT_SPD on a
 * non-positive pivot. */
int orc_cholesky(int32_t n, double *a);
/* z = L^-T L^-1 r by forward then backward substitution. */
void orc_cholesky_solve(int32_t n, const double *L, const double *r, double *z);
/* The iterative coarsest solver of Section 5 with the l1-Jacobi
 * preconditioner of the GPU runs: CG on A x = b from x = 0, preconditioned
 * by the diagonal m (z = r / m), stopped as soon as ||r_k||_2 < rtol ||b||_2
 * or after maxit iterations. Returns the number of iterations (0 for b = 0,
 * which gives x = 0). */
int32_t orc_coarse_pcg(const orc_csr *A, const double *m, const double *b, double rtol,
                       int32_t maxit, double *x);

/* ---- hierarchy ------------------------------------------------------------ */

typedef struct orc_hier orc_hier;

/* Builds the hierarchy (see oracle.c for the level loop). w0 may be NULL
 * (all ones). The input matrix is copied. */
int orc_setup(const orc_csr *A, const double *w0, int32_t sweeps,
              int32_t max_coarse, int32_t max_levels, orc_hier **out);
/* As orc_setup; smooth = 1 builds every next level with the smoothed
 * prolongator Pbar_l instead of the tentative P_l (which still chooses the
 * aggregates and restricts w), and the cycles restrict with Pbar^T and
 * prolongate with Pbar. */
int orc_setup_opts(const orc_csr *A, const double *w0, int32_t sweeps, int32_t max_coarse,
                   int32_t max_levels, int32_t smooth, orc_hier **out);
void orc_free(orc_hier *h);

int32_t orc_num_levels(const orc_hier *h);
/* level l: size, nnz, and copies of its arrays (caller-allocated). */
int64_t orc_level_n(const orc_hier *h, int32_t l);
int64_t orc_level_nnz(const orc_hier *h, int32_t l);
void orc_level_csr(const orc_hier *h, int32_t l, int32_t *rp, int32_t *ci,
                   double *val);
/* composed aggregate map and prolongator values of level l (l < nlev-1) */
void orc_level_transfer(const orc_hier *h, int32_t l, int32_t *agg, double *p);
void orc_level_l1diag(const orc_hier *h, int32_t l, double *m);
void orc_level_w(const orc_hier *h, int32_t l, double *w);
/* number of pairwise sweeps actually run when building level l+1 */
int32_t orc_level_sweeps(const orc_hier *h, int32_t l);
/* smoothed prolongator of level l (smooth hierarchies): nnz, CSR copy
 * (n_l + 1 offsets), and its omega */
int64_t orc_level_pbar_nnz(const orc_hier *h, int32_t l);
void orc_level_pbar(const orc_hier *h, int32_t l, int32_t *rp, int32_t *ci, double *val);
double orc_level_omega(const orc_hier *h, int32_t l);
/* coarsest Cholesky factor, row-major n_L x n_L */
void orc_coarse_factor(const orc_hier *h, double *L);
/* Coarsest solver of the hierarchy's cycles: solver 0 applies the dense
 * Cholesky factor (the default), solver 1 runs orc_coarse_pcg with the
 * coarsest level's l1-Jacobi diagonal, rtol and maxit. */
void orc_set_coarse_solver(orc_hier *h, int32_t solver, double rtol, int32_t maxit);

/* One V-cycle z = B_l r on level l, eq. (amg) with pre/post l1-Jacobi. */
void orc_vcycle(const orc_hier *h, int32_t l, int32_t pre, int32_t post,
                const double *r, double *z);

/* Preconditioned CG on A_0 with the V-cycle as preconditioner.
 * x holds x0 on entry, the iterate on exit. Stops when
 * ||r_k||_2 <= rtol ||b||_2 (recursive residual) or after maxit iterations.
 * out[0] = iterations, out[1] = converged (0/1), out[2] = recursive
 * relative residual, out[3] = true relative residual ||b - A x|| / ||b||. */
int orc_pcg(const orc_hier *h, int32_t pre, int32_t post, const double *b,
            double *x, double rtol, int32_t maxit, double *out);
/* K-cycle on level l (Section 3.1): as orc_vcycle, with the coarse
 * correction on every level other than the finest and the coarsest given by
 * two flexible-CG iterations preconditioned by the K-cycle on that level. */
void orc_kcycle(const orc_hier *h, int32_t l, int32_t pre, int32_t post,
                const double *r, double *z);
/* The two flexible-CG iterations of the K-cycle on level m, from x = 0. */
void orc_fcg2(const orc_hier *h, int32_t m, int32_t pre, int32_t post, const double *b,
              double *x);
/* Flexible CG (truncation 1) with the V-cycle (kcycle = 0) or K-cycle (1)
 * as preconditioner; arguments and outputs as orc_pcg. */
int orc_fcg(const orc_hier *h, int32_t kcycle, int32_t pre, int32_t post, const double *b,
            double *x, double rtol, int32_t maxit, double *out);

#ifdef __cplusplus
}
#endif
#endif
