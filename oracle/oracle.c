/*
 * Plain FP64 CPU oracle for matching-based AMG-preconditioned CG.
 *
 * TEST INFRASTRUCTURE: loaded only by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark. It is deliberately serial and simple so
 * that each step can be read against the paper:
 *
 *   Section 3.1   A_{l+1} = P_l^T A_l P_l and the V-cycle of eq. (amg)
 *   Section 3.2   eq. (weights), maximum-weight matching (half-approximate,
 *                 locally dominant class), eq. (prolongator), restriction
 *                 of w to the coarse level, products of pairwise sweeps
 *   Section 3.3   l1-Jacobi, eq. (l1weights) with blocks of size one
 *   Section 5     CG outer iteration, relative residual stop, coarsest size
 *
 * Readings of points the paper leaves open (all pinned by tests):
 *   - ties in the matching are broken by the strict key
 *     (weight descending, lo ascending, hi ascending); under a strict key the
 *     locally-dominant algorithm and the greedy scan give the same matching;
 *   - the maximum-product objective and its log transform order edges the
 *     same way as c itself, so the matching is taken on c directly;
 *   - coarse indices are numbered by the smallest member of each aggregate;
 *   - one level runs `sweeps` pairwise sweeps; a sweep that matches nothing
 *     ends the level's sweeps; a level whose size does not shrink becomes
 *     the coarsest (an error if it exceeds ORC_MAX_DENSE);
 *   - the coarsest level is factored by dense Cholesky; the alternative
 *     iterative coarsest solver (CG with the l1-Jacobi diagonal) stops on
 *     the first ||r_k|| < rtol ||b||, strictly, from a zero guess.
 *
 * Arithmetic: IEEE binary64, round to nearest, built with -ffp-contract=off
 * and without fast-math. Every sum starts from its first term and runs in
 * the order stated next to it.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_DENSE 4096
#define ORC_MAX_LEVELS 64

/* ------------------------------------------------------------------------ */
/* small helpers                                                            */
/* ------------------------------------------------------------------------ */

static int same_bits(double a, double b) {
  uint64_t x, y;
  memcpy(&x, &a, 8);
  memcpy(&y, &b, 8);
  return x == y;
}

/* position of column j in row i, or -1 (binary search, columns ascending) */
static int64_t find_entry(const orc_csr *A, int32_t i, int32_t j) {
  int64_t lo = A->rp[i], hi = (int64_t)A->rp[i + 1] - 1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (A->ci[mid] == j) return mid;
    if (A->ci[mid] < j) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

static double diag_of(const orc_csr *A, int32_t i) {
  int64_t k = find_entry(A, i, i);
  return k >= 0 ? A->val[k] : 0.0;
}

static int i32_cmp(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

static double dot(int64_t n, const double *x, const double *y) {
  if (n == 0) return 0.0;
  double s = x[0] * y[0];
  for (int64_t i = 1; i < n; ++i) s = s + x[i] * y[i];
  return s;
}

static int csr_alloc(orc_csr *A, int32_t n, int64_t nnz) {
  A->n = n;
  A->nnz = nnz;
  A->rp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
  A->ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  A->val = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  if (!A->rp || !A->ci || !A->val) {
    orc_csr_free(A);
    return ORC_ERR_OOM;
  }
  return ORC_OK;
}

void orc_csr_free(orc_csr *A) {
  if (!A) return;
  free(A->rp);
  free(A->ci);
  free(A->val);
  A->rp = NULL;
  A->ci = NULL;
  A->val = NULL;
  A->n = 0;
  A->nnz = 0;
}

static int csr_copy(const orc_csr *A, orc_csr *B) {
  int st = csr_alloc(B, A->n, A->nnz);
  if (st) return st;
  memcpy(B->rp, A->rp, sizeof(int32_t) * ((size_t)A->n + 1));
  memcpy(B->ci, A->ci, sizeof(int32_t) * (size_t)A->nnz);
  memcpy(B->val, A->val, sizeof(double) * (size_t)A->nnz);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* single steps                                                             */
/* ------------------------------------------------------------------------ */

void orc_spmv(const orc_csr *A, const double *x, double *y) {
  for (int32_t i = 0; i < A->n; ++i) {
    int64_t b = A->rp[i], e = A->rp[i + 1];
    double s = 0.0;
    if (e > b) {
      s = A->val[b] * x[A->ci[b]];
      for (int64_t k = b + 1; k < e; ++k) s = s + A->val[k] * x[A->ci[k]];
    }
    y[i] = s;
  }
}

int orc_check(const orc_csr *A) {
  if (A->n <= 0 || A->rp[0] != 0 || (int64_t)A->rp[A->n] != A->nnz) return ORC_ERR_ARG;
  for (int32_t i = 0; i < A->n; ++i) {
    if (A->rp[i + 1] < A->rp[i]) return ORC_ERR_ARG;
    for (int64_t k = A->rp[i]; k < A->rp[i + 1]; ++k) {
      if (A->ci[k] < 0 || A->ci[k] >= A->n) return ORC_ERR_ARG;
      if (k > A->rp[i] && A->ci[k] <= A->ci[k - 1]) return ORC_ERR_ARG;
      if (!isfinite(A->val[k])) return ORC_ERR_ARG;
    }
  }
  for (int32_t i = 0; i < A->n; ++i) {
    int64_t d = find_entry(A, i, i);
    if (d < 0 || !(A->val[d] > 0.0)) return ORC_ERR_NOT_SPD;
  }
  for (int32_t i = 0; i < A->n; ++i) {
    for (int64_t k = A->rp[i]; k < A->rp[i + 1]; ++k) {
      int64_t t = find_entry(A, A->ci[k], i);
      if (t < 0 || !same_bits(A->val[t], A->val[k])) return ORC_ERR_NOT_SYMMETRIC;
    }
  }
  return ORC_OK;
}

int64_t orc_num_edges(const orc_csr *A) {
  int64_t ne = 0;
  for (int32_t i = 0; i < A->n; ++i)
    for (int64_t k = A->rp[i]; k < A->rp[i + 1]; ++k)
      if (A->ci[k] > i) ++ne;
  return ne;
}

/* eq. (weights) */
void orc_edge_weights(const orc_csr *A, const double *w, int32_t *lo,
                      int32_t *hi, double *c) {
  int64_t e = 0;
  for (int32_t i = 0; i < A->n; ++i) {
    double aii = diag_of(A, i);
    for (int64_t k = A->rp[i]; k < A->rp[i + 1]; ++k) {
      int32_t j = A->ci[k];
      if (j <= i) continue;
      double a = A->val[k];
      double ajj = diag_of(A, j);
      double num = ((2.0 * a) * w[i]) * w[j];
      double den = (aii * w[i]) * w[i] + (ajj * w[j]) * w[j];
      lo[e] = i;
      hi[e] = j;
      c[e] = 1.0 - num / den;
      ++e;
    }
  }
}

/* sort key for the matching: c descending, then lo ascending, hi ascending */
typedef struct {
  double c;
  int32_t lo, hi;
} edge_key;

static int edge_cmp(const void *pa, const void *pb) {
  const edge_key *a = (const edge_key *)pa, *b = (const edge_key *)pb;
  if (a->c > b->c) return -1;
  if (a->c < b->c) return 1;
  if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
  if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;
  return 0;
}

int64_t orc_greedy_matching(int32_t n, int64_t ne, const int32_t *lo,
                            const int32_t *hi, const double *c, int32_t *mate) {
  edge_key *ek = (edge_key *)malloc(sizeof(edge_key) * (size_t)(ne > 0 ? ne : 1));
  for (int64_t e = 0; e < ne; ++e) {
    ek[e].c = c[e];
    ek[e].lo = lo[e];
    ek[e].hi = hi[e];
  }
  qsort(ek, (size_t)ne, sizeof(edge_key), edge_cmp);
  for (int32_t v = 0; v < n; ++v) mate[v] = -1;
  int64_t nm = 0;
  for (int64_t e = 0; e < ne; ++e) {
    int32_t a = ek[e].lo, b = ek[e].hi;
    if (a != b && mate[a] < 0 && mate[b] < 0) {
      mate[a] = b;
      mate[b] = a;
      ++nm;
    }
  }
  free(ek);
  return nm;
}

int32_t orc_number_aggregates(int32_t n, const int32_t *mate, int32_t *agg) {
  for (int32_t v = 0; v < n; ++v) agg[v] = -1;
  int32_t next = 0;
  for (int32_t v = 0; v < n; ++v) {
    if (agg[v] >= 0) continue;
    agg[v] = next;
    if (mate[v] >= 0) agg[mate[v]] = next;
    ++next;
  }
  return next;
}

/* eq. (prolongator): orthonormal projection of w on each pair, w_s/|w_s| on
 * singletons. */
void orc_pairwise_prolongator(int32_t n, const int32_t *mate, const double *w,
                              double *p) {
  for (int32_t v = 0; v < n; ++v) {
    if (mate[v] < 0) {
      p[v] = w[v] / fabs(w[v]);
    } else {
      int32_t i = v < mate[v] ? v : mate[v];
      int32_t j = v < mate[v] ? mate[v] : v;
      double s = w[i] * w[i] + w[j] * w[j];
      p[v] = w[v] / sqrt(s);
    }
  }
}

void orc_restrict(int32_t n, int32_t nc, const int32_t *agg, const double *p,
                  const double *v, double *vc) {
  char *seen = (char *)calloc((size_t)(nc > 0 ? nc : 1), 1);
  for (int32_t i = 0; i < n; ++i) { /* ascending i within every aggregate */
    int32_t I = agg[i];
    double t = p[i] * v[i];
    if (!seen[I]) {
      vc[I] = t;
      seen[I] = 1;
    } else {
      vc[I] = vc[I] + t;
    }
  }
  for (int32_t I = 0; I < nc; ++I)
    if (!seen[I]) vc[I] = 0.0;
  free(seen);
}

/* y = M x for a rectangular CSR M (rows summed over ascending columns;
 * an empty row gives 0) */
static void csr_apply(const orc_csr *M, const double *x, double *y) {
  for (int32_t i = 0; i < M->n; ++i) {
    int64_t k = M->rp[i];
    double s = 0.0;
    if (k < M->rp[i + 1]) {
      s = M->val[k] * x[M->ci[k]];
      for (++k; k < M->rp[i + 1]; ++k) s = s + M->val[k] * x[M->ci[k]];
    }
    y[i] = s;
  }
}

/* one Galerkin term of the pairwise product */
typedef struct {
  int32_t J, lo, hi;
  double t;
} rap_term;

static int rap_cmp(const void *pa, const void *pb) {
  const rap_term *a = (const rap_term *)pa, *b = (const rap_term *)pb;
  if (a->J != b->J) return a->J < b->J ? -1 : 1;
  if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
  if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;
  return 0; /* equal keys carry equal terms (A is bitwise symmetric) */
}

int orc_galerkin_pairwise(const orc_csr *A, int32_t nc, const int32_t *agg,
                          const double *p, orc_csr *Ac) {
  int32_t n = A->n;
  /* members of each aggregate, ascending (at most two) */
  int32_t *m0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)nc);
  int32_t *m1 = (int32_t *)malloc(sizeof(int32_t) * (size_t)nc);
  for (int32_t I = 0; I < nc; ++I) m0[I] = m1[I] = -1;
  for (int32_t i = 0; i < n; ++i) {
    int32_t I = agg[i];
    if (m0[I] < 0) m0[I] = i;
    else if (m1[I] < 0) m1[I] = i;
    else { free(m0); free(m1); return ORC_ERR_ARG; } /* not pairwise */
  }
  int32_t maxrow = 0;
  for (int32_t i = 0; i < n; ++i)
    if (A->rp[i + 1] - A->rp[i] > maxrow) maxrow = A->rp[i + 1] - A->rp[i];
  rap_term *buf = (rap_term *)malloc(sizeof(rap_term) * (size_t)(2 * maxrow + 1));

  /* pass 1: row lengths; pass 2: fill */
  int32_t *rp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nc + 1));
  int32_t *ci = NULL;
  double *vv = NULL;
  rp[0] = 0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int32_t I = 0; I < nc; ++I) {
      int32_t cnt = 0;
      int32_t mem[2] = {m0[I], m1[I]};
      for (int q = 0; q < 2; ++q) {
        int32_t f = mem[q];
        if (f < 0) continue;
        for (int64_t k = A->rp[f]; k < A->rp[f + 1]; ++k) {
          int32_t j = A->ci[k];
          int32_t lo = f < j ? f : j;
          int32_t hi = f < j ? j : f;
          double a = A->val[find_entry(A, lo, hi)]; /* a from row lo */
          buf[cnt].J = agg[j];
          buf[cnt].lo = lo;
          buf[cnt].hi = hi;
          buf[cnt].t = (p[lo] * a) * p[hi];
          ++cnt;
        }
      }
      qsort(buf, (size_t)cnt, sizeof(rap_term), rap_cmp);
      int32_t out = 0;
      for (int32_t k = 0; k < cnt; ++k) {
        if (k == 0 || buf[k].J != buf[k - 1].J) {
          if (pass == 1) {
            ci[rp[I] + out] = buf[k].J;
            vv[rp[I] + out] = buf[k].t;
          }
          ++out;
        } else if (pass == 1) {
          vv[rp[I] + out - 1] = vv[rp[I] + out - 1] + buf[k].t;
        }
      }
      if (pass == 0) rp[I + 1] = rp[I] + out;
    }
    if (pass == 0) {
      ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(rp[nc] > 0 ? rp[nc] : 1));
      vv = (double *)malloc(sizeof(double) * (size_t)(rp[nc] > 0 ? rp[nc] : 1));
    }
  }
  free(buf);
  free(m0);
  free(m1);
  Ac->n = nc;
  Ac->nnz = rp[nc];
  Ac->rp = rp;
  Ac->ci = ci;
  Ac->val = vv;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* smoothed aggregation (the alternative to the K-cycle in Section 3.2)      */
/* ------------------------------------------------------------------------ */

/* omega = 4 / (3 ||D^-1 A||_inf): per row (sum over ascending j of |a_ij|) /
 * a_ii, the maximum over rows, then 4 / (3 max). This is the classical
 * smoothed-aggregation damping 4 / (3 rho(D^-1 A)) with rho estimated by the
 * infinity norm, as the supplement's remark on the smoothed prolongator
 * estimates it. The supplement's table of K with the smoothed prolongator
 * (16^3 Laplacian, HGS, np = 1) is reproduced with this omega; the text's
 * omega = 1 / ||D^-1 A||_inf gives a different K. */
double orc_smoothing_omega(const orc_csr *A) {
  double nrm = 0.0;
  for (int32_t i = 0; i < A->n; ++i) {
    double s = 0.0;
    for (int64_t k = A->rp[i]; k < A->rp[i + 1]; ++k) s = s + fabs(A->val[k]);
    double r = s / diag_of(A, i);
    if (r > nrm) nrm = r;
  }
  return 4.0 / (3.0 * nrm);
}

/* Pbar = (I - omega D^-1 A) P for the tentative prolongator P (one entry
 * p[i] in column agg[i] per row). Row i of Pbar has one entry per distinct
 * aggregate J among the columns of row i of A, J ascending:
 *   s = sum over j ascending with agg[j] = J of a_ij p_j,  t = s / a_ii,
 *   Pbar(i, J) = (J = agg[i] ? p_i : 0) - omega t.
 * Pbar has nc columns. */
int orc_smooth_prolongator(const orc_csr *A, int32_t nc, const int32_t *agg, const double *p,
                           double omega, orc_csr *Pb) {
  int32_t n = A->n;
  int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
  int32_t *cols = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  double *acc = (double *)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
  for (int32_t J = 0; J < nc; ++J) pos[J] = -1;
  int st = csr_alloc(Pb, n, A->nnz); /* at most one entry per entry of A */
  if (st) return st;
  int64_t out = 0;
  Pb->rp[0] = 0;
  for (int32_t i = 0; i < n; ++i) {
    int32_t cnt = 0;
    for (int64_t k = A->rp[i]; k < A->rp[i + 1]; ++k) {
      int32_t j = A->ci[k], J = agg[j];
      double t = A->val[k] * p[j];
      if (pos[J] < 0) {
        pos[J] = cnt;
        cols[cnt++] = J;
        acc[J] = t;
      } else {
        acc[J] = acc[J] + t;
      }
    }
    /* ascending J (insertion sort: a row has few distinct aggregates) */
    for (int32_t a = 1; a < cnt; ++a) {
      int32_t v = cols[a], b = a - 1;
      while (b >= 0 && cols[b] > v) {
        cols[b + 1] = cols[b];
        --b;
      }
      cols[b + 1] = v;
    }
    double aii = diag_of(A, i);
    for (int32_t a = 0; a < cnt; ++a) {
      int32_t J = cols[a];
      double t = acc[J] / aii;
      double base = J == agg[i] ? p[i] : 0.0;
      Pb->ci[out] = J;
      Pb->val[out] = base - omega * t;
      ++out;
      pos[J] = -1;
    }
    Pb->rp[i + 1] = (int32_t)out;
  }
  Pb->nnz = out;
  free(pos);
  free(cols);
  free(acc);
  return ORC_OK;
}

/* C(r, :) = sum over k in [xp[r], xp[r+1]) ascending of coef[k] B(src[k], :):
 * every column's terms coef[k] * b are added in k order onto the first one;
 * columns ascending. B has ncols columns; C has nr rows. */
static int rowcomb(int32_t nr, const int32_t *xp, const int32_t *src, const double *coef,
                   const orc_csr *B, int32_t ncols, orc_csr *C) {
  int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncols > 0 ? ncols : 1));
  int32_t *cols = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncols > 0 ? ncols : 1));
  double *acc = (double *)malloc(sizeof(double) * (size_t)(ncols > 0 ? ncols : 1));
  for (int32_t J = 0; J < ncols; ++J) mark[J] = 0;
  int32_t *rp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nr + 1));
  int64_t cap = 1024, out = 0;
  int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
  double *vv = (double *)malloc(sizeof(double) * (size_t)cap);
  rp[0] = 0;
  for (int32_t r = 0; r < nr; ++r) {
    int32_t cnt = 0;
    for (int32_t k = xp[r]; k < xp[r + 1]; ++k) {
      int32_t s = src[k];
      for (int64_t e = B->rp[s]; e < B->rp[s + 1]; ++e) {
        int32_t J = B->ci[e];
        double t = coef[k] * B->val[e];
        if (!mark[J]) {
          mark[J] = 1;
          cols[cnt++] = J;
          acc[J] = t;
        } else {
          acc[J] = acc[J] + t;
        }
      }
    }
    qsort(cols, (size_t)cnt, sizeof(int32_t), i32_cmp);
    if (out + cnt > cap) {
      while (out + cnt > cap) cap *= 2;
      ci = (int32_t *)realloc(ci, sizeof(int32_t) * (size_t)cap);
      vv = (double *)realloc(vv, sizeof(double) * (size_t)cap);
    }
    for (int32_t a = 0; a < cnt; ++a) {
      ci[out] = cols[a];
      vv[out] = acc[cols[a]];
      mark[cols[a]] = 0;
      ++out;
    }
    rp[r + 1] = (int32_t)out;
  }
  free(mark);
  free(cols);
  free(acc);
  C->n = nr;
  C->nnz = out;
  C->rp = rp;
  C->ci = ci;
  C->val = vv;
  return ORC_OK;
}

/* transpose of an n x ncols CSR: row J lists the rows i holding column J,
 * ascending i */
static int csr_transpose(const orc_csr *A, int32_t ncols, orc_csr *T) {
  int st = csr_alloc(T, ncols, A->nnz);
  if (st) return st;
  for (int32_t J = 0; J <= ncols; ++J) T->rp[J] = 0;
  for (int64_t k = 0; k < A->nnz; ++k) T->rp[A->ci[k] + 1] += 1;
  for (int32_t J = 0; J < ncols; ++J) T->rp[J + 1] += T->rp[J];
  int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncols > 0 ? ncols : 1));
  for (int32_t J = 0; J < ncols; ++J) next[J] = T->rp[J];
  for (int32_t i = 0; i < A->n; ++i)
    for (int64_t k = A->rp[i]; k < A->rp[i + 1]; ++k) {
      int32_t J = A->ci[k];
      T->ci[next[J]] = i;
      T->val[next[J]] = A->val[k];
      ++next[J];
    }
  free(next);
  return ORC_OK;
}

/* A_c = Pbar^T A Pbar (Section 3.1's Galerkin product with the smoothed
 * prolongator): first AP = A Pbar (row i: a_ij Pbar(j, :) over ascending j),
 * then A_c(I, :) = sum over ascending i of Pbar(i, I) AP(i, :); the lower
 * triangle is then replaced by the upper one, so A_c is bitwise symmetric. */
int orc_galerkin_general(const orc_csr *A, const orc_csr *Pb, int32_t nc, orc_csr *Ac) {
  orc_csr AP = {0}, PbT = {0};
  int st = rowcomb(A->n, A->rp, A->ci, A->val, Pb, nc, &AP);
  if (!st) st = csr_transpose(Pb, nc, &PbT);
  if (!st) st = rowcomb(nc, PbT.rp, PbT.ci, PbT.val, &AP, nc, Ac);
  orc_csr_free(&AP);
  orc_csr_free(&PbT);
  if (st) return st;
  for (int32_t I = 0; I < nc; ++I)
    for (int64_t k = Ac->rp[I]; k < Ac->rp[I + 1]; ++k) {
      int32_t J = Ac->ci[k];
      if (J < I) {
        int64_t m = find_entry(Ac, J, I);
        if (m < 0) return ORC_ERR_ARG; /* cannot happen: the pattern is symmetric */
        Ac->val[k] = Ac->val[m];
      }
    }
  return ORC_OK;
}

/* eq. (l1weights), nb = 1 */
void orc_l1_diag(const orc_csr *A, double *m) {
  for (int32_t i = 0; i < A->n; ++i) {
    double aii = 0.0, s = 0.0;
    int first = 1;
    for (int64_t k = A->rp[i]; k < A->rp[i + 1]; ++k) {
      if (A->ci[k] == i) {
        aii = A->val[k];
      } else if (first) {
        s = fabs(A->val[k]);
        first = 0;
      } else {
        s = s + fabs(A->val[k]);
      }
    }
    m[i] = aii + s;
  }
}

/* Algebraically smooth vector (the remark after eq. (prolongator)): nu
 * iterations of the l1-Jacobi smoother on A w = 0 from the sample w,
 * w <- w - (A w) / m, in place. */
void orc_smooth_w(const orc_csr *A, int32_t nu, double *w) {
  int32_t n = A->n;
  double *m = (double *)malloc(sizeof(double) * (size_t)n);
  double *t = (double *)malloc(sizeof(double) * (size_t)n);
  orc_l1_diag(A, m);
  for (int32_t s = 0; s < nu; ++s) {
    orc_spmv(A, w, t);
    for (int32_t i = 0; i < n; ++i) w[i] = w[i] - t[i] / m[i];
  }
  free(m);
  free(t);
}

int orc_cholesky(int32_t n, double *a) {
  for (int32_t j = 0; j < n; ++j) {
    double s = a[(int64_t)j * n + j];
    for (int32_t k = 0; k < j; ++k) s = s - a[(int64_t)j * n + k] * a[(int64_t)j * n + k];
    if (!(s > 0.0)) return ORC_ERR_NOT_SPD;
    double d = sqrt(s);
    a[(int64_t)j * n + j] = d;
    for (int32_t i = j + 1; i < n; ++i) {
      double t = a[(int64_t)i * n + j];
      for (int32_t k = 0; k < j; ++k) t = t - a[(int64_t)i * n + k] * a[(int64_t)j * n + k];
      a[(int64_t)i * n + j] = t / d;
    }
  }
  for (int32_t i = 0; i < n; ++i)
    for (int32_t j = i + 1; j < n; ++j) a[(int64_t)i * n + j] = 0.0;
  return ORC_OK;
}

void orc_cholesky_solve(int32_t n, const double *L, const double *r, double *z) {
  double *y = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int32_t i = 0; i < n; ++i) {
    double t = r[i];
    for (int32_t k = 0; k < i; ++k) t = t - L[(int64_t)i * n + k] * y[k];
    y[i] = t / L[(int64_t)i * n + i];
  }
  for (int32_t i = n - 1; i >= 0; --i) {
    double t = y[i];
    for (int32_t k = i + 1; k < n; ++k) t = t - L[(int64_t)k * n + i] * z[k];
    z[i] = t / L[(int64_t)i * n + i];
  }
  free(y);
}

/* ------------------------------------------------------------------------ */
/* hierarchy                                                                */
/* ------------------------------------------------------------------------ */

struct orc_hier {
  int32_t nlev;
  orc_csr A[ORC_MAX_LEVELS];
  double *w[ORC_MAX_LEVELS];
  int32_t *agg[ORC_MAX_LEVELS]; /* level l -> l+1 composed map */
  double *p[ORC_MAX_LEVELS];    /* composed prolongator values */
  double *m[ORC_MAX_LEVELS];    /* l1-Jacobi diagonal */
  int32_t nsweeps[ORC_MAX_LEVELS];
  int32_t nL;
  double *L; /* coarsest Cholesky factor */
  int32_t coarse_solver; /* 0: Cholesky; 1: orc_coarse_pcg */
  double coarse_rtol;
  int32_t coarse_maxit;
  int32_t smooth;                 /* smoothed prolongators (Pbar) between levels */
  orc_csr Pb[ORC_MAX_LEVELS];     /* level l -> l+1 Pbar, n_l x n_{l+1} */
  orc_csr PbT[ORC_MAX_LEVELS];    /* its transpose */
  double omega[ORC_MAX_LEVELS];
};

void orc_free(orc_hier *h) {
  if (!h) return;
  for (int32_t l = 0; l < ORC_MAX_LEVELS; ++l) {
    orc_csr_free(&h->A[l]);
    free(h->w[l]);
    free(h->agg[l]);
    free(h->p[l]);
    free(h->m[l]);
    orc_csr_free(&h->Pb[l]);
    orc_csr_free(&h->PbT[l]);
  }
  free(h->L);
  free(h);
}

/* One pairwise sweep (Section 3.2) on (A, w): weights, matching, numbering,
 * prolongator, Galerkin product and restriction of w. Returns the number of
 * matched edges (0: nothing produced), or a negative status. */
static int64_t pairwise_sweep(const orc_csr *A, const double *w, orc_csr *Ac,
                              double **wc, int32_t **agg, double **p) {
  int32_t n = A->n;
  int64_t ne = orc_num_edges(A);
  int32_t *lo = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
  int32_t *hi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
  double *c = (double *)malloc(sizeof(double) * (size_t)(ne > 0 ? ne : 1));
  int32_t *mate = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  orc_edge_weights(A, w, lo, hi, c);
  int64_t nm = orc_greedy_matching(n, ne, lo, hi, c, mate);
  free(lo);
  free(hi);
  free(c);
  if (nm == 0) {
    free(mate);
    return 0;
  }
  *agg = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  *p = (double *)malloc(sizeof(double) * (size_t)n);
  int32_t nc = orc_number_aggregates(n, mate, *agg);
  orc_pairwise_prolongator(n, mate, w, *p);
  free(mate);
  int st = orc_galerkin_pairwise(A, nc, *agg, *p, Ac);
  if (st) return -st;
  *wc = (double *)malloc(sizeof(double) * (size_t)nc);
  orc_restrict(n, nc, *agg, *p, w, *wc);
  return nm;
}

int orc_setup(const orc_csr *A0, const double *w0, int32_t sweeps,
              int32_t max_coarse, int32_t max_levels, orc_hier **out) {
  return orc_setup_opts(A0, w0, sweeps, max_coarse, max_levels, 0, out);
}

int orc_setup_opts(const orc_csr *A0, const double *w0, int32_t sweeps, int32_t max_coarse,
                   int32_t max_levels, int32_t smooth, orc_hier **out) {
  *out = NULL;
  if (!A0 || sweeps < 1 || max_coarse < 1 || max_levels < 1) return ORC_ERR_ARG;
  if (max_levels > ORC_MAX_LEVELS) max_levels = ORC_MAX_LEVELS;
  int st = orc_check(A0);
  if (st) return st;
  if (w0)
    for (int32_t i = 0; i < A0->n; ++i)
      if (!(w0[i] != 0.0) || !isfinite(w0[i])) return ORC_ERR_ARG;
  orc_hier *h = (orc_hier *)calloc(1, sizeof(orc_hier));
  h->smooth = smooth ? 1 : 0;
  csr_copy(A0, &h->A[0]);
  h->w[0] = (double *)malloc(sizeof(double) * (size_t)A0->n);
  for (int32_t i = 0; i < A0->n; ++i) h->w[0][i] = w0 ? w0[i] : 1.0;

  int32_t l = 0;
  for (;;) {
    int32_t n = h->A[l].n;
    if (n <= max_coarse || l == max_levels - 1) break;
    /* m pairwise sweeps whose product is P_l (Section 3.2) */
    orc_csr cur = h->A[l];
    double *wcur = h->w[l];
    int own = 0; /* cur/wcur owned by this loop (not the level's) */
    int32_t *agg_c = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *p_c = (double *)malloc(sizeof(double) * (size_t)n);
    int32_t done = 0;
    for (int32_t k = 0; k < sweeps; ++k) {
      orc_csr nxt = {0};
      double *wn = NULL;
      int32_t *ag = NULL;
      double *pk = NULL;
      int64_t nm = pairwise_sweep(&cur, wcur, &nxt, &wn, &ag, &pk);
      if (nm < 0) {
        orc_free(h);
        return (int)(-nm);
      }
      if (nm == 0) break;
      /* compose: P_l(i) = ((p_1(i) p_2(agg_1(i))) p_3(agg_2(agg_1(i)))) */
      for (int32_t i = 0; i < n; ++i) {
        if (k == 0) {
          p_c[i] = pk[i];
          agg_c[i] = ag[i];
        } else {
          int32_t a = agg_c[i];
          p_c[i] = p_c[i] * pk[a];
          agg_c[i] = ag[a];
        }
      }
      free(ag);
      free(pk);
      if (own) {
        orc_csr_free(&cur);
        free(wcur);
      }
      cur = nxt;
      wcur = wn;
      own = 1;
      ++done;
    }
    if (done == 0) { /* nothing matched: this level is the coarsest */
      free(agg_c);
      free(p_c);
      break;
    }
    h->agg[l] = agg_c;
    h->p[l] = p_c;
    h->nsweeps[l] = done;
    h->w[l + 1] = wcur;
    if (h->smooth) {
      /* the tentative product P_l only chose the aggregates and restricted
       * w; the next level is the Galerkin product with Pbar_l */
      int32_t nc = cur.n;
      orc_csr_free(&cur);
      h->omega[l] = orc_smoothing_omega(&h->A[l]);
      st = orc_smooth_prolongator(&h->A[l], nc, agg_c, p_c, h->omega[l], &h->Pb[l]);
      if (!st) st = csr_transpose(&h->Pb[l], nc, &h->PbT[l]);
      if (!st) st = orc_galerkin_general(&h->A[l], &h->Pb[l], nc, &h->A[l + 1]);
      if (st) {
        orc_free(h);
        return st;
      }
    } else {
      h->A[l + 1] = cur;
    }
    ++l;
  }
  h->nlev = l + 1;
  for (int32_t k = 0; k <= l; ++k) {
    h->m[k] = (double *)malloc(sizeof(double) * (size_t)h->A[k].n);
    orc_l1_diag(&h->A[k], h->m[k]);
  }
  /* coarsest: dense Cholesky */
  orc_csr *C = &h->A[l];
  if (C->n > ORC_MAX_DENSE) {
    orc_free(h);
    return ORC_ERR_STALL;
  }
  h->nL = C->n;
  h->L = (double *)calloc((size_t)C->n * (size_t)C->n, sizeof(double));
  for (int32_t i = 0; i < C->n; ++i)
    for (int64_t k = C->rp[i]; k < C->rp[i + 1]; ++k)
      h->L[(int64_t)i * C->n + C->ci[k]] = C->val[k];
  st = orc_cholesky(C->n, h->L);
  if (st) {
    orc_free(h);
    return st;
  }
  *out = h;
  return ORC_OK;
}

int32_t orc_num_levels(const orc_hier *h) { return h->nlev; }
int64_t orc_level_n(const orc_hier *h, int32_t l) { return h->A[l].n; }
int64_t orc_level_nnz(const orc_hier *h, int32_t l) { return h->A[l].nnz; }
int32_t orc_level_sweeps(const orc_hier *h, int32_t l) { return h->nsweeps[l]; }

void orc_level_csr(const orc_hier *h, int32_t l, int32_t *rp, int32_t *ci, double *val) {
  const orc_csr *A = &h->A[l];
  memcpy(rp, A->rp, sizeof(int32_t) * ((size_t)A->n + 1));
  memcpy(ci, A->ci, sizeof(int32_t) * (size_t)A->nnz);
  memcpy(val, A->val, sizeof(double) * (size_t)A->nnz);
}

void orc_level_transfer(const orc_hier *h, int32_t l, int32_t *agg, double *p) {
  memcpy(agg, h->agg[l], sizeof(int32_t) * (size_t)h->A[l].n);
  memcpy(p, h->p[l], sizeof(double) * (size_t)h->A[l].n);
}

void orc_level_l1diag(const orc_hier *h, int32_t l, double *m) {
  memcpy(m, h->m[l], sizeof(double) * (size_t)h->A[l].n);
}

void orc_level_w(const orc_hier *h, int32_t l, double *w) {
  memcpy(w, h->w[l], sizeof(double) * (size_t)h->A[l].n);
}

int64_t orc_level_pbar_nnz(const orc_hier *h, int32_t l) { return h->Pb[l].nnz; }

void orc_level_pbar(const orc_hier *h, int32_t l, int32_t *rp, int32_t *ci, double *val) {
  const orc_csr *P = &h->Pb[l];
  memcpy(rp, P->rp, sizeof(int32_t) * ((size_t)P->n + 1));
  memcpy(ci, P->ci, sizeof(int32_t) * (size_t)P->nnz);
  memcpy(val, P->val, sizeof(double) * (size_t)P->nnz);
}

double orc_level_omega(const orc_hier *h, int32_t l) { return h->omega[l]; }

void orc_coarse_factor(const orc_hier *h, double *L) {
  memcpy(L, h->L, sizeof(double) * (size_t)h->nL * (size_t)h->nL);
}

void orc_set_coarse_solver(orc_hier *h, int32_t solver, double rtol, int32_t maxit) {
  h->coarse_solver = solver;
  h->coarse_rtol = rtol;
  h->coarse_maxit = maxit;
}

/* Hestenes-Stiefel PCG from x = 0 (r_0 = b), preconditioner z = r / m:
 *   q = A p_k, alpha = (r_k, z_k) / (p_k, q), x += alpha p_k, r -= alpha q;
 *   stop if ||r_{k+1}|| < rtol ||b|| or k + 1 = maxit;
 *   z = r / m, beta = (r_{k+1}, z_{k+1}) / (r_k, z_k), p = z + beta p. */
int32_t orc_coarse_pcg(const orc_csr *A, const double *m, const double *b, double rtol,
                       int32_t maxit, double *x) {
  int32_t n = A->n;
  for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
  double bnorm = sqrt(dot(n, b, b));
  if (bnorm == 0.0 || maxit < 1) return 0;
  double *r = (double *)malloc(sizeof(double) * (size_t)n);
  double *z = (double *)malloc(sizeof(double) * (size_t)n);
  double *p = (double *)malloc(sizeof(double) * (size_t)n);
  double *q = (double *)malloc(sizeof(double) * (size_t)n);
  for (int32_t i = 0; i < n; ++i) r[i] = b[i];
  for (int32_t i = 0; i < n; ++i) z[i] = r[i] / m[i];
  for (int32_t i = 0; i < n; ++i) p[i] = z[i];
  double rz0 = dot(n, r, z);
  int32_t it = 0;
  while (it < maxit) {
    orc_spmv(A, p, q);
    double pq = dot(n, p, q);
    if (!(pq > 0.0)) break;
    double step = rz0 / pq;
    for (int32_t i = 0; i < n; ++i) x[i] = x[i] + step * p[i];
    for (int32_t i = 0; i < n; ++i) r[i] = r[i] - step * q[i];
    ++it;
    if (sqrt(dot(n, r, r)) < rtol * bnorm) break;
    for (int32_t i = 0; i < n; ++i) z[i] = r[i] / m[i]; /* preconditioned residual */
    double rz1 = dot(n, r, z);
    double beta = rz1 / rz0;
    rz0 = rz1;
    for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
  }
  free(r);
  free(z);
  free(p);
  free(q);
  return it;
}

static void fcg2(const orc_hier *h, int32_t m, int32_t pre, int32_t post, const double *b,
                 double *x);

/* One application of the multilevel preconditioner on level l.
 * eq. (amg): pre-smoothing M^-1 from a zero guess, coarse correction,
 * post-smoothing M^-T = M^-1 (M diagonal). The coarse correction solves
 * A_{l+1} e = P^T t: on the coarsest level exactly (Cholesky) or by the
 * hierarchy's iterative coarsest solver; else by the same cycle
 * on level l + 1 (V-cycle, kcycle = 0), or by two iterations of flexible CG
 * on level l + 1 preconditioned by the cycle starting there (K-cycle,
 * kcycle = 1; Section 3.1, which applies those FCG iterations on every
 * level but the finest and the coarsest). */
static void cycle(const orc_hier *h, int32_t l, int32_t pre, int32_t post, int kcycle,
                  const double *r, double *z) {
  int32_t L = h->nlev - 1;
  if (l == L) {
    if (h->coarse_solver == 1)
      (void)orc_coarse_pcg(&h->A[L], h->m[L], r, h->coarse_rtol, h->coarse_maxit, z);
    else
      orc_cholesky_solve(h->nL, h->L, r, z);
    return;
  }
  const orc_csr *A = &h->A[l];
  int32_t n = A->n, nc = h->A[l + 1].n;
  const double *m = h->m[l];
  double *t = (double *)malloc(sizeof(double) * (size_t)n);
  double *rc = (double *)malloc(sizeof(double) * (size_t)nc);
  double *zc = (double *)malloc(sizeof(double) * (size_t)nc);
  /* pre-smoothing */
  for (int32_t i = 0; i < n; ++i) z[i] = pre > 0 ? r[i] / m[i] : 0.0;
  for (int32_t s = 1; s < pre; ++s) {
    orc_spmv(A, z, t);
    for (int32_t i = 0; i < n; ++i) z[i] = z[i] + (r[i] - t[i]) / m[i];
  }
  /* residual, restriction, coarse correction, prolongation */
  orc_spmv(A, z, t);
  for (int32_t i = 0; i < n; ++i) t[i] = r[i] - t[i];
  if (h->smooth) csr_apply(&h->PbT[l], t, rc); /* rc = Pbar^T t */
  else orc_restrict(n, nc, h->agg[l], h->p[l], t, rc);
  if (kcycle && l + 1 < L) fcg2(h, l + 1, pre, post, rc, zc);
  else cycle(h, l + 1, pre, post, kcycle, rc, zc);
  if (h->smooth) {
    double *u = (double *)malloc(sizeof(double) * (size_t)n);
    csr_apply(&h->Pb[l], zc, u); /* u = Pbar zc */
    for (int32_t i = 0; i < n; ++i) z[i] = z[i] + u[i];
    free(u);
  } else {
    for (int32_t i = 0; i < n; ++i) z[i] = z[i] + h->p[l][i] * zc[h->agg[l][i]];
  }
  /* post-smoothing */
  for (int32_t s = 0; s < post; ++s) {
    orc_spmv(A, z, t);
    for (int32_t i = 0; i < n; ++i) z[i] = z[i] + (r[i] - t[i]) / m[i];
  }
  free(t);
  free(rc);
  free(zc);
}

/* Two iterations of flexible CG on A_m x = b from x = 0, preconditioned by
 * the K-cycle on level m ([NV2008] as cited in Section 3.1). Each direction
 * is made A-orthogonal to the previous one (FCG with truncation 1):
 *   c1 = K(b), v1 = A c1, rho1 = (c1, v1), s1 = (c1, b) / rho1,
 *   r1 = b - s1 v1,
 *   c2 = K(r1), v2 = A c2, gamma = (c2, v1),
 *   d2 = c2 - (gamma / rho1) c1, rho2 = (d2, A d2) = (c2, v2) - gamma^2 / rho1,
 *   s2 = (d2, r1) / rho2 = (c2, r1) / rho2   ((c1, r1) = 0),
 *   x = s1 c1 + s2 d2 = (s1 - s2 gamma / rho1) c1 + s2 c2.
 * A zero rho1 (b = 0) gives x = 0; a non-positive rho2 stops after the first
 * iteration. */
static void fcg2(const orc_hier *h, int32_t m, int32_t pre, int32_t post, const double *b,
                 double *x) {
  const orc_csr *A = &h->A[m];
  int32_t n = A->n;
  double *c1 = (double *)malloc(sizeof(double) * (size_t)n);
  double *v1 = (double *)malloc(sizeof(double) * (size_t)n);
  double *r1 = (double *)malloc(sizeof(double) * (size_t)n);
  double *c2 = (double *)malloc(sizeof(double) * (size_t)n);
  double *v2 = (double *)malloc(sizeof(double) * (size_t)n);
  cycle(h, m, pre, post, 1, b, c1);
  orc_spmv(A, c1, v1);
  double rho1 = dot(n, c1, v1);
  if (!(rho1 > 0.0)) {
    for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
  } else {
    double s1 = dot(n, c1, b) / rho1;
    for (int32_t i = 0; i < n; ++i) r1[i] = b[i] - s1 * v1[i];
    cycle(h, m, pre, post, 1, r1, c2);
    orc_spmv(A, c2, v2);
    double gamma = dot(n, c2, v1);
    double rho2 = dot(n, c2, v2) - gamma * gamma / rho1;
    if (!(rho2 > 0.0)) {
      for (int32_t i = 0; i < n; ++i) x[i] = s1 * c1[i];
    } else {
      double s2 = dot(n, c2, r1) / rho2;
      double a1 = s1 - s2 * (gamma / rho1);
      for (int32_t i = 0; i < n; ++i) x[i] = a1 * c1[i] + s2 * c2[i];
    }
  }
  free(c1);
  free(v1);
  free(r1);
  free(c2);
  free(v2);
}

void orc_vcycle(const orc_hier *h, int32_t l, int32_t pre, int32_t post,
                const double *r, double *z) {
  cycle(h, l, pre, post, 0, r, z);
}

void orc_kcycle(const orc_hier *h, int32_t l, int32_t pre, int32_t post,
                const double *r, double *z) {
  cycle(h, l, pre, post, 1, r, z);
}

void orc_fcg2(const orc_hier *h, int32_t m, int32_t pre, int32_t post, const double *b,
              double *x) {
  fcg2(h, m, pre, post, b, x);
}

int orc_pcg(const orc_hier *h, int32_t pre, int32_t post, const double *b,
            double *x, double rtol, int32_t maxit, double *out) {
  const orc_csr *A = &h->A[0];
  int32_t n = A->n;
  double *r = (double *)malloc(sizeof(double) * (size_t)n);
  double *z = (double *)malloc(sizeof(double) * (size_t)n);
  double *p = (double *)malloc(sizeof(double) * (size_t)n);
  double *q = (double *)malloc(sizeof(double) * (size_t)n);
  int st = ORC_NOT_CONVERGED;
  int32_t it = 0;
  double bnorm = sqrt(dot(n, b, b));
  double rnorm = 0.0;
  if (bnorm == 0.0) {
    for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
    st = ORC_OK;
    goto done;
  }
  orc_spmv(A, x, q);
  for (int32_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
  rnorm = sqrt(dot(n, r, r));
  if (rnorm <= rtol * bnorm) {
    st = ORC_OK;
    goto done;
  }
  orc_vcycle(h, 0, pre, post, r, z);
  for (int32_t i = 0; i < n; ++i) p[i] = z[i];
  double rho = dot(n, r, z);
  for (it = 1; it <= maxit; ++it) {
    orc_spmv(A, p, q);
    double pq = dot(n, p, q);
    if (!(pq > 0.0) || !(rho > 0.0)) {
      st = ORC_ERR_BREAKDOWN;
      --it;
      break;
    }
    double alpha = rho / pq;
    for (int32_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
    for (int32_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
    rnorm = sqrt(dot(n, r, r));
    if (rnorm <= rtol * bnorm) {
      st = ORC_OK;
      break;
    }
    if (it == maxit) break;
    orc_vcycle(h, 0, pre, post, r, z);
    double rz = dot(n, r, z);
    double beta = rz / rho;
    rho = rz;
    for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
  }
  if (it > maxit) it = maxit;
done:
  out[0] = (double)it;
  out[1] = st == ORC_OK ? 1.0 : 0.0;
  out[2] = bnorm > 0.0 ? rnorm / bnorm : 0.0;
  if (bnorm > 0.0) {
    orc_spmv(A, x, q);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    out[3] = sqrt(dot(n, r, r)) / bnorm;
  } else {
    out[3] = 0.0;
  }
  free(r);
  free(z);
  free(p);
  free(q);
  return st;
}

/* Flexible CG (Section 5 uses FCG as the outer solver) with truncation 1:
 * p_k = z_k - ((z_k, A p_{k-1}) / (p_{k-1}, A p_{k-1})) p_{k-1},
 * alpha_k = (p_k, r_k) / (p_k, A p_k); same start, stop test and outputs as
 * orc_pcg. With a fixed s.p.d. preconditioner it coincides with PCG in exact
 * arithmetic; it is the outer solver of the K-cycle, which is not a fixed
 * linear operator. kcycle selects the preconditioner (0: V-cycle). */
int orc_fcg(const orc_hier *h, int32_t kcycle, int32_t pre, int32_t post, const double *b,
            double *x, double rtol, int32_t maxit, double *out) {
  const orc_csr *A = &h->A[0];
  int32_t n = A->n;
  double *r = (double *)malloc(sizeof(double) * (size_t)n);
  double *z = (double *)malloc(sizeof(double) * (size_t)n);
  double *p = (double *)malloc(sizeof(double) * (size_t)n);
  double *q = (double *)malloc(sizeof(double) * (size_t)n);
  int st = ORC_NOT_CONVERGED;
  int32_t it = 0;
  double bnorm = sqrt(dot(n, b, b));
  double rnorm = 0.0;
  if (bnorm == 0.0) {
    for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
    st = ORC_OK;
    goto done;
  }
  orc_spmv(A, x, q);
  for (int32_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
  rnorm = sqrt(dot(n, r, r));
  if (rnorm <= rtol * bnorm) {
    st = ORC_OK;
    goto done;
  }
  cycle(h, 0, pre, post, kcycle, r, z);
  for (int32_t i = 0; i < n; ++i) p[i] = z[i];
  for (it = 1; it <= maxit; ++it) {
    orc_spmv(A, p, q);
    double pq = dot(n, p, q);
    if (!(pq > 0.0)) {
      st = ORC_ERR_BREAKDOWN;
      --it;
      break;
    }
    double alpha = dot(n, p, r) / pq;
    for (int32_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
    for (int32_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
    rnorm = sqrt(dot(n, r, r));
    if (rnorm <= rtol * bnorm) {
      st = ORC_OK;
      break;
    }
    if (it == maxit) break;
    cycle(h, 0, pre, post, kcycle, r, z);
    double beta = -dot(n, z, q) / pq;
    for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
  }
  if (it > maxit) it = maxit;
done:
  out[0] = (double)it;
  out[1] = st == ORC_OK ? 1.0 : 0.0;
  out[2] = bnorm > 0.0 ? rnorm / bnorm : 0.0;
  if (bnorm > 0.0) {
    orc_spmv(A, x, q);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    out[3] = sqrt(dot(n, r, r)) / bnorm;
  } else {
    out[3] = 0.0;
  }
  free(r);
  free(z);
  free(p);
  free(q);
  return st;
}
