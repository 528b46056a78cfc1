/* A plain C caller of the library (include/amg.h): builds the 7-point
 * Dirichlet Laplacian on an N^3 grid (Section 4's model problem) on the host,
 * copies it to the device with the HIP runtime, builds the hierarchy, solves
 * A x = A u to rtol 1e-8 with the V-cycle, with the K-cycle and with the
 * V-cycle as a non-blocking solve (AMG_ASYNC, amg_query, amg_wait) on an
 * explicitly named device (amg_params.device), and prints one line per
 * solve. For even N it also checks the level-0 aggregates (amg_get_aggregates)
 * against the 2 x 2 x 2 cubes that the matching gives on this problem.
 * Exit status 0 when every solve converges and every check holds. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "amg.h"

#define CHECK_HIP(x)                                        \
  do {                                                      \
    if ((x) != hipSuccess) {                                \
      fprintf(stderr, "HIP error at line %d\n", __LINE__);  \
      return 2;                                             \
    }                                                       \
  } while (0)

/* 1 when the level-0 aggregates are the 2 x 2 x 2 cubes numbered in the
 * order of their smallest member (N even). */
static int cubes_ok(amg_hierarchy *h, int N) {
  const int64_t n = (int64_t)N * N * N;
  int32_t *agg = malloc(sizeof(int32_t) * (size_t)n);
  if (!agg || amg_get_aggregates(h, 0, agg) != AMG_OK) {
    free(agg);
    return 0;
  }
  int ok = 1;
  const int H = N / 2;
  for (int64_t i = 0; i < n && ok; ++i) {
    const int x = (int)(i % N), y = (int)((i / N) % N), z = (int)(i / ((int64_t)N * N));
    ok = agg[i] == x / 2 + H * (y / 2 + H * (z / 2));
  }
  free(agg);
  return ok;
}

static int solve_with(const amg_csr *A, int cycle, int async, const double *db, double *dx,
                      int N) {
  const int64_t n = (int64_t)N * N * N;
  amg_params p;
  amg_params_default(&p);
  p.cycle = cycle;
  if (async) {
    p.flags |= AMG_ASYNC;
    CHECK_HIP(hipGetDevice(&p.device));
  }
  amg_hierarchy *h = NULL;
  amg_status st = amg_setup(A, &p, &h);
  if (st != AMG_OK) {
    fprintf(stderr, "amg_setup: %s\n", amg_status_string(st));
    return 1;
  }
  int32_t nlev = 0;
  amg_num_levels(h, &nlev);
  const int agg_ok = N % 2 == 1 || cubes_ok(h, N);
  CHECK_HIP(hipMemset(dx, 0, sizeof(double) * (size_t)n));
  amg_solve_info info;
  int polls = 0;
  st = amg_pcg_solve(h, db, dx, 1e-8, 500, &info);
  if (async && st == AMG_OK) {
    int32_t done = 0;
    while (amg_query(h, &done) == AMG_OK && !done) ++polls;
    st = amg_wait(h);
  }
  printf("cycle=%s%s levels=%d iterations=%d converged=%d rel_res_true=%.3e aggregates=%s\n",
         cycle == AMG_CYCLE_K ? "K" : "V", async ? " async" : "", nlev, info.iterations,
         info.converged, info.rel_res_true, agg_ok ? "cubes" : "WRONG");
  amg_free(h);
  return st == AMG_OK && info.converged && info.rel_res_true <= 1.001e-8 && agg_ok ? 0 : 1;
}

int main(int argc, char **argv) {
  const int N = argc > 1 ? atoi(argv[1]) : 24;
  const int64_t n = (int64_t)N * N * N;
  int32_t *rp = malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t *ci = malloc(sizeof(int32_t) * (size_t)(7 * n));
  double *va = malloc(sizeof(double) * (size_t)(7 * n));
  double *u = malloc(sizeof(double) * (size_t)n), *b = malloc(sizeof(double) * (size_t)n);
  int64_t nnz = 0;
  for (int z = 0; z < N; ++z)
    for (int y = 0; y < N; ++y)
      for (int x = 0; x < N; ++x) {
        const int64_t i = x + (int64_t)N * (y + (int64_t)N * z);
        rp[i] = (int32_t)nnz;
        const int64_t nb[7] = {z > 0 ? i - (int64_t)N * N : -1, y > 0 ? i - N : -1,
                               x > 0 ? i - 1 : -1,          i,
                               x < N - 1 ? i + 1 : -1,      y < N - 1 ? i + N : -1,
                               z < N - 1 ? i + (int64_t)N * N : -1};
        for (int k = 0; k < 7; ++k) {
          if (nb[k] < 0) continue;
          ci[nnz] = (int32_t)nb[k];
          va[nnz] = nb[k] == i ? 6.0 : -1.0;
          ++nnz;
        }
        u[i] = sin(0.1 * (double)i);
      }
  rp[n] = (int32_t)nnz;
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) s += va[k] * u[ci[k]];
    b[i] = s;
  }
  int32_t *drp, *dci;
  double *dva, *db, *dx;
  CHECK_HIP(hipMalloc((void **)&drp, sizeof(int32_t) * (size_t)(n + 1)));
  CHECK_HIP(hipMalloc((void **)&dci, sizeof(int32_t) * (size_t)nnz));
  CHECK_HIP(hipMalloc((void **)&dva, sizeof(double) * (size_t)nnz));
  CHECK_HIP(hipMalloc((void **)&db, sizeof(double) * (size_t)n));
  CHECK_HIP(hipMalloc((void **)&dx, sizeof(double) * (size_t)n));
  CHECK_HIP(hipMemcpy(drp, rp, sizeof(int32_t) * (size_t)(n + 1), hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(dci, ci, sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(dva, va, sizeof(double) * (size_t)nnz, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(db, b, sizeof(double) * (size_t)n, hipMemcpyHostToDevice));
  amg_csr A = {n, nnz, drp, dci, dva};
  int rc = solve_with(&A, AMG_CYCLE_V, 0, db, dx, N);
  rc |= solve_with(&A, AMG_CYCLE_K, 0, db, dx, N);
  rc |= solve_with(&A, AMG_CYCLE_V, 1, db, dx, N);
  hipFree(drp);
  hipFree(dci);
  hipFree(dva);
  hipFree(db);
  hipFree(dx);
  free(rp);
  free(ci);
  free(va);
  free(u);
  free(b);
  return rc;
}
