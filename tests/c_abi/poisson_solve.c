/* A plain C caller of the library (include/amg.h): builds the 7-point
 * Dirichlet Laplacian on an N^3 grid (Section 4's model problem) on the host,
 * copies it to the device with the HIP runtime, builds the hierarchy, solves
 * A x = A u to rtol 1e-8 with the V-cycle and with the K-cycle, and prints
 * one line per solve. Exit status 0 when both converge. */
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

static int solve_with(const amg_csr *A, int cycle, const double *db, double *dx, int64_t n) {
  amg_params p;
  amg_params_default(&p);
  p.cycle = cycle;
  amg_hierarchy *h = NULL;
  amg_status st = amg_setup(A, &p, &h);
  if (st != AMG_OK) {
    fprintf(stderr, "amg_setup: %s\n", amg_status_string(st));
    return 1;
  }
  int32_t nlev = 0;
  amg_num_levels(h, &nlev);
  CHECK_HIP(hipMemset(dx, 0, sizeof(double) * (size_t)n));
  amg_solve_info info;
  st = amg_pcg_solve(h, db, dx, 1e-8, 500, &info);
  printf("cycle=%s levels=%d iterations=%d converged=%d rel_res_true=%.3e\n",
         cycle == AMG_CYCLE_K ? "K" : "V", nlev, info.iterations, info.converged,
         info.rel_res_true);
  amg_free(h);
  return st == AMG_OK && info.converged && info.rel_res_true <= 1.001e-8 ? 0 : 1;
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
  int rc = solve_with(&A, AMG_CYCLE_V, db, dx, n);
  rc |= solve_with(&A, AMG_CYCLE_K, db, dx, n);
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
