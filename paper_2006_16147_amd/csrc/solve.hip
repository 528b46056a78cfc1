// Solve phase: V-cycle of eq. (amg) with l1-Jacobi smoothing (Section 3.3)
// inside preconditioned CG (Section 5), on one gfx950 GPU.
//
// Every level is stored as sliced ELLPACK with 64-row slices (one slice per
// wavefront, column-major inside the slice), so lane i of a wavefront loads
// row i's k-th value and column index from consecutive addresses; the 7-point
// rows waste about 0.5% to padding. The streaming kernels are HBM-bound:
// each keeps one row per lane and touches every array once.
//
// Kernels of one V-cycle level l < L (zero initial guess):
//   pre_residual : z = M^-1 r ; t = r - A z        (one SpMV, z gathered as r/m)
//   restrict     : r_c = P^T t                     (members in ascending order)
//   ...            level l + 1 ...
//   prolong      : z += P z_c
//   post         : y = z + M^-1 (r - A z)          (one SpMV; on level 0 it
//                                                   also forms (r, y) for CG)
// and on level L a dense solve with the inverse Cholesky factor.
//
// CG scalars live on the device; reductions are two-stage and
// deterministic: each block writes a partial, the last block to arrive sums
// the partials in a fixed order and updates the scalars. Kernels of an
// iteration read a device flag and return at once after convergence, so the
// host can queue several iterations between checks.

#include <chrono>
#include <cmath>

#include "internal.h"

namespace amg {

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// ---------------------------------------------------------------------------
// launch geometry: each block handles a contiguous chunk of rows
// ---------------------------------------------------------------------------

struct Geom {
  int32_t grid;
  int32_t chunk;  // rows per block, a multiple of kBlock
};

Geom geom(int64_t n, bool reduce) {
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks < 1) blocks = 1;
  if (reduce && blocks > kMaxReduceBlocks) {
    int64_t chunk = ((n + kMaxReduceBlocks - 1) / kMaxReduceBlocks + kBlock - 1) / kBlock * kBlock;
    return {ceil_div(n, chunk), (int32_t)chunk};
  }
  return {(int32_t)blocks, kBlock};
}

__device__ __forceinline__ void rows_of_block(int32_t n, int32_t chunk, int32_t *b, int32_t *e) {
  const int32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t bb = (int64_t)lb * chunk;
  *b = (int32_t)bb;
  *e = (int32_t)(bb + chunk < n ? bb + chunk : n);
}

// ---------------------------------------------------------------------------
// deterministic two-stage reductions
// ---------------------------------------------------------------------------

template <int NV>
__device__ void block_sum(double (&v)[NV], double (*sh)[kBlock / kWave]) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double x = v[q];
    for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_down(x, o, kWave);
    if (lane == 0) sh[q][wid] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = sh[q][0];
      for (int k = 1; k < kBlock / kWave; ++k) s += sh[q][k];
      v[q] = s;
    }
  }
}

// Writes this block's partials; returns true in the last block to arrive,
// whose thread 0 then holds the grid totals in v (summed in block order).
template <int NV>
__device__ bool grid_sum(double (&v)[NV], double *partials, unsigned *ticket) {
  __shared__ double sh[NV][kBlock / kWave];
  __shared__ bool last;
  block_sum<NV>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) partials[q * kMaxReduceBlocks + blockIdx.x] = v[q];
    __threadfence();
    const unsigned t = atomicAdd(ticket, 1u);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  // fixed-order sum of the partials: thread k sums blocks k, k+256, ...,
  // then a fixed tree over threads
  double acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock)
      s += partials[q * kMaxReduceBlocks + b];
    acc[q] = s;
  }
  block_sum<NV>(acc, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = acc[q];
    *ticket = 0u;
  }
  return true;
}

// ---------------------------------------------------------------------------
// SELL construction and precision demotion
// ---------------------------------------------------------------------------

__global__ void k_sell_width(int32_t n, int32_t ns, const int32_t *rp, int32_t *w64) {
  const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  const int32_t r0 = s * kSlice, r1 = min(n, r0 + kSlice);
  int32_t w = 0;
  for (int32_t r = r0; r < r1; ++r) w = max(w, rp[r + 1] - rp[r]);
  w64[s] = w * kSlice;
}

__global__ void k_sell_fill(int32_t n, int32_t ns, const int32_t *rp, const int32_t *ci,
                            const double *val, const int32_t *sptr, int32_t *col, double *v64,
                            float *v32) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= (int64_t)ns * kSlice) return;
  const int32_t s = (int32_t)(r / kSlice), lane = (int32_t)(r % kSlice);
  const int32_t base = sptr[s], w = (sptr[s + 1] - base) / kSlice;
  const int32_t b = r < n ? rp[r] : 0, len = r < n ? rp[r + 1] - b : 0;
  for (int32_t k = 0; k < w; ++k) {
    const int64_t idx = base + (int64_t)k * kSlice + lane;
    const bool real = k < len;
    const double a = real ? val[b + k] : 0.0;
    col[idx] = real ? ci[b + k] : (r < n ? (int32_t)r : 0);
    if (v64) v64[idx] = a;
    if (v32) v32[idx] = (float)a;
  }
}

__global__ void k_demote(int64_t n, const double *a, float *b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// ---------------------------------------------------------------------------
// V-cycle kernels. TV: hierarchy precision; TR: type of the level's right-hand
// side (double on level 0, TV below); TO: type of the level's output.
// ---------------------------------------------------------------------------

template <typename TV>
__device__ __forceinline__ void sell_slice(const int32_t *sptr, int32_t row, int32_t *base,
                                           int32_t *w) {
  const int32_t s = row / kSlice;
  *base = sptr[s] + (row % kSlice);
  *w = (sptr[s + 1] - sptr[s]) / kSlice;
}

// z = M^-1 r ; t = r - A z  (z_j gathered as r_j m_j^-1)
template <typename TV, typename TR>
__global__ void __launch_bounds__(kBlock) k_pre_residual(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const TV *__restrict__ val, const TV *__restrict__ minv, const TR *__restrict__ r,
    TV *__restrict__ z, TV *__restrict__ t, const int32_t *__restrict__ done) {
  if (*done) return;
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  for (int32_t row = rb + threadIdx.x; row < re; row += kBlock) {
    int32_t base, w;
    sell_slice<TV>(sptr, row, &base, &w);
    TV acc = 0;
    for (int32_t k = 0; k < w; ++k) {
      const int32_t idx = base + k * kSlice;
      const int32_t j = col[idx];
      acc += val[idx] * ((TV)r[j] * minv[j]);
    }
    const TV ri = (TV)r[row];
    z[row] = ri * minv[row];
    t[row] = ri - acc;
  }
}

// y = z + M^-1 (r - A z); with DOT also (r, y) for CG (rho / beta update)
template <typename TV, typename TR, typename TO, bool DOT>
__global__ void __launch_bounds__(kBlock) k_post(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const TV *__restrict__ val, const TV *__restrict__ minv, const TR *__restrict__ r,
    const TV *__restrict__ z, TO *__restrict__ y, double *partials, unsigned *ticket,
    PcgScal *scal, const int32_t *__restrict__ done) {
  if (*done) return;
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  double d[1] = {0.0};
  for (int32_t row = rb + threadIdx.x; row < re; row += kBlock) {
    int32_t base, w;
    sell_slice<TV>(sptr, row, &base, &w);
    TV acc = 0;
    for (int32_t k = 0; k < w; ++k) {
      const int32_t idx = base + k * kSlice;
      acc += val[idx] * z[col[idx]];
    }
    const TR rr = r[row];
    const TO yo = (TO)(z[row] + ((TV)rr - acc) * minv[row]);
    y[row] = yo;
    if (DOT) d[0] += (double)rr * (double)yo;
  }
  if (DOT) {
    if (grid_sum<1>(d, partials, ticket) && threadIdx.x == 0) {
      const double rz = d[0];
      if (!(rz > 0.0)) {
        scal->done = 3;
      } else if (scal->phase == 0) {
        scal->rho = rz;
        scal->phase = 1;
      } else {
        scal->beta = rz / scal->rho;
        scal->rho = rz;
      }
    }
  }
}

// extra smoothing sweep: y = z + M^-1 (r - A z) (no reduction)
// (k_post with DOT = false)

// z = M^-1 r (first of several pre-smoothing sweeps)
template <typename TV, typename TR>
__global__ void k_jacobi0(int32_t n, const TV *minv, const TR *r, TV *z, const int32_t *done) {
  if (*done) return;
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = (TV)r[i] * minv[i];
}

// t = r - A z
template <typename TV, typename TR>
__global__ void __launch_bounds__(kBlock) k_residual(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const TV *__restrict__ val, const TR *__restrict__ r, const TV *__restrict__ z,
    TV *__restrict__ t, const int32_t *__restrict__ done) {
  if (*done) return;
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  for (int32_t row = rb + threadIdx.x; row < re; row += kBlock) {
    int32_t base, w;
    sell_slice<TV>(sptr, row, &base, &w);
    TV acc = 0;
    for (int32_t k = 0; k < w; ++k) {
      const int32_t idx = base + k * kSlice;
      acc += val[idx] * z[col[idx]];
    }
    t[row] = (TV)r[row] - acc;
  }
}

// r_c(I) = sum over members i of I (ascending) of p_i t_i
template <typename TV>
__global__ void k_restrict(int32_t nc, const int32_t *__restrict__ mptr,
                           const int32_t *__restrict__ mem, const TV *__restrict__ pm,
                           const TV *__restrict__ t, TV *__restrict__ rc,
                           const int32_t *__restrict__ done) {
  if (*done) return;
  const int32_t I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int32_t b = mptr[I], e = mptr[I + 1];
  TV s = 0;
  for (int32_t k = b; k < e; ++k) s += pm[k] * t[mem[k]];
  rc[I] = s;
}

// z += P z_c
template <typename TV>
__global__ void k_prolong(int32_t n, const int32_t *__restrict__ agg, const TV *__restrict__ p,
                          const TV *__restrict__ zc, TV *__restrict__ z,
                          const int32_t *__restrict__ done) {
  if (*done) return;
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] += p[i] * zc[agg[i]];
}

// coarsest level: z = L^-T (L^-1 r) in one workgroup (n <= AMG_MAX_DENSE)
template <typename TI, typename TO>
__global__ void __launch_bounds__(1024) k_coarse_solve(int32_t n, const double *__restrict__ Linv,
                                                       const double *__restrict__ LinvT,
                                                       const TI *__restrict__ r,
                                                       TO *__restrict__ z,
                                                       const int32_t *__restrict__ done) {
  extern __shared__ double sm[];
  if (*done) return;
  double *rs = sm, *ys = sm + n;
  for (int32_t i = threadIdx.x; i < n; i += blockDim.x) rs[i] = (double)r[i];
  __syncthreads();
  for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
    double y = 0.0;
    for (int32_t k = 0; k <= i; ++k) y += LinvT[(int64_t)k * n + i] * rs[k];
    ys[i] = y;
  }
  __syncthreads();
  for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
    double s = 0.0;
    for (int32_t k = i; k < n; ++k) s += Linv[(int64_t)k * n + i] * ys[k];
    z[i] = (TO)s;
  }
}

// (r, z) for CG when the V-cycle has no post-smoother on level 0 to fuse it into
__global__ void __launch_bounds__(kBlock) k_dot_rz(int32_t n, int32_t chunk, const double *r,
                                                   const double *z, double *partials,
                                                   unsigned *ticket, PcgScal *scal,
                                                   const int32_t *done) {
  if (*done) return;
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  double d[1] = {0.0};
  for (int32_t i = rb + threadIdx.x; i < re; i += kBlock) d[0] += r[i] * z[i];
  if (grid_sum<1>(d, partials, ticket) && threadIdx.x == 0) {
    const double rz = d[0];
    if (!(rz > 0.0)) {
      scal->done = 3;
    } else if (scal->phase == 0) {
      scal->rho = rz;
      scal->phase = 1;
    } else {
      scal->beta = rz / scal->rho;
      scal->rho = rz;
    }
  }
}

// ---------------------------------------------------------------------------
// outer CG kernels (FP64)
// ---------------------------------------------------------------------------

__global__ void k_scal_init(PcgScal *s, double rtol, int32_t maxit) {
  s->rho = 0.0;
  s->pq = 0.0;
  s->alpha = 0.0;
  s->beta = 0.0;
  s->rr = 0.0;
  s->bb = 0.0;
  s->rtol = rtol;
  s->tol2 = 0.0;
  s->rr_true = 0.0;
  s->iter = 0;
  s->maxit = maxit;
  s->done = 0;
  s->phase = 0;
}

__device__ __forceinline__ bool converged(double rr, double bb, double rtol) {
  return sqrt(rr) <= rtol * sqrt(bb);
}

// r = b - A x ; (b, b), (r, r)
__global__ void __launch_bounds__(kBlock) k_init_residual(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ b, const double *__restrict__ x,
    double *__restrict__ r, double *partials, unsigned *ticket, PcgScal *scal) {
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  double d[2] = {0.0, 0.0};
  for (int32_t row = rb + threadIdx.x; row < re; row += kBlock) {
    int32_t base, w;
    sell_slice<double>(sptr, row, &base, &w);
    double acc = 0.0;
    for (int32_t k = 0; k < w; ++k) {
      const int32_t idx = base + k * kSlice;
      acc += val[idx] * x[col[idx]];
    }
    const double bi = b[row];
    const double ri = bi - acc;
    r[row] = ri;
    d[0] += bi * bi;
    d[1] += ri * ri;
  }
  if (grid_sum<2>(d, partials, ticket) && threadIdx.x == 0) {
    const double rtol = scal->rtol;
    scal->bb = d[0];
    scal->rr = d[1];
    scal->tol2 = rtol * rtol * d[0];
    if (d[0] == 0.0) scal->done = 4;
    else if (converged(d[1], d[0], rtol)) scal->done = 1;
    else if (scal->maxit <= 0) scal->done = 2;
  }
}

// ||b - A x||^2 at exit
__global__ void __launch_bounds__(kBlock) k_true_residual(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ b, const double *__restrict__ x,
    double *partials, unsigned *ticket, PcgScal *scal) {
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  double d[1] = {0.0};
  for (int32_t row = rb + threadIdx.x; row < re; row += kBlock) {
    int32_t base, w;
    sell_slice<double>(sptr, row, &base, &w);
    double acc = 0.0;
    for (int32_t k = 0; k < w; ++k) {
      const int32_t idx = base + k * kSlice;
      acc += val[idx] * x[col[idx]];
    }
    const double ri = b[row] - acc;
    d[0] += ri * ri;
  }
  if (grid_sum<1>(d, partials, ticket) && threadIdx.x == 0) scal->rr_true = d[0];
}

__global__ void k_zero_if_zero_rhs(int32_t n, double *x, const PcgScal *scal) {
  if (scal->done != 4) return;
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

// q = A p ; (p, q) ; alpha = rho / (p, q)
__global__ void __launch_bounds__(kBlock) k_spmv_dot(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ p, double *__restrict__ q,
    double *partials, unsigned *ticket, PcgScal *scal, const int32_t *__restrict__ done) {
  if (*done) return;
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  double d[1] = {0.0};
  for (int32_t row = rb + threadIdx.x; row < re; row += kBlock) {
    int32_t base, w;
    sell_slice<double>(sptr, row, &base, &w);
    double acc = 0.0;
    for (int32_t k = 0; k < w; ++k) {
      const int32_t idx = base + k * kSlice;
      acc += val[idx] * p[col[idx]];
    }
    q[row] = acc;
    d[0] += p[row] * acc;
  }
  if (grid_sum<1>(d, partials, ticket) && threadIdx.x == 0) {
    const double pq = d[0];
    scal->pq = pq;
    if (!(pq > 0.0)) scal->done = 3;
    else scal->alpha = scal->rho / pq;
  }
}

// x += alpha p ; r -= alpha q ; (r, r) ; stop test
__global__ void __launch_bounds__(kBlock) k_update_xr(int32_t n, int32_t chunk,
                                                      double *__restrict__ x,
                                                      double *__restrict__ r,
                                                      const double *__restrict__ p,
                                                      const double *__restrict__ q,
                                                      double *partials, unsigned *ticket,
                                                      PcgScal *scal,
                                                      const int32_t *__restrict__ done) {
  if (*done) return;
  const double alpha = scal->alpha;
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  double d[1] = {0.0};
  for (int32_t i = rb + threadIdx.x; i < re; i += kBlock) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    d[0] += ri * ri;
  }
  if (grid_sum<1>(d, partials, ticket) && threadIdx.x == 0) {
    scal->rr = d[0];
    scal->iter += 1;
    if (converged(d[0], scal->bb, scal->rtol)) scal->done = 1;
    else if (scal->iter >= scal->maxit) scal->done = 2;
  }
}

// p = z + beta p
__global__ void k_xpay(int32_t n, const double *__restrict__ z, double *__restrict__ p,
                       const PcgScal *__restrict__ scal, const int32_t *__restrict__ done) {
  if (*done) return;
  const double beta = scal->beta;
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = z[i] + beta * p[i];
}

__global__ void k_copy(int32_t n, const double *__restrict__ z, double *__restrict__ p,
                       const int32_t *__restrict__ done) {
  if (*done) return;
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = z[i];
}

inline int32_t grid1(int64_t n) { return ceil_div(n > 0 ? n : 1, kBlock); }

// ---------------------------------------------------------------------------
// host: V-cycle for one hierarchy precision
// ---------------------------------------------------------------------------

template <typename TV>
const TV *vals(const Level &L);
template <>
const double *vals<double>(const Level &L) { return L.S.v64; }
template <>
const float *vals<float>(const Level &L) { return L.S.v32; }
template <typename TV>
const TV *minv(const Level &L);
template <>
const double *minv<double>(const Level &L) { return L.minv64; }
template <>
const float *minv<float>(const Level &L) { return L.minv32; }
template <typename TV>
const TV *pvals(const Level &L);
template <>
const double *pvals<double>(const Level &L) { return L.p64; }
template <>
const float *pvals<float>(const Level &L) { return L.p32; }
template <typename TV>
const TV *pmvals(const Level &L);
template <>
const double *pmvals<double>(const Level &L) { return L.pm64; }
template <>
const float *pmvals<float>(const Level &L) { return L.pm32; }

// pre-smoothing (nu sweeps) + residual on level l: z_l, t_l from right-hand side r
template <typename TV, typename TR>
void launch_down(amg_hierarchy *h, int32_t l, const TR *r, const int32_t *done) {
  hipStream_t s = h->stream;
  Level &L = h->lv[l];
  TV *z = (TV *)L.z, *t = (TV *)L.t, *y = (TV *)L.y;
  const Geom g = geom(L.n, false);
  const int32_t pre = h->params.pre;
  if (pre == 1) {
    k_pre_residual<TV, TR><<<g.grid, kBlock, 0, s>>>(L.n, g.chunk, L.S.sptr, L.S.col, vals<TV>(L),
                                                   minv<TV>(L), r, z, t, done);
    return;
  }
  k_jacobi0<TV, TR><<<grid1(L.n), kBlock, 0, s>>>(L.n, minv<TV>(L), r, z, done);
  for (int32_t k = 1; k < pre; ++k) {
    k_post<TV, TR, TV, false><<<g.grid, kBlock, 0, s>>>(L.n, g.chunk, L.S.sptr, L.S.col,
                                                       vals<TV>(L), minv<TV>(L), r, z, y,
                                                       nullptr, nullptr, nullptr, done);
    std::swap(L.z, L.y);
    z = (TV *)L.z;
    y = (TV *)L.y;
  }
  k_residual<TV, TR><<<g.grid, kBlock, 0, s>>>(L.n, g.chunk, L.S.sptr, L.S.col, vals<TV>(L), r, z,
                                             t, done);
}

// prolongation + post-smoothing on level l; output to `out`
template <typename TV, typename TR, typename TO>
void launch_up(amg_hierarchy *h, int32_t l, const TR *r, const TV *zc, TO *out, bool dot,
               const int32_t *done) {
  hipStream_t s = h->stream;
  Level &L = h->lv[l];
  TV *z = (TV *)L.z, *y = (TV *)L.y;
  k_prolong<TV><<<grid1(L.n), kBlock, 0, s>>>(L.n, L.agg, pvals<TV>(L), zc, z, done);
  const int32_t post = h->params.post;
  for (int32_t k = 0; k + 1 < post; ++k) {
    const Geom g = geom(L.n, false);
    k_post<TV, TR, TV, false><<<g.grid, kBlock, 0, s>>>(L.n, g.chunk, L.S.sptr, L.S.col,
                                                       vals<TV>(L), minv<TV>(L), r, z, y,
                                                       nullptr, nullptr, nullptr, done);
    std::swap(L.z, L.y);
    z = (TV *)L.z;
    y = (TV *)L.y;
  }
  const Geom g = geom(L.n, dot);
  if (dot)
    k_post<TV, TR, TO, true><<<g.grid, kBlock, 0, s>>>(L.n, g.chunk, L.S.sptr, L.S.col,
                                                      vals<TV>(L), minv<TV>(L), r, z, out,
                                                      h->partials, h->ticket, h->scal, done);
  else
    k_post<TV, TR, TO, false><<<g.grid, kBlock, 0, s>>>(L.n, g.chunk, L.S.sptr, L.S.col,
                                                       vals<TV>(L), minv<TV>(L), r, z, out,
                                                       nullptr, nullptr, nullptr, done);
}

template <typename TI, typename TO>
void launch_coarse(amg_hierarchy *h, const TI *r, TO *z, const int32_t *done) {
  const int32_t n = h->C.n;
  const int threads = n <= 64 ? 64 : (n <= 256 ? 256 : 1024);
  k_coarse_solve<TI, TO><<<1, threads, sizeof(double) * 2 * n, h->stream>>>(
      n, h->C.Linv, h->C.LinvT, r, z, done);
}

template <typename TV>
void vcycle_t(amg_hierarchy *h, const double *r0, double *z0, bool dot, const int32_t *done) {
  const int32_t L = (int32_t)h->lv.size() - 1;
  if (L == 0) {
    launch_coarse<double, double>(h, r0, z0, done);
    if (dot) {
      const Geom g = geom(h->lv[0].n, true);
      k_dot_rz<<<g.grid, kBlock, 0, h->stream>>>(h->lv[0].n, g.chunk, r0, z0, h->partials,
                                                 h->ticket, h->scal, done);
    }
    return;
  }
  // down
  launch_down<TV, double>(h, 0, r0, done);
  for (int32_t l = 0; l < L; ++l) {
    Level &F = h->lv[l];
    Level &C = h->lv[l + 1];
    k_restrict<TV><<<grid1(C.n), kBlock, 0, h->stream>>>(C.n, F.mptr, F.mem, pmvals<TV>(F),
                                                         (const TV *)F.t, (TV *)C.r, done);
    if (l + 1 < L) launch_down<TV, TV>(h, l + 1, (const TV *)C.r, done);
  }
  // coarsest
  launch_coarse<TV, TV>(h, (const TV *)h->lv[L].r, (TV *)h->lv[L].y, done);
  // up
  for (int32_t l = L - 1; l >= 1; --l)
    launch_up<TV, TV, TV>(h, l, (const TV *)h->lv[l].r, (const TV *)h->lv[l + 1].y,
                          (TV *)h->lv[l].y, false, done);
  launch_up<TV, double, double>(h, 0, r0, (const TV *)h->lv[1].y, z0, dot, done);
}

amg_status alloc_level_vectors(amg_hierarchy *h, Level &L, size_t vbytes) {
  AMG_TRY(dev_alloc(h, &L.r, vbytes * L.n + 16));
  AMG_TRY(dev_alloc(h, &L.z, vbytes * L.n + 16));
  AMG_TRY(dev_alloc(h, &L.t, vbytes * L.n + 16));
  AMG_TRY(dev_alloc(h, &L.y, vbytes * L.n + 16));
  return AMG_OK;
}

}  // namespace

amg_status build_solve_formats(amg_hierarchy *h) {
  hipStream_t s = h->stream;
  const bool fp32 = h->params.precision == AMG_FP32;
  const size_t vbytes = fp32 ? sizeof(float) : sizeof(double);
  const int32_t nlev = (int32_t)h->lv.size();
  for (int32_t l = 0; l < nlev; ++l) {
    Level &L = h->lv[l];
    const bool coarsest = (l == nlev - 1);
    // level 0 always needs the FP64 SELL for the outer CG; the V-cycle levels
    // need the hierarchy precision; the coarsest uses its dense factor only
    const bool need64 = (l == 0) || (!coarsest && !fp32);
    const bool need32 = !coarsest && fp32;
    if (need64 || need32) {
      Sell &S = L.S;
      S.n = L.n;
      S.nslices = ceil_div(L.n, kSlice);
      int32_t *w64;
      AMG_HIP(hipMallocAsync(reinterpret_cast<void **>(&w64), sizeof(int32_t) * S.nslices + 16, s));
      AMG_TRY(dalloc(h, &S.sptr, (size_t)S.nslices + 1));
      k_sell_width<<<grid1(S.nslices), kBlock, 0, s>>>(L.n, S.nslices, L.rp, w64);
      AMG_TRY(scan_exclusive_i32(w64, S.sptr, S.nslices, s));
      AMG_HIP(hipFreeAsync(w64, s));
      int32_t padded = 0;
      AMG_HIP(hipMemcpyAsync(&padded, S.sptr + S.nslices, sizeof(int32_t),
                             hipMemcpyDeviceToHost, s));
      AMG_HIP(hipStreamSynchronize(s));
      S.nnz_padded = padded;
      AMG_TRY(dalloc(h, &S.col, (size_t)padded));
      if (need64) AMG_TRY(dalloc(h, &S.v64, (size_t)padded));
      if (need32) AMG_TRY(dalloc(h, &S.v32, (size_t)padded));
      k_sell_fill<<<ceil_div((int64_t)S.nslices * kSlice, kBlock), kBlock, 0, s>>>(
          L.n, S.nslices, L.rp, L.ci, L.val, S.sptr, S.col, S.v64, S.v32);
    }
    if (!coarsest) {
      if (fp32) {
        AMG_TRY(dalloc(h, &L.minv32, (size_t)L.n));
        AMG_TRY(dalloc(h, &L.p32, (size_t)L.n));
        AMG_TRY(dalloc(h, &L.pm32, (size_t)L.n));
        k_demote<<<grid1(L.n), kBlock, 0, s>>>(L.n, L.minv64, L.minv32);
        k_demote<<<grid1(L.n), kBlock, 0, s>>>(L.n, L.p64, L.p32);
        k_demote<<<grid1(L.n), kBlock, 0, s>>>(L.n, L.pm64, L.pm32);
      }
    }
    AMG_TRY(alloc_level_vectors(h, L, vbytes));
  }
  // outer CG vectors and scalars
  const int32_t n0 = h->lv[0].n;
  AMG_TRY(dalloc(h, &h->r, (size_t)n0));
  AMG_TRY(dalloc(h, &h->z, (size_t)n0));
  AMG_TRY(dalloc(h, &h->p, (size_t)n0));
  AMG_TRY(dalloc(h, &h->q, (size_t)n0));
  AMG_TRY(dalloc(h, &h->partials, (size_t)kMaxReduceBlocks * 4));
  AMG_TRY(dalloc(h, &h->ticket, 4));
  AMG_TRY(dalloc(h, &h->scal, 1));
  AMG_TRY(dalloc(h, &h->zero_flag, 4));
  AMG_HIP(hipMemsetAsync(h->ticket, 0, sizeof(unsigned) * 4, s));
  AMG_HIP(hipMemsetAsync(h->zero_flag, 0, sizeof(int32_t) * 4, s));
  AMG_HIP(hipMemsetAsync(h->scal, 0, sizeof(PcgScal), s));
  if (!h->scal_host) AMG_HIP(hipHostMalloc(reinterpret_cast<void **>(&h->scal_host), sizeof(PcgScal)));
  return AMG_OK;
}

amg_status vcycle(amg_hierarchy *h, const double *r, double *z, bool fuse_dot,
                  const int32_t *done) {
  if (h->params.precision == AMG_FP32) vcycle_t<float>(h, r, z, fuse_dot, done);
  else vcycle_t<double>(h, r, z, fuse_dot, done);
  AMG_HIP(hipGetLastError());
  return AMG_OK;
}

namespace {

// one CG iteration (after the first preconditioning)
void cg_iteration(amg_hierarchy *h, double *x) {
  hipStream_t s = h->stream;
  Level &L0 = h->lv[0];
  const int32_t n = L0.n;
  const int32_t *done = &h->scal->done;
  const Geom g = geom(n, true);
  k_spmv_dot<<<g.grid, kBlock, 0, s>>>(n, g.chunk, L0.S.sptr, L0.S.col, L0.S.v64, h->p, h->q,
                                       h->partials, h->ticket, h->scal, done);
  k_update_xr<<<g.grid, kBlock, 0, s>>>(n, g.chunk, x, h->r, h->p, h->q, h->partials,
                                        h->ticket + 1, h->scal, done);
  vcycle(h, h->r, h->z, true, done);
  k_xpay<<<grid1(n), kBlock, 0, s>>>(n, h->z, h->p, h->scal, done);
}

}  // namespace

amg_status pcg(amg_hierarchy *h, const double *b, double *x, double rtol, int32_t maxit,
               amg_solve_info *info) {
  const double t0 = now_ms();
  hipStream_t s = h->stream;
  Level &L0 = h->lv[0];
  const int32_t n = L0.n;
  const int32_t *done = &h->scal->done;
  const Geom g = geom(n, true);
  k_scal_init<<<1, 1, 0, s>>>(h->scal, rtol, maxit);
  k_init_residual<<<g.grid, kBlock, 0, s>>>(n, g.chunk, L0.S.sptr, L0.S.col, L0.S.v64, b, x,
                                            h->r, h->partials, h->ticket, h->scal);
  k_zero_if_zero_rhs<<<grid1(n), kBlock, 0, s>>>(n, x, h->scal);
  AMG_TRY(vcycle(h, h->r, h->z, true, done));
  k_copy<<<grid1(n), kBlock, 0, s>>>(n, h->z, h->p, done);
  // iterations in chunks; the chunk length follows the observed convergence
  int32_t queued = 0, chunk = 4;
  double rr_prev = -1.0;
  int32_t it_prev = 0;
  for (;;) {
    AMG_HIP(hipMemcpyAsync(h->scal_host, h->scal, sizeof(PcgScal), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    const PcgScal sc = *h->scal_host;
    if (sc.done) break;
    if (queued >= maxit) break;  // cannot happen: the maxit test sets done
    if (rr_prev > 0.0 && sc.iter > it_prev && sc.rr > 0.0 && sc.rr < rr_prev) {
      const double rate = std::pow(sc.rr / rr_prev, 1.0 / (sc.iter - it_prev));
      const double need = std::log(sc.tol2 / sc.rr) / std::log(rate);
      chunk = need < 1.0 ? 1 : (need > 32.0 ? 32 : (int32_t)std::ceil(need));
    }
    rr_prev = sc.rr;
    it_prev = sc.iter;
    const int32_t c = std::min(chunk, maxit - queued);
    for (int32_t k = 0; k < c; ++k) cg_iteration(h, x);
    AMG_HIP(hipGetLastError());
    queued += c;
  }
  k_true_residual<<<g.grid, kBlock, 0, s>>>(n, g.chunk, L0.S.sptr, L0.S.col, L0.S.v64, b, x,
                                            h->partials, h->ticket, h->scal);
  AMG_HIP(hipMemcpyAsync(h->scal_host, h->scal, sizeof(PcgScal), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  const PcgScal sc = *h->scal_host;
  amg_status st = AMG_OK;
  if (sc.done == 2) st = AMG_NOT_CONVERGED;
  if (sc.done == 3) st = AMG_ERR_BREAKDOWN;
  if (info) {
    info->iterations = sc.iter;
    info->converged = (sc.done == 1 || sc.done == 4) ? 1 : 0;
    info->rel_res = sc.bb > 0.0 ? std::sqrt(sc.rr / sc.bb) : 0.0;
    info->rel_res_true = sc.bb > 0.0 ? std::sqrt(sc.rr_true / sc.bb) : 0.0;
    info->ms = now_ms() - t0;
  }
  return st;
}

amg_status time_kernel(amg_hierarchy *h, int32_t kernel, int32_t level, int32_t reps,
                       double *ms, double *bytes) {
  if (level < 0 || level >= (int32_t)h->lv.size() - 1 || reps < 1) return AMG_ERR_ARG;
  hipStream_t s = h->stream;
  Level &L = h->lv[level];
  const bool fp32 = h->params.precision == AMG_FP32;
  const double V = fp32 ? 4.0 : 8.0;
  const double n = L.n, nnz = (double)L.nnz, nc = h->lv[level + 1].n;
  const double Vr = level == 0 ? 8.0 : V;  // level 0 reads/writes the FP64 CG vectors
  const int32_t *done = h->zero_flag;
  if (kernel == 4 && level != 0) return AMG_ERR_ARG;
  hipEvent_t e0, e1;
  AMG_HIP(hipEventCreate(&e0));
  AMG_HIP(hipEventCreate(&e1));
  auto launch = [&]() {
    const Geom g = geom(L.n, false);
    const Geom gr = geom(L.n, true);
    switch (kernel) {
      case 0:
        if (fp32) {
          if (level == 0)
            k_pre_residual<float, double><<<g.grid, kBlock, 0, s>>>(
                L.n, g.chunk, L.S.sptr, L.S.col, L.S.v32, L.minv32, h->r, (float *)L.z,
                (float *)L.t, done);
          else
            k_pre_residual<float, float><<<g.grid, kBlock, 0, s>>>(
                L.n, g.chunk, L.S.sptr, L.S.col, L.S.v32, L.minv32, (const float *)L.r,
                (float *)L.z, (float *)L.t, done);
        } else {
          k_pre_residual<double, double><<<g.grid, kBlock, 0, s>>>(
              L.n, g.chunk, L.S.sptr, L.S.col, L.S.v64, L.minv64,
              level == 0 ? h->r : (const double *)L.r, (double *)L.z, (double *)L.t, done);
        }
        break;
      case 1:
        if (fp32) {
          if (level == 0)
            k_post<float, double, double, false><<<g.grid, kBlock, 0, s>>>(
                L.n, g.chunk, L.S.sptr, L.S.col, L.S.v32, L.minv32, h->r, (const float *)L.z,
                h->z, nullptr, nullptr, nullptr, done);
          else
            k_post<float, float, float, false><<<g.grid, kBlock, 0, s>>>(
                L.n, g.chunk, L.S.sptr, L.S.col, L.S.v32, L.minv32, (const float *)L.r,
                (const float *)L.z, (float *)L.y, nullptr, nullptr, nullptr, done);
        } else {
          k_post<double, double, double, false><<<g.grid, kBlock, 0, s>>>(
              L.n, g.chunk, L.S.sptr, L.S.col, L.S.v64, L.minv64,
              level == 0 ? h->r : (const double *)L.r, (const double *)L.z,
              level == 0 ? h->z : (double *)L.y, nullptr, nullptr, nullptr, done);
        }
        break;
      case 2:
        if (fp32)
          k_restrict<float><<<grid1(nc), kBlock, 0, s>>>((int32_t)nc, L.mptr, L.mem, L.pm32,
                                                         (const float *)L.t,
                                                         (float *)h->lv[level + 1].r, done);
        else
          k_restrict<double><<<grid1(nc), kBlock, 0, s>>>((int32_t)nc, L.mptr, L.mem, L.pm64,
                                                          (const double *)L.t,
                                                          (double *)h->lv[level + 1].r, done);
        break;
      case 3:
        if (fp32)
          k_prolong<float><<<grid1(L.n), kBlock, 0, s>>>(L.n, L.agg, L.p32,
                                                         (const float *)h->lv[level + 1].y,
                                                         (float *)L.z, done);
        else
          k_prolong<double><<<grid1(L.n), kBlock, 0, s>>>(L.n, L.agg, L.p64,
                                                          (const double *)h->lv[level + 1].y,
                                                          (double *)L.z, done);
        break;
      default:
        k_spmv_dot<<<gr.grid, kBlock, 0, s>>>(L.n, gr.chunk, L.S.sptr, L.S.col, L.S.v64, h->p,
                                              h->q, h->partials, h->ticket, h->scal, done);
        break;
    }
  };
  launch();  // warm
  AMG_HIP(hipEventRecord(e0, s));
  for (int32_t k = 0; k < reps; ++k) launch();
  AMG_HIP(hipEventRecord(e1, s));
  AMG_HIP(hipEventSynchronize(e1));
  float t = 0.f;
  AMG_HIP(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = (double)t / reps;
  // algorithmic bytes: CSR values + int32 columns + int32 row offsets, each
  // vector once
  switch (kernel) {
    case 0: *bytes = nnz * (V + 4) + 4 * (n + 1) + n * (Vr + V + V + V); break;
    case 1: *bytes = nnz * (V + 4) + 4 * (n + 1) + n * (Vr + V + V + Vr); break;
    case 2: *bytes = n * (4 + V + V) + 4 * (nc + 1) + nc * V; break;
    case 3: *bytes = n * (4 + V + V + V) + nc * V; break;
    default: *bytes = nnz * 12 + 4 * (n + 1) + n * 16; break;
  }
  return AMG_OK;
}

}  // namespace amg
