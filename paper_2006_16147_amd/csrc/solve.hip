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
  (void)reduce;
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks < 1) blocks = 1;
  if (blocks > kMaxParts) {
    int64_t chunk = ((n + kMaxParts - 1) / kMaxParts + kBlock - 1) / kBlock * kBlock;
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
// deterministic two-stage reductions: every block writes its partial sums;
// a one-block finalize kernel adds them in block order and updates the CG
// scalars. (No in-kernel cross-block handshake: on gfx950 a device-scope
// fence per block writes back the XCD's L2 and costs more than a launch.)
// ---------------------------------------------------------------------------

template <int NV>
__device__ void block_partial(double (&v)[NV], double *partials) {
  __shared__ double sh[NV][kBlock / kWave];
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
      double t = sh[q][0];
      for (int k = 1; k < kBlock / kWave; ++k) t += sh[q][k];
      partials[(int64_t)q * kMaxParts + blockIdx.x] = t;
    }
  }
}

enum FinOp : int32_t { kFinInit = 0, kFinPQ = 1, kFinRR = 2, kFinRZ = 3, kFinTrue = 4 };

__device__ __forceinline__ bool converged(double rr, double bb, double rtol) {
  return sqrt(rr) <= rtol * sqrt(bb);
}

// Sums nparts partials of one or two quantities in a fixed order and applies
// the CG scalar update of `op`.
__global__ void __launch_bounds__(1024) k_finalize(int32_t op, int32_t nparts,
                                                   const double *__restrict__ partials,
                                                   PcgScal *scal, const int32_t *done) {
  if (done && *done) return;
  __shared__ double sh[2][1024 / kWave];
  const int nv = op == kFinInit ? 2 : 1;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  double tot[2] = {0.0, 0.0};
  for (int q = 0; q < nv; ++q) {
    double a = 0.0;
    for (int32_t b = threadIdx.x; b < nparts; b += blockDim.x) a += partials[(int64_t)q * kMaxParts + b];
    for (int o = kWave / 2; o > 0; o >>= 1) a += __shfl_down(a, o, kWave);
    if (lane == 0) sh[q][wid] = a;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const int nw = blockDim.x / kWave;
  for (int q = 0; q < nv; ++q) {
    double t = sh[q][0];
    for (int k = 1; k < nw; ++k) t += sh[q][k];
    tot[q] = t;
  }
  switch (op) {
    case kFinInit: {
      const double rtol = scal->rtol;
      scal->bb = tot[0];
      scal->rr = tot[1];
      scal->tol2 = rtol * rtol * tot[0];
      if (tot[0] == 0.0) scal->done = 4;
      else if (converged(tot[1], tot[0], rtol)) scal->done = 1;
      else if (scal->maxit <= 0) scal->done = 2;
      break;
    }
    case kFinPQ:
      scal->pq = tot[0];
      if (!(tot[0] > 0.0)) scal->done = 3;
      else scal->alpha = scal->rho / tot[0];
      break;
    case kFinRR:
      scal->rr = tot[0];
      scal->iter += 1;
      if (converged(tot[0], scal->bb, scal->rtol)) scal->done = 1;
      else if (scal->iter >= scal->maxit) scal->done = 2;
      break;
    case kFinRZ:
      if (!(tot[0] > 0.0)) {
        scal->done = 3;
      } else if (scal->phase == 0) {
        scal->rho = tot[0];
        scal->phase = 1;
      } else {
        scal->beta = tot[0] / scal->rho;
        scal->rho = tot[0];
      }
      break;
    default:
      scal->rr_true = tot[0];
      break;
  }
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
    sell_slice(sptr, row, &base, &w);
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

// y = z + M^-1 (r - A z); with DOT also the block partials of (r, y)
template <typename TV, typename TR, typename TO, bool DOT>
__global__ void __launch_bounds__(kBlock) k_post(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const TV *__restrict__ val, const TV *__restrict__ minv, const TR *__restrict__ r,
    const TV *__restrict__ z, TO *__restrict__ y, double *__restrict__ partials,
    const int32_t *__restrict__ done) {
  if (*done) return;
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  double d[1] = {0.0};
  for (int32_t row = rb + threadIdx.x; row < re; row += kBlock) {
    int32_t base, w;
    sell_slice(sptr, row, &base, &w);
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
  if (DOT) block_partial<1>(d, partials);
}

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
    sell_slice(sptr, row, &base, &w);
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

// Coarsest level: z = A_L^-1 r with A_L^-1 = L^-T L^-1 formed from the
// Cholesky factor at setup (row-major, symmetric). One wavefront per row,
// lanes stride the columns (coalesced), so every row's loads are in flight
// together instead of two sequential triangular sweeps.
constexpr int kCoarseWaves = 4;
template <typename TI, typename TO>
__global__ void __launch_bounds__(kWave *kCoarseWaves) k_coarse_solve(
    int32_t n, const double *__restrict__ Ainv, const TI *__restrict__ r, TO *__restrict__ z,
    const int32_t *__restrict__ done) {
  if (*done) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t i = blockIdx.x * kCoarseWaves + threadIdx.x / kWave;
  if (i >= n) return;
  const double *row = Ainv + (int64_t)i * n;
  double s = 0.0;
  for (int32_t k = lane; k < n; k += kWave) s += row[k] * (double)r[k];
  for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_down(s, o, kWave);
  if (lane == 0) z[i] = (TO)s;
}

// partials of (r, z) when level 0 is itself the coarsest level
__global__ void __launch_bounds__(kBlock) k_dot_rz(int32_t n, int32_t chunk, const double *r,
                                                   const double *z, double *partials,
                                                   const int32_t *done) {
  if (*done) return;
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  double d[1] = {0.0};
  for (int32_t i = rb + threadIdx.x; i < re; i += kBlock) d[0] += r[i] * z[i];
  block_partial<1>(d, partials);
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

// r = b - A x ; partials of (b, b), (r, r)
__global__ void __launch_bounds__(kBlock) k_init_residual(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ b, const double *__restrict__ x,
    double *__restrict__ r, double *__restrict__ partials) {
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  double d[2] = {0.0, 0.0};
  for (int32_t row = rb + threadIdx.x; row < re; row += kBlock) {
    int32_t base, w;
    sell_slice(sptr, row, &base, &w);
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
  block_partial<2>(d, partials);
}

// partials of ||b - A x||^2 at exit
__global__ void __launch_bounds__(kBlock) k_true_residual(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ b, const double *__restrict__ x,
    double *__restrict__ partials) {
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  double d[1] = {0.0};
  for (int32_t row = rb + threadIdx.x; row < re; row += kBlock) {
    int32_t base, w;
    sell_slice(sptr, row, &base, &w);
    double acc = 0.0;
    for (int32_t k = 0; k < w; ++k) {
      const int32_t idx = base + k * kSlice;
      acc += val[idx] * x[col[idx]];
    }
    const double ri = b[row] - acc;
    d[0] += ri * ri;
  }
  block_partial<1>(d, partials);
}

__global__ void k_zero_if_zero_rhs(int32_t n, double *x, const PcgScal *scal) {
  if (scal->done != 4) return;
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

// q = A p ; partials of (p, q)
__global__ void __launch_bounds__(kBlock) k_spmv_dot(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ p, double *__restrict__ q,
    double *__restrict__ partials, const int32_t *__restrict__ done) {
  if (*done) return;
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  double d[1] = {0.0};
  for (int32_t row = rb + threadIdx.x; row < re; row += kBlock) {
    int32_t base, w;
    sell_slice(sptr, row, &base, &w);
    double acc = 0.0;
    for (int32_t k = 0; k < w; ++k) {
      const int32_t idx = base + k * kSlice;
      acc += val[idx] * p[col[idx]];
    }
    q[row] = acc;
    d[0] += p[row] * acc;
  }
  block_partial<1>(d, partials);
}

// x += alpha p ; r -= alpha q ; partials of (r, r)
__global__ void __launch_bounds__(kBlock) k_update_xr(int32_t n, int32_t chunk,
                                                      double *__restrict__ x,
                                                      double *__restrict__ r,
                                                      const double *__restrict__ p,
                                                      const double *__restrict__ q,
                                                      double *__restrict__ partials,
                                                      const PcgScal *__restrict__ scal,
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
  block_partial<1>(d, partials);
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

void finalize(amg_hierarchy *h, int32_t op, int32_t nparts, const int32_t *done) {
  k_finalize<<<1, 1024, 0, h->stream>>>(op, nparts, h->partials, h->scal, done);
}

// Pre-smoothing (pre sweeps) and residual on level l from right-hand side r.
// Leaves t_l = r - A z in L.t and returns the buffer that holds z.
template <typename TV, typename TR>
TV *launch_down(amg_hierarchy *h, int32_t l, const TR *r, const int32_t *done) {
  hipStream_t s = h->stream;
  Level &L = h->lv[l];
  TV *z = (TV *)L.z, *tmp = (TV *)L.y, *t = (TV *)L.t;
  const Geom g = geom(L.n, false);
  const int32_t pre = h->params.pre;
  if (pre == 1) {
    k_pre_residual<TV, TR><<<g.grid, kBlock, 0, s>>>(L.n, g.chunk, L.S.sptr, L.S.col, vals<TV>(L),
                                                   minv<TV>(L), r, z, t, done);
    return z;
  }
  k_jacobi0<TV, TR><<<grid1(L.n), kBlock, 0, s>>>(L.n, minv<TV>(L), r, z, done);
  for (int32_t k = 1; k < pre; ++k) {
    k_post<TV, TR, TV, false><<<g.grid, kBlock, 0, s>>>(L.n, g.chunk, L.S.sptr, L.S.col,
                                                       vals<TV>(L), minv<TV>(L), r, z, tmp,
                                                       nullptr, done);
    std::swap(z, tmp);
  }
  k_residual<TV, TR><<<g.grid, kBlock, 0, s>>>(L.n, g.chunk, L.S.sptr, L.S.col, vals<TV>(L), r, z,
                                             t, done);
  return z;
}

// Prolongation into z and post-smoothing on level l; the last sweep writes
// `out` (a buffer other than z and L.t), with the (r, out) partials if dot.
template <typename TV, typename TR, typename TO>
void launch_up(amg_hierarchy *h, int32_t l, const TR *r, TV *z, const TV *zc, TO *out, bool dot,
               const int32_t *done) {
  hipStream_t s = h->stream;
  Level &L = h->lv[l];
  TV *tmp = (TV *)L.t;  // free once the restriction has read it
  k_prolong<TV><<<grid1(L.n), kBlock, 0, s>>>(L.n, L.agg, pvals<TV>(L), zc, z, done);
  const Geom g = geom(L.n, dot);
  const int32_t post = h->params.post;
  for (int32_t k = 0; k + 1 < post; ++k) {
    k_post<TV, TR, TV, false><<<g.grid, kBlock, 0, s>>>(L.n, g.chunk, L.S.sptr, L.S.col,
                                                       vals<TV>(L), minv<TV>(L), r, z, tmp,
                                                       nullptr, done);
    std::swap(z, tmp);
  }
  if (dot) {
    k_post<TV, TR, TO, true><<<g.grid, kBlock, 0, s>>>(L.n, g.chunk, L.S.sptr, L.S.col,
                                                      vals<TV>(L), minv<TV>(L), r, z, out,
                                                      h->partials, done);
    finalize(h, kFinRZ, g.grid, done);
  } else {
    k_post<TV, TR, TO, false><<<g.grid, kBlock, 0, s>>>(L.n, g.chunk, L.S.sptr, L.S.col,
                                                       vals<TV>(L), minv<TV>(L), r, z, out,
                                                       nullptr, done);
  }
}

template <typename TI, typename TO>
void launch_coarse(amg_hierarchy *h, const TI *r, TO *z, const int32_t *done) {
  const int32_t n = h->C.n;
  k_coarse_solve<TI, TO><<<ceil_div(n, kCoarseWaves), kWave * kCoarseWaves, 0, h->stream>>>(
      n, h->C.Ainv, r, z, done);
}

template <typename TV>
void vcycle_t(amg_hierarchy *h, const double *r0, double *z0, bool dot, const int32_t *done) {
  const int32_t L = (int32_t)h->lv.size() - 1;
  if (L == 0) {
    launch_coarse<double, double>(h, r0, z0, done);
    if (dot) {
      const Geom g = geom(h->lv[0].n, true);
      k_dot_rz<<<g.grid, kBlock, 0, h->stream>>>(h->lv[0].n, g.chunk, r0, z0, h->partials, done);
      finalize(h, kFinRZ, g.grid, done);
    }
    return;
  }
  std::vector<TV *> zbuf(L);
  zbuf[0] = launch_down<TV, double>(h, 0, r0, done);
  for (int32_t l = 0; l < L; ++l) {
    Level &F = h->lv[l];
    Level &C = h->lv[l + 1];
    k_restrict<TV><<<grid1(C.n), kBlock, 0, h->stream>>>(C.n, F.mptr, F.mem, pmvals<TV>(F),
                                                         (const TV *)F.t, (TV *)C.r, done);
    if (l + 1 < L) zbuf[l + 1] = launch_down<TV, TV>(h, l + 1, (const TV *)C.r, done);
  }
  launch_coarse<TV, TV>(h, (const TV *)h->lv[L].r, (TV *)h->lv[L].y, done);
  for (int32_t l = L - 1; l >= 1; --l)
    launch_up<TV, TV, TV>(h, l, (const TV *)h->lv[l].r, zbuf[l], (const TV *)h->lv[l + 1].y,
                          (TV *)h->lv[l].y, false, done);
  launch_up<TV, double, double>(h, 0, r0, zbuf[0], (const TV *)h->lv[1].y, z0, dot, done);
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
    // need the hierarchy precision; the coarsest uses its dense inverse only
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
    if (!coarsest && fp32) {
      AMG_TRY(dalloc(h, &L.minv32, (size_t)L.n));
      AMG_TRY(dalloc(h, &L.p32, (size_t)L.n));
      AMG_TRY(dalloc(h, &L.pm32, (size_t)L.n));
      k_demote<<<grid1(L.n), kBlock, 0, s>>>(L.n, L.minv64, L.minv32);
      k_demote<<<grid1(L.n), kBlock, 0, s>>>(L.n, L.p64, L.p32);
      k_demote<<<grid1(L.n), kBlock, 0, s>>>(L.n, L.pm64, L.pm32);
    }
    AMG_TRY(alloc_level_vectors(h, L, vbytes));
  }
  // outer CG vectors and scalars
  const int32_t n0 = h->lv[0].n;
  AMG_TRY(dalloc(h, &h->x, (size_t)n0));
  AMG_TRY(dalloc(h, &h->r, (size_t)n0));
  AMG_TRY(dalloc(h, &h->z, (size_t)n0));
  AMG_TRY(dalloc(h, &h->p, (size_t)n0));
  AMG_TRY(dalloc(h, &h->q, (size_t)n0));
  AMG_TRY(dalloc(h, &h->partials, (size_t)kMaxParts * 2));
  AMG_TRY(dalloc(h, &h->scal, 1));
  AMG_TRY(dalloc(h, &h->zero_flag, 4));
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

// One CG iteration after the first preconditioning. Touches only hierarchy
// buffers (x is the internal copy), so it can be captured once and replayed.
void cg_iteration(amg_hierarchy *h) {
  hipStream_t s = h->stream;
  Level &L0 = h->lv[0];
  const int32_t n = L0.n;
  const int32_t *done = &h->scal->done;
  const Geom g = geom(n, true);
  k_spmv_dot<<<g.grid, kBlock, 0, s>>>(n, g.chunk, L0.S.sptr, L0.S.col, L0.S.v64, h->p, h->q,
                                       h->partials, done);
  finalize(h, kFinPQ, g.grid, done);
  k_update_xr<<<g.grid, kBlock, 0, s>>>(n, g.chunk, h->x, h->r, h->p, h->q, h->partials, h->scal,
                                        done);
  finalize(h, kFinRR, g.grid, done);
  vcycle(h, h->r, h->z, true, done);
  k_xpay<<<grid1(n), kBlock, 0, s>>>(n, h->z, h->p, h->scal, done);
}

// Captures one CG iteration into a hipGraph (once per hierarchy).
amg_status ensure_iteration_graph(amg_hierarchy *h) {
  if (h->iter_exec || h->graph_failed || (h->params.flags & AMG_FLAG_NO_GRAPH)) return AMG_OK;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    h->graph_failed = true;
    return AMG_OK;
  }
  cg_iteration(h);
  hipError_t e = hipStreamEndCapture(h->stream, &g);
  if (e != hipSuccess || !g) {
    (void)hipGetLastError();
    h->graph_failed = true;
    return AMG_OK;
  }
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    (void)hipGraphDestroy(g);
    h->graph_failed = true;
    return AMG_OK;
  }
  h->iter_graph = g;
  h->iter_exec = ex;
  return AMG_OK;
}

}  // namespace

amg_status pcg(amg_hierarchy *h, const double *b, double *x_user, double rtol, int32_t maxit,
               amg_solve_info *info) {
  const double t0 = now_ms();
  hipStream_t s = h->stream;
  Level &L0 = h->lv[0];
  const int32_t n = L0.n;
  const int32_t *done = &h->scal->done;
  const Geom g = geom(n, true);
  AMG_TRY(ensure_iteration_graph(h));
  AMG_HIP(hipMemcpyAsync(h->x, x_user, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  k_scal_init<<<1, 1, 0, s>>>(h->scal, rtol, maxit);
  k_init_residual<<<g.grid, kBlock, 0, s>>>(n, g.chunk, L0.S.sptr, L0.S.col, L0.S.v64, b, h->x,
                                            h->r, h->partials);
  finalize(h, kFinInit, g.grid, nullptr);
  k_zero_if_zero_rhs<<<grid1(n), kBlock, 0, s>>>(n, h->x, h->scal);
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
    if (queued >= maxit) break;  // not reached: the maxit test sets done
    if (rr_prev > 0.0 && sc.iter > it_prev && sc.rr > 0.0 && sc.rr < rr_prev) {
      const double rate = std::pow(sc.rr / rr_prev, 1.0 / (sc.iter - it_prev));
      const double need = std::log(sc.tol2 / sc.rr) / std::log(rate);
      chunk = need < 1.0 ? 1 : (need > 32.0 ? 32 : (int32_t)std::ceil(need));
    }
    rr_prev = sc.rr;
    it_prev = sc.iter;
    const int32_t c = std::min(chunk, maxit - queued);
    for (int32_t k = 0; k < c; ++k) {
      if (h->iter_exec) AMG_HIP(hipGraphLaunch(h->iter_exec, s));
      else cg_iteration(h);
    }
    AMG_HIP(hipGetLastError());
    queued += c;
  }
  k_true_residual<<<g.grid, kBlock, 0, s>>>(n, g.chunk, L0.S.sptr, L0.S.col, L0.S.v64, b, h->x,
                                            h->partials);
  finalize(h, kFinTrue, g.grid, nullptr);
  AMG_HIP(hipMemcpyAsync(x_user, h->x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
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
            k_post<float, double, double, true><<<g.grid, kBlock, 0, s>>>(
                L.n, g.chunk, L.S.sptr, L.S.col, L.S.v32, L.minv32, h->r, (const float *)L.z,
                h->z, h->partials, done);
          else
            k_post<float, float, float, false><<<g.grid, kBlock, 0, s>>>(
                L.n, g.chunk, L.S.sptr, L.S.col, L.S.v32, L.minv32, (const float *)L.r,
                (const float *)L.z, (float *)L.y, nullptr, done);
        } else {
          if (level == 0)
            k_post<double, double, double, true><<<g.grid, kBlock, 0, s>>>(
                L.n, g.chunk, L.S.sptr, L.S.col, L.S.v64, L.minv64, h->r, (const double *)L.z,
                h->z, h->partials, done);
          else
            k_post<double, double, double, false><<<g.grid, kBlock, 0, s>>>(
                L.n, g.chunk, L.S.sptr, L.S.col, L.S.v64, L.minv64, (const double *)L.r,
                (const double *)L.z, (double *)L.y, nullptr, done);
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
        k_spmv_dot<<<g.grid, kBlock, 0, s>>>(L.n, g.chunk, L.S.sptr, L.S.col, L.S.v64, h->p,
                                             h->q, h->partials, done);
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
