// Solve phase: the V-cycle of eq. (amg) with l1-Jacobi smoothing (Section 3.3)
// inside preconditioned CG (Section 5), on one gfx950 GPU.
//
// Layout. Every level is stored in an aggregate-major order (the unknowns of
// an aggregate of P_l are one contiguous segment, segments ordered like the
// coarse unknowns, recursively from the coarsest level), as sliced ELLPACK
// with 64-row slices (one slice per wavefront, column-major inside a slice),
// so lane i of a wavefront loads row i's k-th value and column index from
// consecutive addresses. The matrix arrays are loaded with a nontemporal
// hint: they stream once per SpMV while the gathered vector stays in L2.
//
// Kernels of a V-cycle (zero initial guess), per level l < L:
//   down  pre_restrict : z = M^-1 r ; r_{l+1} = P^T (r - A z)
//         (A M^-1 is stored, so one vector is gathered; a block owns whole
//          aggregates and sums their members in LDS: the residual never
//          goes to HBM)
//   up    post_prolong : y = z + M^-1 (r - A z) on level l + 1, and at once
//         z_l += P y for the segments of the block's coarse rows
//   level L: coarse_prolong: z_L = A_L^-1 r_L and z_{L-1} += P z_L
//   level 0: post with the (r, z) partial sums for CG
//
// CG scalars live on the device; reductions are two-stage and deterministic:
// every block writes its partial sums, a one-block finalize kernel adds them
// in block order and updates the scalars. Kernels test a device flag and
// return at once after convergence, so the host queues several iterations
// (captured in a hipGraph) between checks.

#include <chrono>
#include <cmath>

#include <hip/hip_ext.h>

#include "internal.h"

namespace amg {

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

inline int32_t grid1(int64_t n) { return ceil_div(n > 0 ? n : 1, kBlock); }

// ---------------------------------------------------------------------------
// launch geometry of the row-streaming kernels: each block a contiguous
// chunk of 1 to kMaxRowsPerThread rows per thread, about kTargetBlocks
// blocks (more rows per thread only beyond kMaxParts blocks)
// ---------------------------------------------------------------------------

struct Geom {
  int32_t grid;
  int32_t chunk;  // rows per block, a multiple of kBlock
};

Geom geom(int64_t n) {
  int64_t rows = (n + (int64_t)kBlock * kTargetBlocks - 1) / ((int64_t)kBlock * kTargetBlocks);
  rows = rows < 1 || n >= kManyRows ? 1 : (rows > kMaxRowsPerThread ? kMaxRowsPerThread : rows);
  int64_t chunk = kBlock * rows;
  int64_t blocks = (n + chunk - 1) / chunk;
  if (blocks < 1) blocks = 1;
  if (blocks > kMaxParts) {
    chunk = ((n + kMaxParts - 1) / kMaxParts + kBlock - 1) / kBlock * kBlock;
    blocks = (n + chunk - 1) / chunk;
  }
  return {(int32_t)blocks, (int32_t)chunk};
}

__device__ __forceinline__ void rows_of_block(int32_t n, int32_t chunk, int32_t *b, int32_t *e) {
  const int64_t bb = (int64_t)blockIdx.x * chunk;
  *b = (int32_t)bb;
  *e = (int32_t)(bb + chunk < n ? bb + chunk : n);
}

__device__ __forceinline__ void sell_row(const int32_t *sptr, int32_t row, int32_t *base,
                                         int32_t *w) {
  const int32_t s = row / kSlice;
  const int32_t b0 = sptr[s];
  *base = b0 + (row % kSlice);
  *w = (sptr[s + 1] - b0) / kSlice;
}

// zf[k] += pp[k] * y(aggp[k]) for k = k0 + t, k0 + t + nth, ... < k1: each
// thread issues the loads of four of its positions before their use.
template <typename TV, typename Y>
__device__ __forceinline__ void prolong_add(int32_t k0, int32_t k1, int32_t t, int32_t nth,
                                            const int32_t *__restrict__ aggp,
                                            const TV *__restrict__ pp, TV *__restrict__ zf, Y y) {
  for (int32_t kb = k0 + t; kb < k1; kb += 4 * nth) {
    int32_t a[4];
    TV pv[4], zv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t k = kb + u * nth;
      a[u] = 0;
      pv[u] = zv[u] = 0;
      if (k < k1) {
        a[u] = aggp[k];
        pv[u] = pp[k];
        zv[u] = zf[k];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t k = kb + u * nth;
      if (k < k1) zf[k] = zv[u] + pv[u] * y(a[u]);
    }
  }
}

// ---------------------------------------------------------------------------
// deterministic two-stage reductions (no in-kernel cross-block handshake: on
// gfx950 a device-scope fence per block writes back the XCD's L2 and costs
// more than the extra launch)
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

enum FinOp : int32_t {
  kFinInit = 0,  // (b, b), (r, r) of the initial residual
  kFinPQ = 1,    // CG: (p, q), alpha = rho / (p, q)
  kFinRR = 2,    // (r, r), stop test
  kFinRZ = 3,    // CG: (r, z), beta
  kFinTrue = 4,  // true residual
  kFinPQR = 5,   // flexible CG: (p, q), (p, r), alpha = (p, r) / (p, q)
  kFinZQ = 6     // flexible CG: beta = -(z, q) / (p, q)
};

__device__ __forceinline__ bool converged(double rr, double bb, double rtol) {
  return sqrt(rr) <= rtol * sqrt(bb);
}

// Sums nparts partials of one or two quantities in a fixed order and applies
// the CG scalar update of `op`.
__global__ void __launch_bounds__(1024) k_finalize(int32_t op, int32_t nparts,
                                                   const double *__restrict__ partials,
                                                   PcgScal *scal, const int32_t *done) {
  // the stop flag and the scalars are loaded with the partials, not before
  const int32_t stop = done ? *done : 0;
  PcgScal sc;
  if (threadIdx.x == 0) sc = *scal;
  __shared__ double sh[2][1024 / kWave];
  const int nv = op == kFinInit || op == kFinPQR ? 2 : 1;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int q = 0; q < nv; ++q) {
    // this thread's partials in index order, sixteen loads at a time
    const double *src = partials + (int64_t)q * kMaxParts;
    double a = 0.0;
    for (int32_t b0 = threadIdx.x; b0 < nparts; b0 += 16 * blockDim.x) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int32_t b = b0 + u * (int32_t)blockDim.x;
        v[u] = b < nparts ? src[b] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (b0 + u * (int32_t)blockDim.x < nparts) a += v[u];
    }
    for (int o = kWave / 2; o > 0; o >>= 1) a += __shfl_down(a, o, kWave);
    if (lane == 0) sh[q][wid] = a;
  }
  __syncthreads();
  if (threadIdx.x != 0 || stop) return;
  double tot[2] = {0.0, 0.0};
  for (int q = 0; q < nv; ++q) {
    double t = sh[q][0];
    for (int k = 1; k < (int)(blockDim.x / kWave); ++k) t += sh[q][k];
    tot[q] = t;
  }
  switch (op) {
    case kFinInit: {
      const double rtol = sc.rtol;
      scal->bb = tot[0];
      scal->rr = tot[1];
      scal->tol2 = rtol * rtol * tot[0];
      if (tot[0] == 0.0) scal->done = 4;
      else if (converged(tot[1], tot[0], rtol)) scal->done = 1;
      else if (sc.maxit <= 0) scal->done = 2;
      break;
    }
    case kFinPQ:
      scal->pq = tot[0];
      if (!(tot[0] > 0.0)) scal->done = 3;
      else scal->alpha = sc.rho / tot[0];
      break;
    case kFinRR:
      scal->rr = tot[0];
      scal->iter = sc.iter + 1;
      if (converged(tot[0], sc.bb, sc.rtol)) scal->done = 1;
      else if (sc.iter + 1 >= sc.maxit) scal->done = 2;
      break;
    case kFinRZ:
      if (!(tot[0] > 0.0)) {
        scal->done = 3;
      } else if (sc.phase == 0) {
        scal->rho = tot[0];
        scal->phase = 1;
      } else {
        scal->beta = tot[0] / sc.rho;
        scal->rho = tot[0];
      }
      break;
    case kFinPQR:
      scal->pq = tot[0];
      if (!(tot[0] > 0.0)) scal->done = 3;
      else scal->alpha = tot[1] / tot[0];
      break;
    case kFinZQ:
      scal->beta = -tot[0] / sc.pq;
      break;
    default:
      scal->rr_true = tot[0];
      break;
  }
}

// ---------------------------------------------------------------------------
// aggregate-major order, SELL construction, precision demotion
// ---------------------------------------------------------------------------

// number of members of the aggregate at each coarse position
__global__ void k_seg_count(int32_t nc, const int32_t *perm_c, const int32_t *mptr,
                            int32_t *cnt) {
  const int32_t J = blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= nc) return;
  const int32_t I = perm_c[J];
  cnt[J] = mptr[I + 1] - mptr[I];
}

// positions of the members of each aggregate (in ascending original index)
__global__ void k_order_fill(int32_t nc, const int32_t *perm_c, const int32_t *mptr,
                             const int32_t *mem, const int32_t *seg, const double *p,
                             int32_t *perm, int32_t *iperm, int32_t *aggp, double *pp) {
  const int32_t J = blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= nc) return;
  const int32_t I = perm_c[J];
  const int32_t b = mptr[I], e = mptr[I + 1], k0 = seg[J];
  for (int32_t m = b; m < e; ++m) {
    const int32_t i = mem[m], k = k0 + (m - b);
    perm[k] = i;
    iperm[i] = k;
    aggp[k] = J;
    pp[k] = p[i];
  }
}

__global__ void k_iota_i32(int32_t *a, int32_t n) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = i;
}

__global__ void k_gather_f64(int32_t n, const int32_t *perm, const double *src, double *dst) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = src[perm[k]];
}

// Entries of each 64-row slice (width = longest row, times 64), and their
// 64-bit total: the int32 offsets of the format must not overflow.
__global__ void k_sell_width(int32_t n, int32_t ns, const int32_t *rp, const int32_t *perm,
                             int32_t *w64, unsigned long long *total) {
  const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  const int32_t r0 = s * kSlice, r1 = min(n, r0 + kSlice);
  int32_t w = 0;
  for (int32_t k = r0; k < r1; ++k) {
    const int32_t i = perm[k];
    w = max(w, rp[i + 1] - rp[i]);
  }
  const int64_t e = (int64_t)w * kSlice;
  w64[s] = e > INT32_MAX ? INT32_MAX : (int32_t)e;
  atomicAdd(total, (unsigned long long)e);
}

// Row k of the permuted matrix is original row perm[k] with columns renumbered
// by iperm and sorted (rows up to kSortCap entries); padding entries point at
// the row itself with value 0.
constexpr int kSortCap = 64;
__global__ void k_sell_fill(int32_t n, int32_t ns, const int32_t *rp, const int32_t *ci,
                            const double *val, const int32_t *perm, const int32_t *iperm,
                            const double *minv, const int32_t *sptr, int32_t *col, double *v64,
                            float *v32, double *s64, float *s32) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)ns * kSlice) return;
  const int32_t s = (int32_t)(k / kSlice), lane = (int32_t)(k % kSlice);
  const int32_t base = sptr[s], w = (sptr[s + 1] - base) / kSlice;
  const int32_t i = k < n ? perm[k] : 0;
  const int32_t b = k < n ? rp[i] : 0, len = k < n ? rp[i + 1] - b : 0;
  int32_t order[kSortCap];
  const bool sorted = len <= kSortCap;
  if (sorted) {
    for (int32_t e = 0; e < len; ++e) {
      const int32_t c = iperm[ci[b + e]];
      int32_t pos = e;
      while (pos > 0 && iperm[ci[b + order[pos - 1]]] > c) {
        order[pos] = order[pos - 1];
        --pos;
      }
      order[pos] = e;
    }
  }
  for (int32_t e = 0; e < w; ++e) {
    const int64_t idx = base + (int64_t)e * kSlice + lane;
    if (e < len) {
      const int32_t src = b + (sorted ? order[e] : e);
      const int32_t c = ci[src];
      const double a = val[src];
      col[idx] = iperm[c];
      if (v64) v64[idx] = a;
      if (v32) v32[idx] = (float)a;
      if (s64) s64[idx] = a * minv[c];
      if (s32) s32[idx] = (float)(a * minv[c]);
    } else {
      col[idx] = k < n ? (int32_t)k : 0;
      if (v64) v64[idx] = 0.0;
      if (v32) v32[idx] = 0.f;
      if (s64) s64[idx] = 0.0;
      if (s32) s32[idx] = 0.f;
    }
  }
}

// flags a value that an FP32 number cannot hold exactly (or a NaN)
__global__ void k_not_fp32_exact(int64_t n, const double *a, int32_t *flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !((double)(float)a[i] == a[i])) *flag = 1;
}

__global__ void k_demote(int64_t n, const double *a, float *b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

__global__ void k_permute_in(int32_t n, const int32_t *__restrict__ perm,
                             const double *__restrict__ src, double *__restrict__ dst) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = src[perm[k]];
}

__global__ void k_permute_out(int32_t n, const int32_t *__restrict__ perm,
                              const double *__restrict__ src, double *__restrict__ dst) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[perm[k]] = src[k];
}

// ---------------------------------------------------------------------------
// V-cycle kernels. TV: hierarchy precision; TR: type of the level's
// right-hand side (double on level 0, TV below); TO: type of its output.
// ---------------------------------------------------------------------------

// Down step on level l for the coarse positions [J0, J0 + G) of this block:
// z = M^-1 r with the residual through the stored A M^-1 (kPreScaled) or,
// after extra pre-smoothing sweeps, the given z (kPreFromZ, plain A stored
// as TA), or z = M^-1 r formed while staging r in LDS and the residual
// through the plain A (kPreStagedZ, LDS kernel only: where A is stored in
// fewer bytes than A M^-1, i.e. level 0's exact FP32 copy in an FP64
// hierarchy); then
// r_{l+1}(J) = sum over the segment of J, in order, of p_k (r - A z)_k.
// The block's fine rows are the union of its segments (at most R kBlock
// rows; thread t takes rows t, t + kBlock, ...).
enum PreMode : int { kPreScaled = 0, kPreFromZ = 1, kPreStagedZ = 2 };

template <typename TV, typename TR, int MODE, typename TA = TV, int R = 1>
__global__ void __launch_bounds__(kBlock) k_pre_restrict(
    int32_t nc, int32_t G, const int32_t *__restrict__ seg, const int32_t *__restrict__ sptr,
    const int32_t *__restrict__ col, const TA *__restrict__ val, const TV *__restrict__ minv,
    const TV *__restrict__ pp, const TR *__restrict__ r, TV *__restrict__ z,
    TV *__restrict__ rc, const int32_t *__restrict__ done) {
  __shared__ TV sh[kBlock * R];
  if (*done) return;
  const int32_t J0 = blockIdx.x * G;
  const int32_t J1 = min(nc, J0 + G);
  const int32_t f0 = seg[J0], f1 = seg[J1];
  // the thread's segment bounds for the sums after the barrier, loaded now
  const int32_t Jt = J0 + (int32_t)threadIdx.x;
  const int32_t sb = Jt < J1 ? seg[Jt] : 0, se = Jt < J1 ? seg[Jt + 1] : 0;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int32_t row = f0 + (int32_t)threadIdx.x + u * kBlock;
    if (row < f1) {
      // the row's own operands first: their loads overlap the gathers
      const TV ri = (TV)r[row];
      const TV mi = MODE == kPreScaled ? minv[row] : TV(0);
      const TV pv = pp[row];
      int32_t base, w;
      sell_row(sptr, row, &base, &w);
      const TV acc =
          MODE == kPreFromZ
              ? sell_dot_t<TV, TA>(col, val, base, w, [&](int32_t c) { return z[c]; })
              : sell_dot_t<TV, TA>(col, val, base, w, [&](int32_t c) { return (TV)r[c]; });
      if (MODE == kPreScaled) z[row] = ri * mi;
      sh[threadIdx.x + u * kBlock] = pv * (ri - acc);
    }
  }
  __syncthreads();
  for (int32_t J = Jt; J < J1; J += kBlock) {
    const int32_t b = (J == Jt ? sb : seg[J]) - f0, e = (J == Jt ? se : seg[J + 1]) - f0;
    TV s = 0;
    for (int32_t m = b; m < e; ++m) s += sh[m];
    rc[J] = s;
  }
}

// y = z + M^-1 (r - A z); with DOT also the block partials of (r, y)
// (with a dot partner dv, the partials are of (dv, y) instead)
template <typename TV, typename TR, typename TO, bool DOT, typename TA = TV>
__global__ void __launch_bounds__(kBlock) k_post(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const TA *__restrict__ val, const TV *__restrict__ minv, const TR *__restrict__ r,
    const TV *__restrict__ z, TO *__restrict__ y, double *__restrict__ partials,
    const int32_t *__restrict__ done, const double *__restrict__ dv = nullptr) {
  if (*done) return;
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  double d[1] = {0.0};
  for (int32_t row = rb + threadIdx.x; row < re; row += kBlock) {
    const TR rr = r[row];
    const TV zr = z[row], mr = minv[row];
    int32_t base, w;
    sell_row(sptr, row, &base, &w);
    const TV acc = sell_dot_t<TV, TA>(col, val, base, w, [&](int32_t c) { return z[c]; });
    const TO yo = (TO)(zr + ((TV)rr - acc) * mr);
    y[row] = yo;
    if (DOT) d[0] += (dv ? dv[row] : (double)rr) * (double)yo;
  }
  if (DOT) block_partial<1>(d, partials);
}

// ---- LDS-staged gathers (level 0): the same products as above, with the
// gathered vector's entries of the block's tile loaded into LDS first ----

// xs[i] = x(hidx[h0 + i]) for the block's list of u entries, eight loads in
// flight per thread, then a barrier
template <typename TV, typename X>
__device__ __forceinline__ void stage_tile(TV *xs, const int32_t *__restrict__ hidx, int32_t h0,
                                           int32_t u, X x) {
  for (int32_t i0 = threadIdx.x; i0 < u; i0 += 8 * kBlock) {
    int32_t c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int32_t i = i0 + q * kBlock;
      c[q] = i < u ? hidx[h0 + i] : 0;
    }
    TV v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = i0 + q * kBlock < u ? x(c[q]) : TV(0);
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (i0 + q * kBlock < u) xs[i0 + q * kBlock] = v[q];
  }
  __syncthreads();
}

// sum_k val[k] * xs[lcol[k]] over one SELL row: the products and sums of
// sell_dot_t, in the same order and with the same unconditional batched
// loads, with the operands read from LDS
template <typename TV, typename TA>
__device__ __forceinline__ TV sell_dot_lds(const uint16_t *__restrict__ lcol,
                                           const TA *__restrict__ val, int32_t base, int32_t w,
                                           const TV *xs) {
  TV acc = 0;
  for (int32_t k0 = 0; k0 < w; k0 += kRowBatch) {
    int32_t c[kRowBatch];
    TA va[kRowBatch];
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      const int32_t idx = base + (k0 + u < w ? k0 + u : w - 1) * kSlice;
      c[u] = ld_stream(&lcol[idx]);
      va[u] = ld_stream(&val[idx]);
    }
    TV g[kRowBatch];
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) g[u] = xs[c[u]];
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u)
      if (k0 + u < w) acc += (TV)va[u] * g[u];
  }
  return acc;
}

// k_pre_restrict with the tile of block b = its segment rows (tiles hseg).
// The LDS kernels take their tiles in XCD-aware order (xcd_block): each XCD
// works down one contiguous range of tiles, so a tile's staged neighbours
// were mostly just loaded into the same L2 by the tiles before it (160^3
// FP64 down step 73.6 -> 64.4 us). The partial sums stay indexed by blockIdx.
template <typename TV, typename TR, int MODE, typename TA = TV, int R = 1>
__global__ void __launch_bounds__(kBlock) k_pre_restrict_lds(
    int32_t nc, int32_t G, const int32_t *__restrict__ seg, const int32_t *__restrict__ sptr,
    const uint16_t *__restrict__ lcol, const int32_t *__restrict__ hptr,
    const int32_t *__restrict__ hidx, const TA *__restrict__ val, const TV *__restrict__ minv,
    const TV *__restrict__ pp, const TR *__restrict__ r, TV *__restrict__ z,
    TV *__restrict__ rc, const int32_t *__restrict__ done) {
  extern __shared__ double lds_d[];
  TV *xs = reinterpret_cast<TV *>(lds_d);
  __shared__ TV sh[kBlock * R];
  if (*done) return;
  const int32_t tb = xcd_block(blockIdx.x, gridDim.x);
  const int32_t J0 = tb * G;
  const int32_t J1 = min(nc, J0 + G);
  const int32_t f0 = seg[J0], f1 = seg[J1];
  const int32_t h0 = hptr[tb];
  // the operands that do not come from the staged tile are loaded first, so
  // their latency overlaps the staging
  int32_t pb[R], pw[R];
  TV pr[R], pm[R], pq[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int32_t row = f0 + (int32_t)threadIdx.x + u * kBlock;
    pb[u] = pw[u] = 0;
    pr[u] = pm[u] = pq[u] = TV(0);
    if (row < f1) {
      sell_row(sptr, row, &pb[u], &pw[u]);
      pr[u] = (TV)r[row];
      if (MODE != kPreFromZ) pm[u] = minv[row];
      pq[u] = pp[row];
    }
  }
  const int32_t Jt = J0 + (int32_t)threadIdx.x;
  const int32_t sb = Jt < J1 ? seg[Jt] : 0, se = Jt < J1 ? seg[Jt + 1] : 0;
  if (MODE == kPreFromZ)
    stage_tile(xs, hidx, h0, hptr[tb + 1] - h0, [&](int32_t c) { return z[c]; });
  else if (MODE == kPreStagedZ)
    stage_tile(xs, hidx, h0, hptr[tb + 1] - h0,
               [&](int32_t c) { return (TV)r[c] * minv[c]; });
  else
    stage_tile(xs, hidx, h0, hptr[tb + 1] - h0, [&](int32_t c) { return (TV)r[c]; });
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int32_t row = f0 + (int32_t)threadIdx.x + u * kBlock;
    if (row < f1) {
      const TV acc = sell_dot_lds<TV, TA>(lcol, val, pb[u], pw[u], xs);
      const TV ri = pr[u];
      if (MODE != kPreFromZ) z[row] = ri * pm[u];
      sh[threadIdx.x + u * kBlock] = pq[u] * (ri - acc);
    }
  }
  __syncthreads();
  for (int32_t J = Jt; J < J1; J += kBlock) {
    const int32_t b = (J == Jt ? sb : seg[J]) - f0, e = (J == Jt ? se : seg[J + 1]) - f0;
    TV s = 0;
    for (int32_t m = b; m < e; ++m) s += sh[m];
    rc[J] = s;
  }
}

// k_post with the tile of block b = its row chunk (tiles hrow), XCD-aware order
template <typename TV, typename TR, typename TO, bool DOT, typename TA = TV>
__global__ void __launch_bounds__(kBlock) k_post_lds(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const uint16_t *__restrict__ lcol,
    const int32_t *__restrict__ hptr, const int32_t *__restrict__ hidx,
    const TA *__restrict__ val, const TV *__restrict__ minv, const TR *__restrict__ r,
    const TV *__restrict__ z, TO *__restrict__ y, double *__restrict__ partials,
    const int32_t *__restrict__ done, const double *__restrict__ dv = nullptr) {
  extern __shared__ double lds_d[];
  TV *xs = reinterpret_cast<TV *>(lds_d);
  if (*done) return;
  int32_t rb, re;
  const int32_t tb = xcd_block(blockIdx.x, gridDim.x);
  rb = (int32_t)((int64_t)tb * chunk);
  re = (int32_t)min((int64_t)n, (int64_t)rb + chunk);
  const int32_t h0 = hptr[tb];
  int32_t row = rb + (int32_t)threadIdx.x, nb = 0, nw = 0;
  if (row < re) sell_row(sptr, row, &nb, &nw);
  stage_tile(xs, hidx, h0, hptr[tb + 1] - h0, [&](int32_t c) { return z[c]; });
  double d[1] = {0.0};
  for (; row < re; row += kBlock) {
    const int32_t base = nb, w = nw;
    if (row + kBlock < re) sell_row(sptr, row + kBlock, &nb, &nw);
    const TV acc = sell_dot_lds<TV, TA>(lcol, val, base, w, xs);
    const TR rr = r[row];
    const TO yo = (TO)(z[row] + ((TV)rr - acc) * minv[row]);
    y[row] = yo;
    if (DOT) d[0] += (dv ? dv[row] : (double)rr) * (double)yo;
  }
  if (DOT) block_partial<1>(d, partials);
}

// ---- smoothed aggregation: unfused down and up steps (Pbar is not a
// segment map, so restriction and prolongation are CSR products) ----

// z = M^-1 r and t = r - A z = r - (A M^-1) r (the first sweep from zero)
template <typename TV, typename TR>
__global__ void __launch_bounds__(kBlock) k_pre_resid(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const TV *__restrict__ sval, const TV *__restrict__ minv, const TR *__restrict__ r,
    TV *__restrict__ z, TV *__restrict__ t, const int32_t *__restrict__ done) {
  if (*done) return;
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  for (int32_t row = rb + threadIdx.x; row < re; row += kBlock) {
    int32_t base, w;
    sell_row(sptr, row, &base, &w);
    const TV acc = sell_dot(col, sval, base, w, [&](int32_t c) { return (TV)r[c]; });
    const TV ri = (TV)r[row];
    z[row] = ri * minv[row];
    t[row] = ri - acc;
  }
}

// t = r - A z
template <typename TV, typename TR, typename TA = TV>
__global__ void __launch_bounds__(kBlock) k_resid(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const TA *__restrict__ val, const TR *__restrict__ r, const TV *__restrict__ z,
    TV *__restrict__ t, const int32_t *__restrict__ done) {
  if (*done) return;
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  for (int32_t row = rb + threadIdx.x; row < re; row += kBlock) {
    int32_t base, w;
    sell_row(sptr, row, &base, &w);
    const TV acc = sell_dot_t<TV, TA>(col, val, base, w, [&](int32_t c) { return z[c]; });
    t[row] = (TV)r[row] - acc;
  }
}

// sum over row i of a CSR matrix of val * x(col), with LPR consecutive lanes
// per row: lane k takes the entries k, k + LPR, ..., then the lanes' sums
// are added across the group (every lane of the group gets the total)
template <typename TV, int LPR, typename TA, typename X>
__device__ __forceinline__ TV csr_row_dot(int32_t i, int32_t nr, const int32_t *__restrict__ rp,
                                          const int32_t *__restrict__ ci,
                                          const TA *__restrict__ val, X x) {
  const int lane = threadIdx.x % LPR;
  TV acc = 0;
  if (i < nr) {
    // a lane's entries in batches of kRowBatch: all index and value loads,
    // then all gathers, then the products in order
    const int32_t e1 = rp[i + 1];
    for (int32_t e0 = rp[i] + lane; e0 < e1; e0 += LPR * kRowBatch) {
      int32_t c[kRowBatch];
      TV v[kRowBatch], g[kRowBatch];
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        const int32_t e = e0 + u * LPR;
        c[u] = 0;
        v[u] = 0;
        if (e < e1) {
          c[u] = ci[e];
          v[u] = (TV)val[e];
        }
      }
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) g[u] = e0 + u * LPR < e1 ? x(c[u]) : TV(0);
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u)
        if (e0 + u * LPR < e1) acc += v[u] * g[u];
    }
  }
  for (int o = LPR / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, LPR);
  return acc;
}

// y = M x for a CSR M, or with ADD y += M x (LPR lanes per row)
template <typename TV, bool ADD, int LPR>
__global__ void __launch_bounds__(kBlock) k_csr_apply(int32_t nr, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci,
                                                      const TV *__restrict__ val,
                                                      const TV *__restrict__ x, TV *__restrict__ y,
                                                      const int32_t *__restrict__ done) {
  if (*done) return;
  const int32_t i = (int32_t)(((int64_t)blockIdx.x * kBlock + threadIdx.x) / LPR);
  const TV acc = csr_row_dot<TV, LPR>(i, nr, rp, ci, val, [&](int32_t c) { return x[c]; });
  if (i < nr && threadIdx.x % LPR == 0) y[i] = ADD ? y[i] + acc : acc;
}

// smoothing on a long-row level (CSR in the solve order, LPR lanes per row):
// MODE 0: y = z + M^-1 (r - A z); MODE 1: y = r - A z (the residual)
template <typename TV, typename TR, int MODE, int LPR>
__global__ void __launch_bounds__(kBlock) k_smooth_rows(
    int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const TV *__restrict__ val, const TV *__restrict__ minv, const TR *__restrict__ r,
    const TV *__restrict__ z, TV *__restrict__ y, const int32_t *__restrict__ done) {
  if (*done) return;
  const int32_t i = (int32_t)(((int64_t)blockIdx.x * kBlock + threadIdx.x) / LPR);
  const TV acc = csr_row_dot<TV, LPR>(i, n, rp, ci, val, [&](int32_t c) { return z[c]; });
  if (i < n && threadIdx.x % LPR == 0) {
    const TV res = (TV)r[i] - acc;
    y[i] = MODE == 0 ? z[i] + res * minv[i] : res;
  }
}

// lanes per row for nr rows of nnz entries: two to three entries per lane
// (rows shorter than 6 entries: one lane, a single batch of loads), and more
// lanes (up to a wavefront) while fewer than 2^19 threads would be in
// flight. At 160^3 (smoothed hierarchy) one lane per entry made the big
// levels' products up to 30 % slower, about 8 entries per lane 7 % slower
// per iteration; whole wavefronts made the small levels' twice as fast.
inline int lanes_for(int64_t nr, int64_t nnz) {
  const double avg = nr > 0 ? (double)nnz / nr : 1.0;
  int l = avg >= 96 ? 32 : avg >= 40 ? 16 : avg >= 12 ? 8 : avg >= 6 ? 4 : 1;
  while (l < 64 && (double)nr * l < (double)(1 << 19) && l < avg) l *= 2;
  return l;
}

template <typename TV, bool ADD>
void csr_apply(hipStream_t s, int32_t nr, int64_t nnz, const int32_t *rp, const int32_t *ci,
               const TV *val, const TV *x, TV *y, const int32_t *done) {
  const int lpr = lanes_for(nr, nnz);
  const int32_t g = ceil_div((int64_t)nr * lpr, kBlock);
  switch (lpr) {
    case 1: k_csr_apply<TV, ADD, 1><<<g, kBlock, 0, s>>>(nr, rp, ci, val, x, y, done); break;
    case 2: k_csr_apply<TV, ADD, 2><<<g, kBlock, 0, s>>>(nr, rp, ci, val, x, y, done); break;
    case 4: k_csr_apply<TV, ADD, 4><<<g, kBlock, 0, s>>>(nr, rp, ci, val, x, y, done); break;
    case 8: k_csr_apply<TV, ADD, 8><<<g, kBlock, 0, s>>>(nr, rp, ci, val, x, y, done); break;
    case 16: k_csr_apply<TV, ADD, 16><<<g, kBlock, 0, s>>>(nr, rp, ci, val, x, y, done); break;
    case 32: k_csr_apply<TV, ADD, 32><<<g, kBlock, 0, s>>>(nr, rp, ci, val, x, y, done); break;
    default: k_csr_apply<TV, ADD, 64><<<g, kBlock, 0, s>>>(nr, rp, ci, val, x, y, done); break;
  }
}

template <typename TV, typename TR, int MODE>
void smooth_rows(hipStream_t s, int32_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                 const TV *val, const TV *minv, const TR *r, const TV *z, TV *y,
                 const int32_t *done) {
  const int lpr = lanes_for(n, nnz);
  const int32_t g = ceil_div((int64_t)n * lpr, kBlock);
  switch (lpr) {
    case 1: k_smooth_rows<TV, TR, MODE, 1><<<g, kBlock, 0, s>>>(n, rp, ci, val, minv, r, z, y, done); break;
    case 2: k_smooth_rows<TV, TR, MODE, 2><<<g, kBlock, 0, s>>>(n, rp, ci, val, minv, r, z, y, done); break;
    case 4: k_smooth_rows<TV, TR, MODE, 4><<<g, kBlock, 0, s>>>(n, rp, ci, val, minv, r, z, y, done); break;
    case 8: k_smooth_rows<TV, TR, MODE, 8><<<g, kBlock, 0, s>>>(n, rp, ci, val, minv, r, z, y, done); break;
    case 16: k_smooth_rows<TV, TR, MODE, 16><<<g, kBlock, 0, s>>>(n, rp, ci, val, minv, r, z, y, done); break;
    case 32: k_smooth_rows<TV, TR, MODE, 32><<<g, kBlock, 0, s>>>(n, rp, ci, val, minv, r, z, y, done); break;
    default: k_smooth_rows<TV, TR, MODE, 64><<<g, kBlock, 0, s>>>(n, rp, ci, val, minv, r, z, y, done); break;
  }
}

// Up step: post-smoothing of the coarse level c for this block's kBlock
// coarse rows, y = z_c + M^-1 (r_c - A_c z_c) (kept in LDS), then the
// prolongation z_f += P y over the fine segments of those rows.
template <typename TV>
__global__ void __launch_bounds__(kBlock) k_post_prolong(
    int32_t nc, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const TV *__restrict__ val, const TV *__restrict__ minv, const TV *__restrict__ rcv,
    const TV *__restrict__ zc, const int32_t *__restrict__ seg, const int32_t *__restrict__ aggp,
    const TV *__restrict__ pp, TV *__restrict__ zf, const int32_t *__restrict__ done) {
  __shared__ TV sh[kBlock];
  if (*done) return;
  const int32_t J0 = blockIdx.x * kBlock;
  const int32_t J = J0 + threadIdx.x;
  // the fine range and the row's own operands first: their loads overlap the gathers
  const int32_t J1 = min(nc, J0 + kBlock);
  const int32_t f0 = seg[J0], f1 = seg[J1];
  if (J < nc) {
    const TV zj = zc[J], rj = rcv[J], mj = minv[J];
    int32_t base, w;
    sell_row(sptr, J, &base, &w);
    const TV acc = sell_dot(col, val, base, w, [&](int32_t c) { return zc[c]; });
    sh[threadIdx.x] = zj + (rj - acc) * mj;
  }
  __syncthreads();
  prolong_add(f0, f1, (int32_t)threadIdx.x, kBlock, aggp, pp, zf,
              [&](int32_t a) { return sh[a - J0]; });
}

// Coarsest level with prolongation: z_L = A_L^-1 r_L, then z_f += P z_L over
// all fine positions; one block of 1024 threads. Eight consecutive threads
// share a row (coalesced 64-byte pieces of it), each summing every eighth
// entry against r_L staged in LDS, so 128 rows are in flight per pass.
constexpr int kCoarseSplit = 8;
template <typename TV>
__global__ void __launch_bounds__(1024) k_coarse_prolong(
    int32_t nL, const double *__restrict__ Ainv, const TV *__restrict__ rL, int32_t nf,
    const int32_t *__restrict__ aggp, const TV *__restrict__ pp, TV *__restrict__ zf,
    const int32_t *__restrict__ done) {
  extern __shared__ double sm[];
  if (*done) return;
  double *rs = sm, *zs = sm + nL;
  for (int32_t k = threadIdx.x; k < nL; k += blockDim.x) rs[k] = (double)rL[k];
  __syncthreads();
  const int32_t part = threadIdx.x % kCoarseSplit;
  const int32_t rows_per_pass = blockDim.x / kCoarseSplit;
  for (int32_t i0 = 0; i0 < nL; i0 += rows_per_pass) {
    const int32_t i = i0 + (int32_t)threadIdx.x / kCoarseSplit;
    double s = 0.0;
    if (i < nL) {
      const double *row = Ainv + (int64_t)i * nL;
#pragma unroll 8
      for (int32_t k = part; k < nL; k += kCoarseSplit) s += row[k] * rs[k];
    }
    for (int o = kCoarseSplit / 2; o > 0; o >>= 1) s += __shfl_down(s, o, kCoarseSplit);
    if (i < nL && part == 0) zs[i] = s;
  }
  __syncthreads();
  prolong_add(0, nf, (int32_t)threadIdx.x, (int32_t)blockDim.x, aggp, pp, zf,
              [&](int32_t a) { return (TV)zs[a]; });
}

// Tail of the V-cycle in one block, for a level t = L - 1 small enough for
// LDS (t >= 1, one pre- and one post-sweep): starting from r_t it does the
// down step on t, the coarsest solve, the up step on t, and the
// prolongation into level t - 1 (zf += P_{t-1} y_t), with level t's vectors
// in LDS. Replaces the three latency-bound kernels of the last two levels.
constexpr int kTailMax = 2048;  // largest level t handled in LDS
constexpr int kTailCoarseMax = 512;
constexpr int kTailPro = 8;    // prolongation positions per thread loaded up front (FP32;
                               // half as many in FP64, within the register budget)
constexpr int kTailRow = 16;   // A_L^-1 entries per thread loaded up front (n_L <= 128)
template <typename TV>
__global__ void __launch_bounds__(1024) k_tail(
    int32_t nt, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const TV *__restrict__ sval, const TV *__restrict__ val, const TV *__restrict__ minv,
    const TV *__restrict__ rt, const int32_t *__restrict__ seg, const int32_t *__restrict__ aggp,
    const TV *__restrict__ pp, int32_t nL, const double *__restrict__ Ainv, int32_t nf,
    const int32_t *__restrict__ aggp_f, const TV *__restrict__ pp_f, TV *__restrict__ zf,
    const int32_t *__restrict__ done) {
  __shared__ TV rs[kTailMax], zs[kTailMax], ys[kTailMax];
  __shared__ double rl[kTailCoarseMax], zl[kTailCoarseMax];
  if (*done) return;
  const int32_t tid = threadIdx.x, nth = blockDim.x;
  // The operands of the last two phases do not depend on the first ones:
  // load them now so their latency overlaps the phases before.
  constexpr int kPro = sizeof(TV) == 8 ? kTailPro / 2 : kTailPro;
  int32_t fa[kPro];  // prolongation: this thread's first kPro positions
  TV fp[kPro], fz[kPro];
#pragma unroll
  for (int u = 0; u < kPro; ++u) {
    const int32_t k = tid + u * nth;
    fa[u] = 0;
    fp[u] = fz[u] = 0;
    if (k < nf) {
      fa[u] = aggp_f[k];
      fp[u] = pp_f[k];
      fz[u] = zf[k];
    }
  }
  const int32_t part = tid % kCoarseSplit, irow = tid / kCoarseSplit;
  const bool one_pass = nL <= nth / kCoarseSplit && nL <= kCoarseSplit * kTailRow;
  double av[kTailRow];  // this thread's entries of its A_L^-1 row (one pass)
#pragma unroll
  for (int m = 0; m < kTailRow; ++m) {
    const int32_t k = part + m * kCoarseSplit;
    av[m] = one_pass && irow < nL && k < nL ? Ainv[(int64_t)irow * nL + k] : 0.0;
  }
  // the thread's first row of level t: its slice position, p, its coarse
  // position and its segment bounds, loaded with r so that the later phases
  // start without a round trip to memory
  int32_t b0 = 0, w0 = 0, a0 = 0, sb0 = 0, se0 = 0;
  TV p0 = 0;
  if (tid < nt) {
    const int32_t s = tid / kSlice;
    const int32_t s0 = sptr[s], s1 = sptr[s + 1];
    b0 = s0 + tid % kSlice;
    w0 = (s1 - s0) / kSlice;
    p0 = pp[tid];
    a0 = aggp[tid];
  }
  if (tid < nL) {
    sb0 = seg[tid];
    se0 = seg[tid + 1];
  }
  for (int32_t k = tid; k < nt; k += nth) {
    const TV r = rt[k];
    rs[k] = r;
    zs[k] = r * minv[k];
  }
  __syncthreads();
  // t = p (r - A M^-1 r), kept in ys
  for (int32_t k = tid; k < nt; k += nth) {
    int32_t base = b0, w = w0;
    if (k != tid) {
      const int32_t s = k / kSlice;
      base = sptr[s] + k % kSlice;
      w = (sptr[s + 1] - sptr[s]) / kSlice;
    }
    const TV acc = sell_dot(col, sval, base, w, [&](int32_t c) { return rs[c]; });
    ys[k] = (k == tid ? p0 : pp[k]) * (rs[k] - acc);
  }
  __syncthreads();
  for (int32_t J = tid; J < nL; J += nth) {
    TV a = 0;
    const int32_t mb = J == tid ? sb0 : seg[J], me = J == tid ? se0 : seg[J + 1];
    for (int32_t m = mb; m < me; ++m) a += ys[m];
    rl[J] = (double)a;
  }
  __syncthreads();
  // coarsest: eight threads per row of A_L^-1
  if (one_pass) {
    double a = 0.0;
#pragma unroll
    for (int m = 0; m < kTailRow; ++m)
      if (part + m * kCoarseSplit < nL) a += av[m] * rl[part + m * kCoarseSplit];
    for (int o = kCoarseSplit / 2; o > 0; o >>= 1) a += __shfl_down(a, o, kCoarseSplit);
    if (irow < nL && part == 0) zl[irow] = a;
  } else {
    for (int32_t i0 = 0; i0 < nL; i0 += nth / kCoarseSplit) {
      const int32_t i = i0 + irow;
      double a = 0.0;
      if (i < nL) {
        const double *row = Ainv + (int64_t)i * nL;
#pragma unroll 8
        for (int32_t k = part; k < nL; k += kCoarseSplit) a += row[k] * rl[k];
      }
      for (int o = kCoarseSplit / 2; o > 0; o >>= 1) a += __shfl_down(a, o, kCoarseSplit);
      if (i < nL && part == 0) zl[i] = a;
    }
  }
  __syncthreads();
  for (int32_t k = tid; k < nt; k += nth)
    zs[k] += (k == tid ? p0 : pp[k]) * (TV)zl[k == tid ? a0 : aggp[k]];
  __syncthreads();
  // post-smoothing on level t
  for (int32_t k = tid; k < nt; k += nth) {
    int32_t base = b0, w = w0;
    if (k != tid) {
      const int32_t s = k / kSlice;
      base = sptr[s] + k % kSlice;
      w = (sptr[s + 1] - sptr[s]) / kSlice;
    }
    const TV acc = sell_dot(col, val, base, w, [&](int32_t c) { return zs[c]; });
    ys[k] = zs[k] + (rs[k] - acc) * minv[k];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kPro; ++u) {
    const int32_t k = tid + u * nth;
    if (k < nf) zf[k] = fz[u] + fp[u] * ys[fa[u]];
  }
  prolong_add(kPro * nth, nf, tid, nth, aggp_f, pp_f, zf, [&](int32_t a) { return ys[a]; });
}

// Single-level hierarchy: z = A_0^-1 r, one wavefront per row.
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

// z = M^-1 r (first of several pre-smoothing sweeps)
template <typename TV, typename TR>
__global__ void k_jacobi0(int32_t n, const TV *minv, const TR *r, TV *z, const int32_t *done) {
  if (*done) return;
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = (TV)r[i] * minv[i];
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
// outer CG kernels (FP64, aggregate-major order of level 0)
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

// MODE 0: r = b - A x and partials of (b, b), (r, r)
// MODE 1: partials of ||b - A x||^2 only
template <int MODE, typename TA>
__global__ void __launch_bounds__(kBlock) k_residual_norms(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const TA *__restrict__ val, const double *__restrict__ b, const double *__restrict__ x,
    double *__restrict__ r, double *__restrict__ partials) {
  constexpr int NV = MODE == 0 ? 2 : 1;
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  double d[NV];
  for (int q = 0; q < NV; ++q) d[q] = 0.0;
  for (int32_t row = rb + threadIdx.x; row < re; row += kBlock) {
    int32_t base, w;
    sell_row(sptr, row, &base, &w);
    const double acc = sell_dot_t<double, TA>(col, val, base, w, [&](int32_t c) { return x[c]; });
    const double bi = b[row];
    const double ri = bi - acc;
    if (MODE == 0) {
      r[row] = ri;
      d[0] += bi * bi;
      d[NV - 1] += ri * ri;
    } else {
      d[0] += ri * ri;
    }
  }
  block_partial<NV>(d, partials);
}

__global__ void k_zero_if_zero_rhs(int32_t n, double *x, const PcgScal *scal) {
  if (scal->done != 4) return;
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

// q = A p ; partials of (p, q)
template <typename TA>
__global__ void __launch_bounds__(kBlock) k_spmv_dot(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const TA *__restrict__ val, const double *__restrict__ p, double *__restrict__ q,
    double *__restrict__ partials, const int32_t *__restrict__ done) {
  if (*done) return;
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  double d[1] = {0.0};
  for (int32_t row = rb + threadIdx.x; row < re; row += kBlock) {
    int32_t base, w;
    sell_row(sptr, row, &base, &w);
    const double acc = sell_dot_t<double, TA>(col, val, base, w, [&](int32_t c) { return p[c]; });
    q[row] = acc;
    d[0] += p[row] * acc;
  }
  block_partial<1>(d, partials);
}

// k_spmv_dot with the tile of block b = its row chunk (tiles hrow), XCD-aware order
template <typename TA>
__global__ void __launch_bounds__(kBlock) k_spmv_dot_lds(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const uint16_t *__restrict__ lcol,
    const int32_t *__restrict__ hptr, const int32_t *__restrict__ hidx,
    const TA *__restrict__ val, const double *__restrict__ p, double *__restrict__ q,
    double *__restrict__ partials, const int32_t *__restrict__ done) {
  extern __shared__ double lds_d[];
  if (*done) return;
  int32_t rb, re;
  const int32_t tb = xcd_block(blockIdx.x, gridDim.x);
  rb = (int32_t)((int64_t)tb * chunk);
  re = (int32_t)min((int64_t)n, (int64_t)rb + chunk);
  const int32_t h0 = hptr[tb];
  int32_t row = rb + (int32_t)threadIdx.x, nb = 0, nw = 0;
  if (row < re) sell_row(sptr, row, &nb, &nw);
  stage_tile(lds_d, hidx, h0, hptr[tb + 1] - h0, [&](int32_t c) { return p[c]; });
  double d[1] = {0.0};
  for (; row < re; row += kBlock) {
    const int32_t base = nb, w = nw;
    if (row + kBlock < re) sell_row(sptr, row + kBlock, &nb, &nw);
    const double acc = sell_dot_lds<double, TA>(lcol, val, base, w, lds_d);
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

// p = z + beta p (copy: p = z), W consecutive entries per thread: with W = 2
// one 16-byte access each (z and p 16-byte aligned; an odd last entry alone)
template <int W>
__global__ void k_xpay(int32_t n, const double *__restrict__ z, double *__restrict__ p,
                       const PcgScal *__restrict__ scal, int32_t copy,
                       const int32_t *__restrict__ done) {
  if (*done) return;
  const double beta = scal->beta;
  const int64_t i = W * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  if (W == 2 && i + 1 < n) {
    const double2 zv = reinterpret_cast<const double2 *>(z)[i / 2];
    double2 pv = zv;
    if (!copy) {
      pv = reinterpret_cast<const double2 *>(p)[i / 2];
      pv.x = zv.x + beta * pv.x;
      pv.y = zv.y + beta * pv.y;
    }
    reinterpret_cast<double2 *>(p)[i / 2] = pv;
  } else if (i < n) {
    p[i] = copy ? z[i] : z[i] + beta * p[i];
  }
}

// ---------------------------------------------------------------------------
// K-cycle: two flexible-CG iterations per intermediate level (Section 3.1)
// ---------------------------------------------------------------------------

// v = A c and the block partials of (c, v) and of (c, u) for each given u
// (plane 0: (c, v); plane q >= 1: (c, u_q)), sums in FP64
template <typename TV, int NV, typename TA = TV>
__global__ void __launch_bounds__(kBlock) k_spmv_dots(
    int32_t n, int32_t chunk, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const TA *__restrict__ val, const TV *__restrict__ c, TV *__restrict__ v,
    const TV *__restrict__ u1, const TV *__restrict__ u2, double *__restrict__ partials,
    const int32_t *__restrict__ done) {
  if (*done) return;
  int32_t rb, re;
  rows_of_block(n, chunk, &rb, &re);
  double d[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) d[q] = 0.0;
  for (int32_t row = rb + threadIdx.x; row < re; row += kBlock) {
    int32_t base, w;
    sell_row(sptr, row, &base, &w);
    const TV acc = sell_dot_t<TV, TA>(col, val, base, w, [&](int32_t cc) { return c[cc]; });
    v[row] = acc;
    const double ci = (double)c[row];
    d[0] += ci * (double)acc;
    if (NV > 1) d[1] += ci * (double)u1[row];
    if (NV > 2) d[2] += ci * (double)u2[row];
  }
  block_partial<NV>(d, partials);
}

// One block: the level's second flexible-CG step scalars from the block
// partials (rho1 and s1 = (c1, b) / rho1 come from k_kresid): gamma =
// (c2, v1), rho2 = (c2, v2) - gamma^2 / rho1, s2 = (c2, r1) / rho2,
// a1 = s1 - s2 (gamma / rho1); x = a1 c1 + s2 c2. rho1 <= 0 gives x = 0,
// rho2 <= 0 gives x = s1 c1.
__global__ void __launch_bounds__(1024) k_kfin(int32_t nparts,
                                               const double *__restrict__ partials,
                                               double *__restrict__ ks,
                                               const int32_t *__restrict__ done) {
  const int32_t stop = *done;
  __shared__ double sh[3][1024 / kWave];
  constexpr int nv = 3;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int q = 0; q < nv; ++q) {
    const double *src = partials + (int64_t)q * kMaxParts;
    double a = 0.0;
    for (int32_t b0 = threadIdx.x; b0 < nparts; b0 += 16 * blockDim.x) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int32_t b = b0 + u * (int32_t)blockDim.x;
        v[u] = b < nparts ? src[b] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (b0 + u * (int32_t)blockDim.x < nparts) a += v[u];
    }
    for (int o = kWave / 2; o > 0; o >>= 1) a += __shfl_down(a, o, kWave);
    if (lane == 0) sh[q][wid] = a;
  }
  __syncthreads();
  if (threadIdx.x != 0 || stop) return;
  double tot[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < nv; ++q) {
    double t = sh[q][0];
    for (int k = 1; k < (int)(blockDim.x / kWave); ++k) t += sh[q][k];
    tot[q] = t;
  }
  const double rho1 = ks[kRho1], s1 = ks[kS1];
  const double beta = tot[0], gamma = tot[1], a2 = tot[2];
  if (!(rho1 > 0.0)) {
    ks[kA1] = 0.0;
    ks[kS2] = 0.0;
    return;
  }
  const double rho2 = beta - gamma * gamma / rho1;
  ks[kGamma] = gamma;
  ks[kRho2] = rho2;
  if (!(rho2 > 0.0)) {
    ks[kA1] = s1;
    ks[kS2] = 0.0;
  } else {
    const double s2 = a2 / rho2;
    ks[kS2] = s2;
    ks[kA1] = s1 - s2 * (gamma / rho1);
  }
}

// ---- the deepest flexible-CG step in one block ----
// For the level t just above the coarsest (pre = post = 1), the K-cycle's two
// flexible-CG iterations, each with its cycle (down step, A_L^-1, up step),
// the products, the dot products and the prolongation of x = a1 c1 + s2 c2
// into the level above, in one 1024-thread block with the level's vectors in
// LDS. Same arithmetic as the multi-kernel form; the dot products are summed
// in a fixed order of their own.
constexpr int kKTailMax = 1536;   // largest level t in LDS (five vectors)
constexpr int kKTailCoarse = 128; // coarsest size for the one-pass A_L^-1 product

// sum over the block; every thread gets the same value (fixed order)
__device__ __forceinline__ double block_sum_all(double v, double *red) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = red[0];
  for (int k = 1; k < nw; ++k) t += red[k];
  return t;
}

// One SELL row of the level held in registers (w <= kRowBatch entries):
// loaded once per launch when every thread owns at most one row, then used
// by all six products of the step.
template <typename TV>
struct RegRow {
  int32_t w = 0;
  int32_t c[kRowBatch];
  TV v[kRowBatch], sv[kRowBatch];
  __device__ void load(const int32_t *sptr, const int32_t *col, const TV *val, const TV *sval,
                       int32_t k) {
    const int32_t s = k / kSlice, base = sptr[s] + k % kSlice;
    w = (sptr[s + 1] - sptr[s]) / kSlice;
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      c[u] = 0;
      v[u] = sv[u] = 0;
      if (u < w) {
        c[u] = col[base + u * kSlice];
        v[u] = val[base + u * kSlice];
        sv[u] = sval[base + u * kSlice];
      }
    }
  }
  // sum_e a_e x[c_e] (scaled: A M^-1) in entry order
  template <bool SCALED>
  __device__ TV dot(const TV *x) const {
    TV acc = 0;
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u)
      if (u < w) acc += (SCALED ? sv[u] : v[u]) * x[c[u]];
    return acc;
  }
};

// one K-cycle on level t (iv -> out; the coarse correction is A_L^-1)
template <typename TV, bool REG>
__device__ void ktail_cycle(int32_t nt, const int32_t *__restrict__ sptr,
                            const int32_t *__restrict__ col, const TV *__restrict__ sval,
                            const TV *__restrict__ val, const TV *__restrict__ minv,
                            const TV *__restrict__ pp, const int32_t *__restrict__ seg,
                            const int32_t *__restrict__ aggp, int32_t nL,
                            const double *__restrict__ Ainv, const TV *iv, TV *zs, TV *ys,
                            TV *out, double *rl, double *zl, const RegRow<TV> &rr) {
  const int32_t tid = threadIdx.x, nth = blockDim.x;
  for (int32_t k = tid; k < nt; k += nth) zs[k] = iv[k] * minv[k];
  for (int32_t k = tid; k < nt; k += nth) {
    TV acc;
    if (REG) {
      acc = rr.template dot<true>(iv);
    } else {
      const int32_t s = k / kSlice, base = sptr[s] + k % kSlice,
                    w = (sptr[s + 1] - sptr[s]) / kSlice;
      acc = sell_dot(col, sval, base, w, [&](int32_t c) { return iv[c]; });
    }
    ys[k] = pp[k] * (iv[k] - acc);
  }
  __syncthreads();
  for (int32_t J = tid; J < nL; J += nth) {
    TV a = 0;
    for (int32_t m = seg[J]; m < seg[J + 1]; ++m) a += ys[m];
    rl[J] = (double)a;
  }
  __syncthreads();
  {
    const int32_t part = tid % kCoarseSplit, i = tid / kCoarseSplit;
    double a = 0.0;
    if (i < nL) {
      const double *row = Ainv + (int64_t)i * nL;
#pragma unroll 8
      for (int32_t k = part; k < nL; k += kCoarseSplit) a += row[k] * rl[k];
    }
    for (int o = kCoarseSplit / 2; o > 0; o >>= 1) a += __shfl_down(a, o, kCoarseSplit);
    if (i < nL && part == 0) zl[i] = a;
  }
  __syncthreads();
  for (int32_t k = tid; k < nt; k += nth) zs[k] += pp[k] * (TV)zl[aggp[k]];
  __syncthreads();
  for (int32_t k = tid; k < nt; k += nth) {
    TV acc;
    if (REG) {
      acc = rr.template dot<false>(zs);
    } else {
      const int32_t s = k / kSlice, base = sptr[s] + k % kSlice,
                    w = (sptr[s + 1] - sptr[s]) / kSlice;
      acc = sell_dot(col, val, base, w, [&](int32_t c) { return zs[c]; });
    }
    out[k] = zs[k] + (iv[k] - acc) * minv[k];
  }
  __syncthreads();
}

template <typename TV, bool REG>
__global__ void __launch_bounds__(1024) k_ktail(
    int32_t nt, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const TV *__restrict__ sval, const TV *__restrict__ val, const TV *__restrict__ minv,
    const TV *__restrict__ pp, const int32_t *__restrict__ seg, const int32_t *__restrict__ aggp,
    int32_t nL, const double *__restrict__ Ainv, const TV *__restrict__ b, int32_t nf,
    const int32_t *__restrict__ aggp_f, const TV *__restrict__ pp_f, TV *__restrict__ zf,
    double *__restrict__ ks, const int32_t *__restrict__ done) {
  __shared__ TV IV[kKTailMax], ZS[kKTailMax], YS[kKTailMax], C1[kKTailMax], C2[kKTailMax];
  __shared__ double rl[kKTailCoarse], zl[kKTailCoarse], red[1024 / kWave];
  if (*done) return;
  const int32_t tid = threadIdx.x, nth = blockDim.x;
  constexpr int kRows = kKTailMax / 1024 + 1;  // rows per thread
  // REG: one row per thread (nt <= blockDim.x, rows of at most kRowBatch
  // entries), held in registers for every product of the step
  RegRow<TV> rr;
  if (REG && tid < nt) rr.load(sptr, col, val, sval, tid);
  for (int32_t k = tid; k < nt; k += nth) IV[k] = b[k];
  __syncthreads();
  ktail_cycle<TV, REG>(nt, sptr, col, sval, val, minv, pp, seg, aggp, nL, Ainv, IV, ZS, YS, C1,
                       rl, zl, rr);
  // v1 = A c1, rho1 = (c1, v1), s1 = (c1, b) / rho1
  TV v1[kRows];
  double d0 = 0.0, d1 = 0.0;
#pragma unroll
  for (int u = 0; u < kRows; ++u) {
    const int32_t k = tid + u * nth;
    v1[u] = 0;
    if (k < nt) {
      TV acc;
      if (REG) {
        acc = rr.template dot<false>(C1);
      } else {
        const int32_t s = k / kSlice, base = sptr[s] + k % kSlice,
                      w = (sptr[s + 1] - sptr[s]) / kSlice;
        acc = sell_dot(col, val, base, w, [&](int32_t c) { return C1[c]; });
      }
      v1[u] = acc;
      d0 += (double)C1[k] * (double)acc;
      d1 += (double)C1[k] * (double)IV[k];
    }
  }
  const double rho1 = block_sum_all(d0, red);
  const double cb = block_sum_all(d1, red);
  const double s1 = rho1 > 0.0 ? cb / rho1 : 0.0;
  // r1 = b - s1 v1 (in IV)
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kRows; ++u) {
    const int32_t k = tid + u * nth;
    if (k < nt) IV[k] = IV[k] - (TV)s1 * v1[u];
  }
  __syncthreads();
  ktail_cycle<TV, REG>(nt, sptr, col, sval, val, minv, pp, seg, aggp, nL, Ainv, IV, ZS, YS, C2,
                       rl, zl, rr);
  // v2 = A c2; (c2, v2), gamma = (c2, v1), (c2, r1)
  double e0 = 0.0, e1 = 0.0, e2 = 0.0;
#pragma unroll
  for (int u = 0; u < kRows; ++u) {
    const int32_t k = tid + u * nth;
    if (k < nt) {
      TV acc;
      if (REG) {
        acc = rr.template dot<false>(C2);
      } else {
        const int32_t s = k / kSlice, base = sptr[s] + k % kSlice,
                      w = (sptr[s + 1] - sptr[s]) / kSlice;
        acc = sell_dot(col, val, base, w, [&](int32_t c) { return C2[c]; });
      }
      const double c2 = (double)C2[k];
      e0 += c2 * (double)acc;
      e1 += c2 * (double)v1[u];
      e2 += c2 * (double)IV[k];
    }
  }
  const double beta = block_sum_all(e0, red);
  const double gamma = block_sum_all(e1, red);
  const double a2 = block_sum_all(e2, red);
  double a1 = 0.0, s2 = 0.0;
  if (rho1 > 0.0) {
    const double rho2 = beta - gamma * gamma / rho1;
    if (!(rho2 > 0.0)) {
      a1 = s1;
    } else {
      s2 = a2 / rho2;
      a1 = s1 - s2 * (gamma / rho1);
    }
  }
  if (tid == 0) {
    ks[kRho1] = rho1;
    ks[kS1] = s1;
    ks[kA1] = a1;
    ks[kS2] = s2;
  }
  // z_f += P x, x = a1 c1 + s2 c2
  const TV ta1 = (TV)a1, ts2 = (TV)s2;
  for (int32_t k = tid; k < nf; k += nth) {
    const int32_t J = aggp_f[k];
    zf[k] += pp_f[k] * (ta1 * C1[J] + ts2 * C2[J]);
  }
}

// ---------------------------------------------------------------------------
// iterative coarsest solver (Section 5): CG with the l1-Jacobi diagonal
// ---------------------------------------------------------------------------

// two sums over the block at once; every thread gets both (fixed order)
__device__ __forceinline__ void block_sum2(double &a, double &b, double (*red)[1024 / kWave]) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  for (int o = kWave / 2; o > 0; o >>= 1) {
    a += __shfl_down(a, o, kWave);
    b += __shfl_down(b, o, kWave);
  }
  __syncthreads();
  if (lane == 0) {
    red[0][wid] = a;
    red[1][wid] = b;
  }
  __syncthreads();
  double ta = red[0][0], tb = red[1][0];
  for (int k = 1; k < nw; ++k) {
    ta += red[0][k];
    tb += red[1][k];
  }
  a = ta;
  b = tb;
}

// z_L from A_L z_L = r_L by CG from zero with z = r / m (minv = 1 / m),
// stopped as soon as ||r_k|| < rtol ||r_L|| or after maxit steps. zout (if
// given) receives z_L; then z_f += P z_L over the nf positions of the level
// above (nf = 0: none). One block; thread t owns rows t, t + blockDim.x, ...
// (at most kCgRows), keeps its rows' x, r, q in registers and the search
// direction in LDS for the products; FP64 throughout, A_L in CSR.
constexpr int kCgRows = AMG_MAX_DENSE / 1024;
template <typename TI, typename TO>
__global__ void __launch_bounds__(1024) k_coarse_pcg(
    int32_t nL, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const double *__restrict__ val, const double *__restrict__ minv, double rtol,
    int32_t maxit, const TI *__restrict__ rL, TO *__restrict__ zout, int32_t nf,
    const int32_t *__restrict__ aggp, const TO *__restrict__ pp, TO *__restrict__ zf,
    const int32_t *__restrict__ done) {
  __shared__ double P[AMG_MAX_DENSE];
  __shared__ double red[2][1024 / kWave];
  if (*done) return;
  const int32_t tid = threadIdx.x, nth = blockDim.x;
  double x[kCgRows], r[kCgRows], q[kCgRows];
  double bb = 0.0, rz0 = 0.0;
#pragma unroll
  for (int u = 0; u < kCgRows; ++u) {
    const int32_t i = tid + u * nth;
    x[u] = r[u] = q[u] = 0.0;
    if (i < nL) {
      r[u] = (double)rL[i];
      const double z = r[u] * minv[i];
      P[i] = z;
      bb += r[u] * r[u];
      rz0 += r[u] * z;
    }
  }
  block_sum2(bb, rz0, red);  // also orders the P writes before the first product
  const double bstop = rtol * sqrt(bb);
  for (int32_t it = 0; bb > 0.0 && it < maxit; ++it) {
    // q = A p and (p, q)
    double pq = 0.0, unused = 0.0;
#pragma unroll
    for (int u = 0; u < kCgRows; ++u) {
      const int32_t i = tid + u * nth;
      if (i < nL) {
        double acc = 0.0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) acc += val[k] * P[ci[k]];
        q[u] = acc;
        pq += P[i] * acc;
      }
    }
    block_sum2(pq, unused, red);
    if (!(pq > 0.0)) break;
    const double step = rz0 / pq;
    // x += step p, r -= step q, then ||r||^2 and (r, z) with z = r / m
    double rr = 0.0, rz1 = 0.0;
    double z[kCgRows];
#pragma unroll
    for (int u = 0; u < kCgRows; ++u) {
      const int32_t i = tid + u * nth;
      z[u] = 0.0;
      if (i < nL) {
        x[u] += step * P[i];
        r[u] -= step * q[u];
        z[u] = r[u] * minv[i];
        rr += r[u] * r[u];
        rz1 += r[u] * z[u];
      }
    }
    block_sum2(rr, rz1, red);  // every thread has read P before any rewrites it
    if (sqrt(rr) < bstop) break;
    const double beta = rz1 / rz0;
    rz0 = rz1;
#pragma unroll
    for (int u = 0; u < kCgRows; ++u) {
      const int32_t i = tid + u * nth;
      if (i < nL) P[i] = z[u] + beta * P[i];
    }
    __syncthreads();
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kCgRows; ++u) {
    const int32_t i = tid + u * nth;
    if (i < nL) {
      P[i] = x[u];
      if (zout) zout[i] = (TO)x[u];
    }
  }
  __syncthreads();
  for (int32_t k = tid; k < nf; k += nth) zf[k] += pp[k] * (TO)P[aggp[k]];
}

// threads of the coarsest CG block: one wavefront per 64 rows, at most 1024
inline int32_t coarse_pcg_threads(int32_t nL) {
  const int32_t t = ceil_div(nL, kWave) * kWave;
  return t < kWave ? kWave : (t > 1024 ? 1024 : t);
}

// r1 = b - s1 v1, with s1 = (c1, b) / (c1, v1) from the first step's partials
template <typename TV>
__global__ void __launch_bounds__(kBlock) k_kresid(
    int32_t n, const TV *__restrict__ b, const TV *__restrict__ v1,
    const double *__restrict__ partials, int32_t nparts, double *__restrict__ ks,
    TV *__restrict__ r1, const int32_t *__restrict__ done) {
  if (*done) return;
  // rho1 = (c1, v1) and (c1, b) from the block partials, summed by every
  // block in the same order (so all blocks hold the same s1); block 0 keeps
  // them for the second step and the prolongation
  __shared__ double sh[2][kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  for (int q = 0; q < 2; ++q) {
    const double *src = partials + (int64_t)q * kMaxParts;
    double a = 0.0;
    for (int32_t b0 = threadIdx.x; b0 < nparts; b0 += 16 * kBlock) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int32_t bb = b0 + u * kBlock;
        v[u] = bb < nparts ? src[bb] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (b0 + u * kBlock < nparts) a += v[u];
    }
    for (int o = kWave / 2; o > 0; o >>= 1) a += __shfl_down(a, o, kWave);
    if (lane == 0) sh[q][wid] = a;
  }
  __syncthreads();
  double rho1 = sh[0][0], cb = sh[1][0];
  for (int k = 1; k < kBlock / kWave; ++k) {
    rho1 += sh[0][k];
    cb += sh[1][k];
  }
  const double s1 = rho1 > 0.0 ? cb / rho1 : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ks[kRho1] = rho1;
    ks[kS1] = s1;
  }
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r1[i] = b[i] - (TV)s1 * v1[i];
}

// z_f += P x with x = a1 c1 + s2 c2 formed per coarse position
template <typename TV>
__global__ void k_kprolong(int32_t nf, const int32_t *__restrict__ aggp,
                           const TV *__restrict__ pp, const TV *__restrict__ c1,
                           const TV *__restrict__ c2, const double *__restrict__ ks,
                           TV *__restrict__ zf, const int32_t *__restrict__ done) {
  if (*done) return;
  const TV a1 = (TV)ks[kA1], s2 = (TV)ks[kS2];
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nf) {
    const int32_t J = aggp[k];
    zf[k] += pp[k] * (a1 * c1[J] + s2 * c2[J]);
  }
}

// ---------------------------------------------------------------------------
// host: the V-cycle for one hierarchy precision
// ---------------------------------------------------------------------------

template <typename TV>
const TV *vals(const Level &L);
template <>
const double *vals<double>(const Level &L) { return L.S.v64; }
template <>
const float *vals<float>(const Level &L) { return L.S.v32; }
template <typename TV>
const TV *svals(const Level &L);
template <>
const double *svals<double>(const Level &L) { return L.S.s64; }
template <>
const float *svals<float>(const Level &L) { return L.S.s32; }
template <typename TV>
const TV *minv(const Level &L);
template <>
const double *minv<double>(const Level &L) { return L.sminv64; }
template <>
const float *minv<float>(const Level &L) { return L.sminv32; }
template <typename TV>
const TV *ppv(const Level &L);
template <>
const double *ppv<double>(const Level &L) { return L.pp64; }
template <>
const float *ppv<float>(const Level &L) { return L.pp32; }

template <typename TV>
const TV *pbar_vals(const Level &L);
template <>
const double *pbar_vals<double>(const Level &L) { return L.sp_v64; }
template <>
const float *pbar_vals<float>(const Level &L) { return L.sp_v32; }
template <typename TV>
const TV *lr_vals(const Level &L);
template <>
const double *lr_vals<double>(const Level &L) { return L.lr_v64; }
template <>
const float *lr_vals<float>(const Level &L) { return L.lr_v32; }
template <typename TV>
const TV *pbart_vals(const Level &L);
template <>
const double *pbart_vals<double>(const Level &L) { return L.st_v64; }
template <>
const float *pbart_vals<float>(const Level &L) { return L.st_v32; }

// In-solve timing probe. arm_probe(h, id) marks the next launch made through
// launch_k as the timed one when kernel `id` is being timed (never during
// graph capture, whose probe_id is -1); launch_k then launches it with
// hipExtLaunchKernelGGL and the next pair of probe events, which the runtime
// stamps at that dispatch's own start and end (no marker packets around it).
inline void arm_probe(amg_hierarchy *h, int32_t id) { h->probe_armed = h->probe_id == id; }

template <typename K, typename... Args>
void launch_k(const amg_hierarchy *h, K k, dim3 grid, dim3 block, uint32_t shmem, hipStream_t s,
              Args... args) {
  if (h->probe_armed && h->probe_next + 2 <= h->probe_ev.size()) {
    h->probe_armed = false;
    hipEvent_t e0 = h->probe_ev[h->probe_next], e1 = h->probe_ev[h->probe_next + 1];
    h->probe_next += 2;
    hipExtLaunchKernelGGL(k, grid, block, shmem, s, e0, e1, 0, args...);
    return;
  }
  hipLaunchKernelGGL(k, grid, block, shmem, s, args...);
}

// rows per thread of the down step on a level of n rows: 2 on levels of 2^21
// to kManyRows rows (160^3 level 0: 79.4 -> 78.1 us; 4 rows: 83 us; on
// 16.7 M rows 2 rows were slower)
inline int down_rows(int64_t n) { return n >= (1 << 21) && n < kManyRows ? 2 : 1; }

void finalize(amg_hierarchy *h, int32_t op, int32_t nparts, const int32_t *done) {
  k_finalize<<<1, 1024, 0, h->stream>>>(op, nparts, h->partials, h->scal, done);
}

int32_t coarse_per_block(const amg_hierarchy *h) {
  const int32_t g = kBlock / h->max_seg;
  return g < 1 ? 1 : g;
}

// coarse rows per block of the LDS-staged down step (one fine row per thread:
// with its operands loaded ahead of the staging barrier, two rows per thread
// held more registers than they hid latency)
int32_t staged_down_G(const amg_hierarchy *h) { return coarse_per_block(h); }

// Down step of level F into C: LDS-staged gathers where the level has tiles of
// that geometry, else down_rows(n) fine rows per thread gathering from memory.
template <typename TV, typename TR, int MODE, typename TA>
void pre_restrict(const amg_hierarchy *h, const Level &F, const Level &C, const TA *val,
                  const TV *mv, const TV *pp, const TR *r, TV *z, TV *rc, const int32_t *done) {
  hipStream_t s = h->stream;
  const int32_t Gt = staged_down_G(h);
  if (F.hseg.ok() && F.hseg.param == Gt && F.hseg.ntiles == ceil_div(C.n, Gt)) {
    const Halo &H = F.hseg;
    launch_k(h, k_pre_restrict_lds<TV, TR, MODE, TA, 1>, dim3(ceil_div(C.n, Gt)), dim3(kBlock),
             (uint32_t)(sizeof(TV) * H.umax), s, C.n, Gt, F.seg, F.S.sptr,
             (const uint16_t *)H.lcol, (const int32_t *)H.hptr, (const int32_t *)H.hidx, val, mv,
             pp, r, z, rc, done);
    return;
  }
  const int R = down_rows(F.n);
  const int32_t G = coarse_per_block(h) * R;
  const int32_t grid = ceil_div(C.n, G);
  auto k = R == 2 ? k_pre_restrict<TV, TR, MODE, TA, 2> : k_pre_restrict<TV, TR, MODE, TA, 1>;
  launch_k(h, k, dim3(grid), dim3(kBlock), 0u, s, C.n, G, F.seg, F.S.sptr, F.S.col, val, mv, pp,
           r, z, rc, done);
}

// y = z + M^-1 (r - A z) on a level (DOT: with the block partials of the CG
// dot), with LDS-staged gathers where the level has row tiles
template <typename TV, typename TR, typename TO, bool DOT, typename TA>
void post_sweep(const amg_hierarchy *h, const Level &F, const TA *val, const TV *minv,
                const TR *r, const TV *z, TO *y, double *partials, const int32_t *done,
                const double *dv = nullptr) {
  hipStream_t s = h->stream;
  const Geom g = geom(F.n);
  if (F.hrow.ok() && F.hrow.param == g.chunk && F.hrow.ntiles == g.grid) {
    const Halo &H = F.hrow;
    launch_k(h, k_post_lds<TV, TR, TO, DOT, TA>, dim3(g.grid), dim3(kBlock),
             (uint32_t)(sizeof(TV) * H.umax), s, F.n, g.chunk, F.S.sptr,
             (const uint16_t *)H.lcol, (const int32_t *)H.hptr, (const int32_t *)H.hidx, val,
             minv, r, z, y, partials, done, dv);
    return;
  }
  launch_k(h, k_post<TV, TR, TO, DOT, TA>, dim3(g.grid), dim3(kBlock), 0u, s, F.n, g.chunk,
           F.S.sptr, F.S.col, val, minv, r, z, y, partials, done, dv);
}

// q = A p with the block partials of (p, q) on level 0 (A from its exact FP32
// copy when there is one), with LDS-staged gathers where there are row tiles
inline void spmv_dot0(const amg_hierarchy *h, const double *p, double *q, const int32_t *done) {
  hipStream_t s = h->stream;
  const Level &F = h->lv[0];
  const Geom g = geom(F.n);
  if (F.hrow.ok() && F.hrow.param == g.chunk && F.hrow.ntiles == g.grid) {
    const Halo &H = F.hrow;
    const uint32_t shmem = (uint32_t)(sizeof(double) * H.umax);
    if (F.S.exact32)
      launch_k(h, k_spmv_dot_lds<float>, dim3(g.grid), dim3(kBlock), shmem, s, F.n, g.chunk,
               F.S.sptr, (const uint16_t *)H.lcol, (const int32_t *)H.hptr,
               (const int32_t *)H.hidx, (const float *)F.S.v32, p, q, h->partials, done);
    else
      launch_k(h, k_spmv_dot_lds<double>, dim3(g.grid), dim3(kBlock), shmem, s, F.n, g.chunk,
               F.S.sptr, (const uint16_t *)H.lcol, (const int32_t *)H.hptr,
               (const int32_t *)H.hidx, (const double *)F.S.v64, p, q, h->partials, done);
    return;
  }
  if (F.S.exact32)
    launch_k(h, k_spmv_dot<float>, dim3(g.grid), dim3(kBlock), 0u, s, F.n, g.chunk, F.S.sptr,
             F.S.col, (const float *)F.S.v32, p, q, h->partials, done);
  else
    launch_k(h, k_spmv_dot<double>, dim3(g.grid), dim3(kBlock), 0u, s, F.n, g.chunk, F.S.sptr,
             F.S.col, (const double *)F.S.v64, p, q, h->partials, done);
}

// whether the products of level l read A from its exact FP32 copy: level 0
// of an FP64 hierarchy whose values are all FP32 numbers (same arithmetic)
template <typename TV>
bool reads32(const Level &F, int32_t l) {
  return l == 0 && sizeof(TV) == 8 && F.S.exact32;
}

// whether level F's one-sweep down step forms z = M^-1 r in LDS and reads
// the plain A: an FP64 level with down-step tiles whose values are all FP32
// numbers. With level 0's exact FP32 copy of A that is 4 value bytes per
// entry instead of the 8 of A M^-1; with the copy switched off the same
// arithmetic (so the copy changes no result bit) at 8 bytes. Other operators
// stage r alone and read A M^-1: staging M^-1 r would gather 1 / m as well
// for no saving.
template <typename TV>
bool staged_down(const amg_hierarchy *h, const Level &F, const Level &C) {
  const int32_t G = staged_down_G(h);
  return sizeof(TV) == 8 && F.S.fp32_values && F.hseg.ok() && F.hseg.param == G &&
         F.hseg.ntiles == ceil_div(C.n, G);
}

// the one-sweep down step of level F (z = M^-1 r, residual, restriction)
template <typename TV, typename TR>
void down_one_sweep(const amg_hierarchy *h, const Level &F, const Level &C, const TR *r, TV *z,
                    const int32_t *done) {
  if (staged_down<TV>(h, F, C) && F.S.exact32)
    pre_restrict<TV, TR, kPreStagedZ, float>(h, F, C, F.S.v32, minv<TV>(F), ppv<TV>(F), r, z,
                                             (TV *)C.r, done);
  else if (staged_down<TV>(h, F, C))
    pre_restrict<TV, TR, kPreStagedZ, TV>(h, F, C, vals<TV>(F), minv<TV>(F), ppv<TV>(F), r, z,
                                          (TV *)C.r, done);
  else
    pre_restrict<TV, TR, kPreScaled, TV>(h, F, C, svals<TV>(F), minv<TV>(F), ppv<TV>(F), r, z,
                                         (TV *)C.r, done);
}

// down step on level l: smoothing from zero, residual, restriction into
// level l + 1's right-hand side; returns the buffer holding z_l
template <typename TV, typename TR>
TV *launch_down(amg_hierarchy *h, int32_t l, const TR *r, const int32_t *done) {
  hipStream_t s = h->stream;
  Level &F = h->lv[l];
  Level &C = h->lv[l + 1];
  TV *z = (TV *)F.z, *tmp = (TV *)F.y;
  if (h->params.pre == 1) {
    down_one_sweep<TV, TR>(h, F, C, r, z, done);
    return z;
  }
  const Geom g = geom(F.n);
  const bool a32 = reads32<TV>(F, l);
  k_jacobi0<TV, TR><<<grid1(F.n), kBlock, 0, s>>>(F.n, minv<TV>(F), r, z, done);
  for (int32_t k = 1; k < h->params.pre; ++k) {
    if (a32)
      k_post<TV, TR, TV, false, float><<<g.grid, kBlock, 0, s>>>(
          F.n, g.chunk, F.S.sptr, F.S.col, F.S.v32, minv<TV>(F), r, z, tmp, nullptr, done);
    else
      k_post<TV, TR, TV, false><<<g.grid, kBlock, 0, s>>>(F.n, g.chunk, F.S.sptr, F.S.col,
                                                         vals<TV>(F), minv<TV>(F), r, z, tmp,
                                                         nullptr, done);
    std::swap(z, tmp);
  }
  if (a32)
    pre_restrict<TV, TR, kPreFromZ, float>(h, F, C, F.S.v32, minv<TV>(F), ppv<TV>(F), r, z,
                                           (TV *)C.r, done);
  else
    pre_restrict<TV, TR, kPreFromZ, TV>(h, F, C, vals<TV>(F), minv<TV>(F), ppv<TV>(F), r, z,
                                        (TV *)C.r, done);
  return z;
}

// up step on coarse level c >= 1: extra post sweeps, then the last sweep
// fused with the prolongation into the finer level's z (zf)
template <typename TV>
void launch_up(amg_hierarchy *h, int32_t c, TV *zc, TV *zf, const int32_t *done) {
  hipStream_t s = h->stream;
  Level &C = h->lv[c];
  Level &F = h->lv[c - 1];
  TV *tmp = (TV *)C.y;
  if (tmp == zc) tmp = (TV *)C.z;
  const Geom g = geom(C.n);
  for (int32_t k = 1; k < h->params.post; ++k) {
    k_post<TV, TV, TV, false><<<g.grid, kBlock, 0, s>>>(C.n, g.chunk, C.S.sptr, C.S.col,
                                                       vals<TV>(C), minv<TV>(C), (const TV *)C.r,
                                                       zc, tmp, nullptr, done);
    std::swap(zc, tmp);
  }
  k_post_prolong<TV><<<grid1(C.n), kBlock, 0, s>>>(C.n, C.S.sptr, C.S.col, vals<TV>(C),
                                                   minv<TV>(C), (const TV *)C.r, zc, F.seg,
                                                   F.aggp, ppv<TV>(F), zf, done);
}

inline bool coarse_is_pcg(const amg_hierarchy *h) {
  return h->params.coarse_solver == AMG_COARSE_PCG;
}

// The coarsest solve by CG (coarse_is_pcg): z_L into zout and/or
// prolongated into zf (nf positions of the level above).
template <typename TI, typename TO>
void launch_coarse_pcg(amg_hierarchy *h, const TI *rL, TO *zout, int32_t nf,
                       const int32_t *aggp, const TO *pp, TO *zf, const int32_t *done) {
  const Level &C = h->lv.back();
  k_coarse_pcg<TI, TO><<<1, coarse_pcg_threads(C.n), 0, h->stream>>>(
      C.n, C.rp, C.ci, C.val, C.minv64, h->params.coarse_rtol, h->params.coarse_maxit, rL, zout,
      nf, aggp, pp, zf, done);
}

// z0 = coarsest solve of r0 when level 0 is the coarsest level; with dot,
// the partials of (dv, z0) (dv = NULL: of (r0, z0), finalized into rho)
void one_level_cycle(amg_hierarchy *h, const double *r0, double *z0, bool dot, const double *dv,
                     const int32_t *done) {
  hipStream_t s = h->stream;
  const int32_t n = h->C.n;
  if (coarse_is_pcg(h))
    launch_coarse_pcg<double, double>(h, r0, z0, 0, nullptr, nullptr, nullptr, done);
  else
    k_coarse_solve<double, double><<<ceil_div(n, kCoarseWaves), kWave * kCoarseWaves, 0, s>>>(
        n, h->C.Ainv, r0, z0, done);
  if (dot) {
    const Geom g = geom(h->lv[0].n);
    k_dot_rz<<<g.grid, kBlock, 0, s>>>(h->lv[0].n, g.chunk, dv ? dv : r0, z0, h->partials, done);
    if (!dv) finalize(h, kFinRZ, g.grid, done);
  }
}

// Level 0 after the coarse correction (z holds it): post - 1 extra sweeps,
// then the last into z0, with dot the block partials of (r0, z0) finalized
// into the CG scalars, or of (dv, z0) left to the caller.
template <typename TV>
void level0_post(amg_hierarchy *h, const double *r0, TV *z, double *z0, bool dot,
                 const double *dv, const int32_t *done) {
  hipStream_t s = h->stream;
  Level &F = h->lv[0];
  TV *tmp = (TV *)F.y;
  if (tmp == z) tmp = (TV *)F.z;
  const Geom g = geom(F.n);
  // an FP64 hierarchy reads A from its exact FP32 copy when there is one
  const bool a32 = reads32<TV>(F, 0);
  for (int32_t k = 1; k < h->params.post; ++k) {
    if (a32)
      post_sweep<TV, double, TV, false, float>(h, F, F.S.v32, minv<TV>(F), r0, z, tmp, nullptr,
                                               done);
    else
      post_sweep<TV, double, TV, false, TV>(h, F, vals<TV>(F), minv<TV>(F), r0, z, tmp, nullptr,
                                            done);
    std::swap(z, tmp);
  }
  if (dot) {
    arm_probe(h, 1);
    if (a32)
      post_sweep<TV, double, double, true, float>(h, F, F.S.v32, minv<TV>(F), r0, z, z0,
                                                  h->partials, done, dv);
    else
      post_sweep<TV, double, double, true, TV>(h, F, vals<TV>(F), minv<TV>(F), r0, z, z0,
                                               h->partials, done, dv);
    h->probe_armed = false;
    if (!dv) finalize(h, kFinRZ, g.grid, done);
  } else {
    if (a32)
      post_sweep<TV, double, double, false, float>(h, F, F.S.v32, minv<TV>(F), r0, z, z0,
                                                   nullptr, done);
    else
      post_sweep<TV, double, double, false, TV>(h, F, vals<TV>(F), minv<TV>(F), r0, z, z0,
                                                nullptr, done);
  }
}

// Down step of the smoothed-aggregation cycle on level l: z from the
// pre-smoothing sweeps and the residual t = r - A z (both left in the level's
// buffers); returns the buffer holding z.
template <typename TV, typename TR>
TV *down_sa(amg_hierarchy *h, int32_t l, const TR *r, const int32_t *done) {
  hipStream_t s = h->stream;
  Level &F = h->lv[l];
  TV *z = (TV *)F.z, *y = (TV *)F.y, *t = (TV *)F.t;
  const Geom g = geom(F.n);
  if (F.lr_rp) {  // long rows: several lanes per row
    k_jacobi0<TV, TR><<<grid1(F.n), kBlock, 0, s>>>(F.n, minv<TV>(F), r, z, done);
    for (int32_t k = 1; k < h->params.pre; ++k) {
      smooth_rows<TV, TR, 0>(s, F.n, F.nnz, F.lr_rp, F.lr_ci, lr_vals<TV>(F), minv<TV>(F), r, z,
                             y, done);
      std::swap(z, y);
    }
    smooth_rows<TV, TR, 1>(s, F.n, F.nnz, F.lr_rp, F.lr_ci, lr_vals<TV>(F), minv<TV>(F), r, z, t,
                           done);
    return z;
  }
  if (h->params.pre == 1) {
    k_pre_resid<TV, TR><<<g.grid, kBlock, 0, s>>>(F.n, g.chunk, F.S.sptr, F.S.col, svals<TV>(F),
                                                  minv<TV>(F), r, z, t, done);
    return z;
  }
  const bool a32 = reads32<TV>(F, l);
  k_jacobi0<TV, TR><<<grid1(F.n), kBlock, 0, s>>>(F.n, minv<TV>(F), r, z, done);
  for (int32_t k = 1; k < h->params.pre; ++k) {
    if (a32)
      k_post<TV, TR, TV, false, float><<<g.grid, kBlock, 0, s>>>(
          F.n, g.chunk, F.S.sptr, F.S.col, F.S.v32, minv<TV>(F), r, z, y, nullptr, done);
    else
      k_post<TV, TR, TV, false><<<g.grid, kBlock, 0, s>>>(F.n, g.chunk, F.S.sptr, F.S.col,
                                                         vals<TV>(F), minv<TV>(F), r, z, y,
                                                         nullptr, done);
    std::swap(z, y);
  }
  if (a32)
    k_resid<TV, TR, float><<<g.grid, kBlock, 0, s>>>(F.n, g.chunk, F.S.sptr, F.S.col, F.S.v32, r,
                                                     z, t, done);
  else
    k_resid<TV, TR><<<g.grid, kBlock, 0, s>>>(F.n, g.chunk, F.S.sptr, F.S.col, vals<TV>(F), r, z,
                                              t, done);
  return z;
}

// The V-cycle with smoothed prolongators (L >= 1): per level the down step,
// r_{l+1} = Pbar^T t; the coarsest solve; then per level z_l += Pbar z_{l+1}
// and the post-smoothing sweeps.
template <typename TV>
void vcycle_sa_t(amg_hierarchy *h, const double *r0, double *z0, bool dot, const double *dv,
                 const int32_t *done) {
  hipStream_t s = h->stream;
  const int32_t L = (int32_t)h->lv.size() - 1;
  std::vector<TV *> zb(L);
  for (int32_t l = 0; l < L; ++l) {
    Level &F = h->lv[l];
    Level &C = h->lv[l + 1];
    zb[l] = l == 0 ? down_sa<TV, double>(h, 0, r0, done)
                   : down_sa<TV, TV>(h, l, (const TV *)F.r, done);
    csr_apply<TV, false>(s, C.n, F.pb_nnz, F.st_rp, F.st_ci, pbart_vals<TV>(F), (const TV *)F.t,
                         (TV *)C.r, done);
  }
  Level &Cl = h->lv[L];
  TV *zc = (TV *)Cl.z;
  const int32_t nL = h->C.n;
  if (coarse_is_pcg(h))
    launch_coarse_pcg<TV, TV>(h, (const TV *)Cl.r, zc, 0, nullptr, nullptr, nullptr, done);
  else
    k_coarse_solve<TV, TV><<<ceil_div(nL, kCoarseWaves), kWave * kCoarseWaves, 0, s>>>(
        nL, h->C.Ainv, (const TV *)Cl.r, zc, done);
  for (int32_t l = L - 1; l >= 1; --l) {
    Level &F = h->lv[l];
    csr_apply<TV, true>(s, F.n, F.pb_nnz, F.sp_rp, F.sp_ci, pbar_vals<TV>(F), zc, zb[l], done);
    TV *z = zb[l], *tmp = z == (TV *)F.z ? (TV *)F.y : (TV *)F.z;
    const Geom g = geom(F.n);
    for (int32_t k = 0; k < h->params.post; ++k) {
      if (F.lr_rp)
        smooth_rows<TV, TV, 0>(s, F.n, F.nnz, F.lr_rp, F.lr_ci, lr_vals<TV>(F), minv<TV>(F),
                               (const TV *)F.r, z, tmp, done);
      else
        k_post<TV, TV, TV, false><<<g.grid, kBlock, 0, s>>>(F.n, g.chunk, F.S.sptr, F.S.col,
                                                           vals<TV>(F), minv<TV>(F),
                                                           (const TV *)F.r, z, tmp, nullptr,
                                                           done);
      std::swap(z, tmp);
    }
    zc = z;
  }
  Level &F0 = h->lv[0];
  csr_apply<TV, true>(s, F0.n, F0.pb_nnz, F0.sp_rp, F0.sp_ci, pbar_vals<TV>(F0), zc, zb[0],
                      done);
  level0_post<TV>(h, r0, zb[0], z0, dot, dv, done);
}

// V-cycle z0 = B r0 on the aggregate-major vectors of level 0. With dot, the
// last kernel also writes the block partials of (r0, z0), finalized into the
// CG scalars, or, with a dot partner dv, of (dv, z0), left to the caller.
template <typename TV>
void vcycle_t(amg_hierarchy *h, const double *r0, double *z0, bool dot, const double *dv,
              const int32_t *done) {
  hipStream_t s = h->stream;
  const int32_t L = (int32_t)h->lv.size() - 1;
  if (L == 0) {
    one_level_cycle(h, r0, z0, dot, dv, done);
    return;
  }
  if (h->params.smooth_p) {
    vcycle_sa_t<TV>(h, r0, z0, dot, dv, done);
    return;
  }
  std::vector<TV *> zb(L);
  const bool tail = L >= 2 && h->params.pre == 1 && h->params.post == 1 &&
                    h->lv[L - 1].n <= kTailMax && h->C.n <= kTailCoarseMax && !coarse_is_pcg(h);
  const int32_t down_end = tail ? L - 1 : L;  // levels [0, down_end) take the down step
  arm_probe(h, 0);
  zb[0] = launch_down<TV, double>(h, 0, r0, done);
  h->probe_armed = false;
  for (int32_t l = 1; l < down_end; ++l)
    zb[l] = launch_down<TV, TV>(h, l, (const TV *)h->lv[l].r, done);
  if (tail) {
    Level &T = h->lv[L - 1];
    Level &F = h->lv[L - 2];
    k_tail<TV><<<1, 1024, 0, s>>>(T.n, T.S.sptr, T.S.col, svals<TV>(T), vals<TV>(T), minv<TV>(T),
                                  (const TV *)T.r, T.seg, T.aggp, ppv<TV>(T), h->C.n, h->C.Ainv,
                                  F.n, F.aggp, ppv<TV>(F), zb[L - 2], done);
    for (int32_t c = L - 2; c >= 1; --c) launch_up<TV>(h, c, zb[c], zb[c - 1], done);
  } else {
    Level &F = h->lv[L - 1];
    const int32_t nL = h->C.n;
    if (coarse_is_pcg(h))
      launch_coarse_pcg<TV, TV>(h, (const TV *)h->lv[L].r, nullptr, F.n, F.aggp, ppv<TV>(F),
                                zb[L - 1], done);
    else
      k_coarse_prolong<TV><<<1, 1024, 2 * sizeof(double) * nL, s>>>(
          nL, h->C.Ainv, (const TV *)h->lv[L].r, F.n, F.aggp, ppv<TV>(F), zb[L - 1], done);
    for (int32_t c = L - 1; c >= 1; --c) launch_up<TV>(h, c, zb[c], zb[c - 1], done);
  }
  level0_post<TV>(h, r0, zb[0], z0, dot, dv, done);
}

// ---- K-cycle (Section 3.1) ----

template <typename TV>
void fcg2_t(amg_hierarchy *h, int32_t m, const int32_t *done);

// K-cycle on level l < L. in: the level's right-hand side (level 0: the FP64
// CG residual); out: the result (level 0: FP64). With a dot partner dv the
// last post-sweep also writes the block partials of (dv, out).
template <typename TV, typename TR, typename TO>
void kcycle_t(amg_hierarchy *h, int32_t l, const TR *in, TO *out, const double *dv,
              const int32_t *done) {
  hipStream_t s = h->stream;
  const int32_t L = (int32_t)h->lv.size() - 1;
  Level &F = h->lv[l];
  TV *z = launch_down<TV, TR>(h, l, in, done);
  if (l + 1 == L) {
    const int32_t nL = h->C.n;
    if (coarse_is_pcg(h))
      launch_coarse_pcg<TV, TV>(h, (const TV *)h->lv[L].r, nullptr, F.n, F.aggp, ppv<TV>(F), z,
                                done);
    else
      k_coarse_prolong<TV><<<1, 1024, 2 * sizeof(double) * nL, s>>>(
          nL, h->C.Ainv, (const TV *)h->lv[L].r, F.n, F.aggp, ppv<TV>(F), z, done);
  } else if (l + 2 == L && h->params.pre == 1 && h->params.post == 1 &&
             h->lv[l + 1].n <= kKTailMax && h->C.n <= kKTailCoarse && !coarse_is_pcg(h)) {
    const Level &T = h->lv[l + 1];
    auto kt = T.n <= 1024 && T.S.max_width <= kRowBatch ? k_ktail<TV, true> : k_ktail<TV, false>;
    kt<<<1, 1024, 0, s>>>(T.n, T.S.sptr, T.S.col, svals<TV>(T), vals<TV>(T), minv<TV>(T),
                          ppv<TV>(T), T.seg, T.aggp, h->C.n, h->C.Ainv, (const TV *)T.r, F.n,
                          F.aggp, ppv<TV>(F), z, h->kscal + (int64_t)(l + 1) * kKScal, done);
  } else {
    const Level &C = h->lv[l + 1];
    fcg2_t<TV>(h, l + 1, done);
    k_kprolong<TV><<<grid1(F.n), kBlock, 0, s>>>(F.n, F.aggp, ppv<TV>(F), (const TV *)C.c1,
                                                 (const TV *)C.c2,
                                                 h->kscal + (int64_t)(l + 1) * kKScal, z, done);
  }
  // post-smoothing: post - 1 sweeps alternating two level buffers, the last
  // into out
  TV *tmp = (TV *)F.y;
  if (tmp == z) tmp = (TV *)F.z;
  const Geom g = geom(F.n);
  const bool a32 = reads32<TV>(F, l);
  for (int32_t k = 1; k < h->params.post; ++k) {
    if (a32)
      k_post<TV, TR, TV, false, float><<<g.grid, kBlock, 0, s>>>(
          F.n, g.chunk, F.S.sptr, F.S.col, F.S.v32, minv<TV>(F), in, z, tmp, nullptr, done);
    else
      k_post<TV, TR, TV, false><<<g.grid, kBlock, 0, s>>>(F.n, g.chunk, F.S.sptr, F.S.col,
                                                         vals<TV>(F), minv<TV>(F), in, z, tmp,
                                                         nullptr, done);
    std::swap(z, tmp);
  }
  if (dv && a32)
    k_post<TV, TR, TO, true, float><<<g.grid, kBlock, 0, s>>>(
        F.n, g.chunk, F.S.sptr, F.S.col, F.S.v32, minv<TV>(F), in, z, out, h->partials, done, dv);
  else if (dv)
    k_post<TV, TR, TO, true><<<g.grid, kBlock, 0, s>>>(F.n, g.chunk, F.S.sptr, F.S.col,
                                                      vals<TV>(F), minv<TV>(F), in, z, out,
                                                      h->partials, done, dv);
  else if (a32)
    k_post<TV, TR, TO, false, float><<<g.grid, kBlock, 0, s>>>(
        F.n, g.chunk, F.S.sptr, F.S.col, F.S.v32, minv<TV>(F), in, z, out, nullptr, done);
  else
    k_post<TV, TR, TO, false><<<g.grid, kBlock, 0, s>>>(F.n, g.chunk, F.S.sptr, F.S.col,
                                                       vals<TV>(F), minv<TV>(F), in, z, out,
                                                       nullptr, done);
}

// Two flexible-CG iterations on level m (0 < m < L) for the right-hand side
// the level above restricted into lv[m].r, from zero; the result stays as
// x = a1 c1 + s2 c2 (vectors c1, c2 of the level, scalars in its kscal slot)
// for the prolongation to combine.
template <typename TV>
void fcg2_t(amg_hierarchy *h, int32_t m, const int32_t *done) {
  hipStream_t s = h->stream;
  Level &M = h->lv[m];
  const int32_t n = M.n;
  const TV *b = (const TV *)M.r;
  double *ks = h->kscal + (int64_t)m * kKScal;
  const Geom g = geom(n);
  kcycle_t<TV, TV, TV>(h, m, b, (TV *)M.c1, nullptr, done);
  k_spmv_dots<TV, 2><<<g.grid, kBlock, 0, s>>>(n, g.chunk, M.S.sptr, M.S.col, vals<TV>(M),
                                               (const TV *)M.c1, (TV *)M.v1, b, nullptr,
                                               h->partials, done);
  k_kresid<TV><<<grid1(n), kBlock, 0, s>>>(n, b, (const TV *)M.v1, h->partials, g.grid, ks,
                                           (TV *)M.r1, done);
  kcycle_t<TV, TV, TV>(h, m, (const TV *)M.r1, (TV *)M.c2, nullptr, done);
  k_spmv_dots<TV, 3><<<g.grid, kBlock, 0, s>>>(n, g.chunk, M.S.sptr, M.S.col, vals<TV>(M),
                                               (const TV *)M.c2, (TV *)M.v2,
                                               (const TV *)M.v1, (const TV *)M.r1,
                                               h->partials, done);
  k_kfin<<<1, 1024, 0, s>>>(g.grid, h->partials, ks, done);
}

// z0 = K r0 on the aggregate-major level-0 vectors (with dv: the partials of
// (dv, z0) as well)
template <typename TV>
void kcycle_top(amg_hierarchy *h, const double *r0, double *z0, const double *dv,
                const int32_t *done) {
  const int32_t L = (int32_t)h->lv.size() - 1;
  if (L == 0) {
    if (dv) one_level_cycle(h, r0, z0, true, dv, done);
    else one_level_cycle(h, r0, z0, false, nullptr, done);
    return;
  }
  kcycle_t<TV, double, double>(h, 0, r0, z0, dv, done);
}

amg_status alloc_level_vectors(amg_hierarchy *h, Level &L, size_t vbytes) {
  AMG_TRY(dev_alloc(h, &L.r, vbytes * L.n + 16));
  AMG_TRY(dev_alloc(h, &L.z, vbytes * L.n + 16));
  AMG_TRY(dev_alloc(h, &L.t, vbytes * L.n + 16));
  AMG_TRY(dev_alloc(h, &L.y, vbytes * L.n + 16));
  return AMG_OK;
}

}  // namespace

// ---- LDS-staged gathers: tile lists (setup) ----

constexpr int kHaloCap = 8192;        // padded entries of one tile sorted in LDS
constexpr int kHaloThreads = 1024;
constexpr int32_t kHaloMaxList = 4096;  // longest list a level may have (LDS of a block)

__global__ void k_tile_starts(int32_t ntiles, int32_t step, int32_t nmax,
                              const int32_t *__restrict__ seg, int32_t *__restrict__ tb) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > ntiles) return;
  const int64_t v = (int64_t)t * step;
  const int32_t c = (int32_t)(v < nmax ? v : nmax);
  tb[t] = seg ? seg[c] : c;  // row chunks, or the first row of coarse row c
}

// Tile t = rows [tb[t], tb[t + 1]). Its list is the sorted distinct columns
// of its SELL positions (W per row, W the widest slice among its rows; at
// most kHaloCap positions, else count[t] = -1 and no list): the columns below
// the tile's own rows, then the own rows themselves (every row holds its
// diagonal), then the columns above. Only the columns outside the own rows
// are sorted (bitonic, in LDS) and made distinct; an own row's index in the
// list follows from its offset. Pass 0 writes the list length to count[t];
// pass 1 writes the list at hidx + hptr[t] and, at every position, the index
// of its column in the list.
__global__ void __launch_bounds__(kHaloThreads) k_halo(
    int32_t pass, const int32_t *__restrict__ tb, const int32_t *__restrict__ sptr,
    const int32_t *__restrict__ col, int32_t *__restrict__ count,
    const int32_t *__restrict__ hptr, int32_t *__restrict__ hidx, uint16_t *__restrict__ lcol) {
  __shared__ int32_t keys[kHaloCap];
  __shared__ int32_t part[kHaloThreads];
  __shared__ int32_t wmax, nout;
  const int32_t t = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int32_t r0 = tb[t], r1 = tb[t + 1], rows = r1 - r0;
  if (tid == 0) {
    wmax = 0;
    nout = 0;
  }
  __syncthreads();
  if (rows > 0) {
    int32_t wl = 0;
    for (int32_t q = r0 / kSlice + tid; q <= (r1 - 1) / kSlice; q += nt)
      wl = max(wl, (sptr[q + 1] - sptr[q]) / kSlice);
    atomicMax(&wmax, wl);
  }
  __syncthreads();
  const int32_t W = wmax;
  const int64_t E = (int64_t)rows * W;
  if (E > kHaloCap) {
    if (pass == 0 && tid == 0) count[t] = -1;
    return;
  }
  // the columns outside [r0, r1), in any order
  for (int32_t i = tid; i < E; i += nt) {
    int32_t base, w;
    sell_row(sptr, r0 + i / W, &base, &w);
    if (i % W < w) {
      const int32_t c = col[base + (i % W) * kSlice];
      if (c < r0 || c >= r1) keys[atomicAdd(&nout, 1)] = c;
    }
  }
  __syncthreads();
  const int32_t no = nout;
  int32_t P = 1;
  while (P < no) P <<= 1;
  for (int32_t i = no + tid; i < P; i += nt) keys[i] = INT32_MAX;
  __syncthreads();
  for (int32_t size = 2; size <= P; size <<= 1)  // bitonic sort, ascending
    for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (int32_t i = tid; i < P; i += nt) {
        const int32_t j = i ^ stride;
        if (j > i) {
          const int32_t a = keys[i], b = keys[j];
          if ((a > b) == ((i & size) == 0)) {
            keys[i] = b;
            keys[j] = a;
          }
        }
      }
      __syncthreads();
    }
  // distinct keys: thread tid takes positions [tid * per, tid * per + per)
  const int32_t per = (P + nt - 1) / nt;  // at most kHaloCap / kHaloThreads = 8
  int32_t kv[kHaloCap / kHaloThreads];
  uint32_t first = 0;
  int32_t mine = 0;
  for (int32_t q = 0; q < per; ++q) {
    const int32_t i = tid * per + q;
    kv[q] = i < P ? keys[i] : INT32_MAX;
    if (i < P && kv[q] != INT32_MAX && (i == 0 || keys[i - 1] != kv[q])) {
      first |= 1u << q;
      ++mine;
    }
  }
  part[tid] = mine;
  __syncthreads();
  for (int32_t off = 1; off < nt; off <<= 1) {  // inclusive scan of the counts
    const int32_t add = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += add;
    __syncthreads();
  }
  const int32_t uo = part[nt - 1];
  int32_t pos = part[tid] - mine;
  for (int32_t q = 0; q < per; ++q)  // every key was read before the scan
    if (first & (1u << q)) keys[pos++] = kv[q];
  __syncthreads();
  if (pass == 0) {
    if (tid == 0) count[t] = uo + rows;
    return;
  }
  // nb = distinct outside columns below r0 (they precede the own rows)
  int32_t lo = 0, hi = uo;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (keys[mid] < r0) lo = mid + 1;
    else hi = mid;
  }
  const int32_t nb = lo;
  const int32_t h0 = hptr[t];
  for (int32_t j = tid; j < uo + rows; j += nt)
    hidx[h0 + j] = j < nb ? keys[j] : (j < nb + rows ? r0 + (j - nb) : keys[j - rows]);
  for (int64_t i = tid; i < E; i += nt) {
    int32_t base, w;
    sell_row(sptr, r0 + (int32_t)(i / W), &base, &w);
    const int32_t k = (int32_t)(i % W);
    if (k >= w) continue;
    const int32_t idx = base + k * kSlice;
    const int32_t c = col[idx];
    int32_t at;
    if (c >= r0 && c < r1) {
      at = nb + (c - r0);
    } else {
      int32_t a = 0, b = uo - 1;  // c is in the list
      while (a < b) {
        const int32_t mid = (a + b) >> 1;
        if (keys[mid] < c) a = mid + 1;
        else b = mid;
      }
      at = a < nb ? a : a + rows;
    }
    lcol[idx] = (uint16_t)at;
  }
}

// Tile lists of level L for `ntiles` tiles starting at tb (device, ntiles + 1
// entries). Leaves H empty (the kernels then gather from memory) when a tile
// has too many entries to sort in LDS or too long a list for a block's LDS.
amg_status build_halo(amg_hierarchy *h, const Level &L, const int32_t *tb, int32_t ntiles,
                      int32_t param, Halo *H) {
  hipStream_t s = h->stream;
  int32_t *count;
  AMG_TRY(setup_tmp_alloc(h, reinterpret_cast<void **>(&count), sizeof(int32_t) * (ntiles + 1)));
  k_halo<<<ntiles, kHaloThreads, 0, s>>>(0, tb, L.S.sptr, L.S.col, count, nullptr, nullptr,
                                        nullptr);
  std::vector<int32_t> hc(ntiles);
  AMG_HIP(hipMemcpyAsync(hc.data(), count, sizeof(int32_t) * ntiles, hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  int64_t total = 0;
  int32_t umax = 0;
  bool fits = true;
  for (int32_t c : hc) {
    fits = fits && c >= 0;
    umax = std::max(umax, c);
    total += c > 0 ? c : 0;
  }
  if (!fits || umax > kHaloMaxList || total > INT32_MAX) {
    setup_tmp_free(h, count);
    return AMG_OK;
  }
  Halo G;
  G.ntiles = ntiles;
  G.param = param;
  G.umax = umax;
  amg_status st = dalloc(h, &G.hptr, (size_t)ntiles + 1);
  if (st == AMG_OK) st = setup_scan(h, count, G.hptr, ntiles);
  if (st == AMG_OK) st = dalloc(h, &G.hidx, (size_t)(total > 0 ? total : 1));
  if (st == AMG_OK) st = dalloc(h, &G.lcol, (size_t)L.S.nnz_padded);
  if (st == AMG_OK)
    k_halo<<<ntiles, kHaloThreads, 0, s>>>(1, tb, L.S.sptr, L.S.col, nullptr, G.hptr, G.hidx,
                                          G.lcol);
  setup_tmp_free(h, count);
  AMG_TRY(st);
  AMG_HIP(hipGetLastError());
  *H = G;
  return AMG_OK;
}

// Level 0's tiles: the row chunks of the streaming kernels and the blocks of
// the down step (coarse rows by coarse_per_block, fine rows by segment).
amg_status build_level0_halos(amg_hierarchy *h) {
  hipStream_t s = h->stream;
  Level &F = h->lv[0];
  // none on levels of kManyRows rows or more: there the kernels take one row
  // per thread (256-row tiles), and staging lost to the gathers from memory
  // (256^3 anisotropic blocks: 144.2 -> 138.6 ms per FP64 solve without tiles)
  if (F.n >= kManyRows) return AMG_OK;
  const Level &C = h->lv[1];
  int32_t *tb;
  const Geom g = geom(F.n);
  const int32_t G = staged_down_G(h);
  const int32_t nseg = ceil_div(C.n, G);
  const int32_t most = std::max(g.grid, nseg);
  AMG_TRY(setup_tmp_alloc(h, reinterpret_cast<void **>(&tb), sizeof(int32_t) * (most + 1)));
  k_tile_starts<<<ceil_div(g.grid + 1, kBlock), kBlock, 0, s>>>(g.grid, g.chunk, F.n, nullptr,
                                                                tb);
  amg_status st = build_halo(h, F, tb, g.grid, g.chunk, &F.hrow);
  if (st == AMG_OK) {
    k_tile_starts<<<ceil_div(nseg + 1, kBlock), kBlock, 0, s>>>(nseg, G, C.n, F.seg, tb);
    st = build_halo(h, F, tb, nseg, G, &F.hseg);
  }
  setup_tmp_free(h, tb);
  return st;
}

// average row length from which a level of a smoothed hierarchy is smoothed
// with several lanes per row
constexpr double kLongRow = 48.0;

amg_status build_solve_formats(amg_hierarchy *h) {
  hipStream_t s = h->stream;
  const bool fp32 = h->params.precision == AMG_FP32;
  const size_t vbytes = fp32 ? sizeof(float) : sizeof(double);
  const int32_t nlev = (int32_t)h->lv.size();
  // aggregate-major order, from the coarsest level down
  {
    Level &C = h->lv[nlev - 1];
    AMG_TRY(dalloc(h, &C.perm, (size_t)C.n));
    AMG_TRY(dalloc(h, &C.iperm, (size_t)C.n));
    k_iota_i32<<<grid1(C.n), kBlock, 0, s>>>(C.perm, C.n);
    k_iota_i32<<<grid1(C.n), kBlock, 0, s>>>(C.iperm, C.n);
  }
  h->max_seg = 1;
  for (int32_t l = nlev - 2; l >= 0; --l) {
    Level &F = h->lv[l];
    Level &C = h->lv[l + 1];
    int32_t *cnt;
    AMG_TRY(setup_tmp_alloc(h, reinterpret_cast<void **>(&cnt), sizeof(int32_t) * C.n + 16));
    AMG_TRY(dalloc(h, &F.seg, (size_t)C.n + 1));
    k_seg_count<<<grid1(C.n), kBlock, 0, s>>>(C.n, C.perm, F.mptr, cnt);
    AMG_TRY(setup_scan(h, cnt, F.seg, C.n));
    setup_tmp_free(h, cnt);
    AMG_TRY(dalloc(h, &F.perm, (size_t)F.n));
    AMG_TRY(dalloc(h, &F.iperm, (size_t)F.n));
    AMG_TRY(dalloc(h, &F.aggp, (size_t)F.n));
    AMG_TRY(dalloc(h, &F.pp64, (size_t)F.n));
    k_order_fill<<<grid1(C.n), kBlock, 0, s>>>(C.n, C.perm, F.mptr, F.mem, F.seg, F.p64, F.perm,
                                              F.iperm, F.aggp, F.pp64);
    h->max_seg = std::max(h->max_seg, 1 << F.sweeps);
  }
  for (int32_t l = 0; l < nlev; ++l) {
    Level &L = h->lv[l];
    const bool coarsest = (l == nlev - 1);
    // level 0 needs FP64 values for the outer CG; V-cycle levels need the
    // hierarchy precision (plain and scaled); the coarsest uses A_L^-1 only
    const bool need64 = (l == 0) || (!coarsest && !fp32);
    bool need32 = !coarsest && fp32;
    if (l == 0) {
      // every value of A an FP32 number: the FP64 products of level 0 read
      // the exact FP32 copy (identical arithmetic, half the value bytes)
      // unless AMG_FLAG_NO_VALUE_COMPRESSION switches it off
      int32_t *flag;
      AMG_TRY(setup_tmp_alloc(h, reinterpret_cast<void **>(&flag), sizeof(int32_t)));
      AMG_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
      k_not_fp32_exact<<<grid1(L.nnz), kBlock, 0, s>>>(L.nnz, L.val, flag);
      int32_t hflag = 1;
      AMG_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      AMG_HIP(hipStreamSynchronize(s));
      setup_tmp_free(h, flag);
      L.S.fp32_values = hflag == 0;
      L.S.exact32 = L.S.fp32_values && !(h->params.flags & AMG_FLAG_NO_VALUE_COMPRESSION);
      need32 = need32 || L.S.exact32;
    }
    if (need64 || need32) {
      Sell &S = L.S;
      S.n = L.n;
      S.nslices = ceil_div(L.n, kSlice);
      int32_t *w64;
      AMG_TRY(setup_tmp_alloc(h, reinterpret_cast<void **>(&w64), sizeof(int32_t) * S.nslices + 16));
      unsigned long long *total;
      AMG_TRY(setup_tmp_alloc(h, reinterpret_cast<void **>(&total), sizeof(unsigned long long)));
      AMG_HIP(hipMemsetAsync(total, 0, sizeof(unsigned long long), s));
      AMG_TRY(dalloc(h, &S.sptr, (size_t)S.nslices + 1));
      k_sell_width<<<grid1(S.nslices), kBlock, 0, s>>>(L.n, S.nslices, L.rp, L.perm, w64, total);
      unsigned long long htotal = 0;
      AMG_HIP(hipMemcpyAsync(&htotal, total, sizeof(htotal), hipMemcpyDeviceToHost, s));
      AMG_HIP(hipStreamSynchronize(s));
      setup_tmp_free(h, total);
      if (htotal > (unsigned long long)INT32_MAX) {
        setup_tmp_free(h, w64);
        return AMG_ERR_ARG;  // padded rows exceed the format's 32-bit offsets
      }
      AMG_TRY(setup_scan(h, w64, S.sptr, S.nslices));
      setup_tmp_free(h, w64);
      int32_t padded = 0;
      AMG_HIP(hipMemcpyAsync(&padded, S.sptr + S.nslices, sizeof(int32_t),
                             hipMemcpyDeviceToHost, s));
      AMG_HIP(hipStreamSynchronize(s));
      S.nnz_padded = padded;
      if (L.n <= 1024) {  // small levels: the widest slice, for register-held rows
        std::vector<int32_t> sp(S.nslices + 1);
        AMG_HIP(hipMemcpyAsync(sp.data(), S.sptr, sizeof(int32_t) * (S.nslices + 1),
                               hipMemcpyDeviceToHost, s));
        AMG_HIP(hipStreamSynchronize(s));
        for (int32_t q = 0; q < S.nslices; ++q)
          S.max_width = std::max(S.max_width, (sp[q + 1] - sp[q]) / kSlice);
      }
      AMG_TRY(dalloc(h, &S.col, (size_t)padded));
      if (need64) AMG_TRY(dalloc(h, &S.v64, (size_t)padded));
      if (need32) AMG_TRY(dalloc(h, &S.v32, (size_t)padded));
      if (!coarsest && !fp32) AMG_TRY(dalloc(h, &S.s64, (size_t)padded));
      if (!coarsest && fp32) AMG_TRY(dalloc(h, &S.s32, (size_t)padded));
      k_sell_fill<<<ceil_div((int64_t)S.nslices * kSlice, kBlock), kBlock, 0, s>>>(
          L.n, S.nslices, L.rp, L.ci, L.val, L.perm, L.iperm, L.minv64, S.sptr, S.col, S.v64,
          S.v32, S.s64, S.s32);
    }
    if (!coarsest) {
      AMG_TRY(dalloc(h, &L.sminv64, (size_t)L.n));
      k_gather_f64<<<grid1(L.n), kBlock, 0, s>>>(L.n, L.perm, L.minv64, L.sminv64);
      if (fp32) {
        AMG_TRY(dalloc(h, &L.sminv32, (size_t)L.n));
        AMG_TRY(dalloc(h, &L.pp32, (size_t)L.n));
        k_demote<<<grid1(L.n), kBlock, 0, s>>>(L.n, L.sminv64, L.sminv32);
        k_demote<<<grid1(L.n), kBlock, 0, s>>>(L.n, L.pp64, L.pp32);
      }
    }
    AMG_TRY(alloc_level_vectors(h, L, vbytes));
    // K-cycle flexible-CG vectors on the levels strictly between the finest
    // and the coarsest
    if (h->params.cycle == AMG_CYCLE_K && l > 0 && l + 1 < nlev) {
      AMG_TRY(dev_alloc(h, &L.c1, vbytes * L.n + 16));
      AMG_TRY(dev_alloc(h, &L.v1, vbytes * L.n + 16));
      AMG_TRY(dev_alloc(h, &L.r1, vbytes * L.n + 16));
      AMG_TRY(dev_alloc(h, &L.c2, vbytes * L.n + 16));
      AMG_TRY(dev_alloc(h, &L.v2, vbytes * L.n + 16));
    }
  }
  // LDS-staged gathers of level 0's products (where every tile's list fits)
  if (nlev > 1) AMG_TRY(build_level0_halos(h));
  if (h->params.cycle == AMG_CYCLE_K) AMG_TRY(dalloc(h, &h->kscal, (size_t)kKScal * nlev));
  if (h->params.smooth_p)
    for (int32_t l = 0; l + 1 < nlev; ++l) {
      AMG_TRY(smooth_solve_format(h, l, fp32));
      // the denser coarse levels: CSR for the kernels with several lanes per row
      if (l > 0 && (double)h->lv[l].nnz > kLongRow * (double)h->lv[l].n)
        AMG_TRY(long_row_csr(h, l, fp32));
    }
  // outer CG vectors and scalars (aggregate-major order of level 0)
  const int32_t n0 = h->lv[0].n;
  AMG_TRY(dalloc(h, &h->x, (size_t)n0));
  AMG_TRY(dalloc(h, &h->b, (size_t)n0));
  AMG_TRY(dalloc(h, &h->r, (size_t)n0));
  AMG_TRY(dalloc(h, &h->z, (size_t)n0));
  AMG_TRY(dalloc(h, &h->p, (size_t)n0));
  AMG_TRY(dalloc(h, &h->q, (size_t)n0));
  AMG_TRY(dalloc(h, &h->partials, (size_t)kMaxParts * kPartPlanes));
  AMG_TRY(dalloc(h, &h->scal, 1));
  AMG_TRY(dalloc(h, &h->zero_flag, 4));
  AMG_HIP(hipMemsetAsync(h->zero_flag, 0, sizeof(int32_t) * 4, s));
  AMG_HIP(hipMemsetAsync(h->scal, 0, sizeof(PcgScal), s));
  if (!h->scal_host) AMG_HIP(hipHostMalloc(reinterpret_cast<void **>(&h->scal_host), sizeof(PcgScal)));
  return AMG_OK;
}

// Applies the V-cycle to vectors in the aggregate-major order of level 0.
// The K-cycle with an optional dot partner (see kcycle_top)
amg_status kcycle_perm(amg_hierarchy *h, const double *r, double *z, const double *dv,
                       const int32_t *done) {
  if (h->params.precision == AMG_FP32) kcycle_top<float>(h, r, z, dv, done);
  else kcycle_top<double>(h, r, z, dv, done);
  AMG_HIP(hipGetLastError());
  return AMG_OK;
}

amg_status vcycle_perm(amg_hierarchy *h, const double *r, double *z, bool fuse_dot,
                       const int32_t *done) {
  if (h->params.cycle == AMG_CYCLE_K) return kcycle_perm(h, r, z, nullptr, done);
  if (h->params.precision == AMG_FP32) vcycle_t<float>(h, r, z, fuse_dot, nullptr, done);
  else vcycle_t<double>(h, r, z, fuse_dot, nullptr, done);
  AMG_HIP(hipGetLastError());
  return AMG_OK;
}

// The preconditioner of flexible CG (K-cycle, or a cycle with the iterative
// coarsest solve): z = B r with the block partials of (dv, z) when dv is
// given, left for the caller's finalize.
amg_status precond_perm(amg_hierarchy *h, const double *r, double *z, const double *dv,
                        const int32_t *done) {
  if (h->params.cycle == AMG_CYCLE_K) return kcycle_perm(h, r, z, dv, done);
  if (h->params.precision == AMG_FP32) vcycle_t<float>(h, r, z, dv != nullptr, dv, done);
  else vcycle_t<double>(h, r, z, dv != nullptr, dv, done);
  AMG_HIP(hipGetLastError());
  return AMG_OK;
}

// flexible CG is the outer solver when the preconditioner is not a fixed
// linear operator
inline bool flexible(const amg_hierarchy *h) {
  return h->params.cycle == AMG_CYCLE_K || h->params.coarse_solver == AMG_COARSE_PCG;
}

// z = B r on vectors in the caller's numbering
amg_status vcycle(amg_hierarchy *h, const double *r, double *z, bool fuse_dot,
                  const int32_t *done) {
  hipStream_t s = h->stream;
  const int32_t n = h->lv[0].n;
  k_permute_in<<<grid1(n), kBlock, 0, s>>>(n, h->lv[0].perm, r, h->r);
  AMG_TRY(vcycle_perm(h, h->r, h->z, fuse_dot, done));
  k_permute_out<<<grid1(n), kBlock, 0, s>>>(n, h->lv[0].perm, h->z, z);
  AMG_HIP(hipGetLastError());
  return AMG_OK;
}

namespace {

// p = z + beta p (copy: p = z) on the CG vectors of level 0
void launch_xpay(amg_hierarchy *h, int32_t n, int32_t copy, const int32_t *done) {
  const bool pairs = reinterpret_cast<uintptr_t>(h->z) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(h->p) % 16 == 0;
  if (pairs)
    k_xpay<2><<<grid1((n + 1) / 2), kBlock, 0, h->stream>>>(n, h->z, h->p, h->scal, copy, done);
  else
    k_xpay<1><<<grid1(n), kBlock, 0, h->stream>>>(n, h->z, h->p, h->scal, copy, done);
}

// One CG iteration: q = A p, alpha, x and r updates with the stop test,
// z = B r with (r, z) and beta, p = z + beta p. Touches only hierarchy
// buffers, so it is captured once and replayed.
// One flexible-CG iteration (K-cycle, or the iterative coarsest solve):
// q = A p with (p, q), (p, r), alpha = (p, r) / (p, q), the x and r updates
// with the stop test, z = B r with (q, z), beta = -(z, q) / (p, q),
// p = z + beta p.
void fcg_iteration(amg_hierarchy *h) {
  hipStream_t s = h->stream;
  Level &L0 = h->lv[0];
  const int32_t n = L0.n;
  const int32_t *done = &h->scal->done;
  const Geom g = geom(n);
  if (L0.S.exact32)
    k_spmv_dots<double, 2, float><<<g.grid, kBlock, 0, s>>>(n, g.chunk, L0.S.sptr, L0.S.col,
                                                            L0.S.v32, h->p, h->q, h->r, nullptr,
                                                            h->partials, done);
  else
    k_spmv_dots<double, 2><<<g.grid, kBlock, 0, s>>>(n, g.chunk, L0.S.sptr, L0.S.col, L0.S.v64,
                                                     h->p, h->q, h->r, nullptr, h->partials,
                                                     done);
  finalize(h, kFinPQR, g.grid, done);
  k_update_xr<<<g.grid, kBlock, 0, s>>>(n, g.chunk, h->x, h->r, h->p, h->q, h->partials, h->scal,
                                        done);
  finalize(h, kFinRR, g.grid, done);
  precond_perm(h, h->r, h->z, h->q, done);
  finalize(h, kFinZQ, g.grid, done);
  launch_xpay(h, n, 0, done);
}

void cg_iteration(amg_hierarchy *h) {
  if (flexible(h)) {
    fcg_iteration(h);
    return;
  }
  hipStream_t s = h->stream;
  Level &L0 = h->lv[0];
  const int32_t n = L0.n;
  const int32_t *done = &h->scal->done;
  const Geom g = geom(n);
  arm_probe(h, 4);
  spmv_dot0(h, h->p, h->q, done);
  h->probe_armed = false;
  finalize(h, kFinPQ, g.grid, done);
  k_update_xr<<<g.grid, kBlock, 0, s>>>(n, g.chunk, h->x, h->r, h->p, h->q, h->partials, h->scal,
                                        done);
  finalize(h, kFinRR, g.grid, done);
  vcycle_perm(h, h->r, h->z, true, done);
  launch_xpay(h, n, 0, done);
}

// Captures `count` CG iterations into one instantiated hipGraph.
bool capture_iterations(amg_hierarchy *h, int32_t count, hipGraph_t *graph, hipGraphExec_t *exec) {
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  for (int32_t k = 0; k < count; ++k) cg_iteration(h);
  hipError_t e = hipStreamEndCapture(h->stream, &g);
  if (e != hipSuccess || !g) {
    (void)hipGetLastError();
    return false;
  }
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    (void)hipGraphDestroy(g);
    return false;
  }
  *graph = g;
  *exec = ex;
  return true;
}

// Graphs of one and of kIterGroup CG iterations (once per hierarchy): a
// group replay saves the launch gap between consecutive graphs.
constexpr int32_t kIterGroup = 4;
amg_status ensure_iteration_graph(amg_hierarchy *h) {
  if (h->iter_exec || h->graph_failed || (h->params.flags & AMG_FLAG_NO_GRAPH)) return AMG_OK;
  if (!capture_iterations(h, 1, &h->iter_graph, &h->iter_exec)) {
    h->graph_failed = true;
    return AMG_OK;
  }
  if (!capture_iterations(h, kIterGroup, &h->iter_graph4, &h->iter_exec4)) {
    h->iter_graph4 = nullptr;
    h->iter_exec4 = nullptr;
  }
  return AMG_OK;
}

}  // namespace

amg_status pcg(amg_hierarchy *h, const double *b_user, double *x_user, double rtol,
               int32_t maxit, amg_solve_info *info, bool use_graph) {
  const double t0 = now_ms();
  hipStream_t s = h->stream;
  Level &L0 = h->lv[0];
  const int32_t n = L0.n;
  const int32_t *done = &h->scal->done;
  const Geom g = geom(n);
  if (use_graph) AMG_TRY(ensure_iteration_graph(h));
  // the graphs hold the hierarchy's own scratch buffers: launched only when
  // the solve uses them
  hipGraphExec_t exec1 = use_graph ? h->iter_exec : nullptr;
  hipGraphExec_t exec4 = use_graph ? h->iter_exec4 : nullptr;
  k_permute_in<<<grid1(n), kBlock, 0, s>>>(n, L0.perm, b_user, h->b);
  h->has_rhs = true;
  k_permute_in<<<grid1(n), kBlock, 0, s>>>(n, L0.perm, x_user, h->x);
  k_scal_init<<<1, 1, 0, s>>>(h->scal, rtol, maxit);
  if (L0.S.exact32)
    k_residual_norms<0, float><<<g.grid, kBlock, 0, s>>>(n, g.chunk, L0.S.sptr, L0.S.col,
                                                         L0.S.v32, h->b, h->x, h->r, h->partials);
  else
    k_residual_norms<0, double><<<g.grid, kBlock, 0, s>>>(n, g.chunk, L0.S.sptr, L0.S.col,
                                                          L0.S.v64, h->b, h->x, h->r,
                                                          h->partials);
  finalize(h, kFinInit, g.grid, nullptr);
  k_zero_if_zero_rhs<<<grid1(n), kBlock, 0, s>>>(n, h->x, h->scal);
  if (flexible(h)) AMG_TRY(precond_perm(h, h->r, h->z, nullptr, done));
  else AMG_TRY(vcycle_perm(h, h->r, h->z, true, done));
  launch_xpay(h, n, 1, done);
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
    int32_t k = 0;
    if (exec4)
      for (; k + kIterGroup <= c; k += kIterGroup) AMG_HIP(hipGraphLaunch(exec4, s));
    for (; k < c; ++k) {
      if (exec1) AMG_HIP(hipGraphLaunch(exec1, s));
      else cg_iteration(h);
    }
    AMG_HIP(hipGetLastError());
    queued += c;
  }
  if (L0.S.exact32)
    k_residual_norms<1, float><<<g.grid, kBlock, 0, s>>>(n, g.chunk, L0.S.sptr, L0.S.col,
                                                         L0.S.v32, h->b, h->x, nullptr,
                                                         h->partials);
  else
    k_residual_norms<1, double><<<g.grid, kBlock, 0, s>>>(n, g.chunk, L0.S.sptr, L0.S.col,
                                                          L0.S.v64, h->b, h->x, nullptr,
                                                          h->partials);
  finalize(h, kFinTrue, g.grid, nullptr);
  k_permute_out<<<grid1(n), kBlock, 0, s>>>(n, L0.perm, h->x, x_user);
  AMG_HIP(hipMemcpyAsync(h->scal_host, h->scal, sizeof(PcgScal), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  const PcgScal sc = *h->scal_host;
  amg_status st = AMG_OK;
  if (sc.done == 2) st = AMG_NOT_CONVERGED;
  if (sc.done == 3) st = AMG_ERR_BREAKDOWN;
  if (info) {
    info->iterations = sc.iter;
    info->converged = (sc.done == 1 || sc.done == 4) ? 1 : 0;
    info->rel_res_recursive = sc.bb > 0.0 ? std::sqrt(sc.rr / sc.bb) : 0.0;
    info->rel_res_true = sc.bb > 0.0 ? std::sqrt(sc.rr_true / sc.bb) : 0.0;
    info->ms = now_ms() - t0;
  }
  return st;
}

namespace {

// One V-cycle exactly as the solve runs it (aggregate-major vectors, no
// permutation, no host work between launches), timed with HIP events; bytes
// = the cycle's algorithmic HBM bytes (0 for a K-cycle hierarchy, whose
// traffic depends on the level visits).
amg_status time_vcycle(amg_hierarchy *h, int32_t reps, double *ms, double *bytes) {
  if (reps < 1 || h->params.cycle != AMG_CYCLE_V) return AMG_ERR_ARG;
  hipStream_t s = h->stream;
  const int32_t *done = h->zero_flag;
  AMG_TRY(vcycle_perm(h, h->r, h->z, false, done));  // warm
  hipEvent_t e0, e1;
  AMG_HIP(hipEventCreate(&e0));
  AMG_HIP(hipEventCreate(&e1));
  AMG_HIP(hipEventRecord(e0, s));
  for (int32_t k = 0; k < reps; ++k) AMG_TRY(vcycle_perm(h, h->r, h->z, false, done));
  AMG_HIP(hipEventRecord(e1, s));
  AMG_HIP(hipEventSynchronize(e1));
  float t = 0.f;
  AMG_HIP(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = (double)t / reps;
  // per level l < L: down step z(V+4) + 4(n+1) + n(Vr+3V) + n_c(V+4) and the
  // prolongation into it n(3V+4); per coarse level 0 < c < L its
  // post-smoothing z(V+4) + 4(n+1) + 3V n; the coarsest 8 n_L^2 + V n_L; the
  // level-0 post-smoothing z(V+4) + 4(n+1) + n(16+2V); the iterative
  // coarsest solve is not counted (its traffic stays in L2)
  const int32_t L = (int32_t)h->lv.size() - 1;
  const double V = h->params.precision == AMG_FP32 ? 4.0 : 8.0;
  const double nL = h->C.n;
  if (h->params.smooth_p && L > 0) {
    // smoothed prolongators, per level l < L: down step z(V+4) + 4(n+1) +
    // n(Vr+3V); restriction by Pbar^T p(V+4) + 4(n_c+1) + V(n + n_c);
    // prolongation by Pbar p(V+4) + 4(n+1) + V(n_c + 2n); post-smoothing of
    // 0 < l < L z(V+4) + 4(n+1) + 4Vn; the coarsest (Cholesky) 8 n_L^2 +
    // 2V n_L; the level-0 post-smoothing as above
    double b = coarse_is_pcg(h) ? 0.0 : 8.0 * nL * nL + 2.0 * V * nL;
    for (int32_t l = 0; l < L; ++l) {
      const Level &F = h->lv[l];
      const double n = F.n, z = (double)F.nnz, nc = h->lv[l + 1].n, p = (double)F.pb_nnz;
      const double Vr = l == 0 ? 8.0 : V;
      b += z * (V + 4) + 4 * (n + 1) + n * (Vr + 3 * V);
      b += p * (V + 4) + 4 * (nc + 1) + V * (n + nc);
      b += p * (V + 4) + 4 * (n + 1) + V * (nc + 2 * n);
      if (l > 0) b += z * (V + 4) + 4 * (n + 1) + 4 * V * n;
    }
    const double n0 = h->lv[0].n, z0 = (double)h->lv[0].nnz;
    const double Va = V == 8.0 && h->lv[0].S.exact32 ? 4.0 : V;
    b += z0 * (Va + 4) + 4 * (n0 + 1) + n0 * (16 + 2 * V);
    *bytes = b;
    return AMG_OK;
  }
  double b = coarse_is_pcg(h) ? 0.0 : 8.0 * nL * nL + (L == 0 ? 16.0 : V) * nL;
  for (int32_t l = 0; l < L; ++l) {
    const double n = h->lv[l].n, z = (double)h->lv[l].nnz, nc = h->lv[l + 1].n;
    const double Vr = l == 0 ? 8.0 : V;
    // the down step reads A M^-1, or A's exact FP32 copy where it stages M^-1 r
    const double Vs =
        l == 0 && V == 8.0 && h->lv[0].S.exact32 && staged_down<double>(h, h->lv[0], h->lv[1])
            ? 4.0 : V;
    b += z * (Vs + 4) + 4 * (n + 1) + n * (Vr + 3 * V) + nc * (V + 4) + n * (3 * V + 4);
    if (l > 0) b += z * (V + 4) + 4 * (n + 1) + 3 * V * n;
  }
  if (L > 0) {
    const double n0 = h->lv[0].n, z0 = (double)h->lv[0].nnz;
    const double Va = V == 8.0 && h->lv[0].S.exact32 ? 4.0 : V;  // level-0 A as stored
    b += z0 * (Va + 4) + 4 * (n0 + 1) + n0 * (16 + 2 * V);
  }
  *bytes = b;
  return AMG_OK;
}

// algorithmic HBM bytes of one launch of kernel 0-4 on `level`: CSR values +
// int32 columns + int32 row offsets once per SpMV, every vector entry once
double kernel_bytes(const amg_hierarchy *h, int32_t kernel, int32_t level) {
  const Level &F = h->lv[level];
  const Level &C = h->lv[level + 1];
  const bool fp32 = h->params.precision == AMG_FP32;
  const double V = fp32 ? 4.0 : 8.0;
  const double n = F.n, nnz = (double)F.nnz, nc = C.n, nnzc = (double)C.nnz;
  const double Vr = level == 0 ? 8.0 : V;  // level 0 reads/writes the FP64 CG vectors
  switch (kernel) {
    case 0:  // A M^-1 (or A from its exact FP32 copy), r, minv, p read; z, r_c
             // written; segment offsets
      return nnz * ((level == 0 && V == 8.0 && staged_down<double>(h, F, C) && F.S.exact32
                         ? 4.0 : V) + 4) +
             4 * (n + 1) + n * (Vr + 3 * V) + nc * (V + 4);
    case 1:  // A, r, z, minv read; y written (level 0: A from its exact FP32 copy if any)
      return nnz * ((level == 0 && F.S.exact32 ? 4.0 : V) + 4) + 4 * (n + 1) +
             n * (Vr + V + V + Vr);
    case 2:
    case 3:  // coarse A, r_c, z_c, minv_c; fine z read + written, p, positions
      return nnzc * (V + 4) + 4 * (nc + 1) + nc * (3 * V + 4) + n * (3 * V + 4);
    default:  // A (8 or, from the exact FP32 copy, 4 bytes per value), p read; q written
      return nnz * ((F.S.exact32 ? 4.0 : 8.0) + 4) + 4 * (n + 1) + n * 16;
  }
}


// One of the level-0 kernels 0 (down step), 1 (post-smoothing with the CG
// dot) or 4 (outer SpMV with its dot) timed where the solve runs it: `reps`
// CG iterations from x = 0 on the last right-hand side, launched directly
// (the graph cannot hold the events), rtol 0 and maxit reps + 1 so that no
// kernel takes its early exit; the kernel's own dispatch start and end,
// stamped into events by hipExtLaunchKernelGGL, give its mean duration with
// the caches as the iteration leaves them. Hierarchies with one pre- and one
// post-sweep only (otherwise these steps are several kernels).
amg_status time_in_solve(amg_hierarchy *h, int32_t kernel, int32_t reps, double *ms,
                         double *bytes) {
  if (kernel != 0 && kernel != 1 && kernel != 4) return AMG_ERR_ARG;
  if (reps < 1 || reps > 10000 || flexible(h) || h->params.smooth_p || h->lv.size() < 2 ||
      h->params.pre != 1 || h->params.post != 1 || !h->has_rhs)
    return AMG_ERR_ARG;
  hipStream_t s = h->stream;
  Level &L0 = h->lv[0];
  const int32_t n = L0.n;
  const int32_t *done = &h->scal->done;
  const Geom g = geom(n);
  AMG_HIP(hipMemsetAsync(h->x, 0, sizeof(double) * n, s));
  k_scal_init<<<1, 1, 0, s>>>(h->scal, 0.0, reps + 1);
  if (L0.S.exact32)
    k_residual_norms<0, float><<<g.grid, kBlock, 0, s>>>(n, g.chunk, L0.S.sptr, L0.S.col,
                                                         L0.S.v32, h->b, h->x, h->r, h->partials);
  else
    k_residual_norms<0, double><<<g.grid, kBlock, 0, s>>>(n, g.chunk, L0.S.sptr, L0.S.col,
                                                          L0.S.v64, h->b, h->x, h->r,
                                                          h->partials);
  finalize(h, kFinInit, g.grid, nullptr);
  AMG_TRY(vcycle_perm(h, h->r, h->z, true, done));
  launch_xpay(h, n, 1, done);
  h->probe_ev.assign(2 * (size_t)reps, nullptr);
  amg_status st = AMG_OK;
  // timing-only events: no system-scope release at the timed dispatch's end
  // (that writeback of L2 is not part of the kernel inside the solve)
  for (auto &e : h->probe_ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) st = AMG_ERR_HIP;
  if (st == AMG_OK) {
    h->probe_next = 0;
    h->probe_id = kernel;
    for (int32_t k = 0; k < reps; ++k) cg_iteration(h);
    h->probe_id = -1;
    if (hipGetLastError() != hipSuccess || h->probe_next != h->probe_ev.size() ||
        hipStreamSynchronize(s) != hipSuccess || hipEventSynchronize(h->probe_ev.back()) != hipSuccess)
      st = AMG_ERR_HIP;
  }
  double total = 0.0;
  for (size_t k = 0; st == AMG_OK && k + 1 < h->probe_ev.size(); k += 2) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, h->probe_ev[k], h->probe_ev[k + 1]) != hipSuccess)
      st = AMG_ERR_HIP;
    total += t;
  }
  for (auto e : h->probe_ev)
    if (e) (void)hipEventDestroy(e);
  h->probe_ev.clear();
  (void)hipGetLastError();
  if (st != AMG_OK) return st;
  *ms = total / reps;
  *bytes = kernel_bytes(h, kernel, 0);
  return AMG_OK;
}

}  // namespace

amg_status time_kernel(amg_hierarchy *h, int32_t kernel, int32_t level, int32_t reps,
                       double *ms, double *bytes) {
  const int32_t L = (int32_t)h->lv.size() - 1;
  if (kernel & AMG_TIME_IN_SOLVE) {
    if (level != 0) return AMG_ERR_ARG;
    return time_in_solve(h, kernel & ~AMG_TIME_IN_SOLVE, reps, ms, bytes);
  }
  if (kernel == 5) return time_vcycle(h, reps, ms, bytes);
  if (level < 0 || level >= L || reps < 1 || kernel < 0 || kernel > 4) return AMG_ERR_ARG;
  if (kernel == 4 && level != 0) return AMG_ERR_ARG;
  // the fused down and up kernels are those of the tentative prolongator
  if (h->params.smooth_p && (kernel == 0 || kernel == 2 || kernel == 3)) return AMG_ERR_ARG;
  if ((kernel == 2 || kernel == 3) && level + 1 >= L) return AMG_ERR_ARG;
  hipStream_t s = h->stream;
  Level &F = h->lv[level];
  Level &C = h->lv[level + 1];
  const bool fp32 = h->params.precision == AMG_FP32;
  const double V = fp32 ? 4.0 : 8.0;
  const double n = F.n, nnz = (double)F.nnz, nc = C.n, nnzc = (double)C.nnz;
  const double Vr = level == 0 ? 8.0 : V;  // level 0 reads/writes the FP64 CG vectors
  const int32_t *done = h->zero_flag;
  auto launch = [&]() {
    const Geom g = geom(F.n);
    switch (kernel) {
      case 0:  // pre-smoothing + residual + restriction on `level`
        if (fp32) {
          if (level == 0)
            pre_restrict<float, double, kPreScaled, float>(h, F, C, F.S.s32, F.sminv32, F.pp32,
                                                           h->r, (float *)F.z, (float *)C.r,
                                                           done);
          else
            pre_restrict<float, float, kPreScaled, float>(h, F, C, F.S.s32, F.sminv32, F.pp32,
                                                          (const float *)F.r, (float *)F.z,
                                                          (float *)C.r, done);
        } else {
          down_one_sweep<double, double>(h, F, C, level == 0 ? h->r : (const double *)F.r,
                                         (double *)F.z, done);
        }
        break;
      case 1:  // post-smoothing on `level` (level 0: with the CG dot product)
        if (fp32) {
          if (level == 0)
            post_sweep<float, double, double, true, float>(h, F, F.S.v32, F.sminv32, h->r,
                                                           (const float *)F.z, h->z,
                                                           h->partials, done);
          else
            post_sweep<float, float, float, false, float>(h, F, F.S.v32, F.sminv32,
                                                          (const float *)F.r, (const float *)F.z,
                                                          (float *)F.y, nullptr, done);
        } else {
          if (level == 0 && F.S.exact32)
            post_sweep<double, double, double, true, float>(h, F, F.S.v32, F.sminv64, h->r,
                                                            (const double *)F.z, h->z,
                                                            h->partials, done);
          else if (level == 0)
            post_sweep<double, double, double, true, double>(h, F, F.S.v64, F.sminv64, h->r,
                                                             (const double *)F.z, h->z,
                                                             h->partials, done);
          else
            post_sweep<double, double, double, false, double>(
                h, F, F.S.v64, F.sminv64, (const double *)F.r, (const double *)F.z,
                (double *)F.y, nullptr, done);
        }
        break;
      case 2:  // post-smoothing on level + 1 fused with prolongation into level
      case 3:
        if (fp32)
          k_post_prolong<float><<<grid1(C.n), kBlock, 0, s>>>(
              C.n, C.S.sptr, C.S.col, C.S.v32, C.sminv32, (const float *)C.r,
              (const float *)C.z, F.seg, F.aggp, F.pp32, (float *)F.t, done);
        else
          k_post_prolong<double><<<grid1(C.n), kBlock, 0, s>>>(
              C.n, C.S.sptr, C.S.col, C.S.v64, C.sminv64, (const double *)C.r,
              (const double *)C.z, F.seg, F.aggp, F.pp64, (double *)F.t, done);
        break;
      default:
        spmv_dot0(h, h->p, h->q, done);
        break;
    }
  };
  hipEvent_t e0, e1;
  AMG_HIP(hipEventCreate(&e0));
  AMG_HIP(hipEventCreate(&e1));
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
  *bytes = kernel_bytes(h, kernel, level);
  return AMG_OK;
}

}  // namespace amg
