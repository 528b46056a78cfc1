// Multi-right-hand-side PCG: k independent CG recurrences (one per column,
// each with its own alpha, beta and stop test, Section 5) share one V-cycle
// of eq. (amg) applied to the whole n x k block per iteration.
//
// Blocks are row-major (entry (i, j) at i k + j), so a row's k values are
// contiguous and one matrix entry is read once for all k columns: the matrix
// bytes of every SpMV are amortised over the block. A wavefront covers
// 64 / KT rows x KT columns; KT (the column tile, equivalently the rows per
// wavefront) is chosen per hierarchy and k by timing the level-0 smoother
// kernel over {4, 8, 16, 32, 64}. One iteration is captured in a hipGraph.
// Converged columns are frozen (x, r, p no longer updated); the iteration's
// kernels stop launching work once every column has stopped.

#include <chrono>
#include <cmath>
#include <cstdint>
#include <new>
#include <type_traits>

#include "internal.h"

namespace amg {

namespace {

constexpr int kBatchBlocks = 4096;  // x-blocks of a streaming batch kernel
enum ColField { cRho = 0, cPq, cAlpha, cBeta, cRr, cBb, cRtol, cRrTrue, kColFields };
enum BatchOp { bInit = 0, bPq, bRr, bRz0, bRz, bTrue };

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

__device__ __forceinline__ void sell_row(const int32_t *sptr, int32_t row, int32_t *base,
                                         int32_t *w) {
  const int32_t s = row / kSlice;
  *base = sptr[s] + (row % kSlice);
  *w = (sptr[s + 1] - sptr[s]) / kSlice;
}

// Row groups of kBlock / KT rows are dealt to the blocks in turn, in the
// XCD-aware block order (group g to logical block g mod gridDim.x). The blocks
// resident at one time then work on one window of neighbouring rows, so the
// n x k rows they gather (256 bytes each at k = 32 in FP64) are reused from
// L2; contiguous chunks per block spread the resident blocks over the whole
// matrix and fetched the gathered block about three times from memory.
__device__ __forceinline__ int64_t first_group() { return xcd_block(blockIdx.x, gridDim.x); }

// per-column block partial: threads of one column (same lane % KT) are summed
template <int KT>
__device__ void column_partial(double d, bool valid, int32_t j, int32_t k, double *out) {
  __shared__ double sh[kBlock];
  sh[threadIdx.x] = valid ? d : 0.0;
  __syncthreads();
  if (threadIdx.x < KT && valid) {
    double s = sh[threadIdx.x];
    for (int g = 1; g < kBlock / KT; ++g) s += sh[g * KT + threadIdx.x];
    out[(int64_t)blockIdx.x * k + j] = s;
  }
}

// Register tiling over columns: the sparse-product kernels give each thread
// kCpt columns of its row (j, j + KT, ...), so one load of a row's column
// indices and values feeds kCpt gathers, and each lane keeps kCpt times as
// many gathers in flight.
constexpr int kCpt = 2;

// acc[q] = sum_e val[e] * x(col[e], q) over one SELL row, entries in order,
// loads issued in batches of kRowBatch entries
template <typename TV, typename X>
__device__ __forceinline__ void sell_dot_cols(const int32_t *__restrict__ col,
                                              const TV *__restrict__ val, int32_t base,
                                              int32_t w, X x, TV (&acc)[kCpt]) {
#pragma unroll
  for (int q = 0; q < kCpt; ++q) acc[q] = 0;
  for (int32_t k0 = 0; k0 < w; k0 += kRowBatch) {
    int32_t c[kRowBatch];
    TV v[kRowBatch], g[kRowBatch][kCpt];
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      c[u] = 0;
      v[u] = 0;
      if (k0 + u < w) {
        const int32_t idx = base + (k0 + u) * kSlice;
        c[u] = ld_stream(&col[idx]);
        v[u] = ld_stream(&val[idx]);
      }
    }
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u)
#pragma unroll
      for (int q = 0; q < kCpt; ++q) g[u][q] = k0 + u < w ? x(c[u], q) : TV(0);
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u)
      if (k0 + u < w)
#pragma unroll
        for (int q = 0; q < kCpt; ++q) acc[q] += v[u] * g[u][q];
  }
}

// VW consecutive values of a block row as one 16-byte vector: the down step,
// the outer SpMV, the prolongation, the CG update and p = z + b p have a form
// with VW columns per thread for k a multiple of VW and 16-byte aligned blocks
// (kv = k / VW vectors per row), with a quarter (FP32) or half (FP64) of the
// threads or gathers and memory instructions.
template <typename TV>
struct Vec16;
template <>
struct Vec16<float> {
  using T = float4;
  static constexpr int width = 4;
};
template <>
struct Vec16<double> {
  using T = double2;
  static constexpr int width = 2;
};

// N consecutive values at p (N values 16-byte aligned when N fills whole
// 16-byte vectors of T)
template <typename T, int N>
__device__ __forceinline__ void ld_vals(const T *p, T (&out)[N]) {
  using V = typename Vec16<T>::T;
  constexpr int W = Vec16<T>::width;
  if constexpr (N % W == 0) {
#pragma unroll
    for (int c = 0; c < N / W; ++c) {
      const V v = reinterpret_cast<const V *>(p)[c];
      const T *e = reinterpret_cast<const T *>(&v);
#pragma unroll
      for (int q = 0; q < W; ++q) out[c * W + q] = e[q];
    }
  } else {
#pragma unroll
    for (int q = 0; q < N; ++q) out[q] = p[q];
  }
}

template <typename T, int N>
__device__ __forceinline__ void st_vals(T *p, const T (&in)[N]) {
  using V = typename Vec16<T>::T;
  constexpr int W = Vec16<T>::width;
  if constexpr (N % W == 0) {
#pragma unroll
    for (int c = 0; c < N / W; ++c) {
      V v;
      T *e = reinterpret_cast<T *>(&v);
#pragma unroll
      for (int q = 0; q < W; ++q) e[q] = in[c * W + q];
      reinterpret_cast<V *>(p)[c] = v;
    }
  } else {
#pragma unroll
    for (int q = 0; q < N; ++q) p[q] = in[q];
  }
}

// ---------------------------------------------------------------------------
// V-cycle kernels on n x k blocks
// ---------------------------------------------------------------------------

template <typename TV, typename TR, int KT>
__global__ void __launch_bounds__(kBlock) kb_pre_residual(
    int32_t n, int32_t k, const int32_t *__restrict__ sptr,
    const int32_t *__restrict__ col, const TV *__restrict__ val, const TV *__restrict__ minv,
    const TR *__restrict__ R, TV *__restrict__ Z, TV *__restrict__ T,
    const int32_t *__restrict__ stop) {
  if (*stop) return;
  const int32_t j0 = blockIdx.y * (KT * kCpt) + threadIdx.x % KT;
  if (j0 >= k) return;
  int32_t jc[kCpt];
  bool ok[kCpt];
#pragma unroll
  for (int q = 0; q < kCpt; ++q) {
    jc[q] = j0 + q * KT;
    ok[q] = jc[q] < k;
  }
  for (int64_t grp = first_group(); grp * (kBlock / KT) < n; grp += gridDim.x) {
    const int32_t row = (int32_t)(grp * (kBlock / KT)) + (int32_t)threadIdx.x / KT;
    if (row >= n) continue;
    int32_t base, w;
    sell_row(sptr, row, &base, &w);
    TV acc[kCpt];  // val holds A M^-1
    sell_dot_cols(col, val, base, w,
                  [&](int32_t c, int q) { return ok[q] ? (TV)R[(int64_t)c * k + jc[q]] : TV(0); },
                  acc);
    const TV mi = minv[row];
#pragma unroll
    for (int q = 0; q < kCpt; ++q) {
      if (!ok[q]) continue;
      const int64_t o = (int64_t)row * k + jc[q];
      const TV ri = (TV)R[o];
      Z[o] = ri * mi;
      T[o] = ri - acc[q];
    }
  }
}

// Indices and values of entries k0 .. k0 + kRowBatch - 1 of a SELL row (0
// past its end). The KT lanes of a row would all load the same addresses;
// with SHF lane u loads entry u and the others take it by shuffle (needs
// KT >= kRowBatch and every lane of the row active).
template <int KT, bool SHF, typename TA>
__device__ __forceinline__ void row_batch(const int32_t *__restrict__ col,
                                          const TA *__restrict__ val, int32_t base, int32_t k0,
                                          int32_t w, int32_t (&c)[kRowBatch],
                                          TA (&va)[kRowBatch]) {
  if constexpr (SHF && KT >= kRowBatch) {
    const int32_t lane = (int32_t)threadIdx.x % KT;
    int32_t cl = 0;
    TA vl = 0;
    if (lane < kRowBatch && k0 + lane < w) {
      const int32_t idx = base + (k0 + lane) * kSlice;
      cl = ld_stream(&col[idx]);
      vl = ld_stream(&val[idx]);
    }
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      c[u] = __shfl(cl, u, KT);
      va[u] = __shfl(vl, u, KT);
    }
  } else {
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      c[u] = 0;
      va[u] = 0;
      if (k0 + u < w) {
        const int32_t idx = base + (k0 + u) * kSlice;
        c[u] = ld_stream(&col[idx]);
        va[u] = ld_stream(&val[idx]);
      }
    }
  }
}

// kb_pre_residual for a residual block already in the hierarchy precision,
// with VW consecutive columns per lane and each gathered block row entry
// loaded as one 16-byte vector (k a multiple of VW, blocks 16-byte aligned,
// kv = k / VW); the same sums in the same order
template <typename TV, int KT, bool SHF>
__global__ void __launch_bounds__(kBlock) kb_pre_residual_v(
    int32_t n, int32_t kv, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const TV *__restrict__ val, const TV *__restrict__ minv, const TV *__restrict__ R,
    TV *__restrict__ Z, TV *__restrict__ T, const int32_t *__restrict__ stop) {
  using V = typename Vec16<TV>::T;
  constexpr int VW = Vec16<TV>::width;
  if (*stop) return;
  const int32_t jv = blockIdx.y * KT + threadIdx.x % KT;
  if (jv >= kv) return;
  const V *Rv = reinterpret_cast<const V *>(R);
  for (int64_t grp = first_group(); grp * (kBlock / KT) < n; grp += gridDim.x) {
    const int32_t row = (int32_t)(grp * (kBlock / KT)) + (int32_t)threadIdx.x / KT;
    if (row >= n) continue;
    int32_t base, w;
    sell_row(sptr, row, &base, &w);
    TV acc[VW];
#pragma unroll
    for (int q = 0; q < VW; ++q) acc[q] = 0;
    for (int32_t k0 = 0; k0 < w; k0 += kRowBatch) {
      int32_t c[kRowBatch];
      TV v[kRowBatch];
      V g[kRowBatch];
      row_batch<KT, SHF>(col, val, base, k0, w, c, v);
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u)
        if (k0 + u < w) g[u] = Rv[(int64_t)c[u] * kv + jv];
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u)
        if (k0 + u < w) {
          const TV *gu = reinterpret_cast<const TV *>(&g[u]);
#pragma unroll
          for (int q = 0; q < VW; ++q) acc[q] += v[u] * gu[q];
        }
    }
    const TV mi = minv[row];
    const int64_t o = (int64_t)row * kv + jv;
    const V r = Rv[o];
    const TV *ri = reinterpret_cast<const TV *>(&r);
    V z, t;
    TV *zo = reinterpret_cast<TV *>(&z), *to = reinterpret_cast<TV *>(&t);
#pragma unroll
    for (int q = 0; q < VW; ++q) {
      zo[q] = ri[q] * mi;
      to[q] = ri[q] - acc[q];
    }
    reinterpret_cast<V *>(Z)[o] = z;
    reinterpret_cast<V *>(T)[o] = t;
  }
}

template <typename TV, typename TR, typename TO, int KT, bool DOT>
__global__ void __launch_bounds__(kBlock) kb_post(
    int32_t n, int32_t k, const int32_t *__restrict__ sptr,
    const int32_t *__restrict__ col, const TV *__restrict__ val, const TV *__restrict__ minv,
    const TR *__restrict__ R, const TV *__restrict__ Z, TO *__restrict__ Y,
    double *__restrict__ partials, const int32_t *__restrict__ stop) {
  if (*stop) return;
  const int32_t j0 = blockIdx.y * (KT * kCpt) + threadIdx.x % KT;
  int32_t jc[kCpt];
  bool ok[kCpt];
#pragma unroll
  for (int q = 0; q < kCpt; ++q) {
    jc[q] = j0 + q * KT;
    ok[q] = jc[q] < k;
  }
  double d[kCpt];
#pragma unroll
  for (int q = 0; q < kCpt; ++q) d[q] = 0.0;
  if (ok[0]) {
    for (int64_t grp = first_group(); grp * (kBlock / KT) < n; grp += gridDim.x) {
      const int32_t row = (int32_t)(grp * (kBlock / KT)) + (int32_t)threadIdx.x / KT;
      if (row >= n) continue;
      int32_t base, w;
      sell_row(sptr, row, &base, &w);
      TV acc[kCpt];
      sell_dot_cols(col, val, base, w,
                    [&](int32_t c, int q) { return ok[q] ? Z[(int64_t)c * k + jc[q]] : TV(0); },
                    acc);
      const TV mi = minv[row];
#pragma unroll
      for (int q = 0; q < kCpt; ++q) {
        if (!ok[q]) continue;
        const int64_t o = (int64_t)row * k + jc[q];
        const TR rr = R[o];
        const TO yo = (TO)(Z[o] + ((TV)rr - acc[q]) * mi);
        Y[o] = yo;
        if (DOT) d[q] += (double)rr * (double)yo;
      }
    }
  }
  if (DOT) {
#pragma unroll
    for (int q = 0; q < kCpt; ++q) {
      if (q) __syncthreads();
      column_partial<KT>(d[q], ok[q], jc[q], k, partials);
    }
  }
}

// kb_post with VW = Vec16<TV>::width consecutive columns per lane and each
// gathered entry of Z loaded as one 16-byte vector (k a multiple of VW, blocks
// 16-byte aligned, kv = k / VW); the same sums in the same order
template <typename TV, typename TR, typename TO, int KT, bool DOT, bool SHF>
__global__ void __launch_bounds__(kBlock) kb_post_v(
    int32_t n, int32_t kv, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const TV *__restrict__ val, const TV *__restrict__ minv, const TR *__restrict__ R,
    const TV *__restrict__ Z, TO *__restrict__ Y, double *__restrict__ partials,
    const int32_t *__restrict__ stop) {
  using V = typename Vec16<TV>::T;
  constexpr int VW = Vec16<TV>::width;
  if (*stop) return;
  const int32_t jv = blockIdx.y * KT + threadIdx.x % KT;
  const int32_t k = VW * kv, j = VW * jv;
  const bool ok = jv < kv;
  const V *Zv = reinterpret_cast<const V *>(Z);
  double d[VW];
#pragma unroll
  for (int q = 0; q < VW; ++q) d[q] = 0.0;
  if (ok) {
    for (int64_t grp = first_group(); grp * (kBlock / KT) < n; grp += gridDim.x) {
      const int32_t row = (int32_t)(grp * (kBlock / KT)) + (int32_t)threadIdx.x / KT;
      if (row >= n) continue;
      int32_t base, w;
      sell_row(sptr, row, &base, &w);
      TV acc[VW];
#pragma unroll
      for (int q = 0; q < VW; ++q) acc[q] = 0;
      for (int32_t k0 = 0; k0 < w; k0 += kRowBatch) {
        int32_t c[kRowBatch];
        TV v[kRowBatch];
        V g[kRowBatch];
        row_batch<KT, SHF>(col, val, base, k0, w, c, v);
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u)
          if (k0 + u < w) g[u] = Zv[(int64_t)c[u] * kv + jv];
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u)
          if (k0 + u < w) {
            const TV *gu = reinterpret_cast<const TV *>(&g[u]);
#pragma unroll
            for (int q = 0; q < VW; ++q) acc[q] += v[u] * gu[q];
          }
      }
      const TV mi = minv[row];
      const int64_t o = (int64_t)row * k + j;
      TR rr[VW];
      TV zz[VW];
      TO yo[VW];
      ld_vals(R + o, rr);
      ld_vals(Z + o, zz);
#pragma unroll
      for (int q = 0; q < VW; ++q) {
        yo[q] = (TO)(zz[q] + ((TV)rr[q] - acc[q]) * mi);
        if (DOT) d[q] += (double)rr[q] * (double)yo[q];
      }
      st_vals(Y + o, yo);
    }
  }
  if (DOT) {
#pragma unroll
    for (int q = 0; q < VW; ++q) {
      if (q) __syncthreads();
      column_partial<KT>(d[q], ok, j + q, k, partials);
    }
  }
}

// T = R - A Z (the residual after extra pre-smoothing sweeps)
template <typename TV, typename TR, int KT>
__global__ void __launch_bounds__(kBlock) kb_resid(
    int32_t n, int32_t k, const int32_t *__restrict__ sptr,
    const int32_t *__restrict__ col, const TV *__restrict__ val, const TR *__restrict__ R,
    const TV *__restrict__ Z, TV *__restrict__ T, const int32_t *__restrict__ stop) {
  if (*stop) return;
  const int32_t j0 = blockIdx.y * (KT * kCpt) + threadIdx.x % KT;
  if (j0 >= k) return;
  int32_t jc[kCpt];
  bool ok[kCpt];
#pragma unroll
  for (int q = 0; q < kCpt; ++q) {
    jc[q] = j0 + q * KT;
    ok[q] = jc[q] < k;
  }
  for (int64_t grp = first_group(); grp * (kBlock / KT) < n; grp += gridDim.x) {
    const int32_t row = (int32_t)(grp * (kBlock / KT)) + (int32_t)threadIdx.x / KT;
    if (row >= n) continue;
    int32_t base, w;
    sell_row(sptr, row, &base, &w);
    TV acc[kCpt];
    sell_dot_cols(col, val, base, w,
                  [&](int32_t c, int q) { return ok[q] ? Z[(int64_t)c * k + jc[q]] : TV(0); },
                  acc);
#pragma unroll
    for (int q = 0; q < kCpt; ++q) {
      if (!ok[q]) continue;
      const int64_t o = (int64_t)row * k + jc[q];
      T[o] = (TV)R[o] - acc[q];
    }
  }
}


// The kernels that take one thread per element (the CG update, p = z + b p,
// restriction, prolongation) choose their column tile from k alone: the
// smallest tile covering k, at most 64. One block then reads and writes whole
// rows; with a narrower tile an FP32 row (4k bytes) is split into partial
// cache lines that two blocks fetch and write separately, and the restriction
// and prolongation fetched twice their bytes that way.
bool aligned16(const void *p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; }

int32_t row_tile(int32_t k) { return k <= 4 ? 4 : k <= 8 ? 8 : k <= 16 ? 16 : k <= 32 ? 32 : 64; }

template <typename F>
void with_row_tile(int32_t k, F &&f) {
  switch (row_tile(k)) {
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    case 32: f(std::integral_constant<int, 32>{}); break;
    default: f(std::integral_constant<int, 64>{}); break;
  }
}

// R_c(J) = sum over the segment of J (aggregate-major positions), in order,
// of p_m T(m)
template <typename TV, int KT>
__global__ void kb_restrict(int32_t nc, int32_t k, const int32_t *__restrict__ seg,
                            const TV *__restrict__ pp, const TV *__restrict__ T,
                            TV *__restrict__ Rc, const int32_t *__restrict__ stop) {
  if (*stop) return;
  const int32_t j = blockIdx.y * KT + threadIdx.x % KT;
  const int64_t I = (int64_t)blockIdx.x * (kBlock / KT) + threadIdx.x / KT;
  if (j >= k || I >= nc) return;
  const int32_t b = seg[I], e = seg[I + 1];
  TV s = 0;
  for (int32_t m0 = b; m0 < e; m0 += 8) {  // loads of eight members before their use
    TV pv[8], tv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      pv[u] = tv[u] = 0;
      if (m0 + u < e) {
        pv[u] = pp[m0 + u];
        tv[u] = T[(int64_t)(m0 + u) * k + j];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (m0 + u < e) s += pv[u] * tv[u];
  }
  Rc[I * k + j] = s;
}

template <typename TV, int KT>
__global__ void kb_prolong(int32_t n, int32_t k, const int32_t *__restrict__ aggp,
                           const TV *__restrict__ pp, const TV *__restrict__ Zc,
                           TV *__restrict__ Z, const int32_t *__restrict__ stop) {
  if (*stop) return;
  const int32_t j = blockIdx.y * KT + threadIdx.x % KT;
  const int64_t i = (int64_t)blockIdx.x * (kBlock / KT) + threadIdx.x / KT;
  if (j >= k || i >= n) return;
  Z[i * k + j] += pp[i] * Zc[(int64_t)aggp[i] * k + j];
}

// the prolongation with VW consecutive columns per thread
template <typename TV, int KT>
__global__ void kb_prolong_v(int32_t n, int32_t kv, const int32_t *__restrict__ aggp,
                             const TV *__restrict__ pp, const TV *__restrict__ Zc,
                             TV *__restrict__ Z, const int32_t *__restrict__ stop) {
  using V = typename Vec16<TV>::T;
  constexpr int VW = Vec16<TV>::width;
  if (*stop) return;
  const int32_t jv = blockIdx.y * KT + threadIdx.x % KT;
  const int64_t i = (int64_t)blockIdx.x * (kBlock / KT) + threadIdx.x / KT;
  if (jv >= kv || i >= n) return;
  const TV p = pp[i];
  const V c = reinterpret_cast<const V *>(Zc)[(int64_t)aggp[i] * kv + jv];
  V *zp = reinterpret_cast<V *>(Z) + i * kv + jv;
  V z = *zp;
  const TV *cv = reinterpret_cast<const TV *>(&c);
  TV *zv = reinterpret_cast<TV *>(&z);
#pragma unroll
  for (int q = 0; q < VW; ++q) zv[q] += p * cv[q];
  *zp = z;
}

// row permutation of an n x k block: Dst(q) = Src(perm q) (IN) or
// Dst(perm q) = Src(q) (OUT)
template <bool IN>
__global__ void kb_permute_rows(int32_t n, int32_t k, const int32_t *__restrict__ perm,
                                const double *__restrict__ Src, double *__restrict__ Dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * k) return;
  const int64_t q = e / k, j = e % k;
  if (IN) Dst[e] = Src[(int64_t)perm[q] * k + j];
  else Dst[(int64_t)perm[q] * k + j] = Src[e];
}

// Z = A_L^-1 R on the coarsest level, one thread per (row, column)
template <typename TI, typename TO>
__global__ void kb_coarse(int32_t nL, int32_t k, const double *__restrict__ Ainv,
                          const TI *__restrict__ R, TO *__restrict__ Z,
                          const int32_t *__restrict__ stop) {
  if (*stop) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nL * k) return;
  const int32_t i = (int32_t)(e / k), j = (int32_t)(e % k);
  const double *row = Ainv + (int64_t)i * nL;
  double s = 0.0;
  for (int32_t m0 = 0; m0 < nL; m0 += 8) {  // loads of eight terms before their use
    double av[8], rv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      av[u] = rv[u] = 0.0;
      if (m0 + u < nL) {
        av[u] = row[m0 + u];
        rv[u] = (double)R[(int64_t)(m0 + u) * k + j];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (m0 + u < nL) s += av[u] * rv[u];
  }
  Z[e] = (TO)s;
}

// ---------------------------------------------------------------------------
// per-column CG kernels (FP64)
// ---------------------------------------------------------------------------

template <int KT>
__global__ void __launch_bounds__(kBlock) kb_spmv(
    int32_t n, int32_t k, const int32_t *__restrict__ sptr,
    const int32_t *__restrict__ col, const double *__restrict__ val,
    const double *__restrict__ Xin, const double *__restrict__ B, double *__restrict__ Out,
    float *__restrict__ OutF, double *__restrict__ partials, int32_t mode,
    const int32_t *__restrict__ stop) {
  // mode 0: Out = A Xin, partials (Xin, Out)         (q = A p, (p, q))
  // mode 1: Out = B - A Xin, partials (B, B), (Out, Out)   (initial residual);
  //         OutF (if not null) = float(Out)
  // mode 2: partials (B - A Xin)^2 only               (true residual)
  if (stop && *stop) return;
  const int32_t j0 = blockIdx.y * (KT * kCpt) + threadIdx.x % KT;
  int32_t jc[kCpt];
  bool ok[kCpt];
#pragma unroll
  for (int q = 0; q < kCpt; ++q) {
    jc[q] = j0 + q * KT;
    ok[q] = jc[q] < k;
  }
  double d0[kCpt], d1[kCpt];
#pragma unroll
  for (int q = 0; q < kCpt; ++q) d0[q] = d1[q] = 0.0;
  if (ok[0]) {
    for (int64_t grp = first_group(); grp * (kBlock / KT) < n; grp += gridDim.x) {
      const int32_t row = (int32_t)(grp * (kBlock / KT)) + (int32_t)threadIdx.x / KT;
      if (row >= n) continue;
      int32_t base, w;
      sell_row(sptr, row, &base, &w);
      double acc[kCpt];
      sell_dot_cols(
          col, val, base, w,
          [&](int32_t c, int q) { return ok[q] ? Xin[(int64_t)c * k + jc[q]] : 0.0; }, acc);
#pragma unroll
      for (int q = 0; q < kCpt; ++q) {
        if (!ok[q]) continue;
        const int64_t o = (int64_t)row * k + jc[q];
        if (mode == 0) {
          Out[o] = acc[q];
          d0[q] += Xin[o] * acc[q];
        } else {
          const double bi = B[o], ri = bi - acc[q];
          if (mode == 1) {
            Out[o] = ri;
            if (OutF) OutF[o] = (float)ri;
            d0[q] += bi * bi;
            d1[q] += ri * ri;
          } else {
            d0[q] += ri * ri;
          }
        }
      }
    }
  }
  const int64_t plane = (int64_t)kBatchBlocks * k;
#pragma unroll
  for (int q = 0; q < kCpt; ++q) {
    if (q) __syncthreads();
    column_partial<KT>(d0[q], ok[q], jc[q], k, partials);
    if (mode == 1) {
      __syncthreads();
      column_partial<KT>(d1[q], ok[q], jc[q], k, partials + plane);
    }
  }
}

// kb_spmv with two consecutive columns per lane, each gathered block row
// entry loaded as one 16-byte vector (k even, blocks 16-byte aligned, kv =
// k / 2): half the gather instructions; the same sums in the same order
template <int KT, typename TA, bool SHF>
__global__ void __launch_bounds__(kBlock) kb_spmv_v(
    int32_t n, int32_t kv, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
    const TA *__restrict__ val, const double *__restrict__ Xin,
    const double *__restrict__ B, double *__restrict__ Out, float *__restrict__ OutF,
    double *__restrict__ partials, int32_t mode, const int32_t *__restrict__ stop) {
  if (stop && *stop) return;
  const int32_t jv = blockIdx.y * KT + threadIdx.x % KT;
  const int32_t k = 2 * kv, j = 2 * jv;
  const bool ok = jv < kv;
  const double2 *X2 = reinterpret_cast<const double2 *>(Xin);
  double d0[2] = {0.0, 0.0}, d1[2] = {0.0, 0.0};
  if (ok) {
    for (int64_t grp = first_group(); grp * (kBlock / KT) < n; grp += gridDim.x) {
      const int32_t row = (int32_t)(grp * (kBlock / KT)) + (int32_t)threadIdx.x / KT;
      if (row >= n) continue;
      int32_t base, w;
      sell_row(sptr, row, &base, &w);
      double a0 = 0.0, a1 = 0.0;
      for (int32_t k0 = 0; k0 < w; k0 += kRowBatch) {
        int32_t c[kRowBatch];
        TA va[kRowBatch];  // as stored: converted at the product, not inside the guard
        double2 g[kRowBatch];
        row_batch<KT, SHF>(col, val, base, k0, w, c, va);
        double v[kRowBatch];
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u) v[u] = (double)va[u];
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u)
          g[u] = k0 + u < w ? X2[(int64_t)c[u] * kv + jv] : make_double2(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u)
          if (k0 + u < w) {
            a0 += v[u] * g[u].x;
            a1 += v[u] * g[u].y;
          }
      }
      const int64_t o = (int64_t)row * kv + jv;
      if (mode == 0) {
        reinterpret_cast<double2 *>(Out)[o] = make_double2(a0, a1);
        const double2 xo = X2[o];
        d0[0] += xo.x * a0;
        d0[1] += xo.y * a1;
      } else {
        const double2 bi = reinterpret_cast<const double2 *>(B)[o];
        const double r0 = bi.x - a0, r1 = bi.y - a1;
        if (mode == 1) {
          reinterpret_cast<double2 *>(Out)[o] = make_double2(r0, r1);
          if (OutF) reinterpret_cast<float2 *>(OutF)[o] = make_float2((float)r0, (float)r1);
          d0[0] += bi.x * bi.x;
          d0[1] += bi.y * bi.y;
          d1[0] += r0 * r0;
          d1[1] += r1 * r1;
        } else {
          d0[0] += r0 * r0;
          d0[1] += r1 * r1;
        }
      }
    }
  }
  const int64_t plane = (int64_t)kBatchBlocks * k;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    if (q) __syncthreads();
    column_partial<KT>(d0[q], ok, j + q, k, partials);
    if (mode == 1) {
      __syncthreads();
      column_partial<KT>(d1[q], ok, j + q, k, partials + plane);
    }
  }
}

// per-column partials of (U, V) (a level-0 coarsest solve has no smoother
// to fuse the CG dot product into)
template <int KT>
__global__ void __launch_bounds__(kBlock) kb_dot(int32_t n, int32_t k,
                                                 const double *__restrict__ U,
                                                 const double *__restrict__ V,
                                                 double *__restrict__ partials,
                                                 const int32_t *__restrict__ stop) {
  if (*stop) return;
  const int32_t j = blockIdx.y * KT + threadIdx.x % KT;
  const bool valid = j < k;
  double d = 0.0;
  if (valid)
    for (int64_t grp = first_group(); grp * (kBlock / KT) < n; grp += gridDim.x) {
      const int32_t row = (int32_t)(grp * (kBlock / KT)) + (int32_t)threadIdx.x / KT;
      if (row < n) d += U[(int64_t)row * k + j] * V[(int64_t)row * k + j];
    }
  column_partial<KT>(d, valid, j, k, partials);
}

template <int KT>
__global__ void __launch_bounds__(kBlock) kb_update(int32_t n, int32_t k,
                                                    double *__restrict__ X,
                                                    double *__restrict__ R,
                                                    float *__restrict__ Rf,
                                                    const double *__restrict__ P,
                                                    const double *__restrict__ Q,
                                                    const double *__restrict__ colv,
                                                    const int32_t *__restrict__ done,
                                                    double *__restrict__ partials,
                                                    const int32_t *__restrict__ stop) {
  if (*stop) return;
  const int32_t j = blockIdx.y * KT + threadIdx.x % KT;
  const bool valid = j < k;
  const bool live = valid && done[j] == 0;
  const double alpha = valid ? colv[cAlpha * k + j] : 0.0;
  double d = 0.0;
  if (live) {
    for (int64_t grp = first_group(); grp * (kBlock / KT) < n; grp += gridDim.x) {
      const int32_t row = (int32_t)(grp * (kBlock / KT)) + (int32_t)threadIdx.x / KT;
      if (row >= n) continue;
      const int64_t o = (int64_t)row * k + j;
      X[o] += alpha * P[o];
      const double ri = R[o] - alpha * Q[o];
      R[o] = ri;
      if (Rf) Rf[o] = (float)ri;
      d += ri * ri;
    }
  }
  column_partial<KT>(d, valid, j, k, partials);
}

template <int KT, typename TZ = double>
__global__ void kb_xpay(int32_t n, int32_t k, const TZ *__restrict__ Z,
                        double *__restrict__ P, const double *__restrict__ colv,
                        const int32_t *__restrict__ done, int32_t copy,
                        const int32_t *__restrict__ stop) {
  if (*stop) return;
  const int32_t j = blockIdx.y * KT + threadIdx.x % KT;
  const int64_t i = (int64_t)blockIdx.x * (kBlock / KT) + threadIdx.x / KT;
  if (j >= k || i >= n || done[j]) return;
  const int64_t o = i * k + j;
  const double z = (double)Z[o];
  P[o] = copy ? z : z + colv[cBeta * k + j] * P[o];
}

// r -= alpha q with two columns per thread (k even, blocks 16-byte aligned),
// the FP32 copy of r and the (r, r) partials; a converged column's half of r
// is stored back unchanged, and its partial sum is zero as in the one-value
// form. x += alpha p is left to kb_xpay_v, which reads p anyway: one block
// read fewer per iteration, the same arithmetic.
template <int KT>
__global__ void __launch_bounds__(kBlock) kb_update_v(int32_t n, int32_t kv,
                                                      double *__restrict__ R,
                                                      float *__restrict__ Rf,
                                                      const double *__restrict__ Q,
                                                      const double *__restrict__ colv,
                                                      const int32_t *__restrict__ done,
                                                      double *__restrict__ partials,
                                                      const int32_t *__restrict__ stop) {
  if (*stop) return;
  const int32_t jv = blockIdx.y * KT + threadIdx.x % KT;
  const int32_t k = 2 * kv, j = 2 * jv;
  const bool valid = jv < kv;
  const bool live0 = valid && done[j] == 0, live1 = valid && done[j + 1] == 0;
  const double a0 = live0 ? colv[cAlpha * k + j] : 0.0;
  const double a1 = live1 ? colv[cAlpha * k + j + 1] : 0.0;
  double d0 = 0.0, d1 = 0.0;
  if (live0 || live1) {
    double2 *R2 = reinterpret_cast<double2 *>(R);
    const double2 *Q2 = reinterpret_cast<const double2 *>(Q);
    float2 *Rf2 = reinterpret_cast<float2 *>(Rf);
    for (int64_t grp = first_group(); grp * (kBlock / KT) < n; grp += gridDim.x) {
      const int32_t row = (int32_t)(grp * (kBlock / KT)) + (int32_t)threadIdx.x / KT;
      if (row >= n) continue;
      const int64_t o = (int64_t)row * kv + jv;
      double2 r = R2[o];
      const double2 q = Q2[o];
      if (live0) {
        r.x = r.x - a0 * q.x;
        d0 += r.x * r.x;
      }
      if (live1) {
        r.y = r.y - a1 * q.y;
        d1 += r.y * r.y;
      }
      R2[o] = r;
      if (Rf) Rf2[o] = make_float2((float)r.x, (float)r.y);
    }
  }
  column_partial<KT>(d0, valid, j, k, partials);
  __syncthreads();
  column_partial<KT>(d1, valid, j + 1, k, partials);
}

// The end of an iteration with two columns per thread (k even, blocks
// 16-byte aligned): x += alpha p for the columns whose alpha this iteration
// set (xpend; also those that converged or broke down since, which is why
// the kernel runs when every column has stopped), then p = z + beta p for
// the live ones; a stopped column's half of p is stored back unchanged.
template <int KT, typename TZ>
__global__ void kb_xpay_v(int32_t n, int32_t kv, const TZ *__restrict__ Z,
                          double *__restrict__ P, double *__restrict__ X,
                          const double *__restrict__ colv, const int32_t *__restrict__ done,
                          const int32_t *__restrict__ xpend) {
  const int32_t jv = blockIdx.y * KT + threadIdx.x % KT;
  const int64_t i = (int64_t)blockIdx.x * (kBlock / KT) + threadIdx.x / KT;
  if (jv >= kv || i >= n) return;
  const int32_t k = 2 * kv, j = 2 * jv;
  const bool live0 = done[j] == 0, live1 = done[j + 1] == 0;
  const bool xp0 = xpend[j] != 0, xp1 = xpend[j + 1] != 0;
  if (!live0 && !live1 && !xp0 && !xp1) return;
  const int64_t o = i * kv + jv;
  double2 v = reinterpret_cast<double2 *>(P)[o];
  if (xp0 || xp1) {
    double2 x = reinterpret_cast<double2 *>(X)[o];
    if (xp0) x.x += colv[cAlpha * k + j] * v.x;
    if (xp1) x.y += colv[cAlpha * k + j + 1] * v.y;
    reinterpret_cast<double2 *>(X)[o] = x;
  }
  if (!live0 && !live1) return;
  double2 z;
  if constexpr (std::is_same<TZ, float>::value) {
    const float2 zf = reinterpret_cast<const float2 *>(Z)[o];
    z = make_double2((double)zf.x, (double)zf.y);
  } else {
    z = reinterpret_cast<const double2 *>(Z)[o];
  }
  if (live0) v.x = z.x + colv[cBeta * k + j] * v.x;
  if (live1) v.y = z.y + colv[cBeta * k + j + 1] * v.y;
  reinterpret_cast<double2 *>(P)[o] = v;
}

template <int KT>
__global__ void kb_zero_cols(int32_t n, int32_t k, double *__restrict__ X,
                             const int32_t *__restrict__ done) {
  const int32_t j = blockIdx.y * KT + threadIdx.x % KT;
  const int64_t i = (int64_t)blockIdx.x * (kBlock / KT) + threadIdx.x / KT;
  if (j >= k || i >= n || done[j] != 4) return;
  X[i * k + j] = 0.0;
}

__global__ void kb_init_cols(int32_t k, double rtol, int32_t maxit, double *colv, int32_t *iter,
                             int32_t *done, int32_t *xpend, int32_t *stop) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) *stop = 0;
  if (j >= k) return;
  for (int f = 0; f < kColFields; ++f) colv[f * k + j] = 0.0;
  colv[cRtol * k + j] = rtol;
  iter[j] = 0;
  xpend[j] = 0;
  done[j] = maxit < 0 ? 2 : 0;
}

// per-column fixed-order sum of the block partials and the CG update of op
__global__ void __launch_bounds__(kBlock) kb_finalize(int32_t op, int32_t nparts, int32_t k,
                                                      const double *__restrict__ partials,
                                                      double *__restrict__ colv,
                                                      int32_t *__restrict__ iter,
                                                      int32_t *__restrict__ done,
                                                      int32_t *__restrict__ xpend, int32_t maxit,
                                                      const int32_t *__restrict__ stop) {
  const int32_t j = blockIdx.x;
  // the previous iteration's x update has been applied by now (also in
  // iterations queued after every column stopped)
  if (op == bPq && threadIdx.x == 0) xpend[j] = 0;
  if (stop && *stop) return;
  __shared__ double sh[2][kBlock / kWave];
  const int nv = op == bInit ? 2 : 1;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int64_t plane = (int64_t)kBatchBlocks * k;
  for (int q = 0; q < nv; ++q) {
    double a = 0.0;
    for (int32_t b = threadIdx.x; b < nparts; b += kBlock) a += partials[q * plane + (int64_t)b * k + j];
    for (int o = kWave / 2; o > 0; o >>= 1) a += __shfl_down(a, o, kWave);
    if (lane == 0) sh[q][wid] = a;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double tot[2] = {0.0, 0.0};
  for (int q = 0; q < nv; ++q) {
    double t = sh[q][0];
    for (int w = 1; w < kBlock / kWave; ++w) t += sh[q][w];
    tot[q] = t;
  }
  double *c = colv;
  const double rtol = c[cRtol * k + j];
  if (op == bTrue) {
    c[cRrTrue * k + j] = tot[0];
    return;
  }
  if (op == bInit) {
    c[cBb * k + j] = tot[0];
    c[cRr * k + j] = tot[1];
    if (done[j]) return;
    if (tot[0] == 0.0) done[j] = 4;
    else if (sqrt(tot[1]) <= rtol * sqrt(tot[0])) done[j] = 1;
    else if (maxit <= 0) done[j] = 2;
    return;
  }
  if (done[j]) return;
  switch (op) {
    case bPq:
      c[cPq * k + j] = tot[0];
      if (!(tot[0] > 0.0)) {
        done[j] = 3;
      } else {
        c[cAlpha * k + j] = c[cRho * k + j] / tot[0];
        xpend[j] = 1;
      }
      break;
    case bRr:
      c[cRr * k + j] = tot[0];
      iter[j] += 1;
      if (sqrt(tot[0]) <= rtol * sqrt(c[cBb * k + j])) done[j] = 1;
      else if (iter[j] >= maxit) done[j] = 2;
      break;
    case bRz0:
      if (!(tot[0] > 0.0)) done[j] = 3;
      else c[cRho * k + j] = tot[0];
      break;
    default:  // bRz
      if (!(tot[0] > 0.0)) {
        done[j] = 3;
      } else {
        c[cBeta * k + j] = tot[0] / c[cRho * k + j];
        c[cRho * k + j] = tot[0];
      }
      break;
  }
}

__global__ void kb_all_done(int32_t k, const int32_t *done, int32_t *stop) {
  if (threadIdx.x != 0) return;
  int32_t all = 1;
  for (int32_t j = 0; j < k; ++j) all &= done[j] != 0 ? 1 : 0;
  *stop = all;
}

// the vector kernels' tile for kv vectors per row: row_tile(kv) scaled by
// the autotuned 2^vshift, kept within 4..64
template <typename F>
void with_vec_tile(const Batch &B, int32_t kv, F &&f) {
  int32_t t = row_tile(kv);
  t = B.vshift > 0 ? t << B.vshift : t >> -B.vshift;
  with_row_tile(t < 4 ? 4 : (t > 64 ? 64 : t), f);
}

// ---------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------

struct BGeom {
  dim3 grid;
};

// streaming geometry: one x-block per row group of kBlock / kt rows, at most
// kBatchBlocks (the blocks then take further groups in turn)
BGeom bgeom(int64_t n, int32_t k, int kt) {
  const int64_t rpp = kBlock / kt;  // rows per group
  int64_t groups = (n + rpp - 1) / rpp;
  int64_t bx = groups < kBatchBlocks ? groups : kBatchBlocks;
  if (bx < 1) bx = 1;
  return {dim3((unsigned)bx, (unsigned)((k + kt - 1) / kt))};
}

// grid of the column-tiled sparse-product kernels (kCpt columns per thread)
dim3 tgrid(const BGeom &g, int32_t k, int kt) {
  return dim3(g.grid.x, (unsigned)((k + kt * kCpt - 1) / (kt * kCpt)));
}

dim3 egrid(int64_t n, int32_t k, int kt) {  // one thread per element
  const int64_t rpb = kBlock / kt;
  return dim3((unsigned)((n + rpb - 1) / rpb), (unsigned)((k + kt - 1) / kt));
}

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

void bfinalize(amg_hierarchy *h, int32_t op, int32_t nparts, int32_t maxit, const int32_t *stop) {
  Batch &B = *h->batch;
  kb_finalize<<<B.k, kBlock, 0, h->stream>>>(op, nparts, B.k, B.partials, B.col, B.iter, B.done,
                                            B.xpend, maxit, stop);
}

// whether the block solve keeps the V-cycle's output in Batch::Zf: an FP32
// hierarchy of more than one level whose final post-smoothing and
// p = z + beta p take their vector forms
bool z32(const amg_hierarchy *h) {
  const Batch &B = *h->batch;
  return B.Zf && h->lv.size() > 1 && B.k % 4 == 0 && aligned16(B.Zf) && aligned16(B.R) &&
         aligned16(B.z[0]) && aligned16(B.y[0]) && aligned16(B.t[0]) && B.k % 2 == 0 &&
         aligned16(B.X) && aligned16(B.P) && aligned16(B.Q) &&
         (!B.Rf || reinterpret_cast<uintptr_t>(B.Rf) % 8 == 0);
}

// one block V-cycle: Z = B_0 R on all k columns; with rz_op >= 0 also the
// per-column (R, Z) and that finalize
template <typename TV, int KT>
void vcycle_b(amg_hierarchy *h, const double *R0, double *Z0, int32_t rz_op, int32_t maxit,
              const int32_t *stop) {
  hipStream_t s = h->stream;
  Batch &B = *h->batch;
  const int32_t k = B.k;
  const int32_t L = (int32_t)h->lv.size() - 1;
  if (L == 0) {
    const int32_t nL = h->C.n;
    kb_coarse<double, double><<<ceil_div((int64_t)nL * k, kBlock), kBlock, 0, s>>>(
        nL, k, h->C.Ainv, R0, Z0, stop);
    if (rz_op >= 0) {
      const BGeom g = bgeom(nL, k, KT);
      kb_dot<KT><<<g.grid, kBlock, 0, s>>>(nL, k, R0, Z0, B.partials, stop);
      bfinalize(h, rz_op, (int32_t)g.grid.x, maxit, stop);
    }
    return;
  }
  // Down: the first pre-sweep from zero with the residual through A M^-1,
  // further sweeps alternating z and y, then the residual of the last one;
  // restriction of the residual t. zc[l] is the buffer holding z_l.
  const int32_t pre = h->params.pre, post = h->params.post;
  // The FP32 hierarchy's level-0 kernels use the residual only rounded to
  // FP32 (except the final sweep's CG dot product): they read B.Rf, which
  // holds float(B.R), and gather 4-byte entries instead of 8-byte ones.
  const TV *R0v = std::is_same<TV, float>::value && R0 == B.R && B.Rf
                      ? reinterpret_cast<const TV *>(B.Rf)
                      : nullptr;
  std::vector<TV *> zc(L), yout(L + 1);
  for (int32_t l = 0; l < L; ++l) {
    Level &F = h->lv[l];
    const BGeom g = bgeom(F.n, k, KT);
    TV *z = (TV *)B.z[l], *y = (TV *)B.y[l], *t = (TV *)B.t[l];
    // the residual of this level in the hierarchy precision, if there is one
    const TV *Rl = l > 0 ? (const TV *)B.r[l]
                         : (R0v ? R0v
                                : (std::is_same<TV, double>::value
                                       ? reinterpret_cast<const TV *>(R0)
                                       : nullptr));
    constexpr int VW = Vec16<TV>::width;
    if (Rl && k % VW == 0 && aligned16(Rl) && aligned16(z) && aligned16(t))
      with_vec_tile(B, k / VW, [&](auto kt) {
        constexpr int KV = decltype(kt)::value;
        const BGeom gv = bgeom(F.n, k / VW, KV);
        if ((k / VW) % KV == 0)  // every lane of a row active: shuffled index loads
          kb_pre_residual_v<TV, KV, true><<<gv.grid, kBlock, 0, s>>>(
              F.n, k / VW, F.S.sptr, F.S.col, svals<TV>(F), minv<TV>(F), Rl, z, t, stop);
        else
          kb_pre_residual_v<TV, KV, false><<<gv.grid, kBlock, 0, s>>>(
              F.n, k / VW, F.S.sptr, F.S.col, svals<TV>(F), minv<TV>(F), Rl, z, t, stop);
      });
    else if (l == 0 && R0v)
      kb_pre_residual<TV, TV, KT><<<tgrid(g, k, KT), kBlock, 0, s>>>(
          F.n, k, F.S.sptr, F.S.col, svals<TV>(F), minv<TV>(F), R0v, z, t, stop);
    else if (l == 0)
      kb_pre_residual<TV, double, KT><<<tgrid(g, k, KT), kBlock, 0, s>>>(
          F.n, k, F.S.sptr, F.S.col, svals<TV>(F), minv<TV>(F), R0, z, t, stop);
    else
      kb_pre_residual<TV, TV, KT><<<tgrid(g, k, KT), kBlock, 0, s>>>(
          F.n, k, F.S.sptr, F.S.col, svals<TV>(F), minv<TV>(F), (const TV *)B.r[l], z,
          t, stop);
    for (int32_t sw = 1; sw < pre; ++sw) {
      if (l == 0 && R0v)
        kb_post<TV, TV, TV, KT, false><<<tgrid(g, k, KT), kBlock, 0, s>>>(
            F.n, k, F.S.sptr, F.S.col, vals<TV>(F), minv<TV>(F), R0v, z, y, nullptr, stop);
      else if (l == 0)
        kb_post<TV, double, TV, KT, false><<<tgrid(g, k, KT), kBlock, 0, s>>>(
            F.n, k, F.S.sptr, F.S.col, vals<TV>(F), minv<TV>(F), R0, z, y, nullptr,
            stop);
      else
        kb_post<TV, TV, TV, KT, false><<<tgrid(g, k, KT), kBlock, 0, s>>>(
            F.n, k, F.S.sptr, F.S.col, vals<TV>(F), minv<TV>(F), (const TV *)B.r[l], z,
            y, nullptr, stop);
      std::swap(z, y);
    }
    if (pre > 1) {
      if (l == 0 && R0v)
        kb_resid<TV, TV, KT><<<tgrid(g, k, KT), kBlock, 0, s>>>(
            F.n, k, F.S.sptr, F.S.col, vals<TV>(F), R0v, z, t, stop);
      else if (l == 0)
        kb_resid<TV, double, KT><<<tgrid(g, k, KT), kBlock, 0, s>>>(
            F.n, k, F.S.sptr, F.S.col, vals<TV>(F), R0, z, t, stop);
      else
        kb_resid<TV, TV, KT><<<tgrid(g, k, KT), kBlock, 0, s>>>(
            F.n, k, F.S.sptr, F.S.col, vals<TV>(F), (const TV *)B.r[l], z, t, stop);
    }
    zc[l] = z;
    const Level &C = h->lv[l + 1];
    with_row_tile(k, [&](auto kt) {
      constexpr int KE = decltype(kt)::value;
      kb_restrict<TV, KE><<<egrid(C.n, k, KE), kBlock, 0, s>>>(C.n, k, F.seg, ppv<TV>(F), t,
                                                              (TV *)B.r[l + 1], stop);
    });
  }
  const int32_t nL = h->C.n;
  yout[L] = (TV *)B.y[L];
  kb_coarse<TV, TV><<<ceil_div((int64_t)nL * k, kBlock), kBlock, 0, s>>>(
      nL, k, h->C.Ainv, (const TV *)B.r[L], yout[L], stop);
  // Up: prolongation of the coarser level's result into z_l, then the post
  // sweeps; each writes a buffer of the level other than its input, and
  // yout[l] records where the last one (l > 0) left y_l.
  for (int32_t l = L - 1; l >= 0; --l) {
    Level &F = h->lv[l];
    constexpr int VW = Vec16<TV>::width;
    if (k % VW == 0 && aligned16(yout[l + 1]) && aligned16(zc[l]))
      with_vec_tile(B, k / VW, [&](auto kt) {
        constexpr int KE = decltype(kt)::value;
        kb_prolong_v<TV, KE><<<egrid(F.n, k / VW, KE), kBlock, 0, s>>>(
            F.n, k / VW, F.aggp, ppv<TV>(F), yout[l + 1], zc[l], stop);
      });
    else
      with_row_tile(k, [&](auto kt) {
        constexpr int KE = decltype(kt)::value;
        kb_prolong<TV, KE><<<egrid(F.n, k, KE), kBlock, 0, s>>>(F.n, k, F.aggp, ppv<TV>(F),
                                                               yout[l + 1], zc[l], stop);
      });
    const BGeom g = bgeom(F.n, k, KT);
    TV *bufs[3] = {(TV *)B.y[l], (TV *)B.z[l], (TV *)B.t[l]};
    TV *z = zc[l];
    auto other = [&](const TV *in) {
      for (TV *b : bufs)
        if (b != in) return b;
      return bufs[0];
    };
    for (int32_t sw = 0; sw < post; ++sw) {
      const bool last = sw + 1 == post;
      if (l > 0) {
        TV *out = other(z);
        kb_post<TV, TV, TV, KT, false><<<tgrid(g, k, KT), kBlock, 0, s>>>(
            F.n, k, F.S.sptr, F.S.col, vals<TV>(F), minv<TV>(F), (const TV *)B.r[l], z,
            out, nullptr, stop);
        z = out;
        if (last) yout[l] = out;
      } else if (!last) {
        TV *out = other(z);
        if (R0v)
          kb_post<TV, TV, TV, KT, false><<<tgrid(g, k, KT), kBlock, 0, s>>>(
              F.n, k, F.S.sptr, F.S.col, vals<TV>(F), minv<TV>(F), R0v, z, out, nullptr,
              stop);
        else
          kb_post<TV, double, TV, KT, false><<<tgrid(g, k, KT), kBlock, 0, s>>>(
              F.n, k, F.S.sptr, F.S.col, vals<TV>(F), minv<TV>(F), R0, z, out, nullptr,
              stop);
        z = out;
      } else if (rz_op >= 0) {
        constexpr int VW = Vec16<TV>::width;
        if (std::is_same<TV, float>::value && Z0 == B.Z && z32(h)) {
          // the FP32 store of z (same numbers, see Batch::Zf)
          int32_t np = 0;
          with_vec_tile(B, k / VW, [&](auto kt) {
            constexpr int KV = decltype(kt)::value;
            const BGeom gv = bgeom(F.n, k / VW, KV);
            if ((k / VW) % KV == 0)
              kb_post_v<TV, double, float, KV, true, true><<<gv.grid, kBlock, 0, s>>>(
                  F.n, k / VW, F.S.sptr, F.S.col, vals<TV>(F), minv<TV>(F), R0, z, B.Zf,
                  B.partials, stop);
            else
              kb_post_v<TV, double, float, KV, true, false><<<gv.grid, kBlock, 0, s>>>(
                  F.n, k / VW, F.S.sptr, F.S.col, vals<TV>(F), minv<TV>(F), R0, z, B.Zf,
                  B.partials, stop);
            np = (int32_t)gv.grid.x;
          });
          bfinalize(h, rz_op, np, maxit, stop);
        } else if (k % VW == 0 && aligned16(R0) && aligned16(z) && aligned16(Z0)) {
          int32_t np = 0;
          with_vec_tile(B, k / VW, [&](auto kt) {
            constexpr int KV = decltype(kt)::value;
            const BGeom gv = bgeom(F.n, k / VW, KV);
            if ((k / VW) % KV == 0)
              kb_post_v<TV, double, double, KV, true, true><<<gv.grid, kBlock, 0, s>>>(
                  F.n, k / VW, F.S.sptr, F.S.col, vals<TV>(F), minv<TV>(F), R0, z, Z0,
                  B.partials, stop);
            else
              kb_post_v<TV, double, double, KV, true, false><<<gv.grid, kBlock, 0, s>>>(
                  F.n, k / VW, F.S.sptr, F.S.col, vals<TV>(F), minv<TV>(F), R0, z, Z0,
                  B.partials, stop);
            np = (int32_t)gv.grid.x;
          });
          bfinalize(h, rz_op, np, maxit, stop);
        } else {
          kb_post<TV, double, double, KT, true><<<tgrid(g, k, KT), kBlock, 0, s>>>(
              F.n, k, F.S.sptr, F.S.col, vals<TV>(F), minv<TV>(F), R0, z, Z0, B.partials,
              stop);
          bfinalize(h, rz_op, (int32_t)g.grid.x, maxit, stop);
        }
      } else {
        kb_post<TV, double, double, KT, false><<<tgrid(g, k, KT), kBlock, 0, s>>>(
            F.n, k, F.S.sptr, F.S.col, vals<TV>(F), minv<TV>(F), R0, z, Z0, nullptr,
            stop);
      }
    }
  }
}

// Launches the vector form of the block SpMV when k and the blocks allow it;
// returns the number of partial rows it wrote, or 0 if it did not launch.
int32_t spmv_vec(amg_hierarchy *h, const double *Xin, const double *Bv, double *Out,
                 float *OutF, int32_t mode, const int32_t *stop) {
  Batch &B = *h->batch;
  Level &L0 = h->lv[0];
  const int32_t n = L0.n, k = B.k;
  if (k % 2 != 0 || !aligned16(Xin) || (Bv && !aligned16(Bv)) || (Out && !aligned16(Out)) ||
      (OutF && reinterpret_cast<uintptr_t>(OutF) % 8 != 0))
    return 0;
  int32_t nparts = 0;
  with_vec_tile(B, k / 2, [&](auto kt) {
    constexpr int KV = decltype(kt)::value;
    const BGeom g = bgeom(n, k / 2, KV);
    // level 0's exact FP32 copy of A when there is one: same numbers, half the bytes
    // with every lane of a row active, the row's index and value loads are
    // shuffled from eight lanes
    const bool shf = (k / 2) % KV == 0;
    if (L0.S.exact32 && shf)
      kb_spmv_v<KV, float, true><<<g.grid, kBlock, 0, h->stream>>>(
          n, k / 2, L0.S.sptr, L0.S.col, L0.S.v32, Xin, Bv, Out, OutF, B.partials, mode, stop);
    else if (L0.S.exact32)
      kb_spmv_v<KV, float, false><<<g.grid, kBlock, 0, h->stream>>>(
          n, k / 2, L0.S.sptr, L0.S.col, L0.S.v32, Xin, Bv, Out, OutF, B.partials, mode, stop);
    else if (shf)
      kb_spmv_v<KV, double, true><<<g.grid, kBlock, 0, h->stream>>>(
          n, k / 2, L0.S.sptr, L0.S.col, L0.S.v64, Xin, Bv, Out, OutF, B.partials, mode, stop);
    else
      kb_spmv_v<KV, double, false><<<g.grid, kBlock, 0, h->stream>>>(
          n, k / 2, L0.S.sptr, L0.S.col, L0.S.v64, Xin, Bv, Out, OutF, B.partials, mode, stop);
    nparts = (int32_t)g.grid.x;
  });
  return nparts;
}

template <int KU>
int32_t launch_update(amg_hierarchy *h, const int32_t *stop) {
  Batch &B = *h->batch;
  const int32_t n = h->lv[0].n, k = B.k;
  const BGeom g = bgeom(n, k, KU);
  kb_update<KU><<<g.grid, kBlock, 0, h->stream>>>(n, k, B.X, B.R, B.Rf, B.P, B.Q, B.col,
                                                  B.done, B.partials, stop);
  return (int32_t)g.grid.x;
}

// whether the CG update and p = z + beta p take their two-column forms
// (x += alpha p then moves into the latter)
bool vec_cg(const Batch &B) {
  return B.k % 2 == 0 && aligned16(B.X) && aligned16(B.R) && aligned16(B.P) &&
         aligned16(B.Q) && aligned16(B.Z) &&
         (!B.Rf || reinterpret_cast<uintptr_t>(B.Rf) % 8 == 0);
}

int32_t cg_update(amg_hierarchy *h, const int32_t *stop) {
  Batch &B = *h->batch;
  const int32_t n = h->lv[0].n, k = B.k;
  int32_t nparts = 0;
  if (vec_cg(B)) {
    with_vec_tile(B, k / 2, [&](auto kt) {
      constexpr int KU = decltype(kt)::value;
      const BGeom g = bgeom(n, k / 2, KU);
      kb_update_v<KU><<<g.grid, kBlock, 0, h->stream>>>(n, k / 2, B.R, B.Rf, B.Q, B.col,
                                                        B.done, B.partials, stop);
      nparts = (int32_t)g.grid.x;
    });
  } else {
    with_row_tile(k, [&](auto kt) { nparts = launch_update<decltype(kt)::value>(h, stop); });
  }
  return nparts;
}

template <typename TV, int KT>
void iteration_b(amg_hierarchy *h, int32_t maxit) {
  hipStream_t s = h->stream;
  Batch &B = *h->batch;
  const int32_t k = B.k;
  Level &L0 = h->lv[0];
  const int32_t n = L0.n;
  const int32_t *stop = B.all_done;
  const BGeom g = bgeom(n, k, KT);
  int32_t np = spmv_vec(h, B.P, nullptr, B.Q, nullptr, 0, stop);
  if (np == 0) {
    kb_spmv<KT><<<tgrid(g, k, KT), kBlock, 0, s>>>(n, k, L0.S.sptr, L0.S.col, L0.S.v64, B.P,
                                          nullptr, B.Q, nullptr, B.partials, 0, stop);
    np = (int32_t)g.grid.x;
  }
  bfinalize(h, bPq, np, maxit, stop);
  bfinalize(h, bRr, cg_update(h, stop), maxit, stop);
  kb_all_done<<<1, 64, 0, s>>>(k, B.done, B.all_done);
  vcycle_b<TV, KT>(h, B.R, B.Z, bRz, maxit, stop);
  if (z32(h))
    with_vec_tile(B, k / 2, [&](auto kt) {
      constexpr int KE = decltype(kt)::value;
      kb_xpay_v<KE, float><<<egrid(n, k / 2, KE), kBlock, 0, s>>>(n, k / 2, B.Zf, B.P, B.X,
                                                                   B.col, B.done, B.xpend);
    });
  else if (vec_cg(B))
    with_vec_tile(B, k / 2, [&](auto kt) {
      constexpr int KE = decltype(kt)::value;
      kb_xpay_v<KE, double><<<egrid(n, k / 2, KE), kBlock, 0, s>>>(n, k / 2, B.Z, B.P, B.X,
                                                                    B.col, B.done, B.xpend);
    });
  else
    with_row_tile(k, [&](auto kt) {
      constexpr int KE = decltype(kt)::value;
      kb_xpay<KE><<<egrid(n, k, KE), kBlock, 0, s>>>(n, k, B.Z, B.P, B.col, B.done, 0, stop);
    });
}

template <typename TV>
void dispatch_iteration(amg_hierarchy *h, int32_t maxit) {
  switch (h->batch->kt) {
    case 4: iteration_b<TV, 4>(h, maxit); break;
    case 8: iteration_b<TV, 8>(h, maxit); break;
    case 16: iteration_b<TV, 16>(h, maxit); break;
    case 32: iteration_b<TV, 32>(h, maxit); break;
    default: iteration_b<TV, 64>(h, maxit); break;
  }
}

template <typename TV>
void dispatch_vcycle(amg_hierarchy *h, const double *R, double *Z, int32_t rz_op, int32_t maxit,
                     const int32_t *stop) {
  switch (h->batch->kt) {
    case 4: vcycle_b<TV, 4>(h, R, Z, rz_op, maxit, stop); break;
    case 8: vcycle_b<TV, 8>(h, R, Z, rz_op, maxit, stop); break;
    case 16: vcycle_b<TV, 16>(h, R, Z, rz_op, maxit, stop); break;
    case 32: vcycle_b<TV, 32>(h, R, Z, rz_op, maxit, stop); break;
    default: vcycle_b<TV, 64>(h, R, Z, rz_op, maxit, stop); break;
  }
}

template <int KT>
void launch_spmv_mode(amg_hierarchy *h, const double *Xin, const double *Bv, double *Out,
                      int32_t mode, int32_t *nparts) {
  Batch &B = *h->batch;
  Level &L0 = h->lv[0];
  const BGeom g = bgeom(L0.n, B.k, KT);
  kb_spmv<KT><<<tgrid(g, B.k, KT), kBlock, 0, h->stream>>>(L0.n, B.k, L0.S.sptr, L0.S.col,
                                                L0.S.v64, Xin, Bv, Out,
                                                mode == 1 && Out == B.R ? B.Rf : nullptr,
                                                B.partials, mode, nullptr);
  *nparts = (int32_t)g.grid.x;
}

void spmv_mode(amg_hierarchy *h, const double *Xin, const double *Bv, double *Out, int32_t mode,
               int32_t *nparts) {
  Batch &B = *h->batch;
  *nparts = spmv_vec(h, Xin, Bv, Out, mode == 1 && Out == B.R ? B.Rf : nullptr, mode, nullptr);
  if (*nparts) return;
  switch (h->batch->kt) {
    case 4: launch_spmv_mode<4>(h, Xin, Bv, Out, mode, nparts); break;
    case 8: launch_spmv_mode<8>(h, Xin, Bv, Out, mode, nparts); break;
    case 16: launch_spmv_mode<16>(h, Xin, Bv, Out, mode, nparts); break;
    case 32: launch_spmv_mode<32>(h, Xin, Bv, Out, mode, nparts); break;
    default: launch_spmv_mode<64>(h, Xin, Bv, Out, mode, nparts); break;
  }
}

template <int KT>
void launch_small(amg_hierarchy *h, int32_t which) {
  Batch &B = *h->batch;
  const int32_t n = h->lv[0].n;
  if (which == 0)
    kb_zero_cols<KT><<<egrid(n, B.k, KT), kBlock, 0, h->stream>>>(n, B.k, B.X, B.done);
  else if (z32(h))
    kb_xpay<KT, float><<<egrid(n, B.k, KT), kBlock, 0, h->stream>>>(n, B.k, B.Zf, B.P, B.col,
                                                                   B.done, 1, B.all_done);
  else
    kb_xpay<KT><<<egrid(n, B.k, KT), kBlock, 0, h->stream>>>(n, B.k, B.Z, B.P, B.col, B.done, 1,
                                                            B.all_done);
}

void small_kernel(amg_hierarchy *h, int32_t which) {
  switch (h->batch->kt) {
    case 4: launch_small<4>(h, which); break;
    case 8: launch_small<8>(h, which); break;
    case 16: launch_small<16>(h, which); break;
    case 32: launch_small<32>(h, which); break;
    default: launch_small<64>(h, which); break;
  }
}

amg_status balloc(amg_hierarchy *h, void **p, size_t bytes) {
  Batch &B = *h->batch;
  AMG_TRY(stream_alloc(h->device, h->stream, p, bytes + 16));
  B.allocs.push_back(*p);
  B.bytes += bytes + 16;
  return AMG_OK;
}

// Allocates every buffer of a batch of k columns into h->batch (whose k is
// still 0: a batch is marked usable only once all of them exist).
amg_status alloc_batch(amg_hierarchy *h, int32_t k) {
  Batch &B = *h->batch;
  const bool fp32 = h->params.precision == AMG_FP32;
  const size_t V = fp32 ? 4 : 8;
  const int32_t nlev = (int32_t)h->lv.size();
  B.r.resize(nlev);
  B.z.resize(nlev);
  B.t.resize(nlev);
  B.y.resize(nlev);
  for (int32_t l = 0; l < nlev; ++l) {
    const size_t e = (size_t)h->lv[l].n * k * V;
    AMG_TRY(balloc(h, &B.r[l], e));
    AMG_TRY(balloc(h, &B.z[l], e));
    AMG_TRY(balloc(h, &B.t[l], e));
    AMG_TRY(balloc(h, &B.y[l], e));
  }
  const size_t e0 = (size_t)h->lv[0].n * k * sizeof(double);
  AMG_TRY(balloc(h, (void **)&B.X, e0));
  AMG_TRY(balloc(h, (void **)&B.Bp, e0));
  AMG_TRY(balloc(h, (void **)&B.R, e0));
  AMG_TRY(balloc(h, (void **)&B.Z, e0));
  AMG_TRY(balloc(h, (void **)&B.P, e0));
  AMG_TRY(balloc(h, (void **)&B.Q, e0));
  if (fp32) AMG_TRY(balloc(h, (void **)&B.Rf, (size_t)h->lv[0].n * k * sizeof(float)));
  if (fp32 && k % 4 == 0 && h->lv.size() > 1)
    AMG_TRY(balloc(h, (void **)&B.Zf, (size_t)h->lv[0].n * k * sizeof(float)));
  AMG_TRY(balloc(h, (void **)&B.partials, sizeof(double) * 2 * kBatchBlocks * (size_t)k));
  AMG_TRY(balloc(h, (void **)&B.col, sizeof(double) * kColFields * (size_t)k));
  AMG_TRY(balloc(h, (void **)&B.iter, sizeof(int32_t) * (size_t)k));
  AMG_TRY(balloc(h, (void **)&B.done, sizeof(int32_t) * (size_t)k));
  AMG_TRY(balloc(h, (void **)&B.xpend, sizeof(int32_t) * (size_t)k));
  AMG_TRY(balloc(h, (void **)&B.all_done, sizeof(int32_t) * 4));
  AMG_HIP(hipHostMalloc((void **)&B.col_host, sizeof(double) * kColFields * (size_t)k));
  AMG_HIP(hipHostMalloc((void **)&B.iter_host, sizeof(int32_t) * (size_t)k));
  AMG_HIP(hipHostMalloc((void **)&B.done_host, sizeof(int32_t) * (size_t)k));
  AMG_HIP(hipMemsetAsync(B.all_done, 0, sizeof(int32_t) * 4, h->stream));
  return AMG_OK;
}

// The batch state for k columns, reallocated when k changes. On any failure
// the partial batch is released and h->batch left null, so a later call
// allocates afresh instead of launching on missing buffers.
amg_status ensure_batch(amg_hierarchy *h, int32_t k) {
  if (h->batch && h->batch->k == k) return AMG_OK;
  if (h->batch) {
    free_batch(h->batch, h->device, h->stream);
    h->batch = nullptr;
    h->batch_bytes = 0;
  }
  h->batch = new (std::nothrow) Batch();
  if (!h->batch) return AMG_ERR_OOM;
  const amg_status st = alloc_batch(h, k);
  if (st != AMG_OK) {
    free_batch(h->batch, h->device, h->stream);
    h->batch = nullptr;
    h->batch_bytes = 0;
    return st;
  }
  h->batch->k = k;
  h->batch_bytes = h->batch->bytes;
  return AMG_OK;
}

__global__ void kb_fill_f64(double *p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Autotuner: the block CG iteration as the solve runs it (direct launches),
// timed for every candidate pair of the one-value kernels' column tile kt
// and the vector kernels' tile shift, so that the choice is made on the
// kernels that run. The state is synthetic but valid (X = 0, right-hand
// sides of ones, then the solve's own prologue, rtol 0), so every kernel
// does its full work; the solve's prologue overwrites it afterwards. The
// tiles set how rows are dealt to blocks and hence the order in which each
// column's dot products are summed: the choice is kept for the hierarchy
// and k, so later solves repeat the same sums.
template <typename TV>
amg_status autotune(amg_hierarchy *h) {
  Batch &B = *h->batch;
  hipStream_t s = h->stream;
  const int32_t n = h->lv[0].n, k = B.k;
  const int64_t nk = (int64_t)n * k;
  kb_fill_f64<<<ceil_div(nk, kBlock), kBlock, 0, s>>>(B.X, nk, 0.0);
  kb_fill_f64<<<ceil_div(nk, kBlock), kBlock, 0, s>>>(B.Bp, nk, 1.0);
  B.kt = 16;
  B.vshift = 0;
  kb_init_cols<<<ceil_div(k, 64), 64, 0, s>>>(k, 0.0, INT32_MAX, B.col, B.iter, B.done,
                                              B.xpend, B.all_done);
  int32_t np = 0;
  spmv_mode(h, B.X, B.Bp, B.R, 1, &np);
  bfinalize(h, bInit, np, INT32_MAX, nullptr);
  kb_all_done<<<1, 64, 0, s>>>(k, B.done, B.all_done);
  dispatch_vcycle<TV>(h, B.R, B.Z, bRz0, INT32_MAX, B.all_done);
  small_kernel(h, 1);  // P = Z
  AMG_HIP(hipGetLastError());
  hipEvent_t e0, e1;
  AMG_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return AMG_ERR_HIP;
  }
  const int cands[5] = {4, 8, 16, 32, 64};
  const int shifts[3] = {0, -1, 1};
  const int nshift = k % 2 == 0 ? 3 : 1;  // vector kernels run only for even k
  float best = 0.f;
  int best_kt = 16, best_vs = 0;
  bool first = true;
  amg_status st = AMG_OK;
  for (int c : cands) {
    if (c > 4 && c / 2 >= k) break;  // wider tiles would only add idle lanes
    for (int q = 0; q < nshift && st == AMG_OK; ++q) {
      B.kt = c;
      B.vshift = shifts[q];
      dispatch_iteration<TV>(h, INT32_MAX);  // warm
      float t = 0.f;
      if (hipEventRecord(e0, s) != hipSuccess) st = AMG_ERR_HIP;
      for (int r = 0; r < 2 && st == AMG_OK; ++r) dispatch_iteration<TV>(h, INT32_MAX);
      if (st == AMG_OK &&
          (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
           hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        st = AMG_ERR_HIP;
      if (st == AMG_OK && (first || t < best)) {
        best = t;
        best_kt = c;
        best_vs = shifts[q];
        first = false;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  B.kt = best_kt;
  B.vshift = best_vs;
  if (st != AMG_OK) {
    (void)hipGetLastError();
    return st;
  }
  AMG_HIP(hipGetLastError());
  return AMG_OK;
}

}  // namespace

void free_batch(Batch *b, int device, hipStream_t s) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (void *p : b->allocs) stream_free(device, s, p);
  if (b->col_host) (void)hipHostFree(b->col_host);
  if (b->iter_host) (void)hipHostFree(b->iter_host);
  if (b->done_host) (void)hipHostFree(b->done_host);
  delete b;
}

amg_status batch_kt(const amg_hierarchy *h, int32_t *kt, int32_t *vshift) {
  *kt = h->batch ? h->batch->kt : 0;
  if (vshift) *vshift = h->batch ? h->batch->vshift : 0;
  return AMG_OK;
}

amg_status pcg_batch(amg_hierarchy *h, int32_t k, const double *Bu, double *Xu, double rtol,
                     int32_t maxit, amg_solve_info *info) {
  const double t0 = now_ms();
  hipStream_t s = h->stream;
  const bool fp32 = h->params.precision == AMG_FP32;
  const int32_t n = h->lv[0].n;
  AMG_TRY(ensure_batch(h, k));
  Batch &B = *h->batch;
  if (B.kt == 0) {
    if (fp32) AMG_TRY(autotune<float>(h));
    else AMG_TRY(autotune<double>(h));
  }
  // capture one iteration (all kernels read their scalars from device memory)
  if (!B.exec && !(h->params.flags & AMG_FLAG_NO_GRAPH)) {
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      if (fp32) dispatch_iteration<float>(h, INT32_MAX);
      else dispatch_iteration<double>(h, INT32_MAX);
      if (hipStreamEndCapture(s, &g) == hipSuccess && g &&
          hipGraphInstantiate(&B.exec, g, nullptr, nullptr, 0) == hipSuccess) {
        B.graph = g;
      } else {
        if (g) (void)hipGraphDestroy(g);
        B.exec = nullptr;
      }
    }
    (void)hipGetLastError();
  }
  const int32_t *perm0 = h->lv[0].perm;
  const int32_t pgrid = ceil_div((int64_t)n * k, kBlock);
  kb_permute_rows<true><<<pgrid, kBlock, 0, s>>>(n, k, perm0, Xu, B.X);
  kb_permute_rows<true><<<pgrid, kBlock, 0, s>>>(n, k, perm0, Bu, B.Bp);
  kb_init_cols<<<ceil_div(k, 64), 64, 0, s>>>(k, rtol, maxit, B.col, B.iter, B.done, B.xpend,
                                              B.all_done);
  int32_t np = 0;
  spmv_mode(h, B.X, B.Bp, B.R, 1, &np);
  bfinalize(h, bInit, np, maxit, nullptr);
  small_kernel(h, 0);  // zero the columns of zero right-hand sides
  kb_all_done<<<1, 64, 0, s>>>(k, B.done, B.all_done);
  if (fp32) dispatch_vcycle<float>(h, B.R, B.Z, bRz0, maxit, B.all_done);
  else dispatch_vcycle<double>(h, B.R, B.Z, bRz0, maxit, B.all_done);
  small_kernel(h, 1);  // P = Z
  // iterations: the graph's finalize kernels test maxit = INT32_MAX, so the
  // per-column maxit is enforced here by the number of iterations queued
  int32_t queued = 0, chunk = 4;
  for (;;) {
    AMG_HIP(hipMemcpyAsync(B.done_host, B.done, sizeof(int32_t) * k, hipMemcpyDeviceToHost, s));
    AMG_HIP(hipMemcpyAsync(B.col_host, B.col, sizeof(double) * kColFields * k,
                           hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    bool all = true;
    double worst = 0.0;
    for (int32_t j = 0; j < k; ++j) {
      if (B.done_host[j]) continue;
      all = false;
      const double rr = B.col_host[cRr * k + j], bb = B.col_host[cBb * k + j];
      const double ratio = bb > 0 ? rr / (rtol * rtol * bb) : 0.0;
      worst = ratio > worst ? ratio : worst;
    }
    if (all || queued >= maxit) break;
    // about 0.25 orders of magnitude of residual per iteration for this
    // preconditioner; queue up to the predicted remainder, at most 16
    int32_t need = worst > 1.0 ? (int32_t)std::ceil(0.5 * std::log10(worst) / 0.25) : 1;
    chunk = need < 1 ? 1 : (need > 16 ? 16 : need);
    const int32_t c = std::min(chunk, maxit - queued);
    for (int32_t it = 0; it < c; ++it) {
      if (B.exec) {
        AMG_HIP(hipGraphLaunch(B.exec, s));
      } else if (fp32) {
        dispatch_iteration<float>(h, INT32_MAX);
      } else {
        dispatch_iteration<double>(h, INT32_MAX);
      }
    }
    AMG_HIP(hipGetLastError());
    queued += c;
  }
  // columns still running at maxit
  AMG_HIP(hipMemcpyAsync(B.iter_host, B.iter, sizeof(int32_t) * k, hipMemcpyDeviceToHost, s));
  spmv_mode(h, B.X, B.Bp, nullptr, 2, &np);
  bfinalize(h, bTrue, np, maxit, nullptr);
  kb_permute_rows<false><<<pgrid, kBlock, 0, s>>>(n, k, perm0, B.X, Xu);
  AMG_HIP(hipMemcpyAsync(B.col_host, B.col, sizeof(double) * kColFields * k,
                         hipMemcpyDeviceToHost, s));
  AMG_HIP(hipMemcpyAsync(B.done_host, B.done, sizeof(int32_t) * k, hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  const double ms = now_ms() - t0;
  amg_status st = AMG_OK;
  for (int32_t j = 0; j < k; ++j) {
    const int32_t d = B.done_host[j];
    if (d == 3) st = AMG_ERR_BREAKDOWN;
    else if ((d == 0 || d == 2) && st == AMG_OK) st = AMG_NOT_CONVERGED;
    if (info) {
      const double bb = B.col_host[cBb * k + j];
      info[j].iterations = B.iter_host[j];
      info[j].converged = (d == 1 || d == 4) ? 1 : 0;
      info[j].rel_res_recursive = bb > 0 ? std::sqrt(B.col_host[cRr * k + j] / bb) : 0.0;
      info[j].rel_res_true = bb > 0 ? std::sqrt(B.col_host[cRrTrue * k + j] / bb) : 0.0;
      info[j].ms = ms;
    }
  }
  return st;
}

}  // namespace amg
