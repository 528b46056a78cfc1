// Hierarchy construction on the GPU: coupled aggregation based on compatible
// weighted matching (Section 3.2) and Galerkin coarse operators (Section 3.1).
//
// Built with -ffp-contract=off: weights, prolongator values, Galerkin sums
// and restricted smooth vectors round exactly as written, so the hierarchy is
// bit-for-bit reproducible and equal to the FP64 reference computation.
//
// Per level l (until n_l <= max_coarse):
//   for each of `sweeps` pairwise sweeps on (A_k, w_k):
//     1. edge weights, eq. (weights), one value per stored entry
//     2. matching: rounds of locally-dominant proposals under the strict key
//        (weight desc, lo asc, hi asc) -- the half-approximate
//        maximum-weight matching class of the paper; under a strict key it
//        equals the greedy matching
//     3. aggregate numbering by smallest member (prefix scan)
//     4. pairwise prolongator, eq. (prolongator)
//     5. A_{k+1} = P_k^T A_k P_k, w_{k+1} = P_k^T w_k
//   P_l = P_1 P_2 ... P_m (composed per fine row), A_{l+1} = A_{k=m}.
// Then the l1-Jacobi diagonal (Section 3.3) and, on the coarsest level, a
// dense Cholesky factor and its triangular inverse.

#include <chrono>
#include <cmath>

#include "internal.h"

namespace amg {

namespace {

constexpr int32_t kFree = -2;
constexpr int32_t kDead = -1;
constexpr int kRapCap = 48;     // per-thread Galerkin row buffer
constexpr int kRapLongCap = 2048;  // per-block buffer for long rows
constexpr int kScanBlock = 1024;
constexpr int kScanPer = 4;

enum : int32_t { kErrArg = 1, kErrSpd = 2, kErrSym = 4 };

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// ---------------------------------------------------------------------------
// exclusive prefix sum (three passes)
// ---------------------------------------------------------------------------

__device__ int32_t block_exclusive_scan(int32_t v, int32_t *total) {
  __shared__ int32_t wsum[kScanBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  int32_t x = v;
  for (int o = 1; o < kWave; o <<= 1) {
    int32_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) wsum[wid] = x;
  __syncthreads();
  if (wid == 0) {
    int32_t s = lane < kScanBlock / kWave ? wsum[lane] : 0;
    for (int o = 1; o < kWave; o <<= 1) {
      int32_t y = __shfl_up(s, o, kWave);
      if (lane >= o) s += y;
    }
    if (lane < kScanBlock / kWave) wsum[lane] = s;
  }
  __syncthreads();
  int32_t off = wid > 0 ? wsum[wid - 1] : 0;
  *total = wsum[kScanBlock / kWave - 1];
  __syncthreads();
  return off + x - v;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_local(const int32_t *in, int32_t *out,
                                                           int32_t *bsum, int32_t n) {
  const int64_t base = ((int64_t)blockIdx.x * kScanBlock + threadIdx.x) * kScanPer;
  int32_t v[kScanPer];
  int32_t s = 0;
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = base + k < n ? in[base + k] : 0;
    s += v[k];
  }
  int32_t total;
  int32_t off = block_exclusive_scan(s, &total);
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < n) out[base + k] = off;
    off += v[k];
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_sums(int32_t *bsum, int32_t nb) {
  int32_t carry = 0;
  for (int32_t c0 = 0; c0 < nb; c0 += kScanBlock * kScanPer) {
    const int32_t base = c0 + threadIdx.x * kScanPer;
    int32_t v[kScanPer];
    int32_t s = 0;
    for (int k = 0; k < kScanPer; ++k) {
      v[k] = base + k < nb ? bsum[base + k] : 0;
      s += v[k];
    }
    int32_t total;
    int32_t off = block_exclusive_scan(s, &total);
    for (int k = 0; k < kScanPer; ++k) {
      if (base + k < nb) bsum[base + k] = carry + off;
      off += v[k];
    }
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ void k_scan_add(int32_t *out, const int32_t *bsum, int32_t n, int32_t nb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += bsum[i / (kScanBlock * kScanPer)];
  if (i == 0) out[n] = bsum[nb];
}

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_fill(T *a, T v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_iota(int32_t *a, int32_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n) a[i] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// input validation: structure, positive diagonal, bitwise symmetry
// ---------------------------------------------------------------------------

__device__ __forceinline__ int64_t find_col(const int32_t *ci, int64_t b, int64_t e, int32_t j) {
  int64_t lo = b, hi = e - 1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    int32_t c = ci[mid];
    if (c == j) return mid;
    if (c < j) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

__global__ void k_validate(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                           const double *val, int32_t *err) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (i == 0 && rp[0] != 0) atomicOr(err, kErrArg);
  if (i == n - 1 && (int64_t)rp[n] != nnz) atomicOr(err, kErrArg);
  const int64_t b = rp[i], e = rp[i + 1];
  if (b < 0 || e < b || e > nnz) {
    atomicOr(err, kErrArg);
    return;
  }
  bool diag = false;
  int32_t flags = 0;
  for (int64_t k = b; k < e; ++k) {
    const int32_t j = ci[k];
    const double a = val[k];
    if (j < 0 || j >= n || (k > b && j <= ci[k - 1]) || !isfinite(a)) {
      flags |= kErrArg;
      break;
    }
    if (j == i) {
      diag = true;
      if (!(a > 0.0)) flags |= kErrSpd;
      continue;
    }
    const int64_t bj = rp[j], ej = rp[j + 1];
    if (bj < 0 || ej < bj || ej > nnz) {
      flags |= kErrArg;
      break;
    }
    const int64_t t = find_col(ci, bj, ej, i);
    if (t < 0 || __double_as_longlong(val[t]) != __double_as_longlong(a)) flags |= kErrSym;
  }
  if (!diag) flags |= kErrSpd;
  if (flags) atomicOr(err, flags);
}

__global__ void k_check_w(int32_t n, const double *w, int32_t *err) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(w[i] != 0.0 && isfinite(w[i]))) atomicOr(err, kErrArg);
}

// One sweep of the smoother on A w = 0: w_out = w - (A w) / m (row sums
// left to right from the first term, as the serial definition)
__global__ void k_smooth_w(int32_t n, const int32_t *rp, const int32_t *ci, const double *val,
                           const double *m, const double *w, double *w_out) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t b = rp[i], e = rp[i + 1];
  double t = 0.0;
  if (e > b) {
    t = val[b] * w[ci[b]];
    for (int32_t k = b + 1; k < e; ++k) t = t + val[k] * w[ci[k]];
  }
  w_out[i] = w[i] - t / m[i];
}

// position of the diagonal entry of each row
__global__ void k_diag_pos(int32_t n, const int32_t *rp, const int32_t *ci, int32_t *dpos) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  dpos[i] = (int32_t)find_col(ci, rp[i], rp[i + 1], i);
}

// ---------------------------------------------------------------------------
// 1. eq. (weights)
// ---------------------------------------------------------------------------

// c = 1 - ((2 a) w_lo w_hi) / ((a_lolo w_lo) w_lo + (a_hihi w_hi) w_hi) for
// each stored off-diagonal entry, computed in (lo, hi) order so that both
// copies of an edge carry the same bits (A is bitwise symmetric).
__global__ void k_weights(int32_t n, const int32_t *rp, const int32_t *ci, const double *val,
                          const int32_t *dpos, const double *w, double *c) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
    const int32_t j = ci[k];
    if (j == i) {
      c[k] = 0.0;
      continue;
    }
    const int32_t lo = min(i, j), hi = max(i, j);
    const double a = val[k];
    const double wl = w[lo], wh = w[hi];
    const double num = ((2.0 * a) * wl) * wh;
    const double den = (val[dpos[lo]] * wl) * wl + (val[dpos[hi]] * wh) * wh;
    c[k] = 1.0 - num / den;
  }
}

// ---------------------------------------------------------------------------
// 2. matching: locally-dominant rounds
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool better(double c1, int32_t lo1, int32_t hi1, double c2,
                                       int32_t lo2, int32_t hi2) {
  if (c1 != c2) return c1 > c2;
  if (lo1 != lo2) return lo1 < lo2;
  return hi1 < hi2;
}

// The best neighbour of v (entries [b, e) of its row) under the strict key
// among those not taken: mate[j] != kFree, or (with cur) a mutual proposal
// in cur. The loads go in batches of eight entries (all indices and weights,
// then all mate and cur entries, then the proposals' proposals), so that a
// vertex's chain of dependent loads does not grow with its degree; the
// comparisons run in entry order. -1: every neighbour is taken.
__device__ __forceinline__ int32_t best_free(int32_t v, int32_t b, int32_t e,
                                             const int32_t *__restrict__ ci,
                                             const double *__restrict__ c,
                                             const int32_t *mate, const int32_t *cur) {
  int32_t best = -1, blo = 0, bhi = 0;
  double bc = 0.0;
  for (int32_t k0 = b; k0 < e; k0 += 8) {
    int32_t j[8];
    double cc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool in = k0 + u < e;
      j[u] = in ? ci[k0 + u] : v;
      cc[u] = in ? c[k0 + u] : 0.0;
    }
    int32_t m[8], cj[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      m[u] = mate[j[u]];
      cj[u] = cur ? cur[j[u]] : -1;
    }
    int32_t back[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) back[u] = cj[u] >= 0 ? cur[cj[u]] : -1;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (k0 + u >= e || j[u] == v) continue;
      if (m[u] != kFree || (cj[u] >= 0 && back[u] == j[u])) continue;
      const int32_t lo = min(v, j[u]), hi = max(v, j[u]);
      if (best < 0 || better(cc[u], lo, hi, bc, blo, bhi)) {
        best = j[u];
        bc = cc[u];
        blo = lo;
        bhi = hi;
      }
    }
  }
  return best;
}

// For every free vertex: keep its proposal if the proposed vertex is still
// free (the free set only shrinks, so it is still the best), else propose to
// the best free neighbour under the strict key; a free vertex with no free
// neighbour becomes a singleton. Flags the round if any vertex still proposes.
__global__ void k_match_propose(int32_t n, const int32_t *rp, const int32_t *ci,
                                const double *c, int32_t *mate, int32_t *cand,
                                int32_t *active) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  bool live = false;
  if (v < n && mate[v] == kFree) {
    const int32_t u = cand[v];
    if (u >= 0 && mate[u] == kFree) {
      live = true;
    } else {
      const int32_t best = best_free(v, rp[v], rp[v + 1], ci, c, mate, nullptr);
      cand[v] = best;
      if (best < 0) mate[v] = kDead; else live = true;
    }
  }
  // one plain store per block that still has a proposing vertex (a per-wave
  // atomic on one counter serialises tens of thousands of waves per round)
  if (__syncthreads_or(live) && threadIdx.x == 0) *active = 1;
}

// Mutual proposals are locally dominant edges: match them.
__global__ void k_match_accept(int32_t n, int32_t *mate, const int32_t *cand) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || mate[v] != kFree) return;
  const int32_t u = cand[v];
  if (u >= 0 && cand[u] == v) mate[v] = u;
}

// One round: accept the mutual proposals of `cur` and, for vertices that stay
// free, write their next proposal into `nxt` (kept while its target stays
// free, else the best free neighbour under the strict key; none: singleton).
// x counts as taken in this round if it was matched or became a singleton
// before it (mate), or is matched in it (mutual proposals in `cur`, which
// nobody writes in this round). A stale read of mate[x] can only show a
// vertex that becomes a singleton in this round as free; a proposal to it is
// then repeated next round, while no free vertex is ever taken for matched.
// `prev` is the previous round's flag (null for the first round of a batch):
// once a round has no proposing vertex left, every free vertex has been
// matched or made a singleton, and the rounds queued after it return at once.
__global__ void k_match_round(int32_t n, const int32_t *rp, const int32_t *ci, const double *c,
                              int32_t *mate, const int32_t *cur, int32_t *nxt,
                              const int32_t *prev, int32_t *active) {
  if (prev && *prev == 0) return;
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  bool live = false;
  if (v < n && mate[v] == kFree) {
    // a free vertex's proposal and row bounds together, then the proposed
    // vertex's state and proposal, then that proposal's target
    const int32_t u = cur[v], b = rp[v], e = rp[v + 1];
    const int32_t cu = u >= 0 ? cur[u] : -1;
    const int32_t mu = u >= 0 ? mate[u] : kFree;
    const int32_t ccu = cu >= 0 ? cur[cu] : -1;
    if (u >= 0 && cu == v) {
      mate[v] = u;
      nxt[v] = u;
    } else if (u >= 0 && mu == kFree && !(cu >= 0 && ccu == u)) {
      nxt[v] = u;  // still free: still the best
      live = true;
    } else {
      const int32_t best = best_free(v, b, e, ci, c, mate, cur);
      nxt[v] = best;
      if (best < 0) mate[v] = kDead; else live = true;
    }
  }
  if (__syncthreads_or(live) && threadIdx.x == 0) *active = 1;
}

// ---------------------------------------------------------------------------
// 3. numbering, 4. eq. (prolongator), restriction of w
// ---------------------------------------------------------------------------

__global__ void k_leader(int32_t n, const int32_t *mate, int32_t *flag) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t m = mate[v];
  flag[v] = (m < 0 || v < m) ? 1 : 0;
}

__global__ void k_assign(int32_t n, const int32_t *mate, const int32_t *id, int32_t *agg,
                         int32_t *lead) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t m = mate[v];
  if (m < 0 || v < m) {
    agg[v] = id[v];
    lead[id[v]] = v;
  } else {
    agg[v] = id[m];
  }
}

// pair {i < j}: p_v = w_v / sqrt(w_i w_i + w_j w_j); singleton: w_s / |w_s|
__global__ void k_pair_prolongator(int32_t n, const int32_t *mate, const double *w, double *p) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t m = mate[v];
  if (m < 0) {
    p[v] = w[v] / fabs(w[v]);
  } else {
    const int32_t i = min(v, m), j = max(v, m);
    const double s = w[i] * w[i] + w[j] * w[j];
    p[v] = w[v] / sqrt(s);
  }
}

// w_{k+1}(I) = sum over members i of I, ascending, of p_i w_i
__global__ void k_restrict_pair(int32_t nc, const int32_t *lead, const int32_t *mate,
                                const double *p, const double *w, double *wc) {
  const int32_t I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int32_t i0 = lead[I], i1 = mate[i0];
  double s = p[i0] * w[i0];
  if (i1 >= 0) s = s + p[i1] * w[i1];
  wc[I] = s;
}

// ---------------------------------------------------------------------------
// 5. pairwise Galerkin product A_c = P^T A P
// ---------------------------------------------------------------------------
// Entry (I, J) sums (p_lo a_lo,hi) p_hi over the stored fine entries (i, j),
// i in I, j in J, mapped to (lo, hi) = (min, max) and taken in ascending
// (lo, hi) order, starting from the first term. Every structural entry is
// kept. Each coarse row is produced in a temporary slot, then compacted.

__global__ void k_rap_inlen(int32_t nc, const int32_t *lead, const int32_t *mate,
                            const int32_t *rp, int32_t *inlen) {
  const int32_t I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int32_t i0 = lead[I], i1 = mate[i0];
  int32_t len = rp[i0 + 1] - rp[i0];
  if (i1 >= 0) len += rp[i1 + 1] - rp[i1];
  inlen[I] = len;
}

__device__ __forceinline__ bool key_less(int32_t J1, int32_t lo1, int32_t hi1, int32_t J2,
                                         int32_t lo2, int32_t hi2) {
  if (J1 != J2) return J1 < J2;
  if (lo1 != lo2) return lo1 < lo2;
  return hi1 < hi2;
}

__global__ void k_rap_rows(int32_t nc, const int32_t *lead, const int32_t *mate,
                           const int32_t *rp, const int32_t *ci, const double *val,
                           const int32_t *agg, const double *p, const int32_t *toff,
                           int32_t *tJ, double *tV, int32_t *cnt, int32_t *ovf,
                           int32_t *novf) {
  const int32_t I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int32_t mem[2] = {lead[I], mate[lead[I]]};
  const int32_t len = toff[I + 1] - toff[I];
  if (len > kRapCap) {
    cnt[I] = 0;
    ovf[atomicAdd(novf, 1)] = I;
    return;
  }
  int32_t J[kRapCap], LO[kRapCap], HI[kRapCap];
  double T[kRapCap];
  int32_t m = 0;
  for (int q = 0; q < 2; ++q) {
    const int32_t f = mem[q];
    if (f < 0) continue;
    for (int32_t k = rp[f]; k < rp[f + 1]; ++k) {
      const int32_t j = ci[k];
      const int32_t lo = min(f, j), hi = max(f, j);
      const double t = (p[lo] * val[k]) * p[hi];
      // insertion into the sorted prefix
      int32_t pos = m;
      const int32_t Jj = agg[j];
      while (pos > 0 && key_less(Jj, lo, hi, J[pos - 1], LO[pos - 1], HI[pos - 1])) {
        J[pos] = J[pos - 1];
        LO[pos] = LO[pos - 1];
        HI[pos] = HI[pos - 1];
        T[pos] = T[pos - 1];
        --pos;
      }
      J[pos] = Jj;
      LO[pos] = lo;
      HI[pos] = hi;
      T[pos] = t;
      ++m;
    }
  }
  const int32_t base = toff[I];
  int32_t out = 0;
  double s = 0.0;
  for (int32_t e = 0; e < m; ++e) {
    if (e == 0 || J[e] != J[e - 1]) {
      if (e > 0) tV[base + out - 1] = s;
      tJ[base + out] = J[e];
      s = T[e];
      ++out;
    } else {
      s = s + T[e];
    }
  }
  if (out > 0) tV[base + out - 1] = s;
  cnt[I] = out;
}

// Rows whose two fine rows hold more than kRapCap entries: one block per row,
// entries ranked in LDS by the same key, then summed in order.
__global__ void __launch_bounds__(256) k_rap_long(
    const int32_t *lead, const int32_t *mate, const int32_t *rp, const int32_t *ci,
    const double *val, const int32_t *agg, const double *p, const int32_t *toff, int32_t *tJ,
    double *tV, int32_t *cnt, const int32_t *ovf, const int32_t *novf, int32_t *err) {
  __shared__ int32_t sJ[kRapLongCap], sLO[kRapLongCap], sHI[kRapLongCap];
  __shared__ double sT[kRapLongCap];
  __shared__ int16_t order[kRapLongCap];
  const int32_t count = *novf;
  for (int32_t o = blockIdx.x; o < count; o += gridDim.x) {
    const int32_t I = ovf[o];
    const int32_t i0 = lead[I], i1 = mate[i0];
    const int32_t l0 = rp[i0 + 1] - rp[i0];
    const int32_t len = toff[I + 1] - toff[I];
    if (len > kRapLongCap) {
      if (threadIdx.x == 0) {
        atomicOr(err, kErrArg);
        cnt[I] = 0;
      }
      continue;
    }
    for (int32_t e = threadIdx.x; e < len; e += blockDim.x) {
      const int32_t f = e < l0 ? i0 : i1;
      const int32_t k = e < l0 ? rp[i0] + e : rp[i1] + (e - l0);
      const int32_t j = ci[k];
      const int32_t lo = min(f, j), hi = max(f, j);
      sJ[e] = agg[j];
      sLO[e] = lo;
      sHI[e] = hi;
      sT[e] = (p[lo] * val[k]) * p[hi];
    }
    __syncthreads();
    for (int32_t e = threadIdx.x; e < len; e += blockDim.x) {
      int32_t rank = 0;
      for (int32_t f = 0; f < len; ++f) {
        const bool lt = key_less(sJ[f], sLO[f], sHI[f], sJ[e], sLO[e], sHI[e]);
        const bool eq = sJ[f] == sJ[e] && sLO[f] == sLO[e] && sHI[f] == sHI[e];
        rank += (lt || (eq && f < e)) ? 1 : 0;
      }
      order[rank] = (int16_t)e;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int32_t base = toff[I];
      int32_t out = 0;
      double s = 0.0;
      int32_t prevJ = -1;
      for (int32_t q = 0; q < len; ++q) {
        const int32_t e = order[q];
        if (q == 0 || sJ[e] != prevJ) {
          if (q > 0) tV[base + out - 1] = s;
          tJ[base + out] = sJ[e];
          s = sT[e];
          prevJ = sJ[e];
          ++out;
        } else {
          s = s + sT[e];
        }
      }
      if (out > 0) tV[base + out - 1] = s;
      cnt[I] = out;
    }
    __syncthreads();
  }
}

__global__ void k_rap_copy(int32_t nc, const int32_t *toff, const int32_t *tJ,
                           const double *tV, const int32_t *rpc, int32_t *cic,
                           double *valc) {
  const int32_t I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int32_t src = toff[I], dst = rpc[I], len = rpc[I + 1] - rpc[I];
  for (int32_t e = 0; e < len; ++e) {
    cic[dst + e] = tJ[src + e];
    valc[dst + e] = tV[src + e];
  }
}

// ---------------------------------------------------------------------------
// composition of sweeps and aggregate member lists
// ---------------------------------------------------------------------------

// P_l(i) = ((p_1(i) p_2(agg_1(i))) p_3(...)), agg_l = ... o agg_2 o agg_1
__global__ void k_compose(int32_t n, const int32_t *agg_k, const double *p_k, int32_t *agg_c,
                          double *p_c, int32_t first) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (first) {
    agg_c[i] = agg_k[i];
    p_c[i] = p_k[i];
  } else {
    const int32_t a = agg_c[i];
    p_c[i] = p_c[i] * p_k[a];
    agg_c[i] = agg_k[a];
  }
}

__global__ void k_member_size(int32_t nc, const int32_t *lead, const int32_t *mate,
                              const int32_t *mptr, int32_t *size) {
  const int32_t I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int32_t a = lead[I], b = mate[a];
  int32_t s = mptr[a + 1] - mptr[a];
  if (b >= 0) s += mptr[b + 1] - mptr[b];
  size[I] = s;
}

__global__ void k_member_merge(int32_t nc, const int32_t *lead, const int32_t *mate,
                               const int32_t *mptr, const int32_t *mem, const int32_t *mptr_n,
                               int32_t *mem_n) {
  const int32_t I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int32_t a = lead[I], b = mate[a];
  int32_t pa = mptr[a], ea = mptr[a + 1];
  int32_t pb = b >= 0 ? mptr[b] : 0, eb = b >= 0 ? mptr[b + 1] : 0;
  int32_t o = mptr_n[I];
  while (pa < ea || pb < eb) {
    if (pb >= eb || (pa < ea && mem[pa] < mem[pb])) mem_n[o++] = mem[pa++];
    else mem_n[o++] = mem[pb++];
  }
}

// ---------------------------------------------------------------------------
// l1-Jacobi diagonal, eq. (l1weights) with blocks of one row
// ---------------------------------------------------------------------------

__global__ void k_l1_diag(int32_t n, const int32_t *rp, const int32_t *ci, const double *val,
                          double *m, double *minv) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double aii = 0.0, s = 0.0;
  bool first = true;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
    if (ci[k] == i) {
      aii = val[k];
    } else if (first) {
      s = fabs(val[k]);
      first = false;
    } else {
      s = s + fabs(val[k]);
    }
  }
  const double mi = aii + s;
  m[i] = mi;
  minv[i] = 1.0 / mi;
}

// ---------------------------------------------------------------------------
// coarsest level: dense Cholesky A_L = L L^T and L^-1
// ---------------------------------------------------------------------------

__global__ void k_dense_scatter(int32_t n, const int32_t *rp, const int32_t *ci,
                                const double *val, double *D) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) D[(int64_t)i * n + ci[k]] = val[k];
}

// Right-looking Cholesky of a row-major n x n matrix in one workgroup; the
// lower triangle becomes L, the strict upper triangle is zeroed.
__global__ void __launch_bounds__(1024) k_cholesky(int32_t n, double *D, int32_t *err) {
  __shared__ int32_t bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int32_t k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      const double d = D[(int64_t)k * n + k];
      if (!(d > 0.0)) bad = 1;
      else D[(int64_t)k * n + k] = sqrt(d);
    }
    __syncthreads();
    if (bad) break;
    const double d = D[(int64_t)k * n + k];
    for (int32_t i = k + 1 + threadIdx.x; i < n; i += blockDim.x) D[(int64_t)i * n + k] /= d;
    __syncthreads();
    // trailing update of the lower triangle, threads in rows of 32 over (i, j)
    for (int32_t i = k + 1 + (int32_t)threadIdx.x / 32; i < n; i += (int32_t)blockDim.x / 32)
      for (int32_t j = k + 1 + (int32_t)threadIdx.x % 32; j <= i; j += 32)
        D[(int64_t)i * n + j] -= D[(int64_t)i * n + k] * D[(int64_t)j * n + k];
    __syncthreads();
  }
  if (bad) {
    if (threadIdx.x == 0) atomicOr(err, kErrSpd);
    return;
  }
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += blockDim.x) {
    const int32_t i = (int32_t)(e / n), j = (int32_t)(e % n);
    if (j > i) D[e] = 0.0;
  }
}

// k_cholesky on the packed lower triangle held in LDS (n (n + 1) / 2 doubles,
// up to 64 KB: n <= 127): the same steps on the same numbers, with every
// access of the n steps in LDS instead of L2.
constexpr int kCholLdsMax = 127;
static_assert(kCholLdsMax * (kCholLdsMax + 1) / 2 * sizeof(double) <= 65536, "LDS triangle");
__global__ void __launch_bounds__(1024) k_cholesky_lds(int32_t n, double *D, int32_t *err) {
  extern __shared__ double tri[];  // row i of the lower triangle at i (i + 1) / 2
  __shared__ int32_t bad;
  auto at = [&](int32_t i, int32_t j) -> double & { return tri[i * (i + 1) / 2 + j]; };
  for (int32_t e = threadIdx.x; e < n * (n + 1) / 2; e += blockDim.x) {
    int32_t i = (int32_t)((sqrt(8.0 * e + 1.0) - 1.0) / 2.0);
    while (i * (i + 1) / 2 > e) --i;
    while ((i + 1) * (i + 2) / 2 <= e) ++i;
    tri[e] = D[(int64_t)i * n + (e - i * (i + 1) / 2)];
  }
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int32_t k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      const double d = at(k, k);
      if (!(d > 0.0)) bad = 1;
      else at(k, k) = sqrt(d);
    }
    __syncthreads();
    if (bad) break;
    const double d = at(k, k);
    for (int32_t i = k + 1 + threadIdx.x; i < n; i += blockDim.x) at(i, k) /= d;
    __syncthreads();
    for (int32_t i = k + 1 + (int32_t)threadIdx.x / 32; i < n; i += (int32_t)blockDim.x / 32)
      for (int32_t j = k + 1 + (int32_t)threadIdx.x % 32; j <= i; j += 32)
        at(i, j) -= at(i, k) * at(j, k);
    __syncthreads();
  }
  if (bad) {
    if (threadIdx.x == 0) atomicOr(err, kErrSpd);
    return;
  }
  for (int32_t e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int32_t i = e / n, j = e % n;
    D[e] = j > i ? 0.0 : at(i, j);
  }
}

// X = L^-1, one block per column j: forward substitution of L x = e_j in its
// right-looking form. Once x_i = t_i / L_ii is known, every later row r takes
// off its term L_ri x_i, so each partial sum t_r loses its terms in the order
// k = j, j + 1, ..., r - 1 of the row-by-row substitution (the same numbers).
// t and the diagonal of L live in LDS; each thread owns the rows tid + s *
// kTriThreads and loads their entries of the next column of L while the
// current step runs, so a step waits on no memory access.
constexpr int kTriThreads = 256;
static_assert(AMG_MAX_DENSE % kTriThreads == 0, "whole rows per thread");
static_assert(2 * sizeof(double) * AMG_MAX_DENSE <= 65536, "t and the diagonal fit in LDS");
template <int S>  // rows per thread: S * kTriThreads >= n
__global__ void __launch_bounds__(kTriThreads) k_tri_inverse(int32_t n,
                                                             const double *__restrict__ L,
                                                             double *__restrict__ X) {
  extern __shared__ double tri_sh[];  // t[n], then the diagonal of L
  double *t = tri_sh, *dg = tri_sh + n;
  const int32_t j = blockIdx.x, tid = threadIdx.x;
  for (int32_t r = tid; r < n; r += kTriThreads) {
    t[r] = r == j ? 1.0 : 0.0;
    dg[r] = L[(int64_t)r * n + r];
    if (r < j) X[(int64_t)r * n + j] = 0.0;
  }
  double ln[S];  // this thread's rows' entries of column i of L
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const int32_t r = tid + q * kTriThreads;
    ln[q] = r > j && r < n ? L[(int64_t)r * n + j] : 0.0;
  }
  __syncthreads();
  for (int32_t i = j; i < n; ++i) {
    const double x = t[i] / dg[i];
    if (tid == 0) X[(int64_t)i * n + j] = x;
    double lc[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
      const int32_t r = tid + q * kTriThreads;
      lc[q] = ln[q];
      ln[q] = r > i + 1 && r < n ? L[(int64_t)r * n + i + 1] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < S; ++q) {
      const int32_t r = tid + q * kTriThreads;
      if (r > i && r < n) t[r] -= lc[q] * x;
    }
    __syncthreads();
  }
}

// A^-1 = L^-T L^-1: entry (i, j) sums X(k, i) X(k, j) over k >= max(i, j)
__global__ void k_inverse_from_factor(int32_t n, const double *X, double *Ainv) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int32_t i = (int32_t)(e / n), j = (int32_t)(e % n);
  double s = 0.0;
  for (int32_t k = max(i, j); k < n; ++k) s += X[(int64_t)k * n + i] * X[(int64_t)k * n + j];
  Ainv[e] = s;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

inline int32_t grid(int64_t n) { return ceil_div(n > 0 ? n : 1, kBlock); }

// block count of the exclusive scan of n values (its block sums take nb + 1)
int32_t scan_blocks(int32_t n) { return ceil_div(n > 0 ? n : 1, kScanBlock * kScanPer); }

// exclusive scan with the caller's block-sum scratch (scan_blocks(n) + 1 ints)
void scan_exclusive_i32_with(const int32_t *in, int32_t *out, int32_t n, int32_t *bsum,
                             hipStream_t s) {
  const int32_t nb = scan_blocks(n);
  k_scan_local<<<nb, kScanBlock, 0, s>>>(in, out, bsum, n);
  k_scan_sums<<<1, kScanBlock, 0, s>>>(bsum, nb);
  k_scan_add<<<grid((int64_t)n + 1), kBlock, 0, s>>>(out, bsum, n, nb);
}

// Device memory for the temporaries of one setup call: a few large pool
// blocks, cut in order and given back together when the setup ends. On this
// runtime a stream-ordered allocation or free takes tens of microseconds of
// host time, a setup needs hundreds of them, and between its latency-bound
// kernels the GPU waits for the host; cut from the arena they cost nothing,
// at the price of keeping every temporary of the setup until its end.
struct Arena {
  int device;
  hipStream_t s;
  size_t chunk;  // block size: a quarter of the first sweep's temporaries, 1-256 MB
  std::vector<void *> blocks;
  char *cur = nullptr;
  size_t left = 0;
  Arena(const amg_hierarchy *h, int64_t n, int64_t nnz) : device(h->device), s(h->stream) {
    const double q = (36.0 * (double)n + 32.0 * (double)nnz) / 4;
    const double mb = double(1 << 20);
    chunk = (size_t)(q < mb ? mb : (q > 256 * mb ? 256 * mb : q));
    chunk = (chunk + (1 << 20) - 1) / (1 << 20) * (1 << 20);
  }
  Arena(const Arena &) = delete;
  Arena &operator=(const Arena &) = delete;
  ~Arena() {
    for (void *p : blocks) stream_free(device, s, p);
  }
  amg_status get(void **p, size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    if (bytes > chunk / 4) {  // a large request gets a block of its own
      void *q = nullptr;
      AMG_TRY(stream_alloc(device, s, &q, bytes));
      blocks.push_back(q);
      *p = q;
      return AMG_OK;
    }
    if (bytes > left) {
      void *q = nullptr;
      AMG_TRY(stream_alloc(device, s, &q, chunk));
      blocks.push_back(q);
      cur = static_cast<char *>(q);
      left = chunk;
    }
    *p = cur;
    cur += bytes;
    left -= bytes;
    return AMG_OK;
  }
};

// temporaries of one setup call (not owned by the hierarchy): cut from the
// setup's arena while one runs (dropping them then does nothing), else pool
// allocations released in stream order when dropped or destroyed
struct Tmp {
  int device;
  hipStream_t s;
  Arena *arena;
  std::vector<void *> ptrs;
  explicit Tmp(const amg_hierarchy *h)
      : device(h->device), s(h->stream), arena(static_cast<Arena *>(h->setup_arena)) {}
  Tmp(const Tmp &) = delete;
  Tmp &operator=(const Tmp &) = delete;
  ~Tmp() {
    for (void *p : ptrs) stream_free(device, s, p);
  }
  template <typename T>
  amg_status get(T **p, size_t count) {
    void *q = nullptr;
    if (arena) {
      AMG_TRY(arena->get(&q, count * sizeof(T) + 16));
    } else {
      AMG_TRY(stream_alloc(device, s, &q, count * sizeof(T) + 16));
      ptrs.push_back(q);
    }
    *p = reinterpret_cast<T *>(q);
    return AMG_OK;
  }
  void drop(void *p) {
    for (auto &q : ptrs)
      if (q == p) {
        stream_free(device, s, q);
        q = nullptr;
      }
  }
  // exclusive scan of n values, its block sums in this object's memory
  amg_status scan(const int32_t *in, int32_t *out, int32_t n) {
    int32_t *bsum = nullptr;
    AMG_TRY(get(&bsum, (size_t)scan_blocks(n) + 1));
    scan_exclusive_i32_with(in, out, n, bsum, s);
    return AMG_OK;
  }
};

amg_status read_i32(const int32_t *dev, int32_t *host, hipStream_t s) {
  AMG_HIP(hipMemcpyAsync(host, dev, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

amg_status map_err(int32_t flags) {
  if (flags & kErrArg) return AMG_ERR_ARG;
  if (flags & kErrSpd) return AMG_ERR_NOT_SPD;
  if (flags & kErrSym) return AMG_ERR_NOT_SYMMETRIC;
  return AMG_OK;
}

// A matrix of the current sweep: either a level's (borrowed) or a temporary.
struct Mat {
  int32_t n = 0;
  int64_t nnz = 0;
  int32_t *rp = nullptr, *ci = nullptr;
  double *val = nullptr;
  double *w = nullptr;
};

// One pairwise sweep on A (Section 3.2). On return with nc < n, the outputs
// hold the coarse matrix and vectors; nc == n means nothing was matched.
struct SweepOut {
  Mat Ac;
  int32_t nc = 0;
  int32_t *agg = nullptr;   // fine -> coarse (n)
  double *p = nullptr;      // pairwise prolongator values (n)
  int32_t *lead = nullptr;  // coarse -> smallest member (nc)
  int32_t *mate = nullptr;  // n
  int32_t rounds = 0;
};

amg_status pairwise_sweep(amg_hierarchy *h, Tmp &tmp, const Mat &A, SweepOut &o,
                          double *t_match, double *t_number, double *t_rap) {
  hipStream_t s = h->stream;
  const int32_t n = A.n;
  double t0 = now_ms();
  int32_t *dpos, *mate, *cand, *cand2, *counters;
  double *c;
  AMG_TRY(tmp.get(&dpos, n));
  AMG_TRY(tmp.get(&c, A.nnz));
  AMG_TRY(tmp.get(&mate, n));
  AMG_TRY(tmp.get(&cand, n));
  AMG_TRY(tmp.get(&cand2, n));
  constexpr int kMaxBatch = 128;
  AMG_TRY(tmp.get(&counters, kMaxBatch));
  k_diag_pos<<<grid(n), kBlock, 0, s>>>(n, A.rp, A.ci, dpos);
  k_weights<<<grid(n), kBlock, 0, s>>>(n, A.rp, A.ci, A.val, dpos, A.w, c);
  k_fill<int32_t><<<grid(n), kBlock, 0, s>>>(mate, kFree, n);
  k_fill<int32_t><<<grid(n), kBlock, 0, s>>>(cand, -1, n);
  // matching rounds in batches; the host reads the per-round counters after
  // each batch (rounds past the last live one do nothing)
  // first proposals, then one fused accept-and-propose kernel per round with
  // the proposals double-buffered; the last round's accept is applied after
  // rounds queued after the last live one return at once, so batches can be
  // long: 8, 16, ... up to kMaxBatch rounds between host checks
  int32_t rounds = 0, batch = 8;
  int32_t hc[kMaxBatch];
  int32_t *cur = cand, *nxt = cand2;
  k_fill<int32_t><<<1, kMaxBatch, 0, s>>>(counters, 0, kMaxBatch);
  k_match_propose<<<grid(n), kBlock, 0, s>>>(n, A.rp, A.ci, c, mate, cur, counters);
  for (;;) {
    k_fill<int32_t><<<1, kMaxBatch, 0, s>>>(counters, 0, kMaxBatch);
    for (int32_t r = 0; r < batch; ++r) {
      k_match_round<<<grid(n), kBlock, 0, s>>>(n, A.rp, A.ci, c, mate, cur, nxt,
                                               r > 0 ? counters + r - 1 : nullptr, counters + r);
      std::swap(cur, nxt);
    }
    AMG_HIP(hipMemcpyAsync(hc, counters, sizeof(int32_t) * batch, hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    int32_t r = 0;
    while (r < batch && hc[r] > 0) ++r;
    rounds += r;
    if (r < batch) break;
    if (rounds > n + 2) return AMG_ERR_HIP;  // cannot happen: one edge per round at least
    batch = batch * 2 > kMaxBatch ? kMaxBatch : batch * 2;
  }
  // the proposals of the last live round may still hold mutual pairs
  k_match_accept<<<grid(n), kBlock, 0, s>>>(n, mate, cur);
  o.rounds = rounds;
  o.mate = mate;
  tmp.drop(cand2);
  tmp.drop(cand);
  tmp.drop(c);
  double t1 = now_ms();
  *t_match += t1 - t0;

  // numbering
  int32_t *flag, *id;
  AMG_TRY(tmp.get(&flag, n));
  AMG_TRY(tmp.get(&id, n + 1));
  k_leader<<<grid(n), kBlock, 0, s>>>(n, mate, flag);
  AMG_TRY(tmp.scan(flag, id, n));
  int32_t nc = 0;
  AMG_TRY(read_i32(id + n, &nc, s));
  o.nc = nc;
  if (nc == n) {
    *t_number += now_ms() - t1;
    return AMG_OK;
  }
  AMG_TRY(tmp.get(&o.agg, n));
  AMG_TRY(tmp.get(&o.lead, nc));
  AMG_TRY(tmp.get(&o.p, n));
  k_assign<<<grid(n), kBlock, 0, s>>>(n, mate, id, o.agg, o.lead);
  k_pair_prolongator<<<grid(n), kBlock, 0, s>>>(n, mate, A.w, o.p);
  tmp.drop(flag);
  tmp.drop(id);
  double t2 = now_ms();
  *t_number += t2 - t1;

  // Galerkin product and restricted w
  int32_t *inlen, *toff, *tJ, *cnt, *ovf, *novf, *err;
  double *tV;
  AMG_TRY(tmp.get(&inlen, nc));
  AMG_TRY(tmp.get(&toff, nc + 1));
  AMG_TRY(tmp.get(&cnt, nc));
  AMG_TRY(tmp.get(&ovf, nc));
  AMG_TRY(tmp.get(&novf, 2));
  err = novf + 1;
  k_fill<int32_t><<<1, 2, 0, s>>>(novf, 0, 2);
  k_rap_inlen<<<grid(nc), kBlock, 0, s>>>(nc, o.lead, mate, A.rp, inlen);
  AMG_TRY(tmp.scan(inlen, toff, nc));
  AMG_TRY(tmp.get(&tJ, A.nnz));
  AMG_TRY(tmp.get(&tV, A.nnz));
  k_rap_rows<<<grid(nc), kBlock, 0, s>>>(nc, o.lead, mate, A.rp, A.ci, A.val, o.agg, o.p, toff,
                                         tJ, tV, cnt, ovf, novf);
  k_rap_long<<<256, 256, 0, s>>>(o.lead, mate, A.rp, A.ci, A.val, o.agg, o.p, toff, tJ, tV, cnt,
                                 ovf, novf, err);
  int32_t herr = 0;
  AMG_TRY(read_i32(err, &herr, s));
  if (herr) return AMG_ERR_ARG;  // a coarse row gathers more than kRapLongCap entries
  Mat &C = o.Ac;
  C.n = nc;
  AMG_TRY(tmp.get(&C.rp, nc + 1));
  AMG_TRY(tmp.scan(cnt, C.rp, nc));
  int32_t nnzc = 0;
  AMG_TRY(read_i32(C.rp + nc, &nnzc, s));
  C.nnz = nnzc;
  AMG_TRY(tmp.get(&C.ci, nnzc));
  AMG_TRY(tmp.get(&C.val, nnzc));
  AMG_TRY(tmp.get(&C.w, nc));
  k_rap_copy<<<grid(nc), kBlock, 0, s>>>(nc, toff, tJ, tV, C.rp, C.ci, C.val);
  k_restrict_pair<<<grid(nc), kBlock, 0, s>>>(nc, o.lead, mate, o.p, A.w, C.w);
  AMG_HIP(hipStreamSynchronize(s));
  tmp.drop(inlen);
  tmp.drop(toff);
  tmp.drop(tJ);
  tmp.drop(tV);
  tmp.drop(cnt);
  tmp.drop(ovf);
  tmp.drop(dpos);
  *t_rap += now_ms() - t2;
  return AMG_OK;
}

// copy a temporary matrix into hierarchy-owned level storage
amg_status adopt_level(amg_hierarchy *h, const Mat &M, Level &L) {
  hipStream_t s = h->stream;
  L.n = M.n;
  L.nnz = M.nnz;
  AMG_TRY(dalloc(h, &L.rp, (size_t)M.n + 1));
  AMG_TRY(dalloc(h, &L.ci, (size_t)M.nnz));
  AMG_TRY(dalloc(h, &L.val, (size_t)M.nnz));
  AMG_TRY(dalloc(h, &L.w, (size_t)M.n));
  AMG_HIP(hipMemcpyAsync(L.rp, M.rp, sizeof(int32_t) * (M.n + 1), hipMemcpyDeviceToDevice, s));
  AMG_HIP(hipMemcpyAsync(L.ci, M.ci, sizeof(int32_t) * M.nnz, hipMemcpyDeviceToDevice, s));
  AMG_HIP(hipMemcpyAsync(L.val, M.val, sizeof(double) * M.nnz, hipMemcpyDeviceToDevice, s));
  AMG_HIP(hipMemcpyAsync(L.w, M.w, sizeof(double) * M.n, hipMemcpyDeviceToDevice, s));
  return AMG_OK;
}

}  // namespace

amg_status setup_tmp_alloc(amg_hierarchy *h, void **p, size_t bytes) {
  if (h->setup_arena) return static_cast<Arena *>(h->setup_arena)->get(p, bytes);
  return stream_alloc(h->device, h->stream, p, bytes);
}

void setup_tmp_free(amg_hierarchy *h, void *p) {
  if (!h->setup_arena) stream_free(h->device, h->stream, p);
}

amg_status setup_scan(amg_hierarchy *h, const int32_t *in, int32_t *out, int32_t n) {
  int32_t *bsum = nullptr;
  AMG_TRY(setup_tmp_alloc(h, reinterpret_cast<void **>(&bsum),
                          sizeof(int32_t) * ((size_t)scan_blocks(n) + 1)));
  scan_exclusive_i32_with(in, out, n, bsum, h->stream);
  setup_tmp_free(h, bsum);
  return AMG_OK;
}

amg_status scan_exclusive_i32(const int32_t *in, int32_t *out, int32_t n, hipStream_t s) {
  const int32_t nb = scan_blocks(n);
  int32_t *bsum = nullptr;
  AMG_HIP(hipMallocAsync(reinterpret_cast<void **>(&bsum), sizeof(int32_t) * (nb + 1), s));
  scan_exclusive_i32_with(in, out, n, bsum, s);
  AMG_HIP(hipFreeAsync(bsum, s));
  return AMG_OK;
}

amg_status build_hierarchy(amg_hierarchy *h, const amg_csr *A) {
  hipStream_t s = h->stream;
  const amg_params &P = h->params;
  const int32_t n0 = (int32_t)A->n;
  double T[8] = {0};
  double t_start = now_ms();
  // every temporary of this setup comes from one arena (declared before the
  // Tmp objects, so it outlives them), detached again on every way out
  Arena arena(h, A->n, A->nnz);
  struct Attach {
    amg_hierarchy *h;
    ~Attach() { h->setup_arena = nullptr; }
  } attach{h};
  h->setup_arena = &arena;
  Tmp tmp(h);

  // validation
  int32_t *err;
  AMG_TRY(tmp.get(&err, 1));
  k_fill<int32_t><<<1, 1, 0, s>>>(err, 0, 1);
  if (!(P.flags & AMG_FLAG_SKIP_CHECKS))
    k_validate<<<grid(n0), kBlock, 0, s>>>(n0, A->nnz, A->row_ptr, A->col, A->val, err);
  if (P.w) k_check_w<<<grid(n0), kBlock, 0, s>>>(n0, P.w, err);
  int32_t herr = 0;
  AMG_TRY(read_i32(err, &herr, s));
  AMG_TRY(map_err(herr));
  T[0] = now_ms() - t_start;

  // level 0: a copy of A and w
  h->lv.clear();
  h->lv.emplace_back();
  {
    Level &L0 = h->lv[0];
    L0.n = n0;
    L0.nnz = A->nnz;
    AMG_TRY(dalloc(h, &L0.rp, (size_t)n0 + 1));
    AMG_TRY(dalloc(h, &L0.ci, (size_t)A->nnz));
    AMG_TRY(dalloc(h, &L0.val, (size_t)A->nnz));
    AMG_TRY(dalloc(h, &L0.w, (size_t)n0));
    AMG_HIP(hipMemcpyAsync(L0.rp, A->row_ptr, sizeof(int32_t) * (n0 + 1),
                           hipMemcpyDeviceToDevice, s));
    AMG_HIP(hipMemcpyAsync(L0.ci, A->col, sizeof(int32_t) * A->nnz, hipMemcpyDeviceToDevice, s));
    AMG_HIP(hipMemcpyAsync(L0.val, A->val, sizeof(double) * A->nnz, hipMemcpyDeviceToDevice, s));
    if (P.w)
      AMG_HIP(hipMemcpyAsync(L0.w, P.w, sizeof(double) * n0, hipMemcpyDeviceToDevice, s));
    else
      k_fill<double><<<grid(n0), kBlock, 0, s>>>(L0.w, 1.0, n0);
    // algebraically smooth w: w_sweeps l1-Jacobi sweeps on A w = 0 from the
    // sample; the result must still have no zero entry
    if (P.w_sweeps > 0) {
      double *m, *minv, *w2;
      AMG_TRY(tmp.get(&m, n0));
      AMG_TRY(tmp.get(&minv, n0));
      AMG_TRY(tmp.get(&w2, n0));
      k_l1_diag<<<grid(n0), kBlock, 0, s>>>(n0, L0.rp, L0.ci, L0.val, m, minv);
      double *src = L0.w, *dst = w2;
      for (int32_t k = 0; k < P.w_sweeps; ++k) {
        k_smooth_w<<<grid(n0), kBlock, 0, s>>>(n0, L0.rp, L0.ci, L0.val, m, src, dst);
        std::swap(src, dst);
      }
      if (src != L0.w)
        AMG_HIP(hipMemcpyAsync(L0.w, src, sizeof(double) * n0, hipMemcpyDeviceToDevice, s));
      k_fill<int32_t><<<1, 1, 0, s>>>(err, 0, 1);
      k_check_w<<<grid(n0), kBlock, 0, s>>>(n0, L0.w, err);
      AMG_TRY(read_i32(err, &herr, s));
      AMG_TRY(map_err(herr));
    }
  }

  double t_match = 0, t_number = 0, t_rap = 0, t_compose = 0;
  for (int32_t l = 0;; ++l) {
    const int32_t n = h->lv[l].n;
    if (n <= P.max_coarse || l == P.max_levels - 1) break;
    Mat cur{h->lv[l].n, h->lv[l].nnz, h->lv[l].rp, h->lv[l].ci, h->lv[l].val, h->lv[l].w};
    Tmp sweep_tmp(h);  // intermediate sweep matrices
    int32_t *agg_c = nullptr, *mptr = nullptr, *mem = nullptr;
    double *p_c = nullptr;
    AMG_TRY(sweep_tmp.get(&agg_c, n));
    AMG_TRY(sweep_tmp.get(&p_c, n));
    AMG_TRY(sweep_tmp.get(&mptr, n + 1));
    AMG_TRY(sweep_tmp.get(&mem, n));
    k_iota<<<grid((int64_t)n + 1), kBlock, 0, s>>>(mptr, n);
    k_iota<<<grid(n), kBlock, 0, s>>>(mem, n - 1);
    int32_t done = 0, rounds = 0;
    std::vector<Tmp *> owners;
    Tmp *prev_owner = nullptr;
    for (int32_t k = 0; k < P.sweeps; ++k) {
      Tmp *own = new Tmp(h);
      SweepOut o;
      amg_status st = pairwise_sweep(h, *own, cur, o, &t_match, &t_number, &t_rap);
      if (st != AMG_OK) {
        delete own;
        delete prev_owner;
        return st;
      }
      rounds += o.rounds;
      if (o.nc == cur.n) {  // nothing matched: end this level's sweeps
        delete own;
        break;
      }
      double tc = now_ms();
      k_compose<<<grid(n), kBlock, 0, s>>>(n, o.agg, o.p, agg_c, p_c, k == 0 ? 1 : 0);
      int32_t *msz, *mptr_n, *mem_n;
      AMG_TRY(sweep_tmp.get(&msz, o.nc));
      AMG_TRY(sweep_tmp.get(&mptr_n, o.nc + 1));
      AMG_TRY(sweep_tmp.get(&mem_n, n));
      k_member_size<<<grid(o.nc), kBlock, 0, s>>>(o.nc, o.lead, o.mate, mptr, msz);
      AMG_TRY(sweep_tmp.scan(msz, mptr_n, o.nc));
      k_member_merge<<<grid(o.nc), kBlock, 0, s>>>(o.nc, o.lead, o.mate, mptr, mem, mptr_n,
                                                   mem_n);
      AMG_HIP(hipStreamSynchronize(s));
      sweep_tmp.drop(mptr);
      sweep_tmp.drop(mem);
      sweep_tmp.drop(msz);
      mptr = mptr_n;
      mem = mem_n;
      // the previous sweep's matrix is no longer needed
      delete prev_owner;
      prev_owner = own;
      cur = o.Ac;
      ++done;
      t_compose += now_ms() - tc;
    }
    if (done == 0) {  // level l does not coarsen: it is the coarsest
      delete prev_owner;
      break;
    }
    double tc = now_ms();
    Level &F = h->lv[l];
    F.sweeps = done;
    F.rounds = rounds;
    AMG_TRY(dalloc(h, &F.agg, (size_t)n));
    AMG_TRY(dalloc(h, &F.p64, (size_t)n));
    AMG_TRY(dalloc(h, &F.mptr, (size_t)cur.n + 1));
    AMG_TRY(dalloc(h, &F.mem, (size_t)n));
    AMG_HIP(hipMemcpyAsync(F.agg, agg_c, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    AMG_HIP(hipMemcpyAsync(F.p64, p_c, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    AMG_HIP(hipMemcpyAsync(F.mptr, mptr, sizeof(int32_t) * (cur.n + 1), hipMemcpyDeviceToDevice,
                           s));
    AMG_HIP(hipMemcpyAsync(F.mem, mem, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    if (P.smooth_p) {
      // the tentative product chose the aggregates and restricted w; the
      // next level is the Galerkin product with the smoothed prolongator
      const double tr = now_ms();
      int32_t *crp, *cci;
      double *cval;
      int64_t cnnz = 0;
      const int32_t nc = cur.n;
      AMG_TRY(smooth_level(h, F, nc, agg_c, p_c, &crp, &cci, &cval, &cnnz));
      h->lv.emplace_back();
      Level &Cn = h->lv[l + 1];
      Cn.n = nc;
      Cn.nnz = cnnz;
      Cn.rp = crp;
      Cn.ci = cci;
      Cn.val = cval;
      AMG_TRY(dalloc(h, &Cn.w, (size_t)nc));
      AMG_HIP(hipMemcpyAsync(Cn.w, cur.w, sizeof(double) * nc, hipMemcpyDeviceToDevice, s));
      tc += now_ms() - tr;  // counted as Galerkin time, not composition
      t_rap += now_ms() - tr;
    } else {
      h->lv.emplace_back();
      AMG_TRY(adopt_level(h, cur, h->lv[l + 1]));
    }
    AMG_HIP(hipStreamSynchronize(s));
    delete prev_owner;
    t_compose += now_ms() - tc;
  }
  T[1] = t_match;
  T[2] = t_number;
  T[3] = t_rap;
  T[4] = t_compose;

  // smoother diagonals
  double ts = now_ms();
  const int32_t nlev = (int32_t)h->lv.size();
  // (the coarsest level too when its system is solved by CG with them)
  const int32_t nsmooth = h->params.coarse_solver == AMG_COARSE_PCG ? nlev : nlev - 1;
  for (int32_t l = 0; l < nsmooth; ++l) {
    Level &L = h->lv[l];
    AMG_TRY(dalloc(h, &L.m, (size_t)L.n));
    AMG_TRY(dalloc(h, &L.minv64, (size_t)L.n));
    k_l1_diag<<<grid(L.n), kBlock, 0, s>>>(L.n, L.rp, L.ci, L.val, L.m, L.minv64);
  }
  // coarsest: dense Cholesky and the inverse factor
  {
    Level &L = h->lv[nlev - 1];
    const int32_t nL = L.n;
    if (nL > AMG_MAX_DENSE) return AMG_ERR_STALL;
    double *D;
    AMG_TRY(tmp.get(&D, (size_t)nL * nL));
    AMG_HIP(hipMemsetAsync(D, 0, sizeof(double) * (size_t)nL * nL, s));
    k_dense_scatter<<<grid(nL), kBlock, 0, s>>>(nL, L.rp, L.ci, L.val, D);
    k_fill<int32_t><<<1, 1, 0, s>>>(err, 0, 1);
    if (nL <= kCholLdsMax)
      k_cholesky_lds<<<1, 1024, sizeof(double) * (size_t)nL * (nL + 1) / 2, s>>>(nL, D, err);
    else
      k_cholesky<<<1, 1024, 0, s>>>(nL, D, err);
    AMG_TRY(read_i32(err, &herr, s));
    if (herr) return AMG_ERR_NOT_SPD;
    h->C.n = nL;
    AMG_TRY(dalloc(h, &h->C.Linv, (size_t)nL * nL));
    AMG_TRY(dalloc(h, &h->C.Ainv, (size_t)nL * nL));
    const size_t tri_lds = 2 * sizeof(double) * (size_t)nL;  // <= 64 KB (nL <= AMG_MAX_DENSE)
    if (nL <= kTriThreads)
      k_tri_inverse<1><<<nL, kTriThreads, tri_lds, s>>>(nL, D, h->C.Linv);
    else if (nL <= 4 * kTriThreads)
      k_tri_inverse<4><<<nL, kTriThreads, tri_lds, s>>>(nL, D, h->C.Linv);
    else
      k_tri_inverse<AMG_MAX_DENSE / kTriThreads><<<nL, kTriThreads, tri_lds, s>>>(nL, D,
                                                                                  h->C.Linv);
    k_inverse_from_factor<<<grid((int64_t)nL * nL), kBlock, 0, s>>>(nL, h->C.Linv, h->C.Ainv);
    AMG_HIP(hipStreamSynchronize(s));
  }
  T[5] = now_ms() - ts;
  double tf = now_ms();
  AMG_TRY(build_solve_formats(h));
  AMG_HIP(hipStreamSynchronize(s));
  T[6] = now_ms() - tf;
  T[7] = now_ms() - t_start;
  for (int k = 0; k < 8; ++k) h->setup_ms[k] = T[k];
  return AMG_OK;
}

}  // namespace amg
