// Smoothed aggregation on the GPU (the alternative to the K-cycle in
// Section 3.2): omega = 4 / (3 ||D^-1 A||_inf) (the damping 4 / (3 rho(D^-1 A))
// with rho estimated by the infinity norm, which reproduces the supplement's
// convergence constant of the smoothed prolongator), the smoothed prolongator
// Pbar = (I - omega D^-1 A) P of the composed tentative P, and the next level
// Pbar^T A Pbar; plus Pbar and Pbar^T in the solve numbering.
//
// Every product is formed as expand - sort - reduce. Each output row's terms
// are written in a fixed order (the order of the row's entries, then of the
// entries of the rows they select); a stable radix sort on (row, column)
// brings the terms of one position together without changing their order;
// one thread then adds each run's terms onto the first, in order. The sums
// are exactly the sequential sums of the definitions, so the hierarchy is the
// same bit for bit on every run (built with -ffp-contract=off).

#include <cstring>
#include <map>
#include <mutex>
#include <utility>

#include "internal.h"

namespace amg {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;  // elements per thread in a block's tile
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;  // one digit per thread of a block
static_assert(kRadix == kSortThreads, "one thread per digit");

inline int32_t grid(int64_t n) { return ceil_div(n > 0 ? n : 1, kBlock); }

// bits needed for the values 0 .. n - 1
int bits_for(int64_t n) {
  int b = 0;
  while ((int64_t(1) << b) < n) ++b;
  return b;
}

// Temporaries of the smoothed setup: carved from one workspace per device
// that grows on demand (blocks of at least twice the previous size) and is
// kept until the process ends; a Scratch holds the device's workspace lock
// for its lifetime, so smoothed setups on one device take turns. A product
// takes a dozen buffers of up to several GiB; allocating and freeing them per
// call (through the stream-ordered pool or hipMalloc/hipFree) cost far more
// than the kernels, up to seconds per call once such blocks had been freed.
struct Workspace {
  std::mutex m;
  std::vector<std::pair<char *, size_t>> blocks;
};

Workspace &workspace(int device) {
  static std::mutex guard;
  static std::map<int, Workspace *> all;
  std::lock_guard<std::mutex> g(guard);
  Workspace *&w = all[device];
  if (!w) w = new Workspace();  // process lifetime
  return *w;
}

struct Scratch {
  hipStream_t s;
  Workspace &ws;
  std::unique_lock<std::mutex> lock;
  size_t block = 0, used = 0;  // current block and bytes taken from it
  explicit Scratch(const amg_hierarchy *h)
      : s(h->stream), ws(workspace(h->device)), lock(ws.m) {}
  Scratch(const Scratch &) = delete;
  Scratch &operator=(const Scratch &) = delete;
  ~Scratch() { (void)hipStreamSynchronize(s); }  // the next user may be another stream
  template <typename T>
  amg_status get(T **p, size_t count) {
    const size_t bytes = (count * sizeof(T) + 16 + 255) & ~size_t(255);
    while (block < ws.blocks.size() && used + bytes > ws.blocks[block].second) {
      ++block;
      used = 0;
    }
    if (block == ws.blocks.size()) {
      size_t sz = size_t(256) << 20;
      for (const auto &b : ws.blocks) sz = b.second * 2 > sz ? b.second * 2 : sz;
      if (bytes > sz) sz = bytes;
      void *q = nullptr;
      AMG_HIP(hipMalloc(&q, sz));
      ws.blocks.emplace_back(reinterpret_cast<char *>(q), sz);
      used = 0;
    }
    *p = reinterpret_cast<T *>(ws.blocks[block].first + used);
    used += bytes;
    return AMG_OK;
  }
};

// ---------------------------------------------------------------------------
// stable LSD radix sort of (64-bit key, double) pairs, 8 bits per pass
// ---------------------------------------------------------------------------

// digit counts of each block's tile, digit-major: hist[d * nblocks + block]
__global__ void __launch_bounds__(kSortThreads) k_radix_hist(int32_t count,
                                                            const uint64_t *__restrict__ key,
                                                            int shift, int32_t nblocks,
                                                            int32_t *__restrict__ hist) {
  __shared__ int32_t c[kRadix];
  c[threadIdx.x] = 0;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * kSortTile;
  for (int u = 0; u < kSortItems; ++u) {
    const int64_t i = t0 + (int64_t)u * kSortThreads + threadIdx.x;
    if (i < count) atomicAdd(&c[(key[i] >> shift) & (kRadix - 1)], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = c[threadIdx.x];
}

// Writes every element of the block's tile to its place: the exclusive scan
// of the digit-major counts (offs) gives where the block's run of each digit
// starts; inside the tile, elements keep their index order (rounds of one
// element per thread, waves in order, lanes in order).
__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(
    int32_t count, const uint64_t *__restrict__ key, const double *__restrict__ val, int shift,
    int32_t nblocks, const int32_t *__restrict__ offs, uint64_t *__restrict__ key_out,
    double *__restrict__ val_out) {
  constexpr int kW = kSortThreads / kWave;
  __shared__ int32_t base[kRadix];
  __shared__ int32_t wcnt[kW][kRadix];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  base[tid] = offs[(int64_t)tid * nblocks + blockIdx.x];
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
  const int64_t t0 = (int64_t)blockIdx.x * kSortTile;
  for (int u = 0; u < kSortItems; ++u) {
    for (int w = 0; w < kW; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const int64_t i = t0 + (int64_t)u * kSortThreads + tid;
    const bool ok = i < count;
    uint64_t k = 0;
    double v = 0.0;
    int d = 0;
    if (ok) {
      k = key[i];
      v = val[i];
      d = (int)((k >> shift) & (kRadix - 1));
    }
    // lanes of this wave holding the same digit
    uint64_t m = __ballot(ok);
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const int rank = __popcll(m & below);
    if (ok && rank == 0) wcnt[wid][d] = __popcll(m);
    __syncthreads();
    {  // digit tid: where each wave's group starts, and the block's new base
      int32_t sacc = base[tid];
      for (int w = 0; w < kW; ++w) {
        const int32_t c = wcnt[w][tid];
        wcnt[w][tid] = sacc;
        sacc += c;
      }
      base[tid] = sacc;
    }
    __syncthreads();
    if (ok) {
      const int32_t pos = wcnt[wid][d] + rank;
      key_out[pos] = k;
      val_out[pos] = v;
    }
    __syncthreads();
  }
}

// sorts count pairs by the low `bits` bits of the key, stably; *key and *val
// point at the sorted arrays on return (buffers of the scratch set)
amg_status radix_sort(Scratch &S, int32_t count, int bits, uint64_t **key, double **val) {
  if (count <= 1 || bits <= 0) return AMG_OK;
  hipStream_t s = S.s;
  const int32_t nblocks = ceil_div(count, kSortTile);
  if ((int64_t)nblocks * kRadix >= INT32_MAX) return AMG_ERR_ARG;
  uint64_t *k2;
  double *v2;
  int32_t *hist, *offs;
  AMG_TRY(S.get(&k2, (size_t)count));
  AMG_TRY(S.get(&v2, (size_t)count));
  AMG_TRY(S.get(&hist, (size_t)nblocks * kRadix));
  AMG_TRY(S.get(&offs, (size_t)nblocks * kRadix + 1));
  for (int shift = 0; shift < bits; shift += kRadixBits) {
    k_radix_hist<<<nblocks, kSortThreads, 0, s>>>(count, *key, shift, nblocks, hist);
    AMG_TRY(scan_exclusive_i32(hist, offs, nblocks * kRadix, s));
    k_radix_scatter<<<nblocks, kSortThreads, 0, s>>>(count, *key, *val, shift, nblocks, offs, k2,
                                                     v2);
    std::swap(*key, k2);
    std::swap(*val, v2);
  }
  AMG_HIP(hipGetLastError());
  return AMG_OK;
}

// ---------------------------------------------------------------------------
// sorted (row << cb | column, term) pairs -> CSR with the runs summed in order
// ---------------------------------------------------------------------------

__global__ void k_heads(int32_t count, const uint64_t *__restrict__ key, int32_t *__restrict__ h) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) h[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

__global__ void k_run_start(int32_t count, const int32_t *__restrict__ h,
                            const int32_t *__restrict__ run, int32_t *__restrict__ start) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count && h[i]) start[run[i]] = (int32_t)i;
  if (i == 0) start[run[count]] = count;  // run[count] = number of runs
}

// one thread per run: the first term, then the others added in order
__global__ void k_run_sum(int32_t nrun, const int32_t *__restrict__ start,
                          const uint64_t *__restrict__ key, const double *__restrict__ val,
                          int cb, int32_t *__restrict__ row_of, int32_t *__restrict__ col,
                          double *__restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrun) return;
  const int32_t b = start[r], e = start[r + 1];
  double v = val[b];
  for (int32_t t = b + 1; t < e; ++t) v = v + val[t];
  out[r] = v;
  const uint64_t k = key[b];
  col[r] = (int32_t)(k & ((uint64_t(1) << cb) - 1));
  row_of[r] = (int32_t)(k >> cb);
}

// rp[q] = first run of row q (runs are sorted by row); rp[nrows] = nrun
__global__ void k_row_ptr(int32_t nrun, int32_t nrows, const int32_t *__restrict__ row_of,
                          int32_t *__restrict__ rp) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s > nrun) return;
  const int32_t lo = s == 0 ? -1 : row_of[s - 1];
  const int32_t hi = s == nrun ? nrows : row_of[s];
  for (int32_t q = lo + 1; q <= hi; ++q) rp[q] = (int32_t)s;
}

// destination of a reduced CSR: owned by the hierarchy or by the scratch set
struct CsrOut {
  int32_t *rp = nullptr, *ci = nullptr;
  double *val = nullptr;
  int64_t nnz = 0;
};

template <typename Alloc>
amg_status reduce_sorted(Scratch &S, int32_t count, const uint64_t *key, const double *val,
                         int32_t nrows, int cb, Alloc alloc, CsrOut *out) {
  hipStream_t s = S.s;
  int32_t *h, *run;
  AMG_TRY(S.get(&h, (size_t)count + 1));
  AMG_TRY(S.get(&run, (size_t)count + 1));
  k_heads<<<grid(count), kBlock, 0, s>>>(count, key, h);
  AMG_TRY(scan_exclusive_i32(h, run, count, s));
  int32_t nrun = 0;
  AMG_HIP(hipMemcpyAsync(&nrun, run + count, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  int32_t *start, *row_of;
  AMG_TRY(S.get(&start, (size_t)nrun + 1));
  AMG_TRY(S.get(&row_of, (size_t)nrun + 1));
  AMG_TRY(alloc(&out->rp, (size_t)nrows + 1, &out->ci, &out->val, (size_t)nrun));
  k_run_start<<<grid((int64_t)count + 1), kBlock, 0, s>>>(count, h, run, start);
  k_run_sum<<<grid(nrun), kBlock, 0, s>>>(nrun, start, key, val, cb, row_of, out->ci, out->val);
  k_row_ptr<<<grid((int64_t)nrun + 1), kBlock, 0, s>>>(nrun, nrows, row_of, out->rp);
  AMG_HIP(hipGetLastError());
  out->nnz = nrun;
  return AMG_OK;
}

// ---------------------------------------------------------------------------
// the three products and the transposes
// ---------------------------------------------------------------------------

// (sum over ascending j of |a_ij|) / a_ii per row; maximum over rows (the
// bits of non-negative doubles order like the values)
__global__ void k_absnorm(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                          const double *__restrict__ val, unsigned long long *__restrict__ mx) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double sum = 0.0, aii = 0.0;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
    sum = sum + fabs(val[k]);
    if (ci[k] == i) aii = val[k];
  }
  const double r = sum / aii;
  atomicMax(mx, (unsigned long long)__double_as_longlong(r));
}

// terms of Pbar's sums s(i, J) = sum over j with agg[j] = J of a_ij p_j, in
// the order of row i's entries (one term per entry of A)
__global__ void k_pbar_terms(int32_t n, const int32_t *__restrict__ rp,
                             const int32_t *__restrict__ ci, const double *__restrict__ val,
                             const int32_t *__restrict__ agg, const double *__restrict__ p,
                             int cb, uint64_t *__restrict__ key, double *__restrict__ term) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
    const int32_t j = ci[k];
    key[k] = ((uint64_t)i << cb) | (uint64_t)agg[j];
    term[k] = val[k] * p[j];
  }
}

// Pbar(i, J) = (J = agg[i] ? p_i : 0) - omega (s / a_ii), in place
__global__ void k_pbar_finish(int32_t n, const int32_t *__restrict__ prp,
                              const int32_t *__restrict__ pci, double *__restrict__ pval,
                              const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                              const double *__restrict__ val, const int32_t *__restrict__ agg,
                              const double *__restrict__ p, double omega) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double aii = 0.0;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
    if (ci[k] == i) aii = val[k];
  for (int32_t e = prp[i]; e < prp[i + 1]; ++e) {
    const double t = pval[e] / aii;
    const double base = pci[e] == agg[i] ? p[i] : 0.0;
    pval[e] = base - omega * t;
  }
}

// number of terms each combining entry k (coef_k, row src_k of B) brings:
// the length of B's row src_k; the int64 total for the overflow check
__global__ void k_comb_count(int64_t nk, const int32_t *__restrict__ src,
                             const int32_t *__restrict__ brp, int32_t *__restrict__ cnt,
                             unsigned long long *__restrict__ total) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  const int32_t j = src[k];
  const int32_t c = brp[j + 1] - brp[j];
  cnt[k] = c;
  atomicAdd(total, (unsigned long long)c);
}

// row of each combining entry (k in [xp[r], xp[r+1]) belongs to row r)
__global__ void k_entry_rows(int32_t nr, const int32_t *__restrict__ xp,
                             int32_t *__restrict__ row) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nr) return;
  for (int32_t k = xp[r]; k < xp[r + 1]; ++k) row[k] = r;
}

// The terms coef_k * B(src_k, e): entry k's terms occupy [off[k], off[k+1])
// in the order k ascending, then e ascending (entries of one row are
// consecutive in k). Each block writes one tile of consecutive terms
// (coalesced); a term finds its entry by binary search among the offsets of
// the tile's entries, staged in LDS (every entry brings at least one term,
// so a tile spans at most kCombTile + 1 entries).
constexpr int kCombPer = 8;
constexpr int kCombTile = kBlock * kCombPer;
__global__ void __launch_bounds__(kBlock) k_comb_terms(
    int32_t count, int32_t nk, const int32_t *__restrict__ row, const int32_t *__restrict__ src,
    const double *__restrict__ coef, const int32_t *__restrict__ brp,
    const int32_t *__restrict__ bci, const double *__restrict__ bval,
    const int32_t *__restrict__ off, int cb, uint64_t *__restrict__ key,
    double *__restrict__ term) {
  __shared__ int32_t so[kCombTile + 2];
  __shared__ int32_t kfirst, kcount;
  const int32_t T0 = blockIdx.x * kCombTile;
  const int32_t T1 = min(count, T0 + kCombTile);
  if (threadIdx.x == 0) {
    // last entry with off <= T0, and last entry with off <= T1 - 1
    int32_t lo = 0, hi = nk - 1;
    while (lo < hi) {
      const int32_t mid = lo + (hi - lo + 1) / 2;
      if (off[mid] <= T0) lo = mid;
      else hi = mid - 1;
    }
    int32_t lo2 = lo, hi2 = nk - 1;
    while (lo2 < hi2) {
      const int32_t mid = lo2 + (hi2 - lo2 + 1) / 2;
      if (off[mid] <= T1 - 1) lo2 = mid;
      else hi2 = mid - 1;
    }
    kfirst = lo;
    kcount = lo2 - lo + 1;
  }
  __syncthreads();
  const int32_t k0 = kfirst, nkt = kcount;
  for (int32_t q = threadIdx.x; q <= nkt; q += kBlock) so[q] = off[k0 + q];
  __syncthreads();
  for (int u = 0; u < kCombPer; ++u) {
    const int32_t t = T0 + u * kBlock + (int32_t)threadIdx.x;
    if (t >= T1) break;
    int32_t lo = 0, hi = nkt - 1;  // last local entry with so <= t
    while (lo < hi) {
      const int32_t mid = lo + (hi - lo + 1) / 2;
      if (so[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    const int32_t k = k0 + lo;
    const int32_t e = brp[src[k]] + (t - so[lo]);
    key[t] = ((uint64_t)row[k] << cb) | (uint64_t)bci[e];
    term[t] = coef[k] * bval[e];
  }
}

// entries of an nr-row CSR re-keyed as (rowmap(column) << cb | colmap(row)),
// i.e. transposed, with optional renumbering of both sides (NULL: identity)
__global__ void k_transpose_keys(int32_t nr, const int32_t *__restrict__ rp,
                                 const int32_t *__restrict__ ci, const double *__restrict__ val,
                                 const int32_t *__restrict__ map_row,
                                 const int32_t *__restrict__ map_col, int cb,
                                 uint64_t *__restrict__ key, double *__restrict__ v) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nr) return;
  const uint64_t iq = map_row ? (uint64_t)map_row[i] : (uint64_t)i;
  for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
    const int32_t J = ci[e];
    key[e] = ((uint64_t)(map_col ? map_col[J] : J) << cb) | iq;
    v[e] = val[e];
  }
}

// entries re-keyed as (map_row(row) << cb | map_col(column)), not transposed
__global__ void k_renumber_keys(int32_t nr, const int32_t *__restrict__ rp,
                                const int32_t *__restrict__ ci, const double *__restrict__ val,
                                const int32_t *__restrict__ map_row,
                                const int32_t *__restrict__ map_col, int cb,
                                uint64_t *__restrict__ key, double *__restrict__ v) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nr) return;
  const uint64_t iq = (uint64_t)map_row[i];
  for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
    key[e] = (iq << cb) | (uint64_t)map_col[ci[e]];
    v[e] = val[e];
  }
}

// lower triangle := upper triangle, so the product is bitwise symmetric
__global__ void k_mirror_lower(int32_t n, const int32_t *__restrict__ rp,
                               const int32_t *__restrict__ ci, double *__restrict__ val,
                               int32_t *__restrict__ err) {
  const int32_t I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= n) return;
  for (int32_t k = rp[I]; k < rp[I + 1]; ++k) {
    const int32_t J = ci[k];
    if (J >= I) break;
    int32_t lo = rp[J], hi = rp[J + 1] - 1, m = -1;
    while (lo <= hi) {
      const int32_t mid = lo + (hi - lo) / 2;
      if (ci[mid] == I) {
        m = mid;
        break;
      }
      if (ci[mid] < I) lo = mid + 1;
      else hi = mid - 1;
    }
    if (m < 0) {
      atomicOr(err, 1);
      return;
    }
    val[k] = val[m];
  }
}

__global__ void k_demote_f64(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// sum_k coef_k B(src_k, :) for every row r < nr into a CSR with ncols
// columns (terms in k then e order, runs summed in order)
template <typename Alloc>
amg_status row_combination(Scratch &S, int32_t nr, const int32_t *xp, const int32_t *src,
                           const double *coef, const int32_t *brp, const int32_t *bci,
                           const double *bval, int32_t ncols, Alloc alloc, CsrOut *out) {
  hipStream_t s = S.s;
  int32_t nk = 0;  // combining entries
  AMG_HIP(hipMemcpyAsync(&nk, xp + nr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  int32_t *cnt, *off, *row;
  unsigned long long *total;
  AMG_TRY(S.get(&cnt, (size_t)nk + 1));
  AMG_TRY(S.get(&off, (size_t)nk + 1));
  AMG_TRY(S.get(&row, (size_t)nk + 1));
  AMG_TRY(S.get(&total, 1));
  AMG_HIP(hipMemsetAsync(total, 0, sizeof(unsigned long long), s));
  k_comb_count<<<grid(nk), kBlock, 0, s>>>(nk, src, brp, cnt, total);
  k_entry_rows<<<grid(nr), kBlock, 0, s>>>(nr, xp, row);
  unsigned long long htotal = 0;
  AMG_HIP(hipMemcpyAsync(&htotal, total, sizeof(htotal), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  if (htotal >= (unsigned long long)(INT32_MAX - kSortTile)) return AMG_ERR_ARG;
  const int32_t count = (int32_t)htotal;
  AMG_TRY(scan_exclusive_i32(cnt, off, nk, s));
  uint64_t *key;
  double *term;
  AMG_TRY(S.get(&key, (size_t)count + 1));
  AMG_TRY(S.get(&term, (size_t)count + 1));
  const int cb = bits_for(ncols);
  if (count > 0)
    k_comb_terms<<<ceil_div(count, kCombTile), kBlock, 0, s>>>(count, nk, row, src, coef, brp,
                                                               bci, bval, off, cb, key, term);
  AMG_TRY(radix_sort(S, count, cb + bits_for(nr), &key, &term));
  return reduce_sorted(S, count, key, term, nr, cb, alloc, out);
}

}  // namespace

amg_status smooth_level(amg_hierarchy *h, Level &F, int32_t nc, const int32_t *agg,
                        const double *p, int32_t **rp, int32_t **ci, double **val,
                        int64_t *nnz) {
  hipStream_t s = h->stream;
  const int32_t n = F.n;
  Scratch S(h);
  // hierarchy-owned and scratch destinations
  auto owned = [&](int32_t **r, size_t nr1, int32_t **c, double **v, size_t nz) -> amg_status {
    AMG_TRY(dalloc(h, r, nr1));
    AMG_TRY(dalloc(h, c, nz));
    AMG_TRY(dalloc(h, v, nz));
    return AMG_OK;
  };
  auto scratch = [&](int32_t **r, size_t nr1, int32_t **c, double **v, size_t nz) -> amg_status {
    AMG_TRY(S.get(r, nr1));
    AMG_TRY(S.get(c, nz));
    AMG_TRY(S.get(v, nz));
    return AMG_OK;
  };
  // omega
  unsigned long long *mx;
  AMG_TRY(S.get(&mx, 1));
  AMG_HIP(hipMemsetAsync(mx, 0, sizeof(unsigned long long), s));
  k_absnorm<<<grid(n), kBlock, 0, s>>>(n, F.rp, F.ci, F.val, mx);
  unsigned long long hmx = 0;
  AMG_HIP(hipMemcpyAsync(&hmx, mx, sizeof(hmx), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  double nrm;
  std::memcpy(&nrm, &hmx, sizeof(double));
  if (!(nrm > 0.0) || !std::isfinite(nrm)) return AMG_ERR_NOT_SPD;
  F.omega = 4.0 / (3.0 * nrm);
  // Pbar: one term per entry of A, reduced per (i, J), then finished
  {
    const int32_t count = (int32_t)F.nnz;
    uint64_t *key;
    double *term;
    AMG_TRY(S.get(&key, (size_t)count + 1));
    AMG_TRY(S.get(&term, (size_t)count + 1));
    const int cb = bits_for(nc);
    k_pbar_terms<<<grid(n), kBlock, 0, s>>>(n, F.rp, F.ci, F.val, agg, p, cb, key, term);
    AMG_TRY(radix_sort(S, count, cb + bits_for(n), &key, &term));
    CsrOut Pb;
    AMG_TRY(reduce_sorted(S, count, key, term, n, cb, owned, &Pb));
    k_pbar_finish<<<grid(n), kBlock, 0, s>>>(n, Pb.rp, Pb.ci, Pb.val, F.rp, F.ci, F.val, agg, p,
                                             F.omega);
    F.pb_rp = Pb.rp;
    F.pb_ci = Pb.ci;
    F.pb_val = Pb.val;
    F.pb_nnz = Pb.nnz;
  }
  // AP = A Pbar: row i combines the rows j of Pbar with the coefficients a_ij
  CsrOut AP;
  AMG_TRY(row_combination(S, n, F.rp, F.ci, F.val, F.pb_rp, F.pb_ci, F.pb_val, nc, scratch,
                          &AP));
  // Pbar^T (rows J, entries ascending i)
  CsrOut PT;
  {
    const int32_t count = (int32_t)F.pb_nnz;
    uint64_t *key;
    double *v;
    AMG_TRY(S.get(&key, (size_t)count + 1));
    AMG_TRY(S.get(&v, (size_t)count + 1));
    const int cb = bits_for(n);
    k_transpose_keys<<<grid(n), kBlock, 0, s>>>(n, F.pb_rp, F.pb_ci, F.pb_val, nullptr, nullptr,
                                                cb, key, v);
    AMG_TRY(radix_sort(S, count, cb + bits_for(nc), &key, &v));
    AMG_TRY(reduce_sorted(S, count, key, v, nc, cb, scratch, &PT));
  }
  // A_c = Pbar^T AP: row I combines the rows i of AP with Pbar(i, I)
  CsrOut Ac;
  AMG_TRY(row_combination(S, nc, PT.rp, PT.ci, PT.val, AP.rp, AP.ci, AP.val, nc, owned, &Ac));
  int32_t *err;
  AMG_TRY(S.get(&err, 1));
  AMG_HIP(hipMemsetAsync(err, 0, sizeof(int32_t), s));
  k_mirror_lower<<<grid(nc), kBlock, 0, s>>>(nc, Ac.rp, Ac.ci, Ac.val, err);
  int32_t herr = 0;
  AMG_HIP(hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  if (herr) return AMG_ERR_ARG;
  *rp = Ac.rp;
  *ci = Ac.ci;
  *val = Ac.val;
  *nnz = Ac.nnz;
  return AMG_OK;
}

amg_status long_row_csr(amg_hierarchy *h, int32_t l, bool fp32) {
  hipStream_t s = h->stream;
  Level &F = h->lv[l];
  const int32_t n = F.n;
  const int32_t count = (int32_t)F.nnz;
  Scratch S(h);
  auto owned = [&](int32_t **r, size_t nr1, int32_t **c, double **v, size_t nz) -> amg_status {
    AMG_TRY(dalloc(h, r, nr1));
    AMG_TRY(dalloc(h, c, nz));
    AMG_TRY(dalloc(h, v, nz));
    return AMG_OK;
  };
  uint64_t *key;
  double *v;
  AMG_TRY(S.get(&key, (size_t)count + 1));
  AMG_TRY(S.get(&v, (size_t)count + 1));
  const int cb = bits_for(n);
  k_renumber_keys<<<grid(n), kBlock, 0, s>>>(n, F.rp, F.ci, F.val, F.iperm, F.iperm, cb, key, v);
  AMG_TRY(radix_sort(S, count, 2 * cb, &key, &v));
  CsrOut M;
  AMG_TRY(reduce_sorted(S, count, key, v, n, cb, owned, &M));
  F.lr_rp = M.rp;
  F.lr_ci = M.ci;
  F.lr_v64 = M.val;
  if (fp32) {
    AMG_TRY(dalloc(h, &F.lr_v32, (size_t)count));
    k_demote_f64<<<grid(count), kBlock, 0, s>>>(count, F.lr_v64, F.lr_v32);
  }
  AMG_HIP(hipGetLastError());
  AMG_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

amg_status smooth_solve_format(amg_hierarchy *h, int32_t l, bool fp32) {
  hipStream_t s = h->stream;
  Level &F = h->lv[l];
  const Level &C = h->lv[l + 1];
  const int32_t n = F.n, nc = C.n;
  const int32_t count = (int32_t)F.pb_nnz;
  Scratch S(h);
  auto owned = [&](int32_t **r, size_t nr1, int32_t **c, double **v, size_t nz) -> amg_status {
    AMG_TRY(dalloc(h, r, nr1));
    AMG_TRY(dalloc(h, c, nz));
    AMG_TRY(dalloc(h, v, nz));
    return AMG_OK;
  };
  uint64_t *key;
  double *v;
  AMG_TRY(S.get(&key, (size_t)count + 1));
  AMG_TRY(S.get(&v, (size_t)count + 1));
  // Pbar by fine position, columns by coarse position
  {
    const int cb = bits_for(nc);
    k_renumber_keys<<<grid(n), kBlock, 0, s>>>(n, F.pb_rp, F.pb_ci, F.pb_val, F.iperm, C.iperm,
                                               cb, key, v);
    uint64_t *k1 = key;
    double *v1 = v;
    AMG_TRY(radix_sort(S, count, cb + bits_for(n), &k1, &v1));
    CsrOut P;
    AMG_TRY(reduce_sorted(S, count, k1, v1, n, cb, owned, &P));
    F.sp_rp = P.rp;
    F.sp_ci = P.ci;
    F.sp_v64 = P.val;
  }
  // Pbar^T by coarse position, entries by fine position
  {
    const int cb = bits_for(n);
    k_transpose_keys<<<grid(n), kBlock, 0, s>>>(n, F.pb_rp, F.pb_ci, F.pb_val, F.iperm, C.iperm,
                                                cb, key, v);
    uint64_t *k1 = key;
    double *v1 = v;
    AMG_TRY(radix_sort(S, count, cb + bits_for(nc), &k1, &v1));
    CsrOut T;
    AMG_TRY(reduce_sorted(S, count, k1, v1, nc, cb, owned, &T));
    F.st_rp = T.rp;
    F.st_ci = T.ci;
    F.st_v64 = T.val;
  }
  if (fp32) {
    AMG_TRY(dalloc(h, &F.sp_v32, (size_t)count));
    AMG_TRY(dalloc(h, &F.st_v32, (size_t)count));
    k_demote_f64<<<grid(count), kBlock, 0, s>>>(count, F.sp_v64, F.sp_v32);
    k_demote_f64<<<grid(count), kBlock, 0, s>>>(count, F.st_v64, F.st_v32);
  }
  AMG_HIP(hipGetLastError());
  AMG_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

}  // namespace amg
