// Internal declarations of the gfx950 matching-AMG library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdint>
#include <thread>
#include <vector>

#include "amg.h"

namespace amg {

// ---------------------------------------------------------------------------
// error handling: every host routine returns amg_status
// ---------------------------------------------------------------------------
#define AMG_HIP(call)                                  \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) {                            \
      (void)hipGetLastError();                         \
      return e_ == hipErrorOutOfMemory ? AMG_ERR_OOM   \
                                       : AMG_ERR_HIP;  \
    }                                                  \
  } while (0)

#define AMG_TRY(call)                  \
  do {                                 \
    amg_status s_ = (call);            \
    if (s_ != AMG_OK) return s_;       \
  } while (0)

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kSlice = 64;       // rows per SELL slice (one wavefront)
constexpr int kBlock = 256;      // threads per block of the streaming kernels
// most blocks of a reducing kernel (the partials buffer)
constexpr int kMaxParts = 65536;
// Row-streaming kernels on levels of fewer than kManyRows rows give each
// thread 1 to 4 rows, aiming at about kTargetBlocks blocks: at 160^3 (4000
// blocks of 1024 rows) a solve measured 3 % faster than with one row per
// thread (more loads in flight, fewer partials to finalize); 16 rows per
// thread was 16 % slower. Larger levels keep one row per thread: on the
// anisotropic 256^3 problem (16.7 M rows) 4 rows were 5 % slower.
constexpr int kTargetBlocks = 4096;
constexpr int kMaxRowsPerThread = 4;
constexpr int64_t kManyRows = int64_t(1) << 23;
constexpr int kPartPlanes = 3;  // partial-sum planes (dot products per reduction)
// K-cycle scalars of one level's two flexible-CG iterations
enum KScal : int32_t { kRho1 = 0, kS1, kGamma, kRho2, kS2, kA1, kKScal = 8 };
constexpr int kNumXcd = 8;       // MI355X: 8 XCDs, blocks dispatched round-robin

// Solve-phase PCG scalars, resident on the device.
struct PcgScal {
  double rho;     // (r, z) of the current iterate
  double pq;      // (p, A p)
  double alpha, beta;
  double rr;      // (r, r)
  double bb;      // (b, b)
  double rtol;
  double tol2;    // (rtol ||b||)^2
  double rr_true; // (b - A x, b - A x) at exit
  int32_t iter;
  int32_t maxit;
  int32_t done;   // 0 running, 1 converged, 2 maxit, 3 breakdown, 4 zero rhs
  int32_t phase;  // 0: next (r, z) initialises rho; 1: it also forms beta
};

// Sliced ELLPACK, 64 rows per slice, column-major inside a slice so that
// lane i of a wavefront reads row i's k-th entry at consecutive addresses.
// v*: the matrix values; s*: the values scaled by the column's inverse
// l1-Jacobi diagonal (A M^-1), used where the smoother's first sweep from a
// zero guess is folded into the residual.
struct Sell {
  int32_t n = 0;
  int32_t nslices = 0;
  int64_t nnz_padded = 0;
  int32_t *sptr = nullptr;  // nslices + 1 element offsets (multiples of 64)
  int32_t *col = nullptr;
  double *v64 = nullptr;
  float *v32 = nullptr;
  double *s64 = nullptr;
  float *s32 = nullptr;
  int32_t max_width = 0;  // widest slice (entries per row); set for levels of <= 1024 rows
  // every value of A is an FP32 number (checked on level 0 also when the
  // FP32 copy is switched off); exact32: v32 holds A exactly and the FP64
  // kernels of level 0 read it (half the value bytes, identical arithmetic)
  bool fp32_values = false;
  bool exact32 = false;
};

// LDS-staged gathers. The rows of a level are split into tiles, one per
// block of a kernel; for every tile, hidx[hptr[t] .. hptr[t + 1]) lists the
// distinct columns its rows reference, ascending, and lcol, laid out like
// Sell::col, holds at each SELL position the index of that position's column
// in its tile's list. A block loads its tile's entries of the gathered
// vector into LDS once (each distinct column once, contiguous runs
// coalesced), then every row product reads its operands from LDS: about 1.7
// global loads per row on a 7-point level instead of 7 gathers, and 2-byte
// instead of 4-byte column indices.
struct Halo {
  int32_t ntiles = 0;
  int32_t param = 0;         // the launch geometry the tiles follow (row chunk, or
                             // coarse rows per block of the down step)
  int32_t umax = 0;          // longest list: LDS entries of one block
  int32_t *hptr = nullptr;   // ntiles + 1 offsets into hidx
  int32_t *hidx = nullptr;
  uint16_t *lcol = nullptr;  // local column index at every SELL position
  bool ok() const { return lcol != nullptr; }
};

// A level holds its setup data in the original numbering of that level and
// its solve data in an aggregate-major order: the unknowns of every
// aggregate of P_l form one contiguous segment, and the segments follow the
// order of the coarse unknowns on level l + 1 (itself aggregate-major). The
// coarsest level keeps its numbering.
struct Level {
  int32_t n = 0;
  int64_t nnz = 0;
  // setup data, original numbering
  int32_t *rp = nullptr, *ci = nullptr;  // FP64 CSR of A_l
  double *val = nullptr;
  double *w = nullptr;       // smooth vector restricted to this level
  double *m = nullptr;       // l1-Jacobi diagonal
  double *minv64 = nullptr;  // 1 / m
  int32_t *agg = nullptr;    // fine row -> coarse index (absent on the coarsest level)
  double *p64 = nullptr;     // P(i, agg[i])
  int32_t *mptr = nullptr;   // coarse index -> range of its members in mem
  int32_t *mem = nullptr;    // members, ascending inside each aggregate
  // solve data, aggregate-major positions
  int32_t *perm = nullptr;   // position -> original index
  int32_t *iperm = nullptr;  // original index -> position
  Sell S;                    // A_l permuted
  // LDS-staged gathers on level 0 (when every tile's list fits): tiles of
  // the row chunks of the streaming kernels (post-smoothing, outer SpMV) and
  // of the down step's blocks of segments
  Halo hrow, hseg;
  double *sminv64 = nullptr; // 1 / m by position
  float *sminv32 = nullptr;
  int32_t *seg = nullptr;    // n_{l+1} + 1 segment starts, by coarse position
  int32_t *aggp = nullptr;   // coarse position of each position
  double *pp64 = nullptr;    // prolongator value of each position
  float *pp32 = nullptr;
  // V-cycle work vectors in the hierarchy precision
  void *r = nullptr, *z = nullptr, *t = nullptr, *y = nullptr;
  // K-cycle flexible-CG vectors (levels strictly between the finest and the
  // coarsest): preconditioned residuals c1, c2, their products v1 = A c1,
  // v2 = A c2, and the second residual r1
  void *c1 = nullptr, *v1 = nullptr, *r1 = nullptr, *c2 = nullptr, *v2 = nullptr;
  // smoothed aggregation: Pbar = (I - omega D^-1 A) P to the next level, in
  // the setup numbering (CSR, n x n_{l+1}), and in the solve numbering as
  // Pbar (rows by position, sp_*) and Pbar^T (rows by coarse position, st_*)
  double omega = 0.0;
  int32_t *pb_rp = nullptr, *pb_ci = nullptr;
  double *pb_val = nullptr;
  int64_t pb_nnz = 0;
  int32_t *sp_rp = nullptr, *sp_ci = nullptr, *st_rp = nullptr, *st_ci = nullptr;
  double *sp_v64 = nullptr, *st_v64 = nullptr;
  float *sp_v32 = nullptr, *st_v32 = nullptr;
  // levels with long rows (the denser coarse levels of smoothed aggregation):
  // A in CSR in the solve numbering, for kernels with several lanes per row
  int32_t *lr_rp = nullptr, *lr_ci = nullptr;
  double *lr_v64 = nullptr;
  float *lr_v32 = nullptr;
  int32_t sweeps = 0;
  int32_t rounds = 0;
};

struct Coarse {
  int32_t n = 0;
  double *Linv = nullptr;   // L^-1, row-major n x n (lower triangular)
  double *Ainv = nullptr;   // A_L^-1 = L^-T L^-1, row-major n x n
};

// Multi-right-hand-side state: n_l x k row-major blocks on every level, the
// FP64 CG blocks on level 0 and per-column CG scalars.
struct Batch {
  int32_t k = 0;
  int32_t kt = 0;  // autotuned column tile of the one-value kernels (rows per
                   // wavefront = 64 / kt)
  int32_t vshift = 0;  // autotuned: the vector kernels (2 FP64 or 4 FP32 columns per
                       // lane, kv vectors per row) use tiles of row_tile(kv) x 2^vshift
  std::vector<void *> r, z, t, y;  // per level, hierarchy precision
  // level-0 CG blocks, rows in the aggregate-major order of level 0
  double *X = nullptr, *Bp = nullptr, *R = nullptr, *Z = nullptr, *P = nullptr, *Q = nullptr;
  // FP32 hierarchy only: float(R), kept by whichever kernel writes R, so the
  // level-0 kernels that only use R rounded to FP32 gather 4-byte entries
  float *Rf = nullptr;
  // FP32 hierarchy, k a multiple of 4: the V-cycle's output z. The level-0
  // post-smoothing computes it in FP32, so the FP32 store holds the same
  // numbers as the FP64 block Z in half the bytes (written once, read by
  // p = z + beta p)
  float *Zf = nullptr;
  double *partials = nullptr;  // 2 x kBatchBlocks x k
  double *col = nullptr;       // per-column scalars, 8 x k (see batch.hip)
  int32_t *iter = nullptr, *done = nullptr, *all_done = nullptr;
  // per column: 1 while the iteration's x += alpha p is still to be applied
  // (by p = z + beta p in the two-column form, which reads p anyway)
  int32_t *xpend = nullptr;
  double *col_host = nullptr;  // pinned mirrors
  int32_t *iter_host = nullptr, *done_host = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<void *> allocs;
  size_t bytes = 0;
};

void free_batch(Batch *b, int device, hipStream_t s);  // releases on stream s

}  // namespace amg

struct amg_hierarchy {
  int device = 0;
  hipStream_t stream = nullptr;       // the library's own work stream
  hipStream_t user_stream = nullptr;  // amg_params.stream (NULL: default stream)
  hipEvent_t join_event = nullptr;    // orders the work stream after the caller's
  amg_params params{};
  std::vector<amg::Level> lv;
  amg::Coarse C;
  // outer PCG state (FP64, level-0 size)
  // CG vectors, in the aggregate-major order of level 0
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *b = nullptr;
  int32_t max_seg = 1;            // largest aggregate (segment) of any level
  double *partials = nullptr;     // kPartPlanes x kMaxParts block partial sums
  double *kscal = nullptr;  // K-cycle scalars, kKScal per level
  amg::PcgScal *scal = nullptr;   // device
  amg::PcgScal *scal_host = nullptr;  // pinned mirror
  void *setup_arena = nullptr;  // the running setup's temporaries (setup.hip), else null
  int32_t *zero_flag = nullptr;   // device int 0 (for kernels outside CG)
  // batch (multi-right-hand-side) solve state, allocated for the last k used
  amg::Batch *batch = nullptr;
  size_t batch_bytes = 0;
  // graph of one CG iteration
  hipGraphExec_t iter_exec = nullptr;  // one CG iteration
  hipGraph_t iter_graph = nullptr;
  hipGraphExec_t iter_exec4 = nullptr;  // kIterGroup CG iterations
  hipGraph_t iter_graph4 = nullptr;
  bool graph_failed = false;
  // in-solve kernel timing (amg_time_kernel with AMG_TIME_IN_SOLVE): while
  // probe_id names a kernel, events are recorded right before and after each
  // of its launches, pairwise into probe_ev
  int32_t probe_id = -1;
  mutable bool probe_armed = false;  // the next probed launch is the timed one
  std::vector<hipEvent_t> probe_ev;
  mutable size_t probe_next = 0;
  bool has_rhs = false;  // a right-hand side was given to amg_pcg_solve
  // AMG_ASYNC: the solve in flight runs on this host thread (joined by
  // amg_wait, or by the next call on the hierarchy); its status is kept here
  std::thread worker;
  bool async_pending = false;
  std::atomic<int> async_finished{0};
  amg_status async_status = AMG_OK;
  // bookkeeping: the pool blocks the hierarchy's arrays are cut from (see
  // dev_alloc), the bytes requested, and the free tail of the current block
  std::vector<void *> allocs;
  size_t bytes = 0;
  char *block_cur = nullptr;
  size_t block_left = 0;
  double setup_ms[8] = {0};
};

namespace amg {

// allocation owned by the hierarchy (freed in amg_free)
// Device memory of the library comes from one stream-ordered pool per device
// (allocation and release are ordered on the given stream and never wait for
// the whole device, unlike hipFree); freed memory up to kPoolKeepBytes stays
// reserved in the pool for reuse. Without pool support: hipMalloc / hipFree.
constexpr uint64_t kPoolKeepBytes = 8ull << 30;
amg_status stream_alloc(int device, hipStream_t s, void **p, size_t bytes);
void stream_free(int device, hipStream_t s, void *p);
amg_status dev_alloc(amg_hierarchy *h, void **p, size_t bytes);
template <typename T>
inline amg_status dalloc(amg_hierarchy *h, T **p, size_t count) {
  return dev_alloc(h, reinterpret_cast<void **>(p), count * sizeof(T) + 16);
}

// orders the work stream after everything queued so far on the caller's stream
amg_status join_user_stream(amg_hierarchy *h);

// exclusive prefix sum of n int32 values; writes n + 1 outputs (out[n] = total)
amg_status scan_exclusive_i32(const int32_t *in, int32_t *out, int32_t n, hipStream_t s);

// temporaries of a setup step: cut from the running setup's arena (releasing
// them is then a no-op), else stream-ordered pool memory; and the same scan
// with its block sums taken that way
amg_status setup_tmp_alloc(amg_hierarchy *h, void **p, size_t bytes);
void setup_tmp_free(amg_hierarchy *h, void *p);
amg_status setup_scan(amg_hierarchy *h, const int32_t *in, int32_t *out, int32_t n);

// setup (setup.hip)
amg_status build_hierarchy(amg_hierarchy *h, const amg_csr *A);

// smoothed aggregation (smooth.hip): Pbar of level F from its matrix and the
// composed tentative prolongator (agg, p; nc columns), kept in F, and the next
// level's matrix Pbar^T A Pbar in hierarchy-owned arrays
amg_status smooth_level(amg_hierarchy *h, Level &F, int32_t nc, const int32_t *agg,
                        const double *p, int32_t **rp, int32_t **ci, double **val,
                        int64_t *nnz);
// Pbar and Pbar^T of level l in the solve numbering (needs both levels' perms)
amg_status smooth_solve_format(amg_hierarchy *h, int32_t l, bool fp32);
// level l's A as CSR in the solve numbering (the long-row kernels' format)
amg_status long_row_csr(amg_hierarchy *h, int32_t l, bool fp32);

// solve-phase helpers (solve.hip)
amg_status build_solve_formats(amg_hierarchy *h);
amg_status vcycle(amg_hierarchy *h, const double *r, double *z, bool fuse_dot, const int32_t *done);
amg_status pcg(amg_hierarchy *h, const double *b, double *x, double rtol, int32_t maxit,
               amg_solve_info *info, bool use_graph = true);
// allocation-free solve (noalloc.hip): the solve's scratch in a file-scope
// device array whose address amg_setup looks up once per device
amg_status init_noalloc_scratch(int device);
amg_status pcg_noalloc(amg_hierarchy *h, const double *b, double *x, double rtol, int32_t maxit,
                       amg_solve_info *info);
amg_status pcg_batch(amg_hierarchy *h, int32_t k, const double *B, double *X, double rtol,
                     int32_t maxit, amg_solve_info *info);
amg_status batch_kt(const amg_hierarchy *h, int32_t *kt, int32_t *vshift);
amg_status time_kernel(amg_hierarchy *h, int32_t kernel, int32_t level, int32_t reps,
                       double *ms, double *bytes);

// Streaming load: each matrix value and column index is used once per SpMV,
// so it is loaded with the nontemporal hint and does not evict the gathered
// vector entries from L2 (measured on the 160^3 level-0 smoother: 4.8 ->
// 5.7 TB/s).
template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) {
  return __builtin_nontemporal_load(p);
}

// sum_k val[k] * x(col[k]) over one SELL row, in entry order. Each group of
// up to eight entries issues all its index and value loads, then all its
// gathers, before the first product, so that eight loads per lane are in
// flight instead of one. The loads of a group are unconditional: positions
// past the row's last entry re-read that entry (same cache line) and their
// products are not added, so no load sits behind a branch and no use of a
// loaded value (such as the FP32 -> FP64 conversion of a stored FP32 value)
// forces a wait before the next load is issued.
constexpr int kRowBatch = 8;
// (TA: the stored value type, converted exactly to the accumulation type TV;
// FP32-stored values are used only where every value is an FP32 number)
template <typename TV, typename TA, typename X>
__device__ __forceinline__ TV sell_dot_t(const int32_t *__restrict__ col,
                                         const TA *__restrict__ val, int32_t base, int32_t w,
                                         X x) {
  TV acc = 0;
  for (int32_t k0 = 0; k0 < w; k0 += kRowBatch) {
    int32_t c[kRowBatch];
    TA va[kRowBatch];
    TV g[kRowBatch];
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      const int32_t idx = base + (k0 + u < w ? k0 + u : w - 1) * kSlice;
      c[u] = ld_stream(&col[idx]);
      va[u] = ld_stream(&val[idx]);
    }
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) g[u] = x(c[u]);
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u)
      if (k0 + u < w) acc += (TV)va[u] * g[u];
  }
  return acc;
}

template <typename TV, typename X>
__device__ __forceinline__ TV sell_dot(const int32_t *__restrict__ col, const TV *__restrict__ val,
                                       int32_t base, int32_t w, X x) {
  return sell_dot_t<TV, TV>(col, val, base, w, x);
}

// grid helpers
inline int32_t ceil_div(int64_t a, int64_t b) { return (int32_t)((a + b - 1) / b); }

// XCD-aware block index: blocks are dispatched round-robin over the XCDs, so
// block b runs on XCD b % 8. Remap so that each XCD owns a contiguous range of
// logical blocks (neighbouring rows share that XCD's L2).
__device__ __forceinline__ int32_t xcd_block(int32_t b, int32_t nb) {
  int32_t per = nb / kNumXcd;
  if (per == 0) return b;
  int32_t full = per * kNumXcd;
  if (b >= full) return b;
  return (b % kNumXcd) * per + b / kNumXcd;
}

}  // namespace amg
