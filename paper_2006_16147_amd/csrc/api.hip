// C ABI of the library (include/amg.h): argument checks, hierarchy lifetime,
// introspection. The numerical work is in setup.hip, solve.hip and batch.hip.

#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <system_error>
#include <thread>

#include "internal.h"

namespace amg {

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_pool_mu;
hipMemPool_t g_pool[kMaxDevices] = {};
bool g_pool_tried[kMaxDevices] = {};

// The library's pool on `device`, created on first use; null if the device
// or runtime has no stream-ordered allocator.
hipMemPool_t lib_pool(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_pool_mu);
  if (!g_pool_tried[device]) {
    g_pool_tried[device] = true;
    int supported = 0;
    if (hipDeviceGetAttribute(&supported, hipDeviceAttributeMemoryPoolsSupported, device) !=
            hipSuccess ||
        !supported) {
      (void)hipGetLastError();
      return nullptr;
    }
    hipMemPoolProps props;
    std::memset(&props, 0, sizeof(props));
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = device;
    hipMemPool_t pool = nullptr;
    if (hipMemPoolCreate(&pool, &props) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    uint64_t keep = kPoolKeepBytes;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    g_pool[device] = pool;
  }
  return g_pool[device];
}

}  // namespace

amg_status stream_alloc(int device, hipStream_t s, void **p, size_t bytes) {
  *p = nullptr;
  hipMemPool_t pool = lib_pool(device);
  if (pool) AMG_HIP(hipMallocFromPoolAsync(p, bytes, pool, s));
  else AMG_HIP(hipMalloc(p, bytes));
  return AMG_OK;
}

void stream_free(int device, hipStream_t s, void *p) {
  if (!p) return;
  if (lib_pool(device)) (void)hipFreeAsync(p, s);
  else (void)hipFree(p);
}

namespace {
// Gives the pool's unused memory beyond kPoolKeepBytes back to the device
// (called once a hierarchy's frees have completed): the release threshold
// alone is not relied on to shrink the pool, and a serving loop that builds
// and evicts hierarchies of many sizes would otherwise leave the device's
// memory held by freed blocks.
void pool_trim(int device) {
  hipMemPool_t pool = lib_pool(device);
  if (pool && hipMemPoolTrimTo(pool, kPoolKeepBytes) != hipSuccess) (void)hipGetLastError();
}
}  // namespace

// The hierarchy's arrays are cut in order from pool blocks of 64 bytes per
// level-0 row (1 to 64 MB), larger arrays getting blocks of their own: on this
// runtime each stream-ordered pool allocation costs tens of microseconds of
// host time, and a setup makes about two hundred of them. Everything is
// released together in amg_free.
amg_status dev_alloc(amg_hierarchy *h, void **p, size_t bytes) {
  *p = nullptr;
  const size_t b = (bytes + 255) / 256 * 256;
  const double rows = h->lv.empty() ? 0.0 : (double)h->lv[0].n;
  const double mb = double(1 << 20);
  const size_t block = (size_t)std::min(64 * mb, std::max(mb, 64.0 * rows)) / (1 << 20) * (1 << 20);
  if (b > block / 4) {
    void *q = nullptr;
    AMG_TRY(stream_alloc(h->device, h->stream, &q, b));
    h->allocs.push_back(q);
    h->bytes += bytes;
    *p = q;
    return AMG_OK;
  }
  if (b > h->block_left) {
    void *q = nullptr;
    AMG_TRY(stream_alloc(h->device, h->stream, &q, block));
    h->allocs.push_back(q);
    h->block_cur = static_cast<char *>(q);
    h->block_left = block;
  }
  *p = h->block_cur;
  h->block_cur += b;
  h->block_left -= b;
  h->bytes += bytes;
  return AMG_OK;
}

amg_status join_user_stream(amg_hierarchy *h) {
  AMG_HIP(hipEventRecord(h->join_event, h->user_stream));
  AMG_HIP(hipStreamWaitEvent(h->stream, h->join_event, 0));
  return AMG_OK;
}

}  // namespace amg

using namespace amg;

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Makes `device` current for the guard's lifetime and then restores the
// caller's current device.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int device) {
    if (hipGetDevice(&prev) != hipSuccess) {
      (void)hipGetLastError();
      prev = -1;
      return;
    }
    ok = prev == device || hipSetDevice(device) == hipSuccess;
    if (!ok) (void)hipGetLastError();
  }
  ~DeviceGuard() {
    if (ok && prev >= 0) (void)hipSetDevice(prev);
  }
};

// Joins the solve in flight (AMG_ASYNC); its status stays in async_status
// for amg_wait.
void join_async(const amg_hierarchy *hc) {
  amg_hierarchy *h = const_cast<amg_hierarchy *>(hc);
  if (h->async_pending) {
    if (h->worker.joinable()) h->worker.join();
    h->async_pending = false;
  }
}

// True when p is device memory on `device` and, where the runtime reports
// the allocation's range, [p, p + bytes) lies inside it.
bool device_range(const void *p, size_t bytes, int device) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged) return false;
  if (a.device != device) return false;
  void *base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void *>(p)) != hipSuccess) {
    (void)hipGetLastError();
    return true;  // range unknown to the runtime: nothing more to check
  }
  const uintptr_t lo = reinterpret_cast<uintptr_t>(base), q = reinterpret_cast<uintptr_t>(p);
  return q >= lo && bytes <= size - (q - lo);
}

void destroy(amg_hierarchy *h) {
  if (!h) return;
  join_async(h);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->iter_exec) (void)hipGraphExecDestroy(h->iter_exec);
  if (h->iter_graph) (void)hipGraphDestroy(h->iter_graph);
  if (h->iter_exec4) (void)hipGraphExecDestroy(h->iter_exec4);
  if (h->iter_graph4) (void)hipGraphDestroy(h->iter_graph4);
  if (h->batch) free_batch(h->batch, h->device, h->stream);
  for (void *p : h->allocs) stream_free(h->device, h->stream, p);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  pool_trim(h->device);
  if (h->scal_host) (void)hipHostFree(h->scal_host);
  if (h->join_event) (void)hipEventDestroy(h->join_event);
  if (h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

amg_status check_params(const amg_params *p) {
  if (p->sweeps < 1 || p->sweeps > 8) return AMG_ERR_ARG;
  if (p->max_coarse < 1 || p->max_coarse > AMG_MAX_DENSE) return AMG_ERR_ARG;
  if (p->max_levels < 1 || p->max_levels > 64) return AMG_ERR_ARG;
  if (p->pre < 1 || p->pre > 8 || p->post < 1 || p->post > 8) return AMG_ERR_ARG;
  if (p->precision != AMG_FP64 && p->precision != AMG_FP32) return AMG_ERR_ARG;
  if (p->cycle != AMG_CYCLE_V && p->cycle != AMG_CYCLE_K) return AMG_ERR_ARG;
  if (p->w_sweeps < 0 || p->w_sweeps > 1000) return AMG_ERR_ARG;
  if (p->coarse_solver != AMG_COARSE_CHOLESKY && p->coarse_solver != AMG_COARSE_PCG)
    return AMG_ERR_ARG;
  if (p->smooth_p != 0 && p->smooth_p != 1) return AMG_ERR_ARG;
  if (p->device < -1) return AMG_ERR_ARG;
  if (p->flags & ~(AMG_FLAG_NO_GRAPH | AMG_FLAG_SKIP_CHECKS | AMG_FLAG_NO_VALUE_COMPRESSION |
                   AMG_ASYNC))
    return AMG_ERR_ARG;
  if (p->smooth_p && p->cycle != AMG_CYCLE_V) return AMG_ERR_ARG;
  if (p->coarse_solver == AMG_COARSE_PCG &&
      (p->coarse_maxit < 1 || p->coarse_maxit > 10000 || !(p->coarse_rtol >= 0.0) ||
       !std::isfinite(p->coarse_rtol)))
    return AMG_ERR_ARG;
  return AMG_OK;
}

// Starts `solve` on the hierarchy's worker thread (AMG_ASYNC) or runs it.
template <typename F>
amg_status run_solve(amg_hierarchy *h, F solve) {
  if (!(h->params.flags & AMG_ASYNC)) return solve();
  h->async_status = AMG_OK;
  h->async_finished.store(0);
  try {
    h->worker = std::thread([h, solve]() {
      amg_status st = hipSetDevice(h->device) == hipSuccess ? solve() : AMG_ERR_HIP;
      h->async_status = st;
      h->async_finished.store(1);
    });
  } catch (const std::system_error &) {
    return AMG_ERR_HIP;
  }
  h->async_pending = true;
  return AMG_OK;
}

}  // namespace

extern "C" {

void amg_params_default(amg_params *p) {
  if (!p) return;
  p->sweeps = 3;
  p->max_coarse = 200;
  p->max_levels = 32;
  p->pre = 1;
  p->post = 1;
  p->precision = AMG_FP64;
  p->w = nullptr;
  p->stream = nullptr;
  p->flags = 0;
  p->cycle = AMG_CYCLE_V;
  p->w_sweeps = 0;
  p->coarse_solver = AMG_COARSE_CHOLESKY;
  p->coarse_maxit = 30;
  p->coarse_rtol = 1e-4;
  p->smooth_p = 0;
  p->device = -1;
}

amg_status amg_setup(const amg_csr *A, const amg_params *params, amg_hierarchy **out) {
  if (!out) return AMG_ERR_ARG;
  *out = nullptr;
  if (!A || A->n < 1 || A->n > INT32_MAX - 1 || A->nnz < A->n || A->nnz > INT32_MAX)
    return AMG_ERR_ARG;
  amg_params P;
  if (params) P = *params;
  else amg_params_default(&P);
  AMG_TRY(check_params(&P));
  int device = P.device;
  if (device < 0) {
    if (hipGetDevice(&device) != hipSuccess) return AMG_ERR_HIP;
  } else {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return AMG_ERR_HIP;
    if (device >= count) return AMG_ERR_ARG;
  }
  DeviceGuard guard(device);
  if (!guard.ok) return AMG_ERR_HIP;
  // set-up of the allocation-free solve: the device address of its scratch
  // array, looked up once per device with that device current
  AMG_TRY(init_noalloc_scratch(device));
  const size_t n1 = (size_t)A->n + 1, nz = (size_t)A->nnz;
  if (!device_range(A->row_ptr, 4 * n1, device) || !device_range(A->col, 4 * nz, device) ||
      !device_range(A->val, 8 * nz, device))
    return AMG_ERR_ARG;
  if (P.w && !device_range(P.w, 8 * (size_t)A->n, device)) return AMG_ERR_ARG;
  amg_hierarchy *h = new (std::nothrow) amg_hierarchy();
  if (!h) return AMG_ERR_OOM;
  h->params = P;
  h->params.w = nullptr;  // not retained after setup
  h->params.device = device;
  h->device = device;
  // all work runs on the library's own stream (default priority), ordered
  // after the caller's stream (NULL: the device's default stream) at every
  // entry point; every entry point returns after its work has completed
  h->user_stream = reinterpret_cast<hipStream_t>(P.stream);
  if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->join_event, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    destroy(h);
    return AMG_ERR_HIP;
  }
  if (join_user_stream(h) != AMG_OK) {
    destroy(h);
    return AMG_ERR_HIP;
  }
  amg_params Pw = P;
  h->params.w = Pw.w;
  amg_status st = build_hierarchy(h, A);
  h->params.w = nullptr;
  if (st != AMG_OK) {
    (void)hipGetLastError();
    destroy(h);
    return st;
  }
  *out = h;
  return AMG_OK;
}

amg_status amg_pcg_solve(amg_hierarchy *h, const double *b, double *x, double rtol,
                         int32_t maxit, amg_solve_info *info) {
  if (!h || !b || !x || !(rtol >= 0.0) || maxit < 0) return AMG_ERR_ARG;
  join_async(h);
  DeviceGuard guard(h->device);
  if (!guard.ok) return AMG_ERR_HIP;
  const size_t bytes = sizeof(double) * (size_t)h->lv[0].n;
  if (!device_range(b, bytes, h->device) || !device_range(x, bytes, h->device))
    return AMG_ERR_ARG;
  AMG_TRY(join_user_stream(h));
  return run_solve(h, [=]() { return pcg(h, b, x, rtol, maxit, info); });
}

amg_status amg_pcg_solve_noalloc(amg_hierarchy *h, const double *b, double *x, double rtol,
                                 int32_t maxit, amg_solve_info *info) {
  if (!h || !b || !x || !(rtol >= 0.0) || maxit < 0) return AMG_ERR_ARG;
  join_async(h);
  DeviceGuard guard(h->device);
  if (!guard.ok) return AMG_ERR_HIP;
  const size_t bytes = sizeof(double) * (size_t)h->lv[0].n;
  if (!device_range(b, bytes, h->device) || !device_range(x, bytes, h->device))
    return AMG_ERR_ARG;
  AMG_TRY(join_user_stream(h));
  return pcg_noalloc(h, b, x, rtol, maxit, info);
}

amg_status amg_pcg_solve_batch(amg_hierarchy *h, int32_t k, const double *B, double *X,
                               double rtol, int32_t maxit, amg_solve_info *info) {
  if (!h || k < 0 || !(rtol >= 0.0) || maxit < 0) return AMG_ERR_ARG;
  if (h->params.cycle != AMG_CYCLE_V || h->params.coarse_solver != AMG_COARSE_CHOLESKY ||
      h->params.smooth_p)
    return AMG_ERR_ARG;
  if (k == 0) return AMG_OK;
  if (!B || !X) return AMG_ERR_ARG;
  join_async(h);
  DeviceGuard guard(h->device);
  if (!guard.ok) return AMG_ERR_HIP;
  const size_t bytes = sizeof(double) * (size_t)h->lv[0].n * (size_t)k;
  if (!device_range(B, bytes, h->device) || !device_range(X, bytes, h->device))
    return AMG_ERR_ARG;
  AMG_TRY(join_user_stream(h));
  return run_solve(h, [=]() { return pcg_batch(h, k, B, X, rtol, maxit, info); });
}

amg_status amg_wait(amg_hierarchy *h) {
  if (!h) return AMG_ERR_ARG;
  join_async(h);
  const amg_status st = h->async_status;
  h->async_status = AMG_OK;
  return st;
}

amg_status amg_query(amg_hierarchy *h, int32_t *done) {
  if (!h || !done) return AMG_ERR_ARG;
  *done = !h->async_pending || h->async_finished.load() ? 1 : 0;
  return AMG_OK;
}

amg_status amg_vcycle_apply(amg_hierarchy *h, const double *r, double *z) {
  if (!h || !r || !z) return AMG_ERR_ARG;
  join_async(h);
  DeviceGuard guard(h->device);
  if (!guard.ok) return AMG_ERR_HIP;
  const size_t bytes = sizeof(double) * (size_t)h->lv[0].n;
  if (!device_range(r, bytes, h->device) || !device_range(z, bytes, h->device))
    return AMG_ERR_ARG;
  AMG_TRY(join_user_stream(h));
  AMG_TRY(vcycle(h, r, z, false, h->zero_flag));
  AMG_HIP(hipStreamSynchronize(h->stream));
  return AMG_OK;
}

amg_status amg_set_stream(amg_hierarchy *h, void *stream) {
  if (!h) return AMG_ERR_ARG;
  join_async(h);
  h->user_stream = reinterpret_cast<hipStream_t>(stream);
  return AMG_OK;
}

void amg_free(amg_hierarchy *h) {
  if (!h) return;
  DeviceGuard guard(h->device);
  destroy(h);
}

amg_status amg_num_levels(const amg_hierarchy *h, int32_t *nlev) {
  if (!h || !nlev) return AMG_ERR_ARG;
  *nlev = (int32_t)h->lv.size();
  return AMG_OK;
}

amg_status amg_level_info(const amg_hierarchy *h, int32_t l, int64_t *n, int64_t *nnz) {
  if (!h || l < 0 || l >= (int32_t)h->lv.size()) return AMG_ERR_ARG;
  if (n) *n = h->lv[l].n;
  if (nnz) *nnz = h->lv[l].nnz;
  return AMG_OK;
}

namespace {
// device-to-host copy ordered after all of the hierarchy's queued work
// (a solve in flight included)
amg_status d2h(const amg_hierarchy *h, void *dst, const void *src, size_t bytes) {
  join_async(h);
  DeviceGuard guard(h->device);
  if (!guard.ok) return AMG_ERR_HIP;
  AMG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, h->stream));
  AMG_HIP(hipStreamSynchronize(h->stream));
  return AMG_OK;
}
}  // namespace

amg_status amg_get_level_csr(const amg_hierarchy *h, int32_t l, int32_t *rp, int32_t *ci,
                             double *val) {
  if (!h || l < 0 || l >= (int32_t)h->lv.size()) return AMG_ERR_ARG;
  const Level &L = h->lv[l];
  if (rp) AMG_TRY(d2h(h, rp, L.rp, sizeof(int32_t) * (L.n + 1)));
  if (ci) AMG_TRY(d2h(h, ci, L.ci, sizeof(int32_t) * L.nnz));
  if (val) AMG_TRY(d2h(h, val, L.val, sizeof(double) * L.nnz));
  return AMG_OK;
}

amg_status amg_get_aggregates(const amg_hierarchy *h, int32_t l, int32_t *agg) {
  if (!h || !agg || l < 0 || l + 1 >= (int32_t)h->lv.size()) return AMG_ERR_ARG;
  return d2h(h, agg, h->lv[l].agg, sizeof(int32_t) * h->lv[l].n);
}

amg_status amg_get_transfer(const amg_hierarchy *h, int32_t l, int32_t *agg, double *p) {
  if (!h || l < 0 || l + 1 >= (int32_t)h->lv.size()) return AMG_ERR_ARG;
  const Level &L = h->lv[l];
  if (agg) AMG_TRY(d2h(h, agg, L.agg, sizeof(int32_t) * L.n));
  if (p) AMG_TRY(d2h(h, p, L.p64, sizeof(double) * L.n));
  return AMG_OK;
}

amg_status amg_get_prolongator(const amg_hierarchy *h, int32_t l, int64_t *nnz,
                               int32_t *rp, int32_t *ci, double *val, double *omega) {
  if (!h || !nnz || l < 0 || l + 1 >= (int32_t)h->lv.size() || !h->params.smooth_p)
    return AMG_ERR_ARG;
  const Level &L = h->lv[l];
  *nnz = L.pb_nnz;
  if (omega) *omega = L.omega;
  if (rp) AMG_TRY(d2h(h, rp, L.pb_rp, sizeof(int32_t) * (L.n + 1)));
  if (ci) AMG_TRY(d2h(h, ci, L.pb_ci, sizeof(int32_t) * L.pb_nnz));
  if (val) AMG_TRY(d2h(h, val, L.pb_val, sizeof(double) * L.pb_nnz));
  return AMG_OK;
}

amg_status amg_get_l1diag(const amg_hierarchy *h, int32_t l, double *m) {
  if (!h || !m || l < 0 || l >= (int32_t)h->lv.size()) return AMG_ERR_ARG;
  const Level &L = h->lv[l];
  if (!L.m) return AMG_ERR_ARG;  // the coarsest level has one only for the CG coarsest solve
  AMG_TRY(d2h(h, m, L.m, sizeof(double) * L.n));
  return AMG_OK;
}

amg_status amg_get_w(const amg_hierarchy *h, int32_t l, double *w) {
  if (!h || !w || l < 0 || l >= (int32_t)h->lv.size()) return AMG_ERR_ARG;
  const Level &L = h->lv[l];
  AMG_TRY(d2h(h, w, L.w, sizeof(double) * L.n));
  return AMG_OK;
}

size_t amg_footprint_bytes(const amg_hierarchy *h) {
  if (!h) return 0;
  join_async(h);
  return h->bytes + h->batch_bytes;
}

size_t amg_estimate_footprint(int64_t n, int64_t nnz, const amg_params *params) {
  amg_params P;
  if (params) P = *params;
  else amg_params_default(&P);
  const double V = P.precision == AMG_FP32 ? 4.0 : 8.0;
  const double X = P.precision == AMG_FP32 ? 4.0 : 0.0;  // FP32 copies kept beside FP64
  // geometric bound of the level sizes (coarsening by >= 2 per sweep)
  const double shrink = 1.0 / (1 << (P.sweeps < 1 ? 1 : P.sweeps));
  const double sn = n / (1.0 - shrink), sz = nnz / (1.0 - shrink);
  // SELL padding: ~1 % on the stencil rows of level 0, up to 30 % on Galerkin levels
  const double pad = 1.02 * nnz + 1.3 * (sz - nnz);
  double b = 0;
  b += sz * (4 + 8) + sn * 4;                   // FP64 CSR of every level
  b += sn * (3 * 8 + 4 + 8 + 4 + 4);            // w, m, 1/m, agg, p, mptr, mem
  b += sn * (4 * 4 + 8) + sn * 2 * X;           // perm, iperm, seg, aggp, pp (+ FP32 pp, 1/m)
  b += pad * (4 + 2 * 8 + 2 * X);               // SELL: columns, A, A M^-1 (+ FP32 copies)
  b += 4.0 * 1.02 * nnz;                        // exact FP32 copy of A_0 (when it applies)
  b += 2 * (2.0 * 1.02 * nnz + 4.0 * 2.5 * n);  // level 0's two sets of LDS tile lists
  b += 4 * V * sn;                              // V-cycle vectors
  b += 6 * 8.0 * n;                             // CG vectors (x, r, z, p, q, b)
  b += (double)kPartPlanes * kMaxParts * 8.0;   // block partials
  if (P.cycle == AMG_CYCLE_K) b += 5 * V * (sn - n);  // K-cycle FCG vectors
  // the setup's temporaries (weights, matching state, Galerkin staging, sweep
  // matrices), all held until the setup ends: about twice the first sweep's,
  // plus one partly used arena block (a quarter of the first sweep's)
  b += 2 * (46.0 * n + 28.0 * nnz) + (36.0 * n + 32.0 * nnz) / 4;
  const double nL = P.max_coarse;
  b += 3 * 8.0 * nL * nL;
  if (P.smooth_p) {
    // denser coarse levels (operator complexity up to ~2.2 on 7-point rows,
    // CSR + SELL), Pbar three times (~4 entries per fine row), long-row CSR
    b += 1.4 * nnz * (2 * 12.0 + 8 + 2 * X);
    b += 3 * 4.0 * n * (12.0 + X) + 4 * 3 * sn;
  }
  return (size_t)(b + (1 << 20));
}

amg_status amg_setup_times(const amg_hierarchy *h, double *ms) {
  if (!h || !ms) return AMG_ERR_ARG;
  join_async(h);
  for (int k = 0; k < 8; ++k) ms[k] = h->setup_ms[k];
  return AMG_OK;
}

amg_status amg_matching_rounds(const amg_hierarchy *h, int32_t l, int32_t *rounds) {
  if (!h || !rounds || l < 0 || l >= (int32_t)h->lv.size()) return AMG_ERR_ARG;
  *rounds = h->lv[l].rounds;
  return AMG_OK;
}

amg_status amg_time_kernel(amg_hierarchy *h, int32_t kernel, int32_t level, int32_t reps,
                           double *ms, double *bytes) {
  const int32_t base = kernel & ~AMG_TIME_IN_SOLVE;
  if (!h || !ms || !bytes || kernel < 0 || base > 5) return AMG_ERR_ARG;
  join_async(h);
  DeviceGuard guard(h->device);
  if (!guard.ok) return AMG_ERR_HIP;
  AMG_TRY(join_user_stream(h));
  return time_kernel(h, kernel, level, reps, ms, bytes);
}

amg_status amg_batch_tile(const amg_hierarchy *h, int32_t *kt, int32_t *vshift) {
  if (!h || !kt) return AMG_ERR_ARG;
  join_async(h);
  return batch_kt(h, kt, vshift);
}

const char *amg_status_string(amg_status s) {
  switch (s) {
    case AMG_OK: return "ok";
    case AMG_ERR_ARG: return "invalid argument";
    case AMG_ERR_NOT_SYMMETRIC: return "matrix is not symmetric";
    case AMG_ERR_NOT_SPD: return "matrix is not positive definite";
    case AMG_ERR_STALL: return "coarsening stalled above the dense limit";
    case AMG_ERR_OOM: return "out of device memory";
    case AMG_ERR_HIP: return "HIP runtime error";
    case AMG_ERR_BREAKDOWN: return "CG breakdown";
    case AMG_NOT_CONVERGED: return "not converged";
  }
  return "unknown status";
}

}  // extern "C"
