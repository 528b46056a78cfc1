// Allocation-free variant of the single solve (amg_pcg_solve_noalloc).
//
// amg_pcg_solve keeps its scratch in hierarchy buffers: the block partial
// sums of every reduction (kPartPlanes x kMaxParts doubles), the CG scalars
// and, for the K-cycle, the per-level flexible-CG scalars; and on its first
// call it instantiates the CG-iteration graph, which may allocate. The
// variant takes that scratch from one file-scope device array instead and
// launches the iterations directly, so the call itself allocates nothing:
// no hipMalloc / hipFree, no pool or graph allocation, no pinned host buffer
// (the host mirror of the scalars is the one amg_setup made).
//
// The array is the same for every hierarchy on a device and keeps the last
// call's contents; each call clears the scalars it needs before use. Calls
// on one device that overlap in time (two host threads, or two streams)
// race on it.

#include <mutex>

#include "internal.h"

namespace amg {

namespace {

// layout of the scratch array, in doubles (each region 256-byte aligned)
constexpr size_t kAlign = 256 / sizeof(double);
constexpr size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
constexpr size_t kPartialsAt = 0;
constexpr size_t kPartialsLen = (size_t)kPartPlanes * kMaxParts;
constexpr size_t kScalAt = round_up(kPartialsAt + kPartialsLen);
constexpr size_t kScalLen = round_up((sizeof(PcgScal) + sizeof(double) - 1) / sizeof(double));
constexpr size_t kKScalAt = kScalAt + kScalLen;
constexpr int32_t kKScalLevels = 64;  // amg_params.max_levels is at most 64
constexpr size_t kKScalLen = round_up((size_t)kKScal * kKScalLevels);
constexpr size_t kScratchLen = kKScalAt + kKScalLen;

constexpr int kMaxDevices = 64;

}  // namespace

}  // namespace amg

// the solve's scratch on every device that loads the library (~1.6 MB)
static __device__ __align__(256) double scratch[amg::kScratchLen];

namespace amg {

namespace {

std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

__global__ void k_zero(double *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// Points the hierarchy's scratch pointers at the device array for the
// lifetime of the object and restores them afterwards.
struct ScratchBinding {
  amg_hierarchy *h;
  double *partials, *kscal;
  PcgScal *scal;
  ScratchBinding(amg_hierarchy *hh, double *base)
      : h(hh), partials(hh->partials), kscal(hh->kscal), scal(hh->scal) {
    h->partials = base + kPartialsAt;
    h->scal = reinterpret_cast<PcgScal *>(base + kScalAt);
    if (h->kscal) h->kscal = base + kKScalAt;
  }
  ~ScratchBinding() {
    h->partials = partials;
    h->kscal = kscal;
    h->scal = scal;
  }
};

}  // namespace

// Device address of the scratch array on `device` (current), looked up once
// per device; amg_setup calls it, so the lookup happens at set-up time.
amg_status init_noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return AMG_ERR_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return AMG_OK;
  void *ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return AMG_ERR_HIP;
  }
  g_scratch[device] = static_cast<double *>(ptr);
  return AMG_OK;
}

amg_status pcg_noalloc(amg_hierarchy *h, const double *b, double *x, double rtol, int32_t maxit,
                       amg_solve_info *info) {
  double *base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (h->device >= 0 && h->device < kMaxDevices) base = g_scratch[h->device];
  }
  if (!base) return AMG_ERR_HIP;  // amg_setup found no device address for it
  const int32_t nlev = (int32_t)h->lv.size();
  if (nlev > kKScalLevels) return AMG_ERR_ARG;  // cannot happen: max_levels <= 64
  // the CG scalars and the K-cycle scalars start from zero, as the
  // hierarchy's own buffers do after amg_setup (a fill kernel, not a memset
  // node, so that the sequence stays valid in a captured stream too)
  const int64_t clear = (int64_t)(kScratchLen - kScalAt);
  k_zero<<<(unsigned)((clear + 255) / 256), 256, 0, h->stream>>>(base + kScalAt, clear);
  AMG_HIP(hipGetLastError());
  ScratchBinding bind(h, base);
  return pcg(h, b, x, rtol, maxit, info, /*use_graph=*/false);
}

}  // namespace amg
