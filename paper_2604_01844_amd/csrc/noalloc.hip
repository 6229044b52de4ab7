// fgs_project_views_fwd_noalloc: the rasterizer forward without a caller
// workspace, for callers that cannot allocate device memory.
//
// The lists, records and partial images live in `scratch`, a file-scope
// device array of kScratchBytes that every GPU the library runs on holds
// (its own copy, at its own address) until the process ends. Host code never
// passes the array's name to a kernel or a copy: that name is a host-side
// stand-in, not a device address. The device address is looked up once per
// device, with that device current, and kept in g_scratch[device].
#include <mutex>

#include "fgs_internal.h"

namespace fgs {
namespace {

constexpr uint64_t kScratchBytes = uint64_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];

// Device address of the current device's copy of `scratch`.
int scratch_for_current_device(void **out) {
  int dev = -1;
  FGS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(FGS_E_UNSUPPORTED, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    FGS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(FGS_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return FGS_OK;
}

}  // namespace
}  // namespace fgs

extern "C" int fgs_project_views_fwd_noalloc(const fgs_gaussians *g, const fgs_geom *geom, int32_t view_begin,
                                             int32_t view_count, const fgs_opts *opts, float *img,
                                             void *stream) {
  void *p = nullptr;
  int st = fgs::scratch_for_current_device(&p);
  if (st != FGS_OK) return st;
  fgs_workspace ws{};
  ws.ptr = p;
  ws.bytes = fgs::kScratchBytes;
  st = fgs_project_views_fwd(g, geom, view_begin, view_count, opts, img, &ws, stream);
  if (st == FGS_E_CAPACITY)
    return fgs::fail(FGS_E_CAPACITY,
                     "this call needs at least " + std::to_string((unsigned long long)ws.needed) +
                         " bytes of scratch; the library's fixed scratch holds " +
                         std::to_string((unsigned long long)fgs::kScratchBytes) +
                         " (64 MiB): split the views or call fgs_project_views_fwd with a workspace");
  return st;
}
