// Error reporting and introspection entry points of libfactgs.
#include "fgs_internal.h"

namespace fgs {

namespace {
thread_local std::string g_last_error = "no error";
}

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return FGS_E_HIP;
}

int rast_binning_layout(const fgs_workspace *ws, uint64_t off[9], uint64_t counts[3]);
int vox_binning_layout(const fgs_workspace *ws, uint64_t off[9], uint64_t counts[3]);

}  // namespace fgs

extern "C" const char *fgs_last_error(void) { return fgs::g_last_error.c_str(); }

extern "C" const char *fgs_version(void) { return "factgs-gfx950 0.1"; }

extern "C" int fgs_binning_layout(const fgs_workspace *ws, uint64_t off[9], uint64_t counts[3]) {
  if (!ws || !off || !counts) return fgs::fail(FGS_E_INVALID, "null argument");
  if (ws->kind == 1 || ws->kind == 3) return fgs::rast_binning_layout(ws, off, counts);
  if (ws->kind == 2) return fgs::vox_binning_layout(ws, off, counts);
  return fgs::fail(FGS_E_INVALID, "workspace holds no lists");
}
