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
int rast_workspace_bytes(const fgs_gaussians *g, const fgs_geom *geom, int32_t view_count, const fgs_opts *o,
                         bool forward, uint64_t *fixed_bytes, uint64_t *bytes_per_key);
int vox_workspace_bytes(const fgs_gaussians *g, const fgs_grid *grid, bool forward, uint64_t *fixed_bytes,
                        uint64_t *bytes_per_key);

}  // namespace fgs

extern "C" const char *fgs_last_error(void) { return fgs::g_last_error.c_str(); }

extern "C" const char *fgs_version(void) { return "factgs-gfx950 0.1"; }

extern "C" int fgs_binning_layout(const fgs_workspace *ws, uint64_t off[9], uint64_t counts[3]) {
  if (!ws || !off || !counts) return fgs::fail(FGS_E_INVALID, "null argument");
  if (ws->kind == 1 || ws->kind == 3) return fgs::rast_binning_layout(ws, off, counts);
  if (ws->kind == 2) return fgs::vox_binning_layout(ws, off, counts);
  return fgs::fail(FGS_E_INVALID, "workspace holds no lists");
}

extern "C" int fgs_workspace_query(int32_t op, const fgs_gaussians *g, const fgs_geom *geom, const fgs_grid *grid,
                                   int32_t view_count, const fgs_opts *opts, uint64_t *fixed_bytes,
                                   uint64_t *bytes_per_key) {
  if (!fixed_bytes || !bytes_per_key) return fgs::fail(FGS_E_INVALID, "null output");
  switch (op) {
    case FGS_OP_PROJECT_FWD:
    case FGS_OP_PROJECT_BWD:
      return fgs::rast_workspace_bytes(g, geom, view_count, opts, op == FGS_OP_PROJECT_FWD, fixed_bytes,
                                       bytes_per_key);
    case FGS_OP_VOXELIZE_FWD:
    case FGS_OP_VOXELIZE_BWD:
      return fgs::vox_workspace_bytes(g, grid, op == FGS_OP_VOXELIZE_FWD, fixed_bytes, bytes_per_key);
    default:
      return fgs::fail(FGS_E_INVALID, "workspace query: unknown op");
  }
}
