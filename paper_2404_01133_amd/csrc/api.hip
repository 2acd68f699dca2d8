// Library-wide helpers of the C ABI: status strings, workspace sizes.
#include <stdio.h>

#include "gs_common.h"

namespace gs {

size_t bin_sort_ws_bytes(int64_t rc, int64_t pc);
size_t rasterize_bwd_ws_bytes(int64_t rc, int64_t pc, bool det);

static thread_local char g_err[256];

gs_status set_hip_error(hipError_t e) {
  snprintf(g_err, sizeof(g_err), "GS_ERR_HIP: %s (%s)", hipGetErrorName(e), hipGetErrorString(e));
  return GS_ERR_HIP;
}

}  // namespace gs

extern "C" size_t gs_record_bytes(void) { return sizeof(gs::Record); }

extern "C" size_t gs_workspace_bytes(int32_t which, int64_t record_capacity, int64_t pair_capacity, int32_t n_views,
                                     int32_t width, int32_t height, const gs_tuning* tuning) {
  (void)n_views;
  (void)width;
  (void)height;
  if (record_capacity < 0 || pair_capacity < 0) return 0;
  if (which == GS_WS_BIN_SORT) return gs::bin_sort_ws_bytes(record_capacity, pair_capacity);
  if (which == GS_WS_RASTERIZE_BWD)
    return gs::rasterize_bwd_ws_bytes(record_capacity, pair_capacity,
                                      tuning && (tuning->flags & GS_TUNE_DETERMINISTIC) != 0);
  return 0;
}

extern "C" const char* gs_status_string(gs_status status) {
  switch (status) {
    case GS_OK: return "GS_OK";
    case GS_ERR_INVALID_ARG: return "GS_ERR_INVALID_ARG: a pointer is NULL or a size/shape is out of range";
    case GS_ERR_UNSUPPORTED: return "GS_ERR_UNSUPPORTED: tile shape or batch not supported";
    case GS_ERR_WORKSPACE: return "GS_ERR_WORKSPACE: workspace smaller than gs_workspace_bytes()";
    case GS_ERR_CAPACITY: return "GS_ERR_CAPACITY: a record or pair capacity was exceeded";
    case GS_ERR_HIP: return gs::g_err[0] ? gs::g_err : "GS_ERR_HIP";
    case GS_ERR_SCRATCH:
      return "GS_ERR_SCRATCH: the capacities need more workspace than the static scratch array holds";
    default: return "unknown gs_status";
  }
}
