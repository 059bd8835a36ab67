// Host-side helpers shared by the C-ABI translation units (validation, workspace layout).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/idw.h"
#include "idw_launch.hpp"

namespace idw {

// Byte offsets of the workspace sections and the launch shape chosen for a problem.
struct WsPlan {
  int qf = 8, split_f = 1;
  int64_t chunk_f = 0;
  int qq = 4, split_q = 1;
  int64_t chunk_q = 0;
  int qz = 8, split_z = 1;
  int64_t chunk_z = 0;
  int nbbox = 1, nwg_dp = 1;
  int fused_groups = 0, fused_ranges = 0;  // fused FP32 adjoint decomposition
  int64_t fused_chunk = 0;
  size_t hdr = 0, bbox = 0, flag = 0, bcnt = 0, list = 0, near_min = 0, part_f = 0, part_q = 0, part_z = 0;
  size_t slot_coef = 0, slot_hits = 0, slot_dp = 0, slot_z = 0, slot_den = 0, fpart = 0, wg_dp = 0;
  size_t fwd_total = 0;  // bytes the forward needs (a prefix of the full layout)
  size_t total = 0;      // bytes forward + backward need
  size_t part_x = 0;     // data-coordinate partials, after everything else
  size_t total_x = 0;    // bytes forward + backward need with the data-coordinate gradient
  int fix_cmax = 1;
  // grid of the nearest-distance searches (forward prefix; unused when grid_on is false)
  bool grid_on = false;
  int64_t grid_ncell = 0;  // most cells
  size_t grid_cnt = 0, grid_start = 0, grid_bsum = 0, grid_rec = 0, grid_blist = 0;
};

// Static device scratch of idw_forward_noalloc (the forward's workspace for callers that
// cannot allocate): 64 MiB, enough for the forward at n = m = 2^20 in FP32 (37 MB) and FP64
// (54 MB).
constexpr size_t kScratchBytes = size_t(64) << 20;

int fail(int code, const char* fmt, ...);
void clear_error();
int check_hip(hipError_t e, const char* what);
int check_device();
int validate_points(const idw_points* P, int precision, bool is_data, const char* what);
int validate_common(const idw_points* data, const idw_points* query, double p, int precision,
                    uint32_t flags);
int validate_config(const idw_config* cfg);
int pmode_of(double p);
WsPlan plan_workspace(const idw_points* data, const idw_points* query, int precision,
                      const idw_config* cfg);
DevPts dev_pts(const idw_points* P);
int check_workspace(void* ws, size_t bytes, size_t need);

hipError_t fill_zero(void* p, size_t bytes, hipStream_t st);

}  // namespace idw
