// Host-side launch descriptors shared by the C-ABI layer and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "idw_device.hpp"

namespace idw {

// Everything a forward launch needs; pointers are device pointers.
struct FwdArgs {
  DevPts data;
  int64_t n = 0;
  DevPts query;
  int64_t m = 0;
  int dim = 2;
  int pmode = PM_GEN;
  double p = 2.0;
  unsigned flags = 0;
  int q_per_lane = 8;
  bool kahan = false;  // FP32 sweep with per-pair Kahan compensation
  bool rel = false;    // FP32 relative weights (p >= kRelP): needs rmin
  const unsigned long long* rmin = nullptr;  // [m] nearest squared distance (FP32 bits)
  int split = 1;
  int64_t chunk = 0;  // data points per split chunk (multiple of the tile)
  const double* hdr = nullptr;
  void* out_z = nullptr;
  double* out_den = nullptr;
  uint8_t* flag = nullptr;
  double2* part = nullptr;
  const int* list = nullptr;
  const int* count = nullptr;
  int fix_cmax = 1;              // most data chunks per flagged query in the FP64 fix-up
  double4* fpart = nullptr;      // [kFixGrid] fix-up chunk partials
};

// Everything a backward launch needs.
struct BwdArgs {
  DevPts data;
  int64_t n = 0;
  DevPts query;
  int64_t m = 0;
  int dim = 2;
  int pmode = PM_GEN;
  double p = 2.0;
  unsigned flags = 0;
  int q_per_lane = 4;    // query sweep: queries per lane
  int x_per_lane = 4;    // data sweep: data points per lane
  int split_q = 1;       // data chunks of the query sweep
  int64_t chunk_q = 0;
  int split_z = 1;       // query chunks of the data sweep
  int64_t chunk_z = 0;
  double4* part_q = nullptr;  // [split_q][m] (P, Gx, Gy, Gz)
  double* part_z = nullptr;   // [split_z][n]
  double* part_x = nullptr;   // [split_z][n][dim] data-coordinate sums (null: not requested)
  int fused_groups = 0;       // fused FP32 sweep: query-block groups (= dz partial rows)
  int fused_ranges = 0;       // fused FP32 sweep: data ranges (= query partial rows)
  int64_t fused_chunk = 0;
  const double* hdr = nullptr;
  const void* grad_out = nullptr;
  const void* saved_z = nullptr;
  const double* saved_den = nullptr;
  const uint8_t* route = nullptr;  // [m] settled QueryRoute of each query
  bool rel = false;                // fused FP32 sweep with relative weights (p >= kRelP)
  void* grad_z = nullptr;
  void* grad_q = nullptr;
  void* grad_x = nullptr;
  double* wg_dp = nullptr;      // [num query workgroups] dp partials of the FP32/FP64 sweep
  const int* list = nullptr;    // flagged queries, ascending
  const int* count = nullptr;
  double* slot_coef = nullptr;  // [m] per flagged slot: g/D (or g/h at a hit)
  int* slot_hits = nullptr;     // [m] per flagged slot: hit count h
  double* slot_dp = nullptr;    // [m] per flagged slot: dp contribution
  double* slot_z = nullptr;     // [m] per flagged slot: FP64 Z
  double* slot_den = nullptr;   // [m] per flagged slot: FP64 denominator
  int fix_cmax = 1;
  double4* fpart = nullptr;     // [kFixGrid] fix-up chunk partials
};

// The nearest-distance check of candidate queries (k_near_check).
struct NearArgs {
  DevPts data;
  int64_t n = 0;
  DevPts query;
  int64_t m = 0;  // queries in all (bounds the candidates)
  int dim = 2;
  bool f64 = false;
  bool excl = false;
  const int* list = nullptr;   // candidate query indices
  const int* count = nullptr;  // number of candidates (device)
  const double* hdr = nullptr;
  uint8_t* route = nullptr;    // [m] QueryRoute, settled for the candidates
  unsigned long long* minb = nullptr;  // [m] per-candidate minimum (bits), scratch
  bool all = false;  // every query 0..m-1 (list and count unused); no route is written
};

// The grid of the nearest-distance searches (idw_grid.hpp).
struct GridArgs {
  DevPts data;
  int64_t n = 0;
  DevPts query;
  int64_t m = 0;
  int dim = 2;
  bool f64 = false;
  bool excl = false;
  bool nearest = false;              // search: ring search over all queries, else candidate check
  const double* hdr = nullptr;
  int* hint = nullptr;               // header int slots (flagged count, then GridInt)
  int* cnt = nullptr;                // [ncell_max + 1] cell counts, then scatter cursors
  int* start = nullptr;              // [ncell_max + 1] first record of each cell
  int* bsum = nullptr;               // [scan blocks] block sums of the counts
  int64_t ncell_max = 0;
  void* rec = nullptr;               // [n] P4<T>: scaled coordinates and point index
  const int* list = nullptr;         // candidate check: candidate queries
  uint8_t* route = nullptr;          // candidate check: QueryRoute written per candidate
  unsigned long long* minb = nullptr;  // ring search: nearest squared distance (bits)
  int* blist = nullptr;              // [m] queries handed to the brute-force check
};

constexpr int kTile = 512;        // data points staged in LDS per tile (2 per thread)
constexpr int kFixGrid = 1024;    // workgroups of the FP64 fix-up kernels
constexpr int kCountBlock = 4096; // flags per compaction block (16 per thread)

// Per-layout entry points (one translation unit per layout keeps builds parallel).
#define IDW_DECLARE_LAYOUT(NAME)                                                 \
  hipError_t fwd_sweep_##NAME(const FwdArgs& a, bool f64, hipStream_t st);       \
  hipError_t fwd_fixup_##NAME(const FwdArgs& a, bool f64, hipStream_t st);       \
  hipError_t bbox_##NAME(const DevPts& d, int64_t n, int dim, bool f64, double* part, \
                         int nblocks, hipStream_t st);                           \
  hipError_t bwd_query_##NAME(const BwdArgs& a, bool f64, hipStream_t st);       \
  hipError_t bwd_data_##NAME(const BwdArgs& a, bool f64, hipStream_t st);        \
  hipError_t bwd_datax_##NAME(const BwdArgs& a, bool f64, hipStream_t st);       \
  hipError_t bwd_fixup_##NAME(const BwdArgs& a, bool f64, hipStream_t st);      \
  hipError_t bwd_fused_##NAME(const BwdArgs& a, bool f64, hipStream_t st);       \
  hipError_t near_check_##NAME(const NearArgs& a, hipStream_t st);              \
  hipError_t grid_##NAME(const GridArgs& a, bool build, hipStream_t st);

IDW_DECLARE_LAYOUT(soa)
IDW_DECLARE_LAYOUT(aos)
IDW_DECLARE_LAYOUT(aoas)
IDW_DECLARE_LAYOUT(hybrid)
IDW_DECLARE_LAYOUT(soaos)

// Layout-independent kernels (idw_common.hip).
hipError_t bbox_final(const double* part, int nblocks, int dim, double p, bool f32_scaling,
                      bool rel, double* hdr, hipStream_t st);
hipError_t merge_split(const double2* part, int64_t m, int split, const double* hdr,
                       void* out_z, bool f64, double* out_den, uint8_t* flag, hipStream_t st);
hipError_t compact_flags(const uint8_t* flag, int64_t m, int* bcnt, int* list, int* count,
                         uint8_t want, hipStream_t st);
hipError_t flags_from_den(const double* den, int64_t m, const double* hdr, uint8_t* flag,
                          hipStream_t st);
hipError_t bwd_qmerge(const BwdArgs& a, bool f64, hipStream_t st);
hipError_t bwd_zmerge(const BwdArgs& a, bool f64, hipStream_t st);
hipError_t bwd_xmerge(const BwdArgs& a, int split, bool f64, hipStream_t st);
hipError_t dp_final(const double* wg_dp, int nwg, const double* slot_dp, const int* count,
                    double* grad_p, hipStream_t st);
// Grid geometry and the per-call gates (mode 0: candidate check of hint[0] candidates; mode
// 1: ring search of all m queries), then the exclusive scan of the cell counts.
hipError_t grid_setup(const GridArgs& a, int mode, bool grid_on, hipStream_t st);
hipError_t grid_scan(const GridArgs& a, hipStream_t st);

}  // namespace idw
