// Kernel instantiations for one record layout.  This file is compiled once per layout
// with IDW_LAYOUT (the Layout enum value) and IDW_LAYOUT_NAME (the symbol suffix) defined,
// so the five layouts build as independent translation units.
#include "idw_bwd.hpp"
#include "idw_bwd_fused.hpp"
#include "idw_fwd.hpp"
#include "idw_grid.hpp"
#include "idw_launch.hpp"

#if !defined(IDW_LAYOUT) || !defined(IDW_LAYOUT_NAME)
#error "compile with -DIDW_LAYOUT=<0..4> -DIDW_LAYOUT_NAME=<soa|aos|aoas|hybrid|soaos>"
#endif

#define IDW_CAT2(a, b) a##b
#define IDW_CAT(a, b) IDW_CAT2(a, b)

namespace idw {

hipError_t IDW_CAT(fwd_sweep_, IDW_LAYOUT_NAME)(const FwdArgs& a, bool f64, hipStream_t st) {
  return launch_fwd_sweep<IDW_LAYOUT>(a, f64, st);
}

hipError_t IDW_CAT(fwd_fixup_, IDW_LAYOUT_NAME)(const FwdArgs& a, bool f64, hipStream_t st) {
  return launch_fwd_fixup<IDW_LAYOUT>(a, f64, st);
}

hipError_t IDW_CAT(bbox_, IDW_LAYOUT_NAME)(const DevPts& d, int64_t n, int dim, bool f64,
                                           double* part, int nblocks, hipStream_t st) {
  return launch_bbox<IDW_LAYOUT>(d, n, dim, f64, part, nblocks, st);
}

hipError_t IDW_CAT(bwd_query_, IDW_LAYOUT_NAME)(const BwdArgs& a, bool f64, hipStream_t st) {
  BwdArgs b = a;
  if (f64)
    return a.dim == 3 ? bwd_query_pm<double, 3, IDW_LAYOUT>(b, a.split_q, a.chunk_q, a.part_q, st)
                      : bwd_query_pm<double, 2, IDW_LAYOUT>(b, a.split_q, a.chunk_q, a.part_q, st);
  return a.dim == 3 ? bwd_query_pm<float, 3, IDW_LAYOUT>(b, a.split_q, a.chunk_q, a.part_q, st)
                    : bwd_query_pm<float, 2, IDW_LAYOUT>(b, a.split_q, a.chunk_q, a.part_q, st);
}

hipError_t IDW_CAT(bwd_data_, IDW_LAYOUT_NAME)(const BwdArgs& a, bool f64, hipStream_t st) {
  BwdArgs b = a;
  b.q_per_lane = a.x_per_lane;
  if (f64)
    return a.dim == 3 ? bwd_data_pm<double, 3, IDW_LAYOUT>(b, a.split_z, a.chunk_z, a.part_z, st)
                      : bwd_data_pm<double, 2, IDW_LAYOUT>(b, a.split_z, a.chunk_z, a.part_z, st);
  return a.dim == 3 ? bwd_data_pm<float, 3, IDW_LAYOUT>(b, a.split_z, a.chunk_z, a.part_z, st)
                    : bwd_data_pm<float, 2, IDW_LAYOUT>(b, a.split_z, a.chunk_z, a.part_z, st);
}

hipError_t IDW_CAT(bwd_datax_, IDW_LAYOUT_NAME)(const BwdArgs& a, bool f64, hipStream_t st) {
  if (f64)
    return a.dim == 3 ? bwd_datax_pm<double, 3, IDW_LAYOUT>(a, a.split_z, a.chunk_z, st)
                      : bwd_datax_pm<double, 2, IDW_LAYOUT>(a, a.split_z, a.chunk_z, st);
  return a.dim == 3 ? bwd_datax_pm<float, 3, IDW_LAYOUT>(a, a.split_z, a.chunk_z, st)
                    : bwd_datax_pm<float, 2, IDW_LAYOUT>(a, a.split_z, a.chunk_z, st);
}

hipError_t IDW_CAT(bwd_fixup_, IDW_LAYOUT_NAME)(const BwdArgs& a, bool f64, hipStream_t st) {
  if (f64)
    return a.dim == 3 ? bwd_fix_pm<double, 3, IDW_LAYOUT>(a, st) : bwd_fix_pm<double, 2, IDW_LAYOUT>(a, st);
  return a.dim == 3 ? bwd_fix_pm<float, 3, IDW_LAYOUT>(a, st) : bwd_fix_pm<float, 2, IDW_LAYOUT>(a, st);
}

hipError_t IDW_CAT(near_check_, IDW_LAYOUT_NAME)(const NearArgs& a, hipStream_t st) {
  return launch_near_check<IDW_LAYOUT>(a, st);
}

hipError_t IDW_CAT(grid_, IDW_LAYOUT_NAME)(const GridArgs& a, bool build, hipStream_t st) {
  return launch_grid<IDW_LAYOUT>(a, build, st);
}

hipError_t IDW_CAT(bwd_fused_, IDW_LAYOUT_NAME)(const BwdArgs& a, bool f64, hipStream_t st) {
  if (f64)
    return a.dim == 3 ? bwd_fused_pm<double, 3, IDW_LAYOUT>(a, a.fused_groups, a.fused_ranges, a.fused_chunk, st)
                      : bwd_fused_pm<double, 2, IDW_LAYOUT>(a, a.fused_groups, a.fused_ranges, a.fused_chunk, st);
  return a.dim == 3 ? bwd_fused_pm<float, 3, IDW_LAYOUT>(a, a.fused_groups, a.fused_ranges, a.fused_chunk, st)
                    : bwd_fused_pm<float, 2, IDW_LAYOUT>(a, a.fused_groups, a.fused_ranges, a.fused_chunk, st);
}

}  // namespace idw
