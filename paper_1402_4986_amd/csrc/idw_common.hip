// Layout-independent kernels: extent/threshold header, split merge, deterministic
// compaction of flagged queries, and the final dp reduction.
#include <math.h>

#include "idw_bwd.hpp"
#include "idw_device.hpp"
#include "idw_launch.hpp"

namespace idw {

// Reduces the per-workgroup extent partials and fills the workspace header.
__global__ __launch_bounds__(kWG) void k_bbox_final(const double* __restrict__ part, int nb,
                                                    int dim, double p, int f32s, int rel,
                                                    double* __restrict__ hdr) {
  __shared__ double red[kWG];
  __shared__ double bmn[3], bext[3];
  const int t = threadIdx.x;
  double ext = 0.0;
  if (t < 3) bmn[t] = bext[t] = 0.0;
  __syncthreads();
  for (int d = 0; d < dim; ++d) {
    double mn = __builtin_huge_val(), mx = -__builtin_huge_val();
    for (int b = t; b < nb; b += kWG) {
      mn = fmin(mn, part[b * kBboxStride + d]);
      mx = fmax(mx, part[b * kBboxStride + 3 + d]);
    }
    for (int pass = 0; pass < 2; ++pass) {
      red[t] = pass ? mx : mn;
      __syncthreads();
      for (int s = kWG / 2; s > 0; s >>= 1) {
        if (t < s) red[t] = pass ? fmax(red[t], red[t + s]) : fmin(red[t], red[t + s]);
        __syncthreads();
      }
      if (pass)
        mx = red[0];
      else
        mn = red[0];
      __syncthreads();
    }
    ext = fmax(ext, mx - mn);
    if (t == 0) {
      bmn[d] = mn;
      bext[d] = mx - mn;
    }
  }
  double vm = 0.0;
  for (int b = t; b < nb; b += kWG) vm = fmax(vm, part[b * kBboxStride + 6]);
  red[t] = vm;
  __syncthreads();
  for (int s = kWG / 2; s > 0; s >>= 1) {
    if (t < s) red[t] = fmax(red[t], red[t + s]);
    __syncthreads();
  }
  if (t == 0) {
    fill_header(hdr, ext, red[0], p, f32s != 0, rel != 0);
    const double s = hdr[H_SCALE];
    for (int k = 0; k < 3; ++k) {  // the box in scaled units, for the grid searches
      hdr[H_BMIN + k] = bmn[k] * s;
      hdr[H_BEXT + k] = bext[k] * s;
    }
  }
}

hipError_t bbox_final(const double* part, int nblocks, int dim, double p, bool f32_scaling,
                      bool rel, double* hdr, hipStream_t st) {
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(kWG), 0, st, part, nblocks, dim, p,
                     f32_scaling ? 1 : 0, rel ? 1 : 0, hdr);
  return hipGetLastError();
}

// Merges split partials in chunk order (TwoSum-compensated FP64) and finalises.
template <typename T>
__global__ __launch_bounds__(kWG) void k_merge(const double2* __restrict__ part, int64_t m,
                                               int split, const double* __restrict__ hdr,
                                               T* __restrict__ out_z, double* __restrict__ out_den,
                                               uint8_t* __restrict__ flag) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (i >= m) return;
  double nh = 0.0, nl = 0.0, dh = 0.0, dl = 0.0;
  for (int c = 0; c < split; ++c) {
    const double2 v = part[static_cast<int64_t>(c) * m + i];
    two_sum_acc(nh, nl, v.x);
    two_sum_acc(dh, dl, v.y);
  }
  const double num = nh + nl, den = dh + dl;
  out_z[i] = static_cast<T>(num / den);
  if (out_den) out_den[i] = den * hdr[H_DEN_UNIT];
  flag[i] = route_of(den, hdr, false);
}

hipError_t merge_split(const double2* part, int64_t m, int split, const double* hdr, void* out_z,
                       bool f64, double* out_den, uint8_t* flag, hipStream_t st) {
  dim3 grid(static_cast<unsigned>((m + kWG - 1) / kWG));
  if (f64)
    hipLaunchKernelGGL(k_merge<double>, grid, dim3(kWG), 0, st, part, m, split, hdr,
                       static_cast<double*>(out_z), out_den, flag);
  else
    hipLaunchKernelGGL(k_merge<float>, grid, dim3(kWG), 0, st, part, m, split, hdr,
                       static_cast<float*>(out_z), out_den, flag);
  return hipGetLastError();
}

// Backward route of each query from its saved denominator (caller units); candidates are
// then settled by the same nearest-distance check as in the forward.
__global__ __launch_bounds__(kWG) void k_flags_from_den(const double* __restrict__ den, int64_t m,
                                                        const double* __restrict__ hdr,
                                                        uint8_t* __restrict__ flag) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (i >= m) return;
  const double d = den[i];
  flag[i] = route_of(d, hdr, true);
}

hipError_t flags_from_den(const double* den, int64_t m, const double* hdr, uint8_t* flag,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_flags_from_den, dim3(static_cast<unsigned>((m + kWG - 1) / kWG)),
                     dim3(kWG), 0, st, den, m, hdr, flag);
  return hipGetLastError();
}

// ---- Deterministic, order-preserving compaction of the queries whose route byte equals
// `want` into an index list.  Block b owns bytes [b*4096, (b+1)*4096); thread t owns 16
// consecutive bytes of it. ----
constexpr int kPerThread = kCountBlock / kWG;

__device__ __forceinline__ int local_count(const uint8_t* __restrict__ flag, int64_t m,
                                           int64_t base, uint8_t want) {
  int c = 0;
#pragma unroll
  for (int u = 0; u < kPerThread; ++u) {
    const int64_t i = base + u;
    if (i < m) c += flag[i] == want ? 1 : 0;
  }
  return c;
}

__global__ __launch_bounds__(kWG) void k_count(const uint8_t* __restrict__ flag, int64_t m,
                                               uint8_t want, int* __restrict__ bcnt) {
  __shared__ double red[kWG];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kCountBlock + threadIdx.x * kPerThread;
  const double c = block_sum(static_cast<double>(local_count(flag, m, base, want)), red);
  if (threadIdx.x == 0) bcnt[blockIdx.x] = static_cast<int>(c);
}

// Exclusive scan of the block counts in place (single workgroup), total into *count.
__global__ __launch_bounds__(kWG) void k_scan(int* __restrict__ bcnt, int nb,
                                              int* __restrict__ count) {
  __shared__ int buf[kWG];
  __shared__ int carry;
  const int t = threadIdx.x;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += kWG) {
    const int v = (base + t < nb) ? bcnt[base + t] : 0;
    buf[t] = v;
    __syncthreads();
    for (int off = 1; off < kWG; off <<= 1) {  // Hillis-Steele inclusive scan
      const int add = t >= off ? buf[t - off] : 0;
      __syncthreads();
      buf[t] += add;
      __syncthreads();
    }
    if (base + t < nb) bcnt[base + t] = carry + buf[t] - v;
    __syncthreads();
    if (t == kWG - 1) carry += buf[t];
    __syncthreads();
  }
  if (t == 0) *count = carry;
}

__global__ __launch_bounds__(kWG) void k_emit(const uint8_t* __restrict__ flag, int64_t m,
                                              uint8_t want, const int* __restrict__ boff,
                                              int* __restrict__ list) {
  __shared__ int buf[kWG];
  const int t = threadIdx.x;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kCountBlock + t * kPerThread;
  const int c = local_count(flag, m, base, want);
  buf[t] = c;
  __syncthreads();
  for (int off = 1; off < kWG; off <<= 1) {
    const int add = t >= off ? buf[t - off] : 0;
    __syncthreads();
    buf[t] += add;
    __syncthreads();
  }
  int pos = boff[blockIdx.x] + buf[t] - c;
  for (int u = 0; u < kPerThread; ++u) {
    const int64_t i = base + u;
    if (i < m && flag[i] == want) list[pos++] = static_cast<int>(i);
  }
}

hipError_t compact_flags(const uint8_t* flag, int64_t m, int* bcnt, int* list, int* count,
                         uint8_t want, hipStream_t st) {
  const int nb = static_cast<int>((m + kCountBlock - 1) / kCountBlock);
  hipLaunchKernelGGL(k_count, dim3(nb), dim3(kWG), 0, st, flag, m, want, bcnt);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(kWG), 0, st, bcnt, nb, count);
  hipLaunchKernelGGL(k_emit, dim3(nb), dim3(kWG), 0, st, flag, m, want, bcnt, list);
  return hipGetLastError();
}

// dp = sum of the sweep workgroups' partials (in workgroup order) plus the FP64 fix-up
// slots' partials (in ascending query order).  Single workgroup, fixed-order tree.
__global__ __launch_bounds__(kWG) void k_dp_final(const double* __restrict__ wg_dp, int nwg,
                                                  const double* __restrict__ slot_dp,
                                                  const int* __restrict__ count,
                                                  double* __restrict__ grad_p) {
  __shared__ double red[kWG];
  const int t = threadIdx.x;
  double h = 0.0, l = 0.0;
  for (int b = t; b < nwg; b += kWG) two_sum_acc(h, l, wg_dp[b]);
  const int cnt = *count;
  for (int b = t; b < cnt; b += kWG) two_sum_acc(h, l, slot_dp[b]);
  const double tot = block_sum(h, red) + block_sum(l, red);
  if (t == 0) *grad_p = tot;
}

// ---- grid of the nearest-distance searches: geometry and gates, scan of the counts ----
// Geometry: square cells of side h = (largest box side) / (floor(ncell_max^(1/dim)) - 1),
// at least 2.5 times the near-coincidence distance (so the box q +- r' of the candidate
// check meets at most two cells per axis), hence at most ncell_max cells.
__global__ void k_grid_setup(double* __restrict__ hdr, int* __restrict__ hint, int dim, int64_t ncell_max,
                             int mode, int grid_on, int64_t mall) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const int64_t cand = mode == 1 ? mall : static_cast<int64_t>(hint[0]);
  const bool use = grid_on != 0 && cand > 0 && (mode == 1 || cand >= kGridMinCand);
  hint[GI_FALLBACK] = 0;
  hint[GI_BRUTE] = use ? 0 : static_cast<int>(cand);
  hint[GI_GRID] = use ? static_cast<int>(cand) : 0;
  if (!use) return;
  double emax = 0.0;
  for (int k = 0; k < dim; ++k) emax = fmax(emax, hdr[H_BEXT + k]);
  int base = static_cast<int>(floor(pow(static_cast<double>(ncell_max), 1.0 / dim))) - 1;
  if (base < 1) base = 1;
  auto cells = [&](int b) {  // (b + 1)^dim
    int64_t c = 1;
    for (int k = 0; k < dim; ++k) c *= b + 1;
    return c;
  };
  while (base > 1 && cells(base) > ncell_max) --base;  // pow may round the root up
  double h = fmax(emax / base, 2.5 * sqrt(hdr[H_NEAR_R2]));
  if (!(h > 0.0) || !(h < __builtin_huge_val())) h = 1.0;
  hdr[H_GRID_H] = h;
  hdr[H_GRID_INVH] = 1.0 / h;
  for (int k = 0; k < 3; ++k) {
    int g = 1;
    if (k < dim) {
      const double c = floor(hdr[H_BEXT + k] / h) + 1.0;
      g = c < static_cast<double>(base + 1) ? static_cast<int>(c) : base + 1;
      if (g < 1) g = 1;
    }
    hdr[H_GRID_G + k] = static_cast<double>(g);
  }
}

__device__ __forceinline__ int64_t grid_ncell(const double* __restrict__ hdr) {
  return static_cast<int64_t>(hdr[H_GRID_G]) * static_cast<int64_t>(hdr[H_GRID_G + 1]) *
         static_cast<int64_t>(hdr[H_GRID_G + 2]);
}

constexpr int kScanPer = kGridScanBlock / kWG;  // cells per thread in the count scan

__global__ __launch_bounds__(kWG) void k_grid_blocksum(const int* __restrict__ cnt, const double* __restrict__ hdr,
                                                       const int* __restrict__ hint, int* __restrict__ bsum) {
  __shared__ double red[kWG];
  if (hint[GI_GRID] <= 0) {
    if (threadIdx.x == 0) bsum[blockIdx.x] = 0;
    return;
  }
  const int64_t ncell = grid_ncell(hdr);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kGridScanBlock + threadIdx.x * kScanPer;
  long long c = 0;
  for (int u = 0; u < kScanPer; ++u)
    if (base + u < ncell) c += cnt[base + u];
  const double tot = block_sum(static_cast<double>(c), red);
  if (threadIdx.x == 0) bsum[blockIdx.x] = static_cast<int>(tot);
}

// start[c] = exclusive prefix of the counts; the counts become scatter cursors (= start);
// start[ncell] = the number of points.
__global__ __launch_bounds__(kWG) void k_grid_offsets(int* __restrict__ cnt, const double* __restrict__ hdr,
                                                      const int* __restrict__ hint, const int* __restrict__ boff,
                                                      int* __restrict__ start) {
  __shared__ int buf[kWG];
  if (hint[GI_GRID] <= 0) return;
  const int64_t ncell = grid_ncell(hdr);
  const int t = threadIdx.x;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kGridScanBlock + t * kScanPer;
  int loc[kScanPer];
  int c = 0;
  for (int u = 0; u < kScanPer; ++u) {
    loc[u] = base + u < ncell ? cnt[base + u] : 0;
    c += loc[u];
  }
  buf[t] = c;
  __syncthreads();
  for (int off = 1; off < kWG; off <<= 1) {  // Hillis-Steele inclusive scan
    const int add = t >= off ? buf[t - off] : 0;
    __syncthreads();
    buf[t] += add;
    __syncthreads();
  }
  int pos = boff[blockIdx.x] + buf[t] - c;
  for (int u = 0; u < kScanPer; ++u) {
    const int64_t cell = base + u;
    if (cell < ncell) {
      start[cell] = pos;
      cnt[cell] = pos;
      pos += loc[u];
      if (cell == ncell - 1) start[ncell] = pos;
    }
  }
}

hipError_t grid_setup(const GridArgs& a, int mode, bool grid_on, hipStream_t st) {
  hipLaunchKernelGGL(k_grid_setup, dim3(1), dim3(64), 0, st, const_cast<double*>(a.hdr), a.hint, a.dim,
                     a.ncell_max, mode, grid_on ? 1 : 0, a.m);
  return hipGetLastError();
}

hipError_t grid_scan(const GridArgs& a, hipStream_t st) {
  const int nb = static_cast<int>((a.ncell_max + kGridScanBlock - 1) / kGridScanBlock);
  hipLaunchKernelGGL(k_grid_blocksum, dim3(nb), dim3(kWG), 0, st, a.cnt, a.hdr, a.hint, a.bsum);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(kWG), 0, st, a.bsum, nb, a.hint + GI_TOTAL);
  hipLaunchKernelGGL(k_grid_offsets, dim3(nb), dim3(kWG), 0, st, a.cnt, a.hdr, a.hint, a.bsum, a.start);
  return hipGetLastError();
}

hipError_t bwd_qmerge(const BwdArgs& a, bool f64, hipStream_t st) {
  if (f64)
    return a.dim == 3 ? launch_bwd_qmerge<double, 3>(a, a.split_q, a.part_q, st)
                      : launch_bwd_qmerge<double, 2>(a, a.split_q, a.part_q, st);
  return a.dim == 3 ? launch_bwd_qmerge<float, 3>(a, a.split_q, a.part_q, st)
                    : launch_bwd_qmerge<float, 2>(a, a.split_q, a.part_q, st);
}

hipError_t bwd_xmerge(const BwdArgs& a, int split, bool f64, hipStream_t st) {
  if (f64)
    return a.dim == 3 ? launch_bwd_xmerge<double, 3>(a, split, st) : launch_bwd_xmerge<double, 2>(a, split, st);
  return a.dim == 3 ? launch_bwd_xmerge<float, 3>(a, split, st) : launch_bwd_xmerge<float, 2>(a, split, st);
}

hipError_t bwd_zmerge(const BwdArgs& a, bool f64, hipStream_t st) {
  if (f64) return launch_bwd_zmerge<double>(a, a.split_z, a.part_z, st);
  return launch_bwd_zmerge<float>(a, a.split_z, a.part_z, st);
}

hipError_t dp_final(const double* wg_dp, int nwg, const double* slot_dp, const int* count,
                    double* grad_p, hipStream_t st) {
  hipLaunchKernelGGL(k_dp_final, dim3(1), dim3(kWG), 0, st, wg_dp, nwg, slot_dp, count, grad_p);
  return hipGetLastError();
}

}  // namespace idw

namespace idw {

// Zero fill with a kernel (a memset node is never recorded into a captured graph).
__global__ __launch_bounds__(kWG) void k_fill_zero(uint32_t* __restrict__ p, int64_t words) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x; i < words;
       i += static_cast<int64_t>(gridDim.x) * kWG)
    p[i] = 0u;
}

hipError_t fill_zero(void* p, size_t bytes, hipStream_t st) {
  const int64_t words = static_cast<int64_t>(bytes / 4);
  if (words == 0) return hipSuccess;
  int64_t blocks = (words + kWG - 1) / kWG;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_zero, dim3(static_cast<unsigned>(blocks)), dim3(kWG), 0, st,
                     static_cast<uint32_t*>(p), words);
  return hipGetLastError();
}

}  // namespace idw
