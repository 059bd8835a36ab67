// Batched form: many independent IDW instances (own data, queries, p, dim) in one
// persistent launch, captured with its set-up and merge kernels into one HIP graph.
//
// Host plan: every instance is cut into work items (query block x data chunk); an item's
// cost is proportional to its pair count; items are ordered longest-first so that the
// dynamic claim order below approximates longest-processing-time scheduling.  Device:
// a fixed number of persistent workgroups claim item indices from an integer counter
// (the claim order does not affect any result: every item writes its own partial slot,
// and partials are merged per query in chunk order, so results are bitwise reproducible).
// Each item runs the same LDS-tiled FP32 sweep as idw_forward, dispatched on the
// instance's dimension and weight class.  A merge kernel finalises every query (FP64
// ratio, flags), flagged queries are compacted in order and recomputed in FP64.
// Instances with p >= 6 use relative weights as idw_forward does: a first pass over their
// work items finds every query's nearest squared distance (integer atomic min on the bits
// of the non-negative float, order-independent), and their sweep items scale by it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/idw.h"
#include "idw_api_internal.hpp"
#include "idw_fwd.hpp"

namespace idw {

// Device-side description of one instance.  Layout is aligned AoS (float4 records) for
// data and queries; pointers are caller-owned device memory.
struct BInst {
  const float4* data;
  const float4* query;
  float* out_z;
  double* out_den;
  int64_t n, m;
  int64_t q_off;     // offset of this instance's queries in the flattened query space
  int64_t part_off;  // offset (in double2) of its partials: [split][m]
  int64_t chunk;     // data points per chunk (multiple of kTile)
  int split;
  int dim;
  int pmode;
  int rel;           // relative weights (FP32, p >= kRelP)
  float nhp;         // -p/2
  double p;
};

struct BItem {
  int inst;
  int qblock;
  int chunk;
  int pad;
};

constexpr int kBQ = 4;       // queries per lane in the batched sweep
constexpr int kBHdr = 16;    // header doubles per instance (HdrSlot layout)
constexpr int kBboxBlocks = 32;

// ---- per-instance extent and thresholds (scaled FP32 units), as in idw_forward ----
__global__ __launch_bounds__(kWG) void kb_bbox(const BInst* __restrict__ inst, double* __restrict__ part) {
  __shared__ double red[kWG];
  const int i = blockIdx.y;
  const BInst I = inst[i];
  double mn[3] = {__builtin_huge_val(), __builtin_huge_val(), __builtin_huge_val()};
  double mx[3] = {-__builtin_huge_val(), -__builtin_huge_val(), -__builtin_huge_val()};
  double vm = 0.0;
  for (int64_t j = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x; j < I.n;
       j += static_cast<int64_t>(gridDim.x) * kWG) {
    const float4 r = I.data[j];
    const double c[3] = {r.x, r.y, r.z};
    for (int d = 0; d < I.dim; ++d) {
      mn[d] = fmin(mn[d], c[d]);
      mx[d] = fmax(mx[d], c[d]);
    }
    vm = fmax(vm, fabs(static_cast<double>(I.dim == 3 ? r.w : r.z)));
  }
  const int t = threadIdx.x;
  double* rec = part + (static_cast<int64_t>(i) * gridDim.x + blockIdx.x) * kBboxStride;
  red[t] = vm;
  __syncthreads();
  for (int s = kWG / 2; s > 0; s >>= 1) {
    if (t < s) red[t] = fmax(red[t], red[t + s]);
    __syncthreads();
  }
  if (t == 0) rec[6] = red[0];
  __syncthreads();
  for (int d = 0; d < 3; ++d) {
    for (int pass = 0; pass < 2; ++pass) {
      red[t] = pass ? mx[d] : mn[d];
      __syncthreads();
      for (int s = kWG / 2; s > 0; s >>= 1) {
        if (t < s) red[t] = pass ? fmax(red[t], red[t + s]) : fmin(red[t], red[t + s]);
        __syncthreads();
      }
      if (t == 0) rec[pass * 3 + d] = red[0];
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(64) void kb_bbox_final(const BInst* __restrict__ inst, int count, int nb,
                                                    const double* __restrict__ part,
                                                    double* __restrict__ hdr) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= count) return;
  const BInst I = inst[i];
  const double* rec = part + static_cast<int64_t>(i) * nb * kBboxStride;
  double ext = 0.0, vm = 0.0;
  for (int d = 0; d < I.dim; ++d) {
    double mn = __builtin_huge_val(), mx = -__builtin_huge_val();
    for (int b = 0; b < nb; ++b) {
      mn = fmin(mn, rec[b * kBboxStride + d]);
      mx = fmax(mx, rec[b * kBboxStride + 3 + d]);
    }
    ext = fmax(ext, mx - mn);
  }
  for (int b = 0; b < nb; ++b) vm = fmax(vm, rec[b * kBboxStride + 6]);
  fill_header(hdr + static_cast<int64_t>(i) * kBHdr, ext, vm, I.p, true, I.rel != 0);
}

// ---- nearest squared distance of every query of the relative-weight instances ----
__global__ __launch_bounds__(kWG) void kb_rmin_init(unsigned int* __restrict__ rmin, int64_t mtot) {
  for (int64_t g = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x; g < mtot;
       g += static_cast<int64_t>(gridDim.x) * kWG)
    rmin[g] = __builtin_bit_cast(unsigned int, __builtin_huge_valf());
}

// One workgroup per work item of a relative-weight instance: the item's data chunk goes
// through LDS tiles, each lane keeps the smallest squared distance (scaled FP32 units, the
// arithmetic of the sweep) of its queries and folds it into rmin.
template <int DIM>
__device__ __forceinline__ void kb_rmin_item(const BInst& I, const BItem& it, const double* __restrict__ hdr,
                                             unsigned int* __restrict__ rmin, P4<float> (*tile)[kTile]) {
  const int tid = threadIdx.x;
  const int64_t q0 = static_cast<int64_t>(it.qblock) * (kWG * kBQ);
  const int64_t jb = static_cast<int64_t>(it.chunk) * I.chunk;
  const int64_t je = (jb + I.chunk < I.n) ? jb + I.chunk : I.n;
  const float s = static_cast<float>(hdr[H_SCALE]);
  float qc[kBQ][3], mn[kBQ];
  int64_t qi[kBQ];
#pragma unroll
  for (int k = 0; k < kBQ; ++k) {
    qi[k] = q0 + tid + static_cast<int64_t>(k) * kWG;
    float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
    if (qi[k] < I.m) r = I.query[qi[k]];
    qc[k][0] = r.x * s;
    qc[k][1] = r.y * s;
    qc[k][2] = r.z * s;
    mn[k] = __builtin_huge_valf();
  }
  const int ntiles = static_cast<int>((je - jb + kTile - 1) / kTile);
  for (int t = 0; t < ntiles; ++t) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t j = jb + static_cast<int64_t>(t) * kTile + u * kWG + tid;
      P4<float> r;
      if (j < je) {
        const float4 d = I.data[j];
        r.x = d.x * s;
        r.y = d.y * s;
        r.z = d.z * s;
      } else {  // padding record: infinitely far
        r.x = r.y = r.z = __builtin_huge_valf();
      }
      r.w = 0.f;
      tile[0][u * kWG + tid] = r;
    }
    __syncthreads();
#pragma unroll 4
    for (int jj = 0; jj < kTile; ++jj) {
      const P4<float> d = tile[0][jj];
#pragma unroll
      for (int k = 0; k < kBQ; ++k) {
        const float r2 = sqdist<float, DIM>(qc[k], d);
        mn[k] = r2 < mn[k] ? r2 : mn[k];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kBQ; ++k)
    if (qi[k] < I.m) atomicMin(&rmin[I.q_off + qi[k]], __builtin_bit_cast(unsigned int, mn[k]));
}

__global__ __launch_bounds__(kWG) void kb_rmin(const BInst* __restrict__ inst, const BItem* __restrict__ items,
                                               int nitems, const double* __restrict__ hdr,
                                               unsigned int* __restrict__ rmin) {
  __shared__ P4<float> tile[2][kTile];
  for (int w = blockIdx.x; w < nitems; w += gridDim.x) {  // uniform over the workgroup
    const BItem it = items[w];
    const BInst I = inst[it.inst];
    const double* h = hdr + static_cast<int64_t>(it.inst) * kBHdr;
    if (I.dim == 3)
      kb_rmin_item<3>(I, it, h, rmin, tile);
    else
      kb_rmin_item<2>(I, it, h, rmin, tile);
  }
}

// ---- persistent sweep ----
template <int DIM, int PM, bool REL = false>
__device__ __forceinline__ void kb_item(const BInst& I, const BItem& it, const double* __restrict__ hdr,
                                        double2* __restrict__ part, P4<float> (*tile)[kTile],
                                        const unsigned int* __restrict__ rmin) {
  const int tid = threadIdx.x;
  const int64_t q0 = static_cast<int64_t>(it.qblock) * (kWG * kBQ);
  const int64_t jb = static_cast<int64_t>(it.chunk) * I.chunk;
  const int64_t je = (jb + I.chunk < I.n) ? jb + I.chunk : I.n;
  const float s = static_cast<float>(hdr[H_SCALE]);
  float qc[kBQ][3];
  int64_t qi[kBQ];
#pragma unroll
  for (int k = 0; k < kBQ; ++k) {
    qi[k] = q0 + tid + static_cast<int64_t>(k) * kWG;
    float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
    if (qi[k] < I.m) r = I.query[qi[k]];
    qc[k][0] = r.x * s;
    qc[k][1] = r.y * s;
    qc[k][2] = r.z * s;
  }
  BlockSum<float> nacc[kBQ], dacc[kBQ];
#pragma unroll
  for (int k = 0; k < kBQ; ++k) {
    nacc[k].zero();
    dacc[k].zero();
  }
  float4 rr[2];
  auto fetch = [&](int t) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t j = jb + static_cast<int64_t>(t) * kTile + u * kWG + tid;
      if (j < je) {
        rr[u] = I.data[j];
      } else {
        rr[u] = make_float4(__builtin_huge_valf(), __builtin_huge_valf(), __builtin_huge_valf(), 0.f);
        if (DIM == 2) rr[u].z = 0.f;
      }
    }
  };
  auto put = [&](int b) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      P4<float> r;
      r.x = rr[u].x * s;
      r.y = rr[u].y * s;
      if (DIM == 3) {
        r.z = rr[u].z * s;
        r.w = rr[u].w;
      } else {
        r.z = rr[u].z;
        r.w = 0.f;
      }
      tile[b][u * kWG + tid] = r;
    }
  };
  const int ntiles = static_cast<int>((je - jb + kTile - 1) / kTile);
  float sg[kBQ];  // per-query scale of the relative weights (1: direct weights)
  double fs[kBQ];
#pragma unroll
  for (int k = 0; k < kBQ; ++k) {
    sg[k] = 1.f;
    fs[k] = 1.0;
    if constexpr (REL) {
      if (qi[k] < I.m) rel_from_min(__builtin_bit_cast(float, rmin[I.q_off + qi[k]]), I.p, sg[k], fs[k]);
    }
  }
  fetch(0);
  put(0);
  __syncthreads();
  for (int t = 0; t < ntiles; ++t) {
    if (t + 1 < ntiles) fetch(t + 1);
    fwd_tile<float, DIM, PM, kBQ, false, 4, false, REL>(tile[t & 1], 0, kTile, qc, qi, I.nhp, sg, nacc, dacc);
    if (t + 1 < ntiles) put((t + 1) & 1);
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kBQ; ++k) {
    if (qi[k] < I.m) {
      const double num = nacc[k].value() * fs[k];
      const double den = dacc[k].value() * fs[k];
      part[I.part_off + static_cast<int64_t>(it.chunk) * I.m + qi[k]] = make_double2(num, den);
    }
  }
}

// Persistent workgroups claim work items in list order from an integer counter (which only
// decides which workgroup runs an item, not the arithmetic).  Direct-weight items and the
// relative-weight items of instances with p >= kRelP run in two kernels: with the relative
// variants in the same kernel, the direct-weight sweep measured 12% slower (66.3 against
// 59.4 ms on the 64-instance workload) for the same inner loops.
__device__ __forceinline__ int kb_claim(int* __restrict__ counter, int* claim) {
  if (threadIdx.x == 0) *claim = atomicAdd(counter, 1);
  __syncthreads();
  const int w = *claim;
  __syncthreads();
  return w;  // uniform over the workgroup
}

__global__ __launch_bounds__(kWG) void kb_sweep(const BInst* __restrict__ inst, const BItem* __restrict__ items,
                                                int nitems, int* __restrict__ counter,
                                                const double* __restrict__ hdr,
                                                double2* __restrict__ part) {
  __shared__ P4<float> tile[2][kTile];
  __shared__ int claim;
  for (;;) {
    const int w = kb_claim(counter, &claim);
    if (w >= nitems) break;  // uniform exit: every wave of the workgroup sees the same w
    const BItem it = items[w];
    const BInst I = inst[it.inst];
    const double* h = hdr + static_cast<int64_t>(it.inst) * kBHdr;
    if (I.dim == 3) {
      switch (I.pmode) {
        case PM_1: kb_item<3, PM_1>(I, it, h, part, tile, nullptr); break;
        case PM_2: kb_item<3, PM_2>(I, it, h, part, tile, nullptr); break;
        case PM_3: kb_item<3, PM_3>(I, it, h, part, tile, nullptr); break;
        case PM_4: kb_item<3, PM_4>(I, it, h, part, tile, nullptr); break;
        case PM_25: kb_item<3, PM_25>(I, it, h, part, tile, nullptr); break;
        default: kb_item<3, PM_GEN>(I, it, h, part, tile, nullptr); break;
      }
    } else {
      switch (I.pmode) {
        case PM_1: kb_item<2, PM_1>(I, it, h, part, tile, nullptr); break;
        case PM_2: kb_item<2, PM_2>(I, it, h, part, tile, nullptr); break;
        case PM_3: kb_item<2, PM_3>(I, it, h, part, tile, nullptr); break;
        case PM_4: kb_item<2, PM_4>(I, it, h, part, tile, nullptr); break;
        case PM_25: kb_item<2, PM_25>(I, it, h, part, tile, nullptr); break;
        default: kb_item<2, PM_GEN>(I, it, h, part, tile, nullptr); break;
      }
    }
  }
}

// The work items of the relative-weight instances (p >= kRelP), scaled by each query's
// nearest squared distance from kb_rmin.
__global__ __launch_bounds__(kWG) void kb_sweep_rel(const BInst* __restrict__ inst,
                                                    const BItem* __restrict__ items, int nitems,
                                                    int* __restrict__ counter, const double* __restrict__ hdr,
                                                    double2* __restrict__ part,
                                                    const unsigned int* __restrict__ rmin) {
  __shared__ P4<float> tile[2][kTile];
  __shared__ int claim;
  for (;;) {
    const int w = kb_claim(counter, &claim);
    if (w >= nitems) break;
    const BItem it = items[w];
    const BInst I = inst[it.inst];
    const double* h = hdr + static_cast<int64_t>(it.inst) * kBHdr;
    if (I.dim == 3)
      kb_item<3, PM_GEN, true>(I, it, h, part, tile, rmin);
    else
      kb_item<2, PM_GEN, true>(I, it, h, part, tile, rmin);
  }
}

// Which instance owns flattened query g: binary search over q_off.
__device__ __forceinline__ int find_inst(const BInst* __restrict__ inst, int count, int64_t g) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (inst[mid].q_off <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(kWG) void kb_merge(const BInst* __restrict__ inst, int count, int64_t mtot,
                                                const double* __restrict__ hdr,
                                                const double2* __restrict__ part,
                                                uint8_t* __restrict__ flag) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (g >= mtot) return;
  const int i = find_inst(inst, count, g);
  const BInst I = inst[i];
  const int64_t q = g - I.q_off;
  double nh = 0.0, nl = 0.0, dh = 0.0, dl = 0.0;
  for (int c = 0; c < I.split; ++c) {
    const double2 v = part[I.part_off + static_cast<int64_t>(c) * I.m + q];
    two_sum_acc(nh, nl, v.x);
    two_sum_acc(dh, dl, v.y);
  }
  const double num = nh + nl, den = dh + dl;
  const double* h = hdr + static_cast<int64_t>(i) * kBHdr;
  I.out_z[q] = static_cast<float>(num / den);
  if (I.out_den) I.out_den[q] = den * h[H_DEN_UNIT];
  flag[g] = route_of(den, h, false);
}

template <int DIM, int PM>
__device__ __forceinline__ void kb_fix_one(const BInst& I, int64_t q, double* red, long long* redi) {
  const float4 qr = I.query[q];
  const double qq[3] = {qr.x, qr.y, qr.z};
  NSum num, den;
  double hz = 0.0;
  long long h = 0;
  for (int64_t j = threadIdx.x; j < I.n; j += kWG) {
    const float4 r = I.data[j];
    const double c[3] = {r.x, r.y, r.z};
    const double v = DIM == 3 ? r.w : r.z;
    double r2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double e = qq[d] - c[d];
      r2 += e * e;
    }
    if (r2 == 0.0) {
      ++h;
      hz += v;
    } else {
      const double w = weight<PM>(r2, -0.5 * I.p);
      num.add(w * v);
      den.add(w);
    }
  }
  const double tn = block_sum(num.value(), red);
  const double td = block_sum(den.value(), red);
  const double thz = block_sum(hz, red);
  const long long th = block_sum_i64(h, redi);
  if (threadIdx.x == 0) {
    I.out_z[q] = static_cast<float>(th > 0 ? thz / static_cast<double>(th) : tn / td);
    if (I.out_den) I.out_den[q] = th > 0 ? __builtin_huge_val() : td;
  }
}

// Nearest-distance check of the candidate queries (route F_CANDIDATE), one per workgroup:
// the workgroup strides over its instance's data points, keeps the smallest squared
// distance in the instance's scaled FP32 units (the same arithmetic as k_near_check) and
// reduces it; within 1e-6 of the extent the query goes to FP64, otherwise its sweep result
// stands.
__global__ __launch_bounds__(kWG) void kb_near(const BInst* __restrict__ inst, int count,
                                              const double* __restrict__ hdr, const int* __restrict__ list,
                                              const int* __restrict__ cnt, uint8_t* __restrict__ route) {
  __shared__ float red[kWG];
  const int c = *cnt;
  const int t = threadIdx.x;
  for (int w = blockIdx.x; w < c; w += gridDim.x) {  // uniform over the workgroup
    const int64_t g = list[w];
    const int i = find_inst(inst, count, g);
    const BInst I = inst[i];
    const double* h = hdr + static_cast<int64_t>(i) * kBHdr;
    const float s = static_cast<float>(h[H_SCALE]);
    const float4 qr = I.query[g - I.q_off];
    const float qx = qr.x * s, qy = qr.y * s, qz = qr.z * s;
    float mn = __builtin_huge_valf();
    for (int64_t j = t; j < I.n; j += kWG) {
      const float4 d = I.data[j];
      const float dx = qx - d.x * s, dy = qy - d.y * s;
      float r2 = dx * dx;
      r2 = fmaf(dy, dy, r2);
      if (I.dim == 3) {
        const float dz = qz - d.z * s;
        r2 = fmaf(dz, dz, r2);
      }
      mn = r2 < mn ? r2 : mn;
    }
    red[t] = mn;
    __syncthreads();
    for (int o = kWG / 2; o > 0; o >>= 1) {
      if (t < o) red[t] = red[t + o] < red[t] ? red[t + o] : red[t];
      __syncthreads();
    }
    if (t == 0) route[g] = red[0] < static_cast<float>(h[H_NEAR_R2]) ? F_FP64 : F_FP32;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kWG) void kb_fixup(const BInst* __restrict__ inst, int count,
                                                const int* __restrict__ list, const int* __restrict__ cnt) {
  __shared__ double red[kWG];
  __shared__ long long redi[kWG];
  const int c = *cnt;
  for (int64_t sl = blockIdx.x; sl < c; sl += gridDim.x) {
    const int64_t g = list[sl];
    const int i = find_inst(inst, count, g);
    const BInst I = inst[i];
    const int64_t q = g - I.q_off;
    if (I.dim == 3) {
      switch (I.pmode) {
        case PM_1: kb_fix_one<3, PM_1>(I, q, red, redi); break;
        case PM_2: kb_fix_one<3, PM_2>(I, q, red, redi); break;
        case PM_3: kb_fix_one<3, PM_3>(I, q, red, redi); break;
        case PM_4: kb_fix_one<3, PM_4>(I, q, red, redi); break;
        case PM_25: kb_fix_one<3, PM_25>(I, q, red, redi); break;
        default: kb_fix_one<3, PM_GEN>(I, q, red, redi); break;
      }
    } else {
      switch (I.pmode) {
        case PM_1: kb_fix_one<2, PM_1>(I, q, red, redi); break;
        case PM_2: kb_fix_one<2, PM_2>(I, q, red, redi); break;
        case PM_3: kb_fix_one<2, PM_3>(I, q, red, redi); break;
        case PM_4: kb_fix_one<2, PM_4>(I, q, red, redi); break;
        case PM_25: kb_fix_one<2, PM_25>(I, q, red, redi); break;
        default: kb_fix_one<2, PM_GEN>(I, q, red, redi); break;
      }
    }
  }
}

// Clears the two claim counters (direct-weight and relative-weight items) with a kernel, so
// that no memset node is recorded into the captured graph.
__global__ void kb_reset(int* counter) {
  if (threadIdx.x < 2 && blockIdx.x == 0) counter[threadIdx.x] = 0;
}

}  // namespace idw

using namespace idw;

struct idw_plan {
  int count = 0;
  int nitems = 0;          // work items of the direct-weight instances
  int64_t mtot = 0;
  int64_t part_elems = 0;  // double2 partial slots
  int grid = 0;            // persistent workgroups of the direct-weight sweep
  int grid_rel = 0;        // persistent workgroups of the relative-weight sweep
  int grid_req = 0;        // workgroups asked for (configuration or tuned default), before the
                           // clamp to the number of work items
  int chunk_target = 0;
  int nrel_items = 0;      // work items of the relative-weight instances (nearest pass)
  std::vector<BInst> host_inst;
  BInst* d_inst = nullptr;
  BItem* d_items = nullptr;
  BItem* d_rel_items = nullptr;
  size_t ws_bytes = 0;
  // workspace sections
  size_t o_hdr = 0, o_bbox = 0, o_counter = 0, o_part = 0, o_flag = 0, o_bcnt = 0, o_list = 0, o_count = 0;
  size_t o_rmin = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* graph_ws = nullptr;
};

static size_t al256b(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Defaults of the persistent launch when the configuration leaves them at 0: the values the
// autotuner chose for this architecture, compiled in from its table by the build (item
// length in data points, persistent workgroups; 0 workgroups stands for two per compute
// unit).  Without a table: 16,384-point items, two workgroups per compute unit.
#ifndef IDW_TUNED_BATCH_CHUNK
#define IDW_TUNED_BATCH_CHUNK 16384
#endif
#ifndef IDW_TUNED_BATCH_WORKGROUPS
#define IDW_TUNED_BATCH_WORKGROUPS 0
#endif
static_assert(IDW_TUNED_BATCH_CHUNK > 0 && IDW_TUNED_BATCH_WORKGROUPS >= 0, "tuned batched defaults");

extern "C" {

int idw_batched_defaults(int64_t* chunk, int32_t* workgroups) {
  clear_error();
  if (!chunk || !workgroups) return fail(IDW_EINVAL, "null argument");
  *chunk = (IDW_TUNED_BATCH_CHUNK + kTile - 1) / kTile * kTile;
  *workgroups = IDW_TUNED_BATCH_WORKGROUPS;
  return IDW_OK;
}

int idw_batched_plan_params(const idw_plan* plan, int64_t* chunk, int32_t* workgroups) {
  clear_error();
  if (!plan || !chunk || !workgroups) return fail(IDW_EINVAL, "null argument");
  *chunk = plan->chunk_target;
  *workgroups = plan->grid_req;
  return IDW_OK;
}

int idw_batched_plan_create(const idw_instance* instances, int32_t count, int32_t precision,
                            const idw_config* cfg, idw_plan** out_plan) {
  clear_error();
  if (!out_plan) return fail(IDW_EINVAL, "out_plan is null");
  *out_plan = nullptr;
  if (!instances || count <= 0) return fail(IDW_EINVAL, "at least one instance is required");
  if (precision != IDW_FP32) return fail(IDW_EUNSUPPORTED, "batched plans run the FP32 sweep only");
  if (const int rc0 = validate_config(cfg)) return rc0;
  const int chunk_req = (cfg && cfg->batch_chunk > 0) ? cfg->batch_chunk : IDW_TUNED_BATCH_CHUNK;
  const int chunk_target = static_cast<int>((static_cast<int64_t>(chunk_req) + kTile - 1) / kTile * kTile);
  const int grid_req = (cfg && cfg->batch_workgroups > 0) ? cfg->batch_workgroups : IDW_TUNED_BATCH_WORKGROUPS;
  std::vector<BInst> hi(count);
  int64_t qoff = 0, poff = 0;
  struct Cand {
    BItem it;
    double cost;
  };
  std::vector<Cand> cands;
  for (int i = 0; i < count; ++i) {
    const idw_instance& s = instances[i];
    if (s.data.layout != IDW_AOAS || s.query.layout != IDW_AOAS)
      return fail(IDW_EUNSUPPORTED, "instance %d: batched plans take aligned-AoS (float4) records", i);
    int rc = validate_common(&s.data, &s.query, s.p, precision, 0);
    if (rc) {
      std::string m = idw_last_error();
      return fail(rc, "instance %d: %s", i, m.c_str());
    }
    if (s.query.n > 0 && !s.out_z) return fail(IDW_EINVAL, "instance %d: out_z is null", i);
    BInst& b = hi[i];
    b.data = static_cast<const float4*>(s.data.ptr[0]);
    b.query = static_cast<const float4*>(s.query.ptr[0]);
    b.out_z = static_cast<float*>(s.out_z);
    b.out_den = s.out_den;
    b.n = s.data.n;
    b.m = s.query.n;
    b.dim = s.data.dim;
    const int pm = pmode_of(s.p);
    b.pmode = pm;
    b.rel = s.p >= kRelP ? 1 : 0;
    b.p = s.p;
    b.nhp = static_cast<float>(-0.5 * s.p);
    b.q_off = qoff;
    b.chunk = std::min<int64_t>(chunk_target, (b.n + kTile - 1) / kTile * kTile);
    b.split = static_cast<int>((b.n + b.chunk - 1) / b.chunk);
    b.part_off = poff;
    qoff += b.m;
    poff += static_cast<int64_t>(b.split) * b.m;
    const int64_t qblocks = (b.m + kWG * kBQ - 1) / (kWG * kBQ);
    for (int64_t qb = 0; qb < qblocks; ++qb)
      for (int c = 0; c < b.split; ++c) {
        // Every lane of the workgroup runs the whole chunk whether or not it holds a
        // query, so an item costs its chunk length rounded up to whole tiles.
        const double dn = static_cast<double>(std::min<int64_t>(b.chunk, b.n - c * b.chunk));
        cands.push_back({BItem{i, static_cast<int>(qb), c, 0}, std::ceil(dn / kTile) * kTile});
      }
  }
  // longest first; ties in a fixed order
  std::stable_sort(cands.begin(), cands.end(), [](const Cand& a, const Cand& b) { return a.cost > b.cost; });
  // direct-weight items for kb_sweep, relative-weight items for kb_rmin and kb_sweep_rel,
  // each list longest first
  std::vector<BItem> items, rel_items;
  for (const Cand& c : cands) (hi[c.it.inst].rel ? rel_items : items).push_back(c.it);

  idw_plan* P = new idw_plan();
  P->count = count;
  P->nitems = static_cast<int>(items.size());
  P->nrel_items = static_cast<int>(rel_items.size());
  P->mtot = qoff;
  P->part_elems = poff;
  P->chunk_target = chunk_target;
  P->host_inst = hi;
  int rc = check_device();
  if (rc) {
    delete P;
    return rc;
  }
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  P->grid_req = grid_req > 0 ? grid_req : cus * 2;
  P->grid = std::min(P->grid_req, std::max(P->nitems, 1));
  P->grid_rel = std::min(P->grid_req, std::max(P->nrel_items, 1));
  if (hipMalloc(&P->d_inst, sizeof(BInst) * count) != hipSuccess ||
      hipMalloc(&P->d_items, sizeof(BItem) * std::max<size_t>(1, items.size())) != hipSuccess ||
      hipMalloc(&P->d_rel_items, sizeof(BItem) * std::max<size_t>(1, rel_items.size())) != hipSuccess) {
    idw_batched_plan_destroy(P);
    return fail(IDW_ENOMEM, "plan allocation failed");
  }
  if (hipMemcpy(P->d_inst, hi.data(), sizeof(BInst) * count, hipMemcpyHostToDevice) != hipSuccess ||
      (!items.empty() &&
       hipMemcpy(P->d_items, items.data(), sizeof(BItem) * items.size(), hipMemcpyHostToDevice) != hipSuccess) ||
      (!rel_items.empty() && hipMemcpy(P->d_rel_items, rel_items.data(), sizeof(BItem) * rel_items.size(),
                                       hipMemcpyHostToDevice) != hipSuccess)) {
    idw_batched_plan_destroy(P);
    return fail(IDW_EDEVICE, "plan upload failed");
  }
  // workspace layout
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t at = off;
    off = al256b(off + b);
    return at;
  };
  const int64_t mt = std::max<int64_t>(P->mtot, 1);
  const int64_t nb = (mt + kCountBlock - 1) / kCountBlock;
  P->o_hdr = take(sizeof(double) * kBHdr * count);
  P->o_bbox = take(sizeof(double) * kBboxStride * kBboxBlocks * count);
  P->o_counter = take(sizeof(int) * 4);
  P->o_count = take(sizeof(int) * 4);
  P->o_part = take(sizeof(double2) * std::max<int64_t>(P->part_elems, 1));
  P->o_flag = take(static_cast<size_t>(mt));
  P->o_bcnt = take(sizeof(int) * static_cast<size_t>(nb + 1));
  P->o_list = take(sizeof(int) * static_cast<size_t>(mt));
  P->o_rmin = take(P->nrel_items > 0 ? sizeof(unsigned int) * static_cast<size_t>(mt) : 0);
  P->ws_bytes = off;
  if (hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    idw_batched_plan_destroy(P);
    return fail(IDW_EDEVICE, "stream creation failed");
  }
  *out_plan = P;
  return IDW_OK;
}

int idw_batched_plan_workspace(const idw_plan* plan, size_t* bytes) {
  clear_error();
  if (!plan || !bytes) return fail(IDW_EINVAL, "null argument");
  *bytes = plan->ws_bytes;
  return IDW_OK;
}

static hipError_t enqueue_batched(idw_plan* P, char* ws, hipStream_t st) {
  BInst* di = P->d_inst;
  double* hdr = reinterpret_cast<double*>(ws + P->o_hdr);
  double* bbox = reinterpret_cast<double*>(ws + P->o_bbox);
  int* counter = reinterpret_cast<int*>(ws + P->o_counter);
  int* cnt = reinterpret_cast<int*>(ws + P->o_count);
  double2* part = reinterpret_cast<double2*>(ws + P->o_part);
  uint8_t* flag = reinterpret_cast<uint8_t*>(ws + P->o_flag);
  int* bcnt = reinterpret_cast<int*>(ws + P->o_bcnt);
  int* list = reinterpret_cast<int*>(ws + P->o_list);
  unsigned int* rmin = P->nrel_items > 0 ? reinterpret_cast<unsigned int*>(ws + P->o_rmin) : nullptr;
  hipLaunchKernelGGL(kb_reset, dim3(1), dim3(64), 0, st, counter);
  hipLaunchKernelGGL(kb_bbox, dim3(kBboxBlocks, P->count), dim3(kWG), 0, st, di, bbox);
  hipLaunchKernelGGL(kb_bbox_final, dim3((P->count + 63) / 64), dim3(64), 0, st, di, P->count, kBboxBlocks,
                     bbox, hdr);
  if (P->nrel_items > 0) {  // nearest squared distance of the relative-weight instances' queries
    const int64_t ib = (P->mtot + kWG - 1) / kWG;
    hipLaunchKernelGGL(kb_rmin_init, dim3(static_cast<unsigned>(ib < 4096 ? ib : 4096)), dim3(kWG), 0, st, rmin,
                       P->mtot);
    hipLaunchKernelGGL(kb_rmin, dim3(static_cast<unsigned>(std::min(P->nrel_items, 2048))), dim3(kWG), 0, st, di,
                       P->d_rel_items, P->nrel_items, hdr, rmin);
  }
  if (P->nitems > 0)
    hipLaunchKernelGGL(kb_sweep, dim3(P->grid), dim3(kWG), 0, st, di, P->d_items, P->nitems, counter, hdr, part);
  if (P->nrel_items > 0)
    hipLaunchKernelGGL(kb_sweep_rel, dim3(P->grid_rel), dim3(kWG), 0, st, di, P->d_rel_items, P->nrel_items,
                       counter + 1, hdr, part, rmin);
  if (P->mtot > 0) {
    hipLaunchKernelGGL(kb_merge, dim3(static_cast<unsigned>((P->mtot + kWG - 1) / kWG)), dim3(kWG), 0, st, di,
                       P->count, P->mtot, hdr, part, flag);
    hipError_t e = compact_flags(flag, P->mtot, bcnt, list, cnt, F_CANDIDATE, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kb_near, dim3(1024), dim3(kWG), 0, st, di, P->count, hdr, list, cnt, flag);
    e = compact_flags(flag, P->mtot, bcnt, list, cnt, F_FP64, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kb_fixup, dim3(256), dim3(kWG), 0, st, di, P->count, list, cnt);
  }
  return hipGetLastError();
}

int idw_batched(idw_plan* plan, void* workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  if (!plan) return fail(IDW_EINVAL, "plan is null");
  int rc = check_workspace(workspace, workspace_bytes, plan->ws_bytes);
  if (rc) return rc;
  rc = check_device();
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!plan->exec || plan->graph_ws != workspace) {
    if (plan->exec) {
      (void)hipGraphExecDestroy(plan->exec);
      plan->exec = nullptr;
    }
    if (plan->graph) {
      (void)hipGraphDestroy(plan->graph);
      plan->graph = nullptr;
    }
    hipStream_t cs = plan->cap_stream;
    if ((rc = check_hip(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture"))) return rc;
    hipError_t e = enqueue_batched(plan, static_cast<char*>(workspace), cs);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return check_hip(e != hipSuccess ? e : e2, "graph capture");
    }
    plan->graph = g;
    if ((rc = check_hip(hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0), "graph instantiate"))) return rc;
    plan->graph_ws = workspace;
  }
  return check_hip(hipGraphLaunch(plan->exec, st), "graph launch");
}

void idw_batched_plan_destroy(idw_plan* plan) {
  if (!plan) return;
  (void)hipDeviceSynchronize();
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
  if (plan->d_inst) (void)hipFree(plan->d_inst);
  if (plan->d_items) (void)hipFree(plan->d_items);
  if (plan->d_rel_items) (void)hipFree(plan->d_rel_items);
  delete plan;
}

}  // extern "C"
