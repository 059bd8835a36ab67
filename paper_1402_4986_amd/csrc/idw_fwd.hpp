// Forward sweep of Shepard IDW (Section 2.1, Eq. 1) for gfx950.
//
// One workgroup = 256 lanes x Q queries held in registers.  Data points are streamed
// through LDS in tiles of kTile records (double-buffered: the global loads of tile t+1 are
// in flight while tile t is consumed), and every record is broadcast from LDS to all lanes
// of the wavefront (the shared-memory tiling of Section 4.2, re-derived for wave64).  Each
// lane accumulates sum w*z and sum w for its queries in plain arithmetic over 64-record
// blocks and adds every block sum into an FP64 running sum (a TwoSum pair in the FP64
// sweep), so the sum error is that of a 64-term sum, not of an n-term one.  The ratio is
// taken in FP64.  A query whose
// denominator exceeds the near-coincidence threshold (or is not finite) is flagged for the
// FP64 fix-up kernel, which recomputes it exactly, including the exact-hit rule.
#pragma once

#include <math.h>

#include <type_traits>

#include "idw_device.hpp"
#include "idw_launch.hpp"

namespace idw {

__device__ __forceinline__ float fmaT(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return fma(a, b, c); }

template <typename T>
__device__ __forceinline__ T infT() {
  return __builtin_huge_valf();
}
template <>
__device__ __forceinline__ double infT<double>() {
  return __builtin_huge_val();
}

// Squared distance from query coordinates q to a staged record d.
template <typename T, int DIM>
__device__ __forceinline__ T sqdist(const T (&q)[3], const P4<T>& d) {
  const T dx = q[0] - d.x;
  const T dy = q[1] - d.y;
  T r2 = dx * dx;
  r2 = fmaT(dy, dy, r2);
  if constexpr (DIM == 3) {
    const T dz = q[2] - d.z;
    r2 = fmaT(dz, dz, r2);
  }
  return r2;
}

// Stage one record into LDS form: coordinates scaled by s; {x, y, v, 0} or {x, y, z, v}.
template <typename T, int DIM>
__device__ __forceinline__ P4<T> stage(const T (&c)[3], T v, T s) {
  P4<T> r;
  r.x = c[0] * s;
  r.y = c[1] * s;
  if constexpr (DIM == 3) {
    r.z = c[2] * s;
    r.w = v;
  } else {
    r.z = v;
    r.w = T(0);
  }
  return r;
}

// Kahan-compensated running sum in the working precision, updated on every pair: s carries
// the sum and e the rounding error lost so far (s + e is the compensated sum).
template <typename T>
struct KahanSum {
  T s, e;
  __device__ __forceinline__ void zero() { s = e = T(0); }
  __device__ __forceinline__ void add(T x) {
    const T y = x + e;
    const T t = s + y;
    e = y - (t - s);
    s = t;
  }
  __device__ __forceinline__ double value() const { return static_cast<double>(s) + static_cast<double>(e); }
};

// Consume one LDS tile: for each of the lane's Q queries, accumulate w*z and w.
// KH = false: plain sums over 64-record blocks, each added into a BlockSum.
// KH = true: a Kahan step on every pair into a KahanSum (about 3 more VALU operations per
// accumulator and pair; the accuracy variant).
// REL = true: relative weights, the squared distance multiplied by the query's sigma
// before the weight is taken (one more multiply per pair).
// TAIL = true: only the first `cnt` records of the tile are data (the chunk's last tile);
// the padding records after them are never visited, so that no weight of theirs, however
// small, reaches the denominator.
template <typename T, int DIM, int PM, int Q, bool DIAG, int UNR, bool KH = false, bool REL = false,
          bool TAIL = false, typename Acc>
__device__ __forceinline__ void fwd_tile(const P4<T>* __restrict__ tl, int64_t jt, int cnt,
                                         const T (&qc)[Q][3], const int64_t (&qi)[Q], T nhp,
                                         const T (&sg)[Q], Acc (&num)[Q], Acc (&den)[Q]) {
  constexpr int CH = 64;
  const int lim = TAIL ? cnt : kTile;
  if constexpr (KH) {
#pragma unroll UNR
    for (int jj = 0; jj < lim; ++jj) {
      const P4<T> d = tl[jj];
      const T dv = (DIM == 3) ? d.w : d.z;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        T r2 = sqdist<T, DIM>(qc[k], d);
        if constexpr (REL) r2 *= sg[k];
        T w = weight_sweep<PM>(r2, nhp);
        if constexpr (DIAG) {
          if (jt + jj == qi[k]) w = T(0);
        }
        num[k].add(w * dv);
        den[k].add(w);
      }
    }
    return;
  }
  auto block = [&](int c0) {
    T an[Q], ad[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      an[k] = T(0);
      ad[k] = T(0);
    }
    const int ce = TAIL ? ((lim - c0) < CH ? (lim - c0) : CH) : CH;
#pragma unroll UNR
    for (int jj = 0; jj < ce; ++jj) {
      const P4<T> d = tl[c0 + jj];
      const T dv = (DIM == 3) ? d.w : d.z;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        T r2 = sqdist<T, DIM>(qc[k], d);
        if constexpr (REL) r2 *= sg[k];
        T w = weight_sweep<PM>(r2, nhp);
        if constexpr (DIAG) {
          if (jt + c0 + jj == qi[k]) w = T(0);
        }
        an[k] = fmaT(w, dv, an[k]);
        ad[k] += w;
      }
      // 2-D, one reciprocal per pair, 2 queries per lane: ask the scheduler to interleave
      // each transcendental with six other VALU instructions rather than issue them in
      // runs (1M x 1M p = 2 forward: 179.0 -> 175.6 ms; in 3-D and with 4 queries per lane
      // it measured slower, so those keep the default order).
      if constexpr (sizeof(T) == 4 && DIM == 2 && Q == 2 && (PM == PM_1 || PM == PM_2)) {
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          __builtin_amdgcn_sched_group_barrier(0x002, 6, 0);  // 6 VALU
          __builtin_amdgcn_sched_group_barrier(0x400, 1, 0);  // 1 transcendental
        }
      }
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      num[k].add(an[k]);
      den[k].add(ad[k]);
    }
  };
  // Unrolled over the tile, the compiler keeps every 64-record block's partial sums live
  // until the tile's end and merges them there (159 VGPRs for the FP32 p = 2 sweep against
  // 95 block by block).  Measured at 1M x 1M (16 data chunks): that is 3% faster for the
  // one-transcendental FP32 weights (2-D p = 2: 188.4 against 193.7 ms; p = 1 and 3, and
  // in 3-D, 4-6%) but slower where the weight needs two transcendentals or more registers:
  // FP32 p = 4 (216.6 against 197.8 ms), p = 2.5 (302.0 against 279.2 ms; the 3-D
  // mixture 87.5 against 81.2 ms) and the general-p exp2 / log2 (299.8 against 285.9 ms at
  // p = 1.7), which go block by block.  FP64 differs by at most 2% either way.
  if constexpr (PM == PM_GEN || (sizeof(T) == 4 && (PM == PM_4 || PM == PM_25))) {
#pragma unroll 1
    for (int c0 = 0; c0 < lim; c0 += CH) block(c0);
  } else {
    for (int c0 = 0; c0 < lim; c0 += CH) block(c0);
  }
}

// Finalise one query from its (num, den) in scaled units.
template <typename T>
__device__ __forceinline__ void fwd_finish(int64_t i, double num, double den, const double* hdr,
                                           T* __restrict__ out_z, double* __restrict__ out_den,
                                           uint8_t* __restrict__ out_flag) {
  out_z[i] = static_cast<T>(num / den);
  if (out_den) out_den[i] = den * hdr[H_DEN_UNIT];
  out_flag[i] = route_of(den, hdr, false);
}

// Register-blocking and occupancy knobs of a sweep kernel: UNR = unroll of the per-record
// loop, WPE = minimum waves per SIMD the register allocation must allow.
// Values measured on MI355X (1M queries x 128K data, 2-D, p = 2): FP32 Q = 4 with a 4-deep
// unroll issues 7.4 VALU lane-slots per pair against 8.3 for Q = 8.  With the 16-chunk
// launch at 1M x 1M, Q = 2 (unroll 4) is faster still for the weights with at most one
// transcendental (p = 2: 189.1 -> 179.0 ms; p = 3: 231.4 -> 223.2 ms; 3-D p = 2: 57.8 ->
// 55.0 ms) and within 1% for p = 2.5 and general p, which keep Q = 4.  In FP64, Q = 2 is
// faster for general p (1036 -> 957 ms) and within 1.2% elsewhere; the FP64 sweeps take it.
// At Q = 2 a deeper unroll pays for p = 3 in 2-D (16-deep: 224.5 -> 214.4 ms; 3-D mixture
// 66.5 -> 68.5 ms, so 3-D keeps 4) and for p = 4 (8-deep: 190.8 -> 188.3 ms, 3-D mixture
// 60.6 -> 59.0 ms); for p = 1 and 2 and in FP64 it is 1-3% slower.  At Q = 4 an 8-deep
// unroll pays for the per-pair Kahan sums (3-D mixture, p = 2.5: 130.5 -> 122.9 ms) and the
// relative weights (2-D p = 8: 301.9 -> 285.2 ms) but not for the plain weights (2-D p = 1.5
// 258.9 -> 263.2 ms, p = 2.5 279.1 -> 285.0 ms); the FP64 general-p sweep is faster 2-deep
// (p = 1.7: 931 -> 894 ms, p = 2: 359 -> 364 ms, so only general p takes it).
template <typename T, int Q, int PM = PM_GEN, int DIM = 2, bool KH = false, bool REL = false>
struct SweepTune {
  static constexpr bool kF32 = sizeof(T) == 4;
  static constexpr int UNR = Q >= 8                            ? 2
                             : (kF32 && Q == 4 && (KH || REL)) ? 8
                             : (!kF32 && Q == 2 && PM == PM_GEN) ? 2
                             : (!kF32 || Q != 2)               ? 4
                             : (PM == PM_3 && DIM == 2)        ? 16
                             : PM == PM_4                      ? 8
                                                               : 4;
  static constexpr int WPE = 1;
};

// REL: relative weights; rmin holds each query's nearest squared distance (FP32 bits,
// scaled units, from k_near_check over all queries) and the sums leave the kernel
// multiplied by sigma^(p/2), i.e. in scaled units like those of the direct form.
template <typename T, int DIM, int L, int PM, int Q, int UNR = SweepTune<T, Q, PM, DIM>::UNR,
          int WPE = SweepTune<T, Q>::WPE, bool KH = false, bool REL = false>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_fwd_sweep(DevPts data, int64_t n, DevPts query, int64_t m,
                                                   int64_t chunk, int split, T nhp, unsigned flags,
                                                   const double* __restrict__ hdr,
                                                   T* __restrict__ out_z,
                                                   double* __restrict__ out_den,
                                                   uint8_t* __restrict__ out_flag,
                                                   double2* __restrict__ part,
                                                   const unsigned long long* __restrict__ rmin,
                                                   double p) {
  __shared__ P4<T> tile[2][kTile];
  const int tid = threadIdx.x;
  const int64_t q0 = static_cast<int64_t>(blockIdx.x) * (kWG * Q);
  const int64_t jb = static_cast<int64_t>(blockIdx.y) * chunk;
  const int64_t je = (jb + chunk < n) ? jb + chunk : n;
  const T s = static_cast<T>(hdr[H_SCALE]);

  T qc[Q][3], sg[Q];
  double fs[Q];
  int64_t qi[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    qi[k] = q0 + tid + static_cast<int64_t>(k) * kWG;
    T c[3] = {T(0), T(0), T(0)};
    sg[k] = T(1);
    fs[k] = 1.0;
    if (qi[k] < m) {
      Loader<T, DIM, L>::query(query, qi[k], c);
      if constexpr (REL) {
        float sgf = 1.0f;
        rel_from_min(__builtin_bit_cast(float, static_cast<unsigned int>(rmin[qi[k]])), p, sgf,
                     fs[k]);
        sg[k] = static_cast<T>(sgf);
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) qc[k][d] = c[d] * s;
  }
  using Acc = std::conditional_t<KH, KahanSum<T>, BlockSum<T>>;
  Acc nacc[Q], dacc[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    nacc[k].zero();
    dacc[k].zero();
  }

  T rc[2][3], rv[2];
  auto fetch = [&](int t) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t j = jb + static_cast<int64_t>(t) * kTile + u * kWG + tid;
      if (j < je) {
        Loader<T, DIM, L>::data(data, j, rc[u], rv[u]);
      } else {  // padding record: far away, zero value -> weight (near) 0
        rc[u][0] = rc[u][1] = rc[u][2] = padT<T>();
        rv[u] = T(0);
      }
    }
  };
  auto put = [&](int b) {
#pragma unroll
    for (int u = 0; u < 2; ++u) tile[b][u * kWG + tid] = stage<T, DIM>(rc[u], rv[u], s);
  };

  const int ntiles = static_cast<int>((je - jb + kTile - 1) / kTile);
  const bool excl = (flags & 1u) != 0;
  if constexpr (sizeof(T) == 8 && PM == PM_GEN) pow_table_init(nhp);  // FP64 weight tables (synchronised below)
  fetch(0);
  put(0);
  __syncthreads();
  for (int t = 0; t < ntiles; ++t) {
    if (t + 1 < ntiles) fetch(t + 1);
    const int64_t jt = jb + static_cast<int64_t>(t) * kTile;
    const int cnt = static_cast<int>((je - jt) < kTile ? (je - jt) : kTile);
    const bool diag = excl && jt < q0 + kWG * Q && q0 < jt + kTile;
    if (cnt < kTile) {
      if (diag)
        fwd_tile<T, DIM, PM, Q, true, 1, KH, REL, true>(tile[t & 1], jt, cnt, qc, qi, nhp, sg, nacc, dacc);
      else
        fwd_tile<T, DIM, PM, Q, false, 1, KH, REL, true>(tile[t & 1], jt, cnt, qc, qi, nhp, sg, nacc, dacc);
    } else if (diag) {
      fwd_tile<T, DIM, PM, Q, true, 1, KH, REL>(tile[t & 1], jt, kTile, qc, qi, nhp, sg, nacc, dacc);
    } else {
      fwd_tile<T, DIM, PM, Q, false, UNR, KH, REL>(tile[t & 1], jt, kTile, qc, qi, nhp, sg, nacc, dacc);
    }
    if (t + 1 < ntiles) put((t + 1) & 1);
    __syncthreads();
  }

#pragma unroll
  for (int k = 0; k < Q; ++k) {
    if (qi[k] < m) {
      double num = nacc[k].value();
      double den = dacc[k].value();
      if constexpr (REL) {
        num *= fs[k];
        den *= fs[k];
      }
      if (split == 1)
        fwd_finish<T>(qi[k], num, den, hdr, out_z, out_den, out_flag);
      else
        part[static_cast<int64_t>(blockIdx.y) * m + qi[k]] = make_double2(num, den);
    }
  }
}

// Nearest-distance check of the candidate queries (route F_CANDIDATE, compacted in `list`,
// *count of them), in three kernels:
//  k_near_init   sets each candidate's minimum to +inf;
//  k_near_check  takes work items (block of kWG * Q candidates, data chunk) in turn: the
//                data chunk goes through LDS tiles as in the forward sweep, each query keeps
//                its smallest squared distance in scaled units (the leave-one-out self pair
//                excluded) and folds it into its minimum by an integer atomic min on the
//                bits of the non-negative value (order-independent, so deterministic).  The
//                data range is cut into as many chunks as keep about kNearGrid workgroups
//                busy when the candidates are few, none when they fill the grid;
//  k_near_finish gives a candidate with a data point closer than 1e-6 of the extent
//                F_FP64, the others F_FP32 (their sweep results stand).
// 5 VALU operations per pair (2 sub, mul + fma, min).
constexpr int kNearGrid = 1024;      // workgroups of the nearest-distance check
constexpr int kNearMinChunk = 8192;  // fewest data points per chunk

template <typename T>
__device__ __forceinline__ unsigned long long min_bits(T v) {  // v >= 0: bits order as values
  if constexpr (sizeof(T) == 4)
    return static_cast<unsigned long long>(__builtin_bit_cast(unsigned int, v));
  else
    return __builtin_bit_cast(unsigned long long, v);
}
template <typename T>
__device__ __forceinline__ T from_min_bits(unsigned long long b) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(float, static_cast<unsigned int>(b));
  else
    return __builtin_bit_cast(double, b);
}

// With list == nullptr every query 0..mall-1 takes part (the relative-weight forward needs
// the nearest distance of each query); otherwise the *count queries of list.
template <typename T>
__global__ __launch_bounds__(kWG) void k_near_init(const int* __restrict__ list, const int* __restrict__ count,
                                                   int64_t mall, unsigned long long* __restrict__ minb) {
  const int64_t cnt = list ? static_cast<int64_t>(*count) : mall;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x; i < cnt;
       i += static_cast<int64_t>(gridDim.x) * kWG)
    minb[list ? list[i] : i] = min_bits(infT<T>());
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_near_finish(const int* __restrict__ list, const int* __restrict__ count,
                                                     const unsigned long long* __restrict__ minb,
                                                     const double* __restrict__ hdr, uint8_t* __restrict__ route) {
  const int cnt = *count;
  const T near = static_cast<T>(hdr[H_NEAR_R2]);
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x; i < cnt;
       i += static_cast<int64_t>(gridDim.x) * kWG) {
    const int q = list[i];
    route[q] = from_min_bits<T>(minb[q]) < near ? F_FP64 : F_FP32;
  }
}

template <typename T, int DIM, int L, int Q, bool EXCL>
__global__ __launch_bounds__(kWG) void k_near_check(DevPts data, int64_t n, DevPts query,
                                                    const int* __restrict__ list,
                                                    const int* __restrict__ count, int64_t mall,
                                                    const double* __restrict__ hdr,
                                                    unsigned long long* __restrict__ minb) {
  __shared__ P4<T> tile[2][kTile];
  const int64_t cnt = list ? static_cast<int64_t>(*count) : mall;
  const int tid = threadIdx.x;
  const T s = static_cast<T>(hdr[H_SCALE]);
  constexpr int64_t kQB = static_cast<int64_t>(kWG) * Q;
  const int64_t nblk = (cnt + kQB - 1) / kQB;
  if (nblk == 0) return;
  // data chunks per candidate block: fill the grid when the candidates are few
  int64_t C = kNearGrid / nblk;
  const int64_t cmax = (n + kNearMinChunk - 1) / kNearMinChunk;
  if (C > cmax) C = cmax;
  if (C < 1) C = 1;
  const int64_t len = ((n + C - 1) / C + kTile - 1) / kTile * kTile;
  C = (n + len - 1) / len;
  const int64_t total = nblk * C;
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {  // uniform over the workgroup
    const int64_t b0 = (w / C) * kQB;
    const int64_t jb = (w % C) * len;
    const int64_t je = jb + len < n ? jb + len : n;
    T qc[Q][3], mn[Q];
    int64_t qi[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int64_t slot = b0 + tid + static_cast<int64_t>(k) * kWG;
      qi[k] = slot < cnt ? (list ? list[slot] : slot) : -1;
      T c[3] = {T(0), T(0), T(0)};
      if (qi[k] >= 0) Loader<T, DIM, L>::query(query, qi[k], c);
#pragma unroll
      for (int d = 0; d < 3; ++d) qc[k][d] = c[d] * s;
      mn[k] = infT<T>();
    }
    T rc[2][3], rv[2];
    auto fetch = [&](int t) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int64_t j = jb + static_cast<int64_t>(t) * kTile + u * kWG + tid;
        if (j < je) {
          Loader<T, DIM, L>::data(data, j, rc[u], rv[u]);
        } else {  // padding record: infinitely far
          rc[u][0] = rc[u][1] = rc[u][2] = infT<T>();
          rv[u] = T(0);
        }
      }
    };
    auto put = [&](int b) {
#pragma unroll
      for (int u = 0; u < 2; ++u) tile[b][u * kWG + tid] = stage<T, DIM>(rc[u], rv[u], s);
    };
    const int ntiles = static_cast<int>((je - jb + kTile - 1) / kTile);
    fetch(0);
    put(0);
    __syncthreads();
    for (int t = 0; t < ntiles; ++t) {
      if (t + 1 < ntiles) fetch(t + 1);
      const int64_t jt = jb + static_cast<int64_t>(t) * kTile;
      const P4<T>* tl = tile[t & 1];
#pragma unroll 4
      for (int jj = 0; jj < kTile; ++jj) {
        const P4<T> d = tl[jj];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          T r2 = sqdist<T, DIM>(qc[k], d);
          if constexpr (EXCL) r2 = (jt + jj == qi[k]) ? infT<T>() : r2;
          mn[k] = r2 < mn[k] ? r2 : mn[k];
        }
      }
      if (t + 1 < ntiles) put((t + 1) & 1);
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < Q; ++k)
      if (qi[k] >= 0) atomicMin(&minb[qi[k]], min_bits(mn[k]));
  }
}

// FP64 recomputation of flagged queries.  The pattern of the improved CDP version
// (Section 3.1): a block of threads strides over the data points of one query with
// ceil(len / 256) points per lane, then a block reduction.  When few queries are flagged,
// each query's data range is cut into C chunks swept by different workgroups (C from the
// flagged count, so the grid of kFixGrid workgroups stays busy); chunk partials are
// merged in chunk order by k_fwd_fixmerge.  Exact d == 0 detection, Neumaier sums per lane,
// fixed-order tree reductions.  Writes Z and D (caller units; +inf at an exact hit, whose
// Z is the mean of the coincident values).
__device__ __forceinline__ int fix_chunks(int cnt, int cmax) {
  if (cnt <= 0) return 0;
  int c = kFixGrid / cnt;
  if (c > cmax) c = cmax;
  return c < 1 ? 1 : c;
}

template <typename T, int DIM, int L, int PM>
__global__ __launch_bounds__(kWG) void k_fwd_fixup(DevPts data, int64_t n, DevPts query,
                                                   double nhp, unsigned flags,
                                                   const int* __restrict__ list,
                                                   const int* __restrict__ count, int cmax,
                                                   double4* __restrict__ fpart,
                                                   T* __restrict__ out_z,
                                                   double* __restrict__ out_den) {
  __shared__ double red[kWG];
  __shared__ long long redi[kWG];
  const int cnt = *count;
  const int C = fix_chunks(cnt, cmax);
  const int64_t total = static_cast<int64_t>(cnt) * C;
  const int64_t len = C > 0 ? (n + C - 1) / C : 0;
  const bool excl = (flags & 1u) != 0;
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int sl = static_cast<int>(w / C);
    const int64_t c = w % C;
    const int64_t i = list[sl];
    const int64_t j0 = c * len;
    const int64_t j1 = (j0 + len < n) ? j0 + len : n;
    T qt[3] = {T(0), T(0), T(0)};
    Loader<T, DIM, L>::query(query, i, qt);
    NSum num, den;
    double hz = 0.0;
    long long h = 0;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += kWG) {
      if (excl && j == i) continue;
      T cc[3] = {T(0), T(0), T(0)}, v;
      Loader<T, DIM, L>::data(data, j, cc, v);
      double r2 = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double e = static_cast<double>(qt[d]) - static_cast<double>(cc[d]);
        r2 += e * e;
      }
      if (r2 == 0.0) {
        ++h;
        hz += static_cast<double>(v);
      } else {
        const double wgt = weight<PM>(r2, nhp);
        num.add(wgt * static_cast<double>(v));
        den.add(wgt);
      }
    }
    const double tn = block_sum(num.value(), red);
    const double td = block_sum(den.value(), red);
    const double thz = block_sum(hz, red);
    const long long th = block_sum_i64(h, redi);
    if (threadIdx.x == 0) {
      if (C == 1) {
        const double Z = th > 0 ? thz / static_cast<double>(th) : tn / td;
        out_z[i] = static_cast<T>(Z);
        if (out_den) out_den[i] = th > 0 ? __builtin_huge_val() : td;
      } else {
        fpart[w] = make_double4(tn, td, thz, static_cast<double>(th));
      }
    }
  }
}

// Merges the chunk partials of split fix-up queries (chunk order, TwoSum) and finalises.
template <typename T>
__global__ __launch_bounds__(kWG) void k_fwd_fixmerge(const int* __restrict__ list,
                                                      const int* __restrict__ count, int cmax,
                                                      const double4* __restrict__ fpart,
                                                      T* __restrict__ out_z,
                                                      double* __restrict__ out_den) {
  const int cnt = *count;
  const int C = fix_chunks(cnt, cmax);
  if (C <= 1) return;
  for (int64_t sl = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x; sl < cnt;
       sl += static_cast<int64_t>(gridDim.x) * kWG) {
    double nh = 0.0, nl = 0.0, dh = 0.0, dl = 0.0, hz = 0.0, h = 0.0;
    for (int c = 0; c < C; ++c) {
      const double4 v = fpart[static_cast<int64_t>(sl) * C + c];
      two_sum_acc(nh, nl, v.x);
      two_sum_acc(dh, dl, v.y);
      hz += v.z;
      h += v.w;
    }
    const int64_t i = list[sl];
    const double Z = h > 0.0 ? hz / h : (nh + nl) / (dh + dl);
    out_z[i] = static_cast<T>(Z);
    if (out_den) out_den[i] = h > 0.0 ? __builtin_huge_val() : dh + dl;
  }
}

// Per-workgroup bounding box of the data coordinates and largest |value|, in the
// kBboxStride-double record of each workgroup.
template <typename T, int DIM, int L>
__global__ __launch_bounds__(kWG) void k_bbox(DevPts data, int64_t n, double* __restrict__ part) {
  __shared__ double red[kWG];
  double mn[3] = {__builtin_huge_val(), __builtin_huge_val(), __builtin_huge_val()};
  double mx[3] = {-__builtin_huge_val(), -__builtin_huge_val(), -__builtin_huge_val()};
  double vm = 0.0;
  for (int64_t j = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x; j < n;
       j += static_cast<int64_t>(gridDim.x) * kWG) {
    T c[3] = {T(0), T(0), T(0)}, v;
    Loader<T, DIM, L>::data(data, j, c, v);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      mn[d] = fmin(mn[d], static_cast<double>(c[d]));
      mx[d] = fmax(mx[d], static_cast<double>(c[d]));
    }
    vm = fmax(vm, fabs(static_cast<double>(v)));
  }
  const int t = threadIdx.x;
  red[t] = vm;
  __syncthreads();
  for (int s = kWG / 2; s > 0; s >>= 1) {
    if (t < s) red[t] = fmax(red[t], red[t + s]);
    __syncthreads();
  }
  if (t == 0) part[blockIdx.x * kBboxStride + 6] = red[0];
  __syncthreads();
  for (int d = 0; d < DIM; ++d) {
    for (int pass = 0; pass < 2; ++pass) {
      red[t] = pass ? mx[d] : mn[d];
      __syncthreads();
      for (int s = kWG / 2; s > 0; s >>= 1) {
        if (t < s) red[t] = pass ? fmax(red[t], red[t + s]) : fmin(red[t], red[t + s]);
        __syncthreads();
      }
      if (t == 0) part[blockIdx.x * kBboxStride + pass * 3 + d] = red[0];
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------------------
// Host launchers for one layout (instantiated once per layout translation unit).
// ---------------------------------------------------------------------------------------
template <typename T, int DIM, int L, int PM>
hipError_t launch_fwd_sweep_q(const FwdArgs& a, hipStream_t st) {
  const int Q = a.q_per_lane;
  const int64_t qpb = static_cast<int64_t>(kWG) * Q;
  dim3 grid(static_cast<unsigned>((a.m + qpb - 1) / qpb), static_cast<unsigned>(a.split));
  const T nhp = static_cast<T>(-0.5 * a.p);
  T* z = static_cast<T*>(a.out_z);
#define IDW_FWD_ARGS                                                                          \
  a.data, a.n, a.query, a.m, a.chunk, a.split, nhp, a.flags, a.hdr, z, a.out_den, a.flag, a.part, \
      a.rmin, a.p
#define IDW_FWD_Q(QQ)                                                                       \
  case QQ:                                                                                  \
    hipLaunchKernelGGL((k_fwd_sweep<T, DIM, L, PM, QQ>), grid, dim3(kWG), 0, st, IDW_FWD_ARGS); \
    break;
  if constexpr (sizeof(T) == 4) {
    using KK = SweepTune<T, 4, PM, DIM, true>;         // per-pair Kahan
    using KR = SweepTune<T, 4, PM, DIM, false, true>;  // relative weights
    using KKR = SweepTune<T, 4, PM, DIM, true, true>;
    using K8 = SweepTune<T, 8>;
    if (a.rel) {  // relative weights: general-p form only
      if constexpr (PM == PM_GEN) {
        if (!a.rmin) return hipErrorInvalidValue;
        if (a.kahan) {
          if (Q != 4) return hipErrorInvalidValue;
          hipLaunchKernelGGL((k_fwd_sweep<T, DIM, L, PM, 4, KKR::UNR, KKR::WPE, true, true>), grid, dim3(kWG), 0,
                             st, IDW_FWD_ARGS);
        } else if (Q == 4) {
          hipLaunchKernelGGL((k_fwd_sweep<T, DIM, L, PM, 4, KR::UNR, KR::WPE, false, true>), grid, dim3(kWG), 0,
                             st, IDW_FWD_ARGS);
        } else if (Q == 8) {
          hipLaunchKernelGGL((k_fwd_sweep<T, DIM, L, PM, 8, K8::UNR, K8::WPE, false, true>), grid, dim3(kWG), 0,
                             st, IDW_FWD_ARGS);
        } else {
          return hipErrorInvalidValue;
        }
        return hipGetLastError();
      } else {
        return hipErrorInvalidValue;
      }
    }
    if (a.kahan) {  // per-pair Kahan variant, 4 queries per lane
      if (Q != 4) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_fwd_sweep<T, DIM, L, PM, 4, KK::UNR, KK::WPE, true>), grid, dim3(kWG), 0, st,
                         IDW_FWD_ARGS);
      return hipGetLastError();
    }
    switch (Q) {
      IDW_FWD_Q(2)
      IDW_FWD_Q(4)
      IDW_FWD_Q(8)
      default:
        return hipErrorInvalidValue;
    }
  } else {
    switch (Q) {
      IDW_FWD_Q(2)
      IDW_FWD_Q(4)
      default:
        return hipErrorInvalidValue;
    }
  }
#undef IDW_FWD_Q
#undef IDW_FWD_ARGS
  return hipGetLastError();
}

template <typename T, int DIM, int L>
hipError_t launch_fwd_sweep_pm(const FwdArgs& a, hipStream_t st) {
  switch (a.pmode) {
    case PM_1: return launch_fwd_sweep_q<T, DIM, L, PM_1>(a, st);
    case PM_2: return launch_fwd_sweep_q<T, DIM, L, PM_2>(a, st);
    case PM_3: return launch_fwd_sweep_q<T, DIM, L, PM_3>(a, st);
    case PM_4: return launch_fwd_sweep_q<T, DIM, L, PM_4>(a, st);
    case PM_25: return launch_fwd_sweep_q<T, DIM, L, PM_25>(a, st);
    default: return launch_fwd_sweep_q<T, DIM, L, PM_GEN>(a, st);
  }
}

template <int L>
hipError_t launch_fwd_sweep(const FwdArgs& a, bool f64, hipStream_t st) {
  if (f64) return a.dim == 3 ? launch_fwd_sweep_pm<double, 3, L>(a, st) : launch_fwd_sweep_pm<double, 2, L>(a, st);
  return a.dim == 3 ? launch_fwd_sweep_pm<float, 3, L>(a, st) : launch_fwd_sweep_pm<float, 2, L>(a, st);
}

template <typename T, int DIM, int L, int PM>
hipError_t launch_fwd_fixup_t(const FwdArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((k_fwd_fixup<T, DIM, L, PM>), dim3(kFixGrid), dim3(kWG), 0, st, a.data,
                     a.n, a.query, -0.5 * a.p, a.flags, a.list, a.count, a.fix_cmax, a.fpart,
                     static_cast<T*>(a.out_z), a.out_den);
  hipLaunchKernelGGL((k_fwd_fixmerge<T>), dim3(4), dim3(kWG), 0, st, a.list, a.count, a.fix_cmax,
                     a.fpart, static_cast<T*>(a.out_z), a.out_den);
  return hipGetLastError();
}

template <typename T, int DIM, int L>
hipError_t launch_fwd_fixup_pm(const FwdArgs& a, hipStream_t st) {
  switch (a.pmode) {
    case PM_1: return launch_fwd_fixup_t<T, DIM, L, PM_1>(a, st);
    case PM_2: return launch_fwd_fixup_t<T, DIM, L, PM_2>(a, st);
    case PM_3: return launch_fwd_fixup_t<T, DIM, L, PM_3>(a, st);
    case PM_4: return launch_fwd_fixup_t<T, DIM, L, PM_4>(a, st);
    case PM_25: return launch_fwd_fixup_t<T, DIM, L, PM_25>(a, st);
    default: return launch_fwd_fixup_t<T, DIM, L, PM_GEN>(a, st);
  }
}

template <int L>
hipError_t launch_fwd_fixup(const FwdArgs& a, bool f64, hipStream_t st) {
  if (f64) return a.dim == 3 ? launch_fwd_fixup_pm<double, 3, L>(a, st) : launch_fwd_fixup_pm<double, 2, L>(a, st);
  return a.dim == 3 ? launch_fwd_fixup_pm<float, 3, L>(a, st) : launch_fwd_fixup_pm<float, 2, L>(a, st);
}

template <typename T, int DIM, int L>
hipError_t launch_near_check_t(const NearArgs& a, hipStream_t st) {
  constexpr int Q = sizeof(T) == 4 ? 4 : 2;
  const unsigned gl = static_cast<unsigned>(a.m < 64 * kWG ? (a.m + kWG - 1) / kWG + 1 : 64);
  const int* list = a.all ? nullptr : a.list;
  if (!a.all && !a.list) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_near_init<T>), dim3(gl), dim3(kWG), 0, st, list, a.count, a.m, a.minb);
  if (a.excl)
    hipLaunchKernelGGL((k_near_check<T, DIM, L, Q, true>), dim3(kNearGrid), dim3(kWG), 0, st, a.data, a.n,
                       a.query, list, a.count, a.m, a.hdr, a.minb);
  else
    hipLaunchKernelGGL((k_near_check<T, DIM, L, Q, false>), dim3(kNearGrid), dim3(kWG), 0, st, a.data, a.n,
                       a.query, list, a.count, a.m, a.hdr, a.minb);
  if (!a.all)
    hipLaunchKernelGGL((k_near_finish<T>), dim3(gl), dim3(kWG), 0, st, a.list, a.count, a.minb, a.hdr, a.route);
  return hipGetLastError();
}

template <int L>
hipError_t launch_near_check(const NearArgs& a, hipStream_t st) {
  if (a.f64) return a.dim == 3 ? launch_near_check_t<double, 3, L>(a, st) : launch_near_check_t<double, 2, L>(a, st);
  return a.dim == 3 ? launch_near_check_t<float, 3, L>(a, st) : launch_near_check_t<float, 2, L>(a, st);
}

template <int L>
hipError_t launch_bbox(const DevPts& d, int64_t n, int dim, bool f64, double* part, int nb,
                       hipStream_t st) {
  if (f64) {
    if (dim == 3)
      hipLaunchKernelGGL((k_bbox<double, 3, L>), dim3(nb), dim3(kWG), 0, st, d, n, part);
    else
      hipLaunchKernelGGL((k_bbox<double, 2, L>), dim3(nb), dim3(kWG), 0, st, d, n, part);
  } else {
    if (dim == 3)
      hipLaunchKernelGGL((k_bbox<float, 3, L>), dim3(nb), dim3(kWG), 0, st, d, n, part);
    else
      hipLaunchKernelGGL((k_bbox<float, 2, L>), dim3(nb), dim3(kWG), 0, st, d, n, part);
  }
  return hipGetLastError();
}

}  // namespace idw
