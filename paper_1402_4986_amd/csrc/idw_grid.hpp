// Uniform grid over the data points for the nearest-distance searches (gfx950).
//
// Two steps need, for some queries, the smallest squared distance to the data (scaled
// units, with the arithmetic of the sweeps): the near-coincidence check of candidate
// queries (does a data point lie closer than 1e-6 of the extent?) and, for the relative
// weights of large p, the nearest distance of every query.  By brute force both are one
// more pass over all pairs of the queries concerned (k_near_check: 5 VALU operations per
// pair, about 120 ms at 1M x 1M).  A uniform grid of about four data points per cell
// answers them from a few cells:
//  - build, per call and in the workspace: count the points of every cell (integer
//    atomics), take the exclusive scan of the counts, and scatter every point's scaled
//    coordinates and index into its cell's slots.  The order inside a cell depends on the
//    atomics; only minima are taken over cells, so every result is order-independent;
//  - fixed radius (candidates): the cells that meet the box q +- r', r' just above the
//    near-coincidence distance, at most 2^dim of them;
//  - nearest (relative weights): rings of cells around the query's cell, until no cell
//    left out can hold a closer point.
// Cells come from the monotone map floor((x - bmin) / h), clamped to the grid, evaluated
// in FP64 on the scaled coordinates, so every point within r' of q in each coordinate lies
// in a visited cell.  The squared distances are those of k_near_check (same scaled values,
// same FP32 or FP64 operations), so the minima, and the routes and scales taken from them,
// equal the brute-force ones bit for bit.  A query whose cells hold too many points
// (clustered data) or whose ring search runs long is appended to a list that the
// brute-force kernels settle instead.
#pragma once

#include <math.h>

#include "idw_device.hpp"
#include "idw_fwd.hpp"
#include "idw_launch.hpp"

namespace idw {

// Dense cells: the per-query budget of the fixed-radius check and the ring search before
// a query is handed to the brute-force kernels.  The ring search's cell budget is per
// dimension: in 3-D a query in empty space between clusters visits (2r + 1)^3 cells by
// ring r, and past two rings a failing search costs more than it saves (262,144 points in
// 16 clusters, 1M uniform queries, p = 8: 147 ms forward with 512 cells, 134 ms with 125;
// uniform 3-D points need at most 2 rings and are unchanged at 80 ms).
constexpr int kGridCapPoints = 4096;
constexpr int kGridCapCells2 = 512;  // 2-D
constexpr int kGridCapCells3 = 125;  // 3-D: rings 0..2
constexpr int kGridMaxRing = 8;

struct GridGeom {
  double bmin[3];
  double h, invh;
  int g[3];
};

__device__ __forceinline__ GridGeom grid_geom(const double* __restrict__ hdr) {
  GridGeom G;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    G.bmin[k] = hdr[H_BMIN + k];
    G.g[k] = static_cast<int>(hdr[H_GRID_G + k]);
  }
  G.h = hdr[H_GRID_H];
  G.invh = hdr[H_GRID_INVH];
  return G;
}

// Cell coordinate of scaled coordinate v along one axis (monotone in v).
__device__ __forceinline__ int cell1(double v, double bmin, double invh, int g) {
  double t = floor((v - bmin) * invh);
  t = fmin(fmax(t, 0.0), static_cast<double>(g - 1));
  return static_cast<int>(t);
}

template <typename T>
__device__ __forceinline__ int cell_of(const T (&c)[3], const GridGeom& G) {
  const int i0 = cell1(static_cast<double>(c[0]), G.bmin[0], G.invh, G.g[0]);
  const int i1 = cell1(static_cast<double>(c[1]), G.bmin[1], G.invh, G.g[1]);
  const int i2 = cell1(static_cast<double>(c[2]), G.bmin[2], G.invh, G.g[2]);
  return (i2 * G.g[1] + i1) * G.g[0] + i0;
}

// The point index rides in the fourth slot of a grid record (bit pattern, no arithmetic).
__device__ __forceinline__ float idx_slot(float, int64_t j) {
  return __builtin_bit_cast(float, static_cast<unsigned int>(j));
}
__device__ __forceinline__ double idx_slot(double, int64_t j) {
  return __builtin_bit_cast(double, static_cast<unsigned long long>(j));
}
__device__ __forceinline__ int64_t slot_idx(float v) {
  return static_cast<int64_t>(__builtin_bit_cast(unsigned int, v));
}
__device__ __forceinline__ int64_t slot_idx(double v) {
  return static_cast<int64_t>(__builtin_bit_cast(unsigned long long, v));
}

// Scaled coordinates of data point j, as staged by the sweeps (c * s in T); unused axes 0.
template <typename T, int DIM, int L>
__device__ __forceinline__ void scaled_data(const DevPts& data, int64_t j, T s, T (&c)[3]) {
  T v, r[3] = {T(0), T(0), T(0)};
  Loader<T, DIM, L>::data(data, j, r, v);
  const P4<T> st = stage<T, DIM>(r, v, s);
  c[0] = st.x;
  c[1] = st.y;
  c[2] = DIM == 3 ? st.z : T(0);
}

// ---- build: count, then (after the scan) scatter ----
template <typename T, int DIM, int L>
__global__ __launch_bounds__(kWG) void k_grid_count(DevPts data, int64_t n, const double* __restrict__ hdr,
                                                    const int* __restrict__ hint, int* __restrict__ cnt) {
  if (hint[GI_GRID] <= 0) return;
  const GridGeom G = grid_geom(hdr);
  const T s = static_cast<T>(hdr[H_SCALE]);
  for (int64_t j = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x; j < n;
       j += static_cast<int64_t>(gridDim.x) * kWG) {
    T c[3];
    scaled_data<T, DIM, L>(data, j, s, c);
    atomicAdd(&cnt[cell_of(c, G)], 1);
  }
}

template <typename T, int DIM, int L>
__global__ __launch_bounds__(kWG) void k_grid_scatter(DevPts data, int64_t n, const double* __restrict__ hdr,
                                                      const int* __restrict__ hint, int* __restrict__ cursor,
                                                      P4<T>* __restrict__ rec) {
  if (hint[GI_GRID] <= 0) return;
  const GridGeom G = grid_geom(hdr);
  const T s = static_cast<T>(hdr[H_SCALE]);
  for (int64_t j = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x; j < n;
       j += static_cast<int64_t>(gridDim.x) * kWG) {
    T c[3];
    scaled_data<T, DIM, L>(data, j, s, c);
    const int pos = atomicAdd(&cursor[cell_of(c, G)], 1);
    P4<T> r;
    r.x = c[0];
    r.y = c[1];
    r.z = c[2];
    r.w = idx_slot(T(0), j);
    rec[pos] = r;
  }
}

// Squared distance of a query to a grid record: the operations of sqdist on the same
// scaled values.
template <typename T, int DIM>
__device__ __forceinline__ T grid_r2(const T (&q)[3], const P4<T>& r) {
  return sqdist<T, DIM>(q, r);
}

// ---- fixed-radius check of the candidate queries (list, hint[GI_GRID] of them) ----
// Writes F_FP64 / F_FP32 as k_near_finish would, or appends the query to blist.
template <typename T, int DIM, int L, bool EXCL>
__global__ __launch_bounds__(kWG) void k_grid_check(DevPts query, const int* __restrict__ list,
                                                    const double* __restrict__ hdr, int* __restrict__ hint,
                                                    const int* __restrict__ start, const P4<T>* __restrict__ rec,
                                                    uint8_t* __restrict__ route, int* __restrict__ blist) {
  const int cnt = hint[GI_GRID];
  if (cnt <= 0) return;
  const GridGeom G = grid_geom(hdr);
  const T s = static_cast<T>(hdr[H_SCALE]);
  const T nearT = static_cast<T>(hdr[H_NEAR_R2]);
  // Every point whose computed r2 is below nearT differs from q by less than this in each
  // scaled coordinate (the rounding of the subtraction and the sums is far below 1e-4).
  const double rp = sqrt(hdr[H_NEAR_R2]) * 1.0001;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x; i < cnt;
       i += static_cast<int64_t>(gridDim.x) * kWG) {
    const int64_t q = list[i];
    T c[3] = {T(0), T(0), T(0)};
    Loader<T, DIM, L>::query(query, q, c);
    T qs[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) qs[k] = c[k] * s;
    int lo[3], hi[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double v = static_cast<double>(qs[k]);
      lo[k] = k < DIM ? cell1(v - rp, G.bmin[k], G.invh, G.g[k]) : 0;
      hi[k] = k < DIM ? cell1(v + rp, G.bmin[k], G.invh, G.g[k]) : 0;
    }
    int64_t work = 0;
    for (int z = lo[2]; z <= hi[2]; ++z)
      for (int y = lo[1]; y <= hi[1]; ++y)
        for (int x = lo[0]; x <= hi[0]; ++x) {
          const int id = (z * G.g[1] + y) * G.g[0] + x;
          work += start[id + 1] - start[id];
        }
    if (work > kGridCapPoints) {
      blist[atomicAdd(&hint[GI_FALLBACK], 1)] = static_cast<int>(q);
      continue;
    }
    T mn = infT<T>();
    for (int z = lo[2]; z <= hi[2]; ++z)
      for (int y = lo[1]; y <= hi[1]; ++y)
        for (int x = lo[0]; x <= hi[0]; ++x) {
          const int id = (z * G.g[1] + y) * G.g[0] + x;
          const int e = start[id + 1];
          for (int p = start[id]; p < e; ++p) {
            const P4<T> r = rec[p];
            if (EXCL && slot_idx(r.w) == q) continue;
            const T r2 = grid_r2<T, DIM>(qs, r);
            mn = r2 < mn ? r2 : mn;
          }
        }
    route[q] = mn < nearT ? F_FP64 : F_FP32;
  }
}

// ---- nearest squared distance of queries 0 .. hint[GI_GRID]-1 (ring search) ----
// Writes minb[q] (bits of the minimum, as k_near_check leaves them), or appends q to blist.
template <typename T, int DIM, int L, bool EXCL>
__global__ __launch_bounds__(kWG) void k_grid_nearest(DevPts query, const double* __restrict__ hdr,
                                                      int* __restrict__ hint, const int* __restrict__ start,
                                                      const P4<T>* __restrict__ rec,
                                                      unsigned long long* __restrict__ minb,
                                                      int* __restrict__ blist) {
  const int cnt = hint[GI_GRID];
  if (cnt <= 0) return;
  const GridGeom G = grid_geom(hdr);
  const T s = static_cast<T>(hdr[H_SCALE]);
  // Margins of the stopping test: a point's cell coordinate can be off by about 2^-30 of a
  // cell near a face (FP64 rounding of (x - bmin) / h), and its FP32 r2 below the exact
  // squared distance by a few ulp.
  const double slack = G.h * 0x1p-28;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x; i < cnt;
       i += static_cast<int64_t>(gridDim.x) * kWG) {
    const int64_t q = i;
    T c[3] = {T(0), T(0), T(0)};
    Loader<T, DIM, L>::query(query, q, c);
    T qs[3];
    double qd[3];
    int c0[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      qs[k] = c[k] * s;
      qd[k] = static_cast<double>(qs[k]);
      c0[k] = k < DIM ? cell1(qd[k], G.bmin[k], G.invh, G.g[k]) : 0;
    }
    T best = infT<T>();
    int points = 0, cells = 0;
    bool done = false;
    for (int ring = 0; ring <= kGridMaxRing && !done; ++ring) {
      int lo[3], hi[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        lo[k] = k < DIM ? max(c0[k] - ring, 0) : 0;
        hi[k] = k < DIM ? min(c0[k] + ring, G.g[k] - 1) : 0;
      }
      bool over = false;
      for (int z = lo[2]; z <= hi[2] && !over; ++z)
        for (int y = lo[1]; y <= hi[1] && !over; ++y)
          for (int x = lo[0]; x <= hi[0] && !over; ++x) {
            const int dcheb = max(max(abs(x - c0[0]), abs(y - c0[1])), abs(z - c0[2]));
            if (dcheb != ring) continue;  // inner cells were visited by earlier rings
            const int id = (z * G.g[1] + y) * G.g[0] + x;
            const int b = start[id], e = start[id + 1];
            points += e - b;
            if (++cells > (DIM == 3 ? kGridCapCells3 : kGridCapCells2) || points > kGridCapPoints) {
              over = true;
              break;
            }
            for (int p = b; p < e; ++p) {
              const P4<T> r = rec[p];
              if (EXCL && slot_idx(r.w) == q) continue;
              const T r2 = grid_r2<T, DIM>(qs, r);
              best = r2 < best ? r2 : best;
            }
          }
      if (over) break;
      // Distance from q to the nearest face of the visited block that has cells beyond it.
      double bound = __builtin_huge_val();
      bool more = false;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        if (c0[k] - ring > 0) {
          more = true;
          bound = fmin(bound, qd[k] - (G.bmin[k] + (c0[k] - ring) * G.h));
        }
        if (c0[k] + ring < G.g[k] - 1) {
          more = true;
          bound = fmin(bound, G.bmin[k] + (c0[k] + ring + 1) * G.h - qd[k]);
        }
      }
      if (!more) {
        done = true;  // every cell visited
      } else {
        const double bb = bound - slack;
        if (bb > 0.0 && static_cast<double>(best) < bb * bb * (1.0 - 0x1p-20)) done = true;
      }
    }
    if (done)
      minb[q] = min_bits(best);
    else
      blist[atomicAdd(&hint[GI_FALLBACK], 1)] = static_cast<int>(q);
  }
}

// ---- host launchers for one layout ----
template <typename T, int DIM, int L>
hipError_t launch_grid_build_t(const GridArgs& a, hipStream_t st) {
  const int64_t nb = (a.n + kWG - 1) / kWG;
  const unsigned grid = static_cast<unsigned>(nb < 4096 ? nb : 4096);
  hipLaunchKernelGGL((k_grid_count<T, DIM, L>), dim3(grid), dim3(kWG), 0, st, a.data, a.n, a.hdr, a.hint, a.cnt);
  hipError_t e = grid_scan(a, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_grid_scatter<T, DIM, L>), dim3(grid), dim3(kWG), 0, st, a.data, a.n, a.hdr, a.hint, a.cnt,
                     static_cast<P4<T>*>(a.rec));
  return hipGetLastError();
}

template <typename T, int DIM, int L>
hipError_t launch_grid_search_t(const GridArgs& a, hipStream_t st) {
  const int64_t nb = (a.m + kWG - 1) / kWG;
  const unsigned grid = static_cast<unsigned>(nb < 4096 ? (nb > 0 ? nb : 1) : 4096);
  const P4<T>* rec = static_cast<const P4<T>*>(a.rec);
  if (a.nearest) {
    if (a.excl)
      hipLaunchKernelGGL((k_grid_nearest<T, DIM, L, true>), dim3(grid), dim3(kWG), 0, st, a.query, a.hdr, a.hint,
                         a.start, rec, a.minb, a.blist);
    else
      hipLaunchKernelGGL((k_grid_nearest<T, DIM, L, false>), dim3(grid), dim3(kWG), 0, st, a.query, a.hdr, a.hint,
                         a.start, rec, a.minb, a.blist);
  } else {
    if (a.excl)
      hipLaunchKernelGGL((k_grid_check<T, DIM, L, true>), dim3(grid), dim3(kWG), 0, st, a.query, a.list, a.hdr,
                         a.hint, a.start, rec, a.route, a.blist);
    else
      hipLaunchKernelGGL((k_grid_check<T, DIM, L, false>), dim3(grid), dim3(kWG), 0, st, a.query, a.list, a.hdr,
                         a.hint, a.start, rec, a.route, a.blist);
  }
  return hipGetLastError();
}

template <int L>
hipError_t launch_grid(const GridArgs& a, bool build, hipStream_t st) {
  if (a.f64) {
    if (a.dim == 3) return build ? launch_grid_build_t<double, 3, L>(a, st) : launch_grid_search_t<double, 3, L>(a, st);
    return build ? launch_grid_build_t<double, 2, L>(a, st) : launch_grid_search_t<double, 2, L>(a, st);
  }
  if (a.dim == 3) return build ? launch_grid_build_t<float, 3, L>(a, st) : launch_grid_search_t<float, 3, L>(a, st);
  return build ? launch_grid_build_t<float, 2, L>(a, st) : launch_grid_search_t<float, 2, L>(a, st);
}

}  // namespace idw
