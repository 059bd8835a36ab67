// Adjoint of the IDW forward sweep (Eq. 1 differentiated with respect to z, p and q).
//
// For a query i that is not flagged (no data point within 1e-6 of the extent):
//   dZ_i/dz_j = w_ij / D_i
//   dZ_i/dp   = -(1/D_i) sum_j w_ij (1/2) ln(r2_ij) (z_j - Z_i)
//   dZ_i/dq_i = -(p/D_i) sum_j (w_ij / r2_ij) (z_j - Z_i) (q_i - x_j)
// The centred factor (z_j - Z_i) keeps the p and q sums free of the cancellation of
// sum w ln(r2) z - Z sum w ln(r2).
//
// Three sweeps:
//  * query sweep: lanes own queries, data tiles broadcast from LDS; accumulates
//    P_i = sum w (z - Z) log2(r2) and G_i = sum (w/r2)(z - Z)(q - x) over 64-record
//    blocks added into BlockSum running sums;
//    writes per-(data chunk, query) partials that a merge kernel turns into dq_i and
//    per-workgroup dp partials in a fixed order;
//  * data sweep: lanes own data points, query tiles (q_i, a_i = g_i / D_i) broadcast from
//    LDS; accumulates dz_j = sum_i a_i w_ij;
//  * FP64 fix-up for flagged queries (exact hits and near-coincident points): a per-query
//    workgroup recomputes Z, D, dq and dp exactly, and a data-parallel pass adds their dz
//    (and dx) contributions in ascending query order.
// The gradient with respect to the data coordinates,
//   dZ_i/dx_j = (p/D_i)(w_ij / r2_ij)(z_j - Z_i)(q_i - x_j),
// is a data-direction sum like dz; it has its own data sweep (k_bwd_datax, which also
// yields dz) and rides the fused FP32 sweep.
#pragma once

#include <math.h>

#include "idw_device.hpp"
#include "idw_fwd.hpp"
#include "idw_launch.hpp"

namespace idw {

// w, a factor f for w / r2 (when the position gradient is needed), and log2(r2) (when the
// power gradient is needed), in the cheapest form for the weight class.  For the fast
// classes f = 1/r2 (w / r2 = w f); for general p f = w / r2 itself, taken as
// 2^((-p/2 - 1) log2 r2) with w = f r2, which spares a reciprocal.  wr_times forms
// (w / r2) c from either.  POW (FP64, general p, no dp) takes the weight or w / r2 from the
// tables of pow_t instead: the kernel fills them for the exponent nh - 1 when NDQ, else nh.
template <int PM, bool NDQ, bool NDP, bool POW = false>
__device__ __forceinline__ void wterms(float r2, float nhp, float& w, float& f, float& lg) {
  if constexpr (PM == PM_GEN) {
    lg = __builtin_amdgcn_logf(r2);
    if constexpr (NDQ) {
      f = __builtin_amdgcn_exp2f((nhp - 1.0f) * lg);
      w = f * r2;
    } else {
      w = __builtin_amdgcn_exp2f(nhp * lg);
    }
  } else {
    if constexpr (NDP) lg = __builtin_amdgcn_logf(r2);
    if constexpr (PM == PM_2) {
      w = __builtin_amdgcn_rcpf(r2);
      if constexpr (NDQ) f = w;
    } else if constexpr (PM == PM_1) {
      w = __builtin_amdgcn_rsqf(r2);
      if constexpr (NDQ) f = w * w;
    } else if constexpr (PM == PM_3) {
      const float s = __builtin_amdgcn_rsqf(r2);
      const float s2 = s * s;
      w = s2 * s;
      if constexpr (NDQ) f = s2;
    } else if constexpr (PM == PM_4) {
      const float t = __builtin_amdgcn_rcpf(r2);
      w = t * t;
      if constexpr (NDQ) f = t;
    } else {  // PM_25
      const float s = __builtin_amdgcn_rsqf(r2);
      const float s2 = s * s;
      w = s2 * __builtin_amdgcn_sqrtf(s);
      if constexpr (NDQ) f = s2;
    }
  }
}

template <int PM, bool NDQ, bool NDP, bool POW = false>
__device__ __forceinline__ void wterms(double r2, double nhp, double& w, double& f, double& lg) {
  static_assert(!POW || (PM == PM_GEN && !NDP), "the pow tables serve general p without dp");
  if constexpr (POW) {  // pow_table_init in the kernel
    const double g = pow_t(r2);
    if constexpr (NDQ) {
      f = g;
      w = g * r2;
    } else {
      w = g;
    }
    return;
  }
  if constexpr (NDP || PM == PM_GEN) lg = log2_t(r2);  // log2_table_init in the kernel
  if constexpr (PM == PM_GEN) {  // exp2_table_init in the kernel
    if constexpr (NDQ) {
      f = exp2_t((nhp - 1.0) * lg);
      w = f * r2;
    } else {
      w = exp2_t(nhp * lg);
    }
  } else if constexpr (PM == PM_2) {
    w = rcp64_w(r2);
    if constexpr (NDQ) f = w;
  } else if constexpr (PM == PM_4) {
    const double t = rcp64_w(r2);
    w = t * t;
    if constexpr (NDQ) f = t;
  } else {
    w = weight_sweep<PM>(r2, nhp);
    if constexpr (NDQ) f = rcp64_w(r2);
  }
}

// Whether an FP64 sweep takes its general-p weights from the pow_t tables: only without dp
// (whose log2 r2 the exp2/log2 route shares; a combined log2 and pow measured slower there,
// its registers and LDS costing occupancy).
template <typename T, int PM, bool NDP>
struct PowTab {
  static constexpr bool on = sizeof(T) == 8 && PM == PM_GEN && !NDP;
};

// (w / r2) c from t = w c and wterms' factor f.
template <int PM, typename T>
__device__ __forceinline__ T wr_times(T t, T c, T f) {
  if constexpr (PM == PM_GEN)
    return f * c;
  else
    return t * f;
}

// One LDS tile of the query sweep.  `cnt` records are valid (all of them unless TAIL).
template <typename T, int DIM, int PM, int Q, bool DIAG, bool TAIL, bool NDP, bool NDQ, int UNR>
__device__ __forceinline__ void bwdq_tile(const P4<T>* __restrict__ tl, int cnt, int64_t jt,
                                          const T (&qc)[Q][3], const T (&zq)[Q],
                                          const int64_t (&qi)[Q], T nhp, BlockSum<T> (&P)[Q],
                                          BlockSum<T> (&G)[Q][3]) {
  constexpr int CH = 64;
  const int lim = TAIL ? cnt : kTile;
  // One 64-record block at a time, merged before the next: unrolled over the tile, the
  // compiler keeps every block's sums live to the tile's end (FP32 p = 2 with dp and dq:
  // 127 VGPRs against 78; FP64: 249 against 148).  Measured at 1M x 1M, block by block is
  // 2% faster for dq alone in FP32 and 3% for the FP64 query + data sweeps.
#pragma unroll 1
  for (int c0 = 0; c0 < lim; c0 += CH) {
    T ap[Q], ag[Q][3];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      ap[k] = T(0);
      ag[k][0] = ag[k][1] = ag[k][2] = T(0);
    }
    const int ce = TAIL ? ((lim - c0) < CH ? (lim - c0) : CH) : CH;
#pragma unroll UNR
    for (int jj = 0; jj < ce; ++jj) {
      const P4<T> d = tl[c0 + jj];
      const T dv = (DIM == 3) ? d.w : d.z;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const T dx = qc[k][0] - d.x;
        const T dy = qc[k][1] - d.y;
        T dz = T(0);
        T r2 = dx * dx;
        r2 = fmaT(dy, dy, r2);
        if constexpr (DIM == 3) {
          dz = qc[k][2] - d.z;
          r2 = fmaT(dz, dz, r2);
        }
        T c = dv - zq[k];
        if constexpr (DIAG) {
          if (jt + c0 + jj == qi[k]) {
            r2 = T(1);
            c = T(0);
          }
        }
        T w, f = T(0), lg = T(0);
        wterms<PM, NDQ, NDP, PowTab<T, PM, NDP>::on>(r2, nhp, w, f, lg);
        const T t = w * c;
        if constexpr (NDP) ap[k] = fmaT(t, lg, ap[k]);
        if constexpr (NDQ) {
          const T u = wr_times<PM>(t, c, f);  // (w / r2) (z - Z)
          ag[k][0] = fmaT(u, dx, ag[k][0]);
          ag[k][1] = fmaT(u, dy, ag[k][1]);
          if constexpr (DIM == 3) ag[k][2] = fmaT(u, dz, ag[k][2]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if constexpr (NDP) P[k].add(ap[k]);
      if constexpr (NDQ) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) G[k][d].add(ag[k][d]);
      }
    }
  }
}

// Query sweep: writes part[c * m + i] = (P, Gx, Gy, Gz) in scaled units (double).
// Measured on MI355X: FP32 Q = 2, unroll 4, >= 2 waves per SIMD (13.8 lane-slots per pair
// for 2-D p = 2 with dp and dq, against 14.6 for Q = 4).
template <typename T, int Q>
struct QueryTune {
  static constexpr int UNR = 4;
  static constexpr int WPE = (Q <= 2) ? 2 : 1;
};

template <typename T, int DIM, int L, int PM, int Q, bool NDP, bool NDQ,
          int UNR = QueryTune<T, Q>::UNR, int WPE = QueryTune<T, Q>::WPE>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_bwd_query(DevPts data, int64_t n, DevPts query, int64_t m,
                                                   int64_t chunk, T nhp, unsigned flags,
                                                   const double* __restrict__ hdr,
                                                   const T* __restrict__ saved_z,
                                                   double4* __restrict__ part) {
  __shared__ P4<T> tile[2][kTile];
  const int tid = threadIdx.x;
  const int64_t q0 = static_cast<int64_t>(blockIdx.x) * (kWG * Q);
  const int64_t jb = static_cast<int64_t>(blockIdx.y) * chunk;
  const int64_t je = (jb + chunk < n) ? jb + chunk : n;
  const T s = static_cast<T>(hdr[H_SCALE]);

  T qc[Q][3], zq[Q];
  int64_t qi[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    qi[k] = q0 + tid + static_cast<int64_t>(k) * kWG;
    T c[3] = {T(0), T(0), T(0)};
    zq[k] = T(0);
    if (qi[k] < m) {
      Loader<T, DIM, L>::query(query, qi[k], c);
      zq[k] = saved_z[qi[k]];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) qc[k][d] = c[d] * s;
  }
  BlockSum<T> P[Q], G[Q][3];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    P[k].zero();
#pragma unroll
    for (int d = 0; d < 3; ++d) G[k][d].zero();
  }

  T rc[2][3], rv[2];
  auto fetch = [&](int t) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t j = jb + static_cast<int64_t>(t) * kTile + u * kWG + tid;
      rc[u][0] = rc[u][1] = rc[u][2] = T(0);
      rv[u] = T(0);
      if (j < je) Loader<T, DIM, L>::data(data, j, rc[u], rv[u]);
    }
  };
  auto put = [&](int b) {
#pragma unroll
    for (int u = 0; u < 2; ++u) tile[b][u * kWG + tid] = stage<T, DIM>(rc[u], rv[u], s);
  };

  const int ntiles = static_cast<int>((je - jb + kTile - 1) / kTile);
  const bool excl = (flags & 1u) != 0;
  constexpr bool kPow = PowTab<T, PM, NDP>::on;
  if constexpr (kPow) pow_table_init(NDQ ? nhp - 1.0 : nhp);  // FP64 tables (synchronised below)
  if constexpr (sizeof(T) == 8 && !kPow && (PM == PM_GEN || NDP)) log2_table_init();
  if constexpr (sizeof(T) == 8 && !kPow && PM == PM_GEN) exp2_table_init();
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
        bwdq_tile<T, DIM, PM, Q, true, true, NDP, NDQ, 1>(tile[t & 1], cnt, jt, qc, zq, qi, nhp, P, G);
      else
        bwdq_tile<T, DIM, PM, Q, false, true, NDP, NDQ, 1>(tile[t & 1], cnt, jt, qc, zq, qi, nhp, P, G);
    } else {
      if (diag)
        bwdq_tile<T, DIM, PM, Q, true, false, NDP, NDQ, 1>(tile[t & 1], cnt, jt, qc, zq, qi, nhp, P, G);
      else
        bwdq_tile<T, DIM, PM, Q, false, false, NDP, NDQ, UNR>(tile[t & 1], cnt, jt, qc, zq, qi, nhp, P, G);
    }
    if (t + 1 < ntiles) put((t + 1) & 1);
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    if (qi[k] < m) {
      double4 r;
      r.x = P[k].value();
      r.y = G[k][0].value();
      r.z = G[k][1].value();
      r.w = G[k][2].value();
      part[static_cast<int64_t>(blockIdx.y) * m + qi[k]] = r;
    }
  }
}

// Merges query-sweep partials: dq_i for unflagged queries, dp partial per workgroup.
template <typename T, int DIM>
__global__ __launch_bounds__(kWG) void k_bwd_qmerge(const double4* __restrict__ part, int64_t m,
                                                    int split, double p,
                                                    const double* __restrict__ hdr,
                                                    const T* __restrict__ grad_out,
                                                    const double* __restrict__ saved_den,
                                                    T* __restrict__ grad_q,
                                                    double* __restrict__ wg_dp,
                                                    const uint8_t* __restrict__ route) {
  __shared__ double red[kWG];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  double dpi = 0.0;
  if (i < m) {
    const double D = saved_den[i];
    if (route[i] == F_FP32) {  // the others come from the FP64 fix-up
      double P[2] = {0.0, 0.0}, G[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
      for (int c = 0; c < split; ++c) {
        const double4 v = part[static_cast<int64_t>(c) * m + i];
        two_sum_acc(P[0], P[1], v.x);
        two_sum_acc(G[0][0], G[0][1], v.y);
        two_sum_acc(G[1][0], G[1][1], v.z);
        two_sum_acc(G[2][0], G[2][1], v.w);
      }
      double Ds = D / hdr[H_DEN_UNIT];  // denominator in the sweep's scaled units
      double sig = 1.0;
      // Relative weights: the sweep's sums are sigma^(-p/2) P and sigma^(-p/2 - 1) G, and
      // E = Ds sigma^(-p/2) takes the place of Ds.
      if (hdr[H_REL] != 0.0) {
        float sg = 1.f, k = 0.f;
        double E = 1.0;
        rel_from_den(Ds, p, sg, k, E);
        Ds = E;
        sig = static_cast<double>(sg);
      }
      const double g = static_cast<double>(grad_out[i]);
      // ln(r2) = log2(r2) * ln 2; dZ/dp = -(1/D) sum w (1/2) ln(r2) (z - Z).
      dpi = -(g / Ds) * 0.5 * 0.69314718055994530942 * (P[0] + P[1]);
      if (grad_q) {
        const double f = -(p * g / Ds) * sig * hdr[H_SCALE];
#pragma unroll
        for (int d = 0; d < DIM; ++d) grad_q[i * DIM + d] = static_cast<T>(f * (G[d][0] + G[d][1]));
      }
    }
  }
  const double tot = block_sum(dpi, red);
  if (threadIdx.x == 0 && wg_dp) wg_dp[blockIdx.x] = tot;
}

// One LDS tile of the data sweep: for the lane's Q data points, accumulate a_i * w_ij.
template <typename T, int DIM, int PM, int Q, bool DIAG, int UNR>
__device__ __forceinline__ void bwdd_tile(const P4<T>* __restrict__ tl, int64_t it,
                                          const T (&xc)[Q][3], const int64_t (&xj)[Q], T nhp,
                                          BlockSum<T> (&Zs)[Q]) {
  constexpr int CH = 64;
  for (int c0 = 0; c0 < kTile; c0 += CH) {
    T az[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) az[k] = T(0);
#pragma unroll UNR
    for (int ii = 0; ii < CH; ++ii) {
      const P4<T> d = tl[c0 + ii];
      const T a = (DIM == 3) ? d.w : d.z;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const T r2 = sqdist<T, DIM>(xc[k], d);
        T w = weight_sweep<PM>(r2, nhp);
        if constexpr (DIAG) {
          if (it + c0 + ii == xj[k]) w = T(0);
        }
        az[k] = fmaT(a, w, az[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) Zs[k].add(az[k]);
  }
}

// Data sweep: part[c * n + j] = sum over query chunk c of a_i w_ij (double).
// Measured on MI355X: FP32 Q = 4, unroll 4, >= 2 waves per SIMD (6.8 lane-slots per pair).
template <typename T, int Q>
struct DataTune {
  static constexpr int UNR = 4;
  static constexpr int WPE = 2;
};

template <typename T, int DIM, int L, int PM, int Q, int UNR = DataTune<T, Q>::UNR,
          int WPE = DataTune<T, Q>::WPE>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_bwd_data(DevPts data, int64_t n, DevPts query, int64_t m,
                                                  int64_t chunk, T nhp, unsigned flags,
                                                  const double* __restrict__ hdr,
                                                  const T* __restrict__ grad_out,
                                                  const double* __restrict__ saved_den,
                                                  double* __restrict__ part,
                                                  const uint8_t* __restrict__ route) {
  __shared__ P4<T> tile[2][kTile];
  const int tid = threadIdx.x;
  const int64_t x0 = static_cast<int64_t>(blockIdx.x) * (kWG * Q);
  const int64_t ib = static_cast<int64_t>(blockIdx.y) * chunk;
  const int64_t ie = (ib + chunk < m) ? ib + chunk : m;
  const T s = static_cast<T>(hdr[H_SCALE]);
  const double unit = hdr[H_DEN_UNIT];

  T xc[Q][3];
  int64_t xj[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    xj[k] = x0 + tid + static_cast<int64_t>(k) * kWG;
    T c[3] = {T(0), T(0), T(0)}, v = T(0);
    if (xj[k] < n) Loader<T, DIM, L>::data(data, xj[k], c, v);
#pragma unroll
    for (int d = 0; d < 3; ++d) xc[k][d] = c[d] * s;
  }
  BlockSum<T> Zs[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) Zs[k].zero();

  T rc[2][3], ra[2];
  auto fetch = [&](int t) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t i = ib + static_cast<int64_t>(t) * kTile + u * kWG + tid;
      rc[u][0] = rc[u][1] = rc[u][2] = padT<T>();
      ra[u] = T(0);
      if (i < ie) {
        const double D = saved_den[i];
        if (route[i] == F_FP32) {  // the others are left to the FP64 fix-up
          T c[3] = {T(0), T(0), T(0)};
          Loader<T, DIM, L>::query(query, i, c);
          rc[u][0] = c[0];
          rc[u][1] = c[1];
          rc[u][2] = c[2];
          ra[u] = static_cast<T>(static_cast<double>(grad_out[i]) / (D / unit));
        }
      }
    }
  };
  auto put = [&](int b) {
#pragma unroll
    for (int u = 0; u < 2; ++u) tile[b][u * kWG + tid] = stage<T, DIM>(rc[u], ra[u], s);
  };

  const int ntiles = static_cast<int>((ie - ib + kTile - 1) / kTile);
  const bool excl = (flags & 1u) != 0;
  if constexpr (sizeof(T) == 8 && PM == PM_GEN) pow_table_init(nhp);  // FP64 weight tables (synchronised below)
  fetch(0);
  put(0);
  __syncthreads();
  for (int t = 0; t < ntiles; ++t) {
    if (t + 1 < ntiles) fetch(t + 1);
    const int64_t it = ib + static_cast<int64_t>(t) * kTile;
    const bool diag = excl && it < x0 + kWG * Q && x0 < it + kTile;
    if (diag)
      bwdd_tile<T, DIM, PM, Q, true, 1>(tile[t & 1], it, xc, xj, nhp, Zs);
    else
      bwdd_tile<T, DIM, PM, Q, false, UNR>(tile[t & 1], it, xc, xj, nhp, Zs);
    if (t + 1 < ntiles) put((t + 1) & 1);
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < Q; ++k)
    if (xj[k] < n)
      part[static_cast<int64_t>(blockIdx.y) * n + xj[k]] = Zs[k].value();
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_bwd_zmerge(const double* __restrict__ part, int64_t n,
                                                    int split, T* __restrict__ grad_z) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (j >= n) return;
  double h = 0.0, l = 0.0;
  for (int c = 0; c < split; ++c) two_sum_acc(h, l, part[static_cast<int64_t>(c) * n + j]);
  grad_z[j] = static_cast<T>(h + l);
}

// Coordinate given to queries that a data-direction sweep leaves out (flagged for the FP64
// fix-up, or past the end of the query chunk): far from every scaled data point, with r2
// and every product of the pair terms finite, so that their zero factor a = 0 gives exact
// zeros (an infinite coordinate would turn 0 * (q - x) into NaN).
template <typename T>
__device__ __forceinline__ T farT() {
  return static_cast<T>(0x1p60);
}

// Data sweep with the data-coordinate gradient: lanes own Q data points (scaled coordinates
// and value), query tiles (q_i, a_i) and Z_i are broadcast from LDS.  Accumulates, over
// 64-record blocks as the data sweep,
//   dz_j = sum_i a_i w_ij     and     X_j = sum_i a_i (w_ij / r2_ij)(z_j - Z_i)(q_i - x_j)
// over query chunk c: part_z[c * n + j] and part_x[(c * n + j) * DIM + e] (double).
template <typename T, int DIM, int L, int PM, int Q, int UNR = 2>
__global__ __launch_bounds__(kWG) void k_bwd_datax(DevPts data, int64_t n, DevPts query, int64_t m,
                                                   int64_t chunk, T nhp, unsigned flags,
                                                   const double* __restrict__ hdr,
                                                   const T* __restrict__ grad_out,
                                                   const T* __restrict__ saved_z,
                                                   const double* __restrict__ saved_den,
                                                   double* __restrict__ part_z,
                                                   double* __restrict__ part_x,
                                                   const uint8_t* __restrict__ route) {
  __shared__ P4<T> tile[2][kTile];
  __shared__ T ztl[2][kTile];
  const int tid = threadIdx.x;
  const int64_t x0 = static_cast<int64_t>(blockIdx.x) * (kWG * Q);
  const int64_t ib = static_cast<int64_t>(blockIdx.y) * chunk;
  const int64_t ie = (ib + chunk < m) ? ib + chunk : m;
  const T s = static_cast<T>(hdr[H_SCALE]);
  const double unit = hdr[H_DEN_UNIT];
  const bool excl = (flags & 1u) != 0;

  T xc[Q][3], xv[Q];
  int64_t xj[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    xj[k] = x0 + tid + static_cast<int64_t>(k) * kWG;
    T c[3] = {T(0), T(0), T(0)}, v = T(0);
    if (xj[k] < n) Loader<T, DIM, L>::data(data, xj[k], c, v);
#pragma unroll
    for (int d = 0; d < 3; ++d) xc[k][d] = c[d] * s;
    xv[k] = v;
  }
  BlockSum<T> Zs[Q], Xs[Q][3];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    Zs[k].zero();
#pragma unroll
    for (int d = 0; d < 3; ++d) Xs[k][d].zero();
  }

  T rc[2][3], ra[2], rz[2];
  bool live[2];
  auto fetch = [&](int t) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t i = ib + static_cast<int64_t>(t) * kTile + u * kWG + tid;
      rc[u][0] = rc[u][1] = rc[u][2] = T(0);
      ra[u] = rz[u] = T(0);
      live[u] = false;
      if (i < ie) {
        const double D = saved_den[i];
        if (route[i] == F_FP32) {  // the others are left to the FP64 fix-up
          Loader<T, DIM, L>::query(query, i, rc[u]);
          ra[u] = static_cast<T>(static_cast<double>(grad_out[i]) / (D / unit));
          rz[u] = saved_z[i];
          live[u] = true;
        }
      }
    }
  };
  auto put = [&](int b) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      P4<T> r = stage<T, DIM>(rc[u], ra[u], s);
      if (!live[u]) {
        r.x = r.y = farT<T>();
        if constexpr (DIM == 3) r.z = farT<T>();
      }
      tile[b][u * kWG + tid] = r;
      ztl[b][u * kWG + tid] = rz[u];
    }
  };

  const int ntiles = static_cast<int>((ie - ib + kTile - 1) / kTile);
  if constexpr (sizeof(T) == 8 && PM == PM_GEN) log2_table_init();  // FP64 log2 (synchronised below)
  if constexpr (sizeof(T) == 8 && PM == PM_GEN) exp2_table_init();
  fetch(0);
  put(0);
  __syncthreads();
  for (int t = 0; t < ntiles; ++t) {
    if (t + 1 < ntiles) fetch(t + 1);
    const int64_t it = ib + static_cast<int64_t>(t) * kTile;
    const bool diag = excl && it < x0 + kWG * Q && x0 < it + kTile;
    const P4<T>* tl = tile[t & 1];
    const T* zt = ztl[t & 1];
    // block by block, as the query sweep (the dz + dx sweep: 219 VGPRs against 110 in FP32,
    // 4-5% faster at 1M x 1M in both precisions)
#pragma unroll 1
    for (int c0 = 0; c0 < kTile; c0 += 64) {
      T az[Q], ax[Q][3];
#pragma unroll
      for (int k = 0; k < Q; ++k) az[k] = ax[k][0] = ax[k][1] = ax[k][2] = T(0);
#pragma unroll UNR
      for (int ii = 0; ii < 64; ++ii) {
        const P4<T> d = tl[c0 + ii];
        const T zi = zt[c0 + ii];
        const T a = (DIM == 3) ? d.w : d.z;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          const T e0 = d.x - xc[k][0];  // q - x
          const T e1 = d.y - xc[k][1];
          T e2 = T(0);
          T r2 = e0 * e0;
          r2 = fmaT(e1, e1, r2);
          if constexpr (DIM == 3) {
            e2 = d.z - xc[k][2];
            r2 = fmaT(e2, e2, r2);
          }
          T aa = a;
          if (diag && it + c0 + ii == xj[k]) {  // the leave-one-out self pair
            r2 = T(1);
            aa = T(0);
          }
          T w, f = T(0), lg = T(0);
          wterms<PM, true, false>(r2, nhp, w, f, lg);
          const T aw = aa * w;
          az[k] += aw;
          const T v = wr_times<PM>(aw, aa, f) * (xv[k] - zi);
          ax[k][0] = fmaT(v, e0, ax[k][0]);
          ax[k][1] = fmaT(v, e1, ax[k][1]);
          if constexpr (DIM == 3) ax[k][2] = fmaT(v, e2, ax[k][2]);
        }
      }
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        Zs[k].add(az[k]);
#pragma unroll
        for (int d = 0; d < DIM; ++d) Xs[k][d].add(ax[k][d]);
      }
    }
    if (t + 1 < ntiles) put((t + 1) & 1);
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    if (xj[k] < n) {
      const int64_t r = static_cast<int64_t>(blockIdx.y) * n + xj[k];
      part_z[r] = Zs[k].value();
#pragma unroll
      for (int d = 0; d < DIM; ++d)
        part_x[r * DIM + d] = Xs[k][d].value();
    }
  }
}

// Merges data-coordinate partials in chunk order: dx_j = p s sum_c X_j (s: the sweep's
// coordinate scale, which converts the scaled sums back to caller units).
template <typename T, int DIM>
__global__ __launch_bounds__(kWG) void k_bwd_xmerge(const double* __restrict__ part, int64_t n,
                                                    int split, double p,
                                                    const double* __restrict__ hdr,
                                                    T* __restrict__ grad_x) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (t >= n * DIM) return;
  double h = 0.0, l = 0.0;
  for (int c = 0; c < split; ++c) two_sum_acc(h, l, part[static_cast<int64_t>(c) * n * DIM + t]);
  grad_x[t] = static_cast<T>(p * hdr[H_SCALE] * (h + l));
}

// FP64 fix-up of the adjoint for flagged queries (exact hits and near-coincident points),
// in two passes over the data, each cut into chunks as in k_fwd_fixup:
//   pass 1: D, Z and the hit count of each flagged query;
//   pass 2: P = sum w (1/2) ln(r2) (z - Z) and G = sum (w / r2)(z - Z)(q - x) for the
//           flagged queries without a hit.
// Per slot it leaves the dz coefficient (g / D, or g / h at a hit) and hit count for
// k_bwd_fixz, the dp contribution, and writes dq for its query.
template <typename T>
__device__ __forceinline__ void bwd_fix1_finish(int sl, int64_t i, double num, double den, double h, int dim,
                                                const T* __restrict__ grad_out, T* __restrict__ grad_q,
                                                double* __restrict__ slot_coef, int* __restrict__ slot_hits,
                                                double* __restrict__ slot_dp, double* __restrict__ slot_z,
                                                double* __restrict__ slot_den) {
  const double g = static_cast<double>(grad_out[i]);
  if (h > 0.0) {
    slot_coef[sl] = g / h;
    slot_hits[sl] = static_cast<int>(h);
    slot_dp[sl] = 0.0;
    if (grad_q)
      for (int d = 0; d < dim; ++d) grad_q[i * dim + d] = T(0);
  } else {
    slot_z[sl] = num / den;
    slot_den[sl] = den;
    slot_coef[sl] = g / den;
    slot_hits[sl] = 0;
  }
}

template <typename T, int DIM, int L, int PM>
__global__ __launch_bounds__(kWG) void k_bwd_fix1(DevPts data, int64_t n, DevPts query, double p,
                                                  unsigned flags, const int* __restrict__ list,
                                                  const int* __restrict__ count, int cmax,
                                                  double4* __restrict__ fpart,
                                                  const T* __restrict__ grad_out, T* __restrict__ grad_q,
                                                  double* __restrict__ slot_coef, int* __restrict__ slot_hits,
                                                  double* __restrict__ slot_dp, double* __restrict__ slot_z,
                                                  double* __restrict__ slot_den) {
  __shared__ double red[kWG];
  __shared__ long long redi[kWG];
  const int cnt = *count;
  const int C = fix_chunks(cnt, cmax);
  const int64_t total = static_cast<int64_t>(cnt) * C;
  const int64_t len = C > 0 ? (n + C - 1) / C : 0;
  const bool excl = (flags & 1u) != 0;
  const double nhp = -0.5 * p;
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int sl = static_cast<int>(w / C);
    const int64_t c = w % C;
    const int64_t i = list[sl];
    const int64_t j0 = c * len;
    const int64_t j1 = (j0 + len < n) ? j0 + len : n;
    T qt[3] = {T(0), T(0), T(0)};
    Loader<T, DIM, L>::query(query, i, qt);
    NSum num, den;
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
      } else {
        const double wgt = weight<PM>(r2, nhp);
        num.add(wgt * static_cast<double>(v));
        den.add(wgt);
      }
    }
    const double tn = block_sum(num.value(), red);
    const double td = block_sum(den.value(), red);
    const long long th = block_sum_i64(h, redi);
    if (threadIdx.x == 0) {
      if (C == 1)
        bwd_fix1_finish<T>(sl, i, tn, td, static_cast<double>(th), DIM, grad_out, grad_q, slot_coef,
                           slot_hits, slot_dp, slot_z, slot_den);
      else
        fpart[w] = make_double4(tn, td, 0.0, static_cast<double>(th));
    }
  }
}

template <typename T, int DIM>
__global__ __launch_bounds__(kWG) void k_bwd_fix1_merge(const int* __restrict__ list,
                                                        const int* __restrict__ count, int cmax,
                                                        const double4* __restrict__ fpart,
                                                        const T* __restrict__ grad_out, T* __restrict__ grad_q,
                                                        double* __restrict__ slot_coef,
                                                        int* __restrict__ slot_hits,
                                                        double* __restrict__ slot_dp,
                                                        double* __restrict__ slot_z,
                                                        double* __restrict__ slot_den) {
  const int cnt = *count;
  const int C = fix_chunks(cnt, cmax);
  if (C <= 1) return;
  for (int64_t sl = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x; sl < cnt;
       sl += static_cast<int64_t>(gridDim.x) * kWG) {
    double nh = 0.0, nl = 0.0, dh = 0.0, dl = 0.0, h = 0.0;
    for (int c = 0; c < C; ++c) {
      const double4 v = fpart[static_cast<int64_t>(sl) * C + c];
      two_sum_acc(nh, nl, v.x);
      two_sum_acc(dh, dl, v.y);
      h += v.w;
    }
    bwd_fix1_finish<T>(sl, list[sl], nh + nl, dh + dl, h, DIM, grad_out, grad_q, slot_coef, slot_hits,
                       slot_dp, slot_z, slot_den);
  }
}

template <typename T>
__device__ __forceinline__ void bwd_fix2_finish(int sl, int64_t i, double P, const double (&G)[3], int dim,
                                                double p, const T* __restrict__ grad_out,
                                                T* __restrict__ grad_q, double* __restrict__ slot_dp,
                                                const double* __restrict__ slot_den) {
  const double g = static_cast<double>(grad_out[i]);
  const double D = slot_den[sl];
  slot_dp[sl] = -(g / D) * P;
  if (grad_q)
    for (int d = 0; d < dim; ++d) grad_q[i * dim + d] = static_cast<T>(-(p * g / D) * G[d]);
}

template <typename T, int DIM, int L, int PM>
__global__ __launch_bounds__(kWG) void k_bwd_fix2(DevPts data, int64_t n, DevPts query, double p,
                                                  unsigned flags, const int* __restrict__ list,
                                                  const int* __restrict__ count, int cmax,
                                                  double4* __restrict__ fpart,
                                                  const T* __restrict__ grad_out, T* __restrict__ grad_q,
                                                  const int* __restrict__ slot_hits,
                                                  double* __restrict__ slot_dp,
                                                  const double* __restrict__ slot_z,
                                                  const double* __restrict__ slot_den) {
  __shared__ double red[kWG];
  const int cnt = *count;
  const int C = fix_chunks(cnt, cmax);
  const int64_t total = static_cast<int64_t>(cnt) * C;
  const int64_t len = C > 0 ? (n + C - 1) / C : 0;
  const bool excl = (flags & 1u) != 0;
  const double nhp = -0.5 * p;
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int sl = static_cast<int>(w / C);
    if (slot_hits[sl] > 0) continue;  // uniform over the workgroup
    const int64_t c = w % C;
    const int64_t i = list[sl];
    const int64_t j0 = c * len;
    const int64_t j1 = (j0 + len < n) ? j0 + len : n;
    const double Z = slot_z[sl];
    T qt[3] = {T(0), T(0), T(0)};
    Loader<T, DIM, L>::query(query, i, qt);
    const double q[3] = {static_cast<double>(qt[0]), static_cast<double>(qt[1]), static_cast<double>(qt[2])};
    NSum P, G[3];
    for (int64_t j = j0 + threadIdx.x; j < j1; j += kWG) {
      if (excl && j == i) continue;
      T cc[3] = {T(0), T(0), T(0)}, v;
      Loader<T, DIM, L>::data(data, j, cc, v);
      double e[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        e[d] = q[d] - static_cast<double>(cc[d]);
        r2 += e[d] * e[d];
      }
      const double wgt = weight<PM>(r2, nhp);
      const double cz = static_cast<double>(v) - Z;
      P.add(wgt * 0.5 * log(r2) * cz);
      const double u = (wgt / r2) * cz;
#pragma unroll
      for (int d = 0; d < DIM; ++d) G[d].add(u * e[d]);
    }
    const double tP = block_sum(P.value(), red);
    double tG[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < DIM; ++d) tG[d] = block_sum(G[d].value(), red);
    if (threadIdx.x == 0) {
      if (C == 1)
        bwd_fix2_finish<T>(sl, i, tP, tG, DIM, p, grad_out, grad_q, slot_dp, slot_den);
      else
        fpart[w] = make_double4(tP, tG[0], tG[1], tG[2]);
    }
  }
}

template <typename T, int DIM>
__global__ __launch_bounds__(kWG) void k_bwd_fix2_merge(const int* __restrict__ list,
                                                        const int* __restrict__ count, int cmax,
                                                        const double4* __restrict__ fpart, double p,
                                                        const T* __restrict__ grad_out, T* __restrict__ grad_q,
                                                        const int* __restrict__ slot_hits,
                                                        double* __restrict__ slot_dp,
                                                        const double* __restrict__ slot_den) {
  const int cnt = *count;
  const int C = fix_chunks(cnt, cmax);
  if (C <= 1) return;
  for (int64_t sl = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x; sl < cnt;
       sl += static_cast<int64_t>(gridDim.x) * kWG) {
    if (slot_hits[sl] > 0) continue;
    double P[2] = {0.0, 0.0}, G[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    for (int c = 0; c < C; ++c) {
      const double4 v = fpart[static_cast<int64_t>(sl) * C + c];
      two_sum_acc(P[0], P[1], v.x);
      two_sum_acc(G[0][0], G[0][1], v.y);
      two_sum_acc(G[1][0], G[1][1], v.z);
      two_sum_acc(G[2][0], G[2][1], v.w);
    }
    const double g3[3] = {G[0][0] + G[0][1], G[1][0] + G[1][1], G[2][0] + G[2][1]};
    bwd_fix2_finish<T>(sl, list[sl], P[0] + P[1], g3, DIM, p, grad_out, grad_q, slot_dp, slot_den);
  }
}

// FP64 dz and dx contributions of the flagged queries, added in ascending query order
// (either output may be null).  A query with an exact hit contributes 1/h of its gradient
// to each coincident point's dz and nothing to dx.
template <typename T, int DIM, int L, int PM>
__global__ __launch_bounds__(kWG) void k_bwd_fixz(DevPts data, int64_t n, DevPts query, double p,
                                                  unsigned flags, const int* __restrict__ list,
                                                  const int* __restrict__ count,
                                                  const double* __restrict__ slot_coef,
                                                  const int* __restrict__ slot_hits,
                                                  const double* __restrict__ slot_z,
                                                  T* __restrict__ grad_z, T* __restrict__ grad_x) {
  const int cnt = *count;
  if (cnt == 0) return;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kWG + threadIdx.x;
  if (j >= n) return;
  const bool excl = (flags & 1u) != 0;
  const double nhp = -0.5 * p;
  T c[3] = {T(0), T(0), T(0)}, v;
  Loader<T, DIM, L>::data(data, j, c, v);
  NSum acc, ax[3];
  for (int sl = 0; sl < cnt; ++sl) {
    const int64_t i = list[sl];
    if (excl && i == j) continue;
    T qt[3] = {T(0), T(0), T(0)};
    Loader<T, DIM, L>::query(query, i, qt);
    double e[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      e[d] = static_cast<double>(qt[d]) - static_cast<double>(c[d]);
      r2 += e[d] * e[d];
    }
    if (slot_hits[sl] > 0) {
      if (r2 == 0.0) acc.add(slot_coef[sl]);
    } else {
      const double w = weight<PM>(r2, nhp);
      acc.add(slot_coef[sl] * w);
      if (grad_x) {
        const double u = p * slot_coef[sl] * (w / r2) * (static_cast<double>(v) - slot_z[sl]);
#pragma unroll
        for (int d = 0; d < DIM; ++d) ax[d].add(u * e[d]);
      }
    }
  }
  if (grad_z) grad_z[j] = static_cast<T>(static_cast<double>(grad_z[j]) + acc.value());
  if (grad_x) {
#pragma unroll
    for (int d = 0; d < DIM; ++d)
      grad_x[j * DIM + d] = static_cast<T>(static_cast<double>(grad_x[j * DIM + d]) + ax[d].value());
  }
}

// ---------------------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------------------
template <typename T, int DIM, int L, int PM>
hipError_t launch_bwd_query_t(const BwdArgs& a, int split, int64_t chunk, double4* part,
                              hipStream_t st) {
  const bool ndp = (a.flags & 0x4u) != 0, ndq = (a.flags & 0x8u) != 0;
  const int Q = a.q_per_lane;
  const int64_t qpb = static_cast<int64_t>(kWG) * Q;
  dim3 grid(static_cast<unsigned>((a.m + qpb - 1) / qpb), static_cast<unsigned>(split));
  const T nhp = static_cast<T>(-0.5 * a.p);
  const T* sz = static_cast<const T*>(a.saved_z);
#define IDW_BQ(QQ, DP, DQ)                                                                  \
  hipLaunchKernelGGL((k_bwd_query<T, DIM, L, PM, QQ, DP, DQ>), grid, dim3(kWG), 0, st,      \
                     a.data, a.n, a.query, a.m, chunk, nhp, a.flags, a.hdr, sz, part)
#define IDW_BQ_Q(QQ)                  \
  case QQ:                            \
    if (ndp && ndq)                   \
      IDW_BQ(QQ, true, true);         \
    else if (ndp)                     \
      IDW_BQ(QQ, true, false);        \
    else                              \
      IDW_BQ(QQ, false, true);        \
    break;
  if constexpr (sizeof(T) == 4) {
    switch (Q) {
      IDW_BQ_Q(2)
      IDW_BQ_Q(4)
      default:
        return hipErrorInvalidValue;
    }
  } else {
    switch (Q) {
      IDW_BQ_Q(2)
      default:
        return hipErrorInvalidValue;
    }
  }
#undef IDW_BQ_Q
#undef IDW_BQ
  return hipGetLastError();
}

template <typename T, int DIM, int L, int PM>
hipError_t launch_bwd_data_t(const BwdArgs& a, int split, int64_t chunk, double* part,
                             hipStream_t st) {
  const int Q = a.q_per_lane;
  const int64_t xpb = static_cast<int64_t>(kWG) * Q;
  dim3 grid(static_cast<unsigned>((a.n + xpb - 1) / xpb), static_cast<unsigned>(split));
  const T nhp = static_cast<T>(-0.5 * a.p);
  const T* go = static_cast<const T*>(a.grad_out);
#define IDW_BD_Q(QQ)                                                                        \
  case QQ:                                                                                  \
    hipLaunchKernelGGL((k_bwd_data<T, DIM, L, PM, QQ>), grid, dim3(kWG), 0, st, a.data,     \
                       a.n, a.query, a.m, chunk, nhp, a.flags, a.hdr, go, a.saved_den, part, a.route); \
    break;
  if constexpr (sizeof(T) == 4) {
    switch (Q) {
      IDW_BD_Q(4)
      IDW_BD_Q(8)
      default:
        return hipErrorInvalidValue;
    }
  } else {
    switch (Q) {
      IDW_BD_Q(2)
      default:
        return hipErrorInvalidValue;
    }
  }
#undef IDW_BD_Q
  return hipGetLastError();
}

template <typename T, int DIM, int L, int PM>
hipError_t launch_bwd_fix_t(const BwdArgs& a, hipStream_t st) {
  const T* go = static_cast<const T*>(a.grad_out);
  T* gq = static_cast<T*>(a.grad_q);
  hipLaunchKernelGGL((k_bwd_fix1<T, DIM, L, PM>), dim3(kFixGrid), dim3(kWG), 0, st, a.data, a.n, a.query,
                     a.p, a.flags, a.list, a.count, a.fix_cmax, a.fpart, go, gq, a.slot_coef, a.slot_hits,
                     a.slot_dp, a.slot_z, a.slot_den);
  hipLaunchKernelGGL((k_bwd_fix1_merge<T, DIM>), dim3(4), dim3(kWG), 0, st, a.list, a.count, a.fix_cmax,
                     a.fpart, go, gq, a.slot_coef, a.slot_hits, a.slot_dp, a.slot_z, a.slot_den);
  if (a.flags & 0xcu) {  // dp or dq requested
    hipLaunchKernelGGL((k_bwd_fix2<T, DIM, L, PM>), dim3(kFixGrid), dim3(kWG), 0, st, a.data, a.n, a.query,
                       a.p, a.flags, a.list, a.count, a.fix_cmax, a.fpart, go, gq, a.slot_hits, a.slot_dp,
                       a.slot_z, a.slot_den);
    hipLaunchKernelGGL((k_bwd_fix2_merge<T, DIM>), dim3(4), dim3(kWG), 0, st, a.list, a.count, a.fix_cmax,
                       a.fpart, a.p, go, gq, a.slot_hits, a.slot_dp, a.slot_den);
  }
  if (a.grad_z || a.grad_x)
    hipLaunchKernelGGL((k_bwd_fixz<T, DIM, L, PM>),
                       dim3(static_cast<unsigned>((a.n + kWG - 1) / kWG)), dim3(kWG), 0, st,
                       a.data, a.n, a.query, a.p, a.flags, a.list, a.count, a.slot_coef,
                       a.slot_hits, a.slot_z, static_cast<T*>(a.grad_z), static_cast<T*>(a.grad_x));
  return hipGetLastError();
}

template <typename T, int DIM, int L, int PM>
hipError_t launch_bwd_datax_t(const BwdArgs& a, int split, int64_t chunk, hipStream_t st) {
  constexpr int Q = sizeof(T) == 4 ? 4 : 2;
  const int64_t xpb = static_cast<int64_t>(kWG) * Q;
  dim3 grid(static_cast<unsigned>((a.n + xpb - 1) / xpb), static_cast<unsigned>(split));
  hipLaunchKernelGGL((k_bwd_datax<T, DIM, L, PM, Q>), grid, dim3(kWG), 0, st, a.data, a.n, a.query, a.m,
                     chunk, static_cast<T>(-0.5 * a.p), a.flags, a.hdr, static_cast<const T*>(a.grad_out),
                     static_cast<const T*>(a.saved_z), a.saved_den, a.part_z, a.part_x, a.route);
  return hipGetLastError();
}

// Dispatch helpers over (precision, dim, weight class).
// Backward weight classes: p = 2.5 runs on the general exp2/log2 form, which costs the
// same two transcendentals once log2(r2) is needed for dp.
#define IDW_DISPATCH_PM(FN, T, DIM, L, ...)                              \
  switch (a.pmode) {                                                     \
    case PM_1: return FN<T, DIM, L, PM_1>(__VA_ARGS__);                  \
    case PM_2: return FN<T, DIM, L, PM_2>(__VA_ARGS__);                  \
    case PM_3: return FN<T, DIM, L, PM_3>(__VA_ARGS__);                  \
    case PM_4: return FN<T, DIM, L, PM_4>(__VA_ARGS__);                  \
    default: return FN<T, DIM, L, PM_GEN>(__VA_ARGS__);                  \
  }

template <typename T, int DIM, int L>
hipError_t bwd_query_pm(const BwdArgs& a, int split, int64_t chunk, double4* part, hipStream_t st) {
  IDW_DISPATCH_PM(launch_bwd_query_t, T, DIM, L, a, split, chunk, part, st)
}
template <typename T, int DIM, int L>
hipError_t bwd_data_pm(const BwdArgs& a, int split, int64_t chunk, double* part, hipStream_t st) {
  IDW_DISPATCH_PM(launch_bwd_data_t, T, DIM, L, a, split, chunk, part, st)
}
template <typename T, int DIM, int L>
hipError_t bwd_datax_pm(const BwdArgs& a, int split, int64_t chunk, hipStream_t st) {
  IDW_DISPATCH_PM(launch_bwd_datax_t, T, DIM, L, a, split, chunk, st)
}
template <typename T, int DIM, int L>
hipError_t bwd_fix_pm(const BwdArgs& a, hipStream_t st) {
  IDW_DISPATCH_PM(launch_bwd_fix_t, T, DIM, L, a, st)
}

template <typename T, int DIM>
hipError_t launch_bwd_qmerge(const BwdArgs& a, int split, const double4* part, hipStream_t st) {
  dim3 grid(static_cast<unsigned>((a.m + kWG - 1) / kWG));
  hipLaunchKernelGGL((k_bwd_qmerge<T, DIM>), grid, dim3(kWG), 0, st, part, a.m, split, a.p, a.hdr,
                     static_cast<const T*>(a.grad_out), a.saved_den, static_cast<T*>(a.grad_q),
                     a.wg_dp, a.route);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bwd_zmerge(const BwdArgs& a, int split, const double* part, hipStream_t st) {
  dim3 grid(static_cast<unsigned>((a.n + kWG - 1) / kWG));
  hipLaunchKernelGGL((k_bwd_zmerge<T>), grid, dim3(kWG), 0, st, part, a.n, split,
                     static_cast<T*>(a.grad_z));
  return hipGetLastError();
}

template <typename T, int DIM>
hipError_t launch_bwd_xmerge(const BwdArgs& a, int split, hipStream_t st) {
  dim3 grid(static_cast<unsigned>((a.n * DIM + kWG - 1) / kWG));
  hipLaunchKernelGGL((k_bwd_xmerge<T, DIM>), grid, dim3(kWG), 0, st, a.part_x, a.n, split, a.p, a.hdr,
                     static_cast<T*>(a.grad_x));
  return hipGetLastError();
}

}  // namespace idw
