// Fused FP32 adjoint sweep: the query-direction sums (P_i, G_i, for dp and dq) and the
// data-direction sums (dz_j = sum_i a_i w_ij, a_i = g_i / D_i, and, for the gradient with
// respect to the data coordinates, X_j = sum_i a_i (w_ij / r2_ij)(z_j - Z_i)(q_i - x_j))
// from ONE evaluation of each pair's weight.
//
// Lanes own Q queries each (registers).  Data points are staged in LDS in batches of 64,
// each batch stored twice in a row, so that at step s lane L reads record (L + s) of the
// doubled batch -- data point (L + s) mod 64 -- with a compile-time offset and no bank
// conflicts.  Query-direction sums accumulate per lane as in the query sweep.  For the
// data direction every lane forms s_L = sum_k a_k w_k for its point of the step, and a
// running sum travels one lane per step (v_add_f32 with a wave_rol:1 DPP operand:
// lane L receives the sum held by lane L+1), picking up the contribution of each lane for
// the same data point.  After 64 steps lane L holds the sum over the wave's 64 x Q
// queries for batch point (L - 1) mod 64.  That costs one DPP add per lane per step,
// against a separate data sweep that recomputes every weight.  X_j rides the same rotation
// with one running sum per coordinate.
//
// Work decomposition: workgroup (qg, dr) sweeps data range dr for the query blocks
// qg, qg + G, qg + 2G, ...; it writes the query partials of range dr (as the query sweep
// with a data split) and accumulates its dz partial row qg across its query blocks (the
// data sweep's split-over-queries format), so the existing fixed-order merges apply.
#pragma once

#include "idw_bwd.hpp"
#include "idw_device.hpp"
#include "idw_fwd.hpp"

namespace idw {

constexpr int kBatch = 64;  // data points per rotation batch (one wave)

// Data points per LDS tile: 512 in FP32 (8 batches), 256 in FP64 (the records are twice as
// wide; with 256-thread workgroups the tiles, batches doubled, and the per-wave sums take
// 40 KB of LDS).
template <typename T>
struct FusedShape {
  static constexpr int TILE = sizeof(T) == 8 ? 256 : 512;
  static constexpr int NT = sizeof(T) == 8 ? 256 : 512;  // threads per workgroup
};
constexpr int kFTile = FusedShape<float>::TILE;

// Lane L takes the running sum of lane L+1 (wave rotate left by one); an FP64 value moves
// as its two 32-bit halves.
__device__ __forceinline__ float rotate_in(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x134, 0xF, 0xF, false));
}
__device__ __forceinline__ double rotate_in(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<unsigned int>(b)), 0x134, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<unsigned int>(b >> 32)), 0x134, 0xF, 0xF,
                                             false);
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(static_cast<unsigned int>(hi)) << 32) |
                                        static_cast<unsigned int>(lo));
}

// One 64-point batch.  MASK: some pairs must be skipped (padding records beyond the data
// range, or the leave-one-out self pair); those get r2 = 1 and zero value factors.
// Returns the dz running sum; with NDX, ax holds the X running sums.
// REL: relative weights; the squared distance is multiplied by the query's sigma (sg)
// before the weight terms, log2 r2 = log2(r2 sigma) - k (kq), and the X sums take the
// coefficient a sigma (axq) so that they stay those of the direct form.
template <typename T, int DIM, int PM, int Q, bool NDP, bool NDQ, bool NDX, bool MASK, int UNR, bool REL = false>
__device__ __forceinline__ T bwdf_batch(const P4<T>* __restrict__ rec, int lane, int64_t jb, int64_t je,
                                        bool excl, const T (&qc)[Q][3], const T (&zq)[Q], const T (&aq)[Q],
                                        const T (&sg)[Q], const T (&kq)[Q], const T (&axq)[Q],
                                        const int64_t (&qi)[Q], T nhp, T (&ap)[Q], T (&ag)[Q][3], T (&ax)[3]) {
  T acc = T(0);
  ax[0] = ax[1] = ax[2] = T(0);
  const P4<T>* r0 = rec + lane;
#pragma unroll UNR
  for (int s = 0; s < kBatch; ++s) {
    const P4<T> d = r0[s];
    const T dv = (DIM == 3) ? d.w : d.z;
    T sz = T(0);
    T sx[3] = {T(0), T(0), T(0)};
    int64_t j = 0;
    bool valid = true;
    if constexpr (MASK) {
      j = jb + ((lane + s) & (kBatch - 1));
      valid = j < je;
    }
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
      T a = aq[k];
      T av = REL ? axq[k] : a;
      if constexpr (REL) r2 *= sg[k];
      if constexpr (MASK) {
        if (!valid || (excl && j == qi[k])) {
          r2 = T(1);
          c = T(0);
          a = T(0);
          av = T(0);
        }
      }
      T w, f = T(0), lg = T(0);
      wterms<PM, NDQ || NDX, NDP, PowTab<T, PM, NDP || NDX>::on>(r2, nhp, w, f, lg);
      if constexpr (REL && NDP) lg -= kq[k];
      const T t = w * c;
      if constexpr (NDP) ap[k] = fmaT(t, lg, ap[k]);
      if constexpr (NDQ || NDX) {
        const T u = wr_times<PM>(t, c, f);  // (w / r2)(z - Z)
        if constexpr (NDQ) {
          ag[k][0] = fmaT(u, dx, ag[k][0]);
          ag[k][1] = fmaT(u, dy, ag[k][1]);
          if constexpr (DIM == 3) ag[k][2] = fmaT(u, dz, ag[k][2]);
        }
        if constexpr (NDX) {
          const T v = av * u;
          sx[0] = (k == 0) ? v * dx : fmaT(v, dx, sx[0]);
          sx[1] = (k == 0) ? v * dy : fmaT(v, dy, sx[1]);
          if constexpr (DIM == 3) sx[2] = (k == 0) ? v * dz : fmaT(v, dz, sx[2]);
        }
      }
      sz = (k == 0) ? a * w : fmaT(a, w, sz);
    }
    acc = rotate_in(acc) + sz;
    if constexpr (NDX) {
#pragma unroll
      for (int e = 0; e < DIM; ++e) ax[e] = rotate_in(ax[e]) + sx[e];
    }
  }
  return acc;
}

// Defaults measured on MI355X (1M queries x 256K data, 2-D, p = 2): 512-thread workgroups,
// Q = 2, unroll 2, about 1024 workgroups in the grid: 13.6 VALU lane-slots per pair, against
// 17.3 with 256-thread workgroups and 512 in the grid.
constexpr int kFNT = FusedShape<float>::NT;

// Coordinate given to queries that are left out of a sweep (flagged for the FP64 fix-up):
// far from every scaled data point, yet with r2 (< 3 * 2^120) and every product of the
// pair terms finite, so that their zero factors a = 0 give exact zeros.
constexpr float kFarF = 0x1p60f;

// T = float: the FP32 adjoint (with relative weights for large p); T = double: the FP64
// adjoint (the FP64 one-step and table forms of the weights, no relative weights).
template <typename T, int DIM, int L, int PM, int Q, bool NDP, bool NDQ, bool NDX, bool REL = false, int UNR = 2,
          int WPE = 2, int NT = FusedShape<T>::NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_bwd_fused(
    DevPts data, int64_t n, DevPts query, int64_t m, int64_t chunk, int groups, T nhp, unsigned flags,
    const double* __restrict__ hdr, const T* __restrict__ saved_z, const T* __restrict__ grad_out,
    const double* __restrict__ saved_den, double4* __restrict__ part_q, double* __restrict__ part_z,
    double* __restrict__ part_x, const uint8_t* __restrict__ route, double pd) {
  static_assert(sizeof(T) == 4 || !REL, "FP64: no relative weights");
  constexpr int kFTile = FusedShape<T>::TILE;
  constexpr int kFBatches = kFTile / kBatch;
  __shared__ P4<T> tile[2][2 * kFTile];   // batches stored twice in a row
  constexpr int PPT = kFTile / NT;        // tile points staged per thread
  static_assert(PPT >= 1, "a tile holds at least one point per thread");
  __shared__ T zred[NT / 64][kFTile];     // per-wave dz sums of the current tile
  __shared__ T xred[NDX ? NT / 64 : 1][NDX ? DIM * kFTile : 1];  // per-wave X sums
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int qg = blockIdx.x;
  const int64_t jb = static_cast<int64_t>(blockIdx.y) * chunk;
  const int64_t je = (jb + chunk < n) ? jb + chunk : n;
  const T s = static_cast<T>(hdr[H_SCALE]);
  const double unit = hdr[H_DEN_UNIT];
  const bool excl = (flags & 1u) != 0;
  // FP64 tables (synchronised below); with dx the pow tables cost too much occupancy.
  constexpr bool kPow = PowTab<T, PM, NDP || NDX>::on;
  if constexpr (kPow) pow_table_init(NDQ ? nhp - 1.0 : nhp);
  if constexpr (sizeof(T) == 8 && !kPow && (NDP || PM == PM_GEN)) log2_table_init();
  if constexpr (sizeof(T) == 8 && !kPow && PM == PM_GEN) exp2_table_init();
  const int64_t qpb = static_cast<int64_t>(NT) * Q;
  const int64_t nqb = (m + qpb - 1) / qpb;
  const int ntiles = static_cast<int>((je - jb + kFTile - 1) / kFTile);
  double* zrow = part_z + static_cast<int64_t>(qg) * n;
  double* xrow = NDX ? part_x + static_cast<int64_t>(qg) * n * DIM : nullptr;

  T rc[PPT][3], rv[PPT];
  auto fetch = [&](int t) {
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      const int64_t j = jb + static_cast<int64_t>(t) * kFTile + u * NT + tid;
      rc[u][0] = rc[u][1] = rc[u][2] = T(0);
      rv[u] = T(0);
      if (j < je) Loader<T, DIM, L>::data(data, j, rc[u], rv[u]);
    }
  };
  auto put = [&](int b) {
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      const int p = u * NT + tid;                        // point within the tile
      const int at = (p / kBatch) * (2 * kBatch) + (p % kBatch);
      const P4<T> r = stage<T, DIM>(rc[u], rv[u], s);
      tile[b][at] = r;
      tile[b][at + kBatch] = r;
    }
  };

  int first = 1;
  for (int64_t qb = qg; qb < nqb; qb += groups, first = 0) {
    const int64_t q0 = qb * qpb;
    T qc[Q][3], zq[Q], aq[Q], sg[Q], kq[Q], axq[Q];
    int64_t qi[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      qi[k] = q0 + tid + static_cast<int64_t>(k) * NT;
      T c[3] = {T(0), T(0), T(0)};
      bool ok = false;
      zq[k] = T(0);
      aq[k] = T(0);
      sg[k] = T(1);
      kq[k] = T(0);
      axq[k] = T(0);
      if (qi[k] < m) {
        ok = route[qi[k]] == F_FP32;  // the others are left to the FP64 fix-up
        if (ok) {
          const double D = saved_den[qi[k]];
          Loader<T, DIM, L>::query(query, qi[k], c);
          zq[k] = saved_z[qi[k]];
          const double g = static_cast<double>(grad_out[qi[k]]);
          if constexpr (REL) {
            double E = 1.0;
            float sgf = 1.f, kqf = 0.f;
            rel_from_den(D / unit, pd, sgf, kqf, E);
            sg[k] = sgf;
            kq[k] = kqf;
            aq[k] = static_cast<T>(g / E);
            axq[k] = static_cast<T>(g / E * static_cast<double>(sgf));
          } else {
            aq[k] = static_cast<T>(g / (D / unit));
          }
        }
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) qc[k][d] = ok ? c[d] * s : static_cast<T>(kFarF);
    }
    BlockSum<T> P[Q], G[Q][3];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      P[k].zero();
#pragma unroll
      for (int d = 0; d < 3; ++d) G[k][d].zero();
    }

    fetch(0);
    put(0);
    __syncthreads();
    for (int t = 0; t < ntiles; ++t) {
      if (t + 1 < ntiles) fetch(t + 1);
      const int64_t jt = jb + static_cast<int64_t>(t) * kFTile;
      const bool diag = excl && jt < q0 + qpb && q0 < jt + kFTile;
      const bool tail = jt + kFTile > je;
#pragma unroll 1
      for (int b = 0; b < kFBatches; ++b) {
        T ap[Q], ag[Q][3];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          ap[k] = T(0);
          ag[k][0] = ag[k][1] = ag[k][2] = T(0);
        }
        const P4<T>* rec = tile[t & 1] + b * (2 * kBatch);
        const int64_t jbat = jt + b * kBatch;
        T zs, ax[3];
        if (diag || tail)
          zs = bwdf_batch<T, DIM, PM, Q, NDP, NDQ, NDX, true, 1, REL>(rec, lane, jbat, je, excl, qc, zq, aq, sg, kq,
                                                                     axq, qi, nhp, ap, ag, ax);
        else
          zs = bwdf_batch<T, DIM, PM, Q, NDP, NDQ, NDX, false, UNR, REL>(rec, lane, jbat, je, excl, qc, zq, aq, sg,
                                                                        kq, axq, qi, nhp, ap, ag, ax);
        const int at = b * kBatch + ((lane + kBatch - 1) & (kBatch - 1));
        zred[wave][at] = zs;
        if constexpr (NDX) {
#pragma unroll
          for (int e = 0; e < DIM; ++e) xred[wave][e * kFTile + at] = ax[e];
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
      __syncthreads();  // zred complete; tile t fully consumed
      // dz: sum the waves' partials in wave order and fold into this group's row
#pragma unroll
      for (int u = 0; u < PPT; ++u) {
        const int p = u * NT + tid;
        const int64_t j = jt + p;
        if (j < je) {
          double v = static_cast<double>(zred[0][p]);
#pragma unroll
          for (int w = 1; w < NT / 64; ++w) v += static_cast<double>(zred[w][p]);
          zrow[j] = first ? v : zrow[j] + v;
          if constexpr (NDX) {
#pragma unroll
            for (int e = 0; e < DIM; ++e) {
              double x = static_cast<double>(xred[0][e * kFTile + p]);
#pragma unroll
              for (int w = 1; w < NT / 64; ++w) x += static_cast<double>(xred[w][e * kFTile + p]);
              xrow[j * DIM + e] = first ? x : xrow[j * DIM + e] + x;
            }
          }
        }
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
        part_q[static_cast<int64_t>(blockIdx.y) * m + qi[k]] = r;
      }
    }
  }
  // A group without any query block still owns a partial row: make it zero.
  if (first) {
    for (int64_t j = jb + tid; j < je; j += NT) {
      zrow[j] = 0.0;
      if constexpr (NDX) {
#pragma unroll
        for (int e = 0; e < DIM; ++e) xrow[j * DIM + e] = 0.0;
      }
    }
  }
}

template <typename T, int DIM, int L, int PM, bool REL = false>
hipError_t launch_bwd_fused_t(const BwdArgs& a, int groups, int ranges, int64_t chunk, hipStream_t st) {
  const bool ndp = (a.flags & 0x4u) != 0, ndq = (a.flags & 0x8u) != 0, ndx = a.part_x != nullptr;
  dim3 grid(static_cast<unsigned>(groups), static_cast<unsigned>(ranges));
  const T nhp = static_cast<T>(-0.5 * a.p);
  const T* sz = static_cast<const T*>(a.saved_z);
  const T* go = static_cast<const T*>(a.grad_out);
  constexpr int NT = FusedShape<T>::NT;
#define IDW_BF(DP, DQ, DX)                                                                                  \
  hipLaunchKernelGGL((k_bwd_fused<T, DIM, L, PM, 2, DP, DQ, DX, REL>), grid, dim3(NT), 0, st, a.data, a.n,    \
                     a.query, a.m, chunk, groups, nhp, a.flags, a.hdr, sz, go, a.saved_den, a.part_q, a.part_z, \
                     a.part_x, a.route, a.p)
  // The data-coordinate gradient is instantiated with both query-direction sums (they share
  // its per-pair factors); merges write only what was requested.  With relative weights
  // every request runs here, dz alone included.
  if (ndx)
    IDW_BF(true, true, true);
  else if (ndp && ndq)
    IDW_BF(true, true, false);
  else if (ndp)
    IDW_BF(true, false, false);
  else if (ndq)
    IDW_BF(false, true, false);
  else if constexpr (REL)
    IDW_BF(false, false, false);
  else
    return hipErrorInvalidValue;
#undef IDW_BF
  return hipGetLastError();
}

template <typename T, int DIM, int L>
hipError_t bwd_fused_pm(const BwdArgs& a, int groups, int ranges, int64_t chunk, hipStream_t st) {
  if constexpr (sizeof(T) == 4) {
    if (a.rel)
      return a.pmode == PM_GEN ? launch_bwd_fused_t<T, DIM, L, PM_GEN, true>(a, groups, ranges, chunk, st)
                               : hipErrorInvalidValue;
  } else {
    if (a.rel) return hipErrorInvalidValue;
  }
  switch (a.pmode) {
    case PM_1: return launch_bwd_fused_t<T, DIM, L, PM_1>(a, groups, ranges, chunk, st);
    case PM_2: return launch_bwd_fused_t<T, DIM, L, PM_2>(a, groups, ranges, chunk, st);
    case PM_3: return launch_bwd_fused_t<T, DIM, L, PM_3>(a, groups, ranges, chunk, st);
    case PM_4: return launch_bwd_fused_t<T, DIM, L, PM_4>(a, groups, ranges, chunk, st);
    default: return launch_bwd_fused_t<T, DIM, L, PM_GEN>(a, groups, ranges, chunk, st);
  }
}

}  // namespace idw
