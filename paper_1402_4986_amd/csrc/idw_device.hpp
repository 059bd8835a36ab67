// Device-side building blocks shared by the IDW kernels (gfx950, wave64).
//
//  - record loaders for the five layouts of Sections 3.1-3.5 (SoA, AoS, aligned AoS,
//    SoAoS, hybrid AoS + array of values), templated on element type and dimension;
//  - the weight w = d^-p of Eq. 1 written through r^2 = d^2, with fast forms for
//    p in {1, 2, 3, 4, 2.5} and the exp2/log2 form for any other p;
//  - TwoSum accumulation into (hi, lo) pairs and fixed-order workgroup reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace idw {

enum Layout { L_SOA = 0, L_AOS = 1, L_AOAS = 2, L_HYBRID = 3, L_SOAOS = 4 };

// Weight forms, selected on the host from p.
enum PMode { PM_GEN = 0, PM_1 = 1, PM_2 = 2, PM_3 = 3, PM_4 = 4, PM_25 = 5 };

constexpr int kWG = 256;  // threads per workgroup of every sweep kernel (4 wave64)

// Device-side view of a point set: the raw pointer slots of idw_points.
struct DevPts {
  const void* p[4];
};

// Four-wide record as staged in LDS: {x, y, z-or-value, value-or-pad}.
template <typename T>
struct alignas(4 * sizeof(T)) P4 {
  T x, y, z, w;
};
template <typename T>
struct alignas(2 * sizeof(T)) P2 {
  T x, y;
};

// ---------------------------------------------------------------------------------------
// Record loaders.  c[0..DIM-1] receive coordinates, v the value (data points only).
// ---------------------------------------------------------------------------------------
template <typename T, int DIM, int L>
struct Loader {
  static __device__ __forceinline__ void data(const DevPts& P, int64_t j, T (&c)[3], T& v) {
    if constexpr (L == L_SOA) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) c[k] = static_cast<const T*>(P.p[k])[j];
      v = static_cast<const T*>(P.p[DIM])[j];
    } else if constexpr (L == L_AOS) {
      const T* r = static_cast<const T*>(P.p[0]) + j * (DIM + 1);
#pragma unroll
      for (int k = 0; k < DIM; ++k) c[k] = r[k];
      v = r[DIM];
    } else if constexpr (L == L_AOAS) {
      const P4<T> r = static_cast<const P4<T>*>(P.p[0])[j];
      c[0] = r.x;
      c[1] = r.y;
      if constexpr (DIM == 3) {
        c[2] = r.z;
        v = r.w;
      } else {
        v = r.z;
      }
    } else if constexpr (L == L_HYBRID) {
      const T* r = static_cast<const T*>(P.p[0]) + j * DIM;
#pragma unroll
      for (int k = 0; k < DIM; ++k) c[k] = r[k];
      v = static_cast<const T*>(P.p[1])[j];
    } else {  // L_SOAOS
      if constexpr (DIM == 2) {
        const P2<T> r = static_cast<const P2<T>*>(P.p[0])[j];
        c[0] = r.x;
        c[1] = r.y;
      } else {
        const P4<T> r = static_cast<const P4<T>*>(P.p[0])[j];
        c[0] = r.x;
        c[1] = r.y;
        c[2] = r.z;
      }
      v = static_cast<const P2<T>*>(P.p[1])[j].x;
    }
  }

  static __device__ __forceinline__ void query(const DevPts& P, int64_t i, T (&c)[3]) {
    if constexpr (L == L_SOA) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) c[k] = static_cast<const T*>(P.p[k])[i];
    } else if constexpr (L == L_AOS || L == L_HYBRID) {
      const T* r = static_cast<const T*>(P.p[0]) + i * DIM;
#pragma unroll
      for (int k = 0; k < DIM; ++k) c[k] = r[k];
    } else if constexpr (L == L_AOAS || (L == L_SOAOS && DIM == 3)) {
      const P4<T> r = static_cast<const P4<T>*>(P.p[0])[i];
      c[0] = r.x;
      c[1] = r.y;
      if constexpr (DIM == 3) c[2] = r.z;
    } else {  // L_SOAOS, DIM == 2
      const P2<T> r = static_cast<const P2<T>*>(P.p[0])[i];
      c[0] = r.x;
      c[1] = r.y;
    }
  }
};

// ---------------------------------------------------------------------------------------
// Weight w = d^-p = (r2)^(-p/2) (Eq. 1).  nhp = -p/2 (used by the general form only).
// FP32 uses the hardware transcendentals (about 1 ulp); FP64 uses correctly rounded
// division and square root, and the double exp2/log2 for general p.
// r2 == 0 gives +inf (flagged and recomputed); r2 == +inf (padding) gives 0.
// ---------------------------------------------------------------------------------------
template <int PM>
__device__ __forceinline__ float weight(float r2, float nhp) {
  if constexpr (PM == PM_2) {
    return __builtin_amdgcn_rcpf(r2);
  } else if constexpr (PM == PM_1) {
    return __builtin_amdgcn_rsqf(r2);
  } else if constexpr (PM == PM_3) {
    const float s = __builtin_amdgcn_rsqf(r2);
    return s * s * s;
  } else if constexpr (PM == PM_4) {
    const float t = __builtin_amdgcn_rcpf(r2);
    return t * t;
  } else if constexpr (PM == PM_25) {
    const float s = __builtin_amdgcn_rsqf(r2);
    return s * s * __builtin_amdgcn_sqrtf(s);
  } else {
    return __builtin_amdgcn_exp2f(nhp * __builtin_amdgcn_logf(r2));
  }
}

// 1/a in FP64: the hardware reciprocal estimate refined by two Newton steps (each about
// squares the relative error), then the division fix-up instruction, which returns the
// IEEE result for a = 0, +-inf and NaN (where the Newton steps would give NaN).  Measured
// on MI355X over 2^20 log-uniform a in [2^-40, 2^3]: the estimate is off by up to 2.5e8
// ulp, one step leaves 11 ulp, two steps gave the correctly rounded quotient every time.
// 6 instructions against about 10 for the IEEE division sequence.
__device__ __forceinline__ double rcp64(double a) {
  double y = __builtin_amdgcn_rcp(a);
  double e = fma(-a, y, 1.0);
  y = fma(y, e, y);
  e = fma(-a, y, 1.0);
  y = fma(y, e, y);
  return __builtin_amdgcn_div_fixup(y, a, 1.0);
}

// 1/sqrt(a) in FP64: the hardware estimate refined by two Newton steps; for a = 0, inf and
// NaN the estimate itself (inf, 0, NaN) is returned.  Within 1.0 ulp on MI355X over 2^21
// log-uniform a in [2^-60, 2^60] (about 8 instructions against about 20 for a correctly
// rounded square root and division).
__device__ __forceinline__ double rsq64(double a) {
  const double y0 = __builtin_amdgcn_rsq(a);
  double y = y0;
  double t = a * y;
  double e = fma(-t, y, 1.0);
  y = fma(0.5 * y, e, y);
  t = a * y;
  e = fma(-t, y, 1.0);
  y = fma(0.5 * y, e, y);
  return (a > 0.0 && a < __builtin_huge_val()) ? y : y0;
}

// log2(a) in FP64 for the weights and the power gradient: a = m 2^e with m in
// [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s) with s = (m - 1)/(m + 1), |s| <= 0.172, summed
// as 2 s (1 + s^2/3 + ... + s^20/21) (truncation below 2^-60); log2 a = e + ln m / ln 2.
// log2(0) = -inf, log2(inf) = inf, NaN passes through.  Within 4.1 ulp on MI355X over 2^21
// inputs (log-uniform in [2^-60, 2^60], a quarter within 1e-3 of 1), in about 33
// instructions against about 70 for the library's correctly rounded form.
__device__ __forceinline__ double log2_64(double a) {
  double m = __builtin_amdgcn_frexp_mant(a);
  int e = __builtin_amdgcn_frexp_exp(a);
  const bool low = m < 0.70710678118654752440;
  m = low ? m + m : m;
  e = low ? e - 1 : e;
  const double s = (m - 1.0) * rcp64(m + 1.0);
  const double z = s * s;
  double p = 1.0 / 21.0;
  p = fma(p, z, 1.0 / 19.0);
  p = fma(p, z, 1.0 / 17.0);
  p = fma(p, z, 1.0 / 15.0);
  p = fma(p, z, 1.0 / 13.0);
  p = fma(p, z, 1.0 / 11.0);
  p = fma(p, z, 1.0 / 9.0);
  p = fma(p, z, 1.0 / 7.0);
  p = fma(p, z, 1.0 / 5.0);
  p = fma(p, z, 1.0 / 3.0);
  p = fma(p, z, 1.0);
  const double r = fma((s + s) * p, 1.44269504088896340736, static_cast<double>(e));
  if (a > 0.0 && a < __builtin_huge_val()) return r;
  return a == 0.0 ? -__builtin_huge_val() : a;
}

// The FP64 sweeps' weights need about 1e-14, not correct rounding (the FP64 tolerance is
// 1e-12 of the condition scale): the hardware estimates (relative error below 6e-8 on
// MI355X) refined by ONE Newton step, about 1e-14 relative (11 ulp measured for the
// reciprocal).  No special-case handling: a = 0 or +inf gives NaN, so the sweeps pad with
// far finite records (padT) and route exact hits, whose denominators turn NaN or
// infinite, to the FP64 fix-up, which uses rcp64 / rsq64.
__device__ __forceinline__ double rcp64_w(double a) {
  const double y = __builtin_amdgcn_rcp(a);
  return fma(y, fma(-a, y, 1.0), y);
}
__device__ __forceinline__ double rsq64_w(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  const double t = a * y;
  return fma(0.5 * y, fma(-t, y, 1.0), y);
}

// log2 and exp2 in the FP64 sweeps (the power gradient's log2 r2 and the general-p weight
// 2^(-p/2 log2 r2)), from two 256-entry tables in LDS.  Every lane indexes them with its
// own value; 16-entry tables (conflict-free, but two and four more polynomial terms)
// measured 10-15% slower at 1M x 1M.
//  log2_t: a = 2^e m with m in [1/2, 1) (v_frexp_mant / v_frexp_exp); the top 8 mantissa
//    bits k pick c_k = (1 + (k + 1/2)/256) / 2, whose reciprocal (rounded) and -log2 of that
//    rounded reciprocal the table holds;
//    r = m (1/c_k) - 1 has |r| <= 2^-9 (one rounding, in the fma), and log2(m) =
//    -log2(1/c_k) + log2(1 + r), the latter as r times the series of ln(1 + r) / ln 2
//    through r^5: the first term left out, r^6 / (6 ln 2), is below 1.3e-17, under the
//    rounding of any result but those within 2^-6 of 0 (a within 1% of 1), where the
//    absolute error stays near 1e-17.  The sweeps need absolute accuracy: the power
//    gradient's terms are held relative to sum w |ln r2| (|z| + |Z|), and a general-p weight
//    2^(nh log2 r2) moves by |nh| ln2 times the error, below 3e-16 for p <= 64.  The
//    exponent is added last.  About 11 instructions against about 33 for log2_64.  Positive
//    finite a, subnormals included, are meaningful; a = 0 (an exact hit) gives an unspecified
//    finite value, and the sweeps never keep a result computed from one (such queries are
//    recomputed by the FP64 fix-up, and the data-direction sweeps move them to a far
//    coordinate).  +inf and NaN are not expected (finite padding).
//  exp2_t: k = round(256 x), x = k/256 + f with |f| <= 1/512 (exact); 2^x = 2^(k >> 8)
//    2^((k & 255)/256) 2^f, the table holding 2^(j/256) (rounded) and 2^f its Taylor series
//    in f ln 2 through the fifth power (truncation below 2^-54); v_ldexp applies 2^(k >> 8),
//    with the overflow to +inf and the underflow to subnormals and 0.  x = +inf gives +inf
//    (exact hits), -inf gives 0.
// The tables are static LDS arrays of the kernels that call *_table_init() at their start;
// those synchronise (after staging their first tile) before the first lookup.
constexpr int kLogTab = 256;
constexpr int kExpTab = 256;

__device__ __forceinline__ double2* log2_table() {
  __shared__ double2 tab[kLogTab];
  return tab;
}
__device__ __forceinline__ double* exp2_table() {
  __shared__ double tab[kExpTab];
  return tab;
}

__device__ __forceinline__ void log2_table_init() {
  const int t = threadIdx.x;
  if (t < kLogTab) {
    const double c = 0.5 * (1.0 + (t + 0.5) / kLogTab);
    const double inv = 1.0 / c;
    log2_table()[t] = make_double2(inv, -log2(inv));
  }
}
__device__ __forceinline__ void exp2_table_init() {
  const int t = threadIdx.x;
  if (t < kExpTab) exp2_table()[t] = exp2(static_cast<double>(t) / kExpTab);
}

__device__ __forceinline__ double log2_t(double a) {
  constexpr double L = 1.44269504088896340736;  // 1 / ln 2
  const double m = __builtin_amdgcn_frexp_mant(a);
  const double e = static_cast<double>(__builtin_amdgcn_frexp_exp(a));
  const unsigned int hi = static_cast<unsigned int>(__builtin_bit_cast(unsigned long long, m) >> 32);
  const int k = static_cast<int>((hi >> 12) & (kLogTab - 1));
  const double2 t = log2_table()[k];
  const double r = fma(m, t.x, -1.0);
  double p = L / 5.0;
  p = fma(p, r, -L / 4.0);
  p = fma(p, r, L / 3.0);
  p = fma(p, r, -L / 2.0);
  p = fma(p, r, L);
  return fma(r, p, t.y) + e;
}

__device__ __forceinline__ double exp2_t(double x) {
  constexpr double C1 = 0.69314718055994530942;  // ln 2
  constexpr double C2 = C1 * C1 / 2.0, C3 = C2 * C1 / 3.0, C4 = C3 * C1 / 4.0, C5 = C4 * C1 / 5.0;
  const double xc = fmin(fmax(x, -1100.0), 1100.0);  // NaN -> -1100 (its result is unused)
  const double kd = rint(xc * kExpTab);
  const int k = static_cast<int>(kd);
  const double f = fma(kd, -1.0 / kExpTab, xc);
  double p = C5;
  p = fma(p, f, C4);
  p = fma(p, f, C3);
  p = fma(p, f, C2);
  p = fma(p, f, C1);
  p = fma(p, f, 1.0);
  const double r = __builtin_amdgcn_ldexp(exp2_table()[k & (kExpTab - 1)] * p, k >> 8);
  return x == __builtin_huge_val() ? x : r;
}

// The general-p weight a^nh (nh = -p/2) in the FP64 sweeps that need no log2 (forward, data
// sweep; in the adjoint sweeps without dp, w / r2 = a^(nh - 1) the same way, nh - 1 standing
// for nh below), from two tables filled per call: a = 2^e m, m in [1, 2), k = top 8 bits;
// m = (1 + r) / i_k with i_k the rounded 1/c_k, c_k = 1 + (k + 1/2)/256, |r| <= 2^-9; so
// a^nh = [2^(e nh)] [i_k^(-nh)] (1 + r)^nh, the first two factors from the tables (2048 and
// 256 entries, library exp2 and pow) and the last as its binomial series through r^10
// (truncation below 2^-66 for |nh| <= 33).  Against exp2_t(nh log2_t(a)) the FP64 forward's
// inner loop drops from about 50 to 33 instructions a pair (29 to 19 of them FP64), and the
// rounding no longer grows with |nh log2 a|.  Zero and subnormal a give +inf (exact or
// near-coincident hits, settled by the FP64 fix-up).
constexpr int kPowExp = 2048;

__device__ __forceinline__ double* pow_etable() {
  __shared__ double tab[kPowExp];
  return tab;
}
__device__ __forceinline__ double2* pow_mtable() {
  __shared__ double2 tab[kLogTab];
  return tab;
}
__device__ __forceinline__ double* pow_coef() {
  __shared__ double c[12];
  return c;
}

__device__ __forceinline__ void pow_table_init(double nh) {
  for (int i = threadIdx.x; i < kPowExp; i += blockDim.x) {
    // 2^(e nh) with the product e nh split exactly (hi + lo), so that its rounding does not
    // grow with |e nh|; the last entry (a = +inf) gives weight 0.
    const double e = static_cast<double>(i - 1023);
    const double hi = e * nh;
    const double lo = fma(e, nh, -hi);
    pow_etable()[i] = i < kPowExp - 1 ? exp2(hi) * fma(lo, 0.69314718055994530942, 1.0) : 0.0;
  }
  for (int k = threadIdx.x; k < kLogTab; k += blockDim.x) {
    const double inv = 1.0 / (1.0 + (k + 0.5) / kLogTab);
    pow_mtable()[k] = make_double2(inv, pow(inv, -nh));
  }
  if (threadIdx.x == 0) {  // binomial coefficients C(nh, j), j = 0..10
    double c = 1.0;
    pow_coef()[0] = 1.0;
    for (int j = 1; j <= 10; ++j) {
      c = c * (nh - (j - 1)) / j;
      pow_coef()[j] = c;
    }
  }
}

__device__ __forceinline__ double pow_t(double a) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, a);
  const unsigned int hi = static_cast<unsigned int>(b >> 32);
  const int k = static_cast<int>((hi >> 12) & (kLogTab - 1));
  const int ei = static_cast<int>((hi >> 20) & 0x7ff);
  const double m = __builtin_bit_cast(double, (b & 0x000fffffffffffffull) | 0x3ff0000000000000ull);
  const double2 t = pow_mtable()[k];
  const double r = fma(m, t.x, -1.0);
  const double* c = pow_coef();
  double q = c[10];
#pragma unroll
  for (int j = 9; j >= 0; --j) q = fma(q, r, c[j]);
  const double res = pow_etable()[ei] * t.y * q;
  return a >= 0x1p-1022 ? res : __builtin_huge_val();
}

// Coordinate of padding records in the sweeps' LDS tiles: +inf in FP32 (every weight form
// gives exactly 0 there), a far finite value in FP64 (the one-step forms above give NaN at
// +inf).  The forward sweep never visits them (its last tile is cut to the data count); in
// the data-direction sweeps they carry a zero coefficient, so only their finiteness matters.
template <typename T>
__device__ __forceinline__ T padT() {
  return __builtin_huge_valf();
}
template <>
__device__ __forceinline__ double padT<double>() {
  return 0x1p400;
}

// Weight in the sweeps: weight<PM> in FP32; in FP64 the one-step forms for the fast classes.
template <int PM>
__device__ __forceinline__ float weight_sweep(float r2, float nhp) {
  return weight<PM>(r2, nhp);
}

template <int PM>
__device__ __forceinline__ double weight(double r2, double nhp);

template <int PM>
__device__ __forceinline__ double weight_sweep(double r2, double nhp) {
  if constexpr (PM == PM_2) {
    return rcp64_w(r2);
  } else if constexpr (PM == PM_1) {
    return rsq64_w(r2);
  } else if constexpr (PM == PM_3) {
    const double s = rsq64_w(r2);
    return s * s * s;
  } else if constexpr (PM == PM_4) {
    const double t = rcp64_w(r2);
    return t * t;
  } else if constexpr (PM == PM_25) {
    // d^-2.5 = s^3 / sqrt(s) with s = d^-1: two one-step reciprocal square roots and three
    // multiplies, where s^2 sqrt(s) would pay for the library's correctly rounded square
    // root (about a dozen instructions with its scaling and special cases)
    const double s = rsq64_w(r2);
    return s * s * s * rsq64_w(s);
  } else {  // general p: the tables of pow_t (pow_table_init in the calling kernel)
    return pow_t(r2);
  }
}

template <int PM>
__device__ __forceinline__ double weight(double r2, double nhp) {
  if constexpr (PM == PM_2) {
    return rcp64(r2);
  } else if constexpr (PM == PM_1) {
    return rsq64(r2);
  } else if constexpr (PM == PM_3) {
    const double s = rsq64(r2);
    return s * s * s;
  } else if constexpr (PM == PM_4) {
    const double t = rcp64(r2);
    return t * t;
  } else if constexpr (PM == PM_25) {
    const double s = rsq64(r2);
    return s * s * sqrt(s);
  } else {
    return exp2(nhp * log2_64(r2));
  }
}

// ---------------------------------------------------------------------------------------
// Compensated accumulation: (hi, lo) += x with Knuth's TwoSum (no magnitude assumption).
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void two_sum_acc(T& hi, T& lo, T x) {
  const T s = hi + x;
  const T bb = s - hi;
  const T e = (hi - (s - bb)) + (x - bb);
  hi = s;
  lo += e;
}

// Running sum of a blocked sweep: the plain sum of each 64-record block is added into it.
// FP32 block sums go into one FP64 accumulator (a conversion and an FP64 add, 2 VALU
// operations, where a TwoSum into an FP32 (hi, lo) pair takes 6; the same 2 registers, and
// the FP64 rounding is finer than the pair's); FP64 block sums keep a TwoSum pair.
template <typename T>
struct BlockSum;
template <>
struct BlockSum<float> {
  double s;
  __device__ __forceinline__ void zero() { s = 0.0; }
  __device__ __forceinline__ void add(float x) { s += static_cast<double>(x); }
  __device__ __forceinline__ double value() const { return s; }
};
template <>
struct BlockSum<double> {
  double hi, lo;
  __device__ __forceinline__ void zero() { hi = lo = 0.0; }
  __device__ __forceinline__ void add(double x) { two_sum_acc(hi, lo, x); }
  __device__ __forceinline__ double value() const { return hi + lo; }
};

// Neumaier accumulator for the FP64 fix-up paths.
struct NSum {
  double s = 0.0, c = 0.0;
  __device__ __forceinline__ void add(double v) {
    const double t = s + v;
    if (fabs(s) >= fabs(v))
      c += (s - t) + v;
    else
      c += (v - t) + s;
    s = t;
  }
  __device__ __forceinline__ double value() const { return s + c; }
};

// Fixed-order tree sum over the kWG threads of a workgroup.  `red` is LDS scratch of
// kWG doubles; every thread receives the total.  Contains barriers: call uniformly.
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = kWG / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ long long block_sum_i64(long long v, long long* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = kWG / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const long long r = red[0];
  __syncthreads();
  return r;
}

// Workspace header (doubles), written by the extent kernel of every call.
enum HdrSlot {
  H_SCALE = 0,     // power of two s applied to coordinates in the FP32 sweep (1 for FP64)
  H_THR_S = 1,     // upper flag threshold on the denominator, scaled units
  H_LO_S = 2,      // lower flag threshold on the denominator, scaled units
  H_DEN_UNIT = 3,  // factor s^p converting a scaled denominator to caller units
  H_THR_U = 4,     // upper flag threshold, caller units
  H_LO_U = 5,      // lower flag threshold, caller units
  H_EXTENT = 6,    // data extent (largest side of the bounding box; 1 if degenerate)
  H_VMAX = 7,      // largest |value| of the data points
  H_GEO_S = 8,     // near-coincidence threshold on the denominator, scaled units
  H_GEO_U = 9,     // near-coincidence threshold, caller units
  H_NEAR_R2 = 10,  // squared near-coincidence distance (1e-6 extent s)^2, scaled units
  H_REL = 11,      // 1 when the FP32 sweeps use per-query relative weights (large p), else 0
  H_BMIN = 12,     // [12..14] lower corner of the data bounding box, scaled units
  H_BEXT = 15,     // [15..17] sides of the data bounding box, scaled units
  H_GRID_H = 18,   // side of a grid cell (nearest-distance searches), scaled units
  H_GRID_INVH = 19,
  H_GRID_G = 20,   // [20..22] cells along each axis (1 along unused axes)
  H_COUNT_I = 32   // int slots start at byte 256: [0] flagged count, then GridInt
};

// Int slots of the header after the flagged count, used by the grid searches: the
// candidate check at [1..4], the ring search of every query at [5..8] (the same layout
// shifted by kGridNearestSlots).
enum GridInt {
  GI_FALLBACK = 1,  // queries the grid handed to the brute-force check (appended to a list)
  GI_BRUTE = 2,     // queries the brute-force check takes directly (few candidates)
  GI_GRID = 3,      // queries the grid search takes (0: the grid is not built this call)
  GI_TOTAL = 4      // scan total of the cell counts (the number of data points)
};
constexpr int kGridNearestSlots = 4;

// Grid of the nearest-distance searches: used for n in [kGridMinN, kGridMaxN] (below, the
// brute-force check is as cheap; above, the records would take too much workspace), about
// kGridPerCell points per cell, at most kGridMaxCells cells; the candidate check builds it
// only for at least kGridMinCand candidates (a build costs about one pass over the data).
constexpr int64_t kGridMinN = 65536;
constexpr int64_t kGridMaxN = int64_t(1) << 26;
constexpr int64_t kGridPerCell = 4;
constexpr int64_t kGridMaxCells = int64_t(1) << 22;
constexpr int kGridMinCand = 4096;
constexpr int kGridScanBlock = 4096;  // cells per block of the count scan (16 per thread)

// From this exponent on the FP32 sweeps use relative weights: a query's weights are taken
// relative to a power of two near its largest one, w' = (r2 sigma)^(-p/2) = w sigma^(-p/2)
// with sigma = 2^k chosen per query, so that no weight of Eq. 1 has to fit the FP32 range
// by itself.  (With the direct weights, 1M uniform points at p = 6 already put about one
// query in eight past the FP32-safe bound and into the FP64 recomputation, which then
// costs more than the relative form's nearest-distance pass.)  The forward takes sigma from the query's nearest squared distance (r2min
// sigma in [1/2, 1), so 1 < w'max <= 2^(p/2)); the adjoint takes it from the saved
// denominator (relative denominator E = D / sigma^(p/2) in [1, 2^(p/2))).  Because the
// nearest pairs then have r2 sigma close to 1, the weight's log2 / exp2 evaluation keeps
// about the accuracy it has at small p.
constexpr double kRelP = 6.0;
constexpr double kRelVmax = 4294967296.0;  // 2^32: largest |value| the relative sweeps take

// Adjoint scaling of one query from its denominator Ds (scaled units, finite, > 0):
// sigma = 2^k with k = floor((2/p) log2 Ds) (clamped to the normal FP32 range), E =
// Ds sigma^(-p/2) in [1, 2^(p/2)), and k itself (for log2 r2 = log2(r2 sigma) - k).
__device__ inline void rel_from_den(double Ds, double p, float& sig, float& k, double& E) {
  double kk = floor((2.0 / p) * log2(Ds));
  kk = fmin(fmax(kk, -125.0), 125.0);
  sig = __builtin_amdgcn_ldexpf(1.0f, static_cast<int>(kk));
  k = static_cast<float>(kk);
  E = Ds * exp2(-0.5 * p * kk);
}

// Forward scaling of one query from its nearest squared distance r2min (FP32, scaled
// units): sigma = 2^-e where r2min = m 2^e, m in [1/2, 1), so r2min sigma = m; the sweep's
// sums are multiplied by F = sigma^(p/2) (FP64) to give scaled-unit sums.  A zero,
// subnormal or non-finite r2min (the query is routed to the FP64 fix-up by its
// denominator) gets sigma = 1 when infinite and the clamped exponent otherwise.
__device__ inline void rel_from_min(float r2min, double p, float& sig, double& F) {
  int e = 0;
  if (r2min > 0.0f && r2min < __builtin_huge_valf()) e = __builtin_amdgcn_frexp_expf(r2min);
  if (r2min == 0.0f) e = -125;
  e = e < -125 ? -125 : (e > 125 ? 125 : e);
  sig = __builtin_amdgcn_ldexpf(1.0f, -e);
  F = exp2(-0.5 * p * static_cast<double>(e));
}

// Per-query route after a sweep (flag bytes):
//  F_FP32       the sweep's result stands;
//  F_CANDIDATE  the denominator exceeds (1e-6 extent)^-p: some data point may lie closer
//               than 1e-6 of the extent, or many moderate weights add up to that much (the
//               common case for p near 1 and large n); a check of the nearest distance
//               decides between the other two routes;
//  F_FP64       recomputed in FP64: an exact hit, a data point within 1e-6 of the extent,
//               a denominator past the FP32-safe cap, FP32 underflow, or not finite.
enum QueryRoute : uint8_t { F_FP32 = 0, F_CANDIDATE = 1, F_FP64 = 2 };

// Route of a query from its denominator; `units` selects the scaled (sweep) or the caller
// thresholds of the header.
__device__ __forceinline__ uint8_t route_of(double den, const double* __restrict__ hdr, bool caller_units) {
  const double cap = hdr[caller_units ? H_THR_U : H_THR_S];
  const double lo = hdr[caller_units ? H_LO_U : H_LO_S];
  const double geo = hdr[caller_units ? H_GEO_U : H_GEO_S];
  if (!(den <= cap && den > lo)) return F_FP64;
  return den > geo ? F_CANDIDATE : F_FP32;
}

// Per-workgroup partials of the extent kernels: [0..2] coordinate minima, [3..5] maxima,
// [6] largest |value|, [7] unused.
constexpr int kBboxStride = 8;

// Fills the header from the data extent and largest |value|.
//  s = 2^-e with extent * s in [0.5, 1), in both precisions: an exact scaling that keeps
//    every weight of points inside the box far from overflow and underflow (in FP64 it also
//    keeps the adjoint's w / r2 = d^(-p-2) in range where the caller's units would not, as
//    at coordinates of 1e-90).  Eq. 1 is invariant under it; the denominators leave the
//    sweeps in scaled units and are reported in the caller's as D = D_s s^p.
//  Near-coincidence: a data point closer than 1e-6 of the extent puts the denominator above
//  (1e-6 * extent)^-p, so queries above it are candidates whose nearest distance is then
//  checked against 1e-6 * extent (route_of, k_near_check).
//  Hard cap: a denominator that is not finite, or not above the lower threshold (FP32
//  underflow of the weights), is recomputed in FP64; on the FP32 path so is one above
//  2^80 / max(1, max|value|): below it every weight is at most that and every distance at
//  least 2^-21 (scaled units), which bounds every FP32 term and sum of the forward and
//  adjoint sweeps below 2^125.  Thresholds are finite: for large p, (1e-6 * extent)^-p
//  overflows, and an infinite threshold would pass an infinite denominator.
//  Relative weights (rel, FP32 with p >= kRelP): no weight is held in FP32 by itself, so the
//  cap becomes the value bound alone (every query goes to FP64 when max|value| > kRelVmax),
//  and the lower threshold is 2^(-10 p) (scaled units): a denominator above it has its
//  nearest squared distance below 2^20 n^(2/p), which keeps the adjoint's sigma above
//  2^-21 and its distance factors finite; farther queries are recomputed in FP64.
__device__ inline void fill_header(double* __restrict__ h, double ext, double vmax, double p,
                                   bool f32s, bool rel) {
  if (!(ext > 0.0) || !(ext < __builtin_huge_val())) ext = 1.0;
  int e = 0;
  (void)frexp(ext, &e);
  const double s = ldexp(1.0, -e);
  double cap_s = __DBL_MAX__;
  double lo_s = 0.0;
  if (f32s) {
    cap_s = ldexp(1.0, 80) / fmax(1.0, vmax);
    lo_s = ldexp(1.0, -60);
    if (rel) {
      cap_s = vmax <= kRelVmax ? __DBL_MAX__ : -1.0;
      lo_s = exp2(-10.0 * p);
    }
  }
  const double near = 1e-6 * ext * s;
  const double geo_s = fmin(pow(near, -p), __DBL_MAX__);
  const double unit = pow(s, p);
  h[H_SCALE] = s;
  h[H_THR_S] = cap_s;
  h[H_LO_S] = lo_s;
  h[H_DEN_UNIT] = unit;
  h[H_THR_U] = fmin(cap_s * unit, __DBL_MAX__);
  h[H_LO_U] = lo_s * unit;
  h[H_EXTENT] = ext;
  h[H_VMAX] = vmax;
  h[H_GEO_S] = geo_s;
  h[H_GEO_U] = fmin(geo_s * unit, __DBL_MAX__);
  h[H_NEAR_R2] = near * near;
  h[H_REL] = (f32s && rel) ? 1.0 : 0.0;
}

}  // namespace idw
