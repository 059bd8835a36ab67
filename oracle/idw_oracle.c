/*
 * FP64 reference ("oracle") for Shepard inverse-distance-weighting interpolation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls this
 * file; only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * use it.  It shares no code, header or constant with the HIP library.
 *
 * What it computes (Shepard's weighting function, Section 2.1, Eq. 1):
 *     Z(q) = sum_j w_j(q) z_j / sum_j w_j(q),      w_j(q) = 1 / d(q, x_j)^p
 * with d the Euclidean distance over `dim` coordinates and p > 0 real.
 * Readings taken where the paper is silent (each one is listed in the design notes):
 *   - d is the plain Euclidean distance over all coordinates (Eq. 1 only says "distance");
 *   - the sum runs over all n data points (global IDW: n is the total number of points);
 *   - at d = 0, Eq. 1 is undefined; the result is the mean value of every data point that
 *     coincides exactly with q (the limit of Eq. 1 as q approaches a data point; with a
 *     single coincident point this is that point's value);
 *   - summation order is unspecified; every sum here is Neumaier-compensated so that the
 *     oracle sits closer to the exact value than any GPU path it checks.
 * Gradients follow from differentiating Eq. 1:
 *     dZ/dz_j = w_j / D,   D = sum_j w_j
 *     dZ/dp   = -(1/D) sum_j w_j * (1/2) ln(r2_j) * (z_j - Z)
 *     dZ/dq   = -(p/D) sum_j (w_j / r2_j) * (z_j - Z) * (q - x_j)
 * and at an exact hit (h coincident points): dZ/dz_j = 1/h for each coincident j, and
 * dZ/dp = dZ/dq = 0.  With respect to the data coordinates (w_j depends on x_j through
 * r2_j = |q - x_j|^2 only):
 *     dZ/dx_j = (p/D) (w_j / r2_j) * (z_j - Z) * (q - x_j)
 * so that sum_j dZ/dx_j = -dZ/dq (Z depends on differences q - x_j only); at an exact hit
 * Z is the mean of the coincident values whatever the other points' positions, and
 * dZ/dx_j = 0 (the reading that matches dZ/dq = 0 there).
 *
 * Arrays: coordinates are row-major [count][dim] doubles; values are [n] doubles.
 * `self_index` (nullable) names, per query, one data index to leave out (leave-one-out).
 * All functions are single-threaded plain loops; they return 0 on success and -1 on bad
 * arguments.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct { double s, c; } nsum;

/* Neumaier's improved Kahan summation: s carries the sum, c the running correction. */
static void nadd(nsum* a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v))
    a->c += (a->s - t) + v;
  else
    a->c += (v - t) + a->s;
  a->s = t;
}
static double nval(const nsum* a) { return a->s + a->c; }

static double sqdist(const double* a, const double* b, int dim) {
  double r2 = 0.0;
  for (int k = 0; k < dim; ++k) {
    double d = a[k] - b[k];
    r2 += d * d;
  }
  return r2;
}

/* w = d^-p written through the squared distance: d^-p = (r2)^(-p/2). */
static double weight(double r2, double p) { return pow(r2, -0.5 * p); }

/*
 * Forward sweep.  Per query i writes
 *   Z[i]  interpolated value (Eq. 1, or the hit mean),
 *   D[i]  sum of weights over the non-coincident points (the denominator of Eq. 1),
 *   S[i]  summation scale sum_j w_j |z_j| / D (|Z| at a hit): an upper bound of |Z| used
 *         to express errors relative to the conditioning of the sum (nullable),
 *   H[i]  number of data points that coincide exactly with the query (nullable).
 */
int idw_oracle_forward(int64_t n, int dim, const double* x, const double* z, int64_t m,
                       const double* q, double p, const int64_t* self_index, double* Z,
                       double* D, double* S, int64_t* H) {
  if (n < 1 || m < 0 || (dim != 2 && dim != 3) || !(p > 0.0) || !x || !z || (m && (!q || !Z)))
    return -1;
  for (int64_t i = 0; i < m; ++i) {
    nsum num = {0, 0}, den = {0, 0}, sab = {0, 0}, hz = {0, 0};
    int64_t h = 0;
    const double* qi = q + i * dim;
    for (int64_t j = 0; j < n; ++j) {
      if (self_index && self_index[i] == j) continue;
      double r2 = sqdist(qi, x + j * dim, dim);
      if (r2 == 0.0) {
        ++h;
        nadd(&hz, z[j]);
        continue;
      }
      double w = weight(r2, p);
      nadd(&num, w * z[j]);
      nadd(&den, w);
      nadd(&sab, w * fabs(z[j]));
    }
    double Zi;
    if (h > 0) {
      Zi = nval(&hz) / (double)h;
    } else {
      Zi = nval(&num) / nval(&den);
    }
    Z[i] = Zi;
    if (D) D[i] = nval(&den);
    if (S) S[i] = h > 0 ? fabs(Zi) : nval(&sab) / nval(&den);
    if (H) H[i] = h;
  }
  return 0;
}

/*
 * Adjoint.  Given g[i] = dL/dZ_i, writes
 *   dz[n]      dL/dz_j = sum_i g_i dZ_i/dz_j            (nullable)
 *   dp[1]      dL/dp   = sum_i g_i dZ_i/dp              (nullable)
 *   dq[m*dim]  dL/dq_i = g_i dZ_i/dq_i                  (nullable)
 * and, when the scale pointers are given, the matching sums of absolute terms
 *   dz_scale[n] = sum_i |g_i| w_ij / D_i,  dp_scale[1] = sum_i |g_i| (1/D_i) sum_j |term|,
 *   dq_scale[m] = |g_i| (p/D_i) sum_j (w/r2) |z_j - Z_i| |q_i - x_j|,
 * which bound the conditioning of each sum (errors are stated relative to them).
 * The dp and dq sums are centred on Z_i; near a data point z_j - Z_i is tiny and those
 * sums become sensitive to the last bits of z and Z (a relative perturbation e of the
 * values moves them by about e times the uncentred sums).  dp_cond / dq_cond give those
 * uncentred sums, with |z_j| + |Z_i| in place of |z_j - Z_i| (nullable).
 */
int idw_oracle_backward(int64_t n, int dim, const double* x, const double* z, int64_t m,
                        const double* q, double p, const int64_t* self_index, const double* g,
                        double* dz, double* dp, double* dq, double* dz_scale,
                        double* dp_scale, double* dq_scale, double* dp_cond, double* dq_cond) {
  if (n < 1 || m < 0 || (dim != 2 && dim != 3) || !(p > 0.0) || !x || !z || (m && (!q || !g)))
    return -1;
  nsum* dzs = (nsum*)calloc((size_t)n, sizeof(nsum));
  nsum* dza = (nsum*)calloc((size_t)n, sizeof(nsum));
  if (!dzs || !dza) {
    free(dzs);
    free(dza);
    return -1;
  }
  nsum dpt = {0, 0}, dpa = {0, 0}, dpc = {0, 0};
  for (int64_t i = 0; i < m; ++i) {
    const double* qi = q + i * dim;
    double Zi, Di;
    int64_t h;
    if (idw_oracle_forward(n, dim, x, z, 1, qi, p, self_index ? self_index + i : NULL, &Zi, &Di,
                           NULL, &h) != 0) {
      free(dzs);
      free(dza);
      return -1;
    }
    double gi = g[i];
    if (h > 0) {
      /* Exact hit: Z is the mean of the coincident values. */
      for (int64_t j = 0; j < n; ++j) {
        if (self_index && self_index[i] == j) continue;
        if (sqdist(qi, x + j * dim, dim) == 0.0) {
          nadd(&dzs[j], gi / (double)h);
          nadd(&dza[j], fabs(gi) / (double)h);
        }
      }
      if (dq)
        for (int k = 0; k < dim; ++k) dq[i * dim + k] = 0.0;
      if (dq_scale) dq_scale[i] = 0.0;
      if (dq_cond) dq_cond[i] = 0.0;
      continue;
    }
    nsum P = {0, 0}, Pa = {0, 0}, Pc = {0, 0}, G[3] = {{0, 0}, {0, 0}, {0, 0}}, Ga = {0, 0},
         Gc = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
      if (self_index && self_index[i] == j) continue;
      const double* xj = x + j * dim;
      double r2 = sqdist(qi, xj, dim);
      double w = weight(r2, p);
      double c = z[j] - Zi;
      double lp = w * 0.5 * log(r2) * c;
      nadd(&P, lp);
      nadd(&Pa, fabs(lp));
      const double cabs = fabs(z[j]) + fabs(Zi);
      nadd(&Pc, fabs(w * 0.5 * log(r2)) * cabs);
      double u = (w / r2) * c;
      double ua = 0.0;
      for (int k = 0; k < dim; ++k) {
        double dk = qi[k] - xj[k];
        nadd(&G[k], u * dk);
        ua += fabs(dk);
      }
      nadd(&Ga, fabs(u) * ua);
      nadd(&Gc, (w / r2) * cabs * ua);
      nadd(&dzs[j], gi * w / Di);
      nadd(&dza[j], fabs(gi) * w / Di);
    }
    nadd(&dpt, -gi * nval(&P) / Di);
    nadd(&dpa, fabs(gi) * nval(&Pa) / Di);
    nadd(&dpc, fabs(gi) * nval(&Pc) / Di);
    if (dq)
      for (int k = 0; k < dim; ++k) dq[i * dim + k] = -(p * gi / Di) * nval(&G[k]);
    if (dq_scale) dq_scale[i] = fabs(p * gi / Di) * nval(&Ga);
    if (dq_cond) dq_cond[i] = fabs(p * gi / Di) * nval(&Gc);
  }
  for (int64_t j = 0; j < n; ++j) {
    if (dz) dz[j] = nval(&dzs[j]);
    if (dz_scale) dz_scale[j] = nval(&dza[j]);
  }
  if (dp) dp[0] = nval(&dpt);
  if (dp_scale) dp_scale[0] = nval(&dpa);
  if (dp_cond) dp_cond[0] = nval(&dpc);
  free(dzs);
  free(dza);
  return 0;
}

/*
 * Adjoint with respect to the data coordinates.  Given g[i] = dL/dZ_i, writes
 *   dx[n*dim]   dL/dx_j = sum_i g_i dZ_i/dx_j
 *               = sum_i (p g_i / D_i) (w_ij / r2_ij) (z_j - Z_i) (q_i - x_j)
 * over the queries without an exact hit (a hit query contributes nothing), and, when
 * given, dx_cond[n] = sum_i |p g_i / D_i| (w_ij / r2_ij) (|z_j| + |Z_i|) sum_k |q_ik - x_jk|,
 * the uncentred sum that bounds the sensitivity of dx_j to the last bits of the values
 * (as dq_cond does for dq).  Pairs left out by self_index are skipped.
 */
int idw_oracle_backward_x(int64_t n, int dim, const double* x, const double* z, int64_t m,
                          const double* q, double p, const int64_t* self_index, const double* g,
                          double* dx, double* dx_cond) {
  if (n < 1 || m < 0 || (dim != 2 && dim != 3) || !(p > 0.0) || !x || !z || !dx ||
      (m && (!q || !g)))
    return -1;
  nsum* acc = (nsum*)calloc((size_t)n * (size_t)dim, sizeof(nsum));
  nsum* cnd = (nsum*)calloc((size_t)n, sizeof(nsum));
  if (!acc || !cnd) {
    free(acc);
    free(cnd);
    return -1;
  }
  for (int64_t i = 0; i < m; ++i) {
    const double* qi = q + i * dim;
    double Zi, Di;
    int64_t h;
    if (idw_oracle_forward(n, dim, x, z, 1, qi, p, self_index ? self_index + i : NULL, &Zi, &Di,
                           NULL, &h) != 0) {
      free(acc);
      free(cnd);
      return -1;
    }
    if (h > 0) continue;
    const double a = p * g[i] / Di;
    for (int64_t j = 0; j < n; ++j) {
      if (self_index && self_index[i] == j) continue;
      const double* xj = x + j * dim;
      const double r2 = sqdist(qi, xj, dim);
      const double f = weight(r2, p) / r2;
      const double u = a * f * (z[j] - Zi);
      double ea = 0.0;
      for (int k = 0; k < dim; ++k) {
        const double e = qi[k] - xj[k];
        nadd(&acc[j * dim + k], u * e);
        ea += fabs(e);
      }
      nadd(&cnd[j], fabs(a) * f * (fabs(z[j]) + fabs(Zi)) * ea);
    }
  }
  for (int64_t j = 0; j < n; ++j) {
    for (int k = 0; k < dim; ++k) dx[j * dim + k] = nval(&acc[j * dim + k]);
    if (dx_cond) dx_cond[j] = nval(&cnd[j]);
  }
  free(acc);
  free(cnd);
  return 0;
}
