/*
 * A plain C client of libidw: reads a point set from a binary file, runs idw_forward and
 * idw_backward through the C ABI (device memory from the HIP runtime, default stream) and
 * writes Z, D, dz, dp and dq to a binary file.  Used by tests/test_c_abi.py to show that the
 * boundary needs nothing beyond include/idw.h, libidw.so and the HIP runtime.
 *
 * Input file (little-endian): int64 n, int64 m, int32 dim, int32 pad, double p,
 *   then n*dim doubles x, n doubles z, m*dim doubles q, m doubles g.
 * Output file: m doubles Z, m doubles D, n doubles dz, 1 double dp, m*dim doubles dq.
 * The sweep runs in FP32 on the hybrid layout (packed coordinates + value array).
 * With the single argument --batched-params it instead builds a batched plan with no
 * configuration and prints the launch parameters the plan took.
 * Exit status 0 on success; otherwise the library's error text goes to stderr.
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/idw.h"

#define CHECK_HIP(x)                                                        \
  do {                                                                      \
    if ((x) != hipSuccess) {                                                \
      fprintf(stderr, "HIP error at line %d: %s\n", __LINE__, #x);          \
      return 2;                                                             \
    }                                                                       \
  } while (0)
#define CHECK_IDW(x)                                                        \
  do {                                                                      \
    int rc_ = (x);                                                          \
    if (rc_ != IDW_OK) {                                                    \
      fprintf(stderr, "libidw status %d: %s\n", rc_, idw_last_error());     \
      return 3;                                                             \
    }                                                                       \
  } while (0)

static float* to_f32(const double* a, size_t k) {
  float* r = (float*)malloc(k * sizeof(float));
  for (size_t i = 0; i < k; ++i) r[i] = (float)a[i];
  return r;
}

static void* upload(const void* host, size_t bytes) {
  void* d = NULL;
  if (hipMalloc(&d, bytes ? bytes : 4) != hipSuccess) return NULL;
  if (bytes && hipMemcpy(d, host, bytes, hipMemcpyHostToDevice) != hipSuccess) return NULL;
  return d;
}

/* `--batched-params`: builds a batched plan for one small instance with no configuration
 * and prints the launch parameters it took (the library's compiled-in tuned defaults). */
static int batched_params(void) {
  const int64_t n = 1024, m = 256;
  float* rec = (float*)calloc((size_t)(n + m) * 4, sizeof(float));
  for (int64_t j = 0; j < n + m; ++j) {
    rec[4 * j] = (float)(j % 37) / 37.0f;
    rec[4 * j + 1] = (float)(j % 53) / 53.0f;
    rec[4 * j + 2] = 1.0f;
  }
  void* d = upload(rec, sizeof(float) * 4 * (size_t)n);
  void* q = upload(rec + 4 * n, sizeof(float) * 4 * (size_t)m);
  void* z = NULL;
  CHECK_HIP(hipMalloc(&z, sizeof(float) * m));
  if (!d || !q) return 2;
  idw_instance inst = {{{d, NULL, NULL, NULL}, n, 2, IDW_AOAS}, {{q, NULL, NULL, NULL}, m, 2, IDW_AOAS}, 2.0, z, NULL};
  idw_plan* plan = NULL;
  CHECK_IDW(idw_batched_plan_create(&inst, 1, IDW_FP32, NULL, &plan));
  int64_t chunk = 0, dchunk = 0;
  int32_t wg = 0, dwg = 0;
  CHECK_IDW(idw_batched_plan_params(plan, &chunk, &wg));
  CHECK_IDW(idw_batched_defaults(&dchunk, &dwg));
  idw_batched_plan_destroy(plan);
  printf("plan chunk=%lld workgroups=%d defaults chunk=%lld workgroups=%d\n", (long long)chunk, wg,
         (long long)dchunk, dwg);
  return 0;
}

int main(int argc, char** argv) {
  if (argc == 2 && strcmp(argv[1], "--batched-params") == 0) return batched_params();
  if (argc != 3) {
    fprintf(stderr, "usage: %s input.bin output.bin | --batched-params\n", argv[0]);
    return 1;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 1;
  int64_t n = 0, m = 0;
  int32_t dim = 0, pad = 0;
  double p = 0.0;
  if (fread(&n, 8, 1, f) != 1 || fread(&m, 8, 1, f) != 1 || fread(&dim, 4, 1, f) != 1 ||
      fread(&pad, 4, 1, f) != 1 || fread(&p, 8, 1, f) != 1)
    return 1;
  double* hx = (double*)malloc(sizeof(double) * n * dim);
  double* hz = (double*)malloc(sizeof(double) * n);
  double* hq = (double*)malloc(sizeof(double) * m * dim);
  double* hg = (double*)malloc(sizeof(double) * m);
  if (fread(hx, 8, n * dim, f) != (size_t)(n * dim) || fread(hz, 8, n, f) != (size_t)n ||
      fread(hq, 8, m * dim, f) != (size_t)(m * dim) || fread(hg, 8, m, f) != (size_t)m)
    return 1;
  fclose(f);

  float *fx = to_f32(hx, n * dim), *fz = to_f32(hz, n), *fq = to_f32(hq, m * dim), *fg = to_f32(hg, m);
  void* dx = upload(fx, sizeof(float) * n * dim);
  void* dz_in = upload(fz, sizeof(float) * n);
  void* dq_in = upload(fq, sizeof(float) * m * dim);
  void* dg = upload(fg, sizeof(float) * m);
  if (!dx || !dz_in || !dq_in || !dg) return 2;

  idw_points data = {{dx, dz_in, NULL, NULL}, n, dim, IDW_HYBRID};
  idw_points query = {{dq_in, NULL, NULL, NULL}, m, dim, IDW_HYBRID};
  const uint32_t need = IDW_NEED_DZ | IDW_NEED_DP | IDW_NEED_DQ;
  size_t ws_bytes = 0;
  CHECK_IDW(idw_workspace_size(&data, &query, IDW_FP32, need, NULL, &ws_bytes));
  void *ws = NULL, *Z = NULL, *D = NULL, *gz = NULL, *gp = NULL, *gq = NULL;
  CHECK_HIP(hipMalloc(&ws, ws_bytes));
  CHECK_HIP(hipMalloc(&Z, sizeof(float) * m));
  CHECK_HIP(hipMalloc(&D, sizeof(double) * m));
  CHECK_HIP(hipMalloc(&gz, sizeof(float) * n));
  CHECK_HIP(hipMalloc(&gp, sizeof(double)));
  CHECK_HIP(hipMalloc(&gq, sizeof(float) * m * dim));
  CHECK_IDW(idw_forward(&data, &query, p, IDW_FP32, 0, Z, (double*)D, ws, ws_bytes, NULL, NULL));
  CHECK_IDW(idw_backward(&data, &query, p, IDW_FP32, need, dg, Z, (const double*)D, gz, (double*)gp, gq,
                         NULL, ws, ws_bytes, NULL, NULL));
  CHECK_HIP(hipDeviceSynchronize());

  float* hZ = (float*)malloc(sizeof(float) * m);
  double* hD = (double*)malloc(sizeof(double) * m);
  float* hgz = (float*)malloc(sizeof(float) * n);
  double hgp = 0.0;
  float* hgq = (float*)malloc(sizeof(float) * m * dim);
  CHECK_HIP(hipMemcpy(hZ, Z, sizeof(float) * m, hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(hD, D, sizeof(double) * m, hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(hgz, gz, sizeof(float) * n, hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(&hgp, gp, sizeof(double), hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(hgq, gq, sizeof(float) * m * dim, hipMemcpyDeviceToHost));

  FILE* o = fopen(argv[2], "wb");
  if (!o) return 1;
  for (int64_t i = 0; i < m; ++i) {
    double v = hZ[i];
    fwrite(&v, 8, 1, o);
  }
  fwrite(hD, 8, m, o);
  for (int64_t j = 0; j < n; ++j) {
    double v = hgz[j];
    fwrite(&v, 8, 1, o);
  }
  fwrite(&hgp, 8, 1, o);
  for (int64_t k = 0; k < m * dim; ++k) {
    double v = hgq[k];
    fwrite(&v, 8, 1, o);
  }
  fclose(o);
  printf("c client ok: n=%lld m=%lld dim=%d\n", (long long)n, (long long)m, dim);
  return 0;
}
