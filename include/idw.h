/*
 * idw.h - C ABI of the MI355X (gfx950) Shepard IDW library (libidw.so).
 *
 * The library evaluates Shepard's inverse-distance-weighting interpolant (Section 2.1,
 * Eq. 1 of Mei & Tian, "Performance Impact of Data Layout on the GPU-accelerated IDW
 * Interpolation"):
 *
 *     Z(q) = sum_j w_j(q) z_j / sum_j w_j(q),      w_j(q) = d(q, x_j)^-p,
 *
 * over ALL n data points (global IDW), d the Euclidean distance over dim = 2 or 3
 * coordinates, p > 0 real.  Where Eq. 1 is undefined (d = 0) the result is the mean value
 * of the data points that coincide exactly with q.
 *
 * Conventions shared by every entry point
 *  - Every array pointer is a DEVICE pointer owned by the caller.  The library never frees,
 *    retains or reallocates them; it reads inputs and writes outputs only.
 *  - All work is enqueued asynchronously on `stream` (a hipStream_t passed as void*; NULL
 *    is the legacy default stream).  Entry points never synchronise and never allocate
 *    device memory, except idw_batched_plan_create (documented there).
 *  - Arguments are validated on the host before anything is enqueued; on failure nothing is
 *    enqueued and a non-zero status is returned; idw_last_error() describes it.  Input
 *    values are not scanned: NaN or infinite coordinates/values give undefined results.
 *  - Results are bitwise reproducible for fixed inputs, sizes and configuration (no
 *    floating-point atomics; every sum has a fixed order; the only atomics are integer
 *    ones whose result does not depend on their order: a minimum and a work counter).
 *  - Element type follows the precision: IDW_FP32 and IDW_FP32_KAHAN read and write float
 *    arrays, IDW_FP64 double arrays.  Denominators (out_den, saved_den) and grad_p are
 *    always double.
 *  - FP64 recomputation: a query with a data point closer than 1e-6 of the data extent
 *    (exact hits included), or whose FP32 sums could leave the FP32 range (large |values|,
 *    or large p with the direct weights), is recomputed in FP64; the denominator
 *    nominates candidates and a nearest-distance check settles them.
 *  - Large p in FP32 (p >= 6): the FP32 sweeps take each query's weights relative to a
 *    power of two sigma near its largest one, w' = (d^2 sigma)^(-p/2), so that weights
 *    far outside the FP32 range stay on the FP32 path.  The forward first finds every
 *    query's nearest squared distance (one more pass over all pairs, about 5 operations
 *    each) and takes sigma from it; the adjoint takes sigma from the saved denominator.
 *    Such queries return to FP64 only when max|value| > 2^32 (then all of them) or when
 *    the query's denominator is below 2^(-10 p) in units where the data extent is in
 *    [1/2, 1) (no data point within about 2^10 extents).  A weight below FLT_MIN relative
 *    to its query's largest may be flushed to zero: a value gradient dL/dz_j can lose up
 *    to |g_i| 2^-126 per query i.  With separate_adjoint = 1 the adjoint keeps the direct
 *    weights and their FP64 routing.  Batched plans use the relative weights too.
 */
#ifndef IDW_H
#define IDW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
  IDW_OK = 0,
  IDW_EINVAL = 1,        /* bad argument (size, pointer, alignment, enum, p) */
  IDW_EDEVICE = 2,       /* no usable gfx950 device, or a HIP runtime error */
  IDW_ENOMEM = 3,        /* host/device allocation failed (plan creation only) */
  IDW_EUNSUPPORTED = 4,  /* valid but unsupported combination */
  IDW_EWORKSPACE = 5     /* workspace pointer missing, misaligned or too small */
};

/* Record layouts of a point set (Sections 3.1-3.5).  T is float (IDW_FP32) or double.
 * Data points carry coordinates and a value v; query points carry coordinates only.
 *   IDW_SOA    (Section 3.1) ptr[0..dim-1] = coordinate arrays T[n]; data: ptr[dim] = v[n].
 *   IDW_AOS    (Section 3.2) ptr[0] = packed records {x, y, (z), v} (queries {x, y, (z)}),
 *              no padding, T-aligned.
 *   IDW_AOAS   (Section 3.3, also the built-in float4/double4 form) ptr[0] = records of
 *              four T: {x, y, v, pad} / {x, y, z, v} (queries {x, y, (z), pad}); 16-byte
 *              (float) or 32-byte (double) aligned.
 *   IDW_HYBRID (Section 3.5, AoS + array of values) ptr[0] = packed coordinate records
 *              {x, y, (z)}; data: ptr[1] = v[n].
 *   IDW_SOAOS  (Section 3.4) ptr[0] = aligned coordinate records {x, y} (dim 2) or
 *              {x, y, z, pad} (dim 3), aligned to their size; data: ptr[1] = aligned
 *              value records {v, pad}. */
enum { IDW_SOA = 0, IDW_AOS = 1, IDW_AOAS = 2, IDW_HYBRID = 3, IDW_SOAOS = 4 };

/* Precision of the sweep.
 *   IDW_FP32: float inputs/outputs.  The all-pairs sweep runs in FP32 with blocked sums
 *     (plain FP32 inside 64-point blocks, each block sum added into an FP64 running sum);
 *     the ratio is taken in FP64; queries closer than 1e-6 of the data extent to a data
 *     point (including exact hits) are recomputed entirely in FP64.
 *   IDW_FP64: double inputs/outputs, FP64 sweep with plain FP64 sums inside 64-point
 *     blocks, each block sum merged into a (hi, lo) pair with TwoSum.
 *   IDW_FP32_KAHAN: as IDW_FP32, but the forward sweep updates FP32 (sum, error) pairs with
 *     a Kahan step on every pair instead of summing per block (the accuracy variant; about
 *     1.6x the forward's time).  idw_backward treats it as IDW_FP32; batched plans do not
 *     take it. */
enum { IDW_FP32 = 0, IDW_FP64 = 1, IDW_FP32_KAHAN = 2 };

/* Flags. */
#define IDW_EXCLUDE_SELF 0x1u /* leave-one-out: queries ARE the data set (m == n, same
                                 points in the same order); pair (i, i) is skipped */
#define IDW_NEED_DZ 0x2u      /* idw_backward: compute grad_z */
#define IDW_NEED_DP 0x4u      /* idw_backward: compute grad_p */
#define IDW_NEED_DQ 0x8u      /* idw_backward: compute grad_q */
#define IDW_NEED_DX 0x10u     /* idw_backward: compute grad_x (data coordinates) */

/* A point set.  n >= 0; dim 2 or 3; layout one of IDW_SOA..IDW_SOAOS; unused ptr[] slots
 * are ignored.  For data points n >= 1. */
typedef struct idw_points {
  const void* ptr[4];
  int64_t n;
  int32_t dim;
  int32_t layout;
} idw_points;

/* Optional launch configuration; zero fields select the library default.
 *   queries_per_lane  queries held in registers per lane of the forward sweep (FP32: 2, 4
 *                     or 8, and 4 or 8 for p >= 6; FP32_KAHAN: 4; FP64: 2 or 4; others
 *                     are refused with IDW_EUNSUPPORTED); 0 = FP64: 2; FP32: 2 for p = 1,
 *                     2, 3, 4, else 4 (the default split is computed for 4 then).
 *   split             number of data chunks swept by separate workgroups and merged in a
 *                     fixed order (1..1024); 0 = chosen from n and m so the grid has about
 *                     16384 workgroups, each chunk at least 2048 points (512 where 2048
 *                     would leave fewer than 2048 workgroups), and the partial sums take
 *                     at most 2 GiB
 *   batch_chunk       batched plans: data points per work item (rounded up to 512;
 *                     default: the autotuned value compiled into the library, see
 *                     idw_batched_defaults)
 *   batch_workgroups  batched plans: persistent workgroups (default: the autotuned value,
 *                     or 2 per compute unit when the library was built without a table)
 *   separate_adjoint  idw_backward: 1 = run the query-direction and data-direction sweeps
 *                     separately instead of the fused sweep (same results within the
 *                     stated tolerances; for comparison).  These sweeps use the direct
 *                     weights at every p (see "Large p in FP32").  The fused sweep serves
 *                     requests with dz and dp/dq, or with dx, and in FP32 with p >= 6 any
 *                     request.
 *   near_search       nearest-distance searches (the near-coincidence check of candidate
 *                     queries, and the nearest distance every query needs for the relative
 *                     weights of p >= 6): 0 = a uniform grid over the data points, built in
 *                     the workspace, for 65,536 to 2^26 data points (queries in dense cells
 *                     fall back to brute force), brute force otherwise; 1 = brute force over
 *                     all pairs always (for comparison; the results are the same bit for bit)
 *   reserved          must be zero
 * Negative fields, non-zero reserved fields, and separate_adjoint or near_search outside
 * {0, 1} are rejected with IDW_EINVAL. */
typedef struct idw_config {
  int32_t queries_per_lane;
  int32_t split;
  int32_t batch_chunk;
  int32_t batch_workgroups;
  int32_t separate_adjoint;
  int32_t near_search;
  int32_t reserved[2];
} idw_config;

/* Library version string (static storage). */
const char* idw_version(void);

/* Description of the last error raised on the calling thread (static thread-local
 * storage, valid until the next call on that thread). */
const char* idw_last_error(void);

/* Bytes of a record of `layout` for dim and precision, per pointer slot: writes
 * bytes[0..3] (0 for unused slots).  For data (is_data != 0) or query records.  Host
 * only; never touches the device.  Returns IDW_OK or IDW_EINVAL. */
int idw_record_bytes(int32_t layout, int32_t dim, int32_t precision, int32_t is_data,
                     size_t bytes[4]);

/* Device workspace needed for these point sets with `cfg` (nullable).  With no IDW_NEED_*
 * bit in `flags` it is the forward's need; with any of them it covers idw_forward and
 * idw_backward with those gradients (one workspace then serves both; the forward uses a
 * prefix of it, and a backward without IDW_NEED_DX a prefix of the one with it).  The
 * forward keeps the partial sums of its data chunks (268 MB at n = m = 2^20); the fused
 * adjoint per-range query partials and per-group data partials (3.2 GB there, plus
 * dim x 2.1 GB for IDW_NEED_DX); each such array stays within 2 GiB (dim times that for
 * the dx partials) or one row of the point set, whatever the sizes.  For 65,536 <= n <=
 * 2^26 (and near_search = 0) the forward part holds the grid of the nearest-distance
 * searches: about 18 B per data point (34 B in FP64) and 4 B per query.  Host only. */
int idw_workspace_size(const idw_points* data, const idw_points* query, int32_t precision,
                       uint32_t flags, const idw_config* cfg, size_t* bytes);

/* Forward sweep (Eq. 1).
 *   data, query  point sets (device memory); query->n == m may be 0 (no-op).
 *   p            power parameter, finite, 0 < p <= 64.
 *   flags        0 or IDW_EXCLUDE_SELF.
 *   out_z        [m] interpolated values, element type of `precision`.
 *   out_den      [m] double denominators sum_j w_j in the caller's units (nullable);
 *                +inf for queries that coincide exactly with a data point.  Needed by
 *                idw_backward.
 *   workspace    device buffer of at least idw_workspace_size() bytes, 256-byte aligned;
 *                its contents on entry are irrelevant and on exit unspecified.
 * The workspace is in use until the enqueued work completes; concurrent calls must use
 * different workspaces. */
int idw_forward(const idw_points* data, const idw_points* query, double p, int32_t precision,
                uint32_t flags, void* out_z, double* out_den, void* workspace,
                size_t workspace_bytes, void* stream, const idw_config* cfg);

/* idw_forward for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same computation,
 * with the workspace taken from a static device array of the library (64 MiB per device,
 * held from the first call on that device until the process ends) instead of a caller
 * buffer.  The caller still passes the point sets and out_z / out_den as for idw_forward.
 * With cfg->split 0, where the default data split's partial sums do not fit the array, the
 * largest split that fits is taken: the results are then bit for bit those of idw_forward
 * given that split in cfg (otherwise those of idw_forward with the same cfg).  Sizes whose
 * forward workspace (idw_workspace_size with no IDW_NEED_* bit) exceeds 64 MiB even
 * unsplit are rejected with IDW_EWORKSPACE before anything is enqueued; the benchmark size
 * n = m = 2^20 fits in both precisions.  Allocates nothing and calls no
 * allocating routine.  Every call on a device uses that device's one array, and leaves
 * its contents behind: calls that overlap on one device (other streams, other threads, or
 * a second call before the first has completed on a different stream) race and give
 * undefined results; calls in order on one stream do not.  (With kernel timing switched on
 * by idw_timing_enable, its sweep records HIP events as idw_forward's does.) */
int idw_forward_noalloc(const idw_points* data, const idw_points* query, double p, int32_t precision,
                        uint32_t flags, void* out_z, double* out_den, void* stream, const idw_config* cfg);

/* Adjoint of idw_forward: given grad_out[i] = dL/dZ_i, writes
 *   grad_z [n]       dL/dz_j   (element type of precision)   if flags & IDW_NEED_DZ
 *   grad_p [1]       dL/dp     (double, device)              if flags & IDW_NEED_DP
 *   grad_q [m*dim]   dL/dq_i   row-major, element type       if flags & IDW_NEED_DQ
 *   grad_x [n*dim]   dL/dx_j   row-major, element type       if flags & IDW_NEED_DX
 * (pointers of gradients not requested are ignored and may be null).  saved_z / saved_den
 * are idw_forward's out_z / out_den for the same inputs and p.  The formulas are those of
 * Eq. 1 differentiated: dZ_i/dz_j = w_ij / D_i,
 * dZ_i/dp = -(1/D_i) sum_j w_ij (1/2) ln(d_ij^2) (z_j - Z_i),
 * dZ_i/dq_i = -(p/D_i) sum_j (w_ij / d_ij^2) (z_j - Z_i)(q_i - x_j),
 * dZ_i/dx_j = (p/D_i)(w_ij / d_ij^2)(z_j - Z_i)(q_i - x_j); at an exact hit with h
 * coincident points, dZ_i/dz_j = 1/h for each of them and the other terms are 0.
 * Queries within 1e-6 of the extent of a data point are handled in FP64.  In FP32 with
 * p >= 6 every request (any combination of IDW_NEED_* bits) runs in the fused sweep with
 * relative weights unless cfg->separate_adjoint is 1. */
int idw_backward(const idw_points* data, const idw_points* query, double p, int32_t precision,
                 uint32_t flags, const void* grad_out, const void* saved_z,
                 const double* saved_den, void* grad_z, double* grad_p, void* grad_q,
                 void* grad_x, void* workspace, size_t workspace_bytes, void* stream,
                 const idw_config* cfg);

/* ---- Kernel timing (benchmarks).  When enabled, idw_forward / idw_backward bracket each
 * all-pairs sweep kernel with HIP events recorded on the launch stream.  Not for use
 * under graph capture.  Host-side state is process-wide and mutex-protected. ---- */
enum { IDW_T_FWD_SWEEP = 0, IDW_T_BWD_QUERY = 1, IDW_T_BWD_DATA = 2, IDW_T_BWD_FUSED = 3,
       IDW_T_COUNT = 4 };

/* Enables (on != 0) or disables timing; either way drops pending events and resets the
 * totals. */
int idw_timing_enable(int32_t on);

/* Waits for every recorded event, then returns the total milliseconds and launch count
 * of sweep `which` (IDW_T_*) since the last idw_timing_enable. */
int idw_timing_read(int32_t which, double* total_ms, int64_t* launches);

/* ---- Batched form: many independent instances in one persistent launch. ---- */

/* One instance: its own data, queries, p and outputs (device pointers). */
typedef struct idw_instance {
  idw_points data;
  idw_points query;
  double p;
  void* out_z;      /* [query.n], element type of the plan precision */
  double* out_den;  /* [query.n], nullable */
} idw_instance;

typedef struct idw_plan idw_plan;

/* Builds a plan for `count` instances (host descriptors, copied; the device arrays they
 * name must stay valid while the plan is used).  Precision IDW_FP32 only; every instance
 * uses the IDW_AOAS layout for data and queries, has its own dim (2 or 3), p (any valid
 * p; 1, 2 and 3 have fast forms) and sizes.  The sweep is the FP32 sweep of idw_forward
 * with its FP64 ratio and FP64 fix-up of near-coincident queries; instances with p >= 6
 * use its relative weights (a nearest-distance pass over their work items comes first,
 * see "Large p in FP32" above).  The plan allocates its
 * device work list here (the only allocating entry point) and captures a HIP graph on
 * the first idw_batched call for a given workspace.  `cfg` may be NULL. */
int idw_batched_plan_create(const idw_instance* instances, int32_t count, int32_t precision,
                            const idw_config* cfg, idw_plan** out_plan);

/* Device workspace bytes needed by idw_batched for this plan. */
int idw_batched_plan_workspace(const idw_plan* plan, size_t* bytes);

/* The launch parameters a plan uses: `chunk` = data points per work item (a multiple of
 * 512), `workgroups` = persistent workgroups asked for (the launch takes at most one per
 * work item).  Host only; IDW_EINVAL on a null argument. */
int idw_batched_plan_params(const idw_plan* plan, int64_t* chunk, int32_t* workgroups);

/* The defaults a plan takes where its configuration leaves batch_chunk or batch_workgroups
 * at 0: the parameters the autotuner chose for gfx950 (a table in the source tree), compiled
 * into the library by its build.  `workgroups` = 0 stands for two per compute unit.  Host
 * only, no device needed; IDW_EINVAL on a null argument. */
int idw_batched_defaults(int64_t* chunk, int32_t* workgroups);

/* Runs every instance of the plan: one graph launch on `stream`. */
int idw_batched(idw_plan* plan, void* workspace, size_t workspace_bytes, void* stream);

/* Releases the plan (synchronises with the device first). */
void idw_batched_plan_destroy(idw_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* IDW_H */
