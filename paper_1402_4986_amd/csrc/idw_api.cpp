// C ABI of libidw.so: argument validation, workspace carving, launch configuration and
// dispatch to the per-layout kernel translation units.  No entry point here allocates
// device memory or synchronises.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/idw.h"
#include "idw_api_internal.hpp"
#include "idw_launch.hpp"

namespace idw {

static thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

void clear_error() { g_err.clear(); }

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return IDW_OK;
  return fail(IDW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---- device check: the code objects are built for gfx950 only ----
int check_device() {
  static std::mutex mu;
  static int state[64] = {0};  // 0 unknown, 1 ok, 2 bad
  int dev = 0;
  int cnt = 0;
  if (hipGetDeviceCount(&cnt) != hipSuccess || cnt <= 0)
    return fail(IDW_EDEVICE, "no HIP device available");
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
    return fail(IDW_EDEVICE, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(mu);
  if (state[dev] == 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
      return fail(IDW_EDEVICE, "hipGetDeviceProperties failed");
    state[dev] = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
  }
  if (state[dev] != 1) return fail(IDW_EDEVICE, "device %d is not gfx950", dev);
  return IDW_OK;
}

// ---- validation ----
static size_t elem(int precision) { return precision == IDW_FP64 ? 8 : 4; }
static bool known_precision(int p) { return p == IDW_FP32 || p == IDW_FP64 || p == IDW_FP32_KAHAN; }

int record_bytes(int layout, int dim, int precision, bool is_data, size_t b[4]) {
  for (int k = 0; k < 4; ++k) b[k] = 0;
  if (dim != 2 && dim != 3) return fail(IDW_EINVAL, "dim must be 2 or 3 (got %d)", dim);
  if (!known_precision(precision))
    return fail(IDW_EINVAL, "unknown precision %d", precision);
  const size_t e = elem(precision);
  switch (layout) {
    case IDW_SOA:
      for (int k = 0; k < dim; ++k) b[k] = e;
      if (is_data) b[dim] = e;
      break;
    case IDW_AOS:
      b[0] = e * (dim + (is_data ? 1 : 0));
      break;
    case IDW_AOAS:
      b[0] = 4 * e;
      break;
    case IDW_HYBRID:
      b[0] = e * dim;
      if (is_data) b[1] = e;
      break;
    case IDW_SOAOS:
      b[0] = e * (dim == 2 ? 2 : 4);
      if (is_data) b[1] = 2 * e;
      break;
    default:
      return fail(IDW_EINVAL, "unknown layout %d", layout);
  }
  return IDW_OK;
}

// Required alignment of slot k: the record size for the aligned layouts, else the element.
static size_t slot_align(int layout, int precision, const size_t b[4], int k) {
  if (layout == IDW_AOAS || layout == IDW_SOAOS) return b[k];
  return elem(precision);
}

int validate_points(const idw_points* P, int precision, bool is_data, const char* what) {
  if (!P) return fail(IDW_EINVAL, "%s: null descriptor", what);
  if (P->n < 0) return fail(IDW_EINVAL, "%s: negative count", what);
  if (is_data && P->n < 1) return fail(IDW_EINVAL, "%s: at least one data point is required", what);
  if (P->n > 0x7fffffffLL) return fail(IDW_EINVAL, "%s: count above 2^31-1", what);
  size_t b[4];
  int rc = record_bytes(P->layout, P->dim, precision, is_data, b);
  if (rc != IDW_OK) {
    std::string m = g_err;
    return fail(rc, "%s: %s", what, m.c_str());
  }
  if (P->n == 0) return IDW_OK;
  for (int k = 0; k < 4; ++k) {
    if (!b[k]) continue;
    if (!P->ptr[k]) return fail(IDW_EINVAL, "%s: pointer slot %d is null", what, k);
    const size_t al = slot_align(P->layout, precision, b, k);
    if (reinterpret_cast<uintptr_t>(P->ptr[k]) % al)
      return fail(IDW_EINVAL, "%s: pointer slot %d is not %zu-byte aligned", what, k, al);
  }
  return IDW_OK;
}

static bool same_query_layout(int a, int b) {
  auto canon = [](int l) { return l == IDW_HYBRID ? IDW_AOS : l; };
  return canon(a) == canon(b);
}

int validate_config(const idw_config* cfg) {
  if (!cfg) return IDW_OK;
  for (int k = 0; k < 2; ++k)
    if (cfg->reserved[k] != 0) return fail(IDW_EINVAL, "idw_config.reserved[%d] must be zero", k);
  if (cfg->queries_per_lane < 0 || cfg->split < 0 || cfg->batch_chunk < 0 || cfg->batch_workgroups < 0)
    return fail(IDW_EINVAL, "idw_config fields must not be negative");
  if (cfg->separate_adjoint != 0 && cfg->separate_adjoint != 1)
    return fail(IDW_EINVAL, "idw_config.separate_adjoint must be 0 or 1");
  if (cfg->near_search != 0 && cfg->near_search != 1)
    return fail(IDW_EINVAL, "idw_config.near_search must be 0 or 1");
  return IDW_OK;
}

int validate_common(const idw_points* data, const idw_points* query, double p, int precision,
                    uint32_t flags) {
  if (!known_precision(precision))
    return fail(IDW_EINVAL, "unknown precision %d", precision);
  int rc = validate_points(data, precision, true, "data");
  if (rc) return rc;
  rc = validate_points(query, precision, false, "query");
  if (rc) return rc;
  if (data->dim != query->dim) return fail(IDW_EINVAL, "data and query dims differ");
  if (!same_query_layout(data->layout, query->layout))
    return fail(IDW_EUNSUPPORTED, "query layout must match the data layout (AoS and hybrid "
                                  "query records are the same)");
  if (!(p > 0.0) || !(p <= 64.0)) return fail(IDW_EINVAL, "p must satisfy 0 < p <= 64");
  if (flags & ~(IDW_EXCLUDE_SELF | IDW_NEED_DZ | IDW_NEED_DP | IDW_NEED_DQ | IDW_NEED_DX))
    return fail(IDW_EINVAL, "unknown flag bits 0x%x", flags);
  if ((flags & IDW_EXCLUDE_SELF) && query->n != data->n)
    return fail(IDW_EINVAL, "IDW_EXCLUDE_SELF needs as many queries as data points");
  return IDW_OK;
}

int pmode_of(double p) {
  if (p == 1.0) return PM_1;
  if (p == 2.0) return PM_2;
  if (p == 3.0) return PM_3;
  if (p == 4.0) return PM_4;
  if (p == 2.5) return PM_25;
  return PM_GEN;
}

// ---- launch configuration and workspace layout ----
static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static size_t al256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Partial sums of the split sweeps are kept within this many bytes per array (the chunk
// count is capped by it); the fused adjoint's two partial arrays likewise.
constexpr int64_t kPartBudget = int64_t(1) << 31;

// Splits `len` points into chunks (multiples of the tile) so that `blocks` x chunks is about
// 16384 workgroups, at least 4 tiles per chunk (1 where 4 would leave fewer than 2048
// workgroups) and at most kPartBudget bytes of partials (`unit` bytes per chunk and element
// of the other set, `other` elements).  Every workgroup does the same work, and a grid of
// 1024 workgroups (one per 1024-query block at 1M queries) on the 768 that are resident at
// once loses about 7% to the last, partly empty round; with 16 times as many the loss is
// below 1% (1M x 1M forward: 204.1 -> 189.2 ms).  Below a few tens of thousands of queries
// even 4-tile chunks leave most of the chip idle (10,240^2 forward call, FP64: 166 us with 5
// chunks, 102 us with 20; 32,768^2 FP32: 268 -> 250 us), while from 65,536^2 on the longer
// merge of finer splits outweighs the fuller grid (65,536^2: 789 us with 32 chunks, 803
// with 128), so the smaller minimum applies only to the small grids.
static void choose_split(int64_t len, int64_t blocks, int want_split, int64_t unit, int64_t other, int& split,
                         int64_t& chunk) {
  int64_t s = want_split;
  if (s <= 0) {
    const int64_t target = 16384;
    const int64_t b = blocks > 0 ? blocks : 1;
    s = cdiv(target, b);
    const int64_t s4 = cdiv(len, 4 * kTile);
    s = std::min<int64_t>(s, b * s4 < 2048 ? cdiv(len, kTile) : s4);
    s = std::min<int64_t>(s, std::max<int64_t>(1, kPartBudget / (unit * std::max<int64_t>(other, 1))));
  }
  if (s < 1) s = 1;
  if (s > 1024) s = 1024;
  chunk = cdiv(cdiv(len, s), kTile) * kTile;
  split = static_cast<int>(cdiv(len, chunk));
}

WsPlan plan_workspace(const idw_points* data, const idw_points* query, int precision,
                      const idw_config* cfg) {
  WsPlan w;
  const bool f64 = precision == IDW_FP64;
  const int64_t n = data->n, m = query->n;
  // forward
  w.qf = (cfg && cfg->queries_per_lane) ? cfg->queries_per_lane : 4;
  choose_split(n, cdiv(m, kWG * w.qf), cfg ? cfg->split : 0, sizeof(double2), m, w.split_f, w.chunk_f);
  // backward: query sweep over data chunks, data sweep over query chunks
  w.qq = 2;
  choose_split(n, cdiv(m, kWG * w.qq), 0, sizeof(double4), m, w.split_q, w.chunk_q);
  w.qz = f64 ? 2 : 4;
  choose_split(m > 0 ? m : 1, cdiv(n, kWG * w.qz), 0, sizeof(double), n, w.split_z, w.chunk_z);
  // fused adjoint: workgroup (group, range) sweeps data range `range` for the query blocks
  // group, group + G, ...: about 8192 workgroups in all (of 512 threads in FP32, 256 in
  // FP64), for the reason given at choose_split (1M x 1M: 377.3 ms with 1024, 353.4 with
  // 8192).  Ranges of at most 32K points (at least one tile) and as many groups as the
  // query blocks allow, within kPartBudget for the dz rows (groups x n doubles) and for
  // the query partials (ranges x m double4): 2 GB and 1 GB at n = m = 1M.
  if (m > 0) {
    const int64_t target = 8192;
    const int64_t nqb = cdiv(m, f64 ? 256 * 2 : 512 * 2);
    int64_t r = std::max<int64_t>(cdiv(n, 32768), cdiv(target, nqb));
    r = std::min<int64_t>(r, std::min<int64_t>(cdiv(n, kTile), std::max<int64_t>(1, kPartBudget / (32 * m))));
    r = std::min<int64_t>(r, 32768);  // grid y dimension
    r = std::max<int64_t>(r, 1);
    w.fused_chunk = cdiv(cdiv(n, r), kTile) * kTile;
    w.fused_ranges = static_cast<int>(cdiv(n, w.fused_chunk));
    const int64_t gcap = std::min<int64_t>(nqb, std::max<int64_t>(1, kPartBudget / (8 * n)));
    w.fused_groups = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(gcap, cdiv(target, w.fused_ranges))));
  }
  w.nbbox = static_cast<int>(std::min<int64_t>(1024, cdiv(n, kWG)));
  w.nwg_dp = static_cast<int>(cdiv(m, kWG));
  const int64_t nb = cdiv(m > 0 ? m : 1, kCountBlock);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = al256(off + bytes);
    return at;
  };
  w.hdr = take(512);
  w.bbox = take(sizeof(double) * kBboxStride * static_cast<size_t>(w.nbbox));
  w.flag = take(static_cast<size_t>(m));
  w.bcnt = take(sizeof(int) * static_cast<size_t>(nb + 1));
  w.list = take(sizeof(int) * static_cast<size_t>(m));
  w.near_min = take(sizeof(unsigned long long) * static_cast<size_t>(m));
  w.part_f = take(w.split_f > 1 ? sizeof(double2) * static_cast<size_t>(w.split_f) * m : 0);
  w.fpart = take(sizeof(double4) * kFixGrid);
  w.fix_cmax = static_cast<int>(std::min<int64_t>(kFixGrid, std::max<int64_t>(1, cdiv(n, 4096))));
  // grid of the nearest-distance searches
  w.grid_on = n >= kGridMinN && n <= kGridMaxN && m > 0 && !(cfg && cfg->near_search == 1);
  if (w.grid_on) {
    w.grid_ncell = std::min<int64_t>(kGridMaxCells, std::max<int64_t>(1, n / kGridPerCell));
    const int64_t nb = cdiv(w.grid_ncell, kGridScanBlock);
    w.grid_cnt = take(sizeof(int) * static_cast<size_t>(w.grid_ncell + 1));
    w.grid_start = take(sizeof(int) * static_cast<size_t>(w.grid_ncell + 1));
    w.grid_bsum = take(sizeof(int) * static_cast<size_t>(nb + 1));
    w.grid_rec = take(4 * (f64 ? sizeof(double) : sizeof(float)) * static_cast<size_t>(n));
    w.grid_blist = take(sizeof(int) * static_cast<size_t>(m));
  }
  w.fwd_total = off;  // the forward uses only the sections above
  w.part_q = take(sizeof(double4) * static_cast<size_t>(std::max(w.split_q, w.fused_ranges)) * m);
  w.part_z = take(sizeof(double) * static_cast<size_t>(std::max(w.split_z, w.fused_groups)) * n);
  w.slot_coef = take(sizeof(double) * static_cast<size_t>(m));
  w.slot_hits = take(sizeof(int) * static_cast<size_t>(m));
  w.slot_dp = take(sizeof(double) * static_cast<size_t>(m));
  w.slot_z = take(sizeof(double) * static_cast<size_t>(m));
  w.slot_den = take(sizeof(double) * static_cast<size_t>(m));
  w.wg_dp = take(sizeof(double) * static_cast<size_t>(w.nwg_dp > 0 ? w.nwg_dp : 1));
  w.total = off;
  w.part_x = take(sizeof(double) * static_cast<size_t>(std::max(w.split_z, w.fused_groups)) * n *
                  static_cast<size_t>(data->dim));
  w.total_x = off;
  return w;
}

// ---- per-layout dispatch tables ----
struct LayoutFns {
  hipError_t (*fwd_sweep)(const FwdArgs&, bool, hipStream_t);
  hipError_t (*fwd_fixup)(const FwdArgs&, bool, hipStream_t);
  hipError_t (*bbox)(const DevPts&, int64_t, int, bool, double*, int, hipStream_t);
  hipError_t (*bwd_query)(const BwdArgs&, bool, hipStream_t);
  hipError_t (*bwd_data)(const BwdArgs&, bool, hipStream_t);
  hipError_t (*bwd_datax)(const BwdArgs&, bool, hipStream_t);
  hipError_t (*bwd_fixup)(const BwdArgs&, bool, hipStream_t);
  hipError_t (*bwd_fused)(const BwdArgs&, bool, hipStream_t);
  hipError_t (*near_check)(const NearArgs&, hipStream_t);
  hipError_t (*grid)(const GridArgs&, bool, hipStream_t);
};

#define IDW_FNS(NAME)                                                                   \
  {fwd_sweep_##NAME, fwd_fixup_##NAME, bbox_##NAME,      bwd_query_##NAME, bwd_data_##NAME, \
   bwd_datax_##NAME, bwd_fixup_##NAME, bwd_fused_##NAME, near_check_##NAME, grid_##NAME}
static const LayoutFns kFns[5] = {IDW_FNS(soa), IDW_FNS(aos), IDW_FNS(aoas), IDW_FNS(hybrid), IDW_FNS(soaos)};
#undef IDW_FNS

const LayoutFns& fns(int layout) { return kFns[layout]; }

DevPts dev_pts(const idw_points* P) {
  DevPts d;
  for (int k = 0; k < 4; ++k) d.p[k] = P->ptr[k];
  return d;
}

// ---- static scratch of idw_forward_noalloc ----
// The forward's workspace for callers that cannot allocate: one array per device, held by
// the loaded code object until the process ends.  Host code never passes `scratch` itself
// (on the host it is only a stand-in for the device symbol): the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static int scratch_address(void** out) {
  static std::mutex mu;
  static void* addr[64] = {nullptr};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(IDW_EDEVICE, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(IDW_EDEVICE, "scratch address on device %d: %s", dev, hipGetErrorString(e));
    addr[dev] = ptr;
  }
  *out = addr[dev];
  return IDW_OK;
}

int check_workspace(void* ws, size_t bytes, size_t need) {
  if (!ws) return fail(IDW_EWORKSPACE, "workspace is null");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(IDW_EWORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < need) return fail(IDW_EWORKSPACE, "workspace too small: %zu < %zu bytes", bytes, need);
  return IDW_OK;
}

// Enqueues the extent/threshold header computation (rel: thresholds of the relative-weight
// FP32 sweeps).
hipError_t enqueue_header(const idw_points* data, double p, bool f64, bool rel, char* ws, const WsPlan& w,
                          hipStream_t st) {
  hipError_t e = fns(data->layout).bbox(dev_pts(data), data->n, data->dim, f64,
                                        reinterpret_cast<double*>(ws + w.bbox), w.nbbox, st);
  if (e != hipSuccess) return e;
  return bbox_final(reinterpret_cast<double*>(ws + w.bbox), w.nbbox, data->dim, p, !f64, rel,
                    reinterpret_cast<double*>(ws + w.hdr), st);
}

static GridArgs grid_args(const idw_points* data, const idw_points* query, bool f64, bool excl, char* ws,
                          const WsPlan& w) {
  GridArgs g;
  g.data = dev_pts(data);
  g.n = data->n;
  g.query = dev_pts(query);
  g.m = query->n;
  g.dim = data->dim;
  g.f64 = f64;
  g.excl = excl;
  g.hdr = reinterpret_cast<const double*>(ws + w.hdr);
  g.hint = reinterpret_cast<int*>(ws + w.hdr + 256);
  g.cnt = reinterpret_cast<int*>(ws + w.grid_cnt);
  g.start = reinterpret_cast<int*>(ws + w.grid_start);
  g.bsum = reinterpret_cast<int*>(ws + w.grid_bsum);
  g.ncell_max = w.grid_ncell;
  g.rec = ws + w.grid_rec;
  g.route = reinterpret_cast<uint8_t*>(ws + w.flag);
  g.minb = reinterpret_cast<unsigned long long*>(ws + w.near_min);
  g.blist = reinterpret_cast<int*>(ws + w.grid_blist);
  return g;
}

// Builds the grid when its gate (set by grid_setup) is open: counts, scan, scatter.
static hipError_t grid_build(const LayoutFns& F, const GridArgs& g, hipStream_t st) {
  hipError_t e = fill_zero(g.cnt, sizeof(int) * static_cast<size_t>(g.ncell_max + 1), st);
  if (e != hipSuccess) return e;
  return F.grid(g, true, st);
}

static NearArgs near_args(const idw_points* data, const idw_points* query, bool f64, bool excl, char* ws,
                          const WsPlan& w) {
  NearArgs na;
  na.data = dev_pts(data);
  na.n = data->n;
  na.query = dev_pts(query);
  na.m = query->n;
  na.dim = data->dim;
  na.f64 = f64;
  na.excl = excl;
  na.hdr = reinterpret_cast<const double*>(ws + w.hdr);
  na.route = reinterpret_cast<uint8_t*>(ws + w.flag);
  na.minb = reinterpret_cast<unsigned long long*>(ws + w.near_min);
  return na;
}

// Nearest squared distance of every query (FP32 bits, scaled units) into the near_min
// section: the relative-weight forward sweep takes each query's sigma from it.  With the
// grid: a ring search per query, and the brute-force kernels for the queries it hands
// back; without it: the brute-force kernels over all queries.
static hipError_t nearest_all(const LayoutFns& F, const idw_points* data, const idw_points* query, bool excl,
                              char* ws, const WsPlan& w, hipStream_t st) {
  NearArgs na = near_args(data, query, false, excl, ws, w);
  if (!w.grid_on) {
    na.all = true;
    return F.near_check(na, st);
  }
  GridArgs g = grid_args(data, query, false, excl, ws, w);
  g.nearest = true;
  g.hint += kGridNearestSlots;  // its own gate and counters: the candidate check comes later
  hipError_t e = grid_setup(g, 1, true, st);
  if (e == hipSuccess) e = grid_build(F, g, st);
  if (e == hipSuccess) e = F.grid(g, false, st);
  if (e != hipSuccess) return e;
  na.list = g.blist;  // the queries the ring search handed back
  na.count = g.hint + GI_FALLBACK;
  return F.near_check(na, st);
}

// Settles the route of every query after a sweep (or from the saved denominators): the
// candidates are compacted and checked for a data point within 1e-6 of the extent, then the
// queries routed to FP64 are compacted into the list the fix-ups read.
static hipError_t settle_routes(const LayoutFns& F, const idw_points* data, const idw_points* query,
                                bool f64, bool excl, char* ws, const WsPlan& w, hipStream_t st) {
  uint8_t* route = reinterpret_cast<uint8_t*>(ws + w.flag);
  int* bcnt = reinterpret_cast<int*>(ws + w.bcnt);
  int* list = reinterpret_cast<int*>(ws + w.list);
  int* count = reinterpret_cast<int*>(ws + w.hdr + 256);
  const int64_t m = query->n;
  hipError_t e = compact_flags(route, m, bcnt, list, count, F_CANDIDATE, st);
  if (e != hipSuccess) return e;
  NearArgs na = near_args(data, query, f64, excl, ws, w);
  na.list = list;
  na.count = count;
  if (w.grid_on) {
    // Many candidates: the grid's fixed-radius check, then the brute-force kernels for the
    // candidates it hands back; few: the brute-force kernels for all of them.
    GridArgs g = grid_args(data, query, f64, excl, ws, w);
    g.list = list;
    if ((e = grid_setup(g, 0, true, st)) != hipSuccess) return e;
    na.count = g.hint + GI_BRUTE;
    if ((e = F.near_check(na, st)) != hipSuccess) return e;
    if ((e = grid_build(F, g, st)) != hipSuccess) return e;
    if ((e = F.grid(g, false, st)) != hipSuccess) return e;
    na.list = g.blist;
    na.count = g.hint + GI_FALLBACK;
  }
  if ((e = F.near_check(na, st)) != hipSuccess) return e;
  return compact_flags(route, m, bcnt, list, count, F_FP64, st);
}

// ---- optional event timing of the sweep kernels ----
struct TimingRec {
  int which;
  hipEvent_t a, b;
};
static std::mutex g_tmu;
static bool g_timing = false;
static std::vector<TimingRec> g_pending;
static double g_tot_ms[IDW_T_COUNT];
static int64_t g_launches[IDW_T_COUNT];

template <typename F>
hipError_t timed(int which, hipStream_t st, F&& launch) {
  {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!g_timing) return launch();
  }
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = hipEventRecord(a, st);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, st);
  if (e != hipSuccess) {  // nothing is queued on the events: release them
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    return e;
  }
  std::lock_guard<std::mutex> lk(g_tmu);
  g_pending.push_back({which, a, b});
  return hipSuccess;
}

static int drain_timing(bool accumulate) {
  int rc = IDW_OK;
  for (auto& r : g_pending) {
    if (accumulate && rc == IDW_OK) {
      float ms = 0.f;
      if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
        rc = fail(IDW_EDEVICE, "event timing failed");
      g_tot_ms[r.which] += ms;
      g_launches[r.which] += 1;
    } else {
      (void)hipEventSynchronize(r.b);
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_pending.clear();
  return rc;
}

}  // namespace idw

using namespace idw;

extern "C" {

const char* idw_version(void) { return "idw-gfx950 0.1.0"; }

int idw_timing_enable(int32_t on) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_tmu);
  drain_timing(false);
  for (int k = 0; k < IDW_T_COUNT; ++k) {
    g_tot_ms[k] = 0.0;
    g_launches[k] = 0;
  }
  g_timing = on != 0;
  return IDW_OK;
}

int idw_timing_read(int32_t which, double* total_ms, int64_t* launches) {
  clear_error();
  if (which < 0 || which >= IDW_T_COUNT) return fail(IDW_EINVAL, "unknown timer %d", which);
  std::lock_guard<std::mutex> lk(g_tmu);
  const int rc = drain_timing(true);
  if (total_ms) *total_ms = g_tot_ms[which];
  if (launches) *launches = g_launches[which];
  return rc;
}

const char* idw_last_error(void) { return g_err.c_str(); }

int idw_record_bytes(int32_t layout, int32_t dim, int32_t precision, int32_t is_data,
                     size_t bytes[4]) {
  clear_error();
  if (!bytes) return fail(IDW_EINVAL, "bytes is null");
  return record_bytes(layout, dim, precision, is_data != 0, bytes);
}

int idw_workspace_size(const idw_points* data, const idw_points* query, int32_t precision,
                       uint32_t flags, const idw_config* cfg, size_t* bytes) {
  clear_error();
  if (!bytes) return fail(IDW_EINVAL, "bytes is null");
  int rc = validate_common(data, query, 2.0, precision, flags & ~IDW_EXCLUDE_SELF);
  if (rc) return rc;
  if ((rc = validate_config(cfg))) return rc;
  const WsPlan w = plan_workspace(data, query, precision, cfg);
  *bytes = (flags & IDW_NEED_DX) ? w.total_x
           : (flags & (IDW_NEED_DZ | IDW_NEED_DP | IDW_NEED_DQ)) ? w.total
                                                                 : w.fwd_total;
  return IDW_OK;
}

// The forward's checks and launches on a caller workspace (idw_forward) or on the
// library's static scratch (idw_forward_noalloc).
static int forward_impl(const idw_points* data, const idw_points* query, double p, int32_t precision,
                        uint32_t flags, void* out_z, double* out_den, void* workspace,
                        size_t workspace_bytes, void* stream, const idw_config* cfg, bool static_scratch) {
  int rc = validate_common(data, query, p, precision, flags);
  if (rc) return rc;
  if ((rc = validate_config(cfg))) return rc;
  if (flags & ~IDW_EXCLUDE_SELF) return fail(IDW_EINVAL, "idw_forward accepts only IDW_EXCLUDE_SELF");
  if (cfg && cfg->queries_per_lane) {
    const int q = cfg->queries_per_lane;
    const bool ok = precision == IDW_FP64         ? (q == 2 || q == 4)
                    : precision == IDW_FP32_KAHAN ? q == 4
                    : p >= kRelP                  ? (q == 4 || q == 8)
                                                  : (q == 2 || q == 4 || q == 8);
    if (!ok) return fail(IDW_EUNSUPPORTED, "queries_per_lane %d not built for this precision and p", q);
  }
  if (cfg && (cfg->split < 0 || cfg->split > 1024)) return fail(IDW_EINVAL, "split must be in 0..1024");
  const int64_t m = query->n;
  if (m == 0) return IDW_OK;
  if (!out_z) return fail(IDW_EINVAL, "out_z is null");
  WsPlan w = plan_workspace(data, query, precision, cfg);
  if (static_scratch) {
    // Where the default data split's partial sums do not fit the scratch, take the largest
    // split that does (the same result as idw_forward with that split in cfg).
    if (w.fwd_total > kScratchBytes && !(cfg && cfg->split) && w.split_f > 1) {
      idw_config c{};
      if (cfg) c = *cfg;
      for (c.split = w.split_f - 1; c.split >= 1; --c.split) {
        w = plan_workspace(data, query, precision, &c);
        if (w.fwd_total <= kScratchBytes) break;
      }
    }
    if (w.fwd_total > kScratchBytes)
      return fail(IDW_EWORKSPACE, "idw_forward_noalloc: these sizes need %zu bytes of scratch, above its %zu",
                  w.fwd_total, kScratchBytes);
    rc = check_device();
    if (rc) return rc;
    if ((rc = scratch_address(&workspace))) return rc;
    workspace_bytes = kScratchBytes;
  }
  rc = check_workspace(workspace, workspace_bytes, w.fwd_total);
  if (rc) return rc;
  rc = check_device();
  if (rc) return rc;
  const bool f64 = precision == IDW_FP64;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);

  FwdArgs a;
  a.data = dev_pts(data);
  a.n = data->n;
  a.query = dev_pts(query);
  a.m = m;
  a.dim = data->dim;
  a.pmode = pmode_of(p);
  a.p = p;
  a.flags = flags;
  a.kahan = precision == IDW_FP32_KAHAN;
  // Queries per lane: 2 for the FP32 sweeps whose weight takes at most one transcendental
  // (p = 1, 2, 3, 4) and for every FP64 sweep (general p 1036 -> 957 ms at 1M x 1M; the
  // others within 1.2%), 4 otherwise (the plan's default, which also sets the data split).
  a.q_per_lane = w.qf;
  if (!(cfg && cfg->queries_per_lane) &&
      (f64 || (precision == IDW_FP32 && p < kRelP &&
               (a.pmode == PM_1 || a.pmode == PM_2 || a.pmode == PM_3 || a.pmode == PM_4))))
    a.q_per_lane = 2;
  // Large p in FP32: relative weights, sigma from each query's nearest distance.
  a.rel = !f64 && p >= kRelP;
  a.rmin = reinterpret_cast<const unsigned long long*>(ws + w.near_min);
  a.split = w.split_f;
  a.chunk = w.chunk_f;
  a.hdr = reinterpret_cast<const double*>(ws + w.hdr);
  a.out_z = out_z;
  a.out_den = out_den;
  a.flag = reinterpret_cast<uint8_t*>(ws + w.flag);
  a.part = reinterpret_cast<double2*>(ws + w.part_f);
  a.list = reinterpret_cast<const int*>(ws + w.list);
  a.count = reinterpret_cast<const int*>(ws + w.hdr + 256);
  a.fix_cmax = w.fix_cmax;
  a.fpart = reinterpret_cast<double4*>(ws + w.fpart);

  const LayoutFns& F = fns(data->layout);
  const bool excl = (flags & IDW_EXCLUDE_SELF) != 0;
  if ((rc = check_hip(enqueue_header(data, p, f64, a.rel, ws, w, st), "extent kernels"))) return rc;
  if (a.rel && (rc = check_hip(nearest_all(F, data, query, excl, ws, w, st), "nearest-distance pass")))
    return rc;
  if ((rc = check_hip(timed(IDW_T_FWD_SWEEP, st, [&] { return F.fwd_sweep(a, f64, st); }), "forward sweep")))
    return rc;
  if (a.split > 1 &&
      (rc = check_hip(merge_split(a.part, m, a.split, a.hdr, out_z, f64, out_den, a.flag, st), "merge")))
    return rc;
  if ((rc = check_hip(settle_routes(F, data, query, f64, excl, ws, w, st), "near-coincidence check")))
    return rc;
  if ((rc = check_hip(F.fwd_fixup(a, f64, st), "FP64 fix-up"))) return rc;
  return IDW_OK;
}

int idw_forward(const idw_points* data, const idw_points* query, double p, int32_t precision,
                uint32_t flags, void* out_z, double* out_den, void* workspace,
                size_t workspace_bytes, void* stream, const idw_config* cfg) {
  clear_error();
  return forward_impl(data, query, p, precision, flags, out_z, out_den, workspace, workspace_bytes, stream, cfg,
                      false);
}

int idw_forward_noalloc(const idw_points* data, const idw_points* query, double p, int32_t precision,
                        uint32_t flags, void* out_z, double* out_den, void* stream, const idw_config* cfg) {
  clear_error();
  return forward_impl(data, query, p, precision, flags, out_z, out_den, nullptr, 0, stream, cfg, true);
}

int idw_backward(const idw_points* data, const idw_points* query, double p, int32_t precision,
                 uint32_t flags, const void* grad_out, const void* saved_z,
                 const double* saved_den, void* grad_z, double* grad_p, void* grad_q,
                 void* grad_x, void* workspace, size_t workspace_bytes, void* stream,
                 const idw_config* cfg) {
  clear_error();
  int rc = validate_common(data, query, p, precision, flags);
  if (rc) return rc;
  if ((rc = validate_config(cfg))) return rc;
  const bool ndz = flags & IDW_NEED_DZ, ndp = flags & IDW_NEED_DP, ndq = flags & IDW_NEED_DQ;
  const bool ndx = flags & IDW_NEED_DX;
  if (!(ndz || ndp || ndq || ndx)) return fail(IDW_EINVAL, "no gradient requested (IDW_NEED_* flags)");
  if (ndz && !grad_z) return fail(IDW_EINVAL, "IDW_NEED_DZ set but grad_z is null");
  if (ndp && !grad_p) return fail(IDW_EINVAL, "IDW_NEED_DP set but grad_p is null");
  if (ndq && !grad_q && query->n > 0) return fail(IDW_EINVAL, "IDW_NEED_DQ set but grad_q is null");
  if (ndx && !grad_x) return fail(IDW_EINVAL, "IDW_NEED_DX set but grad_x is null");
  const int64_t m = query->n;
  if (m > 0 && (!grad_out || !saved_z || !saved_den))
    return fail(IDW_EINVAL, "grad_out, saved_z and saved_den are required");
  const WsPlan w = plan_workspace(data, query, precision, cfg);
  rc = check_workspace(workspace, workspace_bytes, ndx ? w.total_x : w.total);
  if (rc) return rc;
  rc = check_device();
  if (rc) return rc;
  const bool f64 = precision == IDW_FP64;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  if (m == 0) {  // no queries: every gradient is zero
    if (ndz && (rc = check_hip(fill_zero(grad_z, static_cast<size_t>(data->n) * elem(precision), st), "fill")))
      return rc;
    if (ndx && (rc = check_hip(fill_zero(grad_x, static_cast<size_t>(data->n) * data->dim * elem(precision), st),
                               "fill")))
      return rc;
    if (ndp && (rc = check_hip(fill_zero(grad_p, sizeof(double), st), "fill"))) return rc;
    return IDW_OK;
  }

  BwdArgs a;
  a.data = dev_pts(data);
  a.n = data->n;
  a.query = dev_pts(query);
  a.m = m;
  a.dim = data->dim;
  a.pmode = pmode_of(p);
  a.p = p;
  a.flags = flags & (IDW_EXCLUDE_SELF | (ndp ? IDW_NEED_DP : 0u) | (ndq ? IDW_NEED_DQ : 0u));
  a.q_per_lane = w.qq;
  a.x_per_lane = w.qz;
  a.split_q = w.split_q;
  a.chunk_q = w.chunk_q;
  a.split_z = w.split_z;
  a.chunk_z = w.chunk_z;
  a.part_q = reinterpret_cast<double4*>(ws + w.part_q);
  a.part_z = reinterpret_cast<double*>(ws + w.part_z);
  a.hdr = reinterpret_cast<const double*>(ws + w.hdr);
  a.grad_out = grad_out;
  a.saved_z = saved_z;
  a.saved_den = saved_den;
  a.grad_z = ndz ? grad_z : nullptr;
  a.grad_q = ndq ? grad_q : nullptr;
  a.grad_x = ndx ? grad_x : nullptr;
  a.part_x = ndx ? reinterpret_cast<double*>(ws + w.part_x) : nullptr;
  a.wg_dp = ndp ? reinterpret_cast<double*>(ws + w.wg_dp) : nullptr;
  a.list = reinterpret_cast<const int*>(ws + w.list);
  a.count = reinterpret_cast<const int*>(ws + w.hdr + 256);
  a.slot_coef = reinterpret_cast<double*>(ws + w.slot_coef);
  a.slot_hits = reinterpret_cast<int*>(ws + w.slot_hits);
  a.slot_dp = reinterpret_cast<double*>(ws + w.slot_dp);
  a.slot_z = reinterpret_cast<double*>(ws + w.slot_z);
  a.slot_den = reinterpret_cast<double*>(ws + w.slot_den);
  a.fix_cmax = w.fix_cmax;
  a.fpart = reinterpret_cast<double4*>(ws + w.fpart);

  const LayoutFns& F = fns(data->layout);
  uint8_t* flag = reinterpret_cast<uint8_t*>(ws + w.flag);
  // Large p in FP32: the fused sweep with relative weights serves every request (the
  // separate sweeps, when asked for, keep the direct weights and their FP64 routing).
  const bool separate = cfg && cfg->separate_adjoint;
  const bool rel = !f64 && p >= kRelP && !separate && w.fused_groups > 0;
  a.rel = rel;
  if ((rc = check_hip(enqueue_header(data, p, f64, rel, ws, w, st), "extent kernels"))) return rc;
  if ((rc = check_hip(flags_from_den(saved_den, m, a.hdr, flag, st), "flags"))) return rc;
  if ((rc = check_hip(settle_routes(F, data, query, f64, (flags & IDW_EXCLUDE_SELF) != 0, ws, w, st),
                      "near-coincidence check")))
    return rc;
  a.route = flag;
  // The fused sweep pays off when both directions are needed: dz with dp or dq, or dx
  // (alone or with the others: its per-pair factors are those of dq).
  const bool fused = rel || (w.fused_groups > 0 && !separate && (ndx || (ndz && (ndp || ndq))));
  if (fused) {  // one sweep for dp/dq and dz (and dx)
    a.fused_groups = w.fused_groups;
    a.fused_ranges = w.fused_ranges;
    a.fused_chunk = w.fused_chunk;
    if ((rc = check_hip(timed(IDW_T_BWD_FUSED, st, [&] { return F.bwd_fused(a, f64, st); }), "fused adjoint sweep")))
      return rc;
    BwdArgs b = a;
    b.split_q = w.fused_ranges;
    b.split_z = w.fused_groups;
    if ((ndp || ndq) && (rc = check_hip(bwd_qmerge(b, f64, st), "query merge"))) return rc;
    if (ndz && (rc = check_hip(bwd_zmerge(b, f64, st), "data merge"))) return rc;
    if (ndx && (rc = check_hip(bwd_xmerge(b, w.fused_groups, f64, st), "data-coordinate merge"))) return rc;
  } else {
    if (ndp || ndq) {
      if ((rc = check_hip(timed(IDW_T_BWD_QUERY, st, [&] { return F.bwd_query(a, f64, st); }), "query sweep")))
        return rc;
      if ((rc = check_hip(bwd_qmerge(a, f64, st), "query merge"))) return rc;
    }
    if (ndx) {  // one data-direction sweep yields dz and dx
      if ((rc = check_hip(timed(IDW_T_BWD_DATA, st, [&] { return F.bwd_datax(a, f64, st); }), "data sweep")))
        return rc;
      if (ndz && (rc = check_hip(bwd_zmerge(a, f64, st), "data merge"))) return rc;
      if ((rc = check_hip(bwd_xmerge(a, w.split_z, f64, st), "data-coordinate merge"))) return rc;
    } else if (ndz) {
      if ((rc = check_hip(timed(IDW_T_BWD_DATA, st, [&] { return F.bwd_data(a, f64, st); }), "data sweep")))
        return rc;
      if ((rc = check_hip(bwd_zmerge(a, f64, st), "data merge"))) return rc;
    }
  }
  if ((rc = check_hip(F.bwd_fixup(a, f64, st), "FP64 fix-up"))) return rc;
  if (ndp && (rc = check_hip(dp_final(a.wg_dp, w.nwg_dp, a.slot_dp, a.count, grad_p, st), "dp reduction")))
    return rc;
  return IDW_OK;
}

}  // extern "C"
