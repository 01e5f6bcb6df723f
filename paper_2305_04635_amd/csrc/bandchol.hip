// Host runtime of the FP64 band Cholesky library for gfx950: argument checks,
// workspaces, the choice of schedule per matrix, and the C-ABI entry points
// declared in bandchol.h.
//
// The factor works on T x T tiles of the band.  Tile (R, C) covers rows
// [R*T, R*T+T) and columns [C*T, C*T+T); the band holds tiles with
// 0 <= R - C <= K, K = ceil(k / T).  In the paper's terms (Algorithm 1,
// Section 3) every diagonal tile is factored by dense Cholesky (potrf), every
// tile below it is solved against it (trsm), and every tile receives the
// rank-T updates L(R,s) L(C,s)^T of the earlier tile columns s (gemm/syrk).
// Two schedules replace the paper's OpenMP task graph (Section 3.1):
//   walk   (walk.hip)    one workgroup factors the whole band; used up to a
//                        settable number of tile diagonals, and for batches;
//   spine  (factor2.hip) one workgroup carries the diagonal chain while the
//                        others take the remaining tile tasks from a queue.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "bandchol.h"

#include "adjoint.h"
#include "common.h"
#include "factor_bwd.h"
#include "mixed.h"
#include "walk.h"

size_t bandchol_solve_workspace(int64_t n, int64_t k);
size_t bandchol_factor2_workspace(int64_t n, int64_t K);
size_t bandchol_factor2_workspace_f32(int64_t n, int64_t K);
hipError_t bandchol_factor2_launch_f32(int64_t n, int64_t k, float* ab, int64_t ldab, int64_t* d_info, void* ws,
                                       int grid_max, hipStream_t st);
hipError_t bandchol_factor2_launch(int64_t n, int64_t k, double* ab, int64_t ldab, int64_t* d_info, void* ws,
                                   int grid_max, hipStream_t st);
hipError_t bandchol_factor2_launch_profiled(int64_t n, int64_t k, double* ab, int64_t ldab, int64_t* d_info, void* ws,
                                            int grid_max, unsigned long long* prof, hipStream_t st);
hipError_t bandchol_solve_launch(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, double* b,
                                 int64_t ldb, void* ws, int num_cus, int64_t* d_status, hipStream_t st);

namespace {

using namespace bandchol;
using bandchol_walk::WalkSys;
using bandchol_walk::WALK_KMAX;

// ----------------------------------------------------------------- host runtime

thread_local char g_err[512] = "";

__global__ void set_info_kernel(int64_t* d_info, int64_t v) { *d_info = v; }
thread_local hipStream_t g_stream = nullptr;

void set_err(const char* what, hipError_t e) {
  snprintf(g_err, sizeof g_err, "%s: %s", what, hipGetErrorString(e));
}

struct DevWork {
  void* ptr = nullptr;
  size_t size = 0;
  void* info_host = nullptr;  // pinned int64 for the synchronous calls
  void* info_dev = nullptr;   // device int64 for the synchronous calls (never reallocated)
  void* mptr = nullptr;       // buffers of the mixed-precision solver (grown on demand)
  size_t msize = 0;
};
std::mutex g_mu;
std::vector<DevWork> g_work;

// Workspace of at least `bytes` on the current device (grown on demand).
void* workspace(size_t bytes, hipError_t* err) {
  int dev = 0;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_work.size() <= dev) g_work.resize(dev + 1);
  DevWork& w = g_work[dev];
  if (w.size < bytes) {
    if (w.ptr) {
      *err = hipDeviceSynchronize();
      if (*err != hipSuccess) return nullptr;
      *err = hipFree(w.ptr);
      w.ptr = nullptr;
      w.size = 0;
      if (*err != hipSuccess) return nullptr;
    }
    size_t want = bytes < (1u << 20) ? (1u << 20) : bytes + bytes / 4;
    *err = hipMalloc(&w.ptr, want);
    if (*err != hipSuccess) { w.ptr = nullptr; return nullptr; }
    w.size = want;
  }
  return w.ptr;
}

// Buffers of the mixed-precision solver on the current device (grown on demand;
// the caller synchronises before reusing them).
void* mixed_buffers(size_t bytes, hipError_t* err) {
  int dev = 0;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_work.size() <= dev) g_work.resize(dev + 1);
  DevWork& w = g_work[dev];
  if (w.msize < bytes) {
    if (w.mptr) {
      *err = hipDeviceSynchronize();
      if (*err == hipSuccess) *err = hipFree(w.mptr);
      w.mptr = nullptr;
      w.msize = 0;
      if (*err != hipSuccess) return nullptr;
    }
    *err = hipMalloc(&w.mptr, bytes);
    if (*err != hipSuccess) { w.mptr = nullptr; return nullptr; }
    w.msize = bytes;
  }
  return w.mptr;
}

// Host (pinned) and device int64 slots used by the synchronous factor call to
// return info.  They live apart from the workspace, which the launch may grow.
bool info_slots(int64_t** h, int64_t** d, hipError_t* err) {
  int dev = 0;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_work.size() <= dev) g_work.resize(dev + 1);
  DevWork& w = g_work[dev];
  if (!w.info_host) {
    *err = hipHostMalloc(&w.info_host, 64, hipHostMallocDefault);
    if (*err != hipSuccess) { w.info_host = nullptr; return false; }
  }
  if (!w.info_dev) {
    *err = hipMalloc(&w.info_dev, 256);
    if (*err != hipSuccess) { w.info_dev = nullptr; return false; }
  }
  *h = (int64_t*)w.info_host;
  *d = (int64_t*)w.info_dev;
  return true;
}

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Number of sub-diagonal tiles of the band (k clipped to n-1).
int tile_diagonals(int64_t n, int64_t k) {
  const int64_t kk = k < n - 1 ? k : (n > 0 ? n - 1 : 0);
  return (int)((kk + T - 1) / T);
}

int g_num_cus = 0;

int num_cus() {
  if (g_num_cus == 0) {
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      g_num_cus = cu;
    else
      g_num_cus = 256;
  }
  return g_num_cus;
}

// Largest sub-diagonal tile count handled by the single-workgroup walk.
int g_walk_kmax = -1;
int walk_kmax() {
  if (g_walk_kmax < 0) {
    g_walk_kmax = 0;   // the spine schedule is faster for a single matrix from K = 1 on
    if (const char* e = getenv("BANDCHOL_WALK_KMAX")) g_walk_kmax = (int)strtol(e, nullptr, 10);
    if (g_walk_kmax > WALK_KMAX) g_walk_kmax = WALK_KMAX;
  }
  return g_walk_kmax;
}

constexpr int64_t MIXED_ITMAX = 30;   // refinement corrections before the FP64 fallback

// ------------------------------------------------------- schedule per bucket
// The factor's schedule is a workgroup count: 1 = the single-workgroup walk,
// more = the spine schedule with that many workgroups.  The count is looked up
// per (floor(log2 n), K) bucket in a table filled by measurement
// (bandchol_tune_factor) or by the caller (bandchol_tune_set); buckets without
// an entry take the rule below.

// Workgroups of the spine schedule that are resident at once (two per CU).
int resident_wgs() { return num_cus() * 2; }

int n_bucket(int64_t n) {
  int b = 0;
  while (b < 62 && (n >> (b + 1)) > 0) ++b;
  return b;
}

// The rule for the spine: the helpers' work per tile column grows with K (the
// tiles of a column, K + 1, each updated by up to K earlier columns), while
// helpers beyond what the columns in flight can feed only contend with the
// spine for memory and matrix cores.  Counts that spread evenly over the CUs
// (a quarter, one or two workgroups per CU) measured better than those
// between them (n = 1e5, k = 1500: 27.7 ms with one per CU, 30.4 with 1.5).
// From K = 12 on the far tiles go in strips of four, which want one
// workgroup per CU (n = 1e5, k = 500, K = 16: 18.5 ms against 19.0 with a
// quarter).
int spine_rule(int K) {
  const int c = num_cus();
  int g = K < 12 ? c / 4 : K <= 55 ? c : 2 * c;
  return g < 2 ? 2 : g;
}

struct TuneEntry {
  int nb = 0, K = 0, wgs = 0;
  int64_t n = 0, k = 0;   // the system it was measured or set for
  double ms = 0.0;        // measured factor time (0 when set by the caller)
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

// Workgroups for the factor of a system with these sizes (before the cap):
// the walk up to the walk limit (by default diagonal matrices only), then the
// table, then the rule.
int schedule_wgs(int64_t n, int K) {
  if (K <= walk_kmax()) return 1;
  const int nb = n_bucket(n);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const TuneEntry& t : g_tune)
      if (t.nb == nb && t.K == K) return t.wgs;
  }
  return spine_rule(K);
}

// The batch table: the same buckets, for systems of a batch plan.  There the
// walk of one system runs beside the walks of all the others in one
// persistent launch, while a system given to the multi-workgroup schedule is
// factored on its own after it, so the best choice differs from that of a
// single matrix; it is kept apart.  Without an entry a batch walks every
// system the walk takes (K <= 15) and gives the others the single-matrix
// choice.
std::vector<TuneEntry> g_btune;

int batch_schedule_wgs(int64_t n, int K) {
  const int nb = n_bucket(n);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const TuneEntry& t : g_btune)
      if (t.nb == nb && t.K == K) return t.wgs;
  }
  if (K <= WALK_KMAX) return 1;
  const int w = schedule_wgs(n, K);
  return w == 1 ? spine_rule(K) : w;
}

void btune_record(int64_t n, int64_t kk, int K, int wgs, double ms) {
  const int nb = n_bucket(n);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (TuneEntry& t : g_btune)
    if (t.nb == nb && t.K == K) {
      t.wgs = wgs, t.n = n, t.k = kk, t.ms = ms;
      return;
    }
  TuneEntry t;
  t.nb = nb, t.K = K, t.wgs = wgs, t.n = n, t.k = kk, t.ms = ms;
  g_btune.push_back(t);
}

// Spine workgroup count after the BANDCHOL_MAX_WG cap (testing aid).
int spine_grid(int want) {
  int grid = want < 2 ? 2 : want;
  if (const char* cap = getenv("BANDCHOL_MAX_WG")) {
    const long v = strtol(cap, nullptr, 10);
    if (v > 0 && v < grid) grid = (int)v;
  }
  return grid;
}

int64_t factor_with(int64_t n, int64_t k, double* ab, int64_t ldab, int64_t* d_info, int wgs, hipStream_t st,
                    void* fixed_ws = nullptr, size_t fixed_size = 0);

// fixed_ws: when not NULL, the spine's working memory is taken from this
// buffer of fixed_size bytes instead of the library's workspace (nothing is
// allocated); a band whose working memory exceeds it is rejected.
int64_t factor_async_impl(int64_t n, int64_t k, double* ab, int64_t ldab, int64_t* d_info, hipStream_t st,
                          void* fixed_ws = nullptr, size_t fixed_size = 0) {
  if (n < 0) return -1;
  if (k < 0) return -2;
  if (ab == nullptr && n > 0) return -3;
  if (ldab < k + 1) return -4;
  if (d_info == nullptr) return -5;
  if (n > ((int64_t)1 << 31) - T) {
    snprintf(g_err, sizeof g_err, "n too large");
    return -1;
  }
  if (n == 0) {
    set_info_kernel<<<1, 1, 0, st>>>(d_info, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_err("factor", e); return BANDCHOL_EHIP; }
    return 0;
  }
  const int K = tile_diagonals(n, k);
  return factor_with(n, k, ab, ldab, d_info, schedule_wgs(n, K), st, fixed_ws, fixed_size);
}

// The factor with a given schedule (1 = walk, else spine workgroups).
int64_t factor_with(int64_t n, int64_t k, double* ab, int64_t ldab, int64_t* d_info, int wgs, hipStream_t st,
                    void* fixed_ws, size_t fixed_size) {
  hipError_t e;
  const int K = tile_diagonals(n, k);
  if (wgs == 1 && K <= WALK_KMAX) {
    const int64_t kk = k < n - 1 ? k : n - 1;
    e = bandchol_walk_single_launch(WalkSys{ab, n, kk, ldab, nullptr, nullptr, 0}, K, d_info, st);
    if (e != hipSuccess) { set_err("factor launch", e); return BANDCHOL_EHIP; }
    return 0;
  }
  const size_t need = bandchol_factor2_workspace(n, K);
  void* w2 = nullptr;
  if (fixed_ws) {
    if (need > fixed_size) {
      snprintf(g_err, sizeof g_err, "factor: n = %lld, k = %lld needs %zu bytes of working memory, more than the %zu "
               "of the fixed scratch array", (long long)n, (long long)k, need, fixed_size);
      return BANDCHOL_ETOOBIG;
    }
    w2 = fixed_ws;
  } else {
    w2 = workspace(need, &e);
    if (!w2) { set_err("workspace", e); return BANDCHOL_EHIP; }
  }
  e = bandchol_factor2_launch(n, k, ab, ldab, d_info, w2, spine_grid(wgs), st);
  if (e != hipSuccess) { set_err("factor launch", e); return BANDCHOL_EHIP; }
  return 0;
}

int64_t solve_async_impl(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, double* b,
                         int64_t ldb, hipStream_t st, int64_t* d_status = nullptr);

int64_t solve_backward_impl(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, const double* x,
                            int64_t ldx, double* g, int64_t ldg, double* gab, int64_t ldgab, hipStream_t st) {
  if (n < 0) return -1;
  if (k < 0) return -2;
  if (nrhs < 0) return -3;
  if (ab == nullptr && n > 0) return -4;
  if (ldab < k + 1) return -5;
  if (x == nullptr && n > 0 && nrhs > 0) return -6;
  if (ldx < (n > 1 ? n : 1)) return -7;
  if (g == nullptr && n > 0 && nrhs > 0) return -8;
  if (ldg < (n > 1 ? n : 1)) return -9;
  if (gab == nullptr && n > 0) return -10;
  if (ldgab < k + 1) return -11;
  if (n == 0) return 0;
  const int64_t kk = k < n - 1 ? k : n - 1;
  if (nrhs > 0) {
    const int64_t rc = solve_async_impl(n, k, nrhs, ab, ldab, g, ldg, st);
    if (rc != 0) return rc;
  }
  const bandchol_adj::AdjSys w{g, x, gab, n, kk, nrhs, ldg, ldx, ldgab};
  const hipError_t e = bandchol_outer_grad_launch1(w, st);
  if (e != hipSuccess) { set_err("solve backward", e); return BANDCHOL_EHIP; }
  return 0;
}

// d_status (device int64, may be NULL): set to BANDCHOL_EHANG when a wait of
// the solve gave up; never cleared here.
int64_t solve_args(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, const double* b,
                   int64_t ldb) {
  if (n < 0) return -1;
  if (k < 0) return -2;
  if (nrhs < 0) return -3;
  if (ab == nullptr && n > 0) return -4;
  if (ldab < k + 1) return -5;
  if (b == nullptr && n > 0 && nrhs > 0) return -6;
  if (ldb < (n > 1 ? n : 1)) return -7;
  return 0;
}

int64_t solve_async_impl(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, double* b,
                         int64_t ldb, hipStream_t st, int64_t* d_status) {
  const int64_t bad = solve_args(n, k, nrhs, ab, ldab, b, ldb);
  if (bad) return bad;
  if (n == 0 || nrhs == 0) return 0;
  const int64_t kk = k < n - 1 ? k : n - 1;
  hipError_t e;
  void* ws = workspace(bandchol_solve_workspace(n, kk), &e);
  if (!ws) { set_err("workspace", e); return BANDCHOL_EHIP; }
  e = bandchol_solve_launch(n, kk, nrhs, ab, ldab, b, ldb, ws, num_cus(), d_status, st);
  if (e != hipSuccess) { set_err("solve launch", e); return BANDCHOL_EHIP; }
  return 0;
}

int64_t factor_f32_impl(int64_t n, int64_t k, float* ab, int64_t ldab, int64_t* d_info, hipStream_t st) {
  if (n < 0) return -1;
  if (k < 0) return -2;
  if (ab == nullptr && n > 0) return -3;
  if (ldab < k + 1) return -4;
  if (d_info == nullptr) return -5;
  if (n > ((int64_t)1 << 31) - T) return -1;
  hipError_t e;
  if (n == 0) {
    set_info_kernel<<<1, 1, 0, st>>>(d_info, 0);
    e = hipGetLastError();
    if (e != hipSuccess) { set_err("factor f32", e); return BANDCHOL_EHIP; }
    return 0;
  }
  void* ws = workspace(bandchol_factor2_workspace_f32(n, tile_diagonals(n, k)), &e);
  if (!ws) { set_err("workspace", e); return BANDCHOL_EHIP; }
  const int K = tile_diagonals(n, k);
  const int wgs = schedule_wgs(n, K);   // no FP32 walk: a walk choice takes the rule
  e = bandchol_factor2_launch_f32(n, k, ab, ldab, d_info, ws, spine_grid(wgs == 1 ? spine_rule(K) : wgs), st);
  if (e != hipSuccess) { set_err("factor f32 launch", e); return BANDCHOL_EHIP; }
  return 0;
}

double from_bits(unsigned long long u) {
  double d;
  memcpy(&d, &u, sizeof d);
  return d;
}

// Mixed-precision solve (see bandchol.h).  Synchronous on `st`.
int64_t mixed_solve_impl(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, const double* b,
                         int64_t ldb, double* x, int64_t ldx, int64_t* iters, int64_t* fallback, hipStream_t st) {
  if (n < 0) return -1;
  if (k < 0) return -2;
  if (nrhs < 0) return -3;
  if (ab == nullptr && n > 0) return -4;
  if (ldab < k + 1) return -5;
  if (b == nullptr && n > 0 && nrhs > 0) return -6;
  if (ldb < (n > 1 ? n : 1)) return -7;
  if (x == nullptr && n > 0 && nrhs > 0) return -8;
  if (ldx < (n > 1 ? n : 1)) return -9;
  if (iters) *iters = 0;
  if (fallback) *fallback = 0;
  if (n == 0 || nrhs == 0) return 0;
  if (n > ((int64_t)1 << 31) - T) return -1;
  const int64_t kk = k < n - 1 ? k : n - 1;
  const int64_t ldl = kk + 1;
  // buffers: L32 (float band), L (widened factor, or the FP64 factor on fallback),
  // R (n x nrhs), norms (2 nrhs + 1), info
  const size_t off_l32 = 0;
  const size_t off_l = align_up(off_l32 + sizeof(float) * (size_t)ldl * n);
  const size_t off_r = align_up(off_l + sizeof(double) * (size_t)ldl * n);
  const size_t off_nrm = align_up(off_r + sizeof(double) * (size_t)n * nrhs);
  const size_t off_info = align_up(off_nrm + sizeof(unsigned long long) * (size_t)(2 * nrhs + 1));
  const size_t total = off_info + 256;
  hipError_t e;
  char* m = (char*)mixed_buffers(total, &e);
  if (!m) { set_err("mixed buffers", e); return BANDCHOL_EHIP; }
  float* l32 = (float*)(m + off_l32);
  double* l = (double*)(m + off_l);
  double* r = (double*)(m + off_r);
  unsigned long long* nrm = (unsigned long long*)(m + off_nrm);
  int64_t* dinfo = (int64_t*)(m + off_info);
  std::vector<unsigned long long> hn(2 * nrhs + 1);
  auto fail = [&](const char* what) {
    set_err(what, e);
    return (int64_t)BANDCHOL_EHIP;
  };
  auto fetch = [&](size_t count) -> bool {
    e = hipMemcpyAsync(hn.data(), nrm, sizeof(unsigned long long) * count, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e == hipSuccess;
  };
  // ||A||_inf: row sums of |A| into R(:, 0), then their maximum
  e = bandchol_residual(n, kk, ab, ldab, nullptr, 0, nullptr, 0, r, n, 1, 1, st);
  if (e == hipSuccess) e = bandchol_colmax(n, 1, r, n, nrm + 2 * nrhs, st);
  if (e != hipSuccess) return fail("mixed: norm");
  // FP32 factor of fl32(A)
  e = bandchol_band_to_f32(n, kk, ab, ldab, l32, ldl, st);
  if (e != hipSuccess) return fail("mixed: convert");
  int64_t* dstatus = dinfo + 1;   // BANDCHOL_EHANG once a solve's wait gave up
  set_info_kernel<<<1, 1, 0, st>>>(dstatus, 0);
  int64_t rc = factor_f32_impl(n, kk, l32, ldl, dinfo, st);
  if (rc != 0) return rc;
  int64_t info32 = 0;
  e = hipMemcpyAsync(&info32, dinfo, sizeof info32, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail("mixed: factor");
  if (!fetch(2 * nrhs + 1)) return fail("mixed: norm");
  const double anrm = from_bits(hn[2 * nrhs]);
  const double tol = sqrt((double)n) * 0x1p-53 * anrm;
  int64_t it = 0, reason = 0;
  if (info32 != 0) reason = 1;
  if (reason == 0) {
    e = bandchol_band_to_f64(n, kk, l32, ldl, l, ldl, st);
    if (e != hipSuccess) return fail("mixed: convert");
    e = hipMemcpy2DAsync(x, sizeof(double) * ldx, b, sizeof(double) * ldb, sizeof(double) * n, nrhs,
                         hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return fail("mixed: copy");
    rc = solve_async_impl(n, kk, nrhs, l, ldl, x, ldx, st, dstatus);
    if (rc != 0) return rc;
    std::vector<double> dprev(nrhs, 0.0);
    for (;;) {
      e = bandchol_residual(n, kk, ab, ldab, x, ldx, b, ldb, r, n, nrhs, 0, st);
      if (e == hipSuccess) e = bandchol_colmax(n, nrhs, r, n, nrm, st);
      if (e == hipSuccess) e = bandchol_colmax(n, nrhs, x, ldx, nrm + nrhs, st);
      if (e != hipSuccess || !fetch(2 * nrhs)) return fail("mixed: residual");
      bool done = true;
      for (int64_t c = 0; c < nrhs; ++c)
        if (!(from_bits(hn[c]) <= tol * from_bits(hn[nrhs + c]))) done = false;
      if (done) break;
      if (it == MIXED_ITMAX) { reason = 2; break; }
      rc = solve_async_impl(n, kk, nrhs, l, ldl, r, n, st, dstatus);
      if (rc != 0) return rc;
      e = bandchol_colmax(n, nrhs, r, n, nrm, st);
      if (e != hipSuccess || !fetch(nrhs)) return fail("mixed: correction");
      bool stall = false;
      for (int64_t c = 0; c < nrhs; ++c)
        if (it > 0 && !(from_bits(hn[c]) <= 0.5 * dprev[c])) stall = true;
      if (stall) { reason = 3; break; }
      for (int64_t c = 0; c < nrhs; ++c) dprev[c] = from_bits(hn[c]);
      e = bandchol_axpy(n, nrhs, x, ldx, r, n, st);
      if (e != hipSuccess) return fail("mixed: update");
      ++it;
    }
  }
  if (iters) *iters = it;
  if (fallback) *fallback = reason;
  // a solve whose wait gave up left x unspecified: report it, whatever the refinement decided
  auto solves_ok = [&]() -> int64_t {
    int64_t status = 0;
    e = hipMemcpyAsync(&status, dstatus, sizeof status, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail("mixed: status");
    if (status == BANDCHOL_EHANG) {
      snprintf(g_err, sizeof g_err, "mixed solve: a device-side wait exceeded its bound");
      return (int64_t)BANDCHOL_EHANG;
    }
    return 0;
  };
  if (reason == 0) return solves_ok();
  // FP64 fallback: factor a copy of A into L, then solve
  e = hipMemcpy2DAsync(l, sizeof(double) * ldl, ab, sizeof(double) * ldab, sizeof(double) * ldl, n,
                       hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return fail("mixed: copy");
  rc = factor_async_impl(n, kk, l, ldl, dinfo, st);
  if (rc != 0) return rc;
  int64_t info64 = 0;
  e = hipMemcpyAsync(&info64, dinfo, sizeof info64, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail("mixed: fallback factor");
  if (info64 != 0) return info64;
  e = hipMemcpy2DAsync(x, sizeof(double) * ldx, b, sizeof(double) * ldb, sizeof(double) * n, nrhs,
                       hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return fail("mixed: copy");
  rc = solve_async_impl(n, kk, nrhs, l, ldl, x, ldx, st, dstatus);
  if (rc != 0) return rc;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail("mixed: fallback solve");
  return solves_ok();
}

// ------------------------------------------- the factor that allocates nothing
// bandchol_factor_noalloc takes the spine's working memory (ticket counter,
// flags, tile inverses, pre-accumulated tiles) from this file-scope device
// array instead of the workspace.  Every device the library runs on holds its
// own copy from module load to process end.  In host code `scratch` names a
// host-side stand-in, not device memory: the kernels receive the address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 20;
__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};   // per device: address of its `scratch`

// Address of the current device's scratch array, looked up once per device
// (with that device current) and kept.
void* scratch_on_current_device(hipError_t* err) {
  int dev = 0;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

// ----------------------------------------------------------------- batches

struct bandchol_batch {
  int device = 0;
  int64_t batch = 0;
  bool has_rhs = false;
  // systems the walk takes (one workgroup each), in the order given
  std::vector<WalkSys> walk;
  std::vector<int64_t> walk_id;   // batch index of walk[j]
  int walk_kmax = 0;              // largest K among them
  // systems with K > WALK_KMAX: multi-workgroup factor and solve, one after another
  std::vector<WalkSys> wide;
  std::vector<int64_t> wide_id;
  std::vector<int> wide_wgs;      // spine workgroups of wide[j] (schedule table or rule, at plan creation)
  // device memory
  void* mem = nullptr;            // descriptors, order, counters, info staging, wide workspace, inverses
  WalkSys* d_sys = nullptr;
  int* d_order = nullptr;
  unsigned* d_queue = nullptr;
  int64_t* d_info_walk = nullptr;
  int64_t* d_walk_id = nullptr;   // batch index of each walk system (device copy)
  void* d_wide_ws = nullptr;
  int grid = 1;
  // adjoint buffers (bandchol_batch_set_adjoint)
  void* adj_mem = nullptr;
  WalkSys* d_sys_adj = nullptr;                   // walk descriptors with b = g
  bandchol_adj::AdjSys* d_adj = nullptr;          // every system (walk and wide)
  std::vector<bandchol_adj::AdjSys> adj;          // host copy, batch order
  std::vector<double*> wide_g;
  int64_t nmax = 0;
};

namespace {

__global__ void scatter_info_kernel(const int64_t* src, const int64_t* idx, int count, int64_t* dst) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < count) dst[idx[j]] = src[j];
}

// Test matrix of the schedule measurement: band (n, kk) in ldab = kk + 1 with
// off-diagonal entries uniform in [-1, 1) from the splitmix64 hash of their
// position and diagonal 2 kk + 2, which exceeds every row's off-diagonal sum:
// symmetric and strictly diagonally dominant, hence positive definite.
__global__ void tune_fill_kernel(double* ab, int64_t n, int64_t kk) {
  const int64_t w = kk + 1, total = n * w;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / w, i = t - j * w;
    double v = 0.0;
    if (i == 0) {
      v = 2.0 * (double)kk + 2.0;
    } else if (j + i < n) {
      uint64_t z = (uint64_t)t + 0x9e3779b97f4a7c15ull;
      z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
      z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
      z ^= z >> 31;
      v = (double)(z >> 11) * 0x1.0p-52 - 1.0;
    }
    ab[t] = v;
  }
}

// One wave runs `steps` dependent steps of the factor's pivot chain -- the
// reciprocal of the pivot (hardware estimate and two Newton steps, as the
// diagonal-tile sweep takes it) and the fused multiply-add that forms the
// next pivot from it -- between two reads of the 100 MHz real-time counter.
// The values stay near the fixed point of d -> 2 - 0.25 / d.
__global__ void pivot_chain_kernel(int64_t steps, double d0, double* out_d, unsigned long long* out_ticks) {
  double d = d0;
  const double p = 2.0, w = 0.5;
  const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
  for (int64_t s = 0; s < steps; ++s) {
    const double dinv = recip(d);
    d = fma(-(w * w), dinv, p);
  }
  const unsigned long long t1 = __builtin_amdgcn_s_memrealtime();
  if (threadIdx.x == 0) {
    *out_d = d;
    *out_ticks = t1 - t0;
  }
}

// Schedules the measurement tries: the walk where it applies, then spine
// workgroup counts up to the resident limit, and the rule's own count.
std::vector<int> tune_candidates(int K) {
  std::vector<int> c;
  if (K <= WALK_KMAX) c.push_back(1);
  if (K == 0) return c;   // a diagonal matrix has no tile tasks for helpers
  const int most = resident_wgs();
  for (int g : {32, 64, 96, 128, 192, 256, 320, 384, 448, 512, 640, 768, 1024})
    if (g <= most) c.push_back(g);
  const int r = spine_rule(K);
  if (std::find(c.begin(), c.end(), r) == c.end()) c.push_back(r);
  return c;
}

void tune_record(int64_t n, int64_t kk, int K, int wgs, double ms) {
  const int nb = n_bucket(n);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (TuneEntry& t : g_tune)
    if (t.nb == nb && t.K == K) {
      t.wgs = wgs, t.n = n, t.k = kk, t.ms = ms;
      return;
    }
  TuneEntry t;
  t.nb = nb, t.K = K, t.wgs = wgs, t.n = n, t.k = kk, t.ms = ms;
  g_tune.push_back(t);
}

}  // namespace

extern "C" {

int64_t bandchol_factor_async(int64_t n, int64_t k, double* ab, int64_t ldab, int64_t* d_info, void* stream) {
  g_err[0] = 0;
  return factor_async_impl(n, k, ab, ldab, d_info, (hipStream_t)stream);
}

int64_t bandchol_solve_async(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, double* b,
                             int64_t ldb, void* stream) {
  g_err[0] = 0;
  return solve_async_impl(n, k, nrhs, ab, ldab, b, ldb, (hipStream_t)stream);
}

int64_t bandchol_factor_noalloc(int64_t n, int64_t k, double* ab, int64_t ldab, int64_t* d_info, void* stream) {
  g_err[0] = 0;
  if (n < 0) return -1;
  if (k < 0) return -2;
  if (ab == nullptr && n > 0) return -3;
  if (ldab < k + 1) return -4;
  if (d_info == nullptr) return -5;
  hipError_t e;
  void* ptr = scratch_on_current_device(&e);
  if (!ptr) { set_err("scratch address", e); return BANDCHOL_EHIP; }
  return factor_async_impl(n, k, ab, ldab, d_info, (hipStream_t)stream, ptr, NOALLOC_SCRATCH_BYTES);
}

int64_t bandchol_factor(int64_t n, int64_t k, double* ab, int64_t ldab) {
  g_err[0] = 0;
  if (n < 0) return -1;
  if (k < 0) return -2;
  if (ab == nullptr && n > 0) return -3;
  if (ldab < k + 1) return -4;
  if (n == 0) return 0;
  hipError_t e;
  int64_t *h = nullptr, *d_info = nullptr;
  if (!info_slots(&h, &d_info, &e)) { set_err("info slots", e); return BANDCHOL_EHIP; }
  int64_t rc = factor_async_impl(n, k, ab, ldab, d_info, g_stream);
  if (rc != 0) return rc;
  e = hipMemcpyAsync(h, d_info, sizeof(int64_t), hipMemcpyDeviceToHost, g_stream);
  if (e == hipSuccess) e = hipStreamSynchronize(g_stream);
  if (e != hipSuccess) { set_err("factor", e); return BANDCHOL_EHIP; }
  if (*h == BANDCHOL_EHANG) snprintf(g_err, sizeof g_err, "factor: a device-side wait exceeded its bound");
  return *h;
}

int64_t bandchol_solve(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, double* b,
                       int64_t ldb) {
  g_err[0] = 0;
  const int64_t bad = solve_args(n, k, nrhs, ab, ldab, b, ldb);
  if (bad || n == 0 || nrhs == 0) return bad;
  hipError_t e;
  int64_t *h = nullptr, *d_status = nullptr;
  if (!info_slots(&h, &d_status, &e)) { set_err("info slots", e); return BANDCHOL_EHIP; }
  set_info_kernel<<<1, 1, 0, g_stream>>>(d_status, 0);
  e = hipGetLastError();
  if (e != hipSuccess) { set_err("solve", e); return BANDCHOL_EHIP; }
  int64_t rc = solve_async_impl(n, k, nrhs, ab, ldab, b, ldb, g_stream, d_status);
  if (rc != 0) return rc;
  e = hipMemcpyAsync(h, d_status, sizeof(int64_t), hipMemcpyDeviceToHost, g_stream);
  if (e == hipSuccess) e = hipStreamSynchronize(g_stream);
  if (e != hipSuccess) { set_err("solve", e); return BANDCHOL_EHIP; }
  if (*h == BANDCHOL_EHANG) {
    snprintf(g_err, sizeof g_err, "solve: a device-side wait exceeded its bound");
    return BANDCHOL_EHANG;
  }
  return 0;
}

int64_t bandchol_set_stream(void* stream) {
  g_stream = (hipStream_t)stream;
  return 0;
}

const char* bandchol_last_error(void) { return g_err; }

void bandchol_finalize(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (size_t d = 0; d < g_work.size(); ++d) {
    if (hipSetDevice((int)d) != hipSuccess) continue;
    (void)hipDeviceSynchronize();
    if (g_work[d].ptr) (void)hipFree(g_work[d].ptr);
    if (g_work[d].info_dev) (void)hipFree(g_work[d].info_dev);
    if (g_work[d].info_host) (void)hipHostFree(g_work[d].info_host);
    if (g_work[d].mptr) (void)hipFree(g_work[d].mptr);
    g_work[d] = DevWork();
  }
  (void)hipSetDevice(cur);
}

int64_t bandchol_tile(void) { return T; }

int64_t bandchol_factor_f32(int64_t n, int64_t k, float* ab, int64_t ldab, int64_t* d_info, void* stream) {
  g_err[0] = 0;
  return factor_f32_impl(n, k, ab, ldab, d_info, (hipStream_t)stream);
}

int64_t bandchol_mixed_solve(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, const double* b,
                             int64_t ldb, double* x, int64_t ldx, int64_t* iters, int64_t* fallback) {
  g_err[0] = 0;
  return mixed_solve_impl(n, k, nrhs, ab, ldab, b, ldb, x, ldx, iters, fallback, g_stream);
}

int64_t bandchol_solve_backward(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, const double* x,
                                int64_t ldx, double* g, int64_t ldg, double* gab, int64_t ldgab, void* stream) {
  g_err[0] = 0;
  return solve_backward_impl(n, k, nrhs, ab, ldab, x, ldx, g, ldg, gab, ldgab, (hipStream_t)stream);
}

int64_t bandchol_factor_backward(int64_t n, int64_t k, const double* l, int64_t ldl, const double* lbar, int64_t ldlb,
                                 double* abar, int64_t ldab, int64_t* d_status, void* stream) {
  g_err[0] = 0;
  if (n < 0) return -1;
  if (k < 0) return -2;
  if (l == nullptr && n > 0) return -3;
  if (ldl < k + 1) return -4;
  if (lbar == nullptr && n > 0) return -5;
  if (ldlb < k + 1) return -6;
  if (abar == nullptr && n > 0) return -7;
  if (ldab < k + 1) return -8;
  if (n > ((int64_t)1 << 31) - T) {
    snprintf(g_err, sizeof g_err, "n too large");
    return -1;
  }
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (n == 0) {
    if (d_status) {
      set_info_kernel<<<1, 1, 0, st>>>(d_status, 0);
      e = hipGetLastError();
      if (e != hipSuccess) { set_err("factor backward", e); return BANDCHOL_EHIP; }
    }
    return 0;
  }
  const int64_t kk = k < n - 1 ? k : n - 1;
  const int K = tile_diagonals(n, k);
  void* ws = workspace(bandchol_fb_workspace(n, K), &e);
  if (!ws) { set_err("workspace", e); return BANDCHOL_EHIP; }
  bandchol_fb::FbSys s{};
  s.l = l, s.ldl = ldl, s.lbar = lbar, s.ldlb = ldlb, s.abar = abar, s.ldab = ldab;
  s.n = n, s.k = kk, s.K = K;
  e = bandchol_fb_launch(s, ws, num_cus(), d_status, st);
  if (e != hipSuccess) { set_err("factor backward launch", e); return BANDCHOL_EHIP; }
  return 0;
}

int64_t bandchol_batch_create(int64_t batch, const int64_t* n, const int64_t* k, double* const* ab,
                              const int64_t* ldab, double* const* b, const int64_t* ldb, bandchol_batch_t* plan) {
  g_err[0] = 0;
  if (batch < 0) return -1;
  if (plan == nullptr) return -8;
  if (batch > 0 && (n == nullptr || k == nullptr || ab == nullptr || ldab == nullptr)) return n == nullptr ? -2 : (k == nullptr ? -3 : (ab == nullptr ? -4 : -5));
  if (b != nullptr && batch > 0 && ldb == nullptr) return -7;
  for (int64_t i = 0; i < batch; ++i) {
    if (n[i] < 0 || n[i] > ((int64_t)1 << 31) - T) return -2;
    if (k[i] < 0) return -3;
    if (ab[i] == nullptr && n[i] > 0) return -4;
    if (ldab[i] < k[i] + 1) return -5;
    if (b != nullptr) {
      if (b[i] == nullptr && n[i] > 0) return -6;
      if (ldb[i] < (n[i] > 1 ? n[i] : 1)) return -7;
    }
  }
  bandchol_batch* p = new bandchol_batch();
  p->batch = batch;
  p->has_rhs = b != nullptr;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { set_err("device", e); delete p; return BANDCHOL_EHIP; }
  size_t inv_doubles = 0, wide_ws = 0;
  std::vector<double> est;
  for (int64_t i = 0; i < batch; ++i) {
    const int64_t kk = k[i] < n[i] - 1 ? k[i] : (n[i] > 0 ? n[i] - 1 : 0);
    const int K = tile_diagonals(n[i], k[i]);
    WalkSys w{ab[i], n[i], kk, ldab[i], nullptr, b ? b[i] : nullptr, b ? ldb[i] : 0};
    const int bw = batch_schedule_wgs(n[i], K);
    if (bw == 1 && K <= WALK_KMAX) {
      p->walk.push_back(w);
      p->walk_id.push_back(i);
      p->walk_kmax = std::max(p->walk_kmax, K);
      inv_doubles += (size_t)((n[i] + T - 1) / T) * T * T;
      est.push_back((double)((n[i] + T - 1) / T) * (10.0 + (double)K * K));
    } else {
      p->wide.push_back(w);
      p->wide_id.push_back(i);
      p->wide_wgs.push_back(bw);
      wide_ws = std::max(wide_ws, std::max(bandchol_factor2_workspace(n[i], K), bandchol_solve_workspace(n[i], kk)));
    }
  }
  const int nw = (int)p->walk.size();
  std::vector<int> order(nw);
  for (int j = 0; j < nw; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return est[x] > est[y]; });
  // one allocation: [descriptors][order][counters][walk info][batch index][wide workspace][inverses]
  const size_t off_sys = 0;
  const size_t off_order = align_up(off_sys + sizeof(WalkSys) * nw);
  const size_t off_queue = align_up(off_order + sizeof(int) * nw);
  const size_t off_info = align_up(off_queue + 256);
  const size_t off_idx = align_up(off_info + sizeof(int64_t) * nw);
  const size_t off_wide = align_up(off_idx + sizeof(int64_t) * nw);
  const size_t off_inv = align_up(off_wide + wide_ws);
  const size_t total = off_inv + sizeof(double) * inv_doubles;
  e = hipMalloc(&p->mem, total > 0 ? total : 256);
  if (e != hipSuccess) { set_err("batch allocation", e); delete p; return BANDCHOL_EHIP; }
  char* base = (char*)p->mem;
  p->d_sys = (WalkSys*)(base + off_sys);
  p->d_order = (int*)(base + off_order);
  p->d_queue = (unsigned*)(base + off_queue);
  p->d_info_walk = (int64_t*)(base + off_info);
  p->d_walk_id = (int64_t*)(base + off_idx);
  p->d_wide_ws = wide_ws ? (void*)(base + off_wide) : nullptr;
  double* inv = (double*)(base + off_inv);
  for (int j = 0; j < nw; ++j) {
    p->walk[j].linv = inv;
    inv += (size_t)((p->walk[j].n + T - 1) / T) * T * T;
  }
  if (nw > 0) {
    e = hipMemcpy(p->d_sys, p->walk.data(), sizeof(WalkSys) * nw, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_order, order.data(), sizeof(int) * nw, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(p->d_walk_id, p->walk_id.data(), sizeof(int64_t) * nw, hipMemcpyHostToDevice);
    if (e != hipSuccess) { set_err("batch upload", e); (void)hipFree(p->mem); delete p; return BANDCHOL_EHIP; }
  }
  // workgroups that fit at once: one per CU (each holds up to ~150 KB of LDS)
  const size_t lds = bandchol_walk_lds_bytes(p->walk_kmax);
  const int per_cu = lds <= 80 * 1024 ? 2 : 1;
  p->grid = std::max(1, std::min(nw, num_cus() * per_cu));
  *plan = p;
  return 0;
}

int64_t bandchol_batch_factor(bandchol_batch_t p, int64_t* d_info, void* stream) {
  g_err[0] = 0;
  if (p == nullptr) return -1;
  if (d_info == nullptr && p->batch > 0) return -2;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  const int nw = (int)p->walk.size();
  if (nw > 0) {
    e = bandchol_walk_batch_factor_launch(p->d_sys, p->d_order, nw, p->walk_kmax, p->d_queue, p->d_info_walk,
                                          p->grid, st);
    if (e == hipSuccess) {
      scatter_info_kernel<<<(nw + 255) / 256, 256, 0, st>>>(p->d_info_walk, p->d_walk_id, nw, d_info);
      e = hipGetLastError();
    }
  }
  for (size_t j = 0; j < p->wide.size() && e == hipSuccess; ++j) {
    const WalkSys& w = p->wide[j];
    e = bandchol_factor2_launch(w.n, w.k, w.ab, w.ldab, d_info + p->wide_id[j], p->d_wide_ws,
                                spine_grid(p->wide_wgs[j]), st);
  }
  if (e != hipSuccess) { set_err("batch factor", e); return BANDCHOL_EHIP; }
  return 0;
}

int64_t bandchol_batch_solve(bandchol_batch_t p, int64_t nrhs, void* stream) {
  g_err[0] = 0;
  if (nrhs < 0) return -1;
  if (p == nullptr) return -3;
  if (!p->has_rhs) return -2;
  if (nrhs == 0) return 0;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  const int nw = (int)p->walk.size();
  if (nw > 0 && nrhs > (int64_t)0x7fffffff) return -1;
  if (nw > 0)
    e = bandchol_walk_batch_solve_launch(p->d_sys, p->d_order, nw, p->walk_kmax, (int)nrhs, p->d_queue + 4,
                                         p->grid, st);
  for (size_t j = 0; j < p->wide.size() && e == hipSuccess; ++j) {
    const WalkSys& w = p->wide[j];
    if (w.n == 0) continue;
    e = bandchol_solve_launch(w.n, w.k, nrhs, w.ab, w.ldab, w.b, w.ldb, p->d_wide_ws, num_cus(), nullptr, st);
  }
  if (e != hipSuccess) { set_err("batch solve", e); return BANDCHOL_EHIP; }
  return 0;
}

int64_t bandchol_batch_set_adjoint(bandchol_batch_t p, double* const* g, double* const* gab, const int64_t* ldgab) {
  g_err[0] = 0;
  if (p == nullptr) return -1;
  if (!p->has_rhs) return -1;
  if (p->batch > 0 && g == nullptr) return -2;
  if (p->batch > 0 && gab == nullptr) return -3;
  if (p->batch > 0 && ldgab == nullptr) return -4;
  // batch index -> system
  std::vector<const WalkSys*> sys(p->batch, nullptr);
  for (size_t j = 0; j < p->walk.size(); ++j) sys[p->walk_id[j]] = &p->walk[j];
  for (size_t j = 0; j < p->wide.size(); ++j) sys[p->wide_id[j]] = &p->wide[j];
  for (int64_t i = 0; i < p->batch; ++i) {
    if (g[i] == nullptr && sys[i]->n > 0) return -2;
    if (gab[i] == nullptr && sys[i]->n > 0) return -3;
    if (ldgab[i] < sys[i]->k + 1) return -4;
  }
  std::vector<WalkSys> walk_adj = p->walk;
  for (size_t j = 0; j < walk_adj.size(); ++j) {
    walk_adj[j].b = g[p->walk_id[j]];
    walk_adj[j].ldb = walk_adj[j].n > 1 ? walk_adj[j].n : 1;
  }
  p->wide_g.clear();
  for (size_t j = 0; j < p->wide.size(); ++j) p->wide_g.push_back(g[p->wide_id[j]]);
  p->adj.clear();
  p->nmax = 0;
  for (int64_t i = 0; i < p->batch; ++i) {
    const WalkSys& w = *sys[i];
    const int64_t ld = w.n > 1 ? w.n : 1;
    p->adj.push_back(bandchol_adj::AdjSys{g[i], w.b, gab[i], w.n, w.k, 0, ld, w.ldb, ldgab[i]});
    p->nmax = std::max(p->nmax, w.n);
  }
  const size_t off_adj = align_up(sizeof(WalkSys) * walk_adj.size());
  const size_t total = off_adj + sizeof(bandchol_adj::AdjSys) * p->adj.size();
  if (p->adj_mem) {
    (void)hipDeviceSynchronize();
    (void)hipFree(p->adj_mem);
    p->adj_mem = nullptr;
  }
  hipError_t e = hipMalloc(&p->adj_mem, total > 0 ? total : 256);
  if (e != hipSuccess) { set_err("adjoint allocation", e); return BANDCHOL_EHIP; }
  p->d_sys_adj = (WalkSys*)p->adj_mem;
  p->d_adj = (bandchol_adj::AdjSys*)((char*)p->adj_mem + off_adj);
  if (!walk_adj.empty())
    e = hipMemcpy(p->d_sys_adj, walk_adj.data(), sizeof(WalkSys) * walk_adj.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !p->adj.empty())
    e = hipMemcpy(p->d_adj, p->adj.data(), sizeof(bandchol_adj::AdjSys) * p->adj.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) { set_err("adjoint upload", e); return BANDCHOL_EHIP; }
  return 0;
}

int64_t bandchol_batch_backward(bandchol_batch_t p, int64_t nrhs, void* stream) {
  g_err[0] = 0;
  if (p == nullptr) return -1;
  if (nrhs < 0 || nrhs > (int64_t)0x7fffffff) return -2;
  if (p->adj_mem == nullptr) return -1;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  const int nw = (int)p->walk.size();
  if (nrhs > 0 && nw > 0)
    e = bandchol_walk_batch_solve_launch(p->d_sys_adj, p->d_order, nw, p->walk_kmax, (int)nrhs, p->d_queue + 8,
                                         p->grid, st);
  for (size_t j = 0; j < p->wide.size() && e == hipSuccess && nrhs > 0; ++j) {
    const WalkSys& w = p->wide[j];
    if (w.n == 0) continue;
    e = bandchol_solve_launch(w.n, w.k, nrhs, w.ab, w.ldab, p->wide_g[j], w.n > 1 ? w.n : 1, p->d_wide_ws,
                              num_cus(), nullptr, st);
  }
  if (e == hipSuccess) e = bandchol_outer_grad_launch(p->d_adj, (int)p->batch, p->nmax, nrhs, st);
  if (e != hipSuccess) { set_err("batch backward", e); return BANDCHOL_EHIP; }
  return 0;
}

void bandchol_batch_destroy(bandchol_batch_t p) {
  if (p == nullptr) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  if (p->mem) (void)hipFree(p->mem);
  if (p->adj_mem) (void)hipFree(p->adj_mem);
  (void)hipSetDevice(cur);
  delete p;
}

int64_t bandchol_batch_tune_set(int64_t n, int64_t k, int64_t wgs) {
  g_err[0] = 0;
  if (n < 1 || n > ((int64_t)1 << 31) - T) return -1;
  if (k < 0) return -2;
  const int K = tile_diagonals(n, k);
  if (wgs < 0 || (wgs == 1 && K > WALK_KMAX) || (wgs > 1 && K == 0) || wgs > resident_wgs()) return -3;
  const int nb = n_bucket(n);
  if (wgs == 0) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_btune.erase(std::remove_if(g_btune.begin(), g_btune.end(),
                                 [&](const TuneEntry& t) { return t.nb == nb && t.K == K; }),
                  g_btune.end());
    return 0;
  }
  btune_record(n, k < n - 1 ? k : n - 1, K, (int)wgs, 0.0);
  return 0;
}

int64_t bandchol_batch_tune_entries(int64_t cap, int64_t* n, int64_t* k, int64_t* wgs, double* ms) {
  g_err[0] = 0;
  if (cap < 0) return -1;
  if (cap > 0 && n == nullptr) return -2;
  if (cap > 0 && k == nullptr) return -3;
  if (cap > 0 && wgs == nullptr) return -4;
  if (cap > 0 && ms == nullptr) return -5;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const int64_t count = (int64_t)g_btune.size();
  for (int64_t i = 0; i < count && i < cap; ++i) {
    n[i] = g_btune[i].n;
    k[i] = g_btune[i].k;
    wgs[i] = g_btune[i].wgs;
    ms[i] = g_btune[i].ms;
  }
  return count;
}

void bandchol_batch_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_btune.clear();
}

int64_t bandchol_batch_tune(int64_t batch, const int64_t* n, const int64_t* k, int64_t reps, int64_t max_buckets,
                            double* ms_out) {
  g_err[0] = 0;
  if (batch < 1) return -1;
  if (n == nullptr) return -2;
  if (k == nullptr) return -3;
  if (reps < 1 || reps > 1000) return -4;
  if (max_buckets < 0) return -5;
  for (int64_t i = 0; i < batch; ++i) {
    if (n[i] < 1 || n[i] > ((int64_t)1 << 31) - T) return -2;
    if (k[i] < 0) return -3;
  }
  // the test bands: diagonally dominant, generated on the device, one allocation
  std::vector<int64_t> kk(batch), ld(batch), off(batch);
  size_t total = 0;
  for (int64_t i = 0; i < batch; ++i) {
    kk[i] = k[i] < n[i] - 1 ? k[i] : n[i] - 1;
    ld[i] = kk[i] + 1;
    off[i] = (int64_t)total;
    total += (size_t)ld[i] * (size_t)n[i];
  }
  hipStream_t st = g_stream;
  double* mem = nullptr;
  int64_t* d_info = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&mem, sizeof(double) * total);
  if (e == hipSuccess) e = hipMalloc(&d_info, sizeof(int64_t) * batch);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  std::vector<double*> ab(batch);
  for (int64_t i = 0; i < batch; ++i) ab[i] = mem + off[i];
  std::vector<int64_t> h_info(batch);
  int64_t rc = 0;
  // median factor time of a plan built from the current batch table; < 0 on failure
  auto measure = [&]() -> double {
    bandchol_batch_t plan = nullptr;
    rc = bandchol_batch_create(batch, n, kk.data(), ab.data(), ld.data(), nullptr, nullptr, &plan);
    if (rc != 0) return -1.0;
    std::vector<float> t;
    for (int64_t r = 0; r <= reps && e == hipSuccess; ++r) {
      for (int64_t i = 0; i < batch && e == hipSuccess; ++i) {
        const int64_t cnt = ld[i] * n[i];
        tune_fill_kernel<<<(unsigned)std::min<int64_t>((cnt + 255) / 256, 8192), 256, 0, st>>>(ab[i], n[i], kk[i]);
        e = hipGetLastError();
      }
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      if (e != hipSuccess) break;
      rc = bandchol_batch_factor(plan, d_info, st);
      if (rc != 0) break;
      e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && r > 0) t.push_back(ms);
    }
    if (e == hipSuccess && rc == 0)
      e = hipMemcpy(h_info.data(), d_info, sizeof(int64_t) * batch, hipMemcpyDeviceToHost);
    bandchol_batch_destroy(plan);
    if (e != hipSuccess || rc != 0) return -1.0;
    for (int64_t i = 0; i < batch; ++i)
      if (h_info[i] != 0) {
        snprintf(g_err, sizeof g_err, "batch tune: factor of test system %lld returned info %lld", (long long)i,
                 (long long)h_info[i]);
        rc = BANDCHOL_EHIP;
        return -1.0;
      }
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
  };
  double best = e == hipSuccess ? measure() : -1.0;
  if (best >= 0.0) {
    // buckets by the walk's work estimate, largest first
    struct Bucket { int nb, K; int64_t n, k; double work; };
    std::vector<Bucket> bk;
    for (int64_t i = 0; i < batch; ++i) {
      const int K = tile_diagonals(n[i], kk[i]), nb = n_bucket(n[i]);
      const double w = (double)((n[i] + T - 1) / T) * (10.0 + (double)K * K);
      bool found = false;
      for (Bucket& b : bk)
        if (b.nb == nb && b.K == K) { b.work += w; found = true; break; }
      if (!found) bk.push_back(Bucket{nb, K, n[i], kk[i], w});
    }
    std::stable_sort(bk.begin(), bk.end(), [](const Bucket& x, const Bucket& y) { return x.work > y.work; });
    for (size_t b = 0; b < bk.size() && (int64_t)b < max_buckets && best >= 0.0; ++b) {
      if (bk[b].K == 0) continue;
      const int cur = batch_schedule_wgs(bk[b].n, bk[b].K);
      int alt = cur == 1 ? spine_rule(bk[b].K) : (bk[b].K <= WALK_KMAX ? 1 : 0);
      if (alt == 0) continue;
      btune_record(bk[b].n, bk[b].k, bk[b].K, alt, 0.0);
      const double t = measure();
      if (t < 0.0) { best = -1.0; break; }
      if (t < 0.99 * best) {
        best = t;
        btune_record(bk[b].n, bk[b].k, bk[b].K, alt, t);
      } else {
        btune_record(bk[b].n, bk[b].k, bk[b].K, cur, best);
      }
    }
  }
  if (e != hipSuccess) {
    set_err("batch tune", e);
    rc = BANDCHOL_EHIP;
  } else if (best < 0.0 && rc == 0) {
    rc = BANDCHOL_EHIP;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (d_info) (void)hipFree(d_info);
  if (mem) (void)hipFree(mem);
  if (rc == 0 && ms_out) *ms_out = best;
  return rc;
}

int64_t bandchol_spine_profile(int64_t n, int64_t k, int64_t reps, double* out, int64_t cap) {
  g_err[0] = 0;
  constexpr int SLOTS = 11;   // as the factor kernel's PROF_* slots
  if (n < 2 || n > ((int64_t)1 << 31) - T) return -1;
  if (k < 1) return -2;
  if (reps < 1 || reps > 100) return -3;
  if (out == nullptr || cap < SLOTS + 2) return -4;
  const int64_t kk = k < n - 1 ? k : n - 1;
  const int K = tile_diagonals(n, kk);
  int wgs = schedule_wgs(n, K);
  if (wgs == 1) wgs = spine_rule(K);
  hipStream_t st = g_stream;
  double* ab = nullptr;
  void* buf = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&ab, sizeof(double) * (size_t)(kk + 1) * (size_t)n);
  if (e == hipSuccess) e = hipMalloc(&buf, 512);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  void* ws = e == hipSuccess ? workspace(bandchol_factor2_workspace(n, K), &e) : nullptr;
  int64_t* d_info = (int64_t*)buf;
  unsigned long long* prof = (unsigned long long*)((char*)buf + 256);
  const int64_t total = (kk + 1) * n;
  float ms = 0.0f;
  for (int64_t r = 0; r < reps && e == hipSuccess; ++r) {
    tune_fill_kernel<<<(unsigned)std::min<int64_t>((total + 255) / 256, 8192), 256, 0, st>>>(ab, n, kk);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = bandchol_factor2_launch_profiled(n, kk, ab, kk + 1, d_info, ws, spine_grid(wgs), prof, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  }
  unsigned long long h[SLOTS] = {};
  int64_t info = 0;
  if (e == hipSuccess) e = hipMemcpy(h, prof, sizeof h, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&info, d_info, sizeof info, hipMemcpyDeviceToHost);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (buf) (void)hipFree(buf);
  if (ab) (void)hipFree(ab);
  if (e != hipSuccess) { set_err("spine profile", e); return BANDCHOL_EHIP; }
  if (info != 0) {
    snprintf(g_err, sizeof g_err, "spine profile: factor returned info %lld", (long long)info);
    return BANDCHOL_EHIP;
  }
  const double steps = h[SLOTS - 1] > 0 ? (double)h[SLOTS - 1] : 1.0;
  for (int i = 0; i < SLOTS - 1; ++i) out[i] = (double)h[i] / steps;
  out[SLOTS - 1] = (double)h[SLOTS - 1];
  out[SLOTS] = ms;
  out[SLOTS + 1] = wgs;
  return 0;
}

int64_t bandchol_pivot_chain_ns(int64_t steps, double* ns_per_step) {
  g_err[0] = 0;
  if (steps < 1 || steps > ((int64_t)1 << 32)) return -1;
  if (ns_per_step == nullptr) return -2;
  hipStream_t st = g_stream;
  void* buf = nullptr;
  hipError_t e = hipMalloc(&buf, 256);
  unsigned long long ticks = 0;
  if (e == hipSuccess) {
    pivot_chain_kernel<<<1, 64, 0, st>>>(steps, 1.9, (double*)buf, (unsigned long long*)((char*)buf + 64));
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(&ticks, (char*)buf + 64, sizeof ticks, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (buf) (void)hipFree(buf);
  if (e != hipSuccess) { set_err("pivot chain probe", e); return BANDCHOL_EHIP; }
  *ns_per_step = (double)ticks * 10.0 / (double)steps;
  return 0;
}

int64_t bandchol_set_walk_limit(int64_t kmax) {
  const int64_t prev = walk_kmax();
  if (kmax < 0) return prev;
  g_walk_kmax = (int)(kmax > WALK_KMAX ? WALK_KMAX : kmax);
  return prev;
}

int64_t bandchol_schedule(int64_t n, int64_t k) {
  g_err[0] = 0;
  if (n < 0 || n > ((int64_t)1 << 31) - T) return -1;
  if (k < 0) return -2;
  if (n == 0) return 0;
  const int wgs = schedule_wgs(n, tile_diagonals(n, k));
  return wgs == 1 ? 1 : spine_grid(wgs);
}

int64_t bandchol_tune_set(int64_t n, int64_t k, int64_t wgs) {
  g_err[0] = 0;
  if (n < 1 || n > ((int64_t)1 << 31) - T) return -1;
  if (k < 0) return -2;
  const int K = tile_diagonals(n, k);
  if (wgs < 0 || (wgs == 1 && K > WALK_KMAX) || (wgs > 1 && K == 0) || wgs > resident_wgs()) return -3;
  if (wgs == 0) {
    const int nb = n_bucket(n);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.erase(std::remove_if(g_tune.begin(), g_tune.end(),
                                [&](const TuneEntry& t) { return t.nb == nb && t.K == K; }),
                 g_tune.end());
    return 0;
  }
  tune_record(n, k < n - 1 ? k : n - 1, K, (int)wgs, 0.0);
  return 0;
}

int64_t bandchol_tune_entries(int64_t cap, int64_t* n, int64_t* k, int64_t* wgs, double* ms) {
  g_err[0] = 0;
  if (cap < 0) return -1;
  if (cap > 0 && n == nullptr) return -2;
  if (cap > 0 && k == nullptr) return -3;
  if (cap > 0 && wgs == nullptr) return -4;
  if (cap > 0 && ms == nullptr) return -5;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const int64_t count = (int64_t)g_tune.size();
  for (int64_t i = 0; i < count && i < cap; ++i) {
    n[i] = g_tune[i].n;
    k[i] = g_tune[i].k;
    wgs[i] = g_tune[i].wgs;
    ms[i] = g_tune[i].ms;
  }
  return count;
}

void bandchol_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}

int64_t bandchol_tune_factor(int64_t n, int64_t k, int64_t reps, int64_t* wgs_out, double* ms_out) {
  g_err[0] = 0;
  if (n < 1 || n > ((int64_t)1 << 31) - T) return -1;
  if (k < 0) return -2;
  if (reps < 1 || reps > 1000) return -3;
  const int64_t kk = k < n - 1 ? k : n - 1;
  const int K = tile_diagonals(n, k);
  const std::vector<int> cand = tune_candidates(K);
  hipStream_t st = g_stream;
  double* ab = nullptr;
  int64_t* d_info = nullptr;
  int64_t* h_info = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int64_t rc = 0;
  int best = 0;
  double best_ms = 0.0;
  hipError_t e = hipMalloc(&ab, sizeof(double) * (size_t)(kk + 1) * (size_t)n);
  if (e == hipSuccess) e = hipMalloc(&d_info, 256);
  if (e == hipSuccess) e = hipHostMalloc(&h_info, 64, hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const int64_t total = (kk + 1) * n;
  const int fill_grid = (int)std::min<int64_t>((total + 255) / 256, 8192);
  std::vector<float> t;
  for (size_t c = 0; c < cand.size() && e == hipSuccess && rc == 0; ++c) {
    t.clear();
    for (int64_t r = 0; r <= reps && e == hipSuccess && rc == 0; ++r) {
      tune_fill_kernel<<<fill_grid, 256, 0, st>>>(ab, n, kk);
      e = hipGetLastError();
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      if (e != hipSuccess) break;
      rc = factor_with(n, kk, ab, kk + 1, d_info, cand[c], st);
      if (rc != 0) break;
      e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipMemcpyAsync(h_info, d_info, sizeof(int64_t), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) break;
      if (*h_info != 0) {
        snprintf(g_err, sizeof g_err, "tune: factor of the test matrix returned info %lld", (long long)*h_info);
        rc = BANDCHOL_EHIP;
        break;
      }
      if (r == 0) {
        if (best > 0 && ms > 2.0 * best_ms) break;   // far behind the best: no timed runs
        continue;
      }
      t.push_back(ms);
    }
    if ((int64_t)t.size() == reps) {
      std::sort(t.begin(), t.end());
      const double med = t[t.size() / 2];
      if (best == 0 || med < best_ms) best = cand[c], best_ms = med;
    }
  }
  if (e != hipSuccess && rc == 0) {
    set_err("tune", e);
    rc = BANDCHOL_EHIP;
  }
  if (rc == 0 && best == 0) {
    snprintf(g_err, sizeof g_err, "tune: no schedule measured");
    rc = BANDCHOL_EHIP;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (h_info) (void)hipHostFree(h_info);
  if (d_info) (void)hipFree(d_info);
  if (ab) (void)hipFree(ab);
  if (rc != 0) return rc;
  tune_record(n, kk, K, best, best_ms);
  if (wgs_out) *wgs_out = best;
  if (ms_out) *ms_out = best_ms;
  return 0;
}

}  // extern "C"
