// FP64 band Cholesky factorization and band solves for gfx950.
//
// The factor walks the band in T x T tiles.  Tile (R, C) covers rows
// [R*T, R*T+T) and columns [C*T, C*T+T); the band holds tiles with
// 0 <= R - C <= K, K = ceil(k / T).  In the paper's terms (Algorithm 1,
// Section 3) every diagonal tile is factored by dense Cholesky (potrf), every
// tile below it is solved against it (trsm), and every tile receives the
// rank-T updates L(R,s) L(C,s)^T of the earlier tile columns s (gemm/syrk).
//
// Scheduling replaces the paper's OpenMP task graph (Section 3.1): one
// persistent kernel; workgroups take tasks from a global counter in a fixed
// topological order and wait on per-tile ready flags, so a task only ever
// waits for tasks that were taken earlier.  Task order per tile column C:
//   D(C)        diagonal tile: acc = A(C,C) - sum_s L(C,s) L(C,s)^T, then a
//               one-wave register sweep that factors it and, in the same
//               instructions, solves the identity against it, giving
//               L(C,C) and L(C,C)^{-T};
//   O(C+d, C)   d = 1..K: acc = A(R,C) - sum_s L(R,s) L(C,s)^T, then
//               L(R,C) = acc * L(C,C)^{-T} (the trsm as an FP64 MFMA product).
// All tile products run on v_mfma_f64_16x16x4.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "bandchol.h"

#include "common.h"

size_t bandchol_solve_workspace(int64_t n);
size_t bandchol_factor2_workspace(int64_t n, int64_t K);
hipError_t bandchol_factor2_launch(int64_t n, int64_t k, double* ab, int64_t ldab, int64_t* d_info, void* ws,
                                   int grid_max, hipStream_t st);
hipError_t bandchol_solve_launch(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, double* b,
                                 int64_t ldb, void* ws, int num_cus, hipStream_t st);

namespace {

using namespace bandchol;

constexpr int NT = 256;      // threads per workgroup (4 waves)
constexpr long long SPIN_LIMIT = 1LL << 25;

struct Work {
  int* flags;          // NB * (K+1) tile-ready flags, tile (R, R-d) at R*(K+1)+d
  double* linvt;       // NB tiles of L(C,C)^{-T}, row-major T x T
  unsigned* queue;     // next task ticket
  int* abort_flag;     // 1 = pivot failure, 2 = wait bound exceeded
  unsigned long long* first_fail;  // smallest failing 1-based column
};

__device__ __forceinline__ int ld_flag(const int* f) {
  return __builtin_amdgcn_readfirstlane(__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Thread 0 waits for up to two flags; the whole workgroup learns whether to go
// on.  Every wave then performs its own acquire before reading tile data.
__device__ bool wg_wait(const int* f1, const int* f2, const Work& w, lds_i* s_ok) {
  if (threadIdx.x == 0) {
    int ok = 1;
    long long spins = 0;
    for (const int* f : {f1, f2}) {
      if (!f) continue;
      while (!ld_flag(f)) {
        if (ld_flag(w.abort_flag)) { ok = 0; break; }
        if (++spins > SPIN_LIMIT) {
          __hip_atomic_store(w.abort_flag, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      if (!ok) break;
    }
    *s_ok = ok;
  }
  __syncthreads();
  int ok = *s_ok;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return ok != 0;
}

// Every wave makes its stores visible device-wide, then one thread raises the flag.
__device__ void wg_publish(int* f) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct FactorParams {
  Band a;
  int NB, K;
  unsigned ntasks;
  Work w;
};

// acc -= L(R,s) L(C,s)^T for this wave's 16x16 block (bi, bj) of the tile.
__device__ __forceinline__ d4 tile_term(const Band& a, int R, int C, int s, int bi, int bj, d4 acc) {
  const int lane = threadIdx.x & 63;
  const int64_t ri = (int64_t)R * T + 16 * bi + (lane & 15);
  const int64_t ci = (int64_t)C * T + 16 * bj + (lane & 15);
  const int64_t j0 = (int64_t)s * T + (lane >> 4);
  double xf[T / 4], yf[T / 4];
#pragma unroll
  for (int q = 0; q < T / 4; ++q) {
    xf[q] = a.ld(ri, j0 + 4 * q);
    yf[q] = a.ld(ci, j0 + 4 * q);
  }
#pragma unroll
  for (int q = 0; q < T / 4; ++q) acc = mfma_xyt(-xf[q], yf[q], acc);
  return acc;
}

// Load tile (R, C) of A into this wave's accumulator block.  Diagonal tile:
// positions past row n-1 get an identity so that the sweep never fails there.
__device__ __forceinline__ d4 tile_load(const Band& a, int R, int C, int bi, int bj) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)R * T + 16 * bi + (lane & 15);
  d4 acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t j = (int64_t)C * T + 16 * bj + 4 * r + (lane >> 4);
    double v = a.ld(i, j);
    if (R == C && i == j && i >= a.n) v = 1.0;
    acc[r] = v;
  }
  return acc;
}

__device__ __forceinline__ void acc_to_lds(lds_d* lds, int bi, int bj, d4 acc) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < 4; ++r) lds[(16 * bj + 4 * r + (lane >> 4)) * LP + 16 * bi + (lane & 15)] = acc[r];
}

// Each task body is compiled on its own (noinline) so that the two term loops
// are never merged into one.
__device__ __attribute__((noinline)) void diag_task(const FactorParams& P, int C, lds_d* lds, lds_d* wbuf, lds_i* s_ok) {
  const Band& a = P.a;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int bi = wave & 1, bj = wave >> 1;
  const bool active = bi >= bj;  // lower blocks only
  d4 acc = {0, 0, 0, 0};
  if (active) acc = tile_load(a, C, C, bi, bj);
  const int s0 = C - P.K > 0 ? C - P.K : 0;
  for (int s = s0; s < C; ++s) {
    if (!wg_wait(&P.w.flags[C * (P.K + 1) + (C - s)], nullptr, P.w, s_ok)) return;
    if (active) acc = tile_term(a, C, C, s, bi, bj, acc);
  }
  if (active) acc_to_lds(lds, bi, bj, acc);
  else acc_to_lds(lds, bi, bj, d4{0, 0, 0, 0});
  __syncthreads();
  if (wave == 0) {
    double row[T];
#pragma unroll
    for (int c = 0; c < T; ++c)
      row[c] = lane < T ? lds[c * LP + lane] : ((lane - T) == c ? 1.0 : 0.0);
    const int fail = sweep_ldlt(row, wbuf);
    if (fail >= 0) {
      const long long col = (long long)C * T + fail;
      if (lane == 0 && col < a.n) {
        atomicMin(P.w.first_fail, (unsigned long long)(col + 1));
        __hip_atomic_store(P.w.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    } else {
      const int64_t i = (int64_t)C * T + lane;
#pragma unroll
      for (int c = 0; c < T; ++c) {
        if (lane < T) {
          if (c <= lane && i < a.n) a.ab[(lane - c) + ((int64_t)C * T + c) * a.ldab] = row[c];
        } else {
          P.w.linvt[(int64_t)C * T * T + (lane - T) * T + c] = row[c];
        }
      }
    }
    if (lane == 0) *s_ok = fail < 0;
  }
  __syncthreads();
  if (!*s_ok) return;
  wg_publish(&P.w.flags[C * (P.K + 1)]);
}

__device__ __attribute__((noinline)) void off_task(const FactorParams& P, int R, int C, lds_d* lds, lds_i* s_ok) {
  const Band& a = P.a;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int bi = wave & 1, bj = wave >> 1;
  d4 acc = tile_load(a, R, C, bi, bj);
  const int s0 = R - P.K > 0 ? R - P.K : 0;
  for (int s = s0; s < C; ++s) {
    if (!wg_wait(&P.w.flags[R * (P.K + 1) + (R - s)], &P.w.flags[C * (P.K + 1) + (C - s)], P.w, s_ok)) return;
    acc = tile_term(a, R, C, s, bi, bj, acc);
  }
  acc_to_lds(lds, bi, bj, acc);
  // L(C,C)^{-T} ready?  (The wait's barrier also orders the LDS writes above.)
  if (!wg_wait(&P.w.flags[C * (P.K + 1)], nullptr, P.w, s_ok)) return;
  // out = acc * L(C,C)^{-T} = X Y^T with X = acc, Y = L(C,C)^{-1}; the upper
  // triangular L^{-T} has zero rows below column 16*bj+15.
  const double* lt = P.w.linvt + (int64_t)C * T * T;
  d4 out = {0, 0, 0, 0};
  const int qmax = (16 * bj + 16) / 4;
#pragma unroll
  for (int q = 0; q < T / 4; ++q) {
    if (q < qmax) {
      const int kk = 4 * q + (lane >> 4);
      const double xf = lds[kk * LP + 16 * bi + (lane & 15)];
      const double yf = lt[kk * T + 16 * bj + (lane & 15)];
      out = mfma_xyt(xf, yf, out);
    }
  }
  const int64_t i = (int64_t)R * T + 16 * bi + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t j = (int64_t)C * T + 16 * bj + 4 * r + (lane >> 4);
    if (a.in_band(i, j)) a.ab[(i - j) + j * a.ldab] = out[r];
  }
  wg_publish(&P.w.flags[R * (P.K + 1) + (R - C)]);
}

__global__ void __launch_bounds__(NT) factor_kernel(FactorParams P) {
  __shared__ double lds[T * LP];
  __shared__ double wbuf[64];
  __shared__ int s_task, s_ok, s_abort;
  for (;;) {
    if (threadIdx.x == 0) {
      s_task = (int)atomicAdd(P.w.queue, 1u);
      s_abort = ld_flag(P.w.abort_flag);
    }
    __syncthreads();
    const unsigned t = (unsigned)s_task;
    if (t >= P.ntasks || s_abort) break;
    const int C = (int)(t / (unsigned)(P.K + 1));
    const int d = (int)(t % (unsigned)(P.K + 1));
    if (C + d < P.NB) {
      if (d == 0) diag_task(P, C, (lds_d*)lds, (lds_d*)wbuf, (lds_i*)&s_ok);
      else off_task(P, C + d, C, (lds_d*)lds, (lds_i*)&s_ok);
    }
    __syncthreads();
  }
}

__global__ void factor_init_kernel(int* flags, int64_t nflags, unsigned* queue, int* abort_flag,
                                   unsigned long long* first_fail) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = g; i < nflags; i += (int64_t)gridDim.x * blockDim.x) flags[i] = 0;
  if (g == 0) {
    *queue = 0;
    *abort_flag = 0;
    *first_fail = 0x7fffffffffffffffULL;
  }
}

__global__ void factor_finish_kernel(const int* abort_flag, const unsigned long long* first_fail, int64_t* d_info) {
  const int ab = *abort_flag;
  const unsigned long long ff = *first_fail;
  *d_info = (ab == 2) ? (int64_t)BANDCHOL_EHANG : (ff == 0x7fffffffffffffffULL ? 0 : (int64_t)ff);
}

// ----------------------------------------------------------------- single-workgroup walk
//
// One workgroup factors one matrix, right-looking and in place, with no
// communication outside the workgroup.  Per tile column C:
//   phase A  wave 0: sweep of the staged diagonal tile -> L(C,C), L(C,C)^{-T};
//            waves 1-3: the work of column C-1 that the next diagonal tile does
//            not wait for: trsm of tiles (C-1+d, C-1), d >= 2, then the updates
//            tile(C-1+dr, C-1+dc) -= L(C-1+dr, C-1) L(C-1+dc, C-1)^T, all pairs but (1,1);
//   phase B  all waves: trsm of tile (C+1, C) (the critical one);
//   phase C  waves 1-3: diag = tile(C+1, C+1) - L(C+1, C) L(C+1, C)^T, staged for the next sweep.
// The current tile column's L tiles stay in LDS (pnl) for the updates.

constexpr int WALK_KMAX = 15;

// Trsm of a tile in place: every output block needs the input row-block over all
// columns, so all input fragments are read before any output is written.
// Fragments of row-block bi of tile (R, C): x[q] = A(R*T + 16 bi + l%16, C*T + 4q + l/16).
__device__ __forceinline__ void rowblk_load(const Band& a, int64_t R, int64_t C, int bi, double (&x)[T / 4]) {
  const int lane = lane_id();
  const int64_t i = R * T + 16 * bi + (lane & 15);
#pragma unroll
  for (int q = 0; q < T / 4; ++q) x[q] = a.ld(i, C * T + 4 * q + (lane >> 4));
}

// out block (bi, bj) = X_rowblk * L^{-T}(:, 16bj..16bj+15); L^{-T} row-major in LDS, upper triangular.
__device__ __forceinline__ d4 blk_trsm_frag(const double (&x)[T / 4], const lds_d* linvt, int bj) {
  const int lane = lane_id();
  const int qmax = 4 * bj + 4;
  d4 out = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < T / 4; ++q)
    if (q < qmax) out = mfma_xyt(x[q], linvt[(4 * q + (lane >> 4)) * T + 16 * bj + (lane & 15)], out);
  return out;
}

// One wave: tile (R, C) <- tile (R, C) * L(C,C)^{-T}, written to global and to an LDS copy.
__device__ __forceinline__ void tile_trsm_wave(const Band& a, int64_t R, int64_t C, const lds_d* linvt, lds_d* lds_out) {
  double x0[T / 4], x1[T / 4];
  rowblk_load(a, R, C, 0, x0);
  rowblk_load(a, R, C, 1, x1);
  const d4 o00 = blk_trsm_frag(x0, linvt, 0), o01 = blk_trsm_frag(x0, linvt, 1);
  const d4 o10 = blk_trsm_frag(x1, linvt, 0), o11 = blk_trsm_frag(x1, linvt, 1);
  blk_to_lds(lds_out, 0, 0, o00); blk_to_lds(lds_out, 0, 1, o01);
  blk_to_lds(lds_out, 1, 0, o10); blk_to_lds(lds_out, 1, 1, o11);
  blk_store(a, R, C, 0, 0, o00); blk_store(a, R, C, 0, 1, o01);
  blk_store(a, R, C, 1, 0, o10); blk_store(a, R, C, 1, 1, o11);
}

struct WalkLds {
  lds_d* diag;    // T*LP
  lds_d* linvt;   // 2 * T*T
  lds_d* pnl;     // K * T*LP
  lds_d* wbuf;    // 64
};

__device__ __forceinline__ WalkLds walk_lds(lds_d* base, int K) {
  WalkLds L;
  L.diag = base;
  L.linvt = L.diag + T * LP;
  L.pnl = L.linvt + 2 * T * T;
  L.wbuf = L.pnl + (size_t)K * T * LP;
  return L;
}

size_t walk_lds_bytes(int K) { return sizeof(double) * ((size_t)T * LP + 2 * T * T + (size_t)K * T * LP + 64); }

// wave 0: factor the staged diagonal tile, store L(C,C), keep L(C,C)^{-T} in LDS
__device__ __attribute__((noinline)) void walk_sweep(const Band& a, int64_t C, const WalkLds& L, lds_d* lt, lds_i* s_fail) {
  const int lane = lane_id();
  double row[T];
#pragma unroll
  for (int c = 0; c < T; ++c) row[c] = lane < T ? L.diag[c * LP + lane] : ((lane - T) == c ? 1.0 : 0.0);
  const int fail = sweep_ldlt(row, L.wbuf);
  if (fail >= 0) {
    if (lane == 0) *s_fail = fail;
    return;
  }
  const int64_t i = C * T + lane;
#pragma unroll
  for (int c = 0; c < T; ++c) {
    if (lane < T) {
      if (c <= lane && i < a.n) *a.at(i, C * T + c) = row[c];
    } else {
      lt[(lane - T) * T + c] = row[c];
    }
  }
}

// waves 1-3: the rest of tile column Cp (trsm of d >= 2, then all updates but the critical one)
__device__ __attribute__((noinline)) void walk_column_rest(const Band& a, int K, int64_t NB, int64_t Cp,
                                                           const WalkLds& L, const lds_d* lt_prev, lds_i* s_sync,
                                                           int sync_target) {
  const int wave = wave_id(), lane = lane_id();
  for (int d = 2; d <= K && Cp + d < NB; ++d)
    if ((d - 2) % 3 == wave - 1) tile_trsm_wave(a, Cp + d, Cp, lt_prev, L.pnl + (size_t)(d - 1) * T * LP);
  int idx = 0;
  // waves 1-3 meet before using each other's panel tiles
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): this wave's LDS writes are done
  if (lane == 0) __hip_atomic_fetch_add(s_sync, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  while (__hip_atomic_load(s_sync, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < sync_target)
    __builtin_amdgcn_s_sleep(1);
  for (int dr = 1; dr <= K && Cp + dr < NB; ++dr) {
    for (int dc = 1; dc <= dr; ++dc) {
      if (dr == 1 && dc == 1) continue;
      for (int blk = 0; blk < 4; ++blk) {
        const int bi = blk & 1, bj = blk >> 1;
        if (dr == dc && bj > bi) continue;
        if (idx++ % 3 != wave - 1) continue;
        d4 acc = blk_load(a, Cp + dr, Cp + dc, bi, bj);
        acc = blk_gemm_lds(L.pnl + (size_t)(dr - 1) * T * LP, L.pnl + (size_t)(dc - 1) * T * LP, bi, bj, acc);
        blk_store(a, Cp + dr, Cp + dc, bi, bj, acc);
      }
    }
  }
}

// Returns info (0 or the 1-based failing column).
__device__ int64_t walk_factor(const Band a, const int K, const WalkLds L, lds_i* s_fail, lds_i* s_sync) {
  const int wave = wave_id();
  const int64_t NB = (a.n + T - 1) / T;
  if (threadIdx.x == 0) { *s_fail = -1; *s_sync = 0; }
  // stage tile (0, 0)
  if (wave >= 1) {
    const int bi = (wave >= 2), bj = (wave == 3);
    blk_to_lds(L.diag, bi, bj, blk_load(a, 0, 0, bi, bj));
  } else {
    blk_to_lds(L.diag, 0, 1, d4{0, 0, 0, 0});
  }
  __syncthreads();
  int sync_target = 0;
  for (int64_t C = 0; C < NB; ++C) {
    lds_d* lt = L.linvt + (C & 1) * T * T;
    const lds_d* lt_prev = L.linvt + ((C + 1) & 1) * T * T;
    // ---------------- phase A
    if (wave == 0) walk_sweep(a, C, L, lt, s_fail);
    else if (C >= 1) walk_column_rest(a, K, NB, C - 1, L, lt_prev, s_sync, sync_target += 3);
    wait_vmem();
    __syncthreads();
    if (*s_fail >= 0) return C * T + *s_fail + 1;
    if (C + 1 >= NB) break;
    // ---------------- phase B: trsm of tile (C+1, C)
    if (K >= 1) {
      const int bi = wave & 1, bj = wave >> 1;
      double x[T / 4];
      rowblk_load(a, C + 1, C, bi, x);
      wait_vmem();
      __syncthreads();   // every wave holds its input before any output is written
      const d4 out = blk_trsm_frag(x, lt, bj);
      blk_to_lds(L.pnl, bi, bj, out);
      blk_store(a, C + 1, C, bi, bj, out);
    }
    wait_vmem();
    __syncthreads();
    // ---------------- phase C: stage tile (C+1, C+1) minus the critical update
    if (wave >= 1) {
      const int bi = (wave >= 2), bj = (wave == 3);
      d4 acc = blk_load(a, C + 1, C + 1, bi, bj);
      if (K >= 1) acc = blk_gemm_lds(L.pnl, L.pnl, bi, bj, acc);
      blk_to_lds(L.diag, bi, bj, acc);
    } else {
      blk_to_lds(L.diag, 0, 1, d4{0, 0, 0, 0});
    }
    __syncthreads();
  }
  return 0;
}

struct WalkSys {
  double* ab;
  int64_t n, k, ldab;
};

__global__ void __launch_bounds__(NT) walk_single_kernel(WalkSys w, int K, int64_t* info) {
  extern __shared__ double lds_dyn[];
  __shared__ int s_fail, s_sync;
  const Band a{(glb_d*)w.ab, w.n, w.k, w.ldab};
  const int64_t res = walk_factor(a, K, walk_lds((lds_d*)lds_dyn, K), (lds_i*)&s_fail, (lds_i*)&s_sync);
  if (threadIdx.x == 0) *info = res;
}

// Persistent: each workgroup takes systems from the queue in the given order.
__global__ void __launch_bounds__(NT) walk_kernel(const WalkSys* sys, const int* order, int nsys, int Kmax,
                                                  unsigned* queue, int64_t* info) {
  extern __shared__ double lds_dyn[];
  __shared__ int s_idx, s_fail, s_sync;
  for (;;) {
    if (threadIdx.x == 0) s_idx = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int t = s_idx;
    if (t >= nsys) break;
    const int id = order ? order[t] : t;
    const WalkSys w = sys[id];
    const int64_t kk = w.k < w.n - 1 ? w.k : (w.n > 0 ? w.n - 1 : 0);
    int K = (int)((kk + T - 1) / T);
    const Band a{(glb_d*)w.ab, w.n, kk, w.ldab};
    int64_t res = 0;
    if (w.n > 0) res = walk_factor(a, K, walk_lds((lds_d*)lds_dyn, Kmax), (lds_i*)&s_fail, (lds_i*)&s_sync);
    if (threadIdx.x == 0) info[id] = res;
    __syncthreads();
  }
}

// ----------------------------------------------------------------- host runtime

thread_local char g_err[512] = "";
thread_local hipStream_t g_stream = nullptr;

void set_err(const char* what, hipError_t e) {
  snprintf(g_err, sizeof g_err, "%s: %s", what, hipGetErrorString(e));
}

struct DevWork {
  void* ptr = nullptr;
  size_t size = 0;
  void* info_host = nullptr;  // pinned int64 for the synchronous calls
  void* info_dev = nullptr;   // device int64 for the synchronous calls (never reallocated)
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

struct FactorLayout {
  int NB, K;
  size_t off_flags, off_linvt, off_misc, total;
};

FactorLayout factor_layout(int64_t n, int64_t k) {
  FactorLayout L;
  L.NB = (int)((n + T - 1) / T);
  L.K = (int)((k + T - 1) / T);
  if (L.K > L.NB - 1) L.K = L.NB - 1 > 0 ? L.NB - 1 : 0;
  L.off_misc = 0;                                   // queue, abort, first_fail, info
  L.off_flags = align_up(64);
  L.off_linvt = align_up(L.off_flags + sizeof(int) * (size_t)L.NB * (L.K + 1));
  L.total = align_up(L.off_linvt + sizeof(double) * (size_t)L.NB * T * T);
  return L;
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
    g_walk_kmax = 2;
    if (const char* e = getenv("BANDCHOL_WALK_KMAX")) g_walk_kmax = (int)strtol(e, nullptr, 10);
    if (g_walk_kmax > WALK_KMAX) g_walk_kmax = WALK_KMAX;
  }
  return g_walk_kmax;
}

bool use_spine() {
  static int v = -1;
  if (v < 0) {
    const char* e = getenv("BANDCHOL_SCHEDULE");
    v = (e && strcmp(e, "tiles") == 0) ? 0 : 1;
  }
  return v == 1;
}

hipError_t walk_attr(size_t lds) {
  static size_t done = 0;
  if (lds <= done) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)walk_single_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)walk_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) done = lds;
  return e;
}

int64_t factor_async_impl(int64_t n, int64_t k, double* ab, int64_t ldab, int64_t* d_info, hipStream_t st) {
  if (n < 0) return -1;
  if (k < 0) return -2;
  if (ab == nullptr && n > 0) return -3;
  if (ldab < k + 1) return -4;
  if (d_info == nullptr) return -5;
  if (n > ((int64_t)1 << 31) - T) {
    snprintf(g_err, sizeof g_err, "n too large");
    return -1;
  }
  hipError_t e;
  const FactorLayout L = factor_layout(n, k);
  if (n > 0 && L.K <= walk_kmax()) {
    const int64_t kk = k < n - 1 ? k : n - 1;
    const size_t lds = walk_lds_bytes(L.K);
    e = walk_attr(lds);
    if (e != hipSuccess) { set_err("walk attributes", e); return BANDCHOL_EHIP; }
    walk_single_kernel<<<1, NT, lds, st>>>(WalkSys{ab, n, kk, ldab}, L.K, d_info);
    e = hipGetLastError();
    if (e != hipSuccess) { set_err("factor launch", e); return BANDCHOL_EHIP; }
    return 0;
  }
  if (n > 0 && use_spine()) {
    void* w2 = workspace(bandchol_factor2_workspace(n, L.K), &e);
    if (!w2) { set_err("workspace", e); return BANDCHOL_EHIP; }
    int grid = num_cus() * 2;
    if (const char* cap = getenv("BANDCHOL_MAX_WG")) {
      const long v = strtol(cap, nullptr, 10);
      if (v > 0 && v < grid) grid = (int)v;
    }
    e = bandchol_factor2_launch(n, k, ab, ldab, d_info, w2, grid, st);
    if (e != hipSuccess) { set_err("factor launch", e); return BANDCHOL_EHIP; }
    return 0;
  }
  char* ws = (char*)workspace(L.total, &e);
  if (!ws) { set_err("workspace", e); return BANDCHOL_EHIP; }
  unsigned* queue = (unsigned*)(ws + 0);
  int* abort_flag = (int*)(ws + 8);
  unsigned long long* first_fail = (unsigned long long*)(ws + 16);
  int* flags = (int*)(ws + L.off_flags);
  const int64_t nflags = (int64_t)L.NB * (L.K + 1);
  factor_init_kernel<<<(unsigned)((nflags + 255) / 256 > 1024 ? 1024 : (nflags + 255) / 256 + 1), 256, 0, st>>>(
      flags, nflags, queue, abort_flag, first_fail);
  if (n > 0) {
    FactorParams P;
    P.a = Band{(glb_d*)ab, n, k, ldab};
    P.NB = L.NB;
    P.K = L.K;
    P.ntasks = (unsigned)((int64_t)L.NB * (L.K + 1));
    P.w = Work{flags, (double*)(ws + L.off_linvt), queue, abort_flag, first_fail};
    int64_t grid = (int64_t)num_cus() * 4;
    if (const char* cap = getenv("BANDCHOL_MAX_WG")) {
      const long v = strtol(cap, nullptr, 10);
      if (v > 0 && v < grid) grid = v;
    }
    if (grid > (int64_t)P.ntasks) grid = P.ntasks;
    if (grid < 1) grid = 1;
    factor_kernel<<<(unsigned)grid, NT, 0, st>>>(P);
  }
  factor_finish_kernel<<<1, 1, 0, st>>>(abort_flag, first_fail, d_info);
  e = hipGetLastError();
  if (e != hipSuccess) { set_err("factor launch", e); return BANDCHOL_EHIP; }
  return 0;
}

int64_t solve_async_impl(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, double* b,
                         int64_t ldb, hipStream_t st) {
  if (n < 0) return -1;
  if (k < 0) return -2;
  if (nrhs < 0) return -3;
  if (ab == nullptr && n > 0) return -4;
  if (ldab < k + 1) return -5;
  if (b == nullptr && n > 0 && nrhs > 0) return -6;
  if (ldb < (n > 1 ? n : 1)) return -7;
  if (n == 0 || nrhs == 0) return 0;
  const int64_t kk = k < n - 1 ? k : n - 1;
  hipError_t e;
  void* ws = workspace(bandchol_solve_workspace(n), &e);
  if (!ws) { set_err("workspace", e); return BANDCHOL_EHIP; }
  e = bandchol_solve_launch(n, kk, nrhs, ab, ldab, b, ldb, ws, num_cus(), st);
  if (e != hipSuccess) { set_err("solve launch", e); return BANDCHOL_EHIP; }
  return 0;
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
  int64_t rc = solve_async_impl(n, k, nrhs, ab, ldab, b, ldb, g_stream);
  if (rc != 0 || n == 0 || nrhs == 0) return rc;
  hipError_t e = hipStreamSynchronize(g_stream);
  if (e != hipSuccess) { set_err("solve", e); return BANDCHOL_EHIP; }
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
    g_work[d] = DevWork();
  }
  (void)hipSetDevice(cur);
}

int64_t bandchol_tile(void) { return T; }

int64_t bandchol_set_walk_limit(int64_t kmax) {
  const int64_t prev = walk_kmax();
  if (kmax < 0) return prev;
  g_walk_kmax = (int)(kmax > WALK_KMAX ? WALK_KMAX : kmax);
  return prev;
}

}  // extern "C"
