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

namespace {

constexpr int T = 32;        // tile width
constexpr int NT = 256;      // threads per workgroup (4 waves)
constexpr int LP = T + 1;    // LDS pitch of a staged tile (column-major)
constexpr long long SPIN_LIMIT = 1LL << 25;

typedef double d4 __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------- device helpers

__device__ __forceinline__ double readlane_d(double v, int lane) {
  int2 p = __builtin_bit_cast(int2, v);
  p.x = __builtin_amdgcn_readlane(p.x, lane);
  p.y = __builtin_amdgcn_readlane(p.y, lane);
  return __builtin_bit_cast(double, p);
}

// One 16x16x4 FP64 MFMA step of D += X Y^T restricted to a 16x16 block, where
// xf and yf are the fragments "lane l holds M[16*blk + l%16][k0 + l/16]" of X
// and Y.  The accumulator then holds, in lane l and register r, the block
// element (row l%16, column 4r + l/16): consecutive lanes are consecutive rows,
// which in the column-major band layout are consecutive addresses.
#ifndef BANDCHOL_MFMA_SWAP
#define BANDCHOL_MFMA_SWAP 1
#endif
__device__ __forceinline__ d4 mfma_xyt(double xf, double yf, d4 acc) {
#if BANDCHOL_MFMA_SWAP
  return __builtin_amdgcn_mfma_f64_16x16x4f64(yf, xf, acc, 0, 0, 0);
#else
  return __builtin_amdgcn_mfma_f64_16x16x4f64(xf, yf, acc, 0, 0, 0);
#endif
}

struct Band {
  double* ab;
  int64_t n, k, ldab;
  __device__ __forceinline__ bool in_band(int64_t i, int64_t j) const {
    int64_t d = i - j;
    return i < n && d >= 0 && d <= k;
  }
  __device__ __forceinline__ double ld(int64_t i, int64_t j) const {
    return in_band(i, j) ? ab[(i - j) + j * ldab] : 0.0;
  }
};

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
__device__ bool wg_wait(const int* f1, const int* f2, const Work& w, int* s_ok) {
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

__device__ __forceinline__ void acc_to_lds(double* lds, int bi, int bj, d4 acc) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < 4; ++r) lds[(16 * bj + 4 * r + (lane >> 4)) * LP + 16 * bi + (lane & 15)] = acc[r];
}

// Dense Cholesky of the staged diagonal tile (lanes 0..T-1 = its rows) with
// the identity rows in lanes T..2T-1 swept along: afterwards lane i < T holds
// row i of L and lane T+b holds row b of L^{-T}.  Right-looking, one column
// per step; the column of L is broadcast with readlane.  Returns the first
// failing local column or -1.
__device__ int sweep_potrf(double (&row)[T]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < T; ++j) {
    const double d = readlane_d(row[j], j);
    if (!(d > 0.0)) return j;
    const double r = sqrt(d);
    const double y = 1.0 / r;
    const double lij = (lane == j) ? r : row[j] * y;
    row[j] = lij;
#pragma unroll
    for (int l = j + 1; l < T; ++l) row[l] = fma(-lij, readlane_d(lij, l), row[l]);
  }
  return -1;
}

// Each task body is compiled on its own (noinline) so that the two term loops
// are never merged into one.
__device__ __attribute__((noinline)) void diag_task(const FactorParams& P, int C, double* lds, int* s_ok) {
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
    const int fail = sweep_potrf(row);
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

__device__ __attribute__((noinline)) void off_task(const FactorParams& P, int R, int C, double* lds, int* s_ok) {
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
      if (d == 0) diag_task(P, C, lds, &s_ok);
      else off_task(P, C + d, C, lds, &s_ok);
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

// ----------------------------------------------------------------- solves

// Per diagonal tile, L(C,C)^{-T} (row-major) from the factor: lanes 0..T-1
// hold the rows of L(C,C), lanes T..2T-1 the identity rows, which are solved
// against L(C,C) column by column.
__global__ void __launch_bounds__(64) solve_tri_inv_kernel(Band a, int NB, double* dinvt) {
  const int C = blockIdx.x, lane = threadIdx.x;
  double row[T];
  const int64_t i = (int64_t)C * T + lane;
#pragma unroll
  for (int c = 0; c < T; ++c) {
    const int64_t j = (int64_t)C * T + c;
    if (lane < T) row[c] = (i >= a.n && i == j) ? 1.0 : a.ld(i, j);
    else row[c] = ((lane - T) == c) ? 1.0 : 0.0;
  }
  const bool rhs = lane >= T;
#pragma unroll
  for (int j = 0; j < T; ++j) {
    const double y = 1.0 / readlane_d(row[j], j);
    const double x = rhs ? row[j] * y : row[j];   // lanes < T keep L
    row[j] = x;
#pragma unroll
    for (int l = j + 1; l < T; ++l) {
      const double llj = readlane_d(x, l);          // L(l, j), from lane l < T
      row[l] = rhs ? fma(-x, llj, row[l]) : row[l];
    }
  }
  if (lane >= T) {
#pragma unroll
    for (int c = 0; c < T; ++c) dinvt[(int64_t)C * T * T + (lane - T) * T + c] = row[c];
  }
}

// Forward solve L y = b for one right-hand side per workgroup.  The rows
// [C*T, C*T+T+k) that still receive updates live in an LDS ring of W slots.
__global__ void __launch_bounds__(NT) solve_fwd_kernel(Band a, int NB, const double* dinvt, double* b, int64_t ldb,
                                                      int W) {
  extern __shared__ double ring[];
  __shared__ double ys[T];
  double* bc = b + (int64_t)blockIdx.x * ldb;
  const int tid = threadIdx.x;
  const int64_t n = a.n, k = a.k;
  const int64_t first = (T + k < n) ? T + k : n;
  for (int64_t r = tid; r < first; r += NT) ring[r & (W - 1)] = bc[r];
  __syncthreads();
  for (int C = 0; C < NB; ++C) {
    const int64_t c0 = (int64_t)C * T;
    const double* lt = dinvt + (int64_t)C * T * T;
    {  // y_C = L(C,C)^{-1} b_C: y[i] = sum_c Linvt[c][i] b[c]; 8 lanes per row
      const int i = tid >> 3, p = tid & 7;
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < T / 8; ++q) {
        const int c = p * (T / 8) + q;
        const double bv = (c0 + c < n) ? ring[(c0 + c) & (W - 1)] : 0.0;
        s = fma(lt[c * T + i], bv, s);
      }
      s += __shfl_xor(s, 1);
      s += __shfl_xor(s, 2);
      s += __shfl_xor(s, 4);
      if (p == 0) {
        ys[i] = s;
        if (c0 + i < n) bc[c0 + i] = s;
      }
    }
    __syncthreads();
    // rows [c0+T, c0+T+k) -= L(r, c0+c) y_c
    const int64_t rlo = c0 + T, rhi = (c0 + T + k < n) ? c0 + T + k : n;
    for (int64_t r = rlo + tid; r < rhi; r += NT) {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int c = 0; c < T; c += 2) {
        s0 = fma(a.ld(r, c0 + c), ys[c], s0);
        s1 = fma(a.ld(r, c0 + c + 1), ys[c + 1], s1);
      }
      ring[r & (W - 1)] -= s0 + s1;
    }
    // rows entering the window for the next tile
    const int64_t elo = c0 + T + k, ehi = (c0 + 2 * T + k < n) ? c0 + 2 * T + k : n;
    for (int64_t r = elo + tid; r < ehi; r += NT) ring[r & (W - 1)] = bc[r];
    __syncthreads();
  }
}

// Back solve L^T x = y, tiles in descending order.  x_C = L(C,C)^{-T} (y_C - z)
// with z_c = sum_{r >= (C+1)T} L(r, c0+c) x_r; the known x of the next k rows
// live in the LDS ring.
__global__ void __launch_bounds__(NT) solve_bwd_kernel(Band a, int NB, const double* dinvt, double* b, int64_t ldb,
                                                      int W) {
  extern __shared__ double ring[];
  __shared__ double zs[T];
  double* bc = b + (int64_t)blockIdx.x * ldb;
  const int tid = threadIdx.x;
  const int64_t n = a.n, k = a.k;
  for (int C = NB - 1; C >= 0; --C) {
    const int64_t c0 = (int64_t)C * T;
    const double* lt = dinvt + (int64_t)C * T * T;
    {  // z_c = y_c - sum_r L(r, c0+c) x_r over r in [c0+T, c0+c+k]
      const int c = tid >> 3, p = tid & 7;
      const int64_t j = c0 + c;
      const int64_t rlo = c0 + T;
      int64_t rhi = j + k + 1;
      if (rhi > n) rhi = n;
      double s = 0.0;
      for (int64_t r = rlo + p; r < rhi; r += 8) s = fma(a.ld(r, j), ring[r & (W - 1)], s);
      s += __shfl_xor(s, 1);
      s += __shfl_xor(s, 2);
      s += __shfl_xor(s, 4);
      if (p == 0) zs[c] = (j < n) ? bc[j] - s : 0.0;
    }
    __syncthreads();
    {  // x_C[i] = sum_c Linvt[i][c] z[c]
      const int i = tid >> 3, p = tid & 7;
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < T / 8; ++q) {
        const int c = p * (T / 8) + q;
        s = fma(lt[i * T + c], zs[c], s);
      }
      s += __shfl_xor(s, 1);
      s += __shfl_xor(s, 2);
      s += __shfl_xor(s, 4);
      if (p == 0 && c0 + i < n) {
        ring[(c0 + i) & (W - 1)] = s;
        bc[c0 + i] = s;
      }
    }
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
  if (!w.info_host) {
    *err = hipHostMalloc(&w.info_host, 64, hipHostMallocDefault);
    if (*err != hipSuccess) { w.info_host = nullptr; return nullptr; }
  }
  return w.ptr;
}

int64_t* info_host() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return (int)g_work.size() > dev ? (int64_t*)g_work[dev].info_host : nullptr;
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
    P.a = Band{ab, n, k, ldab};
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
  const int NB = (int)((n + T - 1) / T);
  int64_t kk = k < n - 1 ? k : n - 1;
  int64_t W = 1;
  while (W < kk + 2 * T) W <<= 1;
  if (W > 8192) {
    snprintf(g_err, sizeof g_err, "bandwidth too large for the solve window (k <= %d)", 8192 - 2 * T);
    return -2;
  }
  hipError_t e;
  const size_t need = align_up(sizeof(double) * (size_t)NB * T * T);
  // the solve uses the top of the same per-device workspace after the factor's part
  const FactorLayout L = factor_layout(n, k);
  char* ws = (char*)workspace(L.total + need, &e);
  if (!ws) { set_err("workspace", e); return BANDCHOL_EHIP; }
  double* dinvt = (double*)(ws + L.total);
  Band a{const_cast<double*>(ab), n, kk, ldab};
  solve_tri_inv_kernel<<<NB, 64, 0, st>>>(a, NB, dinvt);
  solve_fwd_kernel<<<(unsigned)nrhs, NT, W * sizeof(double), st>>>(a, NB, dinvt, b, ldb, (int)W);
  solve_bwd_kernel<<<(unsigned)nrhs, NT, W * sizeof(double), st>>>(a, NB, dinvt, b, ldb, (int)W);
  e = hipGetLastError();
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
  const FactorLayout L = factor_layout(n, k);
  char* ws = (char*)workspace(L.total, &e);
  if (!ws) { set_err("workspace", e); return BANDCHOL_EHIP; }
  int64_t* d_info = (int64_t*)(ws + 24);
  int64_t rc = factor_async_impl(n, k, ab, ldab, d_info, g_stream);
  if (rc != 0) return rc;
  int64_t* h = info_host();
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
    if (g_work[d].ptr) {
      (void)hipDeviceSynchronize();
      (void)hipFree(g_work[d].ptr);
    }
    if (g_work[d].info_host) (void)hipHostFree(g_work[d].info_host);
    g_work[d] = DevWork();
  }
  (void)hipSetDevice(cur);
}

int64_t bandchol_tile(void) { return T; }

}  // extern "C"
