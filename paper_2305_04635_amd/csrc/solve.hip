// Band solves with the factor: forward L Y = B, then back L^T X = Y (gfx950, FP64).
//
// Both directions walk the band in T-row blocks and form each block from the
// previous (or next) K blocks.  One workgroup (the spine, whoever takes ticket
// 0) carries the dependency chain: for block R it applies the contributions of
// the nearest ST blocks itself, then multiplies by the inverse of the diagonal
// tile.  Helper workgroups take the other tickets and pre-accumulate, for each
// block, the contributions of all blocks further away, as soon as those are
// published.  Blocks, partial sums and ready flags pass between workgroups
// through relaxed agent-scope atomic loads and stores (coherent at device
// scope without cache flushes); a flag is raised only after the data stores
// have completed.
#include <stdint.h>

#include "common.h"

namespace bandchol_solve {

using namespace bandchol;

constexpr int NT = 256;
constexpr int ST = 6;            // blocks handled by the spine itself
constexpr int RHS_MAX = 16;      // right-hand sides per launch
constexpr long long SPIN_LIMIT = 1LL << 26;

struct SolveWork {
  int* flag_y;      // NB, block of the result published
  int* flag_z;      // NB, helper partial sum published
  double* z;        // NB * nrhs * T partial sums
  unsigned* queue;  // ticket counter
  int* abort_flag;  // 2 = a wait exceeded its bound
};

struct SolveArgs {
  Band a;
  int NB, K, nrhs;
  const double* dinvt;   // per block, L(C,C)^{-T} row-major
  double* b;
  int64_t ldb;
  SolveWork w;
};

__device__ __forceinline__ double aload(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void astore(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int aflag(const int* p) {
  return __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Thread 0 waits for *f != 0; the result is uniform over the workgroup.
__device__ bool wg_wait(const int* f, int* abort_flag, lds_i* s_ok) {
  if (threadIdx.x == 0) {
    int ok = 1;
    long long spins = 0;
    while (!aflag(f)) {
      if (aflag(abort_flag)) { ok = 0; break; }
      if (++spins > SPIN_LIMIT) {
        __hip_atomic_store(abort_flag, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    *s_ok = ok;
  }
  __syncthreads();
  const int ok = *s_ok;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");  // no load hoisted above the wait
  return ok != 0;
}

__device__ void wg_raise(int* f) {
  wait_vmem();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double red8(double s) {
  s += __shfl_xor(s, 1);
  s += __shfl_xor(s, 2);
  s += __shfl_xor(s, 4);
  return s;
}

// ---------------------------------------------------------------- forward

// y_R = L(R,R)^{-1} (b_R - z_R - sum_{d=1..ST} L(R,R-d) y_{R-d})
__device__ void fwd_spine(const SolveArgs& S, lds_d* ring, lds_d* tl, lds_i* s_ok) {
  const Band& a = S.a;
  const int tid = threadIdx.x, i = tid >> 3, p = tid & 7;
  const int nd = S.K < ST ? S.K : ST;
  for (int R = 0; R < S.NB; ++R) {
    double lf[ST][4], df[4];
#pragma unroll
    for (int d = 1; d <= ST; ++d)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        lf[d - 1][q] = (d <= nd && R - d >= 0) ? a.ld((int64_t)R * T + i, (int64_t)(R - d) * T + 4 * p + q) : 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) df[q] = S.dinvt[(int64_t)R * T * T + (4 * p + q) * T + i];
    const bool has_z = S.K > ST && R > ST;
    if (has_z && !wg_wait(&S.w.flag_z[R], S.w.abort_flag, s_ok)) return;
    const int64_t row = (int64_t)R * T + i;
    for (int r = 0; r < S.nrhs; ++r) {
      double s = 0.0;
#pragma unroll
      for (int d = 1; d <= ST; ++d) {
        if (d > nd || R - d < 0) continue;
        const lds_d* yp = ring + ((R - d) % (ST + 1)) * (T * RHS_MAX) + r * T + 4 * p;
#pragma unroll
        for (int q = 0; q < 4; ++q) s = fma(lf[d - 1][q], yp[q], s);
      }
      s = red8(s);
      if (p == 0) {
        double t = row < a.n ? S.b[r * S.ldb + row] : 0.0;
        if (has_z) t -= aload(S.w.z + ((int64_t)R * S.nrhs + r) * T + i);
        tl[r * T + i] = t - s;
      }
    }
    __syncthreads();
    lds_d* ycur = ring + (R % (ST + 1)) * (T * RHS_MAX);
    for (int r = 0; r < S.nrhs; ++r) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) s = fma(df[q], tl[r * T + 4 * p + q], s);
      s = red8(s);
      if (p == 0) {
        ycur[r * T + i] = s;
        if (row < a.n) astore(S.b + r * S.ldb + row, s);
      }
    }
    wg_raise(&S.w.flag_y[R]);
  }
}

// z_R = sum_{C = R-K}^{R-ST-1} L(R,C) y_C
__device__ void fwd_helper(const SolveArgs& S, int R, lds_i* s_ok) {
  const Band& a = S.a;
  const int tid = threadIdx.x, i = tid >> 3, p = tid & 7;
  const int c0 = R - S.K > 0 ? R - S.K : 0;
  for (int r0 = 0; r0 < S.nrhs; r0 += 8) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int C = c0; C <= R - ST - 1; ++C) {
      if (!wg_wait(&S.w.flag_y[C], S.w.abort_flag, s_ok)) return;
      double lf[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) lf[q] = a.ld((int64_t)R * T + i, (int64_t)C * T + 4 * p + q);
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) {
        if (r0 + rr >= S.nrhs) break;
        const double* yc = S.b + (r0 + rr) * S.ldb + (int64_t)C * T + 4 * p;
        const int64_t rowc = (int64_t)C * T + 4 * p;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (rowc + q < a.n) acc[rr] = fma(lf[q], aload(yc + q), acc[rr]);
      }
    }
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) {
      if (r0 + rr >= S.nrhs) break;
      const double s = red8(acc[rr]);
      if (p == 0) astore(S.w.z + ((int64_t)R * S.nrhs + r0 + rr) * T + i, s);
    }
  }
  wg_raise(&S.w.flag_z[R]);
}

// ---------------------------------------------------------------- back

// x_C = L(C,C)^{-T} (y_C - z_C - sum_{d=1..ST} L(C+d,C)^T x_{C+d})
__device__ void bwd_spine(const SolveArgs& S, lds_d* ring, lds_d* tl, lds_i* s_ok) {
  const Band& a = S.a;
  const int tid = threadIdx.x, c = tid >> 3, p = tid & 7;
  const int nd = S.K < ST ? S.K : ST;
  for (int C = S.NB - 1; C >= 0; --C) {
    double lf[ST][4], df[4];
#pragma unroll
    for (int d = 1; d <= ST; ++d)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        lf[d - 1][q] = (d <= nd && C + d < S.NB) ? a.ld((int64_t)(C + d) * T + 4 * p + q, (int64_t)C * T + c) : 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) df[q] = S.dinvt[(int64_t)C * T * T + c * T + 4 * p + q];
    const bool has_z = S.K > ST && C + ST + 1 < S.NB;
    if (has_z && !wg_wait(&S.w.flag_z[C], S.w.abort_flag, s_ok)) return;
    const int64_t col = (int64_t)C * T + c;
    for (int r = 0; r < S.nrhs; ++r) {
      double s = 0.0;
#pragma unroll
      for (int d = 1; d <= ST; ++d) {
        if (d > nd || C + d >= S.NB) continue;
        const lds_d* xp = ring + ((C + d) % (ST + 1)) * (T * RHS_MAX) + r * T + 4 * p;
#pragma unroll
        for (int q = 0; q < 4; ++q) s = fma(lf[d - 1][q], xp[q], s);
      }
      s = red8(s);
      if (p == 0) {
        double t = col < a.n ? S.b[r * S.ldb + col] : 0.0;
        if (has_z) t -= aload(S.w.z + ((int64_t)C * S.nrhs + r) * T + c);
        tl[r * T + c] = t - s;
      }
    }
    __syncthreads();
    lds_d* xcur = ring + (C % (ST + 1)) * (T * RHS_MAX);
    for (int r = 0; r < S.nrhs; ++r) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) s = fma(df[q], tl[r * T + 4 * p + q], s);
      s = red8(s);
      if (p == 0) {
        xcur[r * T + c] = s;
        if (col < a.n) astore(S.b + r * S.ldb + col, s);
      }
    }
    wg_raise(&S.w.flag_y[C]);
  }
}

// z_C = sum_{R = C+ST+1}^{C+K} L(R,C)^T x_R
__device__ void bwd_helper(const SolveArgs& S, int C, lds_i* s_ok) {
  const Band& a = S.a;
  const int tid = threadIdx.x, c = tid >> 3, p = tid & 7;
  const int r1 = C + S.K < S.NB - 1 ? C + S.K : S.NB - 1;
  for (int r0 = 0; r0 < S.nrhs; r0 += 8) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int R = C + ST + 1; R <= r1; ++R) {
      if (!wg_wait(&S.w.flag_y[R], S.w.abort_flag, s_ok)) return;
      double lf[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) lf[q] = a.ld((int64_t)R * T + 4 * p + q, (int64_t)C * T + c);
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) {
        if (r0 + rr >= S.nrhs) break;
        const double* xr = S.b + (r0 + rr) * S.ldb + (int64_t)R * T + 4 * p;
        const int64_t rowr = (int64_t)R * T + 4 * p;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (rowr + q < a.n) acc[rr] = fma(lf[q], aload(xr + q), acc[rr]);
      }
    }
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) {
      if (r0 + rr >= S.nrhs) break;
      const double s = red8(acc[rr]);
      if (p == 0) astore(S.w.z + ((int64_t)C * S.nrhs + r0 + rr) * T + c, s);
    }
  }
  wg_raise(&S.w.flag_z[C]);
}

// ---------------------------------------------------------------- kernels

template <bool FWD>
__global__ void __launch_bounds__(NT) solve_kernel(SolveArgs S) {
  __shared__ double ring[(ST + 1) * T * RHS_MAX];
  __shared__ double tl[T * RHS_MAX];
  __shared__ int s_ticket, s_ok;
  const int nhelp = (S.K > ST) ? (FWD ? S.NB - ST - 1 : S.NB - ST - 1) : 0;
  for (;;) {
    if (threadIdx.x == 0) s_ticket = (int)atomicAdd(S.w.queue, 1u);
    __syncthreads();
    const int t = s_ticket;
    __syncthreads();
    if (t > nhelp) break;
    if (t == 0) {
      if (FWD) fwd_spine(S, (lds_d*)ring, (lds_d*)tl, (lds_i*)&s_ok);
      else bwd_spine(S, (lds_d*)ring, (lds_d*)tl, (lds_i*)&s_ok);
    } else if (FWD) {
      fwd_helper(S, ST + t, (lds_i*)&s_ok);            // R = ST+1 .. NB-1
    } else {
      bwd_helper(S, S.NB - ST - 1 - t, (lds_i*)&s_ok);  // C = NB-ST-2 .. 0
    }
    if (aflag(S.w.abort_flag)) break;
  }
}

__global__ void solve_clear_kernel(int* flags, int64_t count, unsigned* queue, int* abort_flag) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t x = g; x < count; x += (int64_t)gridDim.x * blockDim.x) flags[x] = 0;
  if (g == 0) { *queue = 0; *abort_flag = 0; }
}

// Per diagonal tile, L(C,C)^{-T} (row-major): lanes 0..T-1 hold the rows of
// L(C,C), lanes T..2T-1 the identity rows, solved against L(C,C) column by column.
__global__ void __launch_bounds__(64) tri_inv_kernel(Band a, int NB, double* dinvt) {
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
    const double y = recip(readlane_d(row[j], j));
    const double x = rhs ? row[j] * y : row[j];
    row[j] = x;
#pragma unroll
    for (int l = j + 1; l < T; ++l) {
      const double llj = readlane_d(x, l);
      row[l] = rhs ? fma(-x, llj, row[l]) : row[l];
    }
  }
  if (rhs) {
#pragma unroll
    for (int c = 0; c < T; ++c) dinvt[(int64_t)C * T * T + (lane - T) * T + c] = row[c];
  }
}

}  // namespace bandchol_solve

// Host side, called by the C-ABI (same library).  Workspace layout, in bytes
// from `ws`: [0,64) queue + abort; flags 2*NB ints; z NB*RHS_MAX*T doubles;
// dinvt NB*T*T doubles.
size_t bandchol_solve_workspace(int64_t n) {
  using namespace bandchol_solve;
  const int64_t NB = (n + T - 1) / T;
  return 256 + ((sizeof(int) * 2 * NB + 255) & ~(size_t)255) + sizeof(double) * (size_t)NB * RHS_MAX * T +
         sizeof(double) * (size_t)NB * T * T;
}

hipError_t bandchol_solve_launch(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, double* b,
                                 int64_t ldb, void* ws, int num_cus, hipStream_t st) {
  using namespace bandchol_solve;
  const int NB = (int)((n + T - 1) / T);
  int K = (int)((k + T - 1) / T);
  if (K > NB - 1) K = NB - 1 > 0 ? NB - 1 : 0;
  char* base = (char*)ws;
  unsigned* queue = (unsigned*)base;
  int* abort_flag = (int*)(base + 8);
  int* flags = (int*)(base + 256);
  const size_t off_z = 256 + ((sizeof(int) * 2 * (size_t)NB + 255) & ~(size_t)255);
  double* z = (double*)(base + off_z);
  double* dinvt = z + (size_t)NB * RHS_MAX * T;
  const Band a{(glb_d*)const_cast<double*>(ab), n, k, ldab};
  tri_inv_kernel<<<NB, 64, 0, st>>>(a, NB, dinvt);
  const int nhelp = K > ST ? NB - ST - 1 : 0;
  int grid = 1 + (nhelp < num_cus * 2 ? nhelp : num_cus * 2);
  for (int64_t r0 = 0; r0 < nrhs; r0 += RHS_MAX) {
    const int nr = (int)(nrhs - r0 < RHS_MAX ? nrhs - r0 : RHS_MAX);
    SolveArgs S{a, NB, K, nr, dinvt, b + r0 * ldb, ldb, SolveWork{flags, flags + NB, z, queue, abort_flag}};
    solve_clear_kernel<<<(2 * NB + 255) / 256 + 1, 256, 0, st>>>(flags, 2 * (int64_t)NB, queue, abort_flag);
    solve_kernel<true><<<grid, NT, 0, st>>>(S);
    solve_clear_kernel<<<(2 * NB + 255) / 256 + 1, 256, 0, st>>>(flags, 2 * (int64_t)NB, queue, abort_flag);
    solve_kernel<false><<<grid, NT, 0, st>>>(S);
  }
  return hipGetLastError();
}
