// Reverse mode of the band factorization (gfx950, FP64): given the factor L of
// A and an upstream gradient Lbar of a loss with respect to L, the gradient
// Abar with respect to the stored band of A.
//
// The forward factorization, in tiles (Algorithm 1, Section 3), does for each
// tile column C: M = L(C,C) = chol of the diagonal tile (potrf); L(R,C) =
// A(R,C) M^{-T} for the tiles below (trsm); A(R,S) -= L(R,C) L(S,C)^T for the
// trailing tiles C < S <= R <= C+K (gemm, syrk).  Its reverse walks the tile
// columns backwards.  W(R,S) denotes the running adjoint of tile (R,S); once
// column S has been reversed it holds Abar(R,S), which is also the adjoint of
// every updated version of A(R,S) (the updates only subtract).  Step C:
//
//   (update)  G(R) = Lbar(R,C) - sum_{C<S<R} Abar(R,S) L(S,C)
//                  - sym(Abar(R,R)) L(R,C) - sum_{R<S<=C+K} Abar(S,R)^T L(S,C),
//             sym(X) = tril(X) + tril(X)^T (the diagonal tile holds its lower
//             triangle only, so its update's adjoint counts it twice);
//   (trsm)    Abar(R,C) = G(R) M^{-1},   Mbar -= tril(Abar(R,C)^T L(R,C));
//   (potrf)   Mbar starts as tril(Lbar(C,C)); with S = M^{-T} Phi(M^T Mbar) M^{-1},
//             Phi = lower triangle with half the diagonal, Abar(C,C) =
//             tril(S + S^T) - diag(S) (a stored entry i > j stands for
//             A(i,j) and A(j,i); the diagonal once).
//
// Schedule: workgroups of one system take the tiles R of a step (one tile
// each, four waves on its four 16 x 16 blocks); workgroup 0 then reduces the
// per-tile contributions to Mbar and reverses the diagonal tile.  One grid
// barrier per step (release/acquire at agent scope) separates the two; the
// only result of the diagonal work the next step needs is Abar(C,C), for the
// tile R = C, which workgroup 0 takes itself.  The partial products of a step
// go to a buffer of two halves used by alternate steps, so that the next step
// can write while workgroup 0 still reads.  With one workgroup per system (the
// batched form) the barrier is a workgroup barrier.
//
// Data: L, Lbar read only; Abar written once per stored entry (may alias
// Lbar: Lbar(R,C) is read only at step C, by the workgroup that overwrites
// it).  The inverses of the diagonal tiles are formed first by their own
// kernel (one wave per tile).  Products on v_mfma_f64_16x16x4f64.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"
#include "factor_bwd.h"

namespace bandchol_fb {

using namespace bandchol;

constexpr int NT = 256;                      // four waves
constexpr long long SPIN_LIMIT = 1LL << 26;  // barrier polls before giving up

struct BandV {
  const glb_d* p;
  int64_t ld, n, k;
  // element (i, j) of the band, zero outside it and past row n-1
  __device__ __forceinline__ double operator()(int64_t i, int64_t j) const {
    const int64_t d = i - j;
    return (i < n && d >= 0 && d <= k) ? p[d + j * ld] : 0.0;
  }
};

__device__ __forceinline__ void band_store(glb_d* p, int64_t ld, int64_t n, int64_t k, int64_t i, int64_t j,
                                           double v) {
  const int64_t d = i - j;
  if (i < n && d >= 0 && d <= k) p[d + j * ld] = v;
}

// M^{-1} of every diagonal tile, column-major T x T: lanes 0..T-1 hold the rows
// of M, lanes T..2T-1 identity rows solved against it column by column, which
// leaves row b of M^{-T} in lane T+b.  Rows past n-1 act as identity rows.
__global__ void __launch_bounds__(64) fb_inverse_kernel(FbSys s) {
  const int64_t NB = (s.n + T - 1) / T;
  const int lane = threadIdx.x;
  const BandV L{(const glb_d*)s.l, s.ldl, s.n, s.k};
  for (int64_t C = blockIdx.x; C < NB; C += gridDim.x) {
    double row[T];
    const int64_t i = C * T + lane;
#pragma unroll
    for (int c = 0; c < T; ++c) {
      const int64_t j = C * T + c;
      if (lane < T) row[c] = (i >= s.n && i == j) ? 1.0 : L(i, j);
      else row[c] = ((lane - T) == c) ? 1.0 : 0.0;
    }
    const bool rhs = lane >= T;
#pragma unroll
    for (int j = 0; j < T; ++j) {
      const double y = 1.0 / readlane(row[j], j);
      const double x = rhs ? row[j] * y : row[j];
      row[j] = x;
#pragma unroll
      for (int l = j + 1; l < T; ++l) {
        const double llj = readlane(x, l);
        row[l] = rhs ? fma(-x, llj, row[l]) : row[l];
      }
    }
    if (rhs) {
      glb_d* out = (glb_d*)s.minv + C * T * T + (lane - T) * T;
#pragma unroll
      for (int c = 0; c < T; ++c) out[c] = row[c];
    }
  }
}

// out = op(a) op(b) for T x T tiles in LDS (column-major, pitch LP); wave w
// forms block (w & 1, w >> 1).  ta / tb: use the transpose.
__device__ __forceinline__ void lds_mm(lds_d* out, const lds_d* a, bool ta, const lds_d* b, bool tb) {
  const int lane = lane_id(), w = wave_id();
  const int bi = w & 1, bj = w >> 1;
  const int i = 16 * bi + (lane & 15), j = 16 * bj + (lane & 15);
  d4 acc = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < T / 4; ++q) {
    const int s = 4 * q + (lane >> 4);
    const double x = ta ? a[i * LP + s] : a[s * LP + i];
    const double y = tb ? b[s * LP + j] : b[j * LP + s];
    acc = mfma_xyt(x, y, acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) out[(16 * bj + 4 * r + (lane >> 4)) * LP + i] = acc[r];
}

struct Lds {
  double minv[T * LP];   // M^{-1} of the step's diagonal tile
  double g[T * LP];      // G(R), then Abar(R,C)
  double m[T * LP];      // diagonal work: M, then scratch
  double mb[T * LP];     // Mbar, then Phi, then S
  double x[T * LP];
};

// Grid barrier among the gridDim.x workgroups of one system: every wave's
// stores are released at agent scope, the counter is raised, and after the
// wait every wave acquires.  Returns false (and raises the abort flag) when a
// wait exceeds its bound or another workgroup has aborted.
__device__ __forceinline__ bool group_barrier(const FbSys& s, unsigned target, lds_i* s_ok) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(s.bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    for (long long spins = 0;; ++spins) {
      if (__hip_atomic_load(s.bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (__hip_atomic_load(s.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
      if (spins > SPIN_LIMIT) {
        __hip_atomic_store(s.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    *s_ok = ok;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return *s_ok != 0;
}

// Step C, tile R = C + 1 + slot: G(R), Abar(R,C) = G M^{-1} (stored), and the
// partial product Abar(R,C)^T L(R,C) into the step's buffer half.
__device__ __forceinline__ void reverse_tile(const FbSys& s, Lds& sh, int64_t C, int64_t R, int64_t Cend, int slot, int half) {
  const int lane = lane_id(), w = wave_id();
  const int bi = w & 1, bj = w >> 1;
  const BandV L{(const glb_d*)s.l, s.ldl, s.n, s.k};
  const BandV Lb{(const glb_d*)s.lbar, s.ldlb, s.n, s.k};
  const BandV W{(const glb_d*)s.abar, s.ldab, s.n, s.k};
  const int64_t r0 = R * T, c0 = C * T;
  const int il = 16 * bi + (lane & 15), jl = 16 * bj + (lane & 15);
  // block (bi, bj) of G, accumulator form: lane l, register r -> (16 bi + l%16, 16 bj + 4 r + l/16)
  d4 acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = Lb(r0 + il, c0 + 16 * bj + 4 * r + (lane >> 4));
  for (int64_t S = C + 1; S <= Cend; ++S) {
    const int64_t s0 = S * T;
#pragma unroll 2
    for (int q = 0; q < T / 4; ++q) {
      const int sl = 4 * q + (lane >> 4);
      double x;
      if (S < R) x = W(r0 + il, s0 + sl);
      else if (S > R) x = W(s0 + sl, r0 + il);
      else x = il >= sl ? (il == sl ? 2.0 : 1.0) * W(r0 + il, r0 + sl) : W(r0 + sl, r0 + il);
      const double y = L(s0 + sl, c0 + jl);
      acc = mfma_xyt(-x, y, acc);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) sh.g[(16 * bj + 4 * r + (lane >> 4)) * LP + il] = acc[r];
  __syncthreads();
  // Abar(R,C) = G M^{-1}
  d4 ab = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < T / 4; ++q) {
    const int sl = 4 * q + (lane >> 4);
    ab = mfma_xyt(sh.g[sl * LP + il], sh.minv[jl * LP + sl], ab);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int cl = 16 * bj + 4 * r + (lane >> 4);
    sh.g[cl * LP + il] = ab[r];
    band_store((glb_d*)s.abar, s.ldab, s.n, s.k, r0 + il, c0 + cl, ab[r]);
  }
  __syncthreads();
  // partial product P = Abar(R,C)^T L(R,C), block (bi, bj)
  d4 p = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < T / 4; ++q) {
    const int sl = 4 * q + (lane >> 4);
    p = mfma_xyt(sh.g[il * LP + sl], L(r0 + sl, c0 + jl), p);
  }
  glb_d* out = (glb_d*)s.part + ((int64_t)half * s.K + slot) * T * T;
#pragma unroll
  for (int r = 0; r < 4; ++r) out[(16 * bj + 4 * r + (lane >> 4)) * T + il] = p[r];
  __syncthreads();
}

// Step C, diagonal tile: Mbar, then Abar(C,C).
__device__ __forceinline__ void reverse_diag(const FbSys& s, Lds& sh, int64_t C, int nslots, int half) {
  const int tid = threadIdx.x;
  const BandV L{(const glb_d*)s.l, s.ldl, s.n, s.k};
  const BandV Lb{(const glb_d*)s.lbar, s.ldlb, s.n, s.k};
  const int64_t c0 = C * T;
  const glb_d* part = (const glb_d*)s.part + (int64_t)half * s.K * T * T;
  for (int e = tid; e < T * T; e += NT) {
    const int r = e % T, c = e / T;
    const int64_t gi = c0 + r;
    sh.m[c * LP + r] = (gi >= s.n && r == c) ? 1.0 : L(gi, c0 + c);
    double v = 0.0;
    if (r >= c) {
      v = Lb(gi, c0 + c);
      for (int t = 0; t < nslots; ++t) v -= part[(int64_t)t * T * T + c * T + r];
    }
    sh.mb[c * LP + r] = v;
  }
  __syncthreads();
  lds_mm((lds_d*)sh.x, (lds_d*)sh.m, true, (lds_d*)sh.mb, false);          // M^T Mbar
  __syncthreads();
  for (int e = tid; e < T * T; e += NT) {          // Phi
    const int r = e % T, c = e / T;
    const double v = sh.x[c * LP + r];
    sh.x[c * LP + r] = r > c ? v : (r == c ? 0.5 * v : 0.0);
  }
  __syncthreads();
  lds_mm((lds_d*)sh.mb, (lds_d*)sh.x, false, (lds_d*)sh.minv, false);      // Phi M^{-1}
  __syncthreads();
  lds_mm((lds_d*)sh.x, (lds_d*)sh.minv, true, (lds_d*)sh.mb, false);       // S = M^{-T} Phi M^{-1}
  __syncthreads();
  for (int e = tid; e < T * T; e += NT) {
    const int r = e % T, c = e / T;
    if (r < c) continue;
    const double v = r == c ? sh.x[c * LP + r] : sh.x[c * LP + r] + sh.x[r * LP + c];
    band_store((glb_d*)s.abar, s.ldab, s.n, s.k, c0 + r, c0 + c, v);
  }
  wait_vmem();
  __syncthreads();
}

__global__ void __launch_bounds__(NT) fb_kernel(FbSys s) {
  __shared__ Lds sh;
  __shared__ int s_ok;
  const int64_t NB = (s.n + T - 1) / T;
  const int g = gridDim.x, wg = blockIdx.x;
  unsigned target = 0;
  for (int64_t C = NB - 1; C >= 0; --C) {
    const int64_t Cend = C + s.K < NB - 1 ? C + s.K : NB - 1;
    const int nslots = (int)(Cend - C);
    const int half = (int)(C & 1);
    for (int e = threadIdx.x; e < T * T; e += NT) {
      const int r = e % T, c = e / T;
      sh.minv[c * LP + r] = ((const glb_d*)s.minv)[C * T * T + c * T + r];
    }
    __syncthreads();
    for (int slot = wg; slot < nslots; slot += g) reverse_tile(s, sh, C, C + 1 + slot, Cend, slot, half);
    if (g > 1) {
      target += (unsigned)g;
      if (!group_barrier(s, target, (lds_i*)&s_ok)) return;
    } else {
      wait_vmem();
      __syncthreads();
    }
    if (wg == 0) reverse_diag(s, sh, C, nslots, half);
  }
}

__global__ void fb_init_kernel(FbSys s) {
  *s.bar = 0;
  *s.abort = 0;
}

__global__ void fb_status_kernel(FbSys s, int64_t* d_status) { *d_status = *s.abort ? (int64_t)-1001 : 0; }

}  // namespace bandchol_fb

size_t bandchol_fb_workspace(int64_t n, int64_t K) {
  using namespace bandchol_fb;
  const int64_t NB = (n + T - 1) / T;
  return 256 + sizeof(double) * ((size_t)NB * T * T + (size_t)2 * (K > 0 ? K : 1) * T * T);
}

// Workspace: the barrier counter and abort flag, then the M^{-1} tiles and
// the two halves of the partial products.  grid_max: workgroups that are
// resident at once (the grid barrier needs all of them running).
hipError_t bandchol_fb_launch(const bandchol_fb::FbSys& in, void* ws, int grid_max, int64_t* d_status,
                              hipStream_t st) {
  using namespace bandchol_fb;
  if (in.n <= 0) return hipSuccess;
  FbSys s = in;
  char* base = (char*)ws;
  const int64_t NB = (s.n + T - 1) / T;
  s.bar = (unsigned*)(base + 0);
  s.abort = (int*)(base + 64);
  s.minv = (double*)(base + 256);
  s.part = s.minv + (size_t)NB * T * T;
  fb_init_kernel<<<1, 1, 0, st>>>(s);
  fb_inverse_kernel<<<(unsigned)(NB < 4096 ? NB : 4096), 64, 0, st>>>(s);
  int g = (int)(s.K > 0 ? s.K : 1);
  if (g > grid_max) g = grid_max;
  if (g < 1) g = 1;
  fb_kernel<<<(unsigned)g, NT, 0, st>>>(s);
  if (d_status) fb_status_kernel<<<1, 1, 0, st>>>(s, d_status);
  return hipGetLastError();
}
