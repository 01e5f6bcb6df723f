// Device building blocks shared by the band Cholesky kernels (gfx950, FP64).
//
// Tiles are T x T (T = 32).  A tile held by a workgroup of 4 waves is split in
// 16 x 16 blocks; in MFMA accumulator form lane l, register r of a block holds
// the element (row l%16, column 4r + l/16), so that consecutive lanes are
// consecutive rows — consecutive addresses in the column-major band layout.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bandchol {

constexpr int T = 32;       // tile width
constexpr int LP = T + 1;   // LDS pitch of a staged tile (column-major)

typedef double d4 __attribute__((ext_vector_type(4)));

// LDS pointers keep their address space across function boundaries, so that
// separately compiled device functions still address LDS with ds_* instructions.
typedef __attribute__((address_space(3))) double lds_d;
typedef __attribute__((address_space(3))) int lds_i;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

__device__ __forceinline__ double readlane_d(double v, int lane) {
  int2 p = __builtin_bit_cast(int2, v);
  p.x = __builtin_amdgcn_readlane(p.x, lane);
  p.y = __builtin_amdgcn_readlane(p.y, lane);
  return __builtin_bit_cast(double, p);
}

// D += X Y^T on one 16x16 block, fragments "lane l holds M[16*blk + l%16][k0 + l/16]".
// The operand order puts the result in the layout described above
// (v_mfma_f64_16x16x4 returns D[4r + l/16][l%16] in lane l, register r).
__device__ __forceinline__ d4 mfma_xyt(double xf, double yf, d4 acc) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(yf, xf, acc, 0, 0, 0);
}

// 1/d from the hardware estimate (about 24 bits) and two Newton-Raphson steps
// r <- r + r (1 - d r), each doubling the correct bits; exact for powers of two.
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// Wait until this wave's outstanding vector memory operations (loads and
// stores) have completed.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

typedef __attribute__((address_space(1))) double glb_d;
typedef __attribute__((address_space(1))) int glb_i;

// Relaxed agent-scope atomic accesses: coherent across the chip's L2 caches
// without cache maintenance; used for data that other workgroups read.
__device__ __forceinline__ double aload(const glb_d* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void astore(glb_d* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct Band {
  glb_d* ab;
  int64_t n, k, ldab;
  __device__ __forceinline__ bool in_band(int64_t i, int64_t j) const {
    const int64_t d = i - j;
    return i < n && d >= 0 && d <= k;
  }
  __device__ __forceinline__ glb_d* at(int64_t i, int64_t j) const { return ab + (i - j) + j * ldab; }
  __device__ __forceinline__ double ld(int64_t i, int64_t j) const { return in_band(i, j) ? *at(i, j) : 0.0; }
};

// A lane's run of band elements A(i, j0 + cs*q), q = 0, 1, ...: the first at p,
// the next ones cs*(ldab-1) doubles apart (A(i, j) sits at ab + i + j*(ldab-1)).
// Element q is in the band iff i < n and 0 <= d0 - cs*q <= k.  Set up once per
// tile so that each element costs one compare and one pointer step.
struct Run {
  glb_d* p;
  int64_t step;
  int d0, ds, k;
  bool row_ok;
  __device__ __forceinline__ bool in(int q) const {
    const int d = d0 - ds * q;
    return row_ok && d >= 0 && d <= k;
  }
  __device__ __forceinline__ glb_d* at(int q) const { return p + step * q; }
  __device__ __forceinline__ double ld(int q) const { return in(q) ? *at(q) : 0.0; }
  __device__ __forceinline__ double ald(int q) const { return in(q) ? aload(at(q)) : 0.0; }
};

__device__ __forceinline__ Run band_run(const Band& a, int64_t i, int64_t j0, int cs) {
  Run r;
  r.p = a.ab + i + j0 * (a.ldab - 1);
  r.step = (int64_t)cs * (a.ldab - 1);
  r.d0 = (int)(i - j0);
  r.ds = cs;
  r.k = (int)(a.k < 0x7fffffff ? a.k : 0x7fffffff);
  r.row_ok = i < a.n;
  return r;
}

// ---------------------------------------------------------------- tile blocks in global memory

// Block (bi, bj) of tile (R, C) into accumulator form.  On a diagonal tile the
// positions past row n-1 get an identity so that the factorization there is trivial.
__device__ __forceinline__ d4 blk_load(const Band& a, int64_t R, int64_t C, int bi, int bj) {
  const int lane = lane_id();
  const Run run = band_run(a, R * T + 16 * bi + (lane & 15), C * T + 16 * bj + (lane >> 4), 4);
  d4 acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double v = run.ld(r);
    if (R == C && !run.row_ok && run.d0 - 4 * r == 0) v = 1.0;
    acc[r] = v;
  }
  return acc;
}

__device__ __forceinline__ void blk_store(const Band& a, int64_t R, int64_t C, int bi, int bj, d4 v) {
  const int lane = lane_id();
  const Run run = band_run(a, R * T + 16 * bi + (lane & 15), C * T + 16 * bj + (lane >> 4), 4);
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (run.in(r)) *run.at(r) = v[r];
}

// ---------------------------------------------------------------- tiles staged in LDS (column-major, pitch LP)

__device__ __forceinline__ void blk_to_lds(lds_d* s, int bi, int bj, d4 v) {
  const int lane = lane_id();
#pragma unroll
  for (int r = 0; r < 4; ++r) s[(16 * bj + 4 * r + (lane >> 4)) * LP + 16 * bi + (lane & 15)] = v[r];
}

// acc -= X_blk(bi) Y_blk(bj)^T, X and Y tiles in LDS (column-major, pitch LP).
__device__ __forceinline__ d4 blk_gemm_lds(const lds_d* x, const lds_d* y, int bi, int bj, d4 acc, int qmax = T / 4) {
  const int lane = lane_id();
#pragma unroll
  for (int q = 0; q < T / 4; ++q) {
    if (q < qmax) {
      const int kk = 4 * q + (lane >> 4);
      acc = mfma_xyt(-x[kk * LP + 16 * bi + (lane & 15)], y[kk * LP + 16 * bj + (lane & 15)], acc);
    }
  }
  return acc;
}

// out = X_blk(bi) * L^{-T}, X in LDS (column-major), L^{-T} row-major T x T in LDS
// with row pitch `pitch` (upper triangular, so k-steps past column 16*bj+15 are zero).
__device__ __forceinline__ d4 blk_trsm_lds(const lds_d* x, const lds_d* linvt, int bi, int bj, int pitch = T) {
  const int lane = lane_id();
  d4 out = {0, 0, 0, 0};
  const int qmax = 4 * bj + 4;
#pragma unroll
  for (int q = 0; q < T / 4; ++q) {
    if (q < qmax) {
      const int kk = 4 * q + (lane >> 4);
      out = mfma_xyt(x[kk * LP + 16 * bi + (lane & 15)], linvt[kk * pitch + 16 * bj + (lane & 15)], out);
    }
  }
  return out;
}

// ---------------------------------------------------------------- diagonal-tile sweep

// Factor the T x T SPD tile whose rows sit in lanes 0..T-1 (row[c] = A(lane, c)),
// while lanes T..2T-1 carry the identity rows, in one wave.
//
// The pivot chain runs in L D L^T form.  For column j the unscaled column
// w_ij = A'(i, j) is final once column j-1 has been applied; it is broadcast
// with readlane (no LDS traffic, so the sweep does not queue behind the MFMA
// operand reads of the other waves) and every row is updated by
// A'(i, l) -= (w_ij / d_j) w_lj, l > j.  Only one division per column is on the
// dependency chain: the next pivot d_{j+1} = A'(j+1,j+1) - w_{j+1,j}^2 / d_j is
// formed directly from two values known before the division.  The square roots
// are taken once at the end, off the chain: both the factor rows (unit factor
// l, L = l D^{1/2}) and the identity rows (which now hold l^{-T} D^{-1}, and
// L^{-T} = l^{-T} D^{-1/2}) are scaled column by column by sqrt(d_c).
// Afterwards lane i < T holds row i of L (upper part unspecified) and lane
// T+b holds row b of L^{-T}.  Returns the first local column whose pivot is
// not > 0 (zero, negative or NaN), or -1.
__device__ __forceinline__ int sweep_ldlt(double (&row)[T], lds_d* wbuf) {
  (void)wbuf;
  const int lane = lane_id();
  double d_mine = 1.0;                    // lane c keeps pivot c
  double dcur = readlane_d(row[0], 0);
  int fail = -1;
  // Straight-line code (no exit per column) so that the scheduler can overlap
  // column j+1's pivot chain with column j's row updates.
#pragma unroll
  for (int j = 0; j < T; ++j) {
    const double d = dcur;
    fail = (fail < 0 && !(d > 0.0)) ? j : fail;
    const double w = row[j];
    double p = 0.0, wn = 0.0;
    if (j + 1 < T) {
      p = readlane_d(row[j + 1], j + 1);
      wn = readlane_d(w, j + 1);
    }
    const double dinv = recip(d);
    d_mine = (lane == j) ? d : d_mine;
    if (j + 1 < T) dcur = fma(-(wn * wn), dinv, p);
    const double q = w * dinv;
    row[j] = (lane == j) ? 1.0 : q;
#pragma unroll
    for (int l = j + 1; l < T; ++l) row[l] = fma(-q, readlane_d(w, l), row[l]);
  }
  const double s_mine = sqrt(d_mine);
#pragma unroll
  for (int c = 0; c < T; ++c) row[c] *= readlane_d(s_mine, c);
  return fail;
}

// The same sweep, with the column broadcast through LDS instead of readlane:
// every lane stores its w_ij, and the values w_lj (l > j) come back two at a
// time with 16-byte broadcast reads (all lanes read the same address).  The
// two values on the pivot chain (the next pivot and its multiplier) still use
// readlane.  wbuf: 2 x 64 doubles of LDS, 16-byte aligned, private to the wave.
typedef double d2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) d2 lds_d2;

__device__ __forceinline__ int sweep_ldlt_lds(double (&row)[T], lds_d* wbuf) {
  const int lane = lane_id();
  double d_mine = 1.0;
  double dcur = readlane_d(row[0], 0);
  int fail = -1;
#pragma unroll
  for (int j = 0; j < T; ++j) {
    lds_d* wb = wbuf + 64 * (j & 1);
    const double d = dcur;
    fail = (fail < 0 && !(d > 0.0)) ? j : fail;
    const double w = row[j];
    wb[lane] = w;
    double p = 0.0, wn = 0.0;
    if (j + 1 < T) {
      p = readlane_d(row[j + 1], j + 1);
      wn = readlane_d(w, j + 1);
    }
    const double dinv = recip(d);
    d_mine = (lane == j) ? d : d_mine;
    if (j + 1 < T) dcur = fma(-(wn * wn), dinv, p);
    const double q = w * dinv;
    row[j] = (lane == j) ? 1.0 : q;
    const lds_d2* wb2 = (const lds_d2*)wb;
#pragma unroll
    for (int l = j + 1; l < T; ++l) {
      double wl;
      if ((l & 1) == 0 && l + 1 < T) {
        const d2 v = wb2[l >> 1];
        wl = v.x;
        row[l + 1] = fma(-q, v.y, row[l + 1]);
      } else if ((l & 1) == 1 && l == j + 1) {
        wl = wb[l];
      } else if ((l & 1) == 1) {
        continue;  // done with its even partner
      } else {
        wl = wb[l];
      }
      row[l] = fma(-q, wl, row[l]);
    }
  }
  const double s_mine = sqrt(d_mine);
#pragma unroll
  for (int c = 0; c < T; ++c) row[c] *= readlane_d(s_mine, c);
  return fail;
}

}  // namespace bandchol
