// Device building blocks shared by the band Cholesky kernels (gfx950), for
// FP64 and FP32 data.
//
// Tiles are T x T (T = 32).  A tile held by a workgroup of 4 waves is split in
// 16 x 16 blocks.  MFMA operands use the fragment form "lane l holds
// M[16*blk + l%16][k0 + l/16]" (the same for both precisions); results come
// back in the accumulator form: lane l, register r holds the element (row
// l%16, column acc_col0(l) + ACC_STEP*r), so that consecutive lanes are
// consecutive rows — consecutive addresses in the column-major band layout.
// The column mapping differs between the two instructions used:
//   v_mfma_f64_16x16x4f64  column 4r + l/16     (ACC_STEP 4)
//   v_mfma_f32_16x16x4f32  column 4(l/16) + r   (ACC_STEP 1)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bandchol {

constexpr int T = 32;       // tile width
constexpr int LP = T + 1;   // LDS pitch of a staged tile (column-major)

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// LDS and global pointers keep their address space across function
// boundaries, so that separately compiled device functions still use ds_* and
// global_* instructions (not flat ones).
template <typename F> using lds_t = __attribute__((address_space(3))) F;
template <typename F> using glb_t = __attribute__((address_space(1))) F;
typedef lds_t<double> lds_d;
typedef lds_t<int> lds_i;
typedef glb_t<double> glb_d;
typedef glb_t<int> glb_i;

template <typename F> struct Prec;
template <> struct Prec<double> {
  typedef d4 v4;
  static constexpr int ACC_STEP = 4;
  __device__ static __forceinline__ int acc_col0(int lane) { return lane >> 4; }
};
template <> struct Prec<float> {
  typedef f4 v4;
  static constexpr int ACC_STEP = 1;
  __device__ static __forceinline__ int acc_col0(int lane) { return 4 * (lane >> 4); }
};
template <typename F> using v4_t = typename Prec<F>::v4;

// With v_mfma_f64_16x16x4f64 an accumulator block (bi, kb) holds, in register
// r, exactly the operand fragment of k-step 4 kb + r of its row block (lane l:
// column 16 kb + 4 r + l/16), so a product's result feeds the next product
// without passing through LDS.  Not so for the FP32 instruction's layout.
template <typename F>
__host__ __device__ constexpr bool acc_is_operand() { return Prec<F>::ACC_STEP == 4; }

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

__device__ __forceinline__ double readlane(double v, int lane) {
  int2 p = __builtin_bit_cast(int2, v);
  p.x = __builtin_amdgcn_readlane(p.x, lane);
  p.y = __builtin_amdgcn_readlane(p.y, lane);
  return __builtin_bit_cast(double, p);
}
__device__ __forceinline__ float readlane(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
__device__ __forceinline__ double readlane_d(double v, int lane) { return readlane(v, lane); }

// D += X Y^T on one 16x16 block from fragments of X and Y; the operand order
// (Y first) puts the result in the accumulator form described above.
__device__ __forceinline__ d4 mfma_xyt(double xf, double yf, d4 acc) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(yf, xf, acc, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_xyt(float xf, float yf, f4 acc) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(yf, xf, acc, 0, 0, 0);
}

// 1/d from the hardware estimate and Newton-Raphson steps r <- r + r (1 - d r),
// each doubling the correct bits; exact for powers of two.  FP64: the estimate
// carries about 24 bits, two steps; FP32: the estimate is within an ulp, one step.
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float recip(float d) {
  const float r = __builtin_amdgcn_rcpf(d);
  const float e = fmaf(-d, r, 1.0f);
  return fmaf(r, e, r);
}

__device__ __forceinline__ double prec_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float prec_sqrt(float x) { return sqrtf(x); }

// Wait until this wave's outstanding vector memory operations (loads and
// stores) have completed.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// The pointer p, hidden from the optimiser (an empty register constraint, no
// instruction): a load from a select between an element and a stand-in is
// otherwise turned into a branch around the load, and the branch makes the
// wave wait for loads still in flight.
template <typename P>
__device__ __forceinline__ P opaque_ptr(P p) {
  uint64_t u = (uint64_t)p;
  asm("" : "+v"(u));
  return (P)u;
}

// Relaxed agent-scope atomic accesses: coherent across the chip's L2 caches
// without cache maintenance; used for data that other workgroups read.
template <typename F>
__device__ __forceinline__ F aload(const glb_t<F>* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename F>
__device__ __forceinline__ void astore(glb_t<F>* p, F v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename F>
struct BandT {
  glb_t<F>* ab;
  int64_t n, k, ldab;
  __device__ __forceinline__ bool in_band(int64_t i, int64_t j) const {
    const int64_t d = i - j;
    return i < n && d >= 0 && d <= k;
  }
  __device__ __forceinline__ glb_t<F>* at(int64_t i, int64_t j) const { return ab + (i - j) + j * ldab; }
  __device__ __forceinline__ F ld(int64_t i, int64_t j) const { return in_band(i, j) ? *at(i, j) : F(0); }
};
typedef BandT<double> Band;

// A lane's run of band elements A(i, j0 + cs*q), q = 0, 1, ...: the first at p,
// the next ones cs*(ldab-1) elements apart (A(i, j) sits at ab + i + j*(ldab-1)).
// Element q is in the band iff i < n and 0 <= d0 - cs*q <= k.  Set up once per
// tile so that each element costs one compare and one pointer step.
template <typename F>
struct RunT {
  glb_t<F>* p;
  int64_t step;
  int d0, ds, k;
  bool row_ok;
  __device__ __forceinline__ bool in(int q) const {
    const int d = d0 - ds * q;
    return row_ok && d >= 0 && d <= k;
  }
  __device__ __forceinline__ glb_t<F>* at(int q) const { return p + step * q; }
  __device__ __forceinline__ F ld(int q) const { return in(q) ? *at(q) : F(0); }
  __device__ __forceinline__ F ald(int q) const { return in(q) ? aload<F>(at(q)) : F(0); }
};
typedef RunT<double> Run;

template <typename F>
__device__ __forceinline__ RunT<F> band_run(const BandT<F>& a, int64_t i, int64_t j0, int cs) {
  RunT<F> r;
  r.p = a.ab + i + j0 * (a.ldab - 1);
  r.step = (int64_t)cs * (a.ldab - 1);
  r.d0 = (int)(i - j0);
  r.ds = cs;
  r.k = (int)(a.k < 0x7fffffff ? a.k : 0x7fffffff);
  r.row_ok = i < a.n;
  return r;
}

// The run of accumulator-form elements of block (bi, bj) of tile (R, C) for this lane.
template <typename F>
__device__ __forceinline__ RunT<F> acc_run(const BandT<F>& a, int64_t R, int64_t C, int bi, int bj) {
  const int lane = lane_id();
  return band_run(a, R * T + 16 * bi + (lane & 15), C * T + 16 * bj + Prec<F>::acc_col0(lane), Prec<F>::ACC_STEP);
}

// ---------------------------------------------------------------- tile blocks in global memory

// Block (bi, bj) of tile (R, C) into accumulator form.  On a diagonal tile the
// positions past row n-1 get an identity so that the factorization there is trivial.
template <typename F>
__device__ __forceinline__ v4_t<F> blk_load(const BandT<F>& a, int64_t R, int64_t C, int bi, int bj) {
  const RunT<F> run = acc_run(a, R, C, bi, bj);
  v4_t<F> acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    F v = run.ld(r);
    if (R == C && !run.row_ok && run.d0 - run.ds * r == 0) v = F(1);
    acc[r] = v;
  }
  return acc;
}

template <typename F>
__device__ __forceinline__ void blk_store(const BandT<F>& a, int64_t R, int64_t C, int bi, int bj, v4_t<F> v) {
  const RunT<F> run = acc_run(a, R, C, bi, bj);
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (run.in(r)) *run.at(r) = v[r];
}

// ---------------------------------------------------------------- tiles staged in LDS (column-major, pitch LP)

// LDS index of accumulator element r of block (bi, bj) for this lane.
template <typename F>
__device__ __forceinline__ int acc_lds_index(int bi, int bj, int r) {
  const int lane = lane_id();
  return (16 * bj + Prec<F>::acc_col0(lane) + Prec<F>::ACC_STEP * r) * LP + 16 * bi + (lane & 15);
}

template <typename F>
__device__ __forceinline__ void blk_to_lds(lds_t<F>* s, int bi, int bj, v4_t<F> v) {
#pragma unroll
  for (int r = 0; r < 4; ++r) s[acc_lds_index<F>(bi, bj, r)] = v[r];
}

template <typename F>
__device__ __forceinline__ v4_t<F> blk_from_lds(const lds_t<F>* s, int bi, int bj) {
  v4_t<F> v;
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = s[acc_lds_index<F>(bi, bj, r)];
  return v;
}

// acc -= X_blk(bi) Y_blk(bj)^T, X and Y tiles in LDS (column-major, pitch LP).
template <typename F>
__device__ __forceinline__ v4_t<F> blk_gemm_lds(const lds_t<F>* x, const lds_t<F>* y, int bi, int bj, v4_t<F> acc,
                                               int qmax = T / 4) {
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
template <typename F>
__device__ __forceinline__ v4_t<F> blk_trsm_lds(const lds_t<F>* x, const lds_t<F>* linvt, int bi, int bj,
                                               int pitch = T) {
  const int lane = lane_id();
  v4_t<F> out = {0, 0, 0, 0};
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
// w_ij = A'(i, j) is final once column j-1 has been applied; every row is
// updated by A'(i, l) -= (w_ij / d_j) w_lj, l > j.  Only one reciprocal per
// column is on the dependency chain: the next pivot
// d_{j+1} = A'(j+1,j+1) - w_{j+1,j}^2 / d_j is formed directly from two values
// known before the reciprocal.  The square roots are taken once at the end, off
// the chain: both the factor rows (unit factor l, L = l D^{1/2}) and the
// identity rows (which now hold l^{-T} D^{-1}, and L^{-T} = l^{-T} D^{-1/2}) are
// scaled column by column by sqrt(d_c).
//
// Two levels: the columns of each half of the tile are swept with updates
// inside that half only, the broadcasts of w_lj done by readlane; the first
// half's update of the second half, A'(i, H+c) -= sum_j q_ij d_j q_{H+c,j}
// (q_ij = w_ij / d_j, the multipliers left in the first half's columns) is one
// rank-H product on the matrix cores, through LDS.  This halves the
// broadcasts, which bound a one-level sweep (two readlanes and the wait
// states after them per element).  `sq` holds at least H x (2T+1) elements
// and `sd` H, both free LDS of this wave (no other wave touches them meanwhile).
//
// Afterwards lane i < T holds row i of L (upper part unspecified) and lane
// T+b holds row b of L^{-T}.  Returns the first local column whose pivot is
// not > 0 (zero, negative or NaN), or -1, found once at the end from the
// pivots kept per lane (after a failed pivot the later columns are garbage,
// which only the failure report sees).  The unit diagonal of the unit factor
// is left as d_j (1 / d_j) rather than set to 1: within the reciprocal's last
// bit of 1, exactly 1 for pivots that are powers of two, and no select per
// column.
template <typename F>
__device__ __forceinline__ void sweep_half(F (&row)[T], int j0, F& dcur, F& d_mine, int& fail) {
  const int lane = lane_id();
  constexpr int H = T / 2;
  // Straight-line code (no exit per column).  Within a column the lane reads
  // of its row updates go first, into distinct scalar registers, and the
  // updates after them, so that the reads overlap instead of each waiting for
  // the previous update; the next column's reciprocal is started before this
  // column's updates (its inputs are known earlier), so that its latency hides
  // behind them.
  F dinv = recip(dcur);
#pragma unroll
  for (int jj = 0; jj < H; ++jj) {
    const int j = j0 + jj;
    const F d = dcur;
    const F w = row[j];
    d_mine = (lane == j) ? d : d_mine;
    const F q = w * dinv;
    F dinv_next = dinv;
    if (jj + 1 < H) {
      const F p = readlane(row[j + 1], j + 1);
      const F wn = readlane(w, j + 1);
      dcur = fma(-(wn * wn), dinv, p);
      dinv_next = recip(dcur);
    }
    row[j] = q;   // lane j: d_j * (1 / d_j), 1 up to the reciprocal's last bit
    F wl[H];
#pragma unroll
    for (int l = j + 1; l < j0 + H; ++l) wl[l - j0] = readlane(w, l);
#pragma unroll
    for (int l = j + 1; l < j0 + H; ++l) row[l] = fma(-q, wl[l - j0], row[l]);
    dinv = dinv_next;
  }
}

struct NoHook {
  __device__ void operator()() const {}
};

// `mid` runs between the two halves (a point some microseconds into the sweep).
template <typename F, typename Hook = NoHook>
__device__ __forceinline__ int sweep_ldlt(F (&row)[T], lds_t<F>* sq, lds_t<F>* sd, Hook mid = Hook()) {
  const int lane = lane_id();
  constexpr int H = T / 2;
  constexpr int QP = 2 * T + 1;           // LDS pitch of a column over the 64 lanes
  F d_mine = F(1);                        // lane c keeps pivot c
  F dcur = readlane(row[0], 0);
  int fail = -1;
  sweep_half(row, 0, dcur, d_mine, fail);
  // Second half -= Q D Q_2^T: Q (64 x H) = the first half's columns of all
  // lanes, Q_2 its rows H..T-1.  Output tile b (lanes 16b .. 16b+15) of the
  // 64 x H product accumulates X Y^T with X = rows of Q and Y = Q_2 D.  Within
  // one wave LDS operations complete in order, so no barrier is needed.
#pragma unroll
  for (int j = 0; j < H; ++j) sq[j * QP + lane] = row[j];
  if (lane < H) sd[lane] = d_mine;
  v4_t<F> acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = v4_t<F>{0, 0, 0, 0};
#pragma unroll
  for (int q4 = 0; q4 < H / 4; ++q4) {
    const int kk = 4 * q4 + (lane >> 4);
    const F y = sq[kk * QP + H + (lane & 15)] * sd[kk];
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = mfma_xyt(sq[kk * QP + 16 * b + (lane & 15)], y, acc[b]);
  }
  // accumulator form (row 16b + l%16, column acc_col0 + ACC_STEP r) -> LDS column-major -> lane rows
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      sq[(Prec<F>::acc_col0(lane) + Prec<F>::ACC_STEP * r) * QP + 16 * b + (lane & 15)] = acc[b][r];
#pragma unroll
  for (int c = 0; c < H; ++c) row[H + c] -= sq[c * QP + lane];
  mid();
  dcur = readlane(row[H], H);
  sweep_half(row, H, dcur, d_mine, fail);
  // column c scaled by sqrt(d_c): the roots broadcast through LDS (lane c
  // writes its own; within one wave LDS accesses complete in order), which
  // keeps 2T lane reads off the vector ALU
  {
    const unsigned long long bad = __ballot(lane < T && !(d_mine > F(0)));
    fail = bad ? (int)__builtin_ctzll(bad) : -1;
  }
  if (lane < T) sd[lane] = prec_sqrt(d_mine);
#pragma unroll
  for (int c = 0; c < T; ++c) row[c] *= sd[c];
  return fail;
}

}  // namespace bandchol
