// Multi-workgroup band Cholesky for wide bands (gfx950; FP64, and FP32 for the
// mixed-precision solver).
//
// Tiles T x T down the band, tile (R, C) for 0 <= R - C <= K.  One workgroup,
// the spine (whoever takes ticket 0), carries the dependency chain along the
// diagonal, one tile column per step:
//   phase A  wave 0: factor the staged diagonal tile (register sweep) ->
//            L(C,C) and L(C,C)^{-T}, published at once;
//            waves 1-3: complete tile (C+1, C) and the next diagonal tile with
//            the one term (column C-1) the helpers could not have applied yet;
//   phase B  all waves: L(C+1, C) = tile * L(C,C)^{-T}, published;
//   phase C  waves 1-3: next diagonal tile -= L(C+1,C) L(C+1,C)^T, staged.
// Helper workgroups take the other tickets, in an order where every task only
// waits for lower tickets or for spine steps:
//   O(R, C), R - C >= 2: acc = A(R,C) - sum_s L(R,s) L(C,s)^T (terms applied as
//            their operand tiles are published), then L(R,C) = acc L(C,C)^{-T};
//   H(m):    the spine's two tiles of step m-1, (m, m-1) and (m, m), with every
//            term but the last one (s <= m-3) applied, published for the spine.
// Data between workgroups moves through relaxed agent-scope atomic loads and
// stores (coherent across the chip without cache flushes); a flag is raised
// after the data stores of the raising wave(s) have completed.
#include <stdint.h>

#include "common.h"

namespace bandchol_f2 {

using namespace bandchol;

constexpr int NT = 256;
// Bound on polls of one flag (each poll sleeps ~64 cycles plus a memory round trip);
// far above any legitimate wait, which lasts a few spine steps.
constexpr long long SPIN_LIMIT = 1LL << 22;


template <typename F>
struct Ws {
  glb_i* tflag;     // NB*(K+1): tile (R, R-d) published, index R*(K+1)+d
  glb_i* hflag;     // NB: pre-accumulated tiles of step m-1 published
  glb_t<F>* linvt;  // NB*T*T: L(C,C)^{-T}, row-major
  glb_t<F>* pre;    // NB*2*T*T: per m, tile (m,m-1) then tile (m,m), column-major
  unsigned* queue;
  glb_i* abort_flag;  // 1 = pivot failure, 2 = wait bound exceeded
  unsigned long long* first_fail;
  const glb_t<F>* zero;  // a zero: masked-off lanes load it, so that operand loads are unconditional
};

template <typename F>
struct Args {
  BandT<F> a;
  int NB, K;
  unsigned ntickets;
  Ws<F> w;
};

__device__ __forceinline__ int aflag(const glb_i* p) {
  return __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void raise_flag(glb_i* p) { __hip_atomic_store(p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// This wave waits for *f (bounded); every lane gets the same answer.
template <typename F>
__device__ __forceinline__ bool wave_wait(const glb_i* f, const Ws<F>& w) {
  glb_i* const abort_flag = w.abort_flag;
  long long spins = 0;
  while (!aflag(f)) {
    if (aflag(abort_flag)) return false;
    if (++spins > SPIN_LIMIT) {
      __hip_atomic_store(abort_flag, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");  // keeps later loads below the wait
  return true;
}

template <typename F>
__device__ __forceinline__ int tidx(const Args<F>& A, int64_t R, int64_t C) { return (int)(R * (A.K + 1) + (R - C)); }

// ---------------------------------------------------------------- block I/O with atomics

// Block (bi, bj) of tile (R, C) in accumulator form (see common.h).  On a
// diagonal tile the positions past row n-1 get an identity.
template <typename F>
__device__ __forceinline__ v4_t<F> ablk_load(const BandT<F>& a, int64_t R, int64_t C, int bi, int bj) {
  const RunT<F> run = acc_run(a, R, C, bi, bj);
  v4_t<F> acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    F v = run.ald(r);
    if (R == C && !run.row_ok && run.d0 - run.ds * r == 0) v = F(1);
    acc[r] = v;
  }
  return acc;
}

template <typename F>
__device__ __forceinline__ void ablk_store(const BandT<F>& a, int64_t R, int64_t C, int bi, int bj, v4_t<F> v) {
  const RunT<F> run = acc_run(a, R, C, bi, bj);
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (run.in(r)) astore(run.at(r), v[r]);
}

// A dense T x T tile in column-major workspace memory, in accumulator form.
template <typename F>
__device__ __forceinline__ int wblk_index(int bi, int bj, int r) {
  const int lane = lane_id();
  return (16 * bj + Prec<F>::acc_col0(lane) + Prec<F>::ACC_STEP * r) * T + 16 * bi + (lane & 15);
}
template <typename F>
__device__ __forceinline__ v4_t<F> wblk_load(const glb_t<F>* t, int bi, int bj) {
  v4_t<F> v;
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = aload<F>(t + wblk_index<F>(bi, bj, r));
  return v;
}
template <typename F>
__device__ __forceinline__ void wblk_store(glb_t<F>* t, int bi, int bj, v4_t<F> v) {
#pragma unroll
  for (int r = 0; r < 4; ++r) astore<F>(t + wblk_index<F>(bi, bj, r), v[r]);
}

// acc -= X_blk(bi) Y_blk(bj)^T with X = tile (Rx, s), Y = tile (Ry, s) from the band.
template <typename F>
__device__ __forceinline__ void term_load(const Args<F>& A, int64_t Rx, int64_t Ry, int64_t s, int bi, int bj,
                                          F (&xf)[T / 4], F (&yf)[T / 4]) {
  const int lane = lane_id();
  const int64_t j0 = s * T + (lane >> 4);
  const RunT<F> x = band_run(A.a, Rx * T + 16 * bi + (lane & 15), j0, 4);
  const RunT<F> y = band_run(A.a, Ry * T + 16 * bj + (lane & 15), j0, 4);
#pragma unroll
  for (int q = 0; q < T / 4; ++q) {
    xf[q] = aload<F>(opaque_ptr(x.in(q) ? x.at(q) : A.w.zero));
    yf[q] = aload<F>(opaque_ptr(y.in(q) ? y.at(q) : A.w.zero));
  }
}

// Only the X operand (block bi of tile (Rx, s)).
template <typename F>
__device__ __forceinline__ void term_load_x(const Args<F>& A, int64_t Rx, int64_t s, int bi, F (&xf)[T / 4]) {
  const int lane = lane_id();
  const RunT<F> x = band_run(A.a, Rx * T + 16 * bi + (lane & 15), s * T + (lane >> 4), 4);
#pragma unroll
  for (int q = 0; q < T / 4; ++q) xf[q] = aload<F>(opaque_ptr(x.in(q) ? x.at(q) : A.w.zero));
}

template <typename F>
__device__ __forceinline__ v4_t<F> term_apply(const F (&xf)[T / 4], const F (&yf)[T / 4], v4_t<F> acc) {
#pragma unroll
  for (int q = 0; q < T / 4; ++q) acc = mfma_xyt(-xf[q], yf[q], acc);
  return acc;
}

// ---------------------------------------------------------------- helpers

// Apply the terms s in [s0, s1) of tile (R, C) (blocks of this wave):
// acc -= L(R,s) L(C,s)^T.  The flags of up to 16 terms are read at once (for a
// fixed tile row they are contiguous, one per lane); within a run of
// published terms the operands of the next term load while the current one
// is on the matrix cores, both steps of each pair always taken (the last term
// of the run stands in past its end) so that the wave's counter of
// outstanding loads stays exact.  Xrow = R, Yrow = C.
template <typename F>
__device__ __forceinline__ bool apply_terms(const Args<F>& A, int64_t R, int64_t C, int64_t s0, int64_t s1, int bi, int bj,
                                            v4_t<F>& acc) {
  const int lane = lane_id();
  int64_t s = s0;
  while (s < s1) {
    const int span = s1 - s < 16 ? (int)(s1 - s) : 16;
    int f = 1;
    if (lane < span) {
      f = __hip_atomic_load(&A.w.tflag[tidx(A, R, s + lane)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (C != R) f &= __hip_atomic_load(&A.w.tflag[tidx(A, C, s + lane)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const unsigned long long bad = __ballot(lane < span && f == 0);
    int64_t e = s + (bad ? (int)__builtin_ctzll(bad) : span);
    if (e == s) {
      if (!wave_wait(&A.w.tflag[tidx(A, R, s)], A.w)) return false;
      if (C != R && !wave_wait(&A.w.tflag[tidx(A, C, s)], A.w)) return false;
      e = s + 1;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");  // keeps the operand loads below the flags
    F x0[T / 4], y0[T / 4], x1[T / 4], y1[T / 4];
    term_load(A, R, C, s, bi, bj, x0, y0);
    term_load(A, R, C, s + 1 < e ? s + 1 : e - 1, bi, bj, x1, y1);
    int64_t u = s;
    for (; u + 1 < e; u += 2) {
      acc = term_apply(x0, y0, acc);
      term_load(A, R, C, u + 2 < e ? u + 2 : e - 1, bi, bj, x0, y0);
      acc = term_apply(x1, y1, acc);
      term_load(A, R, C, u + 3 < e ? u + 3 : e - 1, bi, bj, x1, y1);
    }
    if (u < e) acc = term_apply(x0, y0, acc);
    s = e;
  }
  return true;
}

// Trsm of the accumulator tile held across the 4 waves: out = acc * L(C,C)^{-T}.
template <typename F>
__device__ __forceinline__ v4_t<F> trsm_from_lds(const lds_t<F>* x, const glb_t<F>* linvt_g, int bi, int bj) {
  const int lane = lane_id();
  v4_t<F> out = {0, 0, 0, 0};
  const int qmax = 4 * bj + 4;
  F yf[T / 4];
#pragma unroll
  for (int q = 0; q < T / 4; ++q)
    yf[q] = (q < qmax) ? aload<F>(linvt_g + (4 * q + (lane >> 4)) * T + 16 * bj + (lane & 15)) : F(0);
#pragma unroll
  for (int q = 0; q < T / 4; ++q)
    if (q < qmax) out = mfma_xyt(x[(4 * q + (lane >> 4)) * LP + 16 * bi + (lane & 15)], yf[q], out);
  return out;
}

// The noinline functions below copy their structure arguments into locals
// first: the references point at a stack copy, and after every atomic store or
// fence the fields would otherwise be re-read from memory.
template <typename F>
__device__ __attribute__((noinline)) void task_off(const Args<F>& A_, int64_t R, int64_t C, lds_t<F>* stage,
                                                   lds_i* s_ok) {
  const Args<F> A = A_;
  const int wave = wave_id();
  const int bi = wave & 1, bj = wave >> 1;
  v4_t<F> acc = ablk_load(A.a, R, C, bi, bj);
  const int64_t s0 = R - A.K > 0 ? R - A.K : 0;
  int ok = apply_terms(A, R, C, s0, C, bi, bj, acc) ? 1 : 0;
  if (ok) ok = wave_wait(&A.w.tflag[tidx(A, C, C)], A.w) ? 1 : 0;
  blk_to_lds(stage, bi, bj, acc);
  if (!ok && lane_id() == 0) *s_ok = 0;
  __syncthreads();
  if (*s_ok == 0) return;
  const v4_t<F> out = trsm_from_lds<F>(stage, A.w.linvt + C * T * T, bi, bj);
  ablk_store(A.a, R, C, bi, bj, out);
  wait_vmem();
  __syncthreads();
  if (threadIdx.x == 0) raise_flag(&A.w.tflag[tidx(A, R, C)]);
}

// Two tiles of one column: (R, C) and (R+1, C) share the operand L(C, s) of
// every term, so a term loads three blocks for two outputs and puts twice the
// matrix-core work behind each round trip.  When R > K the first term,
// s = R-K, lies outside the band of row R+1: that operand loads as zero and
// its flag is not checked.  Same run structure as apply_terms.
template <typename F>
__device__ __forceinline__ bool apply_terms2(const Args<F>& A, int64_t R, int64_t C, int64_t s0, int64_t s1, int bi,
                                             int bj, v4_t<F>& acc0, v4_t<F>& acc1) {
  const int lane = lane_id();
  const int64_t s_in1 = R + 1 - A.K;   // first term inside the band for row R+1
  int64_t s = s0;
  while (s < s1) {
    const int span = s1 - s < 16 ? (int)(s1 - s) : 16;
    int f = 1;
    if (lane < span) {
      const int64_t u = s + lane;
      f = __hip_atomic_load(&A.w.tflag[tidx(A, R, u)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
          __hip_atomic_load(&A.w.tflag[tidx(A, C, u)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (u >= s_in1) f &= __hip_atomic_load(&A.w.tflag[tidx(A, R + 1, u)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const unsigned long long bad = __ballot(lane < span && f == 0);
    int64_t e = s + (bad ? (int)__builtin_ctzll(bad) : span);
    if (e == s) {
      if (!wave_wait(&A.w.tflag[tidx(A, R, s)], A.w) || !wave_wait(&A.w.tflag[tidx(A, C, s)], A.w)) return false;
      if (s >= s_in1 && !wave_wait(&A.w.tflag[tidx(A, R + 1, s)], A.w)) return false;
      e = s + 1;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");  // keeps the operand loads below the flags
    F a0[T / 4], b0[T / 4], y0[T / 4], a1[T / 4], b1[T / 4], y1[T / 4];
    term_load(A, R, C, s, bi, bj, a0, y0);
    term_load_x(A, R + 1, s, bi, b0);
    term_load(A, R, C, s + 1 < e ? s + 1 : e - 1, bi, bj, a1, y1);
    term_load_x(A, R + 1, s + 1 < e ? s + 1 : e - 1, bi, b1);
    int64_t u = s;
    for (; u + 1 < e; u += 2) {
      acc0 = term_apply(a0, y0, acc0);
      acc1 = term_apply(b0, y0, acc1);
      term_load(A, R, C, u + 2 < e ? u + 2 : e - 1, bi, bj, a0, y0);
      term_load_x(A, R + 1, u + 2 < e ? u + 2 : e - 1, bi, b0);
      acc0 = term_apply(a1, y1, acc0);
      acc1 = term_apply(b1, y1, acc1);
      term_load(A, R, C, u + 3 < e ? u + 3 : e - 1, bi, bj, a1, y1);
      term_load_x(A, R + 1, u + 3 < e ? u + 3 : e - 1, bi, b1);
    }
    if (u < e) {
      acc0 = term_apply(a0, y0, acc0);
      acc1 = term_apply(b0, y0, acc1);
    }
    s = e;
  }
  return true;
}

template <typename F>
__device__ __attribute__((noinline)) void task_off2(const Args<F>& A_, int64_t R, int64_t C, lds_t<F>* stage,
                                                    lds_i* s_ok) {
  const Args<F> A = A_;
  const int wave = wave_id();
  const int bi = wave & 1, bj = wave >> 1;
  v4_t<F> acc0 = ablk_load(A.a, R, C, bi, bj);
  v4_t<F> acc1 = ablk_load(A.a, R + 1, C, bi, bj);
  const int64_t s0 = R - A.K > 0 ? R - A.K : 0;
  int ok = apply_terms2(A, R, C, s0, C, bi, bj, acc0, acc1) ? 1 : 0;
  if (ok) ok = wave_wait(&A.w.tflag[tidx(A, C, C)], A.w) ? 1 : 0;
  blk_to_lds(stage, bi, bj, acc0);
  blk_to_lds(stage + T * LP, bi, bj, acc1);
  if (!ok && lane_id() == 0) *s_ok = 0;
  __syncthreads();
  if (*s_ok == 0) return;
  const v4_t<F> out0 = trsm_from_lds<F>(stage, A.w.linvt + C * T * T, bi, bj);
  const v4_t<F> out1 = trsm_from_lds<F>(stage + T * LP, A.w.linvt + C * T * T, bi, bj);
  ablk_store(A.a, R, C, bi, bj, out0);
  ablk_store(A.a, R + 1, C, bi, bj, out1);
  wait_vmem();
  __syncthreads();
  if (threadIdx.x == 0) {
    raise_flag(&A.w.tflag[tidx(A, R, C)]);
    raise_flag(&A.w.tflag[tidx(A, R + 1, C)]);
  }
}

// Pre-accumulate the spine's tiles of step m-1: (m, m-1) and (m, m), terms s <= m-3.
template <typename F>
__device__ __attribute__((noinline)) void task_pre(const Args<F>& A_, int64_t m, lds_i* s_ok) {
  const Args<F> A = A_;
  const int wave = wave_id();
  const int64_t s0 = m - A.K > 0 ? m - A.K : 0;
  glb_t<F>* po = A.w.pre + m * 2 * T * T;
  glb_t<F>* pd = po + T * T;
  // waves 0-3: one block of (m, m-1) each; waves 1-3 also one lower block of
  // (m, m).  Both blocks of a wave take each term as soon as its operands are
  // published, so that only the last term is left once the last one arrives.
  int ok = 1;
  const int bi = wave & 1, bj = wave >> 1;
  const int di = (wave >= 2), dj = (wave == 3);
  v4_t<F> acc = ablk_load(A.a, m, m - 1, bi, bj);
  v4_t<F> accd = {0, 0, 0, 0};
  if (wave >= 1) accd = ablk_load(A.a, m, m, di, dj);
  const int lane = lane_id();
  int64_t s = s0;
  while (ok && s < m - 2) {
    // flags of up to 16 terms at once (rows m and m-1), as in apply_terms
    const int span = m - 2 - s < 16 ? (int)(m - 2 - s) : 16;
    int f = 1;
    if (lane < span)
      f = __hip_atomic_load(&A.w.tflag[tidx(A, m, s + lane)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
          __hip_atomic_load(&A.w.tflag[tidx(A, m - 1, s + lane)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long bad = __ballot(lane < span && f == 0);
    int64_t e = s + (bad ? (int)__builtin_ctzll(bad) : span);
    if (e == s) {
      if (!wave_wait(&A.w.tflag[tidx(A, m, s)], A.w) || !wave_wait(&A.w.tflag[tidx(A, m - 1, s)], A.w)) {
        ok = 0;
        break;
      }
      e = s + 1;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");  // keeps the operand loads below the flags
    for (; s < e; ++s) {
      F xf[T / 4], yf[T / 4];
      term_load(A, m, m - 1, s, bi, bj, xf, yf);
      acc = term_apply(xf, yf, acc);
      if (wave >= 1) {
        term_load(A, m, m, s, di, dj, xf, yf);
        accd = term_apply(xf, yf, accd);
      }
    }
  }
  wblk_store(po, bi, bj, acc);
  if (wave >= 1) wblk_store(pd, di, dj, accd);
  if (!ok && lane_id() == 0) *s_ok = 0;
  wait_vmem();
  __syncthreads();
  if (*s_ok == 0) return;
  if (threadIdx.x == 0) raise_flag(&A.w.hflag[m]);
}

// ---------------------------------------------------------------- spine

template <typename F>
struct SpineLds {
  lds_t<F>* diag;    // staged diagonal tile (column-major, LP)
  lds_t<F>* acco;    // staged tile (C+1, C)
  lds_t<F>* accd;    // next diagonal tile before its last update
  lds_t<F>* lcur;    // L(C+1, C)
  lds_t<F>* lprev;   // L(C, C-1)
  lds_t<F>* linvt;   // L(C,C)^{-T}, row-major, row pitch LP
  lds_t<F>* lcc;     // L(C,C) (column-major, LP)
  lds_t<F>* linvt_prev;   // the same two of the previous step, being published
  lds_t<F>* lcc_prev;
};

// Wave 0: the sweep of the staged diagonal tile; L(C,C) and L(C,C)^{-T} go to
// LDS only (both conflict-free: pitch LP); another wave copies them to global
// memory off the critical path.  Takes only scalars and LDS pointers (no
// structures): a structure passed to a noinline function is read back from the
// stack, a memory round trip at the head of the chain.
template <typename F>
__device__ __attribute__((noinline)) void spine_sweep(lds_t<F>* diag, lds_t<F>* lcc, lds_t<F>* linvt, int64_t col0,
                                                      int64_t n, unsigned long long* first_fail, glb_i* abort_flag,
                                                      lds_i* s_fail) {
  const int lane = lane_id();
  F row[T];
#pragma unroll
  for (int c = 0; c < T; ++c) row[c] = lane < T ? diag[c * LP + lane] : ((lane - T) == c ? F(1) : F(0));
  const int fail = sweep_ldlt(row, diag, lcc);  // both free while this wave sweeps
  if (fail >= 0) {
    if (lane == 0) {
      *s_fail = fail;
      const long long col = (long long)col0 + fail;
      if (col < n) atomicMin(first_fail, (unsigned long long)(col + 1));
      __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
#pragma unroll
  for (int c = 0; c < T; ++c) {
    if (lane < T) lcc[c * LP + lane] = row[c];
    else linvt[(lane - T) * LP + c] = row[c];
  }
}

// Waves 1-3 copy the spine's results of step C from LDS to global memory with
// coalesced stores, one part each: wave 1 L(C,C) (lower triangle, from `lcc`),
// wave 2 L(C,C)^{-T} (row-major, for the helpers' trsm, from `linvt`), wave 3
// L(C+1, C) from `lcur` (if `off`).  Does not wait for them.
template <typename F>
__device__ __attribute__((noinline)) void spine_publish(const Args<F>& A_, int64_t C, const lds_t<F>* lcc,
                                                        const lds_t<F>* linvt, const lds_t<F>* lcur, bool off,
                                                        int part) {
  const Args<F> A = A_;
  const BandT<F>& a = A.a;
  const int lane = lane_id();
  const int r = lane & 31;
  // all LDS reads first, then the stores (a store waiting on its own read
  // would serialise the LDS latency)
  F v[T / 2];
  if (part == 1) {
#pragma unroll
    for (int p = 0; p < T / 2; ++p) v[p] = lcc[(2 * p + (lane >> 5)) * LP + r];
    // lane (r, h) stores column 2p + h of row r
    const RunT<F> rd = band_run(a, C * T + r, C * T + (lane >> 5), 2);
#pragma unroll
    for (int p = 0; p < T / 2; ++p)
      if (rd.in(p)) astore(rd.at(p), v[p]);
  } else if (part == 2) {
    glb_t<F>* lt = A.w.linvt + C * T * T;
#pragma unroll
    for (int p = 0; p < T / 2; ++p) {
      const int e = 64 * p + lane;
      v[p] = linvt[(e / T) * LP + (e % T)];
    }
#pragma unroll
    for (int p = 0; p < T / 2; ++p) astore(lt + 64 * p + lane, v[p]);
  } else if (part == 3 && off) {
#pragma unroll
    for (int p = 0; p < T / 2; ++p) v[p] = lcur[(2 * p + (lane >> 5)) * LP + r];
    const RunT<F> ro = band_run(a, (C + 1) * T + r, C * T + (lane >> 5), 2);
#pragma unroll
    for (int p = 0; p < T / 2; ++p)
      if (ro.in(p)) astore(ro.at(p), v[p]);
  }
}

// waves 1-3: tiles (C+1, C) and (C+1, C+1) with everything but the critical
// update.  The 7 lower blocks (4 of (m, C), 3 of (m, m)) go to waves 2 and 3
// three each (b = 0, 2, 4 and 1, 3, 5) and to wave 1 one (b = 6), since wave 1
// also publishes a third of the previous step.  The term s = C-1 uses X = L(m, C-1) for both
// tiles, Y = L(C, C-1) (staged in LDS) for (m, C) and Y = L(m, C-1) for (m, m);
// every global load is issued before the first MFMA.
template <typename F>
__device__ __attribute__((noinline)) void spine_prepare(const Args<F>& A_, int64_t C, const SpineLds<F>& S_,
                                                        lds_i* s_fail) {
  const Args<F> A = A_;
  const SpineLds<F> S = S_;
  const int wave = wave_id();
  const int lane = lane_id();
  const int64_t m = C + 1;
  const bool have_pre = A.K >= 3 && m >= 3;
  const glb_t<F>* po = A.w.pre + m * 2 * T * T;
  const glb_t<F>* pd = po + T * T;
  if (have_pre && !wave_wait(&A.w.hflag[m], A.w)) { if (lane == 0) *s_fail = -2; return; }
  // term s = C-1 needs L(m, C-1) (a helper tile) and L(C, C-1) (S.lprev)
  const bool t1 = C >= 1 && A.K >= 2;
  if (t1 && !wave_wait(&A.w.tflag[tidx(A, m, C - 1)], A.w)) { if (lane == 0) *s_fail = -2; return; }
  v4_t<F> acc[3];
  F x0[T / 4], x1[T / 4];  // fragments of L(m, C-1), rows 0-15 and 16-31
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int b = wave == 1 ? (u == 0 ? 6 : 7) : wave - 2 + 2 * u;
    acc[u] = v4_t<F>{0, 0, 0, 0};
    if (b < 4) {
      const int bi = b & 1, bj = b >> 1;
      acc[u] = have_pre ? wblk_load(po, bi, bj) : ablk_load(A.a, m, C, bi, bj);
    } else if (b < 7) {
      const int bi = (b >= 5), bj = (b == 6);
      acc[u] = have_pre ? wblk_load(pd, bi, bj) : ablk_load(A.a, m, m, bi, bj);
    }
  }
  if (t1) {
    const int64_t j0 = (C - 1) * T + (lane >> 4);
    const RunT<F> r0 = band_run(A.a, m * T + (lane & 15), j0, 4);
    const RunT<F> r1 = band_run(A.a, m * T + 16 + (lane & 15), j0, 4);
#pragma unroll
    for (int q = 0; q < T / 4; ++q) {
      x0[q] = r0.ald(q);
      x1[q] = r1.ald(q);
    }
  }
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int b = wave == 1 ? (u == 0 ? 6 : 7) : wave - 2 + 2 * u;
    if (b < 4) {
      const int bi = b & 1, bj = b >> 1;
      if (t1) {
#pragma unroll
        for (int q = 0; q < T / 4; ++q)
          acc[u] = mfma_xyt(-(bi ? x1[q] : x0[q]), S.lprev[(4 * q + (lane >> 4)) * LP + 16 * bj + (lane & 15)], acc[u]);
      }
      blk_to_lds(S.acco, bi, bj, acc[u]);
    } else if (b < 7) {
      const int bi = (b >= 5), bj = (b == 6);
      if (t1) {
#pragma unroll
        for (int q = 0; q < T / 4; ++q) acc[u] = mfma_xyt(-(bi ? x1[q] : x0[q]), bj ? x1[q] : x0[q], acc[u]);
      }
      blk_to_lds(S.accd, bi, bj, acc[u]);
    }
  }
}

template <typename F>
__device__ void spine(const Args<F>& A, lds_t<F>* base, lds_i* s_fail, lds_i* s_pub) {
  const int wave = wave_id();
  const BandT<F>& a = A.a;
  SpineLds<F> S;
  S.diag = base;
  S.acco = S.diag + T * LP;
  S.accd = S.acco + T * LP;
  S.lcur = S.accd + T * LP;
  S.lprev = S.lcur + T * LP;
  S.linvt = S.lprev + T * LP;
  S.lcc = S.linvt + T * LP;
  S.linvt_prev = S.lcc + T * LP;
  S.lcc_prev = S.linvt_prev + T * LP;
  if (threadIdx.x == 0) {
    *s_fail = -1;
    *s_pub = 0;
  }
  // stage tile (0,0)
  if (wave >= 1) {
    const int bi = (wave >= 2), bj = (wave == 3);
    blk_to_lds(S.diag, bi, bj, ablk_load(a, 0, 0, bi, bj));
  } else {
    blk_to_lds(S.diag, 0, 1, v4_t<F>{0, 0, 0, 0});
  }
  __syncthreads();
  for (int64_t C = 0; C < A.NB; ++C) {
    const bool next = C + 1 < A.NB;
    // waves 1-3 publish step C-1 (its L(C-1,C-1) and inverse sit in the
    // previous-step buffers, L(C,C-1) in lprev) while wave 0 already sweeps
    // step C; each drains its own stores and counts in; the third raises the
    // flags (the prepare below waits, through a helper task, on them)
    if (wave >= 1 && C >= 1) {
      spine_publish(A, C - 1, S.lcc_prev, S.linvt_prev, S.lprev, A.K >= 1, wave);
      wait_vmem();
      if (lane_id() == 0) {
        const int before = __hip_atomic_fetch_add(s_pub, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (before == 3 * (int)C - 1) {
          raise_flag(&A.w.tflag[tidx(A, C - 1, C - 1)]);
          if (A.K >= 1) raise_flag(&A.w.tflag[tidx(A, C, C - 1)]);
        }
      }
    }
    // phase A
    if (wave == 0) spine_sweep<F>(S.diag, S.lcc, S.linvt, C * T, A.a.n, A.w.first_fail, A.w.abort_flag, s_fail);
    else if (next && A.K >= 1) spine_prepare(A, C, S, s_fail);
    else if (next && wave >= 1) {
      const int bi = (wave >= 2), bj = (wave == 3);
      blk_to_lds(S.accd, bi, bj, ablk_load(a, C + 1, C + 1, bi, bj));
    }
    __syncthreads();
    if (*s_fail != -1) return;
    if (!next) {
      if (wave >= 1) spine_publish(A, C, S.lcc, S.linvt, S.lcur, false, wave);
      return;
    }
    // phase B: L(C+1, C) = acco * L(C,C)^{-T}, into LDS
    if (A.K >= 1) {
      const int bi = wave & 1, bj = wave >> 1;
      blk_to_lds(S.lcur, bi, bj, blk_trsm_lds(S.acco, S.linvt, bi, bj, LP));
    }
    __syncthreads();
    // phase C: next diagonal tile (blocks (0,0), (1,0), (1,1) on waves 0, 2, 3)
    if (wave != 1) {
      const int bi = (wave >= 2), bj = (wave == 3);
      v4_t<F> acc = blk_from_lds<F>(S.accd, bi, bj);
      if (A.K >= 1) acc = blk_gemm_lds<F>(S.lcur, S.lcur, bi, bj, acc);
      blk_to_lds<F>(S.diag, bi, bj, acc);
      if (wave == 0) blk_to_lds<F>(S.diag, 0, 1, v4_t<F>{0, 0, 0, 0});
    }
    lds_t<F>* t = S.lprev; S.lprev = S.lcur; S.lcur = t;
    t = S.lcc_prev; S.lcc_prev = S.lcc; S.lcc = t;
    t = S.linvt_prev; S.linvt_prev = S.linvt; S.linvt = t;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- kernel

// Ticket order: 0 = spine; then per column C: O(C+2, C) alone (the spine
// waits on it), O(C+3..C+K, C) in pairs (the last one alone when K is even),
// then H(C+3).
__host__ __device__ __forceinline__ unsigned off_tasks(int K) { return K >= 2 ? 1u + (unsigned)(K - 1) / 2u : 0u; }
__host__ __device__ __forceinline__ unsigned tickets_per_column(int K) {
  return K >= 2 ? off_tasks(K) + (K >= 3 ? 1u : 0u) : 0u;
}

// kind 1: tile (R, C); kind 3: tiles (R, C) and (R+1, C); kind 2: H(R).
template <typename F>
__device__ __forceinline__ void decode(const Args<F>& A, unsigned t, int& kind, int64_t& R, int64_t& C) {
  const unsigned per = tickets_per_column(A.K);
  const unsigned u = t - 1;
  C = u / per;
  const unsigned slot = u % per;
  if (slot == 0) {
    kind = 1;
    R = C + 2;
  } else if (slot < off_tasks(A.K)) {
    R = C + 3 + 2 * (slot - 1);
    kind = (R + 1 <= C + A.K && R + 1 < A.NB) ? 3 : 1;
  } else {
    kind = 2;
    R = C + 3;
  }
}

template <typename F>
__global__ void __launch_bounds__(NT, 2) factor2_kernel(Args<F> A) {
  __shared__ F lds[9 * T * LP];
  __shared__ int s_ticket, s_ok, s_abort, s_pub;
  for (;;) {
    if (threadIdx.x == 0) {
      s_ticket = (int)atomicAdd(A.w.queue, 1u);
      s_abort = aflag(A.w.abort_flag);
    }
    __syncthreads();
    const unsigned t = (unsigned)s_ticket;
    const int stop = s_abort;
    __syncthreads();
    if (threadIdx.x == 0) s_ok = 1;
    __syncthreads();
    if (t >= A.ntickets || stop) break;
    if (t == 0) {
      spine<F>(A, (lds_t<F>*)lds, (lds_i*)&s_ok, (lds_i*)&s_pub);
    } else {
      int kind;
      int64_t R, C;
      decode(A, t, kind, R, C);
      if (R < A.NB) {
        if (kind == 1) task_off<F>(A, R, C, (lds_t<F>*)lds, (lds_i*)&s_ok);
        else if (kind == 3) task_off2<F>(A, R, C, (lds_t<F>*)lds, (lds_i*)&s_ok);
        else task_pre(A, R, (lds_i*)&s_ok);
      }
    }
    __syncthreads();
  }
}

__global__ void factor2_init(glb_i* flags, int64_t count, unsigned* queue, glb_i* abort_flag, unsigned long long* ff,
                             unsigned long long* zero) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t x = g; x < count; x += (int64_t)gridDim.x * blockDim.x) flags[x] = 0;
  if (g == 0) { *queue = 0; *abort_flag = 0; *ff = 0x7fffffffffffffffULL; *zero = 0; }
}

__global__ void factor2_finish(const glb_i* abort_flag, const unsigned long long* ff, int64_t* d_info) {
  const int ab = *abort_flag;
  const unsigned long long f = *ff;
  *d_info = (ab == 2) ? (int64_t)-1001 : (f == 0x7fffffffffffffffULL ? 0 : (int64_t)f);
}

}  // namespace bandchol_f2

// Workspace bytes for n, K (sub-diagonal tile count) and the element size.
static size_t factor2_workspace(int64_t n, int64_t K, size_t elem) {
  using namespace bandchol_f2;
  const int64_t NB = (n + T - 1) / T;
  const size_t flags = sizeof(int) * (size_t)(NB * (K + 1) + NB);
  return 256 + ((flags + 255) & ~(size_t)255) + elem * (size_t)NB * T * T * 3;
}

size_t bandchol_factor2_workspace(int64_t n, int64_t K) { return factor2_workspace(n, K, sizeof(double)); }
size_t bandchol_factor2_workspace_f32(int64_t n, int64_t K) { return factor2_workspace(n, K, sizeof(float)); }

template <typename F>
static hipError_t factor2_launch(int64_t n, int64_t k, F* ab, int64_t ldab, int64_t* d_info, void* ws, int grid_max,
                                 hipStream_t st) {
  using namespace bandchol_f2;
  const int NB = (int)((n + T - 1) / T);
  int K = (int)((k + T - 1) / T);
  if (K > NB - 1) K = NB - 1 > 0 ? NB - 1 : 0;
  char* base = (char*)ws;
  Args<F> A;
  A.a = BandT<F>{(glb_t<F>*)ab, n, k, ldab};
  A.NB = NB;
  A.K = K;
  A.w.queue = (unsigned*)base;
  A.w.abort_flag = (glb_i*)(base + 8);
  A.w.first_fail = (unsigned long long*)(base + 16);
  A.w.zero = (const glb_t<F>*)(base + 64);
  A.w.tflag = (glb_i*)(base + 256);
  A.w.hflag = A.w.tflag + (size_t)NB * (K + 1);
  const size_t flags = sizeof(int) * (size_t)(NB * (K + 1) + NB);
  A.w.linvt = (glb_t<F>*)(base + 256 + ((flags + 255) & ~(size_t)255));
  A.w.pre = A.w.linvt + (size_t)NB * T * T;
  A.ntickets = 1 + tickets_per_column(K) * (unsigned)NB;
  const int64_t nflags = (int64_t)NB * (K + 1) + NB;
  factor2_init<<<(unsigned)((nflags + 255) / 256 > 1024 ? 1024 : (nflags + 255) / 256 + 1), 256, 0, st>>>(
      A.w.tflag, nflags, A.w.queue, A.w.abort_flag, A.w.first_fail, (unsigned long long*)(base + 64));
  int grid = grid_max;
  if ((unsigned)grid > A.ntickets) grid = (int)A.ntickets;
  factor2_kernel<F><<<grid, NT, 0, st>>>(A);
  factor2_finish<<<1, 1, 0, st>>>(A.w.abort_flag, A.w.first_fail, d_info);
  return hipGetLastError();
}

hipError_t bandchol_factor2_launch(int64_t n, int64_t k, double* ab, int64_t ldab, int64_t* d_info, void* ws,
                                   int grid_max, hipStream_t st) {
  return factor2_launch<double>(n, k, ab, ldab, d_info, ws, grid_max, st);
}

hipError_t bandchol_factor2_launch_f32(int64_t n, int64_t k, float* ab, int64_t ldab, int64_t* d_info, void* ws,
                                       int grid_max, hipStream_t st) {
  return factor2_launch<float>(n, k, ab, ldab, d_info, ws, grid_max, st);
}
