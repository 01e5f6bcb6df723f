// Multi-workgroup band Cholesky for wide bands (gfx950; FP64, and FP32 for the
// mixed-precision solver).
//
// Tiles T x T down the band, tile (R, C) for 0 <= R - C <= K.  One workgroup,
// the spine (whoever takes ticket 0), carries the dependency chain along the
// diagonal and the first two sub-diagonals, one tile column per step C:
//   phase A  wave 0: factor the staged diagonal tile (register sweep) ->
//            L(C,C) and L(C,C)^{-T} in LDS;
//            waves 1-3: L(C+1, C-1) from its pre-accumulated sum, the terms
//            the helpers leave and the previous step's L(C-1,C-1)^{-T}; then
//            tile (C+1, C) and the next diagonal tile with the terms s = C-2,
//            C-1;
//   FP64, phase BC: waves 1-3 compute the row blocks of L(C+1, C) = tile *
//            L(C,C)^{-T} that their block of the next diagonal tile needs and
//            subtract L(C+1,C) L(C+1,C)^T from it; wave 0 stores L(C,C) and
//            L(C,C)^{-T};
//   FP32, phase B: all waves: L(C+1, C) = tile * L(C,C)^{-T};
//         phase C: waves 0, 2, 3: next diagonal tile -= L(C+1,C) L(C+1,C)^T.
// Helper workgroups take the other tickets, in an order where every task only
// waits for lower tickets or for spine steps:
//   O(R, C), R - C >= 3: acc = A(R,C) - sum_s L(R,s) L(C,s)^T (terms applied as
//            their operand tiles are published), then L(R,C) = acc L(C,C)^{-T};
//            the tile three below the diagonal alone, then two tiles of one
//            column per task (operands in registers), or for wide bands, from
//            eight below the diagonal on, four per task with the operands
//            staged once per workgroup in LDS;
//   H(m):    the tiles (m, m-1) and (m, m) the spine completes at step m-1,
//            summed over s <= m-4;
//   P(m):    the tile (m, m-2) the spine completes at step m-1, summed over
//            s <= m-4.
// Whatever the spine takes from a helper depends only on spine results at
// least two steps old, so the helpers' round trips stay off its chain.
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
  glb_i* hflag;     // NB: H(m) published
  glb_i* pflag;     // NB: P(m) published
  glb_t<F>* linvt;  // NB*T*T: L(C,C)^{-T}, column-major
  glb_t<F>* pre;    // NB*3*T*T: per m, tiles (m,m-1), (m,m) (from H(m)), (m+1,m-1) (from P(m+1)), column-major
  unsigned* queue;
  glb_i* abort_flag;  // 1 = pivot failure, 2 = wait bound exceeded
  unsigned long long* first_fail;
  glb_i* spine_cu;  // the spine's CU (cu_ident), -1 before it starts
  const glb_t<F>* zero;  // a zero: masked-off lanes load it, so that operand loads are unconditional
  unsigned long long* prof;  // if not null: the spine's phase times, summed over the steps (s_memtime)
};

// Slots of Ws::prof: wave 0's sweep, its wait at the end of phase A, its work
// in phase BC and its wait at the end of it (FP32 schedule: phases B and C);
// per wave w = 1..3 its phase-A work and its wait at the end of phase A; the
// number of steps summed.
enum { PROF_SWEEP, PROF_W0_WAIT, PROF_BC_W0, PROF_BC_WAIT, PROF_W1_WORK, PROF_W1_WAIT, PROF_W2_WORK, PROF_W2_WAIT,
       PROF_W3_WORK, PROF_W3_WAIT, PROF_STEPS, PROF_SLOTS };

__device__ __forceinline__ unsigned long long stamp(bool on) { return on ? __builtin_amdgcn_s_memtime() : 0ull; }

template <typename F>
struct Args {
  BandT<F> a;
  int NB, K;
  unsigned ntickets;
  int spare_spine_cu;  // a helper on the spine's CU stops (only with many workgroups)
  Ws<F> w;
};

// The same value in every lane, in scalar registers.  Arguments of a
// non-inlined function (and structures read through a reference) arrive in
// vector registers; without this every branch on them would be a masked one
// and every address computed from them vector arithmetic.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ unsigned uni(unsigned x) { return (unsigned)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ int64_t uni(int64_t x) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(uint64_t)x);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename P>
__device__ __forceinline__ P* uni(P* p) {
  return (P*)(uintptr_t)uni((int64_t)(uintptr_t)p);
}
template <typename P>
__device__ __forceinline__ __attribute__((address_space(3))) P* uni_lds(__attribute__((address_space(3))) P* p) {
  return (__attribute__((address_space(3))) P*)(uintptr_t)(unsigned)uni((int)(unsigned)(uintptr_t)p);
}

// The fields that the spine's waves 1-3 use in every step, in scalar
// registers; the rest stay in vector registers (all of them in scalar
// registers spilled scalar registers into vector lanes in those waves).
template <typename F>
__device__ __forceinline__ Args<F> uniform_step(const Args<F>& A_) {
  Args<F> A = A_;
  A.a.ab = uni(A_.a.ab), A.a.n = uni(A_.a.n), A.a.k = uni(A_.a.k), A.a.ldab = uni(A_.a.ldab);
  A.NB = uni(A_.NB), A.K = uni(A_.K);
  A.w.tflag = uni(A_.w.tflag), A.w.hflag = uni(A_.w.hflag), A.w.pflag = uni(A_.w.pflag), A.w.pre = uni(A_.w.pre);
  return A;
}

template <typename F>
__device__ __forceinline__ Args<F> uniform(const Args<F>& A_) {
  Args<F> A;
  A.a.ab = uni(A_.a.ab), A.a.n = uni(A_.a.n), A.a.k = uni(A_.a.k), A.a.ldab = uni(A_.a.ldab);
  A.NB = uni(A_.NB), A.K = uni(A_.K), A.ntickets = uni(A_.ntickets), A.spare_spine_cu = uni(A_.spare_spine_cu);
  A.w.tflag = uni(A_.w.tflag), A.w.hflag = uni(A_.w.hflag), A.w.pflag = uni(A_.w.pflag);
  A.w.linvt = uni(A_.w.linvt), A.w.pre = uni(A_.w.pre), A.w.queue = uni(A_.w.queue);
  A.w.abort_flag = uni(A_.w.abort_flag), A.w.first_fail = uni(A_.w.first_fail), A.w.spine_cu = uni(A_.w.spine_cu);
  A.w.zero = uni(A_.w.zero), A.w.prof = uni(A_.w.prof);
  return A;
}

__device__ __forceinline__ int aflag(const glb_i* p) {
  return __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void raise_flag(glb_i* p) { __hip_atomic_store(p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// The CU this wave runs on: HW_ID bits 8-15 (CU, shader array, engine) and the
// XCC number.
__device__ __forceinline__ int cu_ident() {
  const int hw = __builtin_amdgcn_s_getreg(4 | (8 << 6) | (7 << 11));   // HW_ID[15:8]
  const int xcc = __builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11));  // XCC_ID[3:0]
  return hw | (xcc << 8);
}

// This wave waits for *f (bounded); every lane gets the same answer.
template <typename F>
__device__ __forceinline__ bool wave_wait(const glb_i* f, const Ws<F>& w) {
  glb_i* const abort_flag = w.abort_flag;
  long long spins = 0;
  while (!aflag(f)) {
    // the abort flag and the bound every 16th poll: a poll is one memory
    // round trip, and a second load per poll would double the latency at
    // which a raised flag is seen
    if ((++spins & 15) == 0) {
      if (aflag(abort_flag)) return false;
      if (spins > SPIN_LIMIT) {
        __hip_atomic_store(abort_flag, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
    __builtin_amdgcn_s_sleep(1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");  // keeps later loads below the wait
  return true;
}

// One flag per lane (null: none), all polled in one round trip; bounded like wave_wait.
template <typename F>
__device__ __forceinline__ bool wave_wait_lanes(const glb_i* mine, const Ws<F>& w) {
  long long spins = 0;
  for (;;) {
    int v = 1;
    if (mine) v = __hip_atomic_load(mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__ballot(v == 0) == 0) break;
    if ((++spins & 15) == 0) {  // as in wave_wait
      if (aflag(w.abort_flag)) return false;
      if (spins > SPIN_LIMIT) {
        __hip_atomic_store(w.abort_flag, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
    __builtin_amdgcn_s_sleep(1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  return true;
}

// As wave_wait_lanes, with one more flag, `extra` (null: none), polled in
// lane 63 in the same round trips: the first time it reads set, `seen` runs
// (once) and the wait goes on for the others.  Lets a task pick up the
// inverse it will need as soon as that is published, while it still waits
// for its last operands.
template <typename F, typename Seen>
__device__ __forceinline__ bool wave_wait_lanes_or(const glb_i* mine, const glb_i* extra, Seen seen, const Ws<F>& w) {
  const int lane = lane_id();
  long long spins = 0;
  for (;;) {
    const glb_i* p = lane == 63 ? extra : mine;
    int v = 1;
    if (p) v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long z = __ballot(v == 0);
    if (extra && !(z >> 63)) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      seen();
      extra = nullptr;
    }
    if ((z & ~(1ull << 63)) == 0) break;
    if ((++spins & 15) == 0) {  // as in wave_wait
      if (aflag(w.abort_flag)) return false;
      if (spins > SPIN_LIMIT) {
        __hip_atomic_store(w.abort_flag, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
    __builtin_amdgcn_s_sleep(1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  return true;
}

// Up to four flags (null: none), in lanes 0-3.
template <typename F>
__device__ __forceinline__ bool wave_wait4(const glb_i* f0, const glb_i* f1, const glb_i* f2, const glb_i* f3,
                                           const Ws<F>& w) {
  const int lane = lane_id();
  return wave_wait_lanes<F>(lane == 0 ? f0 : lane == 1 ? f1 : lane == 2 ? f2 : lane == 3 ? f3 : nullptr, w);
}

template <typename F>
__device__ __forceinline__ int tidx(const Args<F>& A, int64_t R, int64_t C) { return (int)(R * (A.K + 1) + (R - C)); }

// ---------------------------------------------------------------- block I/O with atomics

// A dense T x T tile in column-major workspace memory, in accumulator form.
template <typename F>
__device__ __forceinline__ int wblk_index(int bi, int bj, int r) {
  const int lane = lane_id();
  return (16 * bj + Prec<F>::acc_col0(lane) + Prec<F>::ACC_STEP * r) * T + 16 * bi + (lane & 15);
}
template <typename F>
__device__ __forceinline__ void wblk_store(glb_t<F>* t, int bi, int bj, v4_t<F> v) {
#pragma unroll
  for (int r = 0; r < 4; ++r) astore<F>(t + wblk_index<F>(bi, bj, r), v[r]);
}

// Block (bi, bj) of tile (R, C) in accumulator form, from `pre` (a dense tile
// in workspace, accumulator order) when not null, else from the band.  The
// four loads are issued unconditionally (positions outside the band read the
// zero word), so that the loads of several blocks stay in flight together: a
// branch around a load, or a use of a value right after its load, makes the
// wave wait for every load still in flight.  On a diagonal tile the positions
// past row n-1 take an identity, applied by blk_ident once a group's loads
// have all been issued.
template <typename F>
__device__ __forceinline__ v4_t<F> blk_issue(const Args<F>& A, const glb_t<F>* pre, int64_t R, int64_t C, int bi,
                                             int bj) {
  const RunT<F> run = acc_run(A.a, R, C, bi, bj);
  v4_t<F> v;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const glb_t<F>* p = pre ? pre + wblk_index<F>(bi, bj, r) : (run.in(r) ? run.at(r) : A.w.zero);
    v[r] = aload<F>(opaque_ptr(p));
  }
  return v;
}

template <typename F>
__device__ __forceinline__ void blk_ident(const BandT<F>& a, int64_t R, int64_t C, int bi, int bj, v4_t<F>& v) {
  if (R != C) return;
  const RunT<F> run = acc_run(a, R, C, bi, bj);
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (!run.row_ok && run.d0 - run.ds * r == 0) v[r] = F(1);
}

template <typename F>
__device__ __forceinline__ void ablk_store(const BandT<F>& a, int64_t R, int64_t C, int bi, int bj, v4_t<F> v) {
  const RunT<F> run = acc_run(a, R, C, bi, bj);
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (run.in(r)) astore(run.at(r), v[r]);
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
// outstanding loads stays exact.  Xrow = R, Yrow = C.  When the wave has to
// wait for the operands of the last term, s1 - 1, it also polls `at_flag`
// (null: not) and runs `at` once that is set (wave_wait_lanes_or).
struct NoAt {
  __device__ void operator()() const {}
};

template <typename F, typename At = NoAt>
__device__ __forceinline__ bool apply_terms(const Args<F>& A, int64_t R, int64_t C, int64_t s0, int64_t s1, int bi, int bj,
                                            v4_t<F>& acc, const glb_i* at_flag = nullptr, At at = At()) {
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
      const glb_i* f0 = &A.w.tflag[tidx(A, R, s)];
      const glb_i* f1 = C != R ? &A.w.tflag[tidx(A, C, s)] : nullptr;
      const bool w = at_flag && s + 1 == s1
                         ? wave_wait_lanes_or<F>(lane == 0 ? f0 : lane == 1 ? f1 : nullptr, at_flag, at, A.w)
                         : wave_wait4<F>(f0, f1, nullptr, nullptr, A.w);
      if (!w) return false;
      e = s + 1;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");  // keeps the operand loads below the flags
    F x0[T / 4], y0[T / 4], x1[T / 4], y1[T / 4];
    term_load(A, R, C, s, bi, bj, x0, y0);
    term_load(A, R, C, s + 1 < e ? s + 1 : e - 1, bi, bj, x1, y1);
    int64_t u = s;
    for (; u + 1 < e; u += 2) {
      acc = term_apply(x0, y0, acc);
      __builtin_amdgcn_sched_barrier(0);
      term_load(A, R, C, u + 2 < e ? u + 2 : e - 1, bi, bj, x0, y0);
      __builtin_amdgcn_sched_barrier(0);
      acc = term_apply(x1, y1, acc);
      __builtin_amdgcn_sched_barrier(0);
      term_load(A, R, C, u + 3 < e ? u + 3 : e - 1, bi, bj, x1, y1);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (u < e) acc = term_apply(x0, y0, acc);
    s = e;
  }
  return true;
}

// The operand fragments of block column bj of L(C,C)^{-T} (column-major in
// global memory; upper triangular, so only the first 4 bj + 4 k-steps), read
// as soon as its flag is seen so that they arrive while the task stages its
// accumulators; used by trsm_frags for every tile of the task.
template <typename F>
__device__ __forceinline__ void linvt_frags(const glb_t<F>* linvt_g, int bj, F (&yf)[T / 4]) {
  const int lane = lane_id();
  const int qmax = 4 * bj + 4;
#pragma unroll
  for (int q = 0; q < T / 4; ++q)
    yf[q] = (q < qmax) ? aload<F>(linvt_g + (16 * bj + (lane & 15)) * T + 4 * q + (lane >> 4)) : F(0);
}
// out = (block row bi of the staged tile x) * (block column bj of the
// inverse); the tile's fragments are all read before the first matrix-core
// step (the scheduling barrier keeps the compiler from sinking each read
// next to its step, with a full LDS wait before each).
template <typename F>
__device__ __forceinline__ v4_t<F> trsm_frags(const lds_t<F>* x, const F (&yf)[T / 4], int bi, int bj) {
  const int lane = lane_id();
  F xf[T / 4];
#pragma unroll
  for (int q = 0; q < T / 4; ++q) xf[q] = x[(4 * q + (lane >> 4)) * LP + 16 * bi + (lane & 15)];
  __builtin_amdgcn_sched_barrier(0);
  v4_t<F> out = {0, 0, 0, 0};
  const int qmax = 4 * bj + 4;
#pragma unroll
  for (int q = 0; q < T / 4; ++q)
    if (q < qmax) out = mfma_xyt(xf[q], yf[q], out);
  return out;
}

// The noinline functions below copy their structure arguments into locals
// first: the references point at a stack copy, and after every atomic store or
// fence the fields would otherwise be re-read from memory.
template <typename F>
__device__ __attribute__((noinline)) void task_off(const Args<F>& A_, int64_t R, int64_t C, lds_t<F>* stage,
                                                   lds_i* s_ok) {
  const Args<F> A = uniform(A_);
  const int wave = wave_id();
  const int bi = wave & 1, bj = wave >> 1;
  v4_t<F> acc = blk_issue<F>(A, nullptr, R, C, bi, bj);
  const int64_t s0 = R - A.K > 0 ? R - A.K : 0;
  // when the inverse is published while the wave still waits for the last
  // term's operands, its fragments load then, off the tail
  F yf[T / 4];
  bool got = false;
  const glb_i* invf = &A.w.tflag[tidx(A, C, C)];
  int ok = apply_terms(A, R, C, s0, C, bi, bj, acc, invf, [&]() {
             linvt_frags<F>(A.w.linvt + C * T * T, bj, yf);
             got = true;
           }) ? 1 : 0;
  if (!got) {
    if (ok) ok = wave_wait(invf, A.w) ? 1 : 0;
    linvt_frags<F>(A.w.linvt + C * T * T, bj, yf);
  }
  blk_to_lds(stage, bi, bj, acc);
  if (!ok && lane_id() == 0) *s_ok = 0;
  __syncthreads();
  if (*s_ok == 0) return;
  const v4_t<F> out = trsm_frags<F>(stage, yf, bi, bj);
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
template <typename F, typename At = NoAt>
__device__ __forceinline__ bool apply_terms2(const Args<F>& A, int64_t R, int64_t C, int64_t s0, int64_t s1, int bi,
                                             int bj, v4_t<F>& acc0, v4_t<F>& acc1, const glb_i* at_flag = nullptr,
                                             At at = At()) {
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
      const glb_i* f0 = &A.w.tflag[tidx(A, R, s)];
      const glb_i* f1 = &A.w.tflag[tidx(A, C, s)];
      const glb_i* f2 = s >= s_in1 ? &A.w.tflag[tidx(A, R + 1, s)] : nullptr;
      const bool w = at_flag && s + 1 == s1
                         ? wave_wait_lanes_or<F>(lane == 0 ? f0 : lane == 1 ? f1 : lane == 2 ? f2 : nullptr, at_flag,
                                                 at, A.w)
                         : wave_wait4<F>(f0, f1, f2, nullptr, A.w);
      if (!w) return false;
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
      __builtin_amdgcn_sched_barrier(0);
      term_load(A, R, C, u + 2 < e ? u + 2 : e - 1, bi, bj, a0, y0);
      term_load_x(A, R + 1, u + 2 < e ? u + 2 : e - 1, bi, b0);
      __builtin_amdgcn_sched_barrier(0);
      acc0 = term_apply(a1, y1, acc0);
      acc1 = term_apply(b1, y1, acc1);
      __builtin_amdgcn_sched_barrier(0);
      term_load(A, R, C, u + 3 < e ? u + 3 : e - 1, bi, bj, a1, y1);
      term_load_x(A, R + 1, u + 3 < e ? u + 3 : e - 1, bi, b1);
      __builtin_amdgcn_sched_barrier(0);
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
  const Args<F> A = uniform(A_);
  const int wave = wave_id();
  const int bi = wave & 1, bj = wave >> 1;
  v4_t<F> acc0 = blk_issue<F>(A, nullptr, R, C, bi, bj);
  v4_t<F> acc1 = blk_issue<F>(A, nullptr, R + 1, C, bi, bj);
  const int64_t s0 = R - A.K > 0 ? R - A.K : 0;
  // one read of the inverse for both tiles; picked up early as in task_off,
  // then parked in this wave's LDS slot (in registers it would be live
  // through the last term's loop, which has none to spare)
  lds_t<F>* park = stage + 2 * T * LP + wave * (T / 4) * 64 + lane_id();
  bool got = false;
  const glb_i* invf = &A.w.tflag[tidx(A, C, C)];
  int ok = apply_terms2(A, R, C, s0, C, bi, bj, acc0, acc1, invf, [&]() {
             F t[T / 4];
             linvt_frags<F>(A.w.linvt + C * T * T, bj, t);
#pragma unroll
             for (int q = 0; q < T / 4; ++q) park[64 * q] = t[q];
             got = true;
           }) ? 1 : 0;
  F yf[T / 4];
  if (got) {
#pragma unroll
    for (int q = 0; q < T / 4; ++q) yf[q] = park[64 * q];
  } else {
    if (ok) ok = wave_wait(invf, A.w) ? 1 : 0;
    linvt_frags<F>(A.w.linvt + C * T * T, bj, yf);
  }
  blk_to_lds(stage, bi, bj, acc0);
  blk_to_lds(stage + T * LP, bi, bj, acc1);
  if (!ok && lane_id() == 0) *s_ok = 0;
  __syncthreads();
  if (*s_ok == 0) return;
  const v4_t<F> out0 = trsm_frags<F>(stage, yf, bi, bj);
  const v4_t<F> out1 = trsm_frags<F>(stage + T * LP, yf, bi, bj);
  ablk_store(A.a, R, C, bi, bj, out0);
  ablk_store(A.a, R + 1, C, bi, bj, out1);
  wait_vmem();
  __syncthreads();
  if (threadIdx.x == 0) {
    raise_flag(&A.w.tflag[tidx(A, R, C)]);
    raise_flag(&A.w.tflag[tidx(A, R + 1, C)]);
  }
}

// Four tiles of one column, O(R0 .. R0+3, C), one per wave (a strip; rows
// past the band or the matrix are absent).  The terms' operands come through
// LDS: per term the workgroup loads the strip's rows of band column block s,
// L(R0..R0+3, s) (in each band column one contiguous run of 4T elements), and
// L(C, s) once, and every wave reads its fragments there.  With operands in
// registers each wave loads its own, so each element of a pair task's
// operands crossed the CU's path to the L2 twice, in half-column pieces that
// straddle cache lines; here once, in whole runs.  The next term's loads are
// in flight while the current one is on the matrix cores.  Wave 0 finds each
// run of published terms and hands its length to the others through LDS, so
// that all waves take the same barriers.
constexpr int SROWS = 4 * T;     // rows of a strip
constexpr int SPX = SROWS + 16;  // LDS pitch of a strip column; 16 mod 32: the fragment reads
constexpr int SPY = T + 16;      // and the L(C, s) pitch cover all banks twice, without conflicts
constexpr int STRIP_D0 = 8;      // strips from the tile STRIP_D0 below the diagonal on (even, >= 6)
constexpr int STRIP_MIN_K = 12;  // and only when K >= STRIP_MIN_K (>= STRIP_D0; below, pairs throughout)

template <typename F>
struct StripLoad {
  F x[SROWS * T / NT];  // strip: element (r, c) with c = 2q + (wave >> 1), r = 64 (wave & 1) + lane
  F y[T * T / NT];      // L(C, s): element (r, c) with c = 8q + 2 wave + (lane >> 5), r = lane & 31
};

template <typename F>
__device__ __forceinline__ void strip_issue(const Args<F>& A, int64_t R0, int64_t C, int64_t s, StripLoad<F>& g) {
  const int wave = wave_id(), lane = lane_id();
  const RunT<F> x = band_run(A.a, R0 * T + 64 * (wave & 1) + lane, s * T + (wave >> 1), 2);
  const RunT<F> y = band_run(A.a, C * T + (lane & 31), s * T + 2 * wave + (lane >> 5), 8);
#pragma unroll
  for (int q = 0; q < SROWS * T / NT; ++q) g.x[q] = aload<F>(opaque_ptr(x.in(q) ? x.at(q) : A.w.zero));
#pragma unroll
  for (int q = 0; q < T * T / NT; ++q) g.y[q] = aload<F>(opaque_ptr(y.in(q) ? y.at(q) : A.w.zero));
}

template <typename F>
__device__ __forceinline__ void strip_put(lds_t<F>* xs, lds_t<F>* ys, const StripLoad<F>& g) {
  const int wave = wave_id(), lane = lane_id();
#pragma unroll
  for (int q = 0; q < SROWS * T / NT; ++q) xs[(2 * q + (wave >> 1)) * SPX + 64 * (wave & 1) + lane] = g.x[q];
#pragma unroll
  for (int q = 0; q < T * T / NT; ++q) ys[(8 * q + 2 * wave + (lane >> 5)) * SPY + (lane & 31)] = g.y[q];
}

// acc[b] -= block (b & 1, b >> 1) of L(R0+wave, s) L(C, s)^T: four independent
// chains.  The fragments of k-step q+1 are read while step q is on the matrix
// cores (the scheduling barriers keep each read ahead of the steps before it).
template <typename F>
__device__ __forceinline__ void strip_apply(const lds_t<F>* xs, const lds_t<F>* ys, int wave, v4_t<F> (&acc)[4]) {
  const int lane = lane_id();
  const lds_t<F>* xw = xs + (lane >> 4) * SPX + T * wave + (lane & 15);
  const lds_t<F>* yw = ys + (lane >> 4) * SPY + (lane & 15);
  F f[2][4];
  f[0][0] = xw[0], f[0][1] = xw[16], f[0][2] = yw[0], f[0][3] = yw[16];
#pragma unroll
  for (int q = 0; q < T / 4; ++q) {
    const int c = q & 1, nx = c ^ 1;
    if (q + 1 < T / 4) {
      f[nx][0] = xw[4 * (q + 1) * SPX], f[nx][1] = xw[4 * (q + 1) * SPX + 16];
      f[nx][2] = yw[4 * (q + 1) * SPY], f[nx][3] = yw[4 * (q + 1) * SPY + 16];
    }
    __builtin_amdgcn_sched_barrier(0);
    acc[0] = mfma_xyt(-f[c][0], f[c][2], acc[0]);
    acc[1] = mfma_xyt(-f[c][1], f[c][2], acc[1]);
    acc[2] = mfma_xyt(-f[c][0], f[c][3], acc[2]);
    acc[3] = mfma_xyt(-f[c][1], f[c][3], acc[3]);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Whether every operand of term u is published (per lane).
template <typename F>
__device__ __forceinline__ int strip_ready(const Args<F>& A, int64_t R0, int64_t C, int64_t u) {
  int f = __hip_atomic_load(&A.w.tflag[tidx(A, C, u)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int64_t R = R0 + w;
    if (R < A.NB && R - u <= A.K)
      f &= __hip_atomic_load(&A.w.tflag[tidx(A, R, u)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return f;
}

// The last term (s = C-1) is not taken through LDS: its operands L(R0.., C-1)
// are the last to be published (by the previous column's strips), so each
// wave waits for its own tile's operands only, loads its fragments itself,
// picks up the inverse meanwhile when that comes first, and publishes its tile
// without waiting for the other three.
template <typename F>
__device__ __attribute__((noinline)) void task_strip(const Args<F>& A_, int64_t R0_, int64_t C_, lds_t<F>* lds,
                                                     lds_i* s_ok, lds_i* s_run) {
  const Args<F> A = uniform(A_);
  const int64_t R0 = uni(R0_), C = uni(C_);
  const int wave = wave_id(), lane = lane_id();
  const int64_t R = R0 + wave;
  const bool mine = R < A.NB && R - C <= A.K;
  v4_t<F> acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = blk_issue<F>(A, nullptr, R, C, b & 1, b >> 1);
  lds_t<F>* xs = lds;
  lds_t<F>* ys = xs + T * SPX;
  const glb_i* invf = &A.w.tflag[tidx(A, C, C)];
  int ok = 1;
  const int64_t s_lo = R0 - A.K > 0 ? R0 - A.K : 0;
  const int64_t s_end = s_lo < C ? C - 1 : C;  // the terms through LDS: [s_lo, s_end)
  int64_t s = s_lo;
  StripLoad<F> g;
  while (s < s_end) {
    if (wave == 0) {
      const int span = s_end - s < 16 ? (int)(s_end - s) : 16;
      const int f = lane < span ? strip_ready(A, R0, C, s + lane) : 1;
      const unsigned long long bad = __ballot(lane < span && f == 0);
      int e = bad ? (int)__builtin_ctzll(bad) : span;
      if (e == 0) {
        const glb_i* mine_f = nullptr;
        if (lane == 0) mine_f = &A.w.tflag[tidx(A, C, s)];
        else if (lane <= 4 && R0 + lane - 1 < A.NB && R0 + lane - 1 - s <= A.K)
          mine_f = &A.w.tflag[tidx(A, R0 + lane - 1, s)];
        e = wave_wait_lanes<F>(mine_f, A.w) ? 1 : -1;
      }
      if (lane == 0) *s_run = e;
    }
    __syncthreads();
    const int e = uni(*s_run);
    if (e < 0) {
      ok = 0;
      break;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");  // keeps the operand loads below the flags
    strip_issue(A, R0, C, s, g);
    wait_vmem();
    strip_put(xs, ys, g);
    __syncthreads();
    for (int u = 0; u < e; ++u) {
      const bool more = u + 1 < e;
      if (more) strip_issue(A, R0, C, s + u + 1, g);
      strip_apply(xs, ys, wave, acc);
      __syncthreads();
      if (more) {
        wait_vmem();
        strip_put(xs, ys, g);
        __syncthreads();
      }
    }
    s += e;
  }
  // From here on each wave goes alone: the LDS terms ended with a barrier, so
  // no wave reads the term buffers any more, and each stages its tile in a
  // region of its own.
  F yf0[T / 4], yf1[T / 4];
  bool got = false;
  if (ok && mine && s_end < C) {
    const int64_t sl = C - 1;
    const glb_i* fy = &A.w.tflag[tidx(A, C, sl)];
    const glb_i* fx = R - sl <= A.K ? &A.w.tflag[tidx(A, R, sl)] : nullptr;  // else L(R, C-1) is outside the band
    ok = wave_wait_lanes_or<F>(lane == 0 ? fy : lane == 1 ? fx : nullptr, invf, [&]() {
           linvt_frags<F>(A.w.linvt + C * T * T, 0, yf0);
           linvt_frags<F>(A.w.linvt + C * T * T, 1, yf1);
           got = true;
         }, A.w) ? 1 : 0;
    F x0[T / 4], x1[T / 4], y0[T / 4], y1[T / 4];
    term_load_x(A, R, sl, 0, x0);
    term_load_x(A, R, sl, 1, x1);
    term_load_x(A, C, sl, 0, y0);
    term_load_x(A, C, sl, 1, y1);
#pragma unroll
    for (int q = 0; q < T / 4; ++q) {
      acc[0] = mfma_xyt(-x0[q], y0[q], acc[0]);
      acc[1] = mfma_xyt(-x1[q], y0[q], acc[1]);
      acc[2] = mfma_xyt(-x0[q], y1[q], acc[2]);
      acc[3] = mfma_xyt(-x1[q], y1[q], acc[3]);
    }
  }
  if (!mine) return;
  if (!got) {
    if (ok) ok = wave_wait(invf, A.w) ? 1 : 0;
    linvt_frags<F>(A.w.linvt + C * T * T, 0, yf0);
    linvt_frags<F>(A.w.linvt + C * T * T, 1, yf1);
  }
  if (!ok) {
    if (lane == 0) *s_ok = 0;
    return;
  }
  lds_t<F>* stage = lds + wave * T * LP;
#pragma unroll
  for (int b = 0; b < 4; ++b) blk_to_lds(stage, b & 1, b >> 1, acc[b]);
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const v4_t<F> out = trsm_frags<F>(stage, (b >> 1) ? yf1 : yf0, b & 1, b >> 1);
    ablk_store(A.a, R, C, b & 1, b >> 1, out);
  }
  wait_vmem();
  if (lane == 0) raise_flag(&A.w.tflag[tidx(A, R, C)]);
}

// H(m): the tiles (m, m-1) and (m, m) the spine completes at step m-1, summed
// over the terms s <= m-4.  Each wave takes one block of (m, m-1) and one of
// (m, m) (waves 1-3 the three lower ones; wave 0 repeats block (0, 0) and
// drops it); every wave loads both row halves of L(m, s) and one of L(m-1, s),
// so that all issue the same loads.  Terms are applied in runs of published
// operands, the next term's operands loading while the current one is on the
// matrix cores, as in apply_terms.
template <typename F>
struct PreOps {
  F x0[T / 4], x1[T / 4], y[T / 4];  // L(m, s) both row halves, L(m-1, s) half bj
};

template <typename F>
__device__ __forceinline__ void pre_load(const Args<F>& A, int64_t m, int64_t s, int bj, PreOps<F>& o) {
  term_load(A, m, m - 1, s, 0, bj, o.x0, o.y);
  term_load_x(A, m, s, 1, o.x1);
}

template <typename F>
__device__ __forceinline__ void pre_apply(const PreOps<F>& o, bool bi, bool di, bool dj, v4_t<F>& acc,
                                          v4_t<F>& accd) {
#pragma unroll
  for (int q = 0; q < T / 4; ++q) {
    acc = mfma_xyt(-(bi ? o.x1[q] : o.x0[q]), o.y[q], acc);
    accd = mfma_xyt(-(di ? o.x1[q] : o.x0[q]), dj ? o.x1[q] : o.x0[q], accd);
  }
}

template <typename F>
__device__ __attribute__((noinline)) void task_pre(const Args<F>& A_, int64_t m, lds_i* s_ok) {
  const Args<F> A = uniform(A_);
  const int wave = wave_id();
  const int lane = lane_id();
  const int64_t s0 = m - A.K > 0 ? m - A.K : 0;
  const int64_t s1 = m - 3;
  glb_t<F>* po = A.w.pre + m * 3 * T * T;
  glb_t<F>* pd = po + T * T;
  const int bi = wave & 1, bj = wave >> 1;
  const int di = (wave >= 2), dj = (wave == 3);
  v4_t<F> acc = blk_issue<F>(A, nullptr, m, m - 1, bi, bj);
  v4_t<F> accd = blk_issue<F>(A, nullptr, m, m, di, dj);
  blk_ident(A.a, m, m, di, dj, accd);
  int ok = 1;
  int64_t s = s0;
  while (s < s1) {
    // flags of up to 16 terms at once, as in apply_terms
    const int span = s1 - s < 16 ? (int)(s1 - s) : 16;
    int f = 1;
    if (lane < span)
      f = __hip_atomic_load(&A.w.tflag[tidx(A, m, s + lane)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
          __hip_atomic_load(&A.w.tflag[tidx(A, m - 1, s + lane)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long bad = __ballot(lane < span && f == 0);
    int64_t e = s + (bad ? (int)__builtin_ctzll(bad) : span);
    if (e == s) {
      if (!wave_wait4<F>(&A.w.tflag[tidx(A, m, s)], &A.w.tflag[tidx(A, m - 1, s)], nullptr, nullptr, A.w)) {
        ok = 0;
        break;
      }
      e = s + 1;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");  // keeps the operand loads below the flags
    PreOps<F> o0, o1;
    pre_load(A, m, s, bj, o0);
    pre_load(A, m, s + 1 < e ? s + 1 : e - 1, bj, o1);
    int64_t u = s;
    for (; u + 1 < e; u += 2) {
      pre_apply(o0, bi, di, dj, acc, accd);
      __builtin_amdgcn_sched_barrier(0);
      pre_load(A, m, u + 2 < e ? u + 2 : e - 1, bj, o0);
      __builtin_amdgcn_sched_barrier(0);
      pre_apply(o1, bi, di, dj, acc, accd);
      __builtin_amdgcn_sched_barrier(0);
      pre_load(A, m, u + 3 < e ? u + 3 : e - 1, bj, o1);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (u < e) pre_apply(o0, bi, di, dj, acc, accd);
    s = e;
  }
  wblk_store(po, bi, bj, acc);
  if (wave >= 1) wblk_store(pd, di, dj, accd);
  if (!ok && lane_id() == 0) *s_ok = 0;
  wait_vmem();
  __syncthreads();
  if (*s_ok == 0) return;
  if (threadIdx.x == 0) raise_flag(&A.w.hflag[m]);
}

// P(m): the tile (m, m-2) the spine completes at step m-1, summed over the
// terms s <= m-4, into the workspace slot of row m-1.  Its last term uses
// L(m, m-4), a tile of the first pair of column m-4, and L(m-2, m-4), which
// the spine publishes at the start of step m-2: one step before it is needed.
template <typename F>
__device__ __attribute__((noinline)) void task_p(const Args<F>& A_, int64_t m, lds_i* s_ok) {
  const Args<F> A = uniform(A_);
  const int wave = wave_id();
  const int bi = wave & 1, bj = wave >> 1;
  v4_t<F> acc = blk_issue<F>(A, nullptr, m, m - 2, bi, bj);
  const int64_t s0 = m - A.K > 0 ? m - A.K : 0;
  const int ok = apply_terms(A, m, m - 2, s0, m - 3, bi, bj, acc) ? 1 : 0;
  wblk_store(A.w.pre + (m - 1) * 3 * T * T + 2 * T * T, bi, bj, acc);
  if (!ok && lane_id() == 0) *s_ok = 0;
  wait_vmem();
  __syncthreads();
  if (*s_ok == 0) return;
  if (threadIdx.x == 0) raise_flag(&A.w.pflag[m]);
}

// ---------------------------------------------------------------- spine

template <typename F>
struct SpineLds {
  lds_t<F>* diag;        // staged diagonal tile D(C) (column-major, LP); scratch of the sweep
  lds_t<F>* sd;          // T values, scratch of the sweep
  lds_t<F>* linvt;       // L(C,C)^{-T}, row-major, row pitch LP
  lds_t<F>* linvt_prev;  // L(C-1,C-1)^{-T}
  lds_t<F>* acco;        // tile (C+1, C) before its trsm
  lds_t<F>* accd;        // tile (C+1, C+1) before its last term
  lds_t<F>* lcur;        // L(C+1, C) from phase B; in phase A first L(C-1, C-2) (two steps old),
                         // then (FP32) the staged tile (C+1, C-1)
  lds_t<F>* lprev;       // L(C, C-1)
  lds_t<F>* l2cur;       // L(C+1, C-1); in phase A first L(C-1, C-3) (two steps old)
  lds_t<F>* l2prev;      // L(C, C-2)
};

template <typename F>
__device__ __forceinline__ SpineLds<F> uniform(const SpineLds<F>& S_) {
  SpineLds<F> S;
  S.diag = uni_lds(S_.diag), S.sd = uni_lds(S_.sd), S.linvt = uni_lds(S_.linvt);
  S.linvt_prev = uni_lds(S_.linvt_prev), S.acco = uni_lds(S_.acco), S.accd = uni_lds(S_.accd);
  S.lcur = uni_lds(S_.lcur), S.lprev = uni_lds(S_.lprev), S.l2cur = uni_lds(S_.l2cur), S.l2prev = uni_lds(S_.l2prev);
  return S;
}

// An inverse from LDS (row-major, pitch LP) to the workspace, column-major:
// store p covers elements 64p .. 64p+63.  Not waited for.
template <typename F>
__device__ __forceinline__ void store_linvt(const lds_t<F>* linvt, glb_t<F>* dst) {
  const int lane = lane_id();
  const int r = lane & 31, h = lane >> 5;
  F v[T / 2];
#pragma unroll
  for (int p = 0; p < T / 2; ++p) v[p] = linvt[r * LP + 2 * p + h];  // element (r, 2p + h)
#pragma unroll
  for (int p = 0; p < T / 2; ++p) astore(dst + 64 * p + lane, v[p]);
}

// Wave 0: the sweep of the staged diagonal tile D(C); L(C,C) replaces the
// tile in its LDS buffer (column-major, pitch LP) and L(C,C)^{-T} goes to
// `linvt` (row-major, pitch LP).  With `flag_prev` (the FP32 schedule), the
// previous step's inverse, `linvt_prev`, is first copied to `lt_prev`, and
// between the two halves of the sweep, once those stores have long
// completed, `flag_prev` is raised: the helpers' trsm takes L(C-1,C-1)^{-T}
// from there.  (The FP64 schedule stores the inverse right after the sweep,
// from wave 0, which is free then, and `flag_stored` is raised here, at the
// start of the next sweep, once those stores have drained.)
template <typename F>
__device__ __forceinline__ void spine_sweep(lds_t<F>* diag, lds_t<F>* sd, lds_t<F>* linvt, const lds_t<F>* linvt_prev,
                                            glb_t<F>* lt_prev, glb_i* flag_prev, glb_i* flag_stored, int64_t C, int64_t n,
                                            unsigned long long* first_fail, glb_i* abort_flag, lds_i* s_fail) {
  const int lane = lane_id();
  if (flag_prev) store_linvt(linvt_prev, lt_prev);
  // every lane reads (lanes >= T a row they then drop for the identity), so
  // that no read sits behind a branch
  F row[T];
#pragma unroll
  for (int c = 0; c < T; ++c) row[c] = diag[c * LP + (lane & (T - 1))];
#pragma unroll
  for (int c = 0; c < T; ++c) row[c] = lane < T ? row[c] : ((lane - T) == c ? F(1) : F(0));
  if (flag_stored) {
    wait_vmem();
    if (lane == 0) raise_flag(flag_stored);
  }
  auto mid = [flag_prev, lane]() {
    if (flag_prev) {
      wait_vmem();
      if (lane == 0) raise_flag(flag_prev);
    }
  };
  const int fail = sweep_ldlt(row, diag, sd, mid);  // the tile is in registers: its LDS is scratch
  if (fail >= 0) {
    if (lane == 0) {
      *s_fail = fail;
      const long long col = (long long)C * T + fail;
      if (col < n) atomicMin(first_fail, (unsigned long long)(col + 1));
      __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  // lane < T: row lane of L(C,C) into diag (column-major); lane >= T: row
  // lane - T of L^{-T} into linvt (row-major); one write per column, each
  // lane through its own base and stride (no branch per column)
  lds_t<F>* const p0 = lane < T ? diag + lane : linvt + (lane - T) * LP;
  const int step = lane < T ? LP : 1;
#pragma unroll
  for (int c = 0; c < T; ++c) p0[c * step] = row[c];
}

// L(C,C) from LDS (column-major, pitch LP) to the band, lower triangle: lane
// (r, h) stores column 2p + h of row r.  Not waited for; four values at a
// time keep the registers it needs inside the kernel few (all sixteen at
// once made wave 0 spill).
template <typename F>
__device__ __forceinline__ void store_lcc(const lds_t<F>* lcc, int64_t C, const BandT<F>& a) {
  const int lane = lane_id();
  const int r = lane & 31, h = lane >> 5;
  const RunT<F> rd = band_run(a, C * T + r, C * T + h, 2);
#pragma unroll 1
  for (int p0 = 0; p0 < T / 2; p0 += 4) {
    F v[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) v[p] = lcc[(2 * (p0 + p) + h) * LP + r];
#pragma unroll
    for (int p = 0; p < 4; ++p)
      if (rd.in(p0 + p)) astore(rd.at(p0 + p), v[p]);
  }
}

// Workgroup barrier for the LDS data of the spine: this wave's LDS accesses
// complete (lgkmcnt(0)), then s_barrier; global stores, which only other
// workgroups read (after a flag raised once they have drained), are not
// waited for.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// The helper flags step C of the spine waits for (null: not needed there).
template <typename F>
struct StepFlags {
  const glb_i* f[4];
};
template <typename F>
__device__ __forceinline__ StepFlags<F> step_flags(const Args<F>& A, int64_t C) {
  const int K = A.K;
  const int64_t m = C + 1;
  StepFlags<F> r;
  r.f[0] = K >= 4 && m >= 4 ? &A.w.hflag[m] : nullptr;                // H(m)
  r.f[1] = K >= 4 && m >= 4 ? &A.w.pflag[m] : nullptr;                // P(m)
  r.f[2] = K >= 3 && C >= 2 ? &A.w.tflag[tidx(A, m, C - 2)] : nullptr;  // L(m, C-2)
  r.f[3] = nullptr;
  return r;
}

// Flags between waves 1-3 inside phase A, where wave 0 is sweeping and no
// workgroup barrier can be used.  A wave's LDS accesses reach the LDS in
// order, so a flag written after a wave's data is seen after that data.
__device__ __forceinline__ void lds_signal(lds_i* f, int v) {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  if (lane_id() == 0) __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ bool lds_wait(lds_i* f, int v) {
  int spins = 0;
  while (__builtin_amdgcn_readfirstlane(__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) < v) {
    if (++spins > (1 << 24)) return false;
    __builtin_amdgcn_s_sleep(0);
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  return true;
}

// The flags of L(C, C-1) and L(C, C-2), raised by the last of waves 1-3 to
// count in once its own stores of them have drained.  In the FP64 schedule
// all those stores were issued in the previous step (L(C, C-2) in its phase A,
// L(C, C-1) in its phase BC), and this runs at the start of phase A, where
// the wait costs little; in the FP32 one wave 1 stores a block of L(C, C-1)
// during phase A, and this runs at its end.
template <typename F>
__device__ __forceinline__ void publish_prev(const Args<F>& A, int64_t C, lds_i* s_pub) {
  wait_vmem();
  if (C >= 1 && lane_id() == 0) {
    const int before = __hip_atomic_fetch_add(s_pub, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (before == 3 * (int)C - 1) {
      if (A.K >= 1) raise_flag(&A.w.tflag[tidx(A, C, C - 1)]);
      if (A.K >= 2 && C >= 2) raise_flag(&A.w.tflag[tidx(A, C, C - 2)]);
    }
  }
}

// FP32 phase A of step C (m = C+1) on waves 1-3, alongside the sweep (the
// FP32 accumulators are not operands, so tiles pass through LDS):
//   * tile (m, C-1): the helpers' sum over s <= C-3 (P(m)), here the term
//     s = C-2 (operand L(C-1, C-2) still in LDS), then L(m, C-1) = tile
//     L(C-1,C-1)^{-T} (the previous sweep's inverse, also still in LDS); row
//     half h on wave 1+h;
//   * tiles (m, C) and (m, m): the helpers' sums over s <= C-3 (H(m)); here
//     s = C-2 (wave 3, all blocks), then s = C-1 with the new L(m, C-1)
//     (waves 1 and 2 their row half, wave 3 block (1, 0) of (m, m));
//   * publication of the previous step (publish_prev) at the end, after wave
//     1 has stored wave 0's block of L(C, C-1) from LDS (after its own loads,
//     which would otherwise wait for that store).
template <typename F>
__device__ __forceinline__ void spine_prepare32(const Args<F>& A, int64_t C, const SpineLds<F>& S, bool next,
                                                lds_i* sync, lds_i* s_pub, lds_i* s_fail, int& early) {
  const int wave = wave_id();
  const int lane = lane_id();
  const int K = A.K;
  const int64_t m = C + 1;
  const bool copy0 = C >= 1 && K >= 1;  // wave 1 stores wave 0's block of L(C, C-1)
  if (next) {
    const bool pre_o = K >= 4 && m >= 4;  // (m, C), (m, m) from H(m)
    const bool pre_p = K >= 4 && m >= 4;  // (m, C-1) from P(m)
    const bool has_p = K >= 2 && C >= 1;  // tile (m, C-1) is inside the band
    const bool t2 = K >= 3 && C >= 2;     // term s = C-2: L(m, C-2)
    const int tag = (int)C + 1;
    // `early`: this lane's flag as read at the end of the previous step (1 if
    // none is needed); all set means no poll now
    bool ok = true;
    if (__ballot(early == 0) != 0) {
      const StepFlags<F> fl = step_flags(A, C);
      ok = wave_wait4(fl.f[0], fl.f[1], fl.f[2], fl.f[3], A.w);
    } else {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");  // keeps the operand loads below the flags
    }
    if (wave == 3) {
      const glb_t<F>* po = A.w.pre + m * 3 * T * T;
      v4_t<F> acc[7];  // blocks 0-3: (m, C), b -> (b & 1, b >> 1); 4-6: (m, m), (0,0) (1,0) (1,1)
      F x3[2][T / 4];
#pragma unroll
      for (int b = 0; b < 7; ++b) {
        const int bi = b < 4 ? (b & 1) : (b >= 5), bj = b < 4 ? (b >> 1) : (b == 6);
        acc[b] = blk_issue<F>(A, pre_o ? po + (b < 4 ? 0 : T * T) : nullptr, m, b < 4 ? C : m, bi, bj);
      }
      if (t2) {
        term_load_x(A, m, C - 2, 0, x3[0]);
        term_load_x(A, m, C - 2, 1, x3[1]);
      }
      if (!pre_o) {
#pragma unroll
        for (int b = 4; b < 7; ++b) blk_ident(A.a, m, m, b >= 5, b == 6, acc[b]);
      }
      if (t2) {
#pragma unroll
        for (int b = 0; b < 7; ++b) {
          const int bi = b < 4 ? (b & 1) : (b >= 5), bj = b < 4 ? (b >> 1) : (b == 6);
#pragma unroll
          for (int q = 0; q < T / 4; ++q) {
            const F y = b < 4 ? S.l2prev[(4 * q + (lane >> 4)) * LP + 16 * bj + (lane & 15)] : x3[bj][q];
            acc[b] = mfma_xyt(-x3[bi][q], y, acc[b]);
          }
        }
      }
#pragma unroll
      for (int b = 0; b < 7; ++b) {
        const int bi = b < 4 ? (b & 1) : (b >= 5), bj = b < 4 ? (b >> 1) : (b == 6);
        blk_to_lds(b < 4 ? S.acco : S.accd, bi, bj, acc[b]);
      }
      lds_signal(&sync[2], tag);
      if (has_p) {
        if (!lds_wait(&sync[0], tag) || !lds_wait(&sync[1], tag)) {
          ok = false;
        } else {
          v4_t<F> v = blk_from_lds<F>(S.accd, 1, 0);
          v = blk_gemm_lds<F>(S.l2cur, S.l2cur, 1, 0, v);
          blk_to_lds(S.accd, 1, 0, v);
        }
      }
    } else {
      const int h = wave - 1;
      if (has_p) {
        v4_t<F> pp[2];
        F x3[T / 4], y1[2][T / 4];
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
          pp[bj] = blk_issue<F>(A, pre_p ? A.w.pre + C * 3 * T * T + 2 * T * T : nullptr, m, C - 1, h, bj);
        if (t2) term_load_x(A, m, C - 2, h, x3);
        // L(C-1, C-2), computed by the spine two steps ago, still sits in the
        // buffer now called lcur: both waves read it before either stages its
        // tile there
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int q = 0; q < T / 4; ++q)
            y1[bj][q] = t2 ? S.lcur[(4 * q + (lane >> 4)) * LP + 16 * bj + (lane & 15)] : F(0);
        lds_signal(&sync[3 + h], tag);
        if (!lds_wait(&sync[4 - h], tag)) ok = false;
        if (t2) {
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) pp[bj] = term_apply(x3, y1[bj], pp[bj]);
        }
        v4_t<F> out[2];  // row half h of L(m, C-1), blocks (h, 0) and (h, 1)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) blk_to_lds(S.lcur, h, bj, pp[bj]);
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) out[bj] = blk_trsm_lds<F>(S.lcur, S.linvt_prev, h, bj, LP);
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          blk_to_lds(S.l2cur, h, bj, out[bj]);
          ablk_store(A.a, m, C - 1, h, bj, out[bj]);
        }
      }
      if (wave == 1 && copy0) ablk_store(A.a, C, C - 1, 0, 0, blk_from_lds<F>(S.lprev, 0, 0));
      lds_signal(&sync[h], tag);
      if (!lds_wait(&sync[2], tag)) {
        ok = false;
      } else if (has_p) {
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          v4_t<F> v = blk_from_lds<F>(S.acco, h, bj);
          v = blk_gemm_lds<F>(S.l2cur, S.lprev, h, bj, v);
          blk_to_lds(S.acco, h, bj, v);
        }
        v4_t<F> v = blk_from_lds<F>(S.accd, h, h);
        v = blk_gemm_lds<F>(S.l2cur, S.l2cur, h, h, v);
        blk_to_lds(S.accd, h, h, v);
      }
    }
    if (!ok && lane == 0) *s_fail = -2;
  } else if (wave == 1 && copy0) {
    ablk_store(A.a, C, C - 1, 0, 0, blk_from_lds<F>(S.lprev, 0, 0));
  }
  publish_prev(A, C, s_pub);
  // the next step's flags, read now and used then (a load in flight meanwhile)
  early = 1;
  if (C + 2 < A.NB && lane < 4) {
    const glb_i* f = step_flags(A, C + 1).f[lane];
    if (f) early = __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Steady-state loads of the FP64 phase A: a dense workspace tile, or a band
// tile that lies wholly inside the band, addressed as a uniform base (scalar
// arithmetic) plus a lane offset, with no per-element test.
template <typename F>
__device__ __forceinline__ int wblk_lane_off() {
  const int lane = lane_id();
  return Prec<F>::acc_col0(lane) * T + (lane & 15);
}
template <typename F>
__device__ __forceinline__ v4_t<F> wblk_ld(const glb_t<F>* tile, int lane_off, int bi, int bj) {
  v4_t<F> v;
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = aload<F>(tile + ((16 * bj + Prec<F>::ACC_STEP * r) * T + 16 * bi) + lane_off);
  return v;
}
// X operand (rows 16 bi .. of tile (Rx, s)) of a tile wholly inside the band
// and above row n: the same elements as term_load_x.
template <typename F>
__device__ __forceinline__ void x_ld(const Args<F>& A, int64_t Rx, int64_t s, int bi, F (&xf)[T / 4]) {
  const int lane = lane_id();
  const int64_t l1 = A.a.ldab - 1;
  const glb_t<F>* base = A.a.ab + (Rx * T + 16 * bi) + s * T * l1;
  const int off = (lane & 15) + (lane >> 4) * (int)l1;
#pragma unroll
  for (int q = 0; q < T / 4; ++q) xf[q] = aload<F>(base + 4 * q * l1 + off);
}
// Whether tile (Rx, Rx-3) lies wholly inside the band and above row n.
template <typename F>
__device__ __forceinline__ bool x3_inside(const Args<F>& A, int64_t Rx) {
  return A.a.k >= 4 * T - 1 && (Rx + 1) * T <= A.a.n;
}

// FP64 phase A of step C (m = C+1) on waves 1-3, alongside the sweep.  Wave
// 1+h (h = 0, 1) owns row half h of the tiles (m, C-1) and (m, C), wave 3 the
// tile (m, m), so that no wave waits for another's matrix-core work except
// wave 3 for L(m, C-1):
//   * row half h of (m, C-1): from P(m) (the helpers' sum over s <= C-3) or
//     the band, the term s = C-2,
//     then L(m, C-1) = that * L(C-1,C-1)^{-T} (the previous sweep's inverse,
//     still in LDS): kept in registers, staged in l2cur and stored;
//   * row half h of (m, C): from H(m) (the helpers' sum over s <= C-3) or the
//     band, the terms s = C-2 and s = C-1 (the latter with L(m, C-1) straight
//     from the registers), staged in acco;
//   * wave 3, (m, m): from H(m) or the band, the term s = C-2, then, once
//     both row halves of L(m, C-1) are in l2cur, s = C-1; staged in accd.
template <typename F>
__device__ __forceinline__ void spine_prepare64(const Args<F>& A, int64_t C, const SpineLds<F>& S, bool next,
                                                lds_i* sync, lds_i* s_pub, lds_i* s_fail, int& early) {
  const int wave = wave_id();
  const int lane = lane_id();
  const int K = A.K;
  const int64_t m = C + 1;
  publish_prev(A, C, s_pub);
  if (next) {
    const bool pre_o = K >= 4 && m >= 4;  // (m, C), (m, m) from H(m)
    const bool pre_p = K >= 4 && m >= 4;  // (m, C-1) from P(m)
    const bool has_p = K >= 2 && C >= 1;  // tile (m, C-1) is inside the band
    const bool t2 = K >= 3 && C >= 2;     // term s = C-2: L(m, C-2)
    // (the term s = C-3 of (m, C-1) is in P(m) wherever the band holds it)
    const int tag = (int)C + 1;
    // `early`: this lane's flag as read at the end of the previous step (1 if
    // none is needed); all set means no poll now
    bool ok = true;
    if (__ballot(early == 0) != 0) {
      const StepFlags<F> fl = step_flags(A, C);
      ok = wave_wait4(fl.f[0], fl.f[1], fl.f[2], fl.f[3], A.w);
    } else {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");  // keeps the operand loads below the flags
    }
    const int loff = wblk_lane_off<F>();
    const bool x3_in = t2 && x3_inside(A, m);
    if (wave == 3) {
      v4_t<F> ad[3];  // blocks (0,0), (1,0), (1,1) of (m, m)
      F x3[2][T / 4];
      if (pre_o) {
#pragma unroll
        for (int b = 0; b < 3; ++b) ad[b] = wblk_ld<F>(A.w.pre + m * 3 * T * T + T * T, loff, b >= 1, b == 2);
      } else {
#pragma unroll
        for (int b = 0; b < 3; ++b) ad[b] = blk_issue<F>(A, nullptr, m, m, b >= 1, b == 2);
      }
      if (x3_in) {
        x_ld(A, m, C - 2, 0, x3[0]);
        x_ld(A, m, C - 2, 1, x3[1]);
      } else if (t2) {
        term_load_x(A, m, C - 2, 0, x3[0]);
        term_load_x(A, m, C - 2, 1, x3[1]);
      }
      if (!pre_o) {
#pragma unroll
        for (int b = 0; b < 3; ++b) blk_ident(A.a, m, m, b >= 1, b == 2, ad[b]);
      }
      if (t2) {
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
          for (int q = 0; q < T / 4; ++q) ad[b] = mfma_xyt(-x3[b >= 1][q], x3[b == 2][q], ad[b]);
      }
      if (has_p) {
        if (!lds_wait(&sync[0], tag) || !lds_wait(&sync[1], tag)) {
          ok = false;
        } else {
#pragma unroll
          for (int b = 0; b < 3; ++b) ad[b] = blk_gemm_lds<F>(S.l2cur, S.l2cur, b >= 1, b == 2, ad[b]);
        }
      }
#pragma unroll
      for (int b = 0; b < 3; ++b) blk_to_lds(S.accd, b >= 1, b == 2, ad[b]);
    } else {
      const int h = wave - 1;
      v4_t<F> ao[2];   // row half h of (m, C)
      v4_t<F> out[2];  // row half h of L(m, C-1)
      F x3[T / 4];
      if (pre_o) {
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) ao[bj] = wblk_ld<F>(A.w.pre + m * 3 * T * T, loff, h, bj);
      } else {
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) ao[bj] = blk_issue<F>(A, nullptr, m, C, h, bj);
      }
      if (x3_in) x_ld(A, m, C - 2, h, x3);
      else if (t2) term_load_x(A, m, C - 2, h, x3);
      if (has_p) {
        v4_t<F> pp[2];
        F y1[2][T / 4];
        if (pre_p) {
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) pp[bj] = wblk_ld<F>(A.w.pre + C * 3 * T * T + 2 * T * T, loff, h, bj);
        } else {
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) pp[bj] = blk_issue<F>(A, nullptr, m, C - 1, h, bj);
        }
        // L(C-1, C-2), computed by the spine two steps ago, still sits in lcur
        // (overwritten only in phase BC)
        if (t2) {
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int q = 0; q < T / 4; ++q) y1[bj][q] = S.lcur[(4 * q + (lane >> 4)) * LP + 16 * bj + (lane & 15)];
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) pp[bj] = term_apply(x3, y1[bj], pp[bj]);
        }
        // L(m, C-1) = P L(C-1,C-1)^{-T} straight from the accumulators
        // (L^{-T} upper triangular: block (h, 0) takes columns 0-15 of P only)
        out[0] = out[1] = v4_t<F>{0, 0, 0, 0};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int kk = 16 * kb + 4 * r + (lane >> 4);
            if (kb == 0) out[0] = mfma_xyt(pp[0][r], S.linvt_prev[kk * LP + (lane & 15)], out[0]);
            out[1] = mfma_xyt(pp[kb][r], S.linvt_prev[kk * LP + 16 + (lane & 15)], out[1]);
          }
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) blk_to_lds(S.l2cur, h, bj, out[bj]);
        lds_signal(&sync[h], tag);
      }
      // (m, C): s = C-2 with L(C, C-2) (l2prev), s = C-1 with L(C, C-1)
      // (lprev); the stores of L(m, C-1) go out between the matrix-core
      // steps of the first term, which leave the wave idle while each runs
      const RunT<F> run0 = acc_run(A.a, m, C - 1, h, 0), run1 = acc_run(A.a, m, C - 1, h, 1);
      if (t2) {
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int q = 0; q < T / 4; ++q) {
            ao[bj] = mfma_xyt(-x3[q], S.l2prev[(4 * q + (lane >> 4)) * LP + 16 * bj + (lane & 15)], ao[bj]);
            if (has_p && (q & 1)) {
              const RunT<F>& run = bj ? run1 : run0;
              if (run.in(q >> 1)) astore(run.at(q >> 1), out[bj][q >> 1]);
            }
          }
      } else if (has_p) {
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) ablk_store(A.a, m, C - 1, h, bj, out[bj]);
      }
      if (has_p) {
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              ao[bj] = mfma_xyt(-out[kb][r], S.lprev[(16 * kb + 4 * r + (lane >> 4)) * LP + 16 * bj + (lane & 15)],
                                ao[bj]);
      }
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) blk_to_lds(S.acco, h, bj, ao[bj]);
    }
    if (!ok && lane == 0) *s_fail = -2;
  }
  // the next step's flags, read now and used then (a load in flight meanwhile)
  early = 1;
  if (C + 2 < A.NB && lane < 4) {
    const glb_i* f = step_flags(A, C + 1).f[lane];
    if (f) early = __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// The spine's steps, one function for wave 0 and one for waves 1-3, each
// called once: no call inside the step loop (a call makes the loop's live
// values spill, and their reloads wait for every store in flight), and the
// kernel's registers, allocated for the helper tasks, stay out of it.  Both
// pass the same three barriers per step.
template <typename F>
__device__ __attribute__((noinline)) void spine_wave0(const Args<F>& A_, const SpineLds<F>& S_, lds_i* s_fail) {
  // (left in vector registers: the sweep needs the scalar registers for its
  // lane reads)
  const Args<F> A = A_;
  SpineLds<F> S = S_;
  const BandT<F>& a = A.a;
  const bool prof = A.w.prof != nullptr;
  unsigned long long p_sweep = 0, p_wait = 0, p_b = 0, p_c = 0, steps = 0;
  for (int64_t C = 0; C < A.NB; ++C) {
    const bool next = C + 1 < A.NB;
    const unsigned long long t0 = stamp(prof);
    // phase A
    spine_sweep<F>(S.diag, S.sd, S.linvt, S.linvt_prev, A.w.linvt + (C - 1) * T * T,
                   !acc_is_operand<F>() && C >= 1 ? &A.w.tflag[tidx(A, C - 1, C - 1)] : nullptr,
                   acc_is_operand<F>() && C >= 1 ? &A.w.tflag[tidx(A, C - 1, C - 1)] : nullptr, C, a.n,
                   A.w.first_fail, A.w.abort_flag, s_fail);
    const unsigned long long t1 = stamp(prof);
    lds_barrier();
    const unsigned long long t2 = stamp(prof);
    if (*s_fail != -1 || !next) {
      if (prof && lane_id() == 0) {
        A.w.prof[PROF_SWEEP] = p_sweep, A.w.prof[PROF_W0_WAIT] = p_wait, A.w.prof[PROF_BC_W0] = p_b;
        A.w.prof[PROF_BC_WAIT] = p_c, A.w.prof[PROF_STEPS] = steps;
      }
      return;
    }
    if constexpr (acc_is_operand<F>()) {
      // phase BC (waves 1-3 finish L(C+1, C) and the next diagonal tile):
      // store L(C,C)^{-T} for the helpers' trsm (its flag is raised at the
      // start of the next sweep, once the stores have drained) and L(C,C), and
      // zero the upper block of the next diagonal tile (staged in accd's buffer)
      store_linvt(S.linvt, A.w.linvt + C * T * T);
      blk_to_lds<F>(S.accd, 0, 1, v4_t<F>{0, 0, 0, 0});
      store_lcc(S.diag, C, a);
      const unsigned long long t3 = stamp(prof);
      lds_t<F>* t = S.diag; S.diag = S.accd; S.accd = t;
      t = S.lprev; S.lprev = S.lcur; S.lcur = t;
      t = S.l2prev; S.l2prev = S.l2cur; S.l2cur = t;
      t = S.linvt_prev; S.linvt_prev = S.linvt; S.linvt = t;
      lds_barrier();
      if (prof) {
        const unsigned long long t4 = stamp(true);
        p_sweep += t1 - t0, p_wait += t2 - t1, p_b += t3 - t2, p_c += t4 - t3, steps += 1;
      }
    } else {
      // phase B: block (0, 0) of L(C+1, C) = acco * L(C,C)^{-T}; wave 1 stores it
      // during the next step
      if (A.K >= 1) blk_to_lds(S.lcur, 0, 0, blk_trsm_lds(S.acco, S.linvt, 0, 0, LP));
      lds_barrier();
      const unsigned long long t3 = stamp(prof);
      // phase C: block (0, 0) of the next diagonal tile, staged in acco's buffer
      v4_t<F> acc = blk_from_lds<F>(S.accd, 0, 0);
      if (A.K >= 1) acc = blk_gemm_lds<F>(S.lcur, S.lcur, 0, 0, acc);
      blk_to_lds<F>(S.acco, 0, 0, acc);
      blk_to_lds<F>(S.acco, 0, 1, v4_t<F>{0, 0, 0, 0});
      lds_t<F>* t = S.diag; S.diag = S.acco; S.acco = t;
      t = S.lprev; S.lprev = S.lcur; S.lcur = t;
      t = S.l2prev; S.l2prev = S.l2cur; S.l2cur = t;
      t = S.linvt_prev; S.linvt_prev = S.linvt; S.linvt = t;
      lds_barrier();
      if (prof) {
        const unsigned long long t4 = stamp(true);
        p_sweep += t1 - t0, p_wait += t2 - t1, p_b += t3 - t2, p_c += t4 - t3, steps += 1;
      }
    }
  }
}

template <typename F>
__device__ __attribute__((noinline)) void spine_waves123(const Args<F>& A_, const SpineLds<F>& S_, lds_i* sync,
                                                         lds_i* s_pub, lds_i* s_fail) {
  const Args<F> A = uniform_step(A_);
  SpineLds<F> S = S_;
  const BandT<F>& a = A.a;
  const int wave = wave_id();
  int early = 0;
  const bool prof = A.w.prof != nullptr;
  unsigned long long p_work = 0, p_wait = 0;
  for (int64_t C = 0; C < A.NB; ++C) {
    const bool next = C + 1 < A.NB;
    const unsigned long long t0 = stamp(prof);
    // phase A
    if constexpr (acc_is_operand<F>()) spine_prepare64(A, C, S, next, sync, s_pub, s_fail, early);
    else spine_prepare32(A, C, S, next, sync, s_pub, s_fail, early);
    const unsigned long long t1 = stamp(prof);
    lds_barrier();
    if (prof) {
      p_work += t1 - t0, p_wait += stamp(true) - t1;
      if (!next && lane_id() == 0) A.w.prof[PROF_W1_WORK + 2 * (wave - 1)] = p_work, A.w.prof[PROF_W1_WAIT + 2 * (wave - 1)] = p_wait;
    }
    if (*s_fail != -1) return;
    if (!next) {
      if (wave == 1) store_lcc(S.diag, C, a);
      return;
    }
    if constexpr (acc_is_operand<F>()) {
      // phase BC: wave w takes block (ci, cj) of the next diagonal tile,
      // (0,0), (1,0), (1,1) for waves 1, 2, 3, and computes row block ci of
      // L(C+1, C) = acco * L(C,C)^{-T}; its accumulators are the operands of
      // that block's last term, so no barrier separates the trsm from it.
      // Waves 1 and 3 stage their row block (for wave 2, which takes row
      // block 0 from there once wave 1 signals, and for the next step) and
      // store it.  The new tile goes to accd's buffer, each wave over the
      // block it read.
      const int ci = wave >= 2, cj = wave == 3;
      v4_t<F> acc = blk_from_lds<F>(S.accd, ci, cj);
      if (A.K >= 1) {
        v4_t<F> oi[2];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) oi[kb] = blk_trsm_lds(S.acco, S.linvt, ci, kb, LP);
        if (wave == 2) {
          // row block 1 in registers, row block 0 from wave 1 through LDS
          if (!lds_wait(&sync[3], (int)C + 1)) {
            if (lane_id() == 0) *s_fail = -2;
          } else {
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
#pragma unroll
              for (int r = 0; r < 4; ++r)
                acc = mfma_xyt(-oi[kb][r], S.lcur[(16 * kb + 4 * r + (lane_id() >> 4)) * LP + (lane_id() & 15)], acc);
          }
        } else {
#pragma unroll
          for (int kb = 0; kb < 2; ++kb) blk_to_lds(S.lcur, ci, kb, oi[kb]);
          if (wave == 1) lds_signal(&sync[3], (int)C + 1);
          // the stores of the row block go out one per matrix-core step of
          // the last term, whose dependent steps would otherwise leave the
          // wave idle while each one runs
          const RunT<F> run0 = acc_run(a, C + 1, C, ci, 0), run1 = acc_run(a, C + 1, C, ci, 1);
#pragma unroll
          for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              acc = mfma_xyt(-oi[kb][r], oi[kb][r], acc);
              const RunT<F>& run = kb ? run1 : run0;
              if (run.in(r)) astore(run.at(r), oi[kb][r]);
            }
        }
      }
      blk_to_lds<F>(S.accd, ci, cj, acc);
      lds_t<F>* t = S.diag; S.diag = S.accd; S.accd = t;
      t = S.lprev; S.lprev = S.lcur; S.lcur = t;
      t = S.l2prev; S.l2prev = S.l2cur; S.l2cur = t;
      t = S.linvt_prev; S.linvt_prev = S.linvt; S.linvt = t;
      lds_barrier();
    } else {
      // phase B: L(C+1, C) = acco * L(C,C)^{-T}, one block per wave, stored now
      if (A.K >= 1) {
        const int bi = wave & 1, bj = wave >> 1;
        const v4_t<F> v = blk_trsm_lds(S.acco, S.linvt, bi, bj, LP);
        blk_to_lds(S.lcur, bi, bj, v);
        ablk_store(a, C + 1, C, bi, bj, v);
      }
      lds_barrier();
      // phase C: blocks (1,0), (1,1) of the next diagonal tile on waves 2, 3,
      // staged in acco's buffer; wave 1 stores L(C,C), which stays in the
      // diagonal tile's buffer until the rotation
      if (wave >= 2) {
        const int bi = 1, bj = (wave == 3);
        v4_t<F> acc = blk_from_lds<F>(S.accd, bi, bj);
        if (A.K >= 1) acc = blk_gemm_lds<F>(S.lcur, S.lcur, bi, bj, acc);
        blk_to_lds<F>(S.acco, bi, bj, acc);
      } else {
        store_lcc(S.diag, C, a);
      }
      lds_t<F>* t = S.diag; S.diag = S.acco; S.acco = t;
      t = S.lprev; S.lprev = S.lcur; S.lcur = t;
      t = S.l2prev; S.l2prev = S.l2cur; S.l2cur = t;
      t = S.linvt_prev; S.linvt_prev = S.linvt; S.linvt = t;
      lds_barrier();
    }
  }
}

template <typename F>
__device__ void spine(const Args<F>& A, lds_t<F>* base, lds_i* s_fail, lds_i* s_pub, lds_i* sync) {
  const int wave = wave_id();
  SpineLds<F> S;
  S.diag = base;
  S.linvt = S.diag + T * LP;
  S.linvt_prev = S.linvt + T * LP;
  S.acco = S.linvt_prev + T * LP;
  S.accd = S.acco + T * LP;
  S.lcur = S.accd + T * LP;
  S.lprev = S.lcur + T * LP;
  S.l2cur = S.lprev + T * LP;
  S.l2prev = S.l2cur + T * LP;
  S.sd = S.l2prev + T * LP;
  if (threadIdx.x == 0) {
    __hip_atomic_store(A.w.spine_cu, cu_ident(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *s_fail = -1;
    *s_pub = 0;
    sync[0] = sync[1] = sync[2] = sync[3] = sync[4] = 0;
  }
  // stage tile (0,0)
  if (wave >= 1) {
    const int bi = (wave >= 2), bj = (wave == 3);
    v4_t<F> v = blk_issue<F>(A, nullptr, 0, 0, bi, bj);
    blk_ident(A.a, 0, 0, bi, bj, v);
    blk_to_lds(S.diag, bi, bj, v);
  } else {
    blk_to_lds(S.diag, 0, 1, v4_t<F>{0, 0, 0, 0});
  }
  lds_barrier();
  if (wave == 0) spine_wave0(A, S, s_fail);
  else spine_waves123(A, S, sync, s_pub, s_fail);
}

// ---------------------------------------------------------------- kernel

// Ticket order: 0 = spine; then per column C the tile O(C+3, C) alone (the
// one the spine takes two steps later, and the head of the chain of tiles
// the helpers hand to each other: a task of its own has half the work per
// term of a pair, so it keeps up sooner), then the pair O(C+4, C), O(C+5, C),
// H(C+4) and P(C+4) (their last terms use the tiles C+3 and C+4), then the
// tiles O(C+6..C+K, C) in pairs (the last one alone when their count is odd),
// except that from K = STRIP_MIN_K on those from O(C+STRIP_D0, C) on go in
// strips of four.
__host__ __device__ __forceinline__ unsigned off_pairs(int K) { return K >= 4 ? (unsigned)(K - 2) / 2u : 0u; }
__host__ __device__ __forceinline__ unsigned tickets_per_column(int K) {
  if (K >= STRIP_MIN_K) return 4u + (STRIP_D0 - 6) / 2 + (unsigned)(K - STRIP_D0 + 4) / 4u;
  return (K >= 3 ? 1u : 0u) + off_pairs(K) + (K >= 4 ? 2u : 0u);
}

// kind 1: tile (R, C); kind 3: tiles (R, C) and (R+1, C); kind 2: H(R); kind 4: P(R);
// kind 5: the strip of tiles (R .. R+3, C).
template <typename F>
__device__ __forceinline__ void decode(const Args<F>& A, unsigned t, int& kind, int64_t& R, int64_t& C) {
  const unsigned per = tickets_per_column(A.K);
  const unsigned u = t - 1;
  C = u / per;
  unsigned k = u % per;
  if (k == 0) {  // K >= 3 whenever there are tickets
    kind = 1;
    R = C + 3;
    return;
  }
  --k;  // from here K >= 4
  if (A.K >= STRIP_MIN_K) {
    if (k == 1) { kind = 2; R = C + 4; return; }
    if (k == 2) { kind = 4; R = C + 4; return; }
    constexpr unsigned mid = (STRIP_D0 - 6) / 2;  // pairs between the first pair and the strips
    if (k >= 3 + mid) { kind = 5; R = C + STRIP_D0 + 4 * (int64_t)(k - 3 - mid); return; }
    R = k == 0 ? C + 4 : C + 6 + 2 * (int64_t)(k - 3);
    kind = (R + 1 < A.NB) ? 3 : 1;  // R + 1 <= C + STRIP_D0 - 1 <= C + K
    return;
  }
  unsigned pair = 0;
  if (k >= 1) {
    --k;
    if (k == 0) { kind = 2; R = C + 4; return; }
    if (k == 1) { kind = 4; R = C + 4; return; }
    pair = k - 1;
  }
  R = C + 4 + 2 * (int64_t)pair;
  kind = (R + 1 <= C + A.K && R + 1 < A.NB) ? 3 : 1;
}

template <typename F>
__global__ void __launch_bounds__(NT, 2) factor2_kernel(Args<F> A) {
  __shared__ F lds[9 * T * LP + T];
  __shared__ int s_ticket, s_ok, s_abort, s_pub, s_sync[5];
  for (;;) {
    if (threadIdx.x == 0) {
      // a helper that shares the spine's CU takes no more tasks: the spine's
      // waves then have the CU's matrix cores to themselves
      const bool beside = A.spare_spine_cu &&
                          __hip_atomic_load(A.w.spine_cu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == cu_ident();
      s_ticket = beside ? -1 : (int)atomicAdd(A.w.queue, 1u);
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
      spine<F>(A, (lds_t<F>*)lds, (lds_i*)&s_ok, (lds_i*)&s_pub, (lds_i*)s_sync);
    } else {
      int kind;
      int64_t R, C;
      decode(A, t, kind, R, C);
      if (R < A.NB) {
        if (kind == 1) task_off<F>(A, R, C, (lds_t<F>*)lds, (lds_i*)&s_ok);
        else if (kind == 3) task_off2<F>(A, R, C, (lds_t<F>*)lds, (lds_i*)&s_ok);
        else if (kind == 5) task_strip<F>(A, R, C, (lds_t<F>*)lds, (lds_i*)&s_ok, (lds_i*)s_sync);
        else if (kind == 2) task_pre(A, R, (lds_i*)&s_ok);
        else task_p(A, R, (lds_i*)&s_ok);
      }
    }
    __syncthreads();
  }
}

__global__ void factor2_init(glb_i* flags, int64_t count, unsigned* queue, glb_i* abort_flag, unsigned long long* ff,
                             unsigned long long* zero, glb_i* spine_cu) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t x = g; x < count; x += (int64_t)gridDim.x * blockDim.x) flags[x] = 0;
  if (g == 0) { *queue = 0; *abort_flag = 0; *ff = 0x7fffffffffffffffULL; *zero = 0; *spine_cu = -1; }
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
  const size_t flags = sizeof(int) * (size_t)(NB * (K + 1) + 2 * NB);
  return 256 + ((flags + 255) & ~(size_t)255) + elem * (size_t)NB * T * T * 4;
}

size_t bandchol_factor2_workspace(int64_t n, int64_t K) { return factor2_workspace(n, K, sizeof(double)); }
size_t bandchol_factor2_workspace_f32(int64_t n, int64_t K) { return factor2_workspace(n, K, sizeof(float)); }

template <typename F>
static hipError_t factor2_launch(int64_t n, int64_t k, F* ab, int64_t ldab, int64_t* d_info, void* ws, int grid_max,
                                 hipStream_t st, unsigned long long* prof = nullptr) {
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
  A.w.spine_cu = (glb_i*)(base + 24);
  A.w.zero = (const glb_t<F>*)(base + 64);
  A.w.prof = prof;
  A.w.tflag = (glb_i*)(base + 256);
  A.w.hflag = A.w.tflag + (size_t)NB * (K + 1);
  A.w.pflag = A.w.hflag + NB;
  const size_t flags = sizeof(int) * (size_t)(NB * (K + 1) + 2 * NB);
  A.w.linvt = (glb_t<F>*)(base + 256 + ((flags + 255) & ~(size_t)255));
  A.w.pre = A.w.linvt + (size_t)NB * T * T;
  A.ntickets = 1 + tickets_per_column(K) * (unsigned)NB;
  const int64_t nflags = (int64_t)NB * (K + 1) + 2 * NB;
  factor2_init<<<(unsigned)((nflags + 255) / 256 > 1024 ? 1024 : (nflags + 255) / 256 + 1), 256, 0, st>>>(
      A.w.tflag, nflags, A.w.queue, A.w.abort_flag, A.w.first_fail, (unsigned long long*)(base + 64), A.w.spine_cu);
  int grid = grid_max;
  if ((unsigned)grid > A.ntickets) grid = (int)A.ntickets;
  A.spare_spine_cu = grid >= 64 ? 1 : 0;  // with few workgroups every helper counts
  factor2_kernel<F><<<grid, NT, 0, st>>>(A);
  factor2_finish<<<1, 1, 0, st>>>(A.w.abort_flag, A.w.first_fail, d_info);
  return hipGetLastError();
}

hipError_t bandchol_factor2_launch(int64_t n, int64_t k, double* ab, int64_t ldab, int64_t* d_info, void* ws,
                                   int grid_max, hipStream_t st) {
  return factor2_launch<double>(n, k, ab, ldab, d_info, ws, grid_max, st);
}

// The FP64 factor with the spine's phase times summed into prof (PROF_SLOTS values).
hipError_t bandchol_factor2_launch_profiled(int64_t n, int64_t k, double* ab, int64_t ldab, int64_t* d_info, void* ws,
                                            int grid_max, unsigned long long* prof, hipStream_t st) {
  return factor2_launch<double>(n, k, ab, ldab, d_info, ws, grid_max, st, prof);
}

hipError_t bandchol_factor2_launch_f32(int64_t n, int64_t k, float* ab, int64_t ldab, int64_t* d_info, void* ws,
                                       int grid_max, hipStream_t st) {
  return factor2_launch<float>(n, k, ab, ldab, d_info, ws, grid_max, st);
}
