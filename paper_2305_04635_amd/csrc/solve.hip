// Band solves with the factor: forward L Y = B, then back L^T X = Y (gfx950, FP64).
//
// Both directions walk the band in blocks of SB = 64 rows (two tiles) and form
// each block from the previous (or next) KS blocks.  One workgroup (the
// spine, whoever takes ticket 0) carries the dependency chain: for block B it
// applies the contributions of the nearest ST blocks itself, then solves with
// the diagonal block.  Helper workgroups take the other tickets and
// pre-accumulate, for each block, the contributions of all blocks further
// away.  A step of the chain costs about the same whatever its width (its
// loads are issued ahead, its arithmetic is short), so blocks of two tiles
// halve the number of steps.
//
// The diagonal block [A 0; C D] (A, C, D tiles) is solved by block
// substitution with precomputed operators, not with the inverse of the whole
// block: forward y1 = A^{-1} t1 and u2 = t2 - (C A^{-1}) t1, then
// y2 = D^{-1} u2; back x2 = D^{-T} t2 and u1 = t1 - (D^{-1} C)^T t2, then
// x1 = A^{-T} u1.  The subtraction comes before the last inverse is applied,
// as in a substitution tile by tile; multiplying by the inverse of the whole
// block would add products of both tile inverses to nearly cancelling terms
// and lose accuracy on ill-conditioned blocks.
//
// Publication without flags: every block of the result and every helper sum is
// written, by relaxed agent-scope atomic stores, into a buffer filled
// beforehand with a signalling NaN.  No arithmetic result is a signalling NaN
// (operations on NaN inputs return quiet ones), so a reader that loads an
// element other than that pattern has the final value: it polls the data
// itself.  The spine never waits for its own stores to drain, and a helper
// sum is ready for the spine one store latency after it is formed.
//
// The spine's operands that do not depend on the chain (its blocks of L, the
// inverse of the diagonal block, the right-hand side and the helper sum) are
// loaded two steps ahead, into two register stages used alternately, so that
// a step costs its arithmetic and two barriers, not memory latencies.
#include <stdint.h>
#include <stdlib.h>

#include "bandchol.h"
#include "common.h"

namespace bandchol_sv {

using namespace bandchol;

typedef double d2 __attribute__((ext_vector_type(2)));
typedef glb_t<d2> glb_d2;

constexpr int SB = 64;               // rows per block
constexpr int NT = 512;              // threads: (i, p) = (tid / 8, tid % 8), row i, columns 8p .. 8p+7
constexpr int QP = 8;                // columns per thread
constexpr int RHS_MAX = 8;           // right-hand sides per launch (thread p completes r = p)
constexpr int ST_MAX = 2;            // most blocks the spine applies itself
constexpr long long SPIN_LIMIT = 1LL << 24;
constexpr long long UNSET = 0x7FF4DEADBEEF0001LL;   // a signalling NaN

struct SolveArgs {
  Band a;
  int NB, KS, nrhs;       // blocks, blocks of bandwidth, right-hand sides
  int64_t NBT;            // NB * SB, the length of a published column
  const glb_d* ops;       // the spine's operands, per block (layout at chunk_len)
  const glb_d* in;        // forward: b; back: the forward result
  int64_t ldin;
  glb_d* pub;             // this direction's result, published (column length NBT)
  glb_d* z;               // helper sums, published: (B * nrhs + r) * SB + i
  glb_d* out;             // back: b, receives the solution; forward: unused
  int64_t ldout;
  unsigned* queue;        // ticket counter
  glb_i* abort_flag;      // 2 = a wait exceeded its bound
  const glb_d* zero;      // QP zeros: masked-off lanes load them, so that every load is unconditional
  glb_d* sink;            // masked-off lanes store here, so that every store is unconditional
};

__device__ __forceinline__ bool unset(double v) { return __double_as_longlong(v) == UNSET; }

// The address to load, hidden from the optimiser: a load whose address is a
// select between a real element and the zero would otherwise be split into a
// branch around a load, and the branch makes the wave wait for loads still in
// flight from earlier steps.  (An empty register constraint, no instruction.)
__device__ __forceinline__ const glb_d* opaque(const glb_d* p) {
  uint64_t u = (uint64_t)p;
  asm("" : "+v"(u));
  return (const glb_d*)u;
}

// A(i, j) of the band or, outside it (j < 0 included), the zero.
__device__ __forceinline__ const glb_d* band_or_zero(const SolveArgs& S, int64_t i, int64_t j) {
  return opaque(j >= 0 && S.a.in_band(i, j) ? S.a.at(i, j) : S.zero);
}

// Polls *p until it is published.  False when the wait gives up: after
// SPIN_LIMIT polls (then the abort flag is raised) or once another wait has.
__device__ __forceinline__ bool await_value(const glb_d* p, glb_i* abort_flag, double& v) {
  for (long long spins = 0;; ++spins) {
    v = aload<double>(p);
    if (!unset(v)) return true;
    if ((spins & 31) == 31) {
      if (aload<int>(abort_flag)) return false;
      if (spins > SPIN_LIMIT) {
        astore<int>(abort_flag, 2);
        return false;
      }
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// v from another lane of the same row of 16, by a DPP control (no LDS trip).
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  int2 h = __builtin_bit_cast(int2, v);
  h.x = __builtin_amdgcn_update_dpp(0, h.x, CTRL, 0xF, 0xF, false);
  h.y = __builtin_amdgcn_update_dpp(0, h.y, CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, h);
}

// Sum over the 8 lanes 8a .. 8a+7, in every one of them: swap neighbours
// (quad_perm 1,0,3,2), swap pairs (quad_perm 2,3,0,1), then add the mirror
// lane of the other quad (row_half_mirror, lane l <-> 7 - l).  The wave must be
// fully active.
__device__ __forceinline__ double red8(double s) {
  s += dpp<0xB1>(s);
  s += dpp<0x4E>(s);
  s += dpp<0x141>(s);
  return s;
}

// sum_q x[q] y[q] over 8 terms, as two chains of 4
__device__ __forceinline__ double dot8(const double (&x)[QP], const lds_d* y) {
  double a0 = x[0] * y[0], a1 = x[4] * y[4];
  a0 = fma(x[1], y[1], a0);
  a1 = fma(x[5], y[5], a1);
  a0 = fma(x[2], y[2], a0);
  a1 = fma(x[6], y[6], a1);
  a0 = fma(x[3], y[3], a0);
  a1 = fma(x[7], y[7], a1);
  return a0 + a1;
}

// sum_q x[o + q] y[q] over 4 terms
__device__ __forceinline__ double dot4(const double (&x)[QP], int o, const lds_d* y) {
  return fma(x[o + 3], y[3], fma(x[o + 2], y[2], fma(x[o + 1], y[1], x[o] * y[0])));
}

// Operands of one spine step, loaded ahead.  Thread (i, p) holds, for the
// step's block B and its neighbours N = B -+ d (d = 1 .. ST):
//   forward: lf[d-1][q] = L(B SB + i, N SB + 8p + q)
//   back:    lf[d-1][q] = L(N SB + 8p + q, B SB + i)
// (zero outside the band and past either end); in df, row i, columns
// 4p .. 4p+3 of the two operators of the diagonal block (see block_operators):
// df[0..3] of P (64 x 32), df[4..7] of R (32 x 32, zero in the rows that P
// completes); and the right-hand side and helper sum of row i for r = p.
template <int ST>
struct Stage {
  double lf[ST][QP];
  double df[QP];
  double bv, zv;
};

// The operand buffer holds, per block B, the ST blocks of L and the inverse of
// the diagonal block that the spine's step on B reads, zero-padded, in the
// order of the threads: block t, elements q = 2h and 2h+1 of thread tid at
// ((t * 4 + h) * NT + tid) * 2.  Every load of a step is then a coalesced
// 16-byte load at a fixed offset from a uniform base.
__host__ __device__ constexpr int64_t chunk_len(int st) { return (int64_t)(st + 1) * SB * SB; }

__device__ __forceinline__ int64_t slot(int t, int h, int tid) { return ((int64_t)(t * 4 + h) * NT + tid) * 2; }

template <bool FWD>
__device__ __forceinline__ int spine_block(const SolveArgs& S, int m) { return FWD ? m : S.NB - 1 - m; }

template <int ST, bool FWD>
__device__ __forceinline__ bool spine_has_z(const SolveArgs& S, int B) {
  return S.KS > ST && (FWD ? B >= ST + 1 : B <= S.NB - ST - 2);
}

template <int ST, bool FWD>
__device__ __forceinline__ void load_l(const SolveArgs& S, int B, int i, int p, Stage<ST>& s) {
  const int tid = threadIdx.x;
  const glb_d* c = S.ops + (int64_t)B * chunk_len(ST);
#pragma unroll
  for (int t = 0; t < ST; ++t)
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const d2 v = *(const glb_d2*)(c + slot(t, h, tid));
      s.lf[t][2 * h] = v.x;
      s.lf[t][2 * h + 1] = v.y;
    }
  // forward reads b (rows < n); back reads the forward result (all NBT rows)
  const int64_t row = (int64_t)B * SB + i;
  const bool on = p < S.nrhs && (FWD ? row < S.a.n : true);
  s.bv = *opaque(on ? S.in + p * S.ldin + row : S.zero);
}

template <int ST, bool FWD>
__device__ __forceinline__ void load_d(const SolveArgs& S, int B, int i, int p, Stage<ST>& s) {
  const int tid = threadIdx.x;
  const glb_d* c = S.ops + (int64_t)B * chunk_len(ST);
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const d2 v = *(const glb_d2*)(c + slot(ST, h, tid));
    s.df[2 * h] = v.x;
    s.df[2 * h + 1] = v.y;
  }
  const bool hz = spine_has_z<ST, FWD>(S, B);
  s.zv = aload<double>(opaque((hz && p < S.nrhs) ? S.z + ((int64_t)B * S.nrhs + p) * SB + i : S.zero));
}

// Ring slot of block N (N may lie up to ST before the first block).
template <int ST>
__device__ __forceinline__ int ring_slot(int N) { return (N + ST + 1) % (ST + 1); }

// Stores a result of row `row` (rhs p) where this lane has one (on), else
// into the sink: the publication buffer (and, back, the solution).  With
// helpers (SH) the publication must be coherent across the chip (an
// agent-scope store); without, only later launches read it, and a plain store
// is enough (it leaves the L2 at the end of the kernel) and cheaper: the
// spine's step at k = 100 took 17 % longer with the agent-scope stores.
template <bool FWD, bool SH>
__device__ __forceinline__ void publish(const SolveArgs& S, bool on, int64_t row, int p, double v) {
  glb_d* dst = (glb_d*)opaque(on ? S.pub + p * S.NBT + row : S.sink);
  if (SH) astore<double>(dst, v);
  else *dst = v;
  if (!FWD) *(glb_d*)opaque(on && p < S.nrhs && row < S.a.n ? S.out + p * S.ldout + row : S.sink) = v;
}

// One spine step on block B = spine_block(m), with the stage loaded for it;
// refills the stage for step m + 2.  False if a wait gave up.
//
// The stage's registers are reloaded while the step's results are still in
// flight.  Every value of the stage is therefore used once on every path
// through the step (not only in the lanes that need it), and every load and
// store is issued on every path: otherwise the compiler cannot tell which
// loads are still pending and waits for all of them before the reload.
template <int ST, bool FWD, bool SH>
__device__ __forceinline__ bool spine_step(const SolveArgs& S, int m, Stage<ST>& s, lds_d* ring, lds_d* tl,
                                           lds_i* s_fail) {
  const int tid = threadIdx.x, i = tid >> 3, p = tid & 7;
  const int B = spine_block<FWD>(S, m);
  const bool hz = spine_has_z<ST, FWD>(S, B);
  // Consumed here on every path (see above); loaded two steps ago.
  double bv = s.bv, zv = s.zv;
  asm volatile("" : "+v"(bv), "+v"(zv));
  // t = b - z - sum_d L(B,N) y_N  (back: L(N,B)^T x_N), one partial sum per
  // neighbour.  Neighbours past either end have zero blocks and read ring
  // slots that were never written (zero).  The loops over the right-hand
  // sides hold LDS reads only (counted apart from the global loads) and are
  // not unrolled, which keeps the registers for the two stages; their first
  // pass is always taken (nrhs >= 1).
  double mine = 0.0;
  int r = 0;
#pragma nounroll
  do {
    double part[ST];
#pragma unroll
    for (int d = 1; d <= ST; ++d) {
      const int N = FWD ? B - d : B + d;
      part[d - 1] = dot8(s.lf[d - 1], ring + ring_slot<ST>(N) * (SB * RHS_MAX) + r * SB + QP * p);
    }
#pragma unroll
    for (int w = 1; w < ST; w *= 2)
#pragma unroll
      for (int d = 0; d + w < ST; d += 2 * w) part[d] += part[d + w];
    const double acc = red8(part[0]);
    mine = p == r ? acc : mine;
  } while (++r < S.nrhs);
  double zz = hz ? zv : 0.0;
  if (hz && p < S.nrhs && unset(zz) && !await_value(S.z + ((int64_t)B * S.nrhs + p) * SB + i, S.abort_flag, zz)) {
    *s_fail = 1;
    zz = 0.0;
  }
  const double tmine = (bv - zz) - mine;
  if (p < S.nrhs) tl[p * SB + i] = tmine;
  // operands of step m + 2 (past the end: the last block again, unused)
  const int b2 = spine_block<FWD>(S, m + 2 < S.NB ? m + 2 : S.NB - 1);
  load_l<ST, FWD>(S, b2, i, p, s);
  __syncthreads();
  // Diagonal block, first half: the rows P completes (forward 0..31, back
  // 32..63) take v = P t_h, the others u = t - v, where t_h is the half of t
  // solved first (forward rows 0..31, back 32..63).
  const int h0 = FWD ? 0 : T;            // first row of t_h
  const bool direct = FWD ? i < T : i >= T;
  mine = 0.0;
  r = 0;
#pragma nounroll
  do {
    const double acc = red8(dot4(s.df, 0, tl + r * SB + h0 + 4 * p));
    mine = p == r ? acc : mine;
  } while (++r < S.nrhs);
  const int64_t row = (int64_t)B * SB + i;
  lds_d* yslot = ring + ring_slot<ST>(B) * (SB * RHS_MAX);
  if (p < S.nrhs) {
    if (direct) yslot[p * SB + i] = mine;
    else tl[p * SB + i] = tmine - mine;
  }
  // The stores are made by every lane (the publication buffers have RHS_MAX
  // columns; masked-off lanes write the sink), for the reason given above.
  publish<FWD, SH>(S, direct, row, p, mine);
  __syncthreads();
  // Second half: the other rows take R u.
  mine = 0.0;
  r = 0;
#pragma nounroll
  do {
    const double acc = red8(dot4(s.df, 4, tl + r * SB + (T - h0) + 4 * p));
    mine = p == r ? acc : mine;
  } while (++r < S.nrhs);
  if (p < S.nrhs && !direct) yslot[p * SB + i] = mine;
  publish<FWD, SH>(S, !direct, row, p, mine);
  load_d<ST, FWD>(S, b2, i, p, s);
  __syncthreads();
  return *s_fail == 0;
}

// Inlined into the kernel: a call here costs more than the few registers the
// kernel then spills (measured both ways).
template <int ST, bool FWD, bool SH>
__device__ __forceinline__ void spine(const SolveArgs& S, lds_d* ring, lds_d* tl, lds_i* s_fail) {
  const int tid = threadIdx.x, i = tid >> 3, p = tid & 7;
  for (int e = tid; e < (ST + 1) * SB * RHS_MAX; e += NT) ring[e] = 0.0;
  Stage<ST> s0, s1;
  const int b1 = spine_block<FWD>(S, S.NB > 1 ? 1 : 0);
  load_l<ST, FWD>(S, spine_block<FWD>(S, 0), i, p, s0);
  load_d<ST, FWD>(S, spine_block<FWD>(S, 0), i, p, s0);
  load_l<ST, FWD>(S, b1, i, p, s1);
  load_d<ST, FWD>(S, b1, i, p, s1);
  __syncthreads();
  // Steps in pairs, both always taken, so that each stage is refilled on every
  // path through the loop body (a stage that might keep its old value would
  // be copied at the loop's end, and the copy waits for the loads).
  int m = 0;
  for (; m + 1 < S.NB; m += 2) {
    if (!spine_step<ST, FWD, SH>(S, m, s0, ring, tl, s_fail)) return;
    if (!spine_step<ST, FWD, SH>(S, m + 1, s1, ring, tl, s_fail)) return;
  }
  if (m < S.NB) spine_step<ST, FWD, SH>(S, m, s0, ring, tl, s_fail);
}

// Helper for block B: z_B = sum over the far neighbours N of L(B,N) y_N
// (forward, N = B-KS .. B-ST-1) or L(N,B)^T x_N (back, N = B+KS .. B+ST+1),
// taken in the order they are published, G blocks and RH right-hand sides per
// round of loads.  All right-hand sides of a block go through the same round
// (RH = RHS_MAX, L loaded once per block), or with one right-hand side G
// blocks do (RH = 1): either way the sums are complete one round trip after the
// newest block appears.  Thread (i, p): row (column) i of B, rows 8p .. 8p+7
// of each N.
template <int ST, bool FWD, int G, int RH>
__device__ __forceinline__ bool helper(const SolveArgs& S, int B, lds_i* s_flag) {
  const int tid = threadIdx.x, i = tid >> 3, p = tid & 7;
  const int nfar = FWD ? (B - ST - 1) - (B - S.KS > 0 ? B - S.KS : 0) + 1
                       : (B + S.KS < S.NB - 1 ? B + S.KS : S.NB - 1) - (B + ST + 1) + 1;
  const int N0 = FWD ? (B - S.KS > 0 ? B - S.KS : 0) : (B + S.KS < S.NB - 1 ? B + S.KS : S.NB - 1);
  const int dir = FWD ? 1 : -1;
  double acc[RH];
#pragma unroll
  for (int r = 0; r < RH; ++r) acc[r] = 0.0;
  for (int g0 = 0; g0 < nfar; g0 += G) {
    double lf[G][QP], yv[G][RH][QP];
    bool miss = false;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const bool on = g0 + g < nfar;
      const int N = N0 + dir * (g0 + g);
#pragma unroll
      for (int q = 0; q < QP; ++q) {
        const int64_t gi = FWD ? (int64_t)B * SB + i : (int64_t)N * SB + QP * p + q;
        const int64_t gj = FWD ? (int64_t)N * SB + QP * p + q : (int64_t)B * SB + i;
        lf[g][q] = *band_or_zero(S, on ? gi : S.a.n, gj);
      }
      const glb_d* yb = S.pub + (int64_t)N * SB + QP * p;
#pragma unroll
      for (int r = 0; r < RH; ++r) {
        const glb_d* yr = opaque(on && r < S.nrhs ? yb + r * S.NBT : S.zero);   // QP zeros there
#pragma unroll
        for (int q = 0; q < QP; ++q) {
          yv[g][r][q] = aload<double>(yr + q);
          miss |= unset(yv[g][r][q]);
        }
      }
    }
    if (__syncthreads_or(miss)) {
      // Not all published yet: thread 0 waits for the last element of the
      // newest block's last right-hand side (one poller per workgroup), then
      // every missing element is awaited on its own.
      const int gl = (nfar - g0 < G ? nfar - g0 : G) - 1;
      const int Nl = N0 + dir * (g0 + gl);
      if (tid == 0) {
        double v;
        *s_flag = await_value(S.pub + (S.nrhs - 1) * S.NBT + (int64_t)Nl * SB + SB - 1, S.abort_flag, v) ? 0 : 1;
      }
      __syncthreads();
      if (*s_flag) return false;
      bool ok = true;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const glb_d* yb = S.pub + (int64_t)(N0 + dir * (g0 + g)) * SB + QP * p;
#pragma unroll
        for (int r = 0; r < RH; ++r)
#pragma unroll
          for (int q = 0; q < QP; ++q)
            if (ok && unset(yv[g][r][q])) ok = await_value(yb + r * S.NBT + q, S.abort_flag, yv[g][r][q]);
      }
      if (__syncthreads_or(!ok)) return false;
    }
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int r = 0; r < RH; ++r)
#pragma unroll
        for (int q = 0; q < QP; ++q) acc[r] = fma(lf[g][q], yv[g][r][q], acc[r]);
  }
#pragma unroll
  for (int r = 0; r < RH; ++r) {
    const double s = red8(acc[r]);
    if (r < S.nrhs && p == r) astore<double>(S.z + ((int64_t)B * S.nrhs + r) * SB + i, s);
  }
  return true;
}

// ---------------------------------------------------------------- kernels

// HV: 0 = no helpers; else the helpers are sized for HV right-hand sides (1,
// 2, 4 or 8, the pass's count rounded up) and read the spine's results while
// the pass runs.  One helper variant per kernel: compiled together, the
// widest set every kernel's register budget.
template <int ST, bool FWD, int HV>
__global__ void __launch_bounds__(NT) solve_kernel(SolveArgs S) {
  __shared__ double ring[(ST + 1) * SB * RHS_MAX];
  __shared__ double tl[SB * RHS_MAX];
  __shared__ int s_ticket, s_flag;
  const int nhelp = S.KS > ST ? S.NB - ST - 1 : 0;
  if (threadIdx.x == 0) s_flag = 0;
  for (;;) {
    if (threadIdx.x == 0) s_ticket = (int)atomicAdd(S.queue, 1u);
    __syncthreads();
    const int t = s_ticket;
    __syncthreads();
    if (t > nhelp) break;
    if (t == 0) {
      spine<ST, FWD, (HV > 0)>(S, (lds_d*)ring, (lds_d*)tl, (lds_i*)&s_flag);
    } else {
      if constexpr (HV > 0) {
        // forward: B = ST+1 .. NB-1; back: B = NB-ST-2 .. 0
        const int B = FWD ? ST + t : S.NB - ST - 1 - t;
        // helpers sized to the pass's right-hand sides (the missing ones would read zeros)
        if (!helper<ST, FWD, (HV <= 2 ? 2 : 1), HV>(S, B, (lds_i*)&s_flag)) break;
      }
    }
    if (s_flag) break;
  }
}

// Fills the first len elements of the 4 publication buffers (stride apart)
// with the unset pattern, zeroes the counters and sets the QP zeros.
__global__ void solve_fill_kernel(glb_d* p, int64_t len, int64_t stride, unsigned* queues, glb_i* abort_flag,
                                  glb_d* zero, int abort_preset) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t x = g; x < 4 * len; x += (int64_t)gridDim.x * blockDim.x)
    p[(x / len) * stride + x % len] = __longlong_as_double(UNSET);
  if (g < QP) zero[g] = 0.0;
  if (g == 0) {
    queues[0] = 0;
    queues[1] = 0;
    *abort_flag = abort_preset;
  }
}

// After a forward + back pair: a wait that gave up (abort flag raised) makes
// the call's status BANDCHOL_EHANG.  The status is only ever set here, never
// cleared: the caller clears it once per call.
__global__ void solve_status_kernel(const glb_i* abort_flag, int64_t* status) {
  if (*abort_flag) *status = BANDCHOL_EHANG;
}

// Per tile C, L(C,C)^{-T} (row-major): lanes 0..T-1 hold the rows of L(C,C),
// lanes T..2T-1 the identity rows, solved against L(C,C) column by column.
// Tiles past the last row come out as the identity.
__global__ void __launch_bounds__(64) tri_inv_kernel(Band a, glb_d* dinvt) {
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

// The operators of the diagonal block B = [A 0; C D] (tiles 2B and 2B+1),
// into LDS with pitch LP: A^{-1} (sa), D^{-1} (sd) from tri_inv_kernel
// (A^{-1}(r, c) = dinvt[c T + r]), and in sc C A^{-1} (forward) or D^{-1} C
// (back).
template <bool FWD>
__device__ __forceinline__ void block_operators(const Band& a, int B, const glb_d* dinvt, lds_d* sa, lds_d* sd,
                                                lds_d* sc) {
  const int tid = threadIdx.x;
  const glb_d* da = dinvt + (int64_t)(2 * B) * T * T;
  const glb_d* dd = da + T * T;
  const int64_t r0 = (int64_t)B * SB;
  for (int e = tid; e < T * T; e += NT) {
    const int r = e % T, c = e / T;
    sa[r * LP + c] = da[c * T + r];
    sd[r * LP + c] = dd[c * T + r];
    sc[r * LP + c] = a.ld(r0 + T + r, r0 + c);
  }
  __syncthreads();
  // two elements per thread, in row r (both inverses lower triangular)
  const int r = tid >> 4, c0 = (tid & 15) * 2;
  double m[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int c = c0 + u;
    double v = 0.0;
    if (FWD)
      for (int k = c; k < T; ++k) v = fma(sc[r * LP + k], sa[k * LP + c], v);
    else
      for (int k = 0; k <= r; ++k) v = fma(sd[r * LP + k], sc[k * LP + c], v);
    m[u] = v;
  }
  __syncthreads();
  sc[r * LP + c0] = m[0];
  sc[r * LP + c0 + 1] = m[1];
  __syncthreads();
}

// Writes the operand buffer of one direction (layout at chunk_len): per
// block B, the ST blocks of L next to it (zero outside the band and past
// either end), then for each thread (i, p), columns 4p .. 4p+3 of row i of
// the diagonal block's operators P and R:
//   forward  P = [A^{-1}; C A^{-1}],   R = [0; D^{-1}]
//   back     P = [(D^{-1} C)^T; D^{-T}], R = [A^{-T}; 0]
template <int ST, bool FWD>
__global__ void __launch_bounds__(NT) prep_kernel(Band a, int NB, const glb_d* dinvt, glb_d* ops) {
  __shared__ double sa[T * LP], sd[T * LP], sc[T * LP];
  const int B = blockIdx.x, tid = threadIdx.x, i = tid >> 3, p = tid & 7;
  block_operators<FWD>(a, B, dinvt, (lds_d*)sa, (lds_d*)sd, (lds_d*)sc);
  glb_d* c = ops + (int64_t)B * chunk_len(ST);
#pragma unroll
  for (int t = 0; t <= ST; ++t) {
    double v[QP];
#pragma unroll
    for (int q = 0; q < QP; ++q) {
      if (t < ST) {
        const int N = FWD ? B - (t + 1) : B + (t + 1);
        const int64_t gi = FWD ? (int64_t)B * SB + i : (int64_t)N * SB + QP * p + q;
        const int64_t gj = FWD ? (int64_t)N * SB + QP * p + q : (int64_t)B * SB + i;
        v[q] = (N >= 0 && N < NB && a.in_band(gi, gj)) ? *a.at(gi, gj) : 0.0;
      } else {
        const int cc = 4 * p + (q & 3);
        const bool lo = i < T;
        const int ih = lo ? i : i - T;
        if (q < 4) {
          if (FWD) v[q] = lo ? sa[ih * LP + cc] : sc[ih * LP + cc];
          else v[q] = lo ? sc[cc * LP + ih] : sd[cc * LP + ih];
        } else {
          if (FWD) v[q] = lo ? 0.0 : sd[ih * LP + cc];
          else v[q] = lo ? sa[cc * LP + ih] : 0.0;
        }
      }
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) *(glb_d2*)(c + slot(t, h, tid)) = d2{v[2 * h], v[2 * h + 1]};
  }
}

template <int ST, int HV>
void launch_pair(const Band& a, const glb_d* dinvt, glb_d* ops, const SolveArgs& f, const SolveArgs& b, int grid,
                 hipStream_t st) {
  prep_kernel<ST, true><<<f.NB, NT, 0, st>>>(a, f.NB, dinvt, ops);
  solve_kernel<ST, true, HV><<<grid, NT, 0, st>>>(f);
  prep_kernel<ST, false><<<f.NB, NT, 0, st>>>(a, f.NB, dinvt, ops);
  solve_kernel<ST, false, HV><<<grid, NT, 0, st>>>(b);
}

// Blocks of the band the spine applies itself: all of them up to ST_MAX,
// rounded up to an instantiated width; beyond, ST_MAX and helpers.
inline int spine_width(int KS) { return KS <= 1 ? 1 : ST_MAX; }

inline int blocks_of_band(int64_t n, int64_t k) {
  const int NB = (int)((n + SB - 1) / SB);
  int KS = (int)((k + SB - 1) / SB);
  if (KS > NB - 1) KS = NB - 1 > 0 ? NB - 1 : 0;
  return KS;
}

}  // namespace bandchol_sv

// Host side, called by the C-ABI (same library).  Workspace layout, in bytes
// from `ws`: [0,256) two ticket counters, the abort flag, (at 64) QP zeros
// and (at 128) the sink; then the publication area, 4 * RHS_MAX * NBT
// doubles (forward result, back result, forward and back helper sums, RHS_MAX
// * NBT each, of which a pass of nrhs right-hand sides uses the first
// nrhs * NBT); then the inverted tiles, 2 * NB * T * T doubles; then the
// operand buffer, NB * chunk_len(ST) doubles.
size_t bandchol_solve_workspace(int64_t n, int64_t k) {
  using namespace bandchol_sv;
  const int64_t NB = (n + SB - 1) / SB, NBT = NB * SB;
  const int ST = spine_width(blocks_of_band(n, k));
  return 256 + sizeof(double) * ((size_t)4 * RHS_MAX * NBT + (size_t)2 * NB * T * T + (size_t)NB * chunk_len(ST));
}

hipError_t bandchol_solve_launch(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, double* b,
                                 int64_t ldb, void* ws, int num_cus, int64_t* d_status, hipStream_t st) {
  using namespace bandchol_sv;
  const int NB = (int)((n + SB - 1) / SB);
  const int64_t NBT = (int64_t)NB * SB;
  const int KS = blocks_of_band(n, k);
  const int ST = spine_width(KS);
  char* base = (char*)ws;
  unsigned* queues = (unsigned*)base;
  glb_i* abort_flag = (glb_i*)(base + 8);
  glb_d* zero = (glb_d*)(base + 64);
  glb_d* sink = (glb_d*)(base + 128);
  glb_d* pubarea = (glb_d*)(base + 256);
  glb_d* dinvt = pubarea + (size_t)4 * RHS_MAX * NBT;
  glb_d* ops = dinvt + (size_t)2 * NB * T * T;
  const Band a{(glb_d*)const_cast<double*>(ab), n, k, ldab};
  tri_inv_kernel<<<2 * NB, 64, 0, st>>>(a, dinvt);
  const int nhelp = KS > ST ? NB - ST - 1 : 0;
  // one workgroup per CU at most: the spine keeps a CU to itself
  const int grid = 1 + nhelp < num_cus ? 1 + nhelp : num_cus;
  // Testing aid: BANDCHOL_TEST_SOLVE_ABORT=1 starts every pass with the abort
  // flag raised, as if a wait had given up, so that the status path can be
  // checked without making any wait actually time out (waits that find their
  // data published never look at the flag; the others return at once).
  const char* preset_env = getenv("BANDCHOL_TEST_SOLVE_ABORT");
  const int preset = (preset_env && preset_env[0] == '1') ? 2 : 0;
  for (int64_t r0 = 0; r0 < nrhs; r0 += RHS_MAX) {
    const int nr = (int)(nrhs - r0 < RHS_MAX ? nrhs - r0 : RHS_MAX);
    const size_t stride = (size_t)RHS_MAX * NBT;
    glb_d* y = pubarea;
    glb_d* x = y + stride;
    glb_d* zf = x + stride;
    glb_d* zb = zf + stride;
    glb_d* bb = (glb_d*)(b + r0 * ldb);
    const SolveArgs F{a, NB, KS, nr, NBT, ops, bb, ldb, y, zf, nullptr, 0, queues, abort_flag, zero, sink};
    const SolveArgs Bk{a, NB, KS, nr, NBT, ops, y, NBT, x, zb, bb, ldb, queues + 1, abort_flag, zero, sink};
    const int64_t len = (int64_t)nr * NBT;
    const int64_t fg = (4 * len + 255) / 256;
    solve_fill_kernel<<<(unsigned)(fg < 2048 ? fg : 2048), 256, 0, st>>>(pubarea, len, (int64_t)stride, queues,
                                                                         abort_flag, zero, preset);
    if (ST == 1) launch_pair<1, 0>(a, dinvt, ops, F, Bk, grid, st);  // KS <= 1: never helpers
    else if (nhelp == 0) launch_pair<ST_MAX, 0>(a, dinvt, ops, F, Bk, grid, st);
    else if (nr == 1) launch_pair<ST_MAX, 1>(a, dinvt, ops, F, Bk, grid, st);
    else if (nr == 2) launch_pair<ST_MAX, 2>(a, dinvt, ops, F, Bk, grid, st);
    else if (nr <= 4) launch_pair<ST_MAX, 4>(a, dinvt, ops, F, Bk, grid, st);
    else launch_pair<ST_MAX, RHS_MAX>(a, dinvt, ops, F, Bk, grid, st);
    if (d_status) solve_status_kernel<<<1, 1, 0, st>>>(abort_flag, d_status);
  }
  return hipGetLastError();
}
