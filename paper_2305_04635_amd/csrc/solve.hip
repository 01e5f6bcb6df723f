// Band solves with the factor: forward L Y = B, then back L^T X = Y (gfx950, FP64).
//
// Both directions walk the band in T-row blocks and form each block from the
// previous (or next) KS blocks.  One workgroup (the spine, whoever takes ticket
// 0) carries the dependency chain: for block B it applies the contributions of
// the nearest ST blocks itself, then multiplies by the inverse of the diagonal
// tile.  Helper workgroups take the other tickets and pre-accumulate, for each
// block, the contributions of all blocks further away.
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
// inverse of the diagonal tile, the right-hand side and the helper sum) are
// loaded two steps ahead, into two register stages used alternately, so that
// a step costs its arithmetic and two barriers, not memory latencies.
#include <stdint.h>

#include "common.h"

namespace bandchol_solve {

using namespace bandchol;

typedef double d2 __attribute__((ext_vector_type(2)));
typedef glb_t<d2> glb_d2;

constexpr int NT = 256;
constexpr int RHS_MAX = 8;           // right-hand sides per launch (thread p completes r = p)
constexpr int G = 4;                 // blocks a helper loads at once
constexpr int HR = 2;                // right-hand sides per helper pass
constexpr int ST_MAX = 8;            // most blocks the spine applies itself
constexpr long long SPIN_LIMIT = 1LL << 24;
constexpr long long UNSET = 0x7FF4DEADBEEF0001LL;   // a signalling NaN

struct SolveArgs {
  Band a;
  int NB, KS, nrhs;
  int64_t NBT;            // NB * T, the length of a published column
  const glb_d* ops;       // the spine's operands, per block (layout below)
  const glb_d* in;        // forward: b; back: the forward result
  int64_t ldin;
  glb_d* pub;             // this direction's result, published (column length NBT)
  glb_d* z;               // helper sums, published: (B * nrhs + r) * T + i
  glb_d* out;             // back: b, receives the solution; forward: unused
  int64_t ldout;
  unsigned* queue;        // ticket counter
  glb_i* abort_flag;      // 2 = a wait exceeded its bound
  const glb_d* zero;      // a zero: masked-off lanes load it, so that every load is unconditional
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

// Operands of one spine step, loaded ahead.  Thread (i, p) = (tid / 8, tid % 8)
// holds, for the step's block B and its neighbours N = B -+ d (d = 1 .. ST):
//   forward: lf[d-1][q] = L(B T + i, N T + 4p + q), df[q] = L(B,B)^{-1}(i, 4p + q)
//   back:    lf[d-1][q] = L(N T + 4p + q, B T + i), df[q] = L(B,B)^{-1}(4p + q, i)
// (zero outside the band and past either end), and the right-hand side and
// helper sum of row i for r = p.
template <int ST>
struct Stage {
  double lf[ST][4];
  double df[4];
  double bv, zv;
};

// The operand buffer holds, per block B, the ST tiles of L and the inverse of
// the diagonal tile that the spine's step on B reads, zero-padded, in the
// order of the threads: tile t, elements q = 2h and 2h+1 of thread tid at
// ((t * 2 + h) * NT + tid) * 2.  Every load of a step is then a coalesced
// 16-byte load at a fixed offset from a uniform base.
__host__ __device__ constexpr int64_t chunk_len(int st) { return (int64_t)(st + 1) * T * T; }

__device__ __forceinline__ int64_t slot(int t, int h, int tid) { return ((int64_t)(t * 2 + h) * NT + tid) * 2; }

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
  for (int t = 0; t < ST; ++t) {
    const d2 lo = *(const glb_d2*)(c + slot(t, 0, tid));
    const d2 hi = *(const glb_d2*)(c + slot(t, 1, tid));
    s.lf[t][0] = lo.x;
    s.lf[t][1] = lo.y;
    s.lf[t][2] = hi.x;
    s.lf[t][3] = hi.y;
  }
  // forward reads b (rows < n); back reads the forward result (all NBT rows)
  const int64_t row = (int64_t)B * T + i;
  const bool on = p < S.nrhs && (FWD ? row < S.a.n : true);
  s.bv = *opaque(on ? S.in + p * S.ldin + row : S.zero);
}

template <int ST, bool FWD>
__device__ __forceinline__ void load_d(const SolveArgs& S, int B, int i, int p, Stage<ST>& s) {
  const int tid = threadIdx.x;
  const glb_d* c = S.ops + (int64_t)B * chunk_len(ST);
  const d2 lo = *(const glb_d2*)(c + slot(ST, 0, tid));
  const d2 hi = *(const glb_d2*)(c + slot(ST, 1, tid));
  s.df[0] = lo.x;
  s.df[1] = lo.y;
  s.df[2] = hi.x;
  s.df[3] = hi.y;
  const bool hz = spine_has_z<ST, FWD>(S, B);
  s.zv = aload<double>(opaque((hz && p < S.nrhs) ? S.z + ((int64_t)B * S.nrhs + p) * T + i : S.zero));
}

// Ring slot of block N (N may lie up to ST before the first block).
template <int ST>
__device__ __forceinline__ int ring_slot(int N) { return (N + ST + 1) % (ST + 1); }

// One spine step on block B = spine_block(m), with the stage loaded for it;
// refills the stage for step m + 2.  False if a wait gave up.
//
// The stage's registers are reloaded while the step's results are still in
// flight.  Every value of the stage is therefore used once on every path
// through the step (not only in the lanes that need it): a register whose
// load might still be pending on some path would make the wave wait for that
// load, and all later ones, before the reload.
template <int ST, bool FWD>
__device__ __forceinline__ bool spine_step(const SolveArgs& S, int m, Stage<ST>& s, lds_d* ring, lds_d* tl,
                                           lds_i* s_fail) {
  const int tid = threadIdx.x, i = tid >> 3, p = tid & 7;
  const int B = spine_block<FWD>(S, m);
  const bool hz = spine_has_z<ST, FWD>(S, B);
  // Consumed here on every path (see above); loaded two steps ago.
  double bv = s.bv, zv = s.zv;
  asm volatile("" : "+v"(bv), "+v"(zv));
  // t = b - z - sum_d L(B,N) y_N  (back: L(N,B)^T x_N), one partial sum per
  // neighbour so that the dependent chains are 4 long.  Neighbours past
  // either end have zero tiles and read ring slots that were never written
  // (zero).  The loops over the right-hand sides are unrolled to their bound,
  // the first one taken always (nrhs >= 1).
  double mine = 0.0;
#pragma unroll
  for (int r = 0; r < RHS_MAX; ++r) {
    if (r > 0 && r >= S.nrhs) break;
    double part[ST];
#pragma unroll
    for (int d = 1; d <= ST; ++d) {
      const int N = FWD ? B - d : B + d;
      const lds_d* yp = ring + ring_slot<ST>(N) * (T * RHS_MAX) + r * T + 4 * p;
      double a0 = s.lf[d - 1][0] * yp[0];
      a0 = fma(s.lf[d - 1][1], yp[1], a0);
      a0 = fma(s.lf[d - 1][2], yp[2], a0);
      part[d - 1] = fma(s.lf[d - 1][3], yp[3], a0);
    }
#pragma unroll
    for (int w = 1; w < ST; w *= 2)
#pragma unroll
      for (int d = 0; d + w < ST; d += 2 * w) part[d] += part[d + w];
    const double acc = red8(part[0]);
    mine = p == r ? acc : mine;
  }
  double zz = hz ? zv : 0.0;
  if (hz && p < S.nrhs && unset(zz) && !await_value(S.z + ((int64_t)B * S.nrhs + p) * T + i, S.abort_flag, zz)) {
    *s_fail = 1;
    zz = 0.0;
  }
  if (p < S.nrhs) tl[p * T + i] = (bv - zz) - mine;
  // operands of step m + 2 (past the end: the last block again, unused)
  const int b2 = spine_block<FWD>(S, m + 2 < S.NB ? m + 2 : S.NB - 1);
  load_l<ST, FWD>(S, b2, i, p, s);
  __syncthreads();
  // y_B = L(B,B)^{-1} t  (back: L(B,B)^{-T} t)
  mine = 0.0;
#pragma unroll
  for (int r = 0; r < RHS_MAX; ++r) {
    if (r > 0 && r >= S.nrhs) break;
    const lds_d* tp = tl + r * T + 4 * p;
    const double acc = red8(fma(s.df[3], tp[3], fma(s.df[2], tp[2], fma(s.df[1], tp[1], s.df[0] * tp[0]))));
    mine = p == r ? acc : mine;
  }
  // The stores are made by every lane (the publication buffers have RHS_MAX
  // columns; the solution's masked-off lanes write the sink): a store that
  // might be skipped would leave the compiler unsure how many operations
  // follow each pending load, and it would wait for more of them.
  const int64_t row = (int64_t)B * T + i;
  if (p < S.nrhs) ring[ring_slot<ST>(B) * (T * RHS_MAX) + p * T + i] = mine;
  astore<double>(S.pub + p * S.NBT + row, mine);
  if (!FWD) *(glb_d*)opaque(p < S.nrhs && row < S.a.n ? S.out + p * S.ldout + row : S.sink) = mine;
  load_d<ST, FWD>(S, b2, i, p, s);
  __syncthreads();
  return *s_fail == 0;
}

template <int ST, bool FWD>
__device__ __forceinline__ void spine(const SolveArgs& S, lds_d* ring, lds_d* tl, lds_i* s_fail) {
  const int tid = threadIdx.x, i = tid >> 3, p = tid & 7;
  for (int e = tid; e < (ST + 1) * T * RHS_MAX; e += NT) ring[e] = 0.0;
  Stage<ST> s0, s1;
  const int b1 = spine_block<FWD>(S, S.NB > 1 ? 1 : 0);
  load_l<ST, FWD>(S, spine_block<FWD>(S, 0), i, p, s0);
  load_d<ST, FWD>(S, spine_block<FWD>(S, 0), i, p, s0);
  load_l<ST, FWD>(S, b1, i, p, s1);
  load_d<ST, FWD>(S, b1, i, p, s1);
  __syncthreads();
  for (int m = 0; m < S.NB; m += 2) {
    if (!spine_step<ST, FWD>(S, m, s0, ring, tl, s_fail)) return;
    if (m + 1 < S.NB && !spine_step<ST, FWD>(S, m + 1, s1, ring, tl, s_fail)) return;
  }
}

// Helper for block B: z_B = sum over the far neighbours N of L(B,N) y_N
// (forward, N = B-KS .. B-ST-1) or L(N,B)^T x_N (back, N = B+KS .. B+ST+1),
// taken in the order they are published, G blocks per round of loads.
// Thread (i, p): row (column) i of B, rows 4p .. 4p+3 of each N.
template <int ST, bool FWD>
__device__ __forceinline__ bool helper(const SolveArgs& S, int B, lds_i* s_flag) {
  const int tid = threadIdx.x, i = tid >> 3, p = tid & 7;
  const int nfar = FWD ? (B - ST - 1) - (B - S.KS > 0 ? B - S.KS : 0) + 1
                       : (B + S.KS < S.NB - 1 ? B + S.KS : S.NB - 1) - (B + ST + 1) + 1;
  const int N0 = FWD ? (B - S.KS > 0 ? B - S.KS : 0) : (B + S.KS < S.NB - 1 ? B + S.KS : S.NB - 1);
  const int dir = FWD ? 1 : -1;
  for (int r0 = 0; r0 < S.nrhs; r0 += HR) {
    const int nr = S.nrhs - r0 < HR ? S.nrhs - r0 : HR;
    double acc[HR];
#pragma unroll
    for (int rr = 0; rr < HR; ++rr) acc[rr] = 0.0;
    for (int g0 = 0; g0 < nfar; g0 += G) {
      double lf[G][4], yv[G][HR][4];
      bool miss = false;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const bool on = g0 + g < nfar;
        const int N = N0 + dir * (g0 + g);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t gi = FWD ? (int64_t)B * T + i : (int64_t)N * T + 4 * p + q;
          const int64_t gj = FWD ? (int64_t)N * T + 4 * p + q : (int64_t)B * T + i;
          lf[g][q] = *band_or_zero(S, on ? gi : S.a.n, gj);
        }
#pragma unroll
        for (int rr = 0; rr < HR; ++rr)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const bool v_on = on && rr < nr;
            yv[g][rr][q] =
                aload<double>(opaque(v_on ? S.pub + (r0 + rr) * S.NBT + (int64_t)N * T + 4 * p + q : S.zero));
            miss |= unset(yv[g][rr][q]);
          }
      }
      if (__syncthreads_or(miss)) {
        // Not all published yet: thread 0 waits for the newest block of the
        // round (one poller per workgroup), then every missing element is
        // awaited on its own.
        const int gl = (nfar - g0 < G ? nfar - g0 : G) - 1;
        const int Nl = N0 + dir * (g0 + gl);
        if (tid == 0) {
          double v;
          *s_flag = await_value(S.pub + (r0 + nr - 1) * S.NBT + (int64_t)Nl * T + T - 1, S.abort_flag, v) ? 0 : 1;
        }
        __syncthreads();
        if (*s_flag) return false;
        bool ok = true;
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int N = N0 + dir * (g0 + g);
#pragma unroll
          for (int rr = 0; rr < HR; ++rr)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (ok && unset(yv[g][rr][q]))
                ok = await_value(S.pub + (r0 + rr) * S.NBT + (int64_t)N * T + 4 * p + q, S.abort_flag, yv[g][rr][q]);
        }
        if (__syncthreads_or(!ok)) return false;
      }
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int rr = 0; rr < HR; ++rr)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[rr] = fma(lf[g][q], yv[g][rr][q], acc[rr]);
    }
#pragma unroll
    for (int rr = 0; rr < HR; ++rr) {
      const double s = red8(acc[rr]);
      if (rr < nr && p == ((r0 + rr) & 7)) astore<double>(S.z + ((int64_t)B * S.nrhs + r0 + rr) * T + i, s);
    }
  }
  return true;
}

// ---------------------------------------------------------------- kernels

template <int ST, bool FWD>
__global__ void __launch_bounds__(NT) solve_kernel(SolveArgs S) {
  __shared__ double ring[(ST + 1) * T * RHS_MAX];
  __shared__ double tl[T * RHS_MAX];
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
      spine<ST, FWD>(S, (lds_d*)ring, (lds_d*)tl, (lds_i*)&s_flag);
    } else {
      // forward: B = ST+1 .. NB-1; back: B = NB-ST-2 .. 0
      const int B = FWD ? ST + t : S.NB - ST - 1 - t;
      if (!helper<ST, FWD>(S, B, (lds_i*)&s_flag)) break;
    }
    if (s_flag) break;
  }
}

// Fills the first len elements of the 4 publication buffers (stride apart)
// with the unset pattern, zeroes the counters and sets the zero element.
__global__ void solve_fill_kernel(glb_d* p, int64_t len, int64_t stride, unsigned* queues, glb_i* abort_flag,
                                  glb_d* zero) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t x = g; x < 4 * len; x += (int64_t)gridDim.x * blockDim.x)
    p[(x / len) * stride + x % len] = __longlong_as_double(UNSET);
  if (g == 0) {
    queues[0] = 0;
    queues[1] = 0;
    *abort_flag = 0;
    *zero = 0.0;
  }
}

// Per diagonal tile, L(C,C)^{-T} (row-major): lanes 0..T-1 hold the rows of
// L(C,C), lanes T..2T-1 the identity rows, solved against L(C,C) column by column.
__global__ void __launch_bounds__(64) tri_inv_kernel(Band a, int NB, glb_d* dinvt) {
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

// Writes the operand buffer of one direction (layout at chunk_len): per
// block B, the ST tiles of L next to it (zero outside the band and past
// either end) and the inverse of its diagonal tile, from dinvt.
template <int ST, bool FWD>
__global__ void __launch_bounds__(NT) prep_kernel(Band a, int NB, const glb_d* dinvt, glb_d* ops) {
  const int B = blockIdx.x, tid = threadIdx.x, i = tid >> 3, p = tid & 7;
  glb_d* c = ops + (int64_t)B * chunk_len(ST);
#pragma unroll
  for (int t = 0; t <= ST; ++t) {
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (t < ST) {
        const int N = FWD ? B - (t + 1) : B + (t + 1);
        const int64_t gi = FWD ? (int64_t)B * T + i : (int64_t)N * T + 4 * p + q;
        const int64_t gj = FWD ? (int64_t)N * T + 4 * p + q : (int64_t)B * T + i;
        v[q] = (N >= 0 && N < NB && a.in_band(gi, gj)) ? *a.at(gi, gj) : 0.0;
      } else {
        const glb_d* di = dinvt + (int64_t)B * T * T;
        v[q] = FWD ? di[(4 * p + q) * T + i] : di[i * T + 4 * p + q];
      }
    }
    *(glb_d2*)(c + slot(t, 0, tid)) = d2{v[0], v[1]};
    *(glb_d2*)(c + slot(t, 1, tid)) = d2{v[2], v[3]};
  }
}

template <int ST>
void launch_pair(const Band& a, const glb_d* dinvt, glb_d* ops, const SolveArgs& f, const SolveArgs& b, int grid,
                 hipStream_t st) {
  prep_kernel<ST, true><<<f.NB, NT, 0, st>>>(a, f.NB, dinvt, ops);
  solve_kernel<ST, true><<<grid, NT, 0, st>>>(f);
  prep_kernel<ST, false><<<f.NB, NT, 0, st>>>(a, f.NB, dinvt, ops);
  solve_kernel<ST, false><<<grid, NT, 0, st>>>(b);
}

// Blocks of the band the spine applies itself: all of them up to ST_MAX,
// rounded up to an instantiated width; beyond, ST_MAX and helpers.
inline int spine_width(int KS) { return KS <= 1 ? 1 : KS <= 2 ? 2 : KS <= 4 ? 4 : ST_MAX; }

inline int tile_blocks_of(int64_t n, int64_t k) {
  const int NB = (int)((n + T - 1) / T);
  int KS = (int)((k + T - 1) / T);
  if (KS > NB - 1) KS = NB - 1 > 0 ? NB - 1 : 0;
  return KS;
}

}  // namespace bandchol_solve

// Host side, called by the C-ABI (same library).  Workspace layout, in bytes
// from `ws`: [0,256) two ticket counters, the abort flag, (at 64) the zero
// element and (at 128) the sink; then the publication area, 4 * RHS_MAX * NBT
// doubles (forward result, back result, forward and back helper sums, RHS_MAX
// * NBT each, of which a pass of nrhs right-hand sides uses the first
// nrhs * NBT); then the inverted diagonal tiles,
// NB * T * T doubles; then the operand buffer, NB * chunk_len(ST) doubles.
size_t bandchol_solve_workspace(int64_t n, int64_t k) {
  using namespace bandchol_solve;
  const int64_t NB = (n + T - 1) / T, NBT = NB * T;
  const int ST = spine_width(tile_blocks_of(n, k));
  return 256 + sizeof(double) * ((size_t)(4 * RHS_MAX + T) * NBT + (size_t)NB * chunk_len(ST));
}

hipError_t bandchol_solve_launch(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, double* b,
                                 int64_t ldb, void* ws, int num_cus, hipStream_t st) {
  using namespace bandchol_solve;
  const int NB = (int)((n + T - 1) / T);
  const int64_t NBT = (int64_t)NB * T;
  const int KS = tile_blocks_of(n, k);
  const int ST = spine_width(KS);
  char* base = (char*)ws;
  unsigned* queues = (unsigned*)base;
  glb_i* abort_flag = (glb_i*)(base + 8);
  glb_d* zero = (glb_d*)(base + 64);
  glb_d* sink = (glb_d*)(base + 128);
  glb_d* pubarea = (glb_d*)(base + 256);
  glb_d* dinvt = pubarea + (size_t)4 * RHS_MAX * NBT;
  glb_d* ops = dinvt + (size_t)NB * T * T;
  const Band a{(glb_d*)const_cast<double*>(ab), n, k, ldab};
  tri_inv_kernel<<<NB, 64, 0, st>>>(a, NB, dinvt);
  const int nhelp = KS > ST ? NB - ST - 1 : 0;
  // one workgroup per CU at most: the spine keeps a CU to itself
  const int grid = 1 + nhelp < num_cus ? 1 + nhelp : num_cus;
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
                                                                         abort_flag, zero);
    switch (ST) {
      case 1: launch_pair<1>(a, dinvt, ops, F, Bk, grid, st); break;
      case 2: launch_pair<2>(a, dinvt, ops, F, Bk, grid, st); break;
      case 4: launch_pair<4>(a, dinvt, ops, F, Bk, grid, st); break;
      default: launch_pair<ST_MAX>(a, dinvt, ops, F, Bk, grid, st); break;
    }
  }
  return hipGetLastError();
}
