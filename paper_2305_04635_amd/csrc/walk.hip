// Single-workgroup band Cholesky ("walk") for narrow bands, and the batched
// factor and solve built on it (gfx950, FP64).
//
// One workgroup factors one matrix, right-looking and in place, with no
// communication outside the workgroup (Algorithm 1's potrf / trsm / syrk+gemm
// steps on T x T tiles, Section 3).  Per tile column C:
//   phase A  wave 0: sweep of the staged diagonal tile -> L(C,C), L(C,C)^{-T};
//            waves 1-3: the work of column C-1 that the next diagonal tile does
//            not wait for: trsm of tiles (C-1+d, C-1), d >= 2, then the updates
//            tile(C-1+dr, C-1+dc) -= L(C-1+dr, C-1) L(C-1+dc, C-1)^T, all pairs but (1,1);
//   phase B  all waves: trsm of tile (C+1, C) (the critical one);
//   phase C  waves 1-3: diag = tile(C+1, C+1) - L(C+1, C) L(C+1, C)^T, staged
//            for the next sweep; wave 0 stores L(C,C)^{-T} when asked to.
// The current tile column's L tiles stay in LDS (pnl) for the updates.
//
// The batched kernels take a descriptor per system and an order (longest
// first); every workgroup takes the next system from an atomic counter.
#include <stdint.h>

#include <mutex>
#include <vector>

#include "common.h"
#include "walk.h"

namespace bandchol_walk {

using namespace bandchol;

constexpr int NT = 256;          // batched solves
constexpr int WALK_WAVES = 8;    // walk: wave 0 sweeps, the others take the tile column's remaining work
constexpr int UPD_WAVES = WALK_WAVES - 1;
constexpr int WALK_NT = 64 * WALK_WAVES;

// ----------------------------------------------------------------- tile helpers

// Fragments of row-block bi of tile (R, C): x[q] = A(R*T + 16 bi + l%16, C*T + 4q + l/16).
__device__ __forceinline__ void rowblk_load(const Band& a, int64_t R, int64_t C, int bi, double (&x)[T / 4]) {
  const int lane = lane_id();
  const Run run = band_run(a, R * T + 16 * bi + (lane & 15), C * T + (lane >> 4), 4);
#pragma unroll
  for (int q = 0; q < T / 4; ++q) x[q] = run.ld(q);
}

// out block (bi, bj) = X_rowblk * L^{-T}(:, 16bj..16bj+15); L^{-T} row-major in LDS
// (pitch LP), upper triangular.
__device__ __forceinline__ d4 blk_trsm_frag(const double (&x)[T / 4], const lds_d* linvt, int bj) {
  const int lane = lane_id();
  const int qmax = 4 * bj + 4;
  d4 out = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < T / 4; ++q)
    if (q < qmax) out = mfma_xyt(x[q], linvt[(4 * q + (lane >> 4)) * LP + 16 * bj + (lane & 15)], out);
  return out;
}

// One wave: tile (R, C) <- tile (R, C) * L(C,C)^{-T}, written to global and to an
// LDS copy.  Every output block needs the input row-block over all columns, so
// all input fragments are read before any output is written.
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

// ----------------------------------------------------------------- band as a buffer resource

// The band from column j0 on as a buffer resource.  A buffer load whose offset
// lies past the resource's size returns zero and such a store is dropped, so
// the accesses of lanes outside the band (and of idle pipeline slots) go to
// offset BUF_OOB and need no branch: every load and store is issued, and the
// compiler can count the outstanding ones exactly.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int BUF_OOB = 0x7fffffff;
constexpr int64_t BUF_MAX = 0x7fff0000;   // resource size cap (bytes); offsets stay below it

struct BandBuf {
  __amdgpu_buffer_rsrc_t rsrc;
  int64_t n, k, ldab, j0;
};

// The same value in every lane, held in scalar registers (arguments of a
// non-inlined function arrive in vector registers; a buffer resource must not).
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni(int64_t x) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(uint64_t)x);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ BandBuf band_buf(const Band& a, int64_t j0) {
  BandBuf b;
  b.n = uni(a.n), b.k = uni(a.k), b.ldab = uni(a.ldab), b.j0 = uni(j0);
  const int64_t left = (b.n - b.j0) * b.ldab * (int64_t)sizeof(double);
  const int64_t base = uni((int64_t)(uintptr_t)(a.ab + j0 * a.ldab));
  b.rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)(uintptr_t)base, (short)0,
                                             (int)(left < BUF_MAX ? left : BUF_MAX), 0x00020000);
  return b;
}

// Whether every element of the tile columns j0/T .. j0/T + K + 1 lies at a byte
// offset below BUF_MAX from column j0.
__device__ __forceinline__ bool band_buf_fits(const Band& a, int K) {
  return (int64_t)(K + 2) * T * a.ldab * (int64_t)sizeof(double) < BUF_MAX;
}

// Byte offsets of this lane's accumulator elements of block (bi, bj) of tile
// (R, C) (BUF_OOB outside the band, or for every lane when !live).
__device__ __forceinline__ void blk_offsets(const BandBuf& b, int64_t R, int64_t C, int bi, int bj, bool live,
                                            int (&off)[4]) {
  // 32-bit arithmetic throughout: rows and columns are below 2^31 and, with
  // band_buf_fits, every offset from column j0 is below BUF_MAX
  const int lane = lane_id();
  const int i = (int)R * T + 16 * bi + (lane & 15);
  const int j = (int)C * T + 16 * bj + Prec<double>::acc_col0(lane);
  const int ldab = (int)b.ldab, k = (int)b.k, n = (int)b.n;
  const int base = (i - j) + (j - (int)b.j0) * ldab;
  const int step = Prec<double>::ACC_STEP * (ldab - 1);
  const bool row = live && i < n;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int d = i - j - Prec<double>::ACC_STEP * r;
    off[r] = (row && d >= 0 && d <= k) ? (base + step * r) * (int)sizeof(double) : BUF_OOB;
  }
}

__device__ __forceinline__ d4 blk_bload(const BandBuf& b, const int (&off)[4]) {
  d4 v;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    v[r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(b.rsrc, off[r], 0, 0));
  return v;
}

// The elements go through scalars: __builtin_bit_cast applied to a vector
// element (v[r]) yields element 0 for every r with this compiler.
__device__ __forceinline__ void blk_bstore(const BandBuf& b, const int (&off)[4], d4 v) {
  const double e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double x = e[r];
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), b.rsrc, off[r], 0, 0);
  }
}

// The trailing tiles of one tile column: (dr, dc), 1 <= dc <= dr <= dmax,
// without (1, 1) (the next diagonal tile's critical update, done in phase C);
// every UPD_WAVES-th one for wave w (1..UPD_WAVES).
struct TileGen {
  int dr, dc, idx, dmax, w;
  __device__ __forceinline__ bool next(int& odr, int& odc) {
    for (;;) {
      if (dr > dmax) return false;
      const int cdr = dr, cdc = dc;
      if (++dc > dr) dc = 1, ++dr;
      if (cdr == 1 && cdc == 1) continue;
      if (idx++ % UPD_WAVES != w - 1) continue;
      odr = cdr, odc = cdc;
      return true;
    }
  }
};

// One tile of the update in flight: its four blocks (acc[bi + 2 bj]) and their
// element offsets (the upper block of a diagonal tile, and every block of a
// dead slot, at BUF_OOB).
struct TileSlot {
  int dr, dc;
  bool live;
  int off[4][4];
  d4 acc[4];
};

__device__ __forceinline__ void tile_issue(const BandBuf& b, int64_t Cp, TileGen& gen, TileSlot& s) {
  s.live = gen.next(s.dr, s.dc);
  if (!s.live) s.dr = s.dc = 1;
#pragma unroll
  for (int blk = 0; blk < 4; ++blk) {
    const int bi = blk & 1, bj = blk >> 1;
    blk_offsets(b, Cp + s.dr, Cp + s.dc, bi, bj, s.live && !(s.dr == s.dc && bj > bi), s.off[blk]);
    s.acc[blk] = blk_bload(b, s.off[blk]);
  }
}

// acc[bi + 2 bj] -= X(bi) Y(bj)^T with X, Y the panel tiles (LDS, column-major,
// pitch LP): per k-step two fragments of each feed four independent MFMAs.
__device__ __forceinline__ void tile_update(const lds_d* x, const lds_d* y, d4 (&acc)[4]) {
  const int lane = lane_id();
#pragma unroll
  for (int q = 0; q < T / 4; ++q) {
    const int kk = 4 * q + (lane >> 4);
    const double x0 = -x[kk * LP + (lane & 15)], x1 = -x[kk * LP + 16 + (lane & 15)];
    const double y0 = y[kk * LP + (lane & 15)], y1 = y[kk * LP + 16 + (lane & 15)];
    acc[0] = mfma_xyt(x0, y0, acc[0]);
    acc[1] = mfma_xyt(x1, y0, acc[1]);
    acc[2] = mfma_xyt(x0, y1, acc[2]);
    acc[3] = mfma_xyt(x1, y1, acc[3]);
  }
}

__device__ __forceinline__ void tile_finish(const BandBuf& b, const lds_d* pnl, lds_d* stB, lds_d* stC,
                                            TileSlot& s) {
  tile_update(pnl + (size_t)(s.dr - 1) * T * LP, pnl + (size_t)(s.dc - 1) * T * LP, s.acc);
  lds_d* st = s.dr == 2 ? (s.dc == 1 ? stB : stC) : nullptr;
  if (st) {
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) blk_to_lds(st, blk & 1, blk >> 1, s.acc[blk]);
    return;
  }
#pragma unroll
  for (int blk = 0; blk < 4; ++blk) blk_bstore(b, s.off[blk], s.acc[blk]);
}

// One panel tile (Cp + d, Cp) of the column's trsm: both row-blocks
// of its current value, x[bi][q] = A(R*T + 16 bi + l%16, Cp*T + 4q + l/16).
struct PanelSlot {
  int d;
  bool live;
  double x[2][T / 4];
};

__device__ __forceinline__ void panel_issue(const BandBuf& b, int64_t Cp, int d, int dmax, PanelSlot& s) {
  const int lane = lane_id();
  s.live = d <= dmax;
  s.d = s.live ? d : 2;
  const int64_t j = Cp * T + (lane >> 4);
#pragma unroll
  for (int bi = 0; bi < 2; ++bi) {
    const int64_t i = (Cp + s.d) * T + 16 * bi + (lane & 15);
    const int base = (int)((i - j) + (j - b.j0) * b.ldab);
#pragma unroll
    for (int q = 0; q < T / 4; ++q) {
      const int64_t dd = i - j - 4 * q;
      const bool in = s.live && i < b.n && dd >= 0 && dd <= b.k;
      const int off = in ? (base + 4 * q * (int)(b.ldab - 1)) * (int)sizeof(double) : BUF_OOB;
      s.x[bi][q] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(b.rsrc, off, 0, 0));
    }
  }
}

// L(Cp + d, Cp) = tile * L(Cp,Cp)^{-T}: into the panel's LDS slot d-1 and back
// to the band.
__device__ __forceinline__ void panel_finish(const BandBuf& b, int64_t Cp, const lds_d* linvt, lds_d* pnl,
                                             PanelSlot& s) {
  lds_d* out = pnl + (size_t)(s.d - 1) * T * LP;
#pragma unroll
  for (int blk = 0; blk < 4; ++blk) {
    const int bi = blk & 1, bj = blk >> 1;
    const d4 o = blk_trsm_frag(s.x[bi], linvt, bj);
    blk_to_lds(out, bi, bj, o);
    int off[4];
    blk_offsets(b, Cp + s.d, Cp, bi, bj, s.live, off);
    blk_bstore(b, off, o);
  }
}

// Up to this many tile diagonals the LDS also holds two staging tiles: the
// next step's tiles (C+1, C) and (C+1, C+1) stay there after their last update
// instead of a round trip through the band.
constexpr int STAGE_KMAX = 13;

struct WalkLds {
  lds_d* diag;    // T*LP
  lds_d* linvt;   // 2 x T*LP (row-major, pitch LP), alternating by column parity
  lds_d* pnl;     // K x T*LP
  lds_d* stB;     // T*LP: tile (C+1, C) before its trsm (null past STAGE_KMAX)
  lds_d* stC;     // T*LP: tile (C+1, C+1) before its last update (null past STAGE_KMAX)
};

__device__ __forceinline__ WalkLds walk_lds(lds_d* base, int K) {
  WalkLds L;
  L.diag = base;
  L.linvt = L.diag + T * LP;
  L.pnl = L.linvt + 2 * T * LP;
  L.stB = K <= STAGE_KMAX ? L.pnl + (size_t)K * T * LP : nullptr;
  L.stC = K <= STAGE_KMAX ? L.stB + T * LP : nullptr;
  return L;
}

// Whether this step's phase-A update leaves tiles (C+1, C) and (C+1, C+1) in
// the staging tiles: there is LDS for them, the update runs on the buffer path,
// and both tiles lie inside the band of the column updated (K >= 2).
__device__ __forceinline__ bool walk_staged(const WalkLds& L, const Band& a, int K);

// ----------------------------------------------------------------- the walk
//
// The noinline functions copy their structure arguments into locals first:
// the references point at a stack copy, and after every store the fields
// would otherwise be re-read from memory.

// wave 0: factor the staged diagonal tile, store L(C,C), keep L(C,C)^{-T} in LDS
__device__ __attribute__((noinline)) void walk_sweep(const Band& a_, int64_t C, const WalkLds& L_, lds_d* lt,
                                                     lds_i* s_fail) {
  const Band a = a_;
  const WalkLds L = L_;
  const int lane = lane_id();
  double row[T];
#pragma unroll
  for (int c = 0; c < T; ++c) row[c] = lane < T ? L.diag[c * LP + lane] : ((lane - T) == c ? 1.0 : 0.0);
  const int fail = sweep_ldlt(row, L.diag, lt);  // both free while this wave sweeps
  if (fail >= 0) {
    if (lane == 0) *s_fail = fail;
    return;
  }
  const Run run = band_run(a, C * T + (lane & 31), C * T, 1);
#pragma unroll
  for (int c = 0; c < T; ++c) {
    if (lane < T) {
      if (run.in(c)) *run.at(c) = row[c];
    } else {
      lt[(lane - T) * LP + c] = row[c];
    }
  }
}

// waves 1-3: the rest of tile column Cp (trsm of d >= 2, then all updates but the critical one)
__device__ __forceinline__ void walk_column_rest(const Band& a_, int K, int64_t NB, int64_t Cp,
                                                           const WalkLds& L_, const lds_d* lt_prev, lds_i* s_sync,
                                                           int sync_target) {
  const Band a = a_;
  const WalkLds L = L_;
  const int wave = wave_id(), lane = lane_id();
  if (band_buf_fits(a, K)) {
    const int64_t Cu = uni(Cp);
    const int dmax = uni((int)(K < NB - 1 - Cu ? K : NB - 1 - Cu));
    const BandBuf bp = band_buf(a, Cu * T);         // the panel's tile column
    const BandBuf b = band_buf(a, (Cu + 1) * T);    // the trailing tile columns
    TileGen gen{1, 1, 0, dmax, uni(wave)};
    TileSlot s0, s1;
    // the panel tiles (Cp + d, Cp), d = 2 .. dmax, every UPD_WAVES-th for this
    // wave, one at a time (a second one in flight cost more in spills than it hid)
    for (int d = 1 + uni(wave); d <= dmax; d += UPD_WAVES) {
      PanelSlot p0;
      panel_issue(bp, Cu, d, dmax, p0);
      panel_finish(bp, Cu, lt_prev, L.pnl, p0);
    }
    // the first update tile's loads after the panel work: issued earlier they
    // kept 48 more registers live through it and the panel loop spilled
    tile_issue(b, Cu, gen, s0);
    // waves 1-7 meet before using each other's panel tiles
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): this wave's LDS writes are done
    if (lane == 0) __hip_atomic_fetch_add(s_sync, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    while (__hip_atomic_load(s_sync, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < sync_target)
      __builtin_amdgcn_s_sleep(1);
    // whole tiles per wave, the next one's loads in flight while the current
    // one is on the matrix cores (two slots, alternating)
    for (;;) {
      if (!s0.live) break;
      tile_issue(b, Cu, gen, s1);
      tile_finish(b, L.pnl, L.stB, L.stC, s0);
      if (!s1.live) break;
      tile_issue(b, Cu, gen, s0);
      tile_finish(b, L.pnl, L.stB, L.stC, s1);
    }
    return;
  }
  for (int d = 2; d <= K && Cp + d < NB; ++d)
    if ((d - 2) % UPD_WAVES == wave - 1) tile_trsm_wave(a, Cp + d, Cp, lt_prev, L.pnl + (size_t)(d - 1) * T * LP);
  int idx = 0;
  // waves 1-7 meet before using each other's panel tiles
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
        if (idx++ % UPD_WAVES != wave - 1) continue;
        d4 acc = blk_load(a, Cp + dr, Cp + dc, bi, bj);
        acc = blk_gemm_lds(L.pnl + (size_t)(dr - 1) * T * LP, L.pnl + (size_t)(dc - 1) * T * LP, bi, bj, acc);
        blk_store(a, Cp + dr, Cp + dc, bi, bj, acc);
      }
    }
  }
}

// wave 0: L(C,C)^{-T} from LDS (pitch LP) to dense row-major T x T global memory
__device__ __forceinline__ void store_linvt(const lds_d* lt, glb_d* dst) {
  const int lane = lane_id();
  double v[T / 2];
#pragma unroll
  for (int p = 0; p < T / 2; ++p) {
    const int e = 64 * p + lane;
    v[p] = lt[(e / T) * LP + (e % T)];
  }
#pragma unroll
  for (int p = 0; p < T / 2; ++p) dst[64 * p + lane] = v[p];
}

__device__ __forceinline__ bool walk_staged(const WalkLds& L, const Band& a, int K) {
  return L.stB != nullptr && K >= 2 && band_buf_fits(a, K);
}

// The step loop of each wave role, one function per role with the phase work
// inlined (a call inside the loop would save and restore registers around it on
// every step).  Both roles pass the same barriers: after phase A, inside phase
// B (K >= 1), after phase B and after phase C.  They return the tile column
// whose sweep failed (the column inside it in *s_fail), or -1.
__device__ __attribute__((noinline)) int64_t walk_wave0(const Band& a_, int K, const WalkLds& L_, double* linv,
                                                       lds_i* s_fail, bool staged) {
  const Band a = a_;
  const WalkLds L = L_;
  const int64_t NB = (a.n + T - 1) / T;
  const int lane = lane_id();
  for (int64_t C = 0; C < NB; ++C) {
    lds_d* lt = L.linvt + (C & 1) * T * LP;
    // ---------------- phase A: sweep of the staged diagonal tile
    walk_sweep(a, C, L, lt, s_fail);
    wait_vmem();
    __syncthreads();
    if (*s_fail >= 0) return C;
    if (C + 1 >= NB) {
      if (linv) store_linvt(lt, (glb_d*)linv + C * T * T);
      break;
    }
    // ---------------- phase B: block (0, 0) of the trsm of tile (C+1, C)
    const bool from_lds = staged && C >= 1;
    if (K >= 1) {
      double x[T / 4];
      if (from_lds) {
#pragma unroll
        for (int q = 0; q < T / 4; ++q) x[q] = L.stB[(4 * q + (lane >> 4)) * LP + (lane & 15)];
      } else {
        rowblk_load(a, C + 1, C, 0, x);
      }
      wait_vmem();
      __syncthreads();
      const d4 out = blk_trsm_frag(x, lt, 0);
      blk_to_lds(L.pnl, 0, 0, out);
      blk_store(a, C + 1, C, 0, 0, out);
    }
    wait_vmem();
    __syncthreads();
    // ---------------- phase C: the upper block of the next diagonal tile, L(C,C)^{-T} out
    blk_to_lds(L.diag, 0, 1, d4{0, 0, 0, 0});
    if (linv) store_linvt(lt, (glb_d*)linv + C * T * T);
    __syncthreads();
  }
  return -1;
}

__device__ __attribute__((noinline)) int64_t walk_waves(const Band& a_, int K, const WalkLds& L_, lds_i* s_fail,
                                                       lds_i* s_sync, bool staged) {
  const Band a = a_;
  const WalkLds L = L_;
  const int64_t NB = (a.n + T - 1) / T;
  const int wave = wave_id(), lane = lane_id();
  int sync_target = 0;
  for (int64_t C = 0; C < NB; ++C) {
    lds_d* lt = L.linvt + (C & 1) * T * LP;
    const lds_d* lt_prev = L.linvt + ((C + 1) & 1) * T * LP;
    // ---------------- phase A: the rest of tile column C-1
    if (C >= 1) walk_column_rest(a, K, NB, C - 1, L, lt_prev, s_sync, sync_target += UPD_WAVES);
    wait_vmem();
    __syncthreads();
    if (*s_fail >= 0) return C;
    if (C + 1 >= NB) break;
    // ---------------- phase B: blocks of the trsm of tile (C+1, C), one per wave 1-3
    const bool from_lds = staged && C >= 1;
    if (K >= 1) {
      const bool mine = wave < 4;
      const int bi = wave & 1, bj = (wave >> 1) & 1;
      double x[T / 4];
      if (mine) {
        if (from_lds) {
#pragma unroll
          for (int q = 0; q < T / 4; ++q) x[q] = L.stB[(4 * q + (lane >> 4)) * LP + 16 * bi + (lane & 15)];
        } else {
          rowblk_load(a, C + 1, C, bi, x);
        }
      }
      wait_vmem();
      __syncthreads();   // every wave holds its input before any output is written
      if (mine) {
        const d4 out = blk_trsm_frag(x, lt, bj);
        blk_to_lds(L.pnl, bi, bj, out);
        blk_store(a, C + 1, C, bi, bj, out);
      }
    }
    wait_vmem();
    __syncthreads();
    // ---------------- phase C: stage tile (C+1, C+1) minus the critical update
    if (wave <= 3) {
      const int bi = (wave >= 2), bj = (wave == 3);
      d4 acc;
      if (from_lds) {
        acc = blk_from_lds(L.stC, bi, bj);
        // rows past n: the identity, as blk_load gives
        const int64_t i = (C + 1) * T + 16 * bi + (lane & 15);
        const int64_t j = (C + 1) * T + 16 * bj + Prec<double>::acc_col0(lane);
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (i >= a.n && i == j + Prec<double>::ACC_STEP * r) acc[r] = 1.0;
      } else {
        acc = blk_load(a, C + 1, C + 1, bi, bj);
      }
      if (K >= 1) acc = blk_gemm_lds(L.pnl, L.pnl, bi, bj, acc);
      blk_to_lds(L.diag, bi, bj, acc);
    }
    __syncthreads();
  }
  return -1;
}

// Returns info (0 or the 1-based failing column).  linv: if not null, receives
// L(C,C)^{-T} (row-major T x T) for every tile column C.
__device__ int64_t walk_factor(const Band a, const int K, const WalkLds L, double* linv, lds_i* s_fail,
                               lds_i* s_sync) {
  const int wave = wave_id();
  const bool staged = walk_staged(L, a, K);
  if (threadIdx.x == 0) { *s_fail = -1; *s_sync = 0; }
  // stage tile (0, 0)
  if (wave >= 1 && wave <= 3) {
    const int bi = (wave >= 2), bj = (wave == 3);
    blk_to_lds(L.diag, bi, bj, blk_load(a, 0, 0, bi, bj));
  } else if (wave == 0) {
    blk_to_lds(L.diag, 0, 1, d4{0, 0, 0, 0});
  }
  __syncthreads();
  const int64_t Cf = wave == 0 ? walk_wave0(a, K, L, linv, s_fail, staged) : walk_waves(a, K, L, s_fail, s_sync, staged);
  return Cf >= 0 ? Cf * T + *s_fail + 1 : 0;
}

__global__ void __launch_bounds__(WALK_NT) walk_single_kernel(WalkSys w, int K, int64_t* info) {
  extern __shared__ double lds_dyn[];
  __shared__ int s_fail, s_sync;
  const Band a{(glb_d*)w.ab, w.n, w.k, w.ldab};
  const int64_t res = walk_factor(a, K, walk_lds((lds_d*)lds_dyn, K), w.linv, (lds_i*)&s_fail, (lds_i*)&s_sync);
  if (threadIdx.x == 0) *info = res;
}

// Batched factor: systems sys[order[t]] for t = 0, 1, ... taken from *queue.
__global__ void __launch_bounds__(WALK_NT) walk_batch_kernel(const WalkSys* sys, const int* order, int nsys, int Kmax,
                                                        unsigned* queue, int64_t* info) {
  extern __shared__ double lds_dyn[];
  __shared__ int s_idx, s_fail, s_sync;
  for (;;) {
    if (threadIdx.x == 0) s_idx = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int t = s_idx;
    if (t >= nsys) break;
    const int id = order[t];
    const WalkSys w = sys[id];
    const int64_t kk = w.k < w.n - 1 ? w.k : (w.n > 0 ? w.n - 1 : 0);
    const int K = (int)((kk + T - 1) / T);
    const Band a{(glb_d*)w.ab, w.n, kk, w.ldab};
    int64_t res = 0;
    if (w.n > 0 && K <= Kmax) res = walk_factor(a, K, walk_lds((lds_d*)lds_dyn, Kmax), w.linv, (lds_i*)&s_fail,
                                                 (lds_i*)&s_sync);
    if (threadIdx.x == 0) info[id] = res;
    __syncthreads();
  }
}

// ----------------------------------------------------------------- batched solves
//
// One workgroup solves one system, block of T rows by block, with up to
// RHS_PASS right-hand sides per pass; the diagonal blocks are applied through
// the inverses L(C,C)^{-T} kept by the factorization, so no block waits on a
// triangular recurrence.  Lane l of every wave owns row (or column) l % 32 and
// the right-hand sides (l / 32) * (RHS_PASS / 2) ... + RHS_PASS / 2 - 1.  The
// last K+1 solution blocks stay in an LDS ring.
//   forward (L Y = B):   s = b_R - sum_{d=1..K} L(R, R-d) y_{R-d};  y_R = L_RR^{-1} s
//   back   (L^T X = Y):  s = y_C - sum_{d=1..K} L(C+d, C)^T x_{C+d}; x_C = L_CC^{-T} s
// Waves split the K off-diagonal tiles; their partial sums meet in LDS.

constexpr int RH = RHS_PASS / 2;   // right-hand sides per lane

__device__ __forceinline__ lds_d* ring_at(lds_d* ring, int64_t blk, int K) {
  return ring + (size_t)(blk % (K + 1)) * T * RHS_PASS;   // [row][rhs]
}

template <bool FWD>
__device__ void solve_one(const Band& a, int K, const glb_d* linv, glb_d* b, int64_t ldb, int r0, int nr,
                          lds_d* ring, lds_d* part) {
  const int wave = wave_id(), lane = lane_id();
  const int i = lane & 31, h = lane >> 5;
  const int64_t NB = (a.n + T - 1) / T;
  for (int64_t it = 0; it < NB; ++it) {
    const int64_t R = FWD ? it : NB - 1 - it;
    // wave 0: this block's row of L(R,R)^{-T} (or of its transpose) and b, loaded
    // before its share of the tiles, so that they are in registers when the
    // partial sums have met (none of them depends on the chain)
    const int64_t gi = R * T + i;
    double ltr[T], bv[RH];
    if (wave == 0) {
      const glb_d* lt = linv + R * T * T;
#pragma unroll
      for (int c = 0; c < T; ++c) ltr[c] = FWD ? lt[c * T + i] : lt[i * T + c];
      const int64_t gic = gi < a.n ? gi : a.n - 1;
#pragma unroll
      for (int t = 0; t < RH; ++t) {
        const int r = h * RH + t;
        const double v = b[(r0 + (r < nr ? r : 0)) * ldb + gic];
        bv[t] = (gi < a.n && r < nr) ? v : 0.0;
      }
    }
    double acc[RH];
#pragma unroll
    for (int t = 0; t < RH; ++t) acc[t] = 0.0;
    for (int d = wave + 1; d <= K; d += 4) {
      const int64_t S = FWD ? R - d : R + d;   // block of the known solution
      if (S < 0 || S >= NB) continue;
      const lds_d* ys = ring_at(ring, S, K);
      if (FWD) {
        // row i of tile (R, S): A(R*T + i, S*T + j), j = 0..T-1
        const Run run = band_run(a, R * T + i, S * T, 1);
        // sixteen loads per round: eight left a round trip per eight elements,
        // all 32 at once (with 256 workgroups issuing) measured slower
#pragma unroll 16
        for (int j = 0; j < T; ++j) {
          const double l = run.ld(j);
#pragma unroll
          for (int t = 0; t < RH; ++t) acc[t] = fma(l, ys[j * RHS_PASS + h * RH + t], acc[t]);
        }
      } else {
        // column i of tile (S, R): A(S*T + j, R*T + i), j = 0..T-1 (consecutive in memory)
        const int64_t gi = R * T + i;
        const int64_t d0 = S * T - gi;   // row offset of j = 0 inside the band column
        const glb_d* col = a.ab + d0 + gi * a.ldab;
#pragma unroll 16
        for (int j = 0; j < T; ++j) {
          const int64_t dj = d0 + j;
          const double l = (S * T + j < a.n && dj <= a.k) ? col[j] : 0.0;
#pragma unroll
          for (int t = 0; t < RH; ++t) acc[t] = fma(l, ys[j * RHS_PASS + h * RH + t], acc[t]);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < RH; ++t) part[(wave * T + i) * RHS_PASS + h * RH + t] = acc[t];
    __syncthreads();
    if (wave == 0) {
      // s = b_R - sum of the partials (row i, this lane's right-hand sides)
      double s[RH];
#pragma unroll
      for (int t = 0; t < RH; ++t) {
        const int r = h * RH + t;
        double v = bv[t];
#pragma unroll
        for (int w = 0; w < 4; ++w) v -= part[(w * T + i) * RHS_PASS + r];
        s[t] = v;
      }
      lds_d* sbuf = part;   // reuse: [row][rhs]
      __builtin_amdgcn_s_waitcnt(0xC07F);
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int t = 0; t < RH; ++t) sbuf[i * RHS_PASS + h * RH + t] = s[t];
      __builtin_amdgcn_s_waitcnt(0xC07F);
      __builtin_amdgcn_wave_barrier();
      // y_i = sum_c Linv(i, c) s_c = sum_c linvt[c][i] s_c;  x_i = sum_c Linv(c, i) s_c = sum_c linvt[i][c] s_c
      double y[RH];
#pragma unroll
      for (int t = 0; t < RH; ++t) y[t] = 0.0;
#pragma unroll
      for (int c = 0; c < T; ++c)
#pragma unroll
        for (int t = 0; t < RH; ++t) y[t] = fma(ltr[c], sbuf[c * RHS_PASS + h * RH + t], y[t]);
      lds_d* yr = ring_at(ring, R, K);
#pragma unroll
      for (int t = 0; t < RH; ++t) {
        const int r = h * RH + t;
        yr[i * RHS_PASS + r] = (gi < a.n) ? y[t] : 0.0;
        if (gi < a.n && r < nr) b[(r0 + r) * ldb + gi] = y[t];
      }
    }
    __syncthreads();
  }
}

template <bool FWD>
__global__ void __launch_bounds__(NT) solve_batch_kernel(const WalkSys* sys, const int* order, int nsys, int Kmax,
                                                         int nrhs, unsigned* queue) {
  extern __shared__ double lds_dyn[];
  __shared__ int s_idx;
  lds_d* part = (lds_d*)lds_dyn;                     // 4 x T x RHS_PASS
  lds_d* ring = part + 4 * T * RHS_PASS;            // (Kmax+1) x T x RHS_PASS
  for (;;) {
    if (threadIdx.x == 0) s_idx = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int t = s_idx;
    if (t >= nsys) break;
    const int id = order[t];
    const WalkSys w = sys[id];
    const int64_t kk = w.k < w.n - 1 ? w.k : (w.n > 0 ? w.n - 1 : 0);
    const int K = (int)((kk + T - 1) / T);
    const Band a{(glb_d*)w.ab, w.n, kk, w.ldab};
    if (w.n > 0 && K <= Kmax && w.b && w.linv) {
      for (int r0 = 0; r0 < nrhs; r0 += RHS_PASS) {
        const int nr = nrhs - r0 < RHS_PASS ? nrhs - r0 : RHS_PASS;
        solve_one<FWD>(a, K, (const glb_d*)w.linv, (glb_d*)w.b, w.ldb, r0, nr, ring, part);
      }
    }
    __syncthreads();
  }
}

__global__ void batch_clear_kernel(unsigned* queue, int count) {
  if (threadIdx.x < count) queue[threadIdx.x] = 0;
}

}  // namespace bandchol_walk

// ----------------------------------------------------------------- host-side launchers

using namespace bandchol_walk;

size_t bandchol_walk_lds_bytes(int K) {
  return sizeof(double) * ((size_t)(3 + K + (K <= STAGE_KMAX ? 2 : 0)) * T * LP);
}

size_t bandchol_solve_batch_lds_bytes(int Kmax) {
  return sizeof(double) * ((size_t)4 * T * RHS_PASS + (size_t)(Kmax + 1) * T * RHS_PASS);
}

// Raises a kernel's dynamic LDS limit once to the most any launch can ask for
// (so that launches under stream capture change no attributes).
static hipError_t set_lds_attr(const void* fn, size_t lds) {
  (void)lds;
  static std::mutex mu;
  static std::vector<const void*> done;
  std::lock_guard<std::mutex> lk(mu);
  for (const void* f : done)
    if (f == fn) return hipSuccess;
  const size_t most = bandchol_walk_lds_bytes(WALK_KMAX) > bandchol_solve_batch_lds_bytes(WALK_KMAX)
                          ? bandchol_walk_lds_bytes(WALK_KMAX)
                          : bandchol_solve_batch_lds_bytes(WALK_KMAX);
  const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)most);
  if (e == hipSuccess) done.push_back(fn);
  return e;
}

hipError_t bandchol_walk_single_launch(const WalkSys& w, int K, int64_t* d_info, hipStream_t st) {
  const size_t lds = bandchol_walk_lds_bytes(K);
  hipError_t e = set_lds_attr((const void*)walk_single_kernel, lds);
  if (e != hipSuccess) return e;
  walk_single_kernel<<<1, WALK_NT, lds, st>>>(w, K, d_info);
  return hipGetLastError();
}

hipError_t bandchol_walk_batch_factor_launch(const WalkSys* d_sys, const int* d_order, int nsys, int Kmax,
                                             unsigned* d_queue, int64_t* d_info, int grid, hipStream_t st) {
  const size_t lds = bandchol_walk_lds_bytes(Kmax);
  hipError_t e = set_lds_attr((const void*)walk_batch_kernel, lds);
  if (e != hipSuccess) return e;
  batch_clear_kernel<<<1, 64, 0, st>>>(d_queue, 1);
  walk_batch_kernel<<<grid, WALK_NT, lds, st>>>(d_sys, d_order, nsys, Kmax, d_queue, d_info);
  return hipGetLastError();
}

hipError_t bandchol_walk_batch_solve_launch(const WalkSys* d_sys, const int* d_order, int nsys, int Kmax, int nrhs,
                                            unsigned* d_queue, int grid, hipStream_t st) {
  const size_t lds = bandchol_solve_batch_lds_bytes(Kmax);
  hipError_t e = set_lds_attr((const void*)solve_batch_kernel<true>, lds);
  if (e == hipSuccess) e = set_lds_attr((const void*)solve_batch_kernel<false>, lds);
  if (e != hipSuccess) return e;
  batch_clear_kernel<<<1, 64, 0, st>>>(d_queue, 2);
  solve_batch_kernel<true><<<grid, NT, lds, st>>>(d_sys, d_order, nsys, Kmax, nrhs, d_queue);
  solve_batch_kernel<false><<<grid, NT, lds, st>>>(d_sys, d_order, nsys, Kmax, nrhs, d_queue + 1);
  return hipGetLastError();
}
