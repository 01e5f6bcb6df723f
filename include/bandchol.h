/*
 * bandchol: FP64 Cholesky factorization of symmetric positive-definite band
 * matrices and the band solves that use the factor, on AMD MI355X (gfx950).
 *
 * Method: A = L L^T with L lower triangular, positive diagonal, and the lower
 * bandwidth k of A.  The factor is unique (Section 2 of Liu, Fredriksson and
 * Markidis, "Parallel Cholesky Factorization for Banded Matrices using
 * OpenMP Tasks", arXiv 2305.04635).  The GPU walks the band in square tiles:
 * each diagonal tile is factored (dense Cholesky), the tiles below it are
 * solved against it (triangular solve), and the tiles further right receive
 * the rank-nb updates (the potrf / trsm / gemm / syrk steps of Algorithm 1,
 * Section 3).  Flop count used for rates: n(k^2 + 3k) (Section 3.2).
 *
 * Storage (all routines): LAPACK lower band layout, column-major,
 *   A(i, j) for 0 <= i - j <= k  at  ab[(i - j) + j * ldab],  ldab >= k + 1
 * (the paper keeps the standard LAPACK band format, Sections 3 and 6).  Rows
 * k+1 .. ldab-1 of every column and the positions past row n-1 in the last k
 * columns are never read or written.  Indices are 0-based; info is 1-based.
 *
 * Pointers: every array argument is a DEVICE pointer on the current HIP
 * device, allocated and owned by the caller.  The library never frees caller
 * memory.  It owns one workspace per device (grown on demand with hipMalloc,
 * released by bandchol_finalize); a call that needs a larger workspace than
 * the one held must therefore not run under stream capture, and growing it
 * frees the old one, which a graph captured earlier may still name: capture
 * only after a call of the same or a larger size has run, and recapture after
 * a larger call or after bandchol_finalize.
 *
 * Concurrency: the single-matrix calls (factor, solve, their _async forms, the
 * FP32 factor, the mixed solve, the solve backward) share that workspace --
 * ticket counters, flags and publication buffers -- and one status slot per
 * device.  Two such calls on one device must not overlap in time, whether
 * issued on different streams or from different threads: order them on one
 * stream or synchronise between them.  Batch plans own their memory and do
 * not share it.
 *
 * Streams: the synchronous calls run on the stream set with
 * bandchol_set_stream for the calling thread (default: the null stream) and
 * wait for it.  The _async calls run on the stream passed in and do not wait.
 *
 * Errors: 0 = success; -i = the i-th argument is illegal (checked before any
 * GPU work); BANDCHOL_EHIP = a HIP runtime error (bandchol_last_error() gives
 * its text); BANDCHOL_EHANG = a device-side wait exceeded its bound (the
 * kernel exited instead of hanging; results unspecified).
 *
 * Inputs must be finite except for NaN, which is reported: a NaN anywhere in
 * the band makes info point at the first pivot it reaches.
 */
#ifndef BANDCHOL_H
#define BANDCHOL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BANDCHOL_EHIP (-1000)
#define BANDCHOL_EHANG (-1001)
#define BANDCHOL_ETOOBIG (-1002)

/*
 * Factor A = L L^T in place (LAPACK pbtrf, uplo = 'L').
 *   n     order of A, n >= 0                                   (bad: -1)
 *   k     number of sub-diagonals, k >= 0; k >= n-1 is the dense case (bad: -2)
 *   ab    device pointer to the band, ldab x n column-major    (NULL with n > 0: -3)
 *   ldab  leading dimension, ldab >= k + 1                     (bad: -4)
 * Returns 0 on success, < 0 on a bad argument or runtime error, or info > 0:
 * the 1-based index of the first column whose pivot A(j,j) - sum_l L(j,l)^2
 * is not positive (zero, negative or NaN), i.e. the leading minor of that
 * order is not positive definite.  After info > 0 the contents of ab are
 * unspecified.  Synchronous: waits for the stream and reads info back.
 */
int64_t bandchol_factor(int64_t n, int64_t k, double* ab, int64_t ldab);

/*
 * Solve A X = B with the factor from bandchol_factor (LAPACK pbtrs, uplo =
 * 'L'): forward L Y = B, then back L^T X = Y.
 *   n -1, k -2, nrhs >= 0 -3, ab (factor) -4, ldab >= k+1 -5,
 *   b device pointer, n x nrhs column-major -6, ldb >= max(1, n) -7.
 * B is overwritten by X.  The factor is not inspected for zero pivots: call
 * only after bandchol_factor returned 0.  Synchronous.  Returns
 * BANDCHOL_EHANG (B then unspecified) when a wait between the solve's
 * workgroups exceeded its bound.
 */
int64_t bandchol_solve(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, double* b,
                       int64_t ldb);

/*
 * Stream-ordered forms.  No host synchronisation.  bandchol_factor_async
 * writes info (as above; 0 on success) to *d_info, a device int64.  Argument
 * codes are returned immediately.  stream is a hipStream_t (NULL = null stream).
 * bandchol_solve_async has no status output: a wait that exceeded its bound
 * (reported as BANDCHOL_EHANG by bandchol_solve) leaves B unspecified.
 */
int64_t bandchol_factor_async(int64_t n, int64_t k, double* ab, int64_t ldab, int64_t* d_info,
                              void* stream);
int64_t bandchol_solve_async(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab,
                             double* b, int64_t ldb, void* stream);

/*
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the factor of
 * bandchol_factor_async (same arguments, same result bit for bit, same
 * schedule) that allocates nothing.  Its working memory (ticket counter,
 * flags, tile inverses and pre-accumulated tiles of the multi-workgroup
 * schedule) lives in a fixed device array of 128 MiB that every GPU the
 * library runs on holds from module load until the process ends; the call
 * makes no hipMalloc, hipFree or other allocating call.  It needs
 *   256 + 256 * ceil(4 (NB (K + 1) + 2 NB) / 256) + 32768 NB bytes,
 *   NB = ceil(n / 32), K = ceil(min(k, n-1) / 32),
 * which fits for n up to about 130000 at any k <= 2000; a larger band returns
 * BANDCHOL_ETOOBIG (nothing launched; bandchol_last_error() gives the sizes).
 * Every call on a GPU shares that GPU's array and leaves its contents behind
 * (the kernels clear what must start at zero): calls that overlap in time on
 * one GPU -- on different streams or from different threads -- race.  The
 * first call on each device looks the array's address up (with that device
 * current).  Argument codes and d_info as bandchol_factor_async.
 */
int64_t bandchol_factor_noalloc(int64_t n, int64_t k, double* ab, int64_t ldab, int64_t* d_info,
                                void* stream);

/* Stream used by the synchronous calls of the calling thread (hipStream_t). */
int64_t bandchol_set_stream(void* stream);

/* Text of the last error in the calling thread ("" if none). */
const char* bandchol_last_error(void);

/* Release the per-device workspaces. */
void bandchol_finalize(void);

/* Tile width the factor uses (the rank of each trailing update). */
int64_t bandchol_tile(void);

/*
 * Tuning: single matrices whose band spans at most `kmax` sub-diagonal tiles
 * (k <= kmax * bandchol_tile()) are factored by one workgroup walking the band;
 * wider bands use the multi-workgroup tile schedule.  kmax is clamped to
 * [0, 15]; the default is 0 (only diagonal matrices walk).  Returns the
 * previous limit; a negative kmax only queries it.  Process-wide; not
 * synchronised with calls running in other threads.  Batch plans always walk
 * systems of up to 15 tile diagonals.
 */
int64_t bandchol_set_walk_limit(int64_t kmax);

/*
 * Latency of one step of the factor's pivot chain on the current device, in
 * nanoseconds: one wave runs `steps` dependent steps of the reciprocal of a
 * pivot (hardware estimate refined by two Newton steps, as the factor takes
 * it) followed by the fused multiply-add that forms the next pivot, timed by
 * the GPU's 100 MHz real-time counter.  A single band's factorization has n
 * such steps one after another, so n times this is a floor for its time at
 * any bandwidth.  1 <= steps <= 2^32 (-1), ns_per_step a host pointer (-2).
 * Synchronous on the stream of bandchol_set_stream; allocates 256 bytes of
 * device memory for the call.
 */
int64_t bandchol_pivot_chain_ns(int64_t steps, double* ns_per_step);

/*
 * Where the time of the diagonal chain goes: factors an (n, k) band (generated
 * on the device as for bandchol_tune_factor) `reps` times with the
 * multi-workgroup schedule (the workgroup count the factor would use, its
 * rule where that is the walk) and the spine's phase times recorded (shader
 * clock, s_memtime), and writes out[0..12]: per step of 32 columns, the cycles
 * of wave 0's diagonal-tile sweep (0), its wait for waves 1-3 at the end of
 * phase A (1), its work in phase BC (the stores of L(C,C) and its inverse,
 * while waves 1-3 finish the next diagonal tile) (2) and its wait for them
 * at the end of that phase (3); for waves 1, 2, 3 the cycles of their
 * phase-A work and of their wait at its end (4..9); the number of steps
 * (10); the last factor's time in ms (11); its workgroup count (12).  n >= 2
 * (-1), k >= 1 (-2), 1 <= reps <= 100 (-3), out with cap >= 13 (-4).
 * Allocates the test band; synchronous; not under stream capture.
 */
int64_t bandchol_spine_profile(int64_t n, int64_t k, int64_t reps, double* out, int64_t cap);

/*
 * Schedule per (n, k) bucket.  The paper picks the dimension of its block
 * grid per problem with a heuristic (block size near 50, no more blocks than
 * cores) and lets users who know their bandwidths and hardware tune it
 * (Section 3, end of the method's overview).  Here the tile is fixed by the
 * matrix instruction and the choice is the number of workgroups that factor
 * one matrix:
 * 1 = the single-workgroup walk, w >= 2 = the tile schedule with w
 * workgroups (one carries the diagonal chain, the rest take tile tasks).
 * Buckets are (floor(log2 n), K) with K = ceil(min(k, n-1) / bandchol_tile()).
 * The factor (FP64, FP32, and the wide systems of batch plans when the plan is
 * created) takes, in this order: the walk for K up to the walk limit
 * (bandchol_set_walk_limit; by default K = 0 only), the table entry of the
 * bucket, else the rule w = CUs/4 for K <= 11, CUs for
 * K <= 55, 2 x CUs above (at least 2).  The FP32 factor has no walk and takes
 * the rule where the choice is 1.  The table is process-wide and guarded by a mutex; it starts empty.
 *
 * bandchol_schedule: the workgroup count the factor of (n, k) would use now,
 * 0 for n = 0; -1 / -2 for a bad n / k.  No GPU work.
 *
 * bandchol_tune_set: record w for the bucket of (n, k), replacing an entry;
 * w = 0 removes the bucket's entry.  Returns -1 / -2 for a bad n / k, -3 when
 * w < 0, w > 2 x CUs, w = 1 with K > 15 (the walk's limit) or w > 1 with
 * K = 0.  No GPU work.
 *
 * bandchol_tune_entries: copies up to `cap` entries (arrays of `cap`
 * elements: the n and k each was recorded for, its w, and its measured
 * median factor time in ms, 0 when set by the caller) and returns the number
 * of entries; cap = 0 only counts (NULL arrays allowed).  -1 when cap < 0,
 * -2 .. -5 for a NULL array with cap > 0.
 *
 * bandchol_tune_clear: empties the table.
 *
 * bandchol_tune_factor: measures the factor of an (n, k) band on the current
 * device, on the stream set for the calling thread, and records the fastest
 * schedule for its bucket.  The test matrix is generated on the device
 * (off-diagonal entries uniform in [-1, 1) from a hash of their position,
 * diagonal 2k + 2: diagonally dominant, so SPD).  Candidates: the walk when
 * K <= 15, and (for K >= 1) 32, 64, 96, 128, 192, 256, 320, 384, 448, 512 ...
 * up to 2 x CUs workgroups plus the rule's count.  Each candidate runs once
 * untimed (dropped when it takes more than twice the best median so far),
 * then `reps` timed runs (1 <= reps <= 1000; events around the factor on the
 * stream); the lowest median wins (ties: the earlier candidate).  Writes the
 * winner and its median (ms) to *wgs_out / *ms_out when not NULL.  Allocates
 * the test band (8 (k+1) n bytes) with hipMalloc and frees it before
 * returning: not for use under stream capture.  Synchronous.  Returns -1 / -2
 * / -3 for a bad n / k / reps, BANDCHOL_EHIP on a HIP error or if a
 * factor fails (the table is then unchanged).  The BANDCHOL_MAX_WG
 * environment cap, when set, applies to the candidates too.
 */
int64_t bandchol_schedule(int64_t n, int64_t k);
int64_t bandchol_tune_set(int64_t n, int64_t k, int64_t wgs);
int64_t bandchol_tune_entries(int64_t cap, int64_t* n, int64_t* k, int64_t* wgs, double* ms);
void bandchol_tune_clear(void);
int64_t bandchol_tune_factor(int64_t n, int64_t k, int64_t reps, int64_t* wgs_out, double* ms_out);

/*
 * FP32 factor: the same factorization in single precision (the trailing
 * products on v_mfma_f32_16x16x4f32, FP32 accumulation), in place on a float
 * band in the same layout.  Arguments and info as bandchol_factor_async
 * (d_info: device int64; -5 when NULL).  Stream-ordered.
 */
int64_t bandchol_factor_f32(int64_t n, int64_t k, float* ab, int64_t ldab, int64_t* d_info, void* stream);

/*
 * Mixed-precision solve of A X = B: factor fl32(A) in FP32, then refine in
 * FP64 (Buttari, Dongarra et al. 2007; LAPACK dsposv): x0 from the FP32
 * factor, then repeat r = b - A x (FP64), d = A32^{-1} r (the FP32 factor
 * widened to FP64), x += d, until every column has
 * ||r||_inf <= sqrt(n) * 2^-53 * ||A||_inf * ||x||_inf.  Falls back to the
 * FP64 factor and solve when the FP32 factor fails (fallback = 1), after 30
 * corrections (2), or when a correction is not at most half the previous one
 * in some column (3); 0 = no fallback.
 *   ab (device, read only) -4 / ldab >= k+1 -5; b (device, n x nrhs) -6 /
 *   ldb >= max(1,n) -7; x (device, n x nrhs, written) -8 / ldx -9; n -1, k -2,
 *   nrhs -3.  iters, fallback: host pointers or NULL.
 * Returns 0, or the info of the FP64 factor (> 0) if the fallback factor fails
 * too, or BANDCHOL_EHANG (x unspecified) when a wait inside one of its band
 * solves exceeded its bound.  Uses internal buffers of about 12 (k+1) n + 8 n nrhs bytes.
 * Synchronous on the stream of bandchol_set_stream.
 */
int64_t bandchol_mixed_solve(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, const double* b,
                             int64_t ldb, double* x, int64_t ldx, int64_t* iters, int64_t* fallback);

/*
 * Reverse mode of the solve, for a loss that depends on x = A^{-1} B through
 * an upstream gradient G = dloss/dX (n x nrhs): the gradient with respect to B
 * is A^{-1} G (A is symmetric), computed with two more band solves on the
 * factor, and the gradient with respect to the stored band of A is
 * -A^{-1} G X^T folded onto the band, since a stored entry A(i, j), i > j,
 * stands for both A(i, j) and A(j, i):
 *   gab(i, j) = -sum_r (lambda(i,r) x(j,r) + lambda(j,r) x(i,r)),  i > j,
 *   gab(i, i) = -sum_r lambda(i,r) x(i,r),       lambda = A^{-1} G.
 * (This is the transpose rule of the linear solve; the paper covers only the
 * forward factorization.)
 *   n -1, k -2, nrhs -3, ab = factor from bandchol_factor -4, ldab >= k+1 -5,
 *   x = solution (device, n x nrhs) -6, ldx >= max(1,n) -7,
 *   g = upstream gradient (device, n x nrhs), overwritten by A^{-1} G -8,
 *   ldg >= max(1,n) -9, gab = band gradient (device, written) -10,
 *   ldgab >= k+1 -11.  Stream-ordered on `stream`; no host synchronisation.
 */
int64_t bandchol_solve_backward(int64_t n, int64_t k, int64_t nrhs, const double* ab, int64_t ldab, const double* x,
                                int64_t ldx, double* g, int64_t ldg, double* gab, int64_t ldgab, void* stream);

/*
 * Reverse mode of the factorization, for a loss that depends on the factor L
 * of A = L L^T through an upstream gradient Lbar = dloss/dL (lower band):
 * the gradient Abar = dloss/dA with respect to the stored band entries A(i, j),
 * i >= j, i.e. the entries the factorization reads (a stored entry below the
 * diagonal stands for both A(i, j) and A(j, i)).  With M = L, for the dense
 * matrix this is Abar(i, j) = S(i, j) + S(j, i) (i > j), Abar(i, i) = S(i, i),
 * S = L^{-T} Phi(L^T Lbar) L^{-1}, Phi = lower triangle with half the
 * diagonal; it is computed tile by tile on the band only, reversing the
 * potrf / trsm / gemm / syrk steps of Algorithm 1 (Section 3) in reverse
 * order.  (The paper covers only the forward factorization.)
 *   n -1, k -2, l = the factor from bandchol_factor (device) -3, ldl >= k+1 -4,
 *   lbar (device, band layout, rows 0..k read) -5, ldlb >= k+1 -6,
 *   abar (device, band layout, rows 0..k written; may be the same array as
 *   lbar with ldab = ldlb) -7, ldab >= k+1 -8.
 * d_status: device int64 or NULL; receives 0, or BANDCHOL_EHANG when a wait
 * between the kernel's workgroups exceeded its bound (abar then unspecified).
 * Stream-ordered on `stream`; uses the library's workspace (about 8 T^2 bytes
 * per tile of n plus 16 T^2 per tile of k, T = bandchol_tile()).
 */
int64_t bandchol_factor_backward(int64_t n, int64_t k, const double* l, int64_t ldl, const double* lbar,
                                 int64_t ldlb, double* abar, int64_t ldab, int64_t* d_status, void* stream);

/*
 * Batches of independent systems of different orders and bandwidths.  The
 * paper's method factors one band at a time; a single band only offers the
 * parallelism of its own tile columns (the paper's evaluation finds its small
 * bandwidths far from the machine's peak, Section 5, and its conclusions point
 * at the little parallelism narrow bands offer, Section 7), so many independent
 * systems are run at once: one
 * workgroup per system, every workgroup taking the next system from an atomic
 * counter, longest first (the estimate is (n / T) * (10 + K^2) with K the
 * number of sub-diagonal tiles).  Systems with more than 15 sub-diagonal
 * tiles (k > 480) are factored one after another with the multi-workgroup
 * schedule instead.
 *
 * bandchol_batch_create builds a plan.  All array arguments are HOST arrays of
 * length `batch`; ab[i] and b[i] are DEVICE pointers owned by the caller and
 * must stay valid while the plan is used:
 *   batch >= 0 (-1); n[i] >= 0 (-2); k[i] >= 0 (-3); ab[i] != NULL when
 *   n[i] > 0 (-4); ldab[i] >= k[i] + 1 (-5); b may be NULL (no solves),
 *   else b[i] != NULL when n[i] > 0 (-6) and ldb[i] >= max(1, n[i]) (-7);
 *   plan != NULL (-8).
 * It allocates device memory (descriptors and the inverses of all diagonal
 * tiles, 8 T^2 bytes per tile column of every system) on the current device,
 * synchronously.  The factor and solve calls below allocate nothing and only
 * launch kernels on `stream`, so they may be captured into a HIP graph and
 * replayed; the plan must be destroyed only after its work has finished.
 *
 * bandchol_batch_factor factors every system in place and writes info per
 * system (as for bandchol_factor) to d_info[0 .. batch-1], a DEVICE int64
 * array.  bandchol_batch_solve(nrhs) overwrites b[i] (n[i] x nrhs,
 * column-major) with the solution, using the factors and the inverses of the
 * diagonal tiles left by the last bandchol_batch_factor on the same plan; call
 * it only for systems whose info was 0.  Returns -1 for nrhs < 0, -2 when
 * the plan has no right-hand sides.
 */
typedef struct bandchol_batch* bandchol_batch_t;

int64_t bandchol_batch_create(int64_t batch, const int64_t* n, const int64_t* k, double* const* ab,
                              const int64_t* ldab, double* const* b, const int64_t* ldb, bandchol_batch_t* plan);
int64_t bandchol_batch_factor(bandchol_batch_t plan, int64_t* d_info, void* stream);
int64_t bandchol_batch_solve(bandchol_batch_t plan, int64_t nrhs, void* stream);
/*
 * Reverse mode for a whole batch (as bandchol_solve_backward per system).
 * bandchol_batch_set_adjoint registers, per system, the upstream gradient
 * g[i] (device, n[i] x nrhs, overwritten by A^{-1} G) and the band gradient
 * gab[i] (device, leading dimension ldgab[i] >= k[i]+1): HOST arrays of
 * length batch; it allocates and uploads descriptors synchronously (-1 plan
 * NULL or created without right-hand sides, -2 g, -3 gab, -4 ldgab).
 * bandchol_batch_backward(nrhs) then only launches kernels on `stream`
 * (capturable), using the factors and inverses of the last
 * bandchol_batch_factor and the solutions X left in b by bandchol_batch_solve
 * (-1 plan NULL or no adjoint buffers, -2 nrhs).
 */
int64_t bandchol_batch_set_adjoint(bandchol_batch_t plan, double* const* g, double* const* gab,
                                   const int64_t* ldgab);
int64_t bandchol_batch_backward(bandchol_batch_t plan, int64_t nrhs, void* stream);

/* Frees the plan's device memory (waits for the device first). */
void bandchol_batch_destroy(bandchol_batch_t plan);

/*
 * Schedule per (n, k) bucket for the systems of batch plans (the tuning of the
 * batched path).  Buckets as for bandchol_schedule.  In a batch, the systems
 * the walk takes run side by side in one persistent launch, one workgroup
 * each, while a system given w >= 2 workgroups is factored on its own with the
 * multi-workgroup schedule after that launch; so the best choice for a
 * bucket depends on the batch, and this table is kept apart from the
 * single-matrix one.  A plan reads it when it is created: the bucket's entry
 * if there is one, else the walk for K <= 15 and the single-matrix choice
 * above (its rule where that choice is the walk).  The tile is T =
 * bandchol_tile() for every choice: it is set by the 16 x 16 x 4 FP64 matrix
 * instruction and the LDS the walk keeps per tile diagonal, not tuned.
 *
 * bandchol_batch_tune_set / _entries / _clear: as bandchol_tune_set /
 * _entries / _clear, on this table.
 *
 * bandchol_batch_tune: measures, on the current device and the stream of
 * bandchol_set_stream, the batched factor of systems of the given orders and
 * bandwidths (HOST arrays of length batch; test bands generated on the
 * device as for bandchol_tune_factor, 8 (k+1) n bytes each, allocated and
 * freed by the call: not under stream capture).  Starting from the current
 * table it takes the buckets in decreasing order of the walk's work estimate
 * (n / T)(10 + K^2) summed over their systems, up to max_buckets of them,
 * tries the other schedule for each (the multi-workgroup schedule with the
 * rule's count where the bucket walks, the walk where it does not and K <=
 * 15), and keeps it when the batch factor's median time over `reps` runs
 * drops by more than 1 %; every bucket tried gets an entry with the choice
 * kept.  *ms_out (may be NULL): the final median in ms.  Returns -1 batch < 1,
 * -2 n (NULL or an n < 1), -3 k, -4 reps outside 1..1000, -5 max_buckets < 0,
 * BANDCHOL_EHIP on a HIP error or a failed factor.  Synchronous.
 */
int64_t bandchol_batch_tune_set(int64_t n, int64_t k, int64_t wgs);
int64_t bandchol_batch_tune_entries(int64_t cap, int64_t* n, int64_t* k, int64_t* wgs, double* ms);
void bandchol_batch_tune_clear(void);
int64_t bandchol_batch_tune(int64_t batch, const int64_t* n, const int64_t* k, int64_t reps, int64_t max_buckets,
                            double* ms_out);

#ifdef __cplusplus
}
#endif

#endif /* BANDCHOL_H */
