// Shared between the walk kernels (walk.hip) and the host runtime (bandchol.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bandchol_walk {

// Largest number of sub-diagonal tiles (K = ceil(k / T)) the single-workgroup
// walk takes: its LDS holds the diagonal tile, two inverses and K panel tiles.
constexpr int WALK_KMAX = 15;
// Right-hand sides per pass of the batched solve.
constexpr int RHS_PASS = 8;

// One system of a batch (also used for a single matrix).
struct WalkSys {
  double* ab;      // band, LAPACK lower layout
  int64_t n, k, ldab;
  double* linv;    // if not null: L(C,C)^{-T} row-major T x T per tile column (written by the factor)
  double* b;       // right-hand sides for the batched solve (n x nrhs column-major), may be null
  int64_t ldb;
};

}  // namespace bandchol_walk

size_t bandchol_walk_lds_bytes(int K);
size_t bandchol_solve_batch_lds_bytes(int Kmax);
hipError_t bandchol_walk_single_launch(const bandchol_walk::WalkSys& w, int K, int64_t* d_info, hipStream_t st);
hipError_t bandchol_walk_batch_factor_launch(const bandchol_walk::WalkSys* d_sys, const int* d_order, int nsys,
                                             int Kmax, unsigned* d_queue, int64_t* d_info, int grid, hipStream_t st);
hipError_t bandchol_walk_batch_solve_launch(const bandchol_walk::WalkSys* d_sys, const int* d_order, int nsys,
                                            int Kmax, int nrhs, unsigned* d_queue, int grid, hipStream_t st);
