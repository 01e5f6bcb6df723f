// Shared between the adjoint kernel (adjoint.hip) and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bandchol_adj {

// One system: lambda and x are n x nrhs column-major; gab is the band gradient
// in the LAPACK lower layout with leading dimension ldg >= k+1.  (The batched
// kernel takes nrhs as an argument and ignores the field.)
struct AdjSys {
  const double* lam;
  const double* x;
  double* gab;
  int64_t n, k, nrhs, ldl, ldx, ldg;
};

}  // namespace bandchol_adj

hipError_t bandchol_outer_grad_launch(const bandchol_adj::AdjSys* d_sys, int nsys, int64_t nmax, int64_t nrhs,
                                      hipStream_t st);
hipError_t bandchol_outer_grad_launch1(const bandchol_adj::AdjSys& sys, hipStream_t st);
