// Shared between the reverse mode of the factorization (factor_bwd.hip) and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bandchol_fb {

struct FbSys {
  const double* l;       // the factor, LAPACK lower band
  int64_t ldl;
  const double* lbar;    // upstream gradient of L on the band
  int64_t ldlb;
  double* abar;          // gradient of the stored band of A (may alias lbar)
  int64_t ldab;
  int64_t n, k;          // k clipped to n-1
  int64_t K;             // sub-diagonal tiles, ceil(k / T)
  double* minv;          // workspace (set by the launch): M^{-1} per diagonal tile
  double* part;          // workspace: 2 x K partial products
  unsigned* bar;         // workspace: grid barrier counter
  int* abort;            // workspace: set when a barrier wait gave up
};

}  // namespace bandchol_fb

size_t bandchol_fb_workspace(int64_t n, int64_t K);
hipError_t bandchol_fb_launch(const bandchol_fb::FbSys& s, void* ws, int grid_max, int64_t* d_status,
                              hipStream_t st);
