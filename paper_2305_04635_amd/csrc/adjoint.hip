// Reverse mode of the band solve (gfx950, FP64).
//
// For loss = sum(w .* x) with x = A^{-1} b and A = L L^T symmetric: the
// adjoint of b is lambda = A^{-1} w (one more pair of band solves with the
// same factor), and the gradient with respect to the stored band is the
// outer product -lambda x^T folded onto the band: an entry A(i, j), i > j,
// stands for both A(i, j) and A(j, i), so
//   g(i, j) = -sum_r (lambda(i,r) x(j,r) + lambda(j,r) x(i,r)),  i > j,
//   g(i, i) = -sum_r lambda(i,r) x(i,r).
// This kernel forms g: one workgroup per band column (grid-stride), its
// threads down the column, so that the writes of a column are contiguous.
// It reads 2 n nrhs values and writes 8 n (k+1) bytes: HBM-bound.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adjoint.h"

namespace bandchol_adj {

typedef __attribute__((address_space(1))) double glb_d;

__device__ __forceinline__ void outer_grad(const AdjSys& w, int64_t nrhs) {
  const glb_d* lam = (const glb_d*)w.lam;
  const glb_d* x = (const glb_d*)w.x;
  glb_d* g = (glb_d*)w.gab;
  for (int64_t j = blockIdx.x; j < w.n; j += gridDim.x) {
    const int64_t dmax = w.k < w.n - 1 - j ? w.k : w.n - 1 - j;
    for (int64_t d = threadIdx.x; d <= dmax; d += blockDim.x) {
      const int64_t i = j + d;
      double v = 0.0;
      for (int64_t r = 0; r < nrhs; ++r) {
        v = fma(-lam[i + r * w.ldl], x[j + r * w.ldx], v);
        if (d > 0) v = fma(-lam[j + r * w.ldl], x[i + r * w.ldx], v);
      }
      g[d + j * w.ldg] = v;
    }
  }
}

// blockIdx.y + y0 = system
__global__ void __launch_bounds__(256) outer_grad_batch_kernel(const AdjSys* sys, int y0, int64_t nrhs) {
  outer_grad(sys[blockIdx.y + y0], nrhs);
}

__global__ void __launch_bounds__(256) outer_grad_kernel(AdjSys w) { outer_grad(w, w.nrhs); }

}  // namespace bandchol_adj

static unsigned columns_grid(int64_t n) { return (unsigned)(n < 8192 ? (n > 0 ? n : 1) : 8192); }

hipError_t bandchol_outer_grad_launch(const bandchol_adj::AdjSys* d_sys, int nsys, int64_t nmax, int64_t nrhs,
                                      hipStream_t st) {
  if (nsys <= 0 || nmax <= 0) return hipSuccess;
  for (int y0 = 0; y0 < nsys; y0 += 65535) {
    const int ny = nsys - y0 < 65535 ? nsys - y0 : 65535;
    bandchol_adj::outer_grad_batch_kernel<<<dim3(columns_grid(nmax), (unsigned)ny), 256, 0, st>>>(d_sys, y0, nrhs);
  }
  return hipGetLastError();
}

hipError_t bandchol_outer_grad_launch1(const bandchol_adj::AdjSys& sys, hipStream_t st) {
  if (sys.n <= 0) return hipSuccess;
  bandchol_adj::outer_grad_kernel<<<columns_grid(sys.n), 256, 0, st>>>(sys);
  return hipGetLastError();
}
