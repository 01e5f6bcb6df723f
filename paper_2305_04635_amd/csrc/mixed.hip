// Kernels of the mixed-precision solver (gfx950): band precision conversions,
// the FP64 residual R = B - A X of the symmetric band, column max-norms and
// the correction update.  The FP32 factor itself is the spine schedule of
// factor2.hip instantiated for float; the correction solves are the FP64 band
// solves run on the FP32 factor widened to FP64.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mixed.h"

namespace bandchol_mixed {

typedef __attribute__((address_space(1))) double glb_d;
typedef __attribute__((address_space(1))) float glb_f;

constexpr int RB = 64;   // rows per workgroup of the residual kernel
constexpr int RP = 8;    // right-hand sides per pass

// Band (k+1) x n, leading dimensions lds/ldd, element by element.
template <typename S, typename D>
__global__ void __launch_bounds__(256) convert_kernel(int64_t n, int64_t k, const S* src, int64_t lds, D* dst,
                                                      int64_t ldd) {
  const int64_t rows = k + 1;
  const int64_t total = rows * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / rows, d = e - j * rows;
    dst[d + j * ldd] = (D)src[d + j * lds];
  }
}

// out(i, r) = b(i, r) - sum_j A(i, j) x(j, r)  (mode 0), or out(i, 0) = sum_j |A(i, j)| (mode 1),
// for rows i in [RB * blockIdx.x, RB * blockIdx.x + RB), right-hand sides [r0, r0 + RP).
// Lane = row.  Waves split the columns: the lower part (j <= i, stored in
// column j at row offset i - j: one contiguous segment per column for the 64
// rows) and the strict upper part (j > i, A(i, j) = A(j, i), stored in
// column i).  Partial sums meet in LDS in a fixed order.
__global__ void __launch_bounds__(256) residual_kernel(int64_t n, int64_t k, const double* ab_, int64_t ldab,
                                                       const double* x_, int64_t ldx, const double* b_, int64_t ldb,
                                                       double* out_, int64_t ldo, int64_t nrhs, int mode) {
  __shared__ double part[4][RB][RP];
  const glb_d* ab = (const glb_d*)ab_;
  const glb_d* x = (const glb_d*)x_;
  const glb_d* b = (const glb_d*)b_;
  glb_d* out = (glb_d*)out_;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * RB;
  const int64_t i = i0 + lane;
  const bool row_ok = i < n;
  for (int64_t r0 = 0; r0 < (mode == 0 ? nrhs : 1); r0 += RP) {
    const int nr = mode == 0 ? (int)(nrhs - r0 < RP ? nrhs - r0 : RP) : 1;
    double acc[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) acc[r] = 0.0;
    // lower part and diagonal: columns j in [i0 - k, i0 + RB)
    const int64_t jlo = i0 - k > 0 ? i0 - k : 0;
    for (int64_t j = jlo + wave; j < i0 + RB && j < n; j += 4) {
      const int64_t d = i - j;
      const double a = (row_ok && d >= 0 && d <= k) ? ab[d + j * ldab] : 0.0;
      if (mode == 1) {
        acc[0] += fabs(a);
      } else {
#pragma unroll
        for (int r = 0; r < RP; ++r)
          if (r < nr) acc[r] = fma(a, x[j + (r0 + r) * ldx], acc[r]);
      }
    }
    // strict upper part: A(i, i + d) = ab[d + i * ldab], d = 1..k
    for (int64_t d = 1 + wave; d <= k; d += 4) {
      const bool in = row_ok && i + d < n;
      const double a = in ? ab[d + i * ldab] : 0.0;
      if (mode == 1) {
        acc[0] += fabs(a);
      } else {
#pragma unroll
        for (int r = 0; r < RP; ++r)
          if (r < nr) acc[r] = fma(a, in ? x[i + d + (r0 + r) * ldx] : 0.0, acc[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < RP; ++r) part[wave][lane][r] = acc[r];
    __syncthreads();
    if (wave == 0 && row_ok) {
      for (int r = 0; r < nr; ++r) {
        const double s = ((part[0][lane][r] + part[1][lane][r]) + part[2][lane][r]) + part[3][lane][r];
        out[i + (r0 + r) * ldo] = mode == 1 ? s : b[i + (r0 + r) * ldb] - s;
      }
    }
    __syncthreads();
  }
}

// maxabs[c] = max_i |v(i, c)| for c < ncol, as the IEEE bit pattern of a
// non-negative double (whose integer order is the numeric order); NaN sorts
// above every number.  maxabs must start at zero.
__global__ void __launch_bounds__(256) colmax_kernel(int64_t n, int64_t ncol, const double* v, int64_t ldv,
                                                     unsigned long long* maxabs) {
  const int64_t c = blockIdx.y;
  unsigned long long m = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(fabs(v[i + c * ldv]));
    m = u > m ? u : m;
  }
  // wave maximum, then one atomic per wave
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_down(m, off, 64);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0 && m) atomicMax(maxabs + c, m);
}

__global__ void fill_u64_kernel(unsigned long long* p, int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = 0;
}

// x(:, c) += d(:, c)
__global__ void __launch_bounds__(256) axpy_kernel(int64_t n, int64_t ncol, double* x, int64_t ldx, const double* d,
                                                   int64_t ldd) {
  const int64_t c = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i + c * ldx] += d[i + c * ldd];
}

static unsigned grid_for(int64_t work, int64_t per) {
  int64_t g = (work + per - 1) / per;
  return (unsigned)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace bandchol_mixed

using namespace bandchol_mixed;

hipError_t bandchol_band_to_f32(int64_t n, int64_t k, const double* src, int64_t lds, float* dst, int64_t ldd,
                                hipStream_t st) {
  convert_kernel<double, float><<<grid_for((k + 1) * n, 1024), 256, 0, st>>>(n, k, src, lds, dst, ldd);
  return hipGetLastError();
}

hipError_t bandchol_band_to_f64(int64_t n, int64_t k, const float* src, int64_t lds, double* dst, int64_t ldd,
                                hipStream_t st) {
  convert_kernel<float, double><<<grid_for((k + 1) * n, 1024), 256, 0, st>>>(n, k, src, lds, dst, ldd);
  return hipGetLastError();
}

hipError_t bandchol_residual(int64_t n, int64_t k, const double* ab, int64_t ldab, const double* x, int64_t ldx,
                             const double* b, int64_t ldb, double* out, int64_t ldo, int64_t nrhs, int mode,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  residual_kernel<<<(unsigned)((n + RB - 1) / RB), 256, 0, st>>>(n, k, ab, ldab, x, ldx, b, ldb, out, ldo, nrhs,
                                                                 mode);
  return hipGetLastError();
}

hipError_t bandchol_colmax(int64_t n, int64_t ncol, const double* v, int64_t ldv, unsigned long long* maxabs,
                           hipStream_t st) {
  fill_u64_kernel<<<grid_for(ncol, 64), 64, 0, st>>>(maxabs, ncol);
  if (n > 0 && ncol > 0) colmax_kernel<<<dim3(grid_for(n, 2048), (unsigned)ncol), 256, 0, st>>>(n, ncol, v, ldv, maxabs);
  return hipGetLastError();
}

hipError_t bandchol_axpy(int64_t n, int64_t ncol, double* x, int64_t ldx, const double* d, int64_t ldd,
                         hipStream_t st) {
  if (n > 0 && ncol > 0) axpy_kernel<<<dim3(grid_for(n, 2048), (unsigned)ncol), 256, 0, st>>>(n, ncol, x, ldx, d, ldd);
  return hipGetLastError();
}
