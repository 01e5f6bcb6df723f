// Kernels of the mixed-precision solver (mixed.hip), called by the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// dst (band, ldd) = src (band, lds), converted element by element.
hipError_t bandchol_band_to_f32(int64_t n, int64_t k, const double* src, int64_t lds, float* dst, int64_t ldd,
                                hipStream_t st);
hipError_t bandchol_band_to_f64(int64_t n, int64_t k, const float* src, int64_t lds, double* dst, int64_t ldd,
                                hipStream_t st);
// mode 0: out = b - A x (n x nrhs); mode 1: out(:, 0) = row sums of |A|.  A symmetric, lower band.
hipError_t bandchol_residual(int64_t n, int64_t k, const double* ab, int64_t ldab, const double* x, int64_t ldx,
                             const double* b, int64_t ldb, double* out, int64_t ldo, int64_t nrhs, int mode,
                             hipStream_t st);
// maxabs[c] = bit pattern of max_i |v(i, c)| (device, ncol entries).
hipError_t bandchol_colmax(int64_t n, int64_t ncol, const double* v, int64_t ldv, unsigned long long* maxabs,
                           hipStream_t st);
// x += d, n x ncol.
hipError_t bandchol_axpy(int64_t n, int64_t ncol, double* x, int64_t ldx, const double* d, int64_t ldd,
                         hipStream_t st);
