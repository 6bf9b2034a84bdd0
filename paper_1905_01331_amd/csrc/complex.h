// Layout kernels of the complex-tensor network (complex.hip, gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace ttn {

// split planes from interleaved (re, im) pairs (z: 2n doubles, 16-byte
// aligned) and back
hipError_t deinterleave_f64(const double* z, double* re, double* im, size_t n, hipStream_t s);
hipError_t interleave_f64(const double* re, const double* im, double* z, size_t n, hipStream_t s);
// real embedding of the complex m x k matrix X = xr + i xi: y (2m x 2k,
// row-major) = [[xr, -xi], [xi, xr]]; products, conjugate transposes and so
// polar factors of complex matrices are those of their embeddings (m <= 32767)
hipError_t embed_complex_f64(const double* xr, const double* xi, double* y, int m, long long k, hipStream_t s);
// the complex m x k matrix whose embedding is nearest to y (2m x 2k) =
// [[P, Q], [R, S]]: xr = (P + S) / 2, xi = (R - Q) / 2 (the projection onto
// embeddings; exact on an embedding)
hipError_t unembed_complex_f64(const double* y, double* xr, double* xi, int m, long long k, hipStream_t s);

}  // namespace ttn
