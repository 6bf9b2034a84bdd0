// The one-work-group blocked Jacobi eigensolver (gfx950): declared apart
// from common.h so that the product kernels' sources stay as they are.
#pragma once
#include <hip/hip_runtime.h>

namespace ttn {

// Largest order the one-work-group blocked solver takes (G, padded to
// blocks of 16, and the sub-problems of one round fit the LDS).
constexpr int JC_LDS_MAXN = 96;

// Eigen-decomposition of the symmetric n x n float64 matrix G (32 < n <=
// JC_LDS_MAXN), in place: on return the diagonal holds the eigenvalues and
// the ROWS of U (n x n) the eigenvectors, G_in = U^T diag U.  One work-group
// per matrix; the calling thread's launch group (grp()) runs its members side
// by side.  info (device int[2]): sweeps run, rotations of the first sweep.
// skip (device flag, may be null): when set the kernel returns at once.
hipError_t jacobi_eig_lds_f64(double* G, double* U, int n, int max_sweeps, double tol, int* info, hipStream_t s,
                              const int* skip);
size_t jacobi_lds_bytes(int n);

// The orders where it beats the one-work-group cyclic solver (measured on
// gfx950): those within 8 of an even number of 16-index blocks.
inline bool jacobi_lds_preferred(int n) {
  if (n <= 32 || n > JC_LDS_MAXN) return false;
  int nb = (n + 15) / 16;
  nb += nb & 1;
  return nb * 16 - n < 8;
}

}  // namespace ttn
