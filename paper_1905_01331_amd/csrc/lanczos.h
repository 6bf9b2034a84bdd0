#pragma once
#include "common.h"

namespace ttn {
hipError_t lz_three_term(double* w, const double* qj, const double* qjm1, const double* alpha, const double* beta, int j,
                         size_t n, const int* stop, hipStream_t s);
hipError_t lz_set_beta(const double* ss, const double* hss, double* beta, int j, double tol, int* stop, int* m_eff,
                       hipStream_t s);
hipError_t lz_next_q(const double* w, double* qn, const double* beta, int j, size_t n, const int* stop, hipStream_t s);
hipError_t lz_build_T(const double* alpha, const double* beta, int m, const int* stop, const int* m_eff, double* T,
                      hipStream_t s);
hipError_t lz_select_lowest(const double* T, const double* V, int m, double* y, double* theta, hipStream_t s);
hipError_t scale_rsqrt(double* x, const double* ss, size_t n, hipStream_t s);
hipError_t residual_vec(const double* Hv, const double* v, const double* lam, double* r, size_t n, hipStream_t s);
hipError_t sign_fix(double* v, size_t n, hipStream_t s);
hipError_t axpy_dev(double* y, const double* x, const double* scale, double factor, size_t n, hipStream_t s);
hipError_t sqrt_inplace(double* x, hipStream_t s);
// out[0] = lam[0], out[1] = (lam[0] + c[0] L) / (L ly)  (c: the shift, on the device)
hipError_t energy_store(const double* lam, const double* c, double L, double ly, double* out, hipStream_t s);
hipError_t ratio_minmax(const double* nrm, int m, double* out, double* run_min, hipStream_t s);
hipError_t running_max(const double* x, double* run_max, hipStream_t s);
hipError_t identity_f64(double* X, int n, hipStream_t s);
hipError_t zero_int(int* x, int n, hipStream_t s);
// Full reorthogonalisation pass against the first nq rows of Q (row length n):
// coef[i] = Q[i].w (i < nq), coef[nq] = w.w (before the update), then
// w -= sum_i coef[i] Q[i].  `part` holds lz_reorth_part_doubles() doubles.
hipError_t lz_reorth(double* w, const double* Q, int nq, size_t n, double* coef, double* part, hipStream_t s);
size_t lz_reorth_part_doubles();
hipError_t lz_alpha(const double* c1, const double* c2, int j, double* alpha, hipStream_t s);
// X <- (X + sign X^T) / 2 in place (sign = +1 symmetric, -1 antisymmetric part)
hipError_t symmetrize_f64(double* X, int n, double sign, hipStream_t s);
}  // namespace ttn
