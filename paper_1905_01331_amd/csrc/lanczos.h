#pragma once
#include "common.h"

namespace ttn {
hipError_t lz_build_T(const double* alpha, const double* beta, int m, const int* stop, const int* m_eff, double* T,
                      hipStream_t s);
hipError_t lz_select_lowest(const double* T, const double* V, int m, double* y, double* theta, hipStream_t s);
hipError_t scale_rsqrt(double* x, const double* ss, size_t n, hipStream_t s);
hipError_t residual_vec(const double* Hv, const double* v, const double* lam, double* r, size_t n, hipStream_t s);
hipError_t sign_fix(double* v, size_t n, hipStream_t s);
hipError_t axpy_dev(double* y, const double* x, const double* scale, double factor, size_t n, hipStream_t s);
hipError_t sqrt_inplace(double* x, hipStream_t s);
// out[0] = lam[0], out[1] = (lam[0] + c[0] L) / (L ly)  (c: the shift, on the device)
// out[0] = lambda, out[1] = (lambda + c L) / (L ly); the previous out[1]
// goes to prev[0] (prev may be null)
hipError_t energy_store(const double* lam, const double* c, double L, double ly, double* out, double* prev,
                        hipStream_t s);
hipError_t ratio_minmax(const double* nrm, int m, double* out, double* run_min, hipStream_t s);
hipError_t running_max(const double* x, double* run_max, hipStream_t s);
hipError_t identity_f64(double* X, int n, hipStream_t s);
hipError_t zero_int(int* x, int n, hipStream_t s);
// p[0..n) = diagonal of G (n x n) in descending order, S[0] = -sum_{p>0} p log2 p
hipError_t spectrum_sorted(const double* G, int n, double* p, double* S, hipStream_t s);
// after a restart: ++runs[0] when done[0] is still 0 (the restart ran), then
// done[0] = 1 when res[0] <= tol max(1, |lam[0]|)
hipError_t lz_mark_done(const double* res, const double* lam, double tol, int* done, int* runs, hipStream_t s);
// Full reorthogonalisation against the first nq rows of Q (row length n), in
// two passes of classical Gram-Schmidt; `part` holds lz_reorth_part_doubles()
// doubles, `nrm` lz_norm_doubles().  For recurrence step j (nq = j + 1):
// first:  c1 = Q^T w (c1[nq] = ||w||^2 before), w -= Q c1;
// final:  c2 = Q^T w, w -= Q c2, alpha[j] = c1[j] + c2[j], beta[j] = ||w||
//         (zero, and stop / m_eff set, when beta[j] <= tol ||H q_j||),
//         q_{j+1} = w / beta[j] into qn, and also into stage when not null.
size_t lz_reorth_part_doubles();
size_t lz_norm_doubles();
hipError_t lz_reorth_first(double* w, const double* Q, int nq, size_t n, double* coef, double* part, hipStream_t s);
hipError_t lz_reorth_final(double* w, const double* Q, int nq, size_t n, const double* c1, double* c2, double* part,
                           double* nrm, double* alpha, double* beta, double tol, int* stop, int* m_eff, double* qn,
                           double* stage, hipStream_t s);
// X <- (X + sign X^T) / 2 in place (sign = +1 symmetric, -1 antisymmetric part)
hipError_t symmetrize_f64(double* X, int n, double sign, hipStream_t s);
}  // namespace ttn
