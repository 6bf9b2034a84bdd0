#pragma once
#include "common.h"

namespace ttn {
hipError_t gemm_plain(Prec prec, const GemmDesc& g, void* scratch, size_t scratch_bytes, hipStream_t s);
// MFMA kernels (float32 / split-bf16); hipErrorNotSupported when the shape or
// the strides do not fit their loaders.
// splits_req > 0 asks for that many split-K slices (clamped to what the
// scratch and K allow); *splits_used (may be null) receives the count run.
hipError_t gemm_mfma(Prec prec, const GemmDesc& g, void* scratch, size_t scratch_bytes, hipStream_t s,
                     int splits_req = 0, int* splits_used = nullptr);
hipError_t splitk_reduce_f32(const GemmDesc& g, int splits, const float* partial, hipStream_t s);
hipError_t splitk_reduce_f64(const GemmDesc& g, int splits, const double* partial, hipStream_t s);
bool gemm_path_mfma_enabled();
// tuned choice for a product (see gemm_tune.cpp): false when none is stored
struct GemmChoice {
  int path;    // 0: MFMA kernels, 1: general kernel
  int splits;  // split-K slices for the MFMA path (0: heuristic)
};
bool gemm_tuned_choice(Prec prec, const GemmDesc& g, hipStream_t s, void* scratch, size_t scratch_bytes,
                       GemmChoice* out);
void gemm_tune_set_mode(int mode);
size_t gemm_tune_entries();
void gemm_tune_clear();
void gemm_set_mfma_enabled(bool on);
}  // namespace ttn
