#pragma once
#include "common.h"

namespace ttn {
hipError_t gemm_plain(Prec prec, const GemmDesc& g, void* scratch, size_t scratch_bytes, hipStream_t s);
// MFMA kernels (float32 / split-bf16); hipErrorNotSupported when the shape or
// the strides do not fit their loaders.
hipError_t gemm_mfma(Prec prec, const GemmDesc& g, void* scratch, size_t scratch_bytes, hipStream_t s);
hipError_t splitk_reduce_f32(const GemmDesc& g, int splits, const float* partial, hipStream_t s);
hipError_t splitk_reduce_f64(const GemmDesc& g, int splits, const double* partial, hipStream_t s);
bool gemm_path_mfma_enabled();
void gemm_set_mfma_enabled(bool on);
}  // namespace ttn
