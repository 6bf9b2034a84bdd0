#pragma once
#include "common.h"

namespace ttn {
hipError_t gemm_plain(Prec prec, const GemmDesc& g, void* scratch, size_t scratch_bytes, hipStream_t s);
// Launch shape of an MFMA product: the output tile (float64: 1 64 x 64,
// 2 128 x 64, 3 64 x 128; 0 the default, 64 x 64) and the order in which tiles
// are handed out (0 default, 1 x fastest, 2 y fastest).  Every choice computes every output element with
// the same instruction sequence and the same split-K partition, so results
// are identical bit for bit; only the speed differs.
struct GemmLaunch {
  int tile = 0;
  int orient = 0;
};
// MFMA kernels (float32 / split-bf16 / float64); hipErrorNotSupported when the
// shape or the strides do not fit their loaders.
hipError_t gemm_mfma(Prec prec, const GemmDesc& g, void* scratch, size_t scratch_bytes, hipStream_t s,
                     const GemmLaunch& how = GemmLaunch());
hipError_t splitk_reduce_f32(const GemmDesc& g, int splits, const float* partial, hipStream_t s);
hipError_t splitk_reduce_f64(const GemmDesc& g, int splits, const double* partial, hipStream_t s);
bool gemm_path_mfma_enabled();
// tuned launch shape of a product (see gemm_tune.cpp): false when none is stored
bool gemm_tuned_choice(Prec prec, const GemmDesc& g, hipStream_t s, void* scratch, size_t scratch_bytes,
                       GemmLaunch* out);
void gemm_tune_set_mode(int mode);
size_t gemm_tune_entries();
void gemm_tune_clear();
// the kept choices as text, one per line (false / -1 on an I/O or format
// error); load merges the file's choices into the table and returns their count
bool gemm_tune_save(const char* path);
int gemm_tune_load(const char* path);
void gemm_set_mfma_enabled(bool on);
}  // namespace ttn
