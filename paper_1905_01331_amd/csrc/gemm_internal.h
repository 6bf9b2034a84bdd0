#pragma once
#include "common.h"

namespace ttn {
hipError_t gemm_plain(Prec prec, const GemmDesc& g, void* scratch, size_t scratch_bytes, hipStream_t s);
}  // namespace ttn
