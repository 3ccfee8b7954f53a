// Quantisation of FP32 tensors to the low-precision storage formats.
#pragma once

#include "common.h"

namespace hoscf {

int quantize(const float* src, int64_t n, int dtype, void* dst, float* scale_dev, void* ws, size_t ws_bytes,
             hipStream_t s);

}  // namespace hoscf
