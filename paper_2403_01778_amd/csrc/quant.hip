// Low-precision copies of a tensor for the precision form: bfloat16 (round to
// nearest even) and OCP FP8 E4M3 with a per-tensor scale amax/448 (round to
// nearest even, saturating at 448).  The scale is computed on the device; the
// max reduction is order-independent, so the codes are deterministic.
#include <algorithm>

#include "common.h"
#include "quant.h"

namespace hoscf {

__global__ __launch_bounds__(256) void amax_kernel(const float* __restrict__ x, int64_t n, unsigned* amax_bits) {
    float m = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        m = fmaxf(m, fabsf(x[i]));
    for (int k = 32; k >= 1; k >>= 1) m = fmaxf(m, __shfl_xor(m, k));
    __shared__ float wm[4];
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float t = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
        // non-negative binary32 values order like their bit patterns
        atomicMax(amax_bits, __float_as_uint(t));
    }
}

__global__ void zero_u32_kernel(unsigned* p) { *p = 0u; }

__global__ void scale_kernel(const unsigned* amax_bits, float* scale) {
    const float amax = __uint_as_float(*amax_bits);
    *scale = amax > 0.f ? __fdiv_rn(amax, 448.0f) : 1.0f;
}

// binary32 -> E4M3 (OCP): RNE on the dropped mantissa bits, subnormals below
// 2^-6, saturation to the largest finite value 448 (code 0x7E).
__device__ __forceinline__ unsigned e4m3_encode(float y) {
    const unsigned b = __float_as_uint(y);
    const unsigned sign = (b >> 31) << 7;
    const float a = fabsf(y);
    if (!(a < 448.0f)) return sign | 0x7Eu;  // also Inf; NaN is not expected
    if (a < 0x1p-6f) return sign | (unsigned)rintf(a * 512.0f);  // m * 2^-9, m in [0, 8]
    const unsigned mant = b & 0x7fffffu;
    unsigned E = ((b >> 23) & 0xffu) - 127u + 7u;
    unsigned r = (mant + 0x7ffffu + ((mant >> 20) & 1u)) >> 20;
    if (r == 8u) {
        r = 0u;
        E += 1u;
    }
    unsigned code = (E << 3) | r;
    if (code > 0x7Eu) code = 0x7Eu;
    return sign | code;
}

__global__ __launch_bounds__(256) void fp8_kernel(const float* __restrict__ x, int64_t n, const float* scale,
                                                  uint8_t* __restrict__ out) {
    const float s = *scale;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = (uint8_t)e4m3_encode(__fdiv_rn(x[i], s));
}

__global__ __launch_bounds__(256) void bf16_kernel(const float* __restrict__ x, int64_t n, uint16_t* __restrict__ out,
                                                   float* scale) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && scale) *scale = 1.0f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const unsigned b = __float_as_uint(x[i]);
        out[i] = (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
    }
}

int quantize(const float* src, int64_t n, int dtype, void* dst, float* scale_dev, void* ws, size_t ws_bytes,
             hipStream_t s) {
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192));
    if (dtype == HOSCF_BF16) {
        hipLaunchKernelGGL(bf16_kernel, dim3(grid), dim3(256), 0, s, src, n, (uint16_t*)dst, scale_dev);
        return hipGetLastError() == hipSuccess ? HOSCF_OK : HOSCF_HIP_ERROR;
    }
    if (dtype != HOSCF_FP8E4M3) return HOSCF_INVALID_ARG;
    if (!ws || ws_bytes < sizeof(unsigned)) return HOSCF_WORKSPACE_TOO_SMALL;
    unsigned* amax = static_cast<unsigned*>(ws);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, s, amax);
    hipLaunchKernelGGL(amax_kernel, dim3(grid), dim3(256), 0, s, src, n, amax);
    hipLaunchKernelGGL(scale_kernel, dim3(1), dim3(1), 0, s, amax, scale_dev);
    hipLaunchKernelGGL(fp8_kernel, dim3(grid), dim3(256), 0, s, src, n, scale_dev, (uint8_t*)dst);
    return hipGetLastError() == hipSuccess ? HOSCF_OK : HOSCF_HIP_ERROR;
}

}  // namespace hoscf
