// BF16 storage helpers shared by the row kernels and the auxiliary kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ntc {

__device__ __forceinline__ float bf16_to_f32(uint16_t b)
{
    return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

// round-to-nearest-even FP32 -> BF16 (inputs are finite)
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

}  // namespace ntc
