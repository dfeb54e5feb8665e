// Wire form of a served frame: one byte per filtered AO value (Section 3.2:
// the AO a client receives fits 8 bits) and one visibility bit per light
// (Section 3.1, Fig. 1).  Memory-bound: a lane handles four pixels.
#include "device.h"
#include "internal.h"

namespace dhr {
namespace {

__device__ __forceinline__ uint8_t quantize(float v) {
#pragma clang fp contract(off)
    if (!(v > 0.0f)) v = 0.0f;  // negative values and NaN
    if (v > 1.0f) v = 1.0f;
    const float s = 255.0f * v;
    return (uint8_t)floorf(s + 0.5f);
}

__global__ __launch_bounds__(256) void encode_kernel(const float* __restrict__ value, uint8_t* __restrict__ q,
                                                     const uint8_t* __restrict__ sc, uint32_t n_lights,
                                                     uint32_t n_shadow, uint8_t* __restrict__ mask, uint64_t n) {
    const uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i0 >= n) return;
    const bool full = i0 + 4 <= n;
    if (value) {
        if (full && (reinterpret_cast<uintptr_t>(value + i0) & 15) == 0 && (reinterpret_cast<uintptr_t>(q + i0) & 3) == 0) {
            const float4 v = *reinterpret_cast<const float4*>(value + i0);
            *reinterpret_cast<uchar4*>(q + i0) = make_uchar4(quantize(v.x), quantize(v.y), quantize(v.z), quantize(v.w));
        } else {
            for (uint64_t i = i0; i < n && i < i0 + 4; ++i) q[i] = quantize(value[i]);
        }
    }
    if (sc) {
        if (full && (n & 3) == 0 && (reinterpret_cast<uintptr_t>(sc) & 3) == 0 &&
            (reinterpret_cast<uintptr_t>(mask) & 3) == 0) {
            uint32_t m[4] = {0, 0, 0, 0};
            for (uint32_t l = 0; l < n_lights; ++l) {
                const uchar4 c = *reinterpret_cast<const uchar4*>(sc + (uint64_t)l * n + i0);
                m[0] |= (2u * c.x >= n_shadow) ? 1u << l : 0u;
                m[1] |= (2u * c.y >= n_shadow) ? 1u << l : 0u;
                m[2] |= (2u * c.z >= n_shadow) ? 1u << l : 0u;
                m[3] |= (2u * c.w >= n_shadow) ? 1u << l : 0u;
            }
            *reinterpret_cast<uchar4*>(mask + i0) = make_uchar4(m[0], m[1], m[2], m[3]);
        } else {
            for (uint64_t i = i0; i < n && i < i0 + 4; ++i) {
                uint32_t m = 0;
                for (uint32_t l = 0; l < n_lights; ++l)
                    if (2u * sc[(uint64_t)l * n + i] >= n_shadow) m |= 1u << l;
                mask[i] = (uint8_t)m;
            }
        }
    }
}

}  // namespace
}  // namespace dhr

extern "C" {

dhr_status dhr_encode_frame(dhr_ctx* ctx, const float* value, uint8_t* q, const uint8_t* shadow_count,
                            uint32_t n_lights, uint32_t n_shadow, uint8_t* mask, uint64_t n, dhr_stream stream) {
    if (!ctx) return DHR_ERR_INVALID_ARG;
    if ((value && !q) || (shadow_count && !mask))
        return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_encode_frame: missing output buffer");
    if (shadow_count && (n_lights < 1 || n_lights > DHR_MAX_LIGHTS || n_shadow < 1))
        return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_encode_frame: n_lights must be 1..8 and n_shadow >= 1");
    if (n > (1ull << 36)) return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_encode_frame: n too large");
    if (n == 0 || (!value && !shadow_count)) return DHR_OK;
    dhr::DeviceGuard g(ctx->device);
    const uint64_t lanes = (n + 3) / 4;
    hipLaunchKernelGGL(dhr::encode_kernel, dim3((uint32_t)((lanes + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), value, q, shadow_count, n_lights, n_shadow, mask, n);
    return dhr::check_launch(ctx, "dhr_encode_frame");
}

}  // extern "C"
