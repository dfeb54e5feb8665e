// Shared pieces of the SVGF kernels (forward and adjoint): frame
// descriptors, parameters and the edge-stopping weights (Section 3.3: depth
// and normal differences, plus the AO-value term of the iterated kernel).
#pragma once

#include "device.h"
#include "internal.h"

namespace dhr {

constexpr int kSvgfTile = 16;            // 16 x 16 pixels per workgroup
constexpr int kSvgfBlock = kSvgfTile * kSvgfTile;

struct SvgfK {
    uint32_t levels;
    float alpha, alpha_m;
    float sz[DHR_MAX_LEVELS], sn[DHR_MAX_LEVELS], sl[DHR_MAX_LEVELS];
    float eps_z, eps_l, cos_min, plane_px;
    uint32_t use_obj, var_min_h, R, fb_level;
    float cap;
};

struct SvgfDesc {
    uint32_t W, H, n_ao, tiles_x;
    const uint8_t* ao;
    const float4* pos;
    const float4* nz;
    const float2* dz;
    const float2* mv;
    const float4* prev_pos;
    const float4* prev_nz;
    const float4* hist_in;
    float4* hist_out;
    float* out;
    float2* save;        // [levels][HW]
    float2* work;        // [2][HW]
    const float2* b0;    // level-0 input when it is not save[0]/work[0]
    float pix;
};
constexpr int kSvgfMaxB = 24;
using SvgfBatch = Batch<SvgfDesc, kSvgfMaxB>;

// The (c, var) input buffer of level l.
__device__ __forceinline__ float2* level_buf(const SvgfDesc& D, uint32_t l) {
    const size_t HW = (size_t)D.W * D.H;
    if (l == 0 && D.b0) return const_cast<float2*>(D.b0);
    return D.save ? D.save + (size_t)l * HW : D.work + (size_t)(l & 1u) * HW;
}

__device__ __forceinline__ void tile_xy(uint32_t t, uint32_t tiles_x, uint32_t& x, uint32_t& y) {
    x = (t % tiles_x) * kSvgfTile + (threadIdx.x % kSvgfTile);
    y = (t / tiles_x) * kSvgfTile + (threadIdx.x / kSvgfTile);
}

// Workgroups are dispatched to the 8 XCDs round-robin by id.  This remap
// (a bijection of [0, nb)) makes consecutive logical tiles share an XCD, so
// tiles that read the same cache lines share its L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nb) {
    const uint32_t q = nb / 8, r = nb % 8, xcd = b % 8, k = b / 8;
    return xcd < r ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

// 1-D taps: B3 spline (1,4,6,4,1)/16 and the (1,2,1)/4 variance prefilter
__device__ __forceinline__ float b3(int a) { return a == 0 ? 0.375f : (a == 1 || a == -1 ? 0.25f : 0.0625f); }
__device__ __forceinline__ float k3(int a) { return a == 0 ? 0.5f : 0.25f; }

// All three edge-stopping terms as one power of two:
//   w = exp2(kz |z_p - z_q| + ke |c_p - c_q| + sigma_n log2(n_p . n_q))
// with kz = -log2(e) / (sigma_z S + eps_z z_p) (S shared by a tap and its
// mirror) and ke = -log2(e) / (sigma_l g + eps_l); zero when n_p . n_q <= 0.
// Hardware exp2 / log2 / rcp (about 1 ulp) replace the library calls and
// divisions of the per-term form; the product is the same function.
constexpr float kNegLog2e = -1.4426950408889634f;

__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// kz of the tap pair (a, b) / (-a, -b) at stride s
__device__ __forceinline__ float depth_coef(float2 dzp, int a, int b, int s, float sz, float eps_zp) {
    const float S = fabsf((float)s * ((float)a * dzp.x + (float)b * dzp.y));
    return kNegLog2e * hw_rcp(fmaf(sz, S, eps_zp));
}

__device__ __forceinline__ float fused_weight(float kz, float ke, float zp, float cp, float3 np, float sn, float4 nq,
                                              float cq) {
    const float x = fminf(dot3(np, f3(nq)), 1.0f);
    const float e = fmaf(kz, fabsf(zp - nq.w), fmaf(ke, fabsf(cp - cq), sn * hw_log2(x)));
    return x > 0.0f ? hw_exp2(e) : 0.0f;
}

}  // namespace dhr
