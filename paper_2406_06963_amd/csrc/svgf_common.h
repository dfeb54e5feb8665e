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

// 1-D taps: B3 spline (1,4,6,4,1)/16 and the (1,2,1)/4 variance prefilter
__device__ __forceinline__ float b3(int a) { return a == 0 ? 0.375f : (a == 1 || a == -1 ? 0.25f : 0.0625f); }
__device__ __forceinline__ float k3(int a) { return a == 0 ? 0.5f : 0.25f; }

// depth term: exp(-|z_p - z_q| / (sigma_z |s (a dzx + b dzy)| + eps z_p))
__device__ __forceinline__ float w_depth(float zp, float zq, float2 dzp, int a, int b, int s, float sz, float eps) {
    const float S = fabsf((float)s * ((float)a * dzp.x + (float)b * dzp.y));
    return expf(-fabsf(zp - zq) / fmaf(sz, S, eps * zp));
}

// normal term: max(0, min(1, n_p . n_q))^sigma_n, 0 when the dot is <= 0
__device__ __forceinline__ float w_normal(float3 np, float3 nq, float sn) {
    const float x = fminf(dot3(np, nq), 1.0f);
    return x > 0.0f ? exp2f(sn * log2f(x)) : 0.0f;
}

}  // namespace dhr
