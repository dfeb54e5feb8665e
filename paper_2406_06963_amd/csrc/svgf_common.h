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
    uint32_t kw;  // a-trous kernel width, 5 or 3
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
    float* ke;           // [HW] prefiltered AO-value coefficient of the current level (in work)
    uint32_t* fb;        // [16 x 16 tiles] tile holds a pixel of short history (in work; filter only)
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

// Variance written for invalid pixels by the a-trous levels, so the variance
// prefilter of the next level finds valid neighbours from (c, var) alone.
// Finite, so a zero tap weight times it stays zero.
constexpr float kNoVar = -3.0e38f;
__device__ __forceinline__ bool has_var(float v) { return v > -1.0e38f; }

// ke = -log2(e) / (sigma_l g + eps_l) with g = sqrt of the 3x3 (1,2,1)/4 blur of
// the variance over valid pixels (G and its weight sk accumulated by the caller)
__device__ __forceinline__ float ke_of(float G, float sk, float sl, float eps_l) {
    return -1.4426950408889634f * __builtin_amdgcn_rcpf(fmaf(sl, __builtin_amdgcn_sqrtf(G * __builtin_amdgcn_rcpf(sk)), eps_l));
}

__device__ __forceinline__ void tile_xy(uint32_t t, uint32_t tiles_x, uint32_t& x, uint32_t& y) {
    x = (t % tiles_x) * kSvgfTile + (threadIdx.x % kSvgfTile);
    y = (t / tiles_x) * kSvgfTile + (threadIdx.x / kSvgfTile);
}

// Fills an N-entry LDS tile: every lane first issues the loads of all its
// entries (load(e) must be safe for every e < N), then stores them, so the
// loads of one lane overlap instead of each waiting for the previous store.
template <int N, class Load, class Store>
__device__ __forceinline__ void stage_tile(Load load, Store store) {
    constexpr int K = (N + kSvgfBlock - 1) / kSvgfBlock;
    decltype(load(0)) v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = (int)threadIdx.x + k * kSvgfBlock;
        if (N % kSvgfBlock == 0 || e < N) v[k] = load(e);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = (int)threadIdx.x + k * kSvgfBlock;
        if (N % kSvgfBlock == 0 || e < N) store(e, v[k]);
    }
}

// Row-class tiles of the a-trous levels at stride s = 2^level: a workgroup
// owns 64 consecutive pixels of 4 rows that are s apart (rows congruent mod
// s); tile t of a frame is column block t % tx, then row class, then block
// of 4s rows.
constexpr int kRowsTX = 64, kRowsTY = kSvgfBlock / kRowsTX;

__host__ __device__ constexpr uint32_t rows_tiles(uint32_t W, uint32_t H, int level) {
    return ((W + kRowsTX - 1) / kRowsTX) * (1u << level) * ((H + (kRowsTY << level) - 1) / (kRowsTY << level));
}

// The adjoint runs levels up to kAdjRowsMax on row-class tiles, deeper levels
// (whose staged neighbourhood would not fit in LDS) on 16 x 16 tiles.
constexpr uint32_t kAdjRowsMax = 4;

__host__ __device__ constexpr uint32_t adjoint_tiles(uint32_t W, uint32_t H, uint32_t level) {
    return level <= kAdjRowsMax ? rows_tiles(W, H, (int)level)
                                : ((W + kSvgfTile - 1) / kSvgfTile) * ((H + kSvgfTile - 1) / kSvgfTile);
}

// Geometry and (c, var) of one staged pixel
struct Staged {
    float4 nz;
    float2 cv;
};

__device__ __forceinline__ bool inside(int qx, int qy, int W, int H) {
    return (unsigned)qx < (unsigned)W && (unsigned)qy < (unsigned)H;
}

// Index of the pixel nearest to (qx, qy) inside the frame: staging loads
// read it unconditionally (no branch per staged pixel) and discard what lies
// outside.
__device__ __forceinline__ size_t clamped_index(int qx, int qy, int W, int H) {
    return (size_t)min(max(qy, 0), H - 1) * (size_t)W + (size_t)min(max(qx, 0), W - 1);
}

// A staged pixel's geometry and (c, var); outside the frame it reads its
// nearest pixel and reports depth 0 (invalid), which the staging stores as a
// zero normal.
__device__ __forceinline__ Staged load_staged(const float4* __restrict__ nz, const float2* __restrict__ cv, int qx,
                                              int qy, int W, int H) {
    const size_t q = clamped_index(qx, qy, W, H);
    Staged r{nz[q], cv[q]};
    if (!inside(qx, qy, W, H)) r.nz.w = 0.0f;
    return r;
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

// The a-trous stencil of radius KR (2: 5x5 B3 taps, 1: 3x3 (1,2,1)/4 taps).
// Tap tp < half_taps<KR> is the tp-th tap after the centre in raster order;
// its mirror (-a, -b) is the matching tap before the centre.
template <int KR>
__device__ __forceinline__ float hk(int a) { return KR == 2 ? b3(a) : k3(a); }
// log2 of the same weights (log2 3/8 = log2 3 - 3), added to a tap's
// exponent instead of multiplying its weight
template <int KR>
__device__ __forceinline__ float lhk(int a) {
    return KR == 2 ? (a == 0 ? -1.4150374992788438f : (a == 1 || a == -1 ? -2.0f : -4.0f)) : (a == 0 ? -1.0f : -2.0f);
}
template <int KR>
constexpr int half_taps = ((2 * KR + 1) * (2 * KR + 1) - 1) / 2;
template <int KR>
constexpr float centre_h = KR == 2 ? 0.140625f : 0.25f;  // h(0, 0)
template <int KR>
__device__ __forceinline__ void tap_ab(int tp, int& a, int& b) {
    const int idx = tp + half_taps<KR> + 1;
    a = idx % (2 * KR + 1) - KR;
    b = idx / (2 * KR + 1) - KR;
}

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

// |s (a dz/dx + b dz/dy)|, the depth change the gradient predicts at tap
// (a, b) of stride s, rounded as b dz/dy, then one fma: with contraction off
// the compiler cannot fuse the other product instead once a and b are
// constants (it would for |a| = 1, |b| = 3), so unrolled and looped code give
// the same bits.  The sum can nearly cancel at grazing angles, where an ulp of
// it moves the weight; the mirror (-a, -b) gives the same bits.
__device__ __forceinline__ float tap_span(float2 dzp, int a, int b, int s) {
#pragma clang fp contract(off)
    return fabsf((float)s * fmaf((float)a, dzp.x, (float)b * dzp.y));
}

// kz of the tap pair (a, b) / (-a, -b) at stride s
__device__ __forceinline__ float depth_coef(float2 dzp, int a, int b, int s, float sz, float eps_zp) {
    return kNegLog2e * hw_rcp(fmaf(sz, tap_span(dzp, a, b, s), eps_zp));
}

__device__ __forceinline__ float fused_weight(float kz, float ke, float zp, float cp, float3 np, float sn, float4 nq,
                                              float cq) {
    const float x = fminf(dot3(np, f3(nq)), 1.0f);
    const float e = fmaf(kz, fabsf(zp - nq.w), fmaf(ke, fabsf(cp - cq), sn * hw_log2(x)));
    return x > 0.0f ? hw_exp2(e) : 0.0f;
}

// One tap of a level whose staged neighbourhood holds a zero normal for
// invalid pixels (so n_p . n_q = 0 and the weight vanishes): accumulates the
// weight sum, the weighted deviation and the squared-weight variance.  The
// stencil weight enters as lh = log2 h in the exponent, h w = exp2(e + lh).
// The normal term clamps n_p . n_q to [0, 1]; at 0 its log2 is -inf, the
// exponent -inf and the weight exactly 0 with no test, provided sn > 0 (the
// parameter block raises sigma_n = 0 to the smallest normal float, whose
// weight x^sn rounds to 1 for every x > 0).
__device__ __forceinline__ void accumulate_tap(float lh, float kz, float ke, float zp, float cp, float3 np, float sn,
                                               float4 nq, float2 cvq, float& Dn, float& Sc, float& Sv) {
    const float x = __builtin_amdgcn_fmed3f(dot3(np, f3(nq)), 0.0f, 1.0f);
    const float d = cvq.x - cp;
    const float e = fmaf(kz, fabsf(zp - nq.w), fmaf(ke, fabsf(d), fmaf(sn, hw_log2(x), lh)));
    const float hw = hw_exp2(e);
    Dn += hw;
    Sc = fmaf(hw, d, Sc);
    Sv = fmaf(hw * hw, cvq.y, Sv);
}

}  // namespace dhr
