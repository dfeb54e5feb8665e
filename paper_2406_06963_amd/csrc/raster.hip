// G-buffer by rasterisation.  The paper's server rasterises the G-buffer
// (Section 2.2: world-space position per pixel) and traces its visibility
// rays from it; rasterising is also far less work than one primary ray per
// pixel through the BVH.  The result is defined as the closest hit of the
// pixel's primary ray (ties: lowest input index), so it must equal the
// ray-traced G-buffer texel for texel: every (pixel, triangle) candidate
// that rasterisation proposes is decided by the same ray-triangle test the
// traversal uses, and the winner is the minimum of (t, input index) packed
// into one 64-bit key per pixel (atomic min; t > 0, so its bits order like
// the values).  Candidates come from a conservative screen box of each
// triangle: the triangle clipped to the camera's near side, projected, grown
// by half a pixel.  A hit point with view depth below the clip distance lies
// closer to the eye than `near_r` (primary rays make at most the corner
// angle with the view axis), so triangles whose plane passes that close are
// tested against the whole frame instead.
//
// Unclipped triangles also get their projected edges: a pixel centre more
// than half a pixel outside one of them is rejected without the exact test.
//
// Passes: clear the keys; one thread
// per triangle projects it and tests the pixels of a small box itself (at
// most kSmallArea pixel centres), or lists it as medium (at most kMidArea) or
// large (one entry per 64 x 64 block of its box); one thread per medium
// triangle tests its box; one wave per large-triangle block tests the 8 x 8
// tiles that come within half a pixel of the triangle, a pixel per lane; one
// thread per pixel turns its key into the texel.
#include <cmath>
#include <cstring>

#include "camera.h"
#include "device.h"
#include "internal.h"

// Each pass recomputes a triangle's screen footprint; without contraction
// every pass computes the same one.
#pragma clang fp contract(off)

namespace dhr {
namespace {

constexpr int kRB = 256;               // threads per workgroup
constexpr uint32_t kSmallArea = 16;    // pixel centres the projecting thread tests itself
constexpr uint32_t kMidArea = 64;      // pixel centres a thread of the medium pass tests
constexpr int kBlockPx = 64;           // side of a large triangle's block
constexpr float kMargin = 0.5f;        // pixels
constexpr float kEdgeRange = 1.0e5f;   // projected coordinates for which edges are used

struct RasterDesc {
    const float4* tris;
    const uint32_t* rec_of;
    uint32_t T, W, H, has_prev;
    CamD cur, prev;
    float inv_tx, inv_ty;  // 1 / tan(fov/2) per axis
    float near_z;          // clip distance along the view axis
    float near_r;          // plane distance below which a triangle takes the whole frame
    unsigned long long* key;  // [HW]
    uint32_t* mid;            // [T]: records of the medium triangles
    uint2* big;               // [cap]: (record, 64 x 64 block of its box) of the large triangles
    unsigned long long* ctr;  // [0] medium triangles, [1] large-triangle blocks
    uint32_t cap;
    float4* pos;
    float4* nz;
    float2* dz;
    float2* mv;
};

__device__ __forceinline__ float3 cam_vec(const float* v) { return f3(v[0], v[1], v[2]); }

// Screen footprint of a triangle: the box of pixel centres that may see it
// and, for an unclipped triangle of nonzero projected area, its edges as
// signed pixel distances (inside >= 0).
struct Screen {
    int x0, y0, x1, y1;
    bool edges;
    float a[3], b[3], c[3];
};

__device__ __forceinline__ bool tri_screen(const RasterDesc& D, float4 v0, float4 e1, float4 e2, Screen& S) {
    const CamD& C = D.cur;
    const float3 eye = cam_vec(C.eye), fwd = cam_vec(C.fwd), rt = cam_vec(C.right), up = cam_vec(C.up);
    const float3 a = f3(v0);
    const float3 V[3] = {a, a + f3(e1), a + f3(e2)};
    S.edges = false;
    // near the eye: the whole frame
    const float3 n = cross3(f3(e1), f3(e2));
    const float nl = sqrtf(dot3(n, n));
    if (nl > 0.0f && fabsf(dot3(eye - a, n)) < D.near_r * nl) {
        S.x0 = 0;
        S.y0 = 0;
        S.x1 = (int)D.W - 1;
        S.y1 = (int)D.H - 1;
        return true;
    }
    float z[3];
    for (int k = 0; k < 3; ++k) z[k] = dot3(V[k] - eye, fwd);
    const float zn = D.near_z;
    if (z[0] < zn && z[1] < zn && z[2] < zn) return false;
    const bool clipped = z[0] < zn || z[1] < zn || z[2] < zn;
    // the triangle clipped to z >= zn: kept vertices and edge crossings
    float lx = INFINITY, hx = -INFINITY, ly = INFINITY, hy = -INFINITY;
    float px[3], py[3];
    auto proj = [&](float3 p, float zc, float& X, float& Y) {
        const float3 v = p - eye;
        const float r = __builtin_amdgcn_rcpf(zc);
        X = fmaf(dot3(v, rt) * r, D.inv_tx, 1.0f) * (0.5f * (float)D.W);
        Y = fmaf(-dot3(v, up) * r, D.inv_ty, 1.0f) * (0.5f * (float)D.H);
        lx = fminf(lx, X);
        hx = fmaxf(hx, X);
        ly = fminf(ly, Y);
        hy = fmaxf(hy, Y);
    };
    for (int k = 0; k < 3; ++k) {
        const int m = k == 2 ? 0 : k + 1;
        if (z[k] >= zn) proj(V[k], z[k], px[k], py[k]);
        if ((z[k] < zn) != (z[m] < zn)) {
            const float s = (zn - z[k]) / (z[m] - z[k]);
            float X, Y;
            proj(V[k] + (V[m] - V[k]) * s, zn, X, Y);
        }
    }
    // pixel centres x + 0.5 within kMargin of the projected box
    constexpr float kBig = 1.0e8f;
    lx = fmaxf(lx, -kBig);
    ly = fmaxf(ly, -kBig);
    hx = fminf(hx, kBig);
    hy = fminf(hy, kBig);
    S.x0 = max((int)ceilf(lx - 0.5f - kMargin), 0);
    S.y0 = max((int)ceilf(ly - 0.5f - kMargin), 0);
    S.x1 = min((int)floorf(hx - 0.5f + kMargin), (int)D.W - 1);
    S.y1 = min((int)floorf(hy - 0.5f + kMargin), (int)D.H - 1);
    if (S.x0 > S.x1 || S.y0 > S.y1) return false;
    if (!clipped && fmaxf(fmaxf(-lx, hx), fmaxf(-ly, hy)) < kEdgeRange) {
        const float area = (px[1] - px[0]) * (py[2] - py[0]) - (py[1] - py[0]) * (px[2] - px[0]);
        if (area != 0.0f) {
            const float sg = area > 0.0f ? 1.0f : -1.0f;
            S.edges = true;
            for (int k = 0; k < 3; ++k) {
                const int m = k == 2 ? 0 : k + 1;
                const float dx = px[m] - px[k], dy = py[m] - py[k];
                const float il = sg * __builtin_amdgcn_rsqf(dx * dx + dy * dy);
                S.a[k] = -dy * il;
                S.b[k] = dx * il;
                S.c[k] = -fmaf(S.a[k], px[k], S.b[k] * py[k]);
                if (!(fabsf(il) < INFINITY)) S.edges = false;
            }
        }
    }
    return true;
}

// Whether pixel centre (x + 0.5, y + 0.5) lies within kMargin of the triangle.
__device__ __forceinline__ bool near_pixel(const Screen& S, int x, int y) {
    if (!S.edges) return true;
    const float X = (float)x + 0.5f, Y = (float)y + 0.5f;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) ok = ok && fmaf(S.a[k], X, fmaf(S.b[k], Y, S.c[k])) >= -kMargin;
    return ok;
}

// Whether any pixel centre of [x0, x1] x [y0, y1] lies within kMargin of the
// triangle (each edge distance is linear: its maximum is at a corner).
__device__ __forceinline__ bool near_tile(const Screen& S, int x0, int y0, int x1, int y1) {
    if (!S.edges) return true;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float X = (S.a[k] > 0.0f ? (float)x1 : (float)x0) + 0.5f;
        const float Y = (S.b[k] > 0.0f ? (float)y1 : (float)y0) + 0.5f;
        ok = ok && fmaf(S.a[k], X, fmaf(S.b[k], Y, S.c[k])) >= -kMargin;
    }
    return ok;
}

// Tests pixel (x, y) against the triangle record and keeps the nearer key.
__device__ __forceinline__ void test_pixel(const RasterDesc& D, float3 eye, float4 v0, float4 e1, float4 e2, int x,
                                           int y) {
    const float t = tri_t_rec(v0, e1, e2, eye, cam_dir(D.cur, x + 0.5f, y + 0.5f));
    if (t > 0.0f)
        atomicMin(D.key + (size_t)y * D.W + x, ((unsigned long long)__float_as_uint(t) << 32) | fbits(v0.w));
}

// Tests the pixels of [x0, x1] x [y0, y1] near the triangle, one thread.
__device__ __forceinline__ void test_box(const RasterDesc& D, const Screen& S, float4 v0, float4 e1, float4 e2, int x0,
                                         int y0, int x1, int y1) {
    const float3 eye = cam_vec(D.cur.eye);
    for (int y = y0; y <= y1; ++y)
        for (int x = x0; x <= x1; ++x)
            if (near_pixel(S, x, y)) test_pixel(D, eye, v0, e1, e2, x, y);
}

__global__ __launch_bounds__(kRB) void clear_kernel(const RasterDesc D) {
    const uint32_t i = blockIdx.x * kRB + threadIdx.x;
    if (i < 2) D.ctr[i] = 0ull;
    if (i >= D.W * D.H) return;
    D.key[i] = ~0ull;
}

__device__ __forceinline__ uint32_t box_area(const Screen& S) {
    return (uint32_t)(S.x1 - S.x0 + 1) * (uint32_t)(S.y1 - S.y0 + 1);
}
__device__ __forceinline__ uint32_t blocks_x(const Screen& S) { return (uint32_t)(S.x1 - S.x0 + kBlockPx) / kBlockPx; }
__device__ __forceinline__ uint32_t blocks_of(const Screen& S) {
    return blocks_x(S) * ((uint32_t)(S.y1 - S.y0 + kBlockPx) / kBlockPx);
}

// Wave-aggregated reservation of n slots per lane on counter c: returns the
// lane's first slot.
__device__ __forceinline__ unsigned long long reserve(unsigned long long* c, uint32_t n) {
    const uint32_t lane = threadIdx.x & 63;
    uint32_t incl = n;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(incl, o, 64);
        if ((int)lane >= o) incl += v;
    }
    const uint32_t total = __shfl(incl, 63, 64);
    unsigned long long base = 0;
    if (lane == 0 && total) base = atomicAdd(c, (unsigned long long)total);
    return __shfl(base, 0, 64) + (incl - n);
}

__global__ __launch_bounds__(kRB) void setup_kernel(const RasterDesc D) {
    const uint32_t k = blockIdx.x * kRB + threadIdx.x;
    float4 v0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), e1 = v0, e2 = v0;
    Screen S;
    bool any = false;
    if (k < D.T) {
        v0 = D.tris[3ull * k];
        e1 = D.tris[3ull * k + 1];
        e2 = D.tris[3ull * k + 2];
        any = tri_screen(D, v0, e1, e2, S);
    }
    const uint32_t area = any ? box_area(S) : 0u;
    if (any && area <= kSmallArea) test_box(D, S, v0, e1, e2, S.x0, S.y0, S.x1, S.y1);
    const bool mid = area > kSmallArea && area <= kMidArea, large = area > kMidArea;
    if (__ballot(mid)) {
        const unsigned long long slot = reserve(D.ctr, mid ? 1u : 0u);
        if (mid) D.mid[slot] = k;
    }
    if (__ballot(large)) {
        const uint32_t nb = large ? blocks_of(S) : 0u;
        const unsigned long long first = reserve(D.ctr + 1, nb);
        for (uint32_t b = 0; b < nb; ++b) {
            if (first + b < (unsigned long long)D.cap) {
                D.big[first + b] = make_uint2(k, b);
            } else {  // past the block buffer: test the block here
                const int bx = S.x0 + (int)(b % blocks_x(S)) * kBlockPx, by = S.y0 + (int)(b / blocks_x(S)) * kBlockPx;
                test_box(D, S, v0, e1, e2, bx, by, min(bx + kBlockPx - 1, S.x1), min(by + kBlockPx - 1, S.y1));
            }
        }
    }
}

// One thread per medium triangle.
__global__ __launch_bounds__(kRB) void mid_kernel(const RasterDesc D) {
    const uint32_t n = (uint32_t)D.ctr[0];
    for (uint32_t i = blockIdx.x * kRB + threadIdx.x; i < n; i += gridDim.x * kRB) {
        const uint32_t rec = D.mid[i];
        const float4 v0 = D.tris[3ull * rec], e1 = D.tris[3ull * rec + 1], e2 = D.tris[3ull * rec + 2];
        Screen S;
        if (tri_screen(D, v0, e1, e2, S)) test_box(D, S, v0, e1, e2, S.x0, S.y0, S.x1, S.y1);
    }
}

// One wave per block of a large triangle: its 8 x 8 tiles that come within
// kMargin of the triangle, one pixel per lane.
__global__ __launch_bounds__(kRB) void big_kernel(const RasterDesc D) {
    const uint32_t wave = (blockIdx.x * kRB + threadIdx.x) >> 6, n_waves = (gridDim.x * kRB) >> 6;
    const uint32_t lane = threadIdx.x & 63;
    const unsigned long long nc = D.ctr[1];
    const uint32_t n = nc < (unsigned long long)D.cap ? (uint32_t)nc : D.cap;
    for (uint32_t i = wave; i < n; i += n_waves) {
        const uint2 e = D.big[i];
        const float4 v0 = D.tris[3ull * e.x], e1 = D.tris[3ull * e.x + 1], e2 = D.tris[3ull * e.x + 2];
        Screen S;
        if (!tri_screen(D, v0, e1, e2, S)) continue;
        const int bx = S.x0 + (int)(e.y % blocks_x(S)) * kBlockPx, by = S.y0 + (int)(e.y / blocks_x(S)) * kBlockPx;
        const int bx1 = min(bx + kBlockPx - 1, S.x1), by1 = min(by + kBlockPx - 1, S.y1);
        const float3 eye = cam_vec(D.cur.eye);
        for (int ty = by; ty <= by1; ty += 8)
            for (int tx = bx; tx <= bx1; tx += 8) {
                if (!near_tile(S, tx, ty, min(tx + 7, bx1), min(ty + 7, by1))) continue;
                const int x = tx + (int)(lane & 7), y = ty + (int)(lane >> 3);
                if (x <= bx1 && y <= by1 && near_pixel(S, x, y)) test_pixel(D, eye, v0, e1, e2, x, y);
            }
    }
}

__global__ __launch_bounds__(kRB) void resolve_kernel(const RasterDesc D) {
    const uint32_t i = blockIdx.x * kRB + threadIdx.x;
    if (i >= D.W * D.H) return;
    const uint32_t x = i % D.W, y = i / D.W;
    const unsigned long long k = D.key[i];
    const float3 d = cam_dir(D.cur, x + 0.5f, y + 0.5f);
    const float4* rec = k == ~0ull ? nullptr : D.tris + 3ull * D.rec_of[(uint32_t)k];
    gbuffer_texel(D.cur, D.prev, D.has_prev != 0, D.W, D.H, x, y, d, rec, __uint_as_float((uint32_t)(k >> 32)),
                  D.pos[i], D.nz[i], D.dz[i], D.mv[i]);
}

// Capacity for large-triangle blocks: half the triangle count plus one per
// 16 pixels (blocks beyond it are tested by the projecting thread).
uint64_t block_cap(uint32_t W, uint32_t H, uint32_t T) { return (uint64_t)W * H / 16 + T / 2 + 64; }

// Workspace layout: keys, medium list, blocks, counters, each region on a
// 256-byte boundary (the 64-bit atomics need 8-byte alignment).
struct RasterLayout {
    uint64_t key, mid, big, ctr, total;
};
constexpr uint64_t round256(uint64_t b) { return (b + 255) & ~255ull; }
RasterLayout raster_layout(uint32_t W, uint32_t H, uint32_t T) {
    RasterLayout L;
    const uint64_t HW = (uint64_t)W * H;
    L.key = 0;
    L.mid = L.key + round256(8 * HW);
    L.big = L.mid + round256(4ull * T);
    L.ctr = L.big + round256(8 * block_cap(W, H, T));
    L.total = L.ctr + 256;
    return L;
}

uint64_t raster_workspace(uint32_t W, uint32_t H, uint32_t T) { return raster_layout(W, H, T).total; }

}  // namespace
}  // namespace dhr

extern "C" {

uint64_t dhr_gbuffer_raster_workspace_bytes(uint32_t W, uint32_t H, uint32_t n_tris) {
    return dhr::raster_workspace(W, H, n_tris);
}

dhr_status dhr_gbuffer_raster(dhr_ctx* ctx, const dhr_bvh* bvh, const dhr_camera* cur, const dhr_camera* prev,
                              uint32_t W, uint32_t H, float* pos, float* nz, float* dz, float* mv, void* work,
                              uint64_t work_bytes, dhr_stream stream) {
    using namespace dhr;
    if (!ctx) return DHR_ERR_INVALID_ARG;
    const char* what = "dhr_gbuffer_raster";
    if (!bvh || bvh->ctx != ctx) return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: bad bvh", what);
    if (bvh->tl || !bvh->rec_of)
        return set_error(ctx, DHR_ERR_UNSUPPORTED, "%s: two-level hierarchies are traced, not rasterised", what);
    if (!cur) return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: camera is NULL", what);
    if (W < 1 || H < 1 || W > DHR_MAX_SIDE || H > DHR_MAX_SIDE)
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: image %ux%u outside 1..16384", what, W, H);
    if (!pos || !nz || !dz || !mv || !work || !aligned16(pos) || !aligned16(nz) || !aligned8(dz) || !aligned8(mv) ||
        !aligned16(work))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: null or misaligned buffer", what);
    const uint32_t T = (uint32_t)bvh->info.n_tris;
    if (work_bytes < raster_workspace(W, H, T))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: work holds %llu bytes, %llu needed", what,
                         (unsigned long long)work_bytes, (unsigned long long)raster_workspace(W, H, T));
    RasterDesc D;
    std::memset(&D, 0, sizeof D);
    if (!make_cam(*cur, W, H, &D.cur) || (prev && !make_cam(*prev, W, H, &D.prev)))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: degenerate camera", what);
    D.tris = bvh->tris;
    D.rec_of = bvh->rec_of;
    D.T = T;
    D.W = W;
    D.H = H;
    D.has_prev = prev ? 1u : 0u;
    // clip distance and the eye neighbourhood it leaves out (cosine of the
    // frame's corner ray: 1 / |(1, tx, ty)|)
    const double em = std::max({std::fabs((double)cur->eye[0]), std::fabs((double)cur->eye[1]),
                                std::fabs((double)cur->eye[2]), 1.0});
    const double zn = 1e-5 * em;
    const double cmin = 1.0 / std::sqrt(1.0 + (double)D.cur.tx * D.cur.tx + (double)D.cur.ty * D.cur.ty);
    D.near_z = (float)zn;
    D.inv_tx = (float)(1.0 / (double)D.cur.tx);
    D.inv_ty = (float)(1.0 / (double)D.cur.ty);
    D.near_r = (float)(1.01 * zn / cmin);
    char* w = static_cast<char*>(work);
    const uint64_t HW = (uint64_t)W * H;
    const RasterLayout L = raster_layout(W, H, T);
    D.key = reinterpret_cast<unsigned long long*>(w + L.key);
    D.mid = reinterpret_cast<uint32_t*>(w + L.mid);
    D.big = reinterpret_cast<uint2*>(w + L.big);
    D.cap = (uint32_t)block_cap(W, H, T);
    D.ctr = reinterpret_cast<unsigned long long*>(w + L.ctr);
    if (!aligned16(D.key) || !aligned16(D.mid) || !aligned16(D.big) || !aligned16(D.ctr))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: workspace layout misaligned", what);
    D.pos = reinterpret_cast<float4*>(pos);
    D.nz = reinterpret_cast<float4*>(nz);
    D.dz = reinterpret_cast<float2*>(dz);
    D.mv = reinterpret_cast<float2*>(mv);
    DeviceGuard g(ctx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uint32_t pix_blocks = (uint32_t)((HW + kRB - 1) / kRB);
    const uint32_t wave_blocks = (uint32_t)std::max(ctx->n_cu, 1) * 8;
    hipLaunchKernelGGL(clear_kernel, dim3(pix_blocks), dim3(kRB), 0, s, D);
    hipLaunchKernelGGL(setup_kernel, dim3((T + kRB - 1) / kRB), dim3(kRB), 0, s, D);
    hipLaunchKernelGGL(mid_kernel, dim3(wave_blocks), dim3(kRB), 0, s, D);
    hipLaunchKernelGGL(big_kernel, dim3(wave_blocks), dim3(kRB), 0, s, D);
    hipLaunchKernelGGL(resolve_kernel, dim3(pix_blocks), dim3(kRB), 0, s, D);
    return check_launch(ctx, what);
}

}  // extern "C"
