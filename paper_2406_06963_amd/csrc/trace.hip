// Ray kernels: the G-buffer of primary rays and the stochastic visibility
// rays (ambient occlusion, Section 3.2; soft shadows, Section 3.1).
//
// Layout: a 128-lane workgroup covers a 16 x 8 pixel tile; a wave's 64 rays
// traverse the tree together (one walk per wave, the stack one LDS column per
// wave): one ray of each pixel of an 8 x 8 square, or, for a stream with an
// even ray count, P rays of each pixel of an 8 x 8/P block.  Jobs of a ragged
// batch are passed by value in the kernel arguments.
#include <cmath>
#include <cstring>
#include <vector>

#include "camera.h"
#include "device.h"
#include "internal.h"

namespace dhr {
namespace {

// A workgroup of kWaves waves covers a kTileW x 8 pixel tile.  Its
// visibility rays come from one 8 x 8 square per wave, squares side by side
// (a square's hit points keep the union of the wave's paths short).  Its
// primary rays come from one kPX x kPY rectangle per wave.  Rectangles wider
// than tall suit primary rays: near a horizon the rows of a square reach
// very different distances, while a strip's pixels stay at one elevation.
// The G-buffer texels pass from one layout to the other through LDS, indexed
// by the pixel's place in the tile.  (One and four waves per workgroup with
// 8 x 8 primary squares measured slower than two on the 1080p terrain.)
#ifndef DHR_PRIMARY_W
#define DHR_PRIMARY_W 16
#endif
#ifndef DHR_WAVES
#define DHR_WAVES 2
#endif
constexpr int kWaves = DHR_WAVES, kBlock = 64 * kWaves, kTileW = 8 * kWaves, kTileH = 8;
constexpr int kPX = DHR_PRIMARY_W, kPY = 64 / kPX, kPWavesX = kTileW / kPX;
static_assert(kPX * kPY == 64 && kPWavesX >= 1 && kPWavesX * (kTileH / kPY) == kWaves,
              "primary-ray rectangles must tile the workgroup");

struct LightD {
    uint32_t kind;
    float v[3];
    float k;
    float radius;
};

struct TraceDesc {
    const float4* nodes;
    const float4* tris;
    const TwoLevel* tl;  // two-level hierarchies: instances and bottom levels (device)
    const float4* pos;
    const float4* nz;
    uint8_t* ao;
    uint8_t* sh;
    uint64_t* bits;
    uint32_t W, H, tiles_x, frame, client, seed, n_ao, ao_off, n_shadow, n_lights;
    float ao_r, eps_abs;
    LightD lights[DHR_MAX_LIGHTS];
};
static_assert(sizeof(TwoLevel) == sizeof(TwoLevelHost) && alignof(TwoLevel) == alignof(TwoLevelHost),
              "the host image of the two-level description must match the kernels'");
constexpr int kTraceMaxB = 12;
using TraceBatch = Batch<TraceDesc, kTraceMaxB>;
static_assert(sizeof(TraceBatch) <= 4000, "kernel arguments too large");

struct GbufDesc {
    const float4* nodes;
    const float4* tris;
    const TwoLevel* tl;
    float4* pos;
    float4* nz;
    float2* dz;
    float2* mv;
    uint32_t W, H, tiles_x, has_prev;
    CamD cur, prev;
};
constexpr int kGbufMaxB = 16;
using GbufBatch = Batch<GbufDesc, kGbufMaxB>;
static_assert(sizeof(GbufBatch) <= 4000, "kernel arguments too large");

// This lane's pixel of tile t in the visibility layout (8 x 8 squares)
// and in the primary-ray layout (kPX x kPY rectangles); `slot` is the
// pixel's place in the tile, y kTileW + x.
__device__ __forceinline__ void vis_pixel(uint32_t t, uint32_t tiles_x, uint32_t& x, uint32_t& y, uint32_t& slot) {
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t lx = w * 8 + (lane & 7), ly = lane >> 3;
    x = (t % tiles_x) * kTileW + lx;
    y = (t / tiles_x) * kTileH + ly;
    slot = ly * kTileW + lx;
}
__device__ __forceinline__ void prim_pixel(uint32_t t, uint32_t tiles_x, uint32_t& x, uint32_t& y, uint32_t& slot) {
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t lx = (w % kPWavesX) * kPX + lane % kPX, ly = (w / kPWavesX) * kPY + lane / kPX;
    x = (t % tiles_x) * kTileW + lx;
    y = (t / tiles_x) * kTileH + ly;
    slot = ly * kTileW + lx;
}

// Ray `sample` of stream st (0 = AO, l + 1 = light l) of pixel (x, y) with
// offset origin o and normal n.  `decided` rays need no tracing: invalid
// pixels, points inside a sphere light (unoccluded), light behind the
// surface (occluded); `occ` then holds the answer.
__device__ __forceinline__ void make_ray(const TraceDesc& D, uint32_t st, uint32_t sample, uint32_t x, uint32_t y,
                                         float3 o, float3 n, bool valid, Ray& r, bool& decided, bool& occ) {
    occ = true;
    decided = !valid;
    r.o = o;
    r.d = n;
    r.tmax = 0.0f;
    if (!valid) return;
    const float2 u = ray_uniforms(D.seed, D.client, x, y, D.frame, st, st == 0 ? D.ao_off + sample : sample);
    if (st == 0) {
        r.d = sample_cosine(n, u.x, u.y);
        r.tmax = D.ao_r;
        return;
    }
    const LightD& L = D.lights[st - 1];
    if (L.kind == 0) {
        r.d = sample_cone(f3(L.v[0], L.v[1], L.v[2]), L.k, u.x, u.y);
        r.tmax = __builtin_inff();
    } else {
        const float3 Dv = f3(L.v[0], L.v[1], L.v[2]) - o;
        const float dist = sqrtf(dot3(Dv, Dv));
        if (dist <= L.radius) {
            decided = true;
            occ = false;
            return;
        }
        const float3 axis = Dv * (1.0f / dist);
        const float rr = L.radius / dist;
        const float q = rr * rr;
        const float k = q / (1.0f + sqrtf(1.0f - q));
        r.d = sample_cone(axis, k, u.x, u.y);
        const float b = dot3(r.d, Dv);
        const float c = dist * dist - L.radius * L.radius;
        r.tmax = b - sqrtf(fmaxf(b * b - c, 0.0f));
    }
    if (dot3(n, r.d) <= 0.0f) {
        decided = true;
        occ = true;
    }
}

// Rays of one pixel a stream traces side by side in one wave: the largest
// power of two up to 8 that divides the stream's ray count.  A wave then
// covers 64 / P pixels (an 8 x 8/P block) with P rays each, whose paths
// through the tree overlap more than those of 64 pixels one ray apart.
__device__ __forceinline__ uint32_t pack_of(uint32_t nr) {
    return (nr % 8 == 0) ? 8 : (nr % 4 == 0) ? 4 : (nr % 2 == 0) ? 2 : 1;
}

// Workgroup LDS of the visibility pass: the stack columns of its waves (two
// per wave for two-level hierarchies), and the block's ray origins, normals
// and per-pixel counts.
template <bool TWO_LEVEL>
struct TraceShared {
    int stack[kStack * (kBlock / 64) * (TWO_LEVEL ? 2 : 1)];
    float4 s_o[kBlock];   // the block's ray origins, w = 1 for a valid pixel
    float4 s_n[kBlock];   // and normals
    uint32_t s_cnt[kBlock];
    unsigned long long s_bits[kBlock];
};

// The visibility rays of one kTileW x 8 block (tile t of job D).  This lane
// brings the G-buffer texel p4, n4 of the pixel at tile slot `ps` (`in_p`
// false beyond the image) and traces for its pixel (x, y) of the visibility
// layout (slot vs, index i; `inside` false beyond the image).  Every lane
// of the workgroup takes part (barriers).  With COUNT, tc and n_rays tally
// this lane's work.
template <bool COUNT, bool TWO_LEVEL, bool WIDE>
__device__ __forceinline__ void trace_block(const TraceDesc& D, uint32_t t, uint32_t ps, bool in_p, float4 p4,
                                            float4 n4, uint32_t x, uint32_t y, uint32_t vs, bool inside, size_t i,
                                            TraceShared<TWO_LEVEL>& S, TravCount& tc, uint32_t& n_rays) {
    const uint32_t tx0 = (t % D.tiles_x) * kTileW, ty0 = (t / D.tiles_x) * kTileH;
    const size_t HW = (size_t)D.W * D.H;
    const bool valid = in_p && n4.w > 0.0f;
    const float3 n = f3(n4);
    const float3 p = f3(p4);
    float eps = D.eps_abs;
    if (!(eps > 0.0f)) eps = fmaxf(1e-3f * D.ao_r, fmaxf(fmaxf(fabsf(p.x), fabsf(p.y)), fabsf(p.z)) * 0x1p-17f);
    const float3 o = p + n * eps;
    S.s_o[ps] = make_float4(o.x, o.y, o.z, valid ? 1.0f : 0.0f);
    S.s_n[ps] = make_float4(n.x, n.y, n.z, 0.0f);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int* wstk = S.stack + w * kStack;
    int* wstk2 = S.stack + (TWO_LEVEL ? (kBlock / 64 + w) * kStack : 0);
    TwoLevel L{};
    if (TWO_LEVEL) L = *D.tl;

    for (uint32_t st = 0; st <= D.n_lights; ++st) {
        const uint32_t nr = st == 0 ? D.n_ao : D.n_shadow;
        const uint32_t P = pack_of(nr);
        uint32_t cnt = 0;
        uint64_t bits = 0;
        if (P > 1) {
            S.s_cnt[threadIdx.x] = 0;
            S.s_bits[threadIdx.x] = 0;
            __syncthreads();
        }
        for (uint32_t it = 0; it < nr; ++it) {
            // P == 1: ray `it` of the lane's own pixel.  P > 1: step it of the
            // stream covers block b = kWaves (it % P) + w of the tile (8 x 8/P
            // pixels of the wave's own square), P rays of each pixel, counted
            // in LDS.
            uint32_t src = vs, s = it, px = x, py = y;
            if (P > 1) {
                const uint32_t b = kWaves * (it % P) + w, q = lane / P;
                const uint32_t lx = (b % kWaves) * 8 + q % 8, ly = (b / kWaves) * (8 / P) + q / 8;
                src = ly * kTileW + lx;
                s = (it / P) * P + lane % P;
                px = tx0 + lx;
                py = ty0 + ly;
            }
            const float4 so = S.s_o[src], sn = S.s_n[src];
            const bool v = so.w > 0.0f;
            Ray r;
            bool decided, occ;
            make_ray(D, st, s, px, py, f3(so), f3(sn), v, r, decided, occ);
            const bool h = TWO_LEVEL ? any_hit_2l(D.nodes, L, r, !decided, wstk, wstk2)
                                     : any_hit<COUNT, WIDE>(D.nodes, D.tris, r, !decided, wstk, &tc);
            if (!decided) occ = h;
            if (COUNT && !decided) ++n_rays;
            if (!v || !occ) {
                if (P == 1) {
                    ++cnt;
                    if (s < 64) bits |= 1ull << s;
                } else {
                    atomicAdd(&S.s_cnt[src], 1u);
                    if (s < 64) atomicOr(&S.s_bits[src], 1ull << s);
                }
            }
        }
        if (P > 1) {
            __syncthreads();
            cnt = S.s_cnt[vs];
            bits = S.s_bits[vs];
        }
        if (inside) {
            if (st == 0)
                D.ao[i] = (uint8_t)cnt;
            else
                D.sh[(size_t)(st - 1) * HW + i] = (uint8_t)cnt;
            if (D.bits) D.bits[(size_t)st * HW + i] = bits;
        }
        __syncthreads();  // s_cnt / s_bits are reused by the next stream
    }
}

// COUNT: the instrumented variant that also tallies rays, node visits, leaf
// visits and triangle tests into `counters` (device uint64[4]).  WIDE: the
// record addressing of single-level trees (device.h; two-level walks are
// always wide).
template <bool COUNT, bool TWO_LEVEL, bool WIDE>
__global__ __launch_bounds__(kBlock) void trace_kernel(const TraceBatch B, unsigned long long* counters) {
    __shared__ TraceShared<TWO_LEVEL> S;
    const int j = find_job(B.tile0, (int)B.n, blockIdx.x);
    const TraceDesc& D = B.d[j];
    const uint32_t t = blockIdx.x - B.tile0[j];
    uint32_t x, y, vs;
    vis_pixel(t, D.tiles_x, x, y, vs);
    const bool inside = x < D.W && y < D.H;
    const size_t i = inside ? (size_t)y * D.W + x : 0;
    TravCount tc;
    uint32_t n_rays = 0;
    trace_block<COUNT, TWO_LEVEL, WIDE>(D, t, vs, inside, D.pos[i], D.nz[i], x, y, vs, inside, i, S, tc, n_rays);
    if (COUNT) {
        // one vector atomic per lane (instrumented runs only)
        atomicAdd(counters + 0, (unsigned long long)n_rays);
        atomicAdd(counters + 1, (unsigned long long)tc.nodes);
        atomicAdd(counters + 2, (unsigned long long)tc.leaves);
        atomicAdd(counters + 3, (unsigned long long)tc.tris);
    }
}

// The G-buffer texel of pixel (x, y) of job D: the closest hit of the ray
// through the pixel centre.  Lanes with live false (beyond the image) take
// part in the walk without a ray.
template <bool TWO_LEVEL, bool WIDE, bool COUNT = false>
__device__ __forceinline__ void texel_of(const GbufDesc& D, uint32_t x, uint32_t y, bool live, int* wstk, int* wstk2,
                                         float4& pos, float4& nz, float2& dz, float2& mv, TravCount* cnt = nullptr) {
    const CamD& C = D.cur;
    const float3 eye = f3(C.eye[0], C.eye[1], C.eye[2]);
    const float3 d = cam_dir(C, x + 0.5f, y + 0.5f);
    float t;
    if (!TWO_LEVEL) {
        const int hit = closest_hit<COUNT, WIDE>(D.nodes, D.tris, eye, d, live, t, wstk, cnt);
        gbuffer_texel(C, D.prev, D.has_prev != 0, D.W, D.H, x, y, d, hit < 0 ? nullptr : D.tris + 3 * hit, t, pos,
                      nz, dz, mv);
        return;
    }
    const TwoLevel L = *D.tl;
    int inst, tri;
    closest_hit_2l(D.nodes, L, eye, d, live, t, inst, tri, wstk, wstk2);
    float4 rec[3];
    if (inst >= 0) {
        // the hit triangle in world space, with the instance's object id
        const float4* I = L.inst + kInstStride * inst;
        const float4 f0 = I[3], f1 = I[4], f2 = I[5], info = I[6];
        const float4* tr = bottom_tris(L, (int)fbits(info.x)) + 3 * tri;
        const float4 v0 = tr[0], e1 = tr[1], e2 = tr[2];
        const float3 w0 = xf_point(f0, f1, f2, f3(v0)), w1 = xf_dir(f0, f1, f2, f3(e1)), w2 = xf_dir(f0, f1, f2, f3(e2));
        const float oid = fbits(info.y) == 0xFFFFFFFFu ? e1.w : info.y;
        rec[0] = make_float4(w0.x, w0.y, w0.z, v0.w);
        rec[1] = make_float4(w1.x, w1.y, w1.z, oid);
        rec[2] = make_float4(w2.x, w2.y, w2.z, 0.0f);
    }
    gbuffer_texel(C, D.prev, D.has_prev != 0, D.W, D.H, x, y, d, inst < 0 ? nullptr : rec, t, pos, nz, dz, mv);
}

template <bool TWO_LEVEL, bool WIDE>
__global__ __launch_bounds__(kBlock) void gbuffer_kernel(const GbufBatch B) {
    __shared__ int stack[kStack * (kBlock / 64) * (TWO_LEVEL ? 2 : 1)];
    const int j = find_job(B.tile0, (int)B.n, blockIdx.x);
    const GbufDesc& D = B.d[j];
    uint32_t x, y, slot;
    prim_pixel(blockIdx.x - B.tile0[j], D.tiles_x, x, y, slot);
    if (x >= D.W || y >= D.H) return;
    const size_t i = (size_t)y * D.W + x;
    int* wstk = stack + (threadIdx.x >> 6) * kStack;
    texel_of<TWO_LEVEL, WIDE>(D, x, y, true, wstk, wstk + (kBlock / 64) * kStack, D.pos[i], D.nz[i], D.dz[i],
                              D.mv[i]);
}

// G-buffer and visibility of a frame in one launch: each workgroup writes the
// texels of its kTileW x 8 block (primary-ray layout), then traces the
// block's visibility rays from them (visibility layout, as trace_kernel).
// The long primary walks of some blocks then overlap other blocks'
// visibility work instead of leaving the device idle behind them.
struct FrameDesc {
    GbufDesc g;
    TraceDesc t;
};
constexpr int kFrameMaxB = 6;
using FrameBatch = Batch<FrameDesc, kFrameMaxB>;
static_assert(sizeof(FrameBatch) <= 4000, "kernel arguments too large");

// COUNT: the instrumented variant (single-level hierarchies), tallying the
// primary and the visibility rays' work into `counters` as trace_kernel does.
template <bool COUNT, bool TWO_LEVEL, bool WIDE>
__global__ __launch_bounds__(kBlock) void frame_kernel(const FrameBatch B, unsigned long long* counters) {
    __shared__ TraceShared<TWO_LEVEL> S;
    const int j = find_job(B.tile0, (int)B.n, blockIdx.x);
    const FrameDesc& F = B.d[j];
    const uint32_t t = blockIdx.x - B.tile0[j];
    uint32_t x, y, ps;
    prim_pixel(t, F.g.tiles_x, x, y, ps);
    const bool inside = x < F.g.W && y < F.g.H;
    const size_t i = inside ? (size_t)y * F.g.W + x : 0;
    const uint32_t w = threadIdx.x >> 6;
    float4 pos, nz;
    float2 dz, mv;
    int* wstk = S.stack + w * kStack;
    TravCount tc;
    texel_of<TWO_LEVEL, WIDE, COUNT>(F.g, x, y, inside, wstk, TWO_LEVEL ? S.stack + (kBlock / 64 + w) * kStack : wstk, pos,
                               nz, dz, mv, &tc);
    if (inside) {
        F.g.pos[i] = pos;
        F.g.nz[i] = nz;
        F.g.dz[i] = dz;
        F.g.mv[i] = mv;
    }
    uint32_t n_rays = inside ? 1 : 0;
    uint32_t vx, vy, vs;
    vis_pixel(t, F.t.tiles_x, vx, vy, vs);
    const bool v_in = vx < F.t.W && vy < F.t.H;
    trace_block<COUNT, TWO_LEVEL, WIDE>(F.t, t, ps, inside, pos, nz, vx, vy, vs, v_in,
                                        v_in ? (size_t)vy * F.t.W + vx : 0, S, tc, n_rays);
    if (COUNT) {
        atomicAdd(counters + 0, (unsigned long long)n_rays);
        atomicAdd(counters + 1, (unsigned long long)tc.nodes);
        atomicAdd(counters + 2, (unsigned long long)tc.leaves);
        atomicAdd(counters + 3, (unsigned long long)tc.tris);
    }
}

__global__ void philox_kernel(uint32_t k0, uint32_t k1, const uint4* __restrict__ ctr, uint4* __restrict__ out,
                              uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = philox4x32_10(ctr[i], k0, k1);
}

// ------------------------------------------------------------------ host side

bool size_ok(uint32_t W, uint32_t H) { return W >= 1 && H >= 1 && W <= DHR_MAX_SIDE && H <= DHR_MAX_SIDE; }

dhr_status check_trace_params(dhr_ctx* ctx, const dhr_trace_params& p) {
    if (!size_ok(p.W, p.H)) return set_error(ctx, DHR_ERR_INVALID_ARG, "trace: image %ux%u outside 1..16384", p.W, p.H);
    if (p.n_ao > 255) return set_error(ctx, DHR_ERR_INVALID_ARG, "trace: n_ao = %u > 255 (the count is one byte)", p.n_ao);
    if (p.n_shadow > 255) return set_error(ctx, DHR_ERR_INVALID_ARG, "trace: n_shadow = %u > 255", p.n_shadow);
    if (p.n_lights > DHR_MAX_LIGHTS) return set_error(ctx, DHR_ERR_INVALID_ARG, "trace: n_lights = %u > 8", p.n_lights);
    if ((uint64_t)p.ao_sample_offset + p.n_ao > 65536)
        return set_error(ctx, DHR_ERR_INVALID_ARG, "trace: AO sample index beyond 65535");
    if (p.n_ao > 0 && !(p.ao_radius > 0.0f && std::isfinite(p.ao_radius)))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "trace: ao_radius must be positive");
    if (!(p.eps_origin_abs >= 0.0f) || !std::isfinite(p.eps_origin_abs))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "trace: eps_origin_abs must be >= 0");
    for (uint32_t l = 0; l < p.n_lights; ++l) {
        const dhr_light& L = p.lights[l];
        bool fin = std::isfinite(L.vec[0]) && std::isfinite(L.vec[1]) && std::isfinite(L.vec[2]);
        if (L.kind == 0) {
            double n2 = (double)L.vec[0] * L.vec[0] + (double)L.vec[1] * L.vec[1] + (double)L.vec[2] * L.vec[2];
            if (!fin || !(n2 > 0.0) || !(L.one_minus_cos >= 0.0f && L.one_minus_cos <= 2.0f))
                return set_error(ctx, DHR_ERR_INVALID_ARG, "trace: light %u: bad direction or cone", l);
        } else if (L.kind == 1) {
            if (!fin || !(L.radius > 0.0f) || !std::isfinite(L.radius))
                return set_error(ctx, DHR_ERR_INVALID_ARG, "trace: light %u: bad sphere", l);
        } else {
            return set_error(ctx, DHR_ERR_INVALID_ARG, "trace: light %u: unknown kind %u", l, L.kind);
        }
    }
    return DHR_OK;
}

void fill_trace_desc(const dhr_bvh* bvh, const dhr_trace_params& p, const float* pos, const float* nz, uint8_t* ao,
                     uint8_t* sh, uint64_t* bits, TraceDesc* d) {
    std::memset(d, 0, sizeof *d);
    d->nodes = bvh->nodes;
    d->tris = bvh->tris;
    d->tl = reinterpret_cast<const TwoLevel*>(bvh->tl);
    d->pos = reinterpret_cast<const float4*>(pos);
    d->nz = reinterpret_cast<const float4*>(nz);
    d->ao = ao;
    d->sh = sh;
    d->bits = bits;
    d->W = p.W;
    d->H = p.H;
    d->tiles_x = (p.W + kTileW - 1) / kTileW;
    d->frame = p.frame;
    d->client = p.client_id;
    d->seed = p.seed;
    d->n_ao = p.n_ao;
    d->ao_off = p.ao_sample_offset;
    d->n_shadow = p.n_shadow;
    d->n_lights = p.n_lights;
    d->ao_r = p.ao_radius;
    d->eps_abs = p.eps_origin_abs;
    for (uint32_t l = 0; l < p.n_lights; ++l) {
        const dhr_light& L = p.lights[l];
        d->lights[l].kind = L.kind;
        d->lights[l].k = L.one_minus_cos;
        d->lights[l].radius = L.radius;
        if (L.kind == 0) {
            double n = std::sqrt((double)L.vec[0] * L.vec[0] + (double)L.vec[1] * L.vec[1] + (double)L.vec[2] * L.vec[2]);
            for (int k = 0; k < 3; ++k) d->lights[l].v[k] = (float)(L.vec[k] / n);
        } else {
            for (int k = 0; k < 3; ++k) d->lights[l].v[k] = L.vec[k];
        }
    }
}

uint32_t tiles_of(uint32_t W, uint32_t H) { return ((W + kTileW - 1) / kTileW) * ((H + kTileH - 1) / kTileH); }

// Launch group of a job's hierarchy: narrow-addressed single level, wide
// single level (node or triangle array beyond 4 GB, or forced by the
// context), two levels.
enum Hier { kNarrow = 0, kWide = 1, kTwoLevel = 2 };
Hier hier_of(const dhr_ctx* ctx, const dhr_bvh* b) {
    if (b->tl) return kTwoLevel;
    const bool fits = b->info.n_nodes <= (1ull << 26) && b->info.n_tris <= (1ull << 26);
    return fits && !ctx->wide_records ? kNarrow : kWide;
}

// Splits jobs (descs[k], tiles[k], hierarchy h[k]) into the three groups.
template <class D>
struct Groups {
    std::vector<D> d[3];
    std::vector<uint32_t> t[3];
    Groups(const std::vector<D>& descs, const std::vector<uint32_t>& tiles, const std::vector<Hier>& h) {
        for (size_t k = 0; k < descs.size(); ++k) {
            d[h[k]].push_back(descs[k]);
            t[h[k]].push_back(tiles[k]);
        }
    }
};

template <class D, int MAXB, class K, class... Extra>
dhr_status launch_batches(dhr_ctx* ctx, const std::vector<D>& descs, const std::vector<uint32_t>& tiles, K kernel,
                          int block, hipStream_t s, const char* what, Extra... extra) {
    for (size_t b = 0; b < descs.size(); b += MAXB) {
        Batch<D, MAXB> B;
        std::memset(&B, 0, sizeof B);
        const size_t n = std::min<size_t>(MAXB, descs.size() - b);
        B.n = (uint32_t)n;
        uint64_t acc = 0;
        for (size_t k = 0; k < n; ++k) {
            B.tile0[k] = (uint32_t)acc;
            B.d[k] = descs[b + k];
            acc += tiles[b + k];
        }
        B.tile0[n] = (uint32_t)acc;
        if (acc == 0) continue;
        if (acc > 0x7FFFFFFFull) return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: batch too large", what);
        hipLaunchKernelGGL(kernel, dim3((uint32_t)acc), dim3(block), 0, s, B, extra...);
        dhr_status st = check_launch(ctx, what);
        if (st != DHR_OK) return st;
    }
    return DHR_OK;
}

dhr_status trace_desc_of(dhr_ctx* ctx, const dhr_trace_job& J, uint32_t k, uint64_t* bits, const char* what,
                         TraceDesc* d) {
    if (!J.bvh || J.bvh->ctx != ctx) return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: job %u: bad bvh", what, k);
    dhr_status st = check_trace_params(ctx, J.params);
    if (st != DHR_OK) return st;
    if (!J.pos || !J.nz || !J.ao_count || !aligned16(J.pos) || !aligned16(J.nz))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: job %u: null or misaligned buffer", what, k);
    if (J.params.n_lights > 0 && !J.shadow_count)
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: job %u: shadow_count is NULL", what, k);
    if (bits && (J.params.n_ao > 64 || J.params.n_shadow > 64 || !aligned8(bits)))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: debug_ray_bits needs n <= 64 rays per stream", what);
    fill_trace_desc(J.bvh, J.params, J.pos, J.nz, J.ao_count, J.shadow_count, bits, d);
    return DHR_OK;
}

dhr_status trace_jobs(dhr_ctx* ctx, const dhr_trace_job* jobs, uint32_t n, const uint64_t* const* bits_per_job,
                      dhr_stream stream, const char* what) {
    std::vector<TraceDesc> descs(n);
    std::vector<uint32_t> tiles(n);
    for (uint32_t k = 0; k < n; ++k) {
        uint64_t* bits = bits_per_job ? const_cast<uint64_t*>(bits_per_job[k]) : nullptr;
        dhr_status st = trace_desc_of(ctx, jobs[k], k, bits, what, &descs[k]);
        if (st != DHR_OK) return st;
        tiles[k] = tiles_of(jobs[k].params.W, jobs[k].params.H);
    }
    std::vector<Hier> h(n);
    for (uint32_t k = 0; k < n; ++k) h[k] = hier_of(ctx, jobs[k].bvh);
    DeviceGuard g(ctx->device);
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(ctx->trace_counters);
    // one launch sequence per hierarchy kind
    const Groups<TraceDesc> G(descs, tiles, h);
    if (cnt && !G.d[kTwoLevel].empty())
        return set_error(ctx, DHR_ERR_UNSUPPORTED, "%s: work counters cover single-level hierarchies only", what);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    dhr_status st = DHR_OK;
    auto go = [&](Hier k, auto kernel) {
        if (st == DHR_OK && !G.d[k].empty())
            st = launch_batches<TraceDesc, kTraceMaxB>(ctx, G.d[k], G.t[k], kernel, kBlock, s, what, cnt);
    };
    if (cnt) {
        go(kNarrow, trace_kernel<true, false, false>);
        go(kWide, trace_kernel<true, false, true>);
    } else {
        go(kNarrow, trace_kernel<false, false, false>);
        go(kWide, trace_kernel<false, false, true>);
    }
    go(kTwoLevel, trace_kernel<false, true, true>);
    return st;
}

dhr_status gbuf_desc_of(dhr_ctx* ctx, const dhr_gbuffer_job& J, uint32_t k, const char* what, GbufDesc* dp) {
    if (!J.bvh || J.bvh->ctx != ctx) return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: job %u: bad bvh", what, k);
    if (!size_ok(J.W, J.H)) return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: image %ux%u outside 1..16384", what, J.W, J.H);
    if (!J.pos || !J.nz || !J.dz || !J.mv || !aligned16(J.pos) || !aligned16(J.nz) || !aligned8(J.dz) ||
        !aligned8(J.mv))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: job %u: null or misaligned buffer", what, k);
    GbufDesc& d = *dp;
    std::memset(&d, 0, sizeof d);
    if (!make_cam(J.cur, J.W, J.H, &d.cur) || (J.has_prev && !make_cam(J.prev, J.W, J.H, &d.prev)))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: job %u: degenerate camera", what, k);
    d.nodes = J.bvh->nodes;
    d.tris = J.bvh->tris;
    d.tl = reinterpret_cast<const TwoLevel*>(J.bvh->tl);
    d.pos = reinterpret_cast<float4*>(J.pos);
    d.nz = reinterpret_cast<float4*>(J.nz);
    d.dz = reinterpret_cast<float2*>(J.dz);
    d.mv = reinterpret_cast<float2*>(J.mv);
    d.W = J.W;
    d.H = J.H;
    d.tiles_x = (J.W + kTileW - 1) / kTileW;
    d.has_prev = J.has_prev ? 1u : 0u;
    return DHR_OK;
}

dhr_status gbuffer_jobs(dhr_ctx* ctx, const dhr_gbuffer_job* jobs, uint32_t n, dhr_stream stream, const char* what) {
    std::vector<GbufDesc> descs(n);
    std::vector<uint32_t> tiles(n);
    for (uint32_t k = 0; k < n; ++k) {
        dhr_status st = gbuf_desc_of(ctx, jobs[k], k, what, &descs[k]);
        if (st != DHR_OK) return st;
        tiles[k] = tiles_of(jobs[k].W, jobs[k].H);
    }
    std::vector<Hier> h(n);
    for (uint32_t k = 0; k < n; ++k) h[k] = hier_of(ctx, jobs[k].bvh);
    DeviceGuard g(ctx->device);
    const Groups<GbufDesc> G(descs, tiles, h);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    dhr_status st = DHR_OK;
    auto go = [&](Hier k, auto kernel) {
        if (st == DHR_OK && !G.d[k].empty())
            st = launch_batches<GbufDesc, kGbufMaxB>(ctx, G.d[k], G.t[k], kernel, kBlock, s, what);
    };
    go(kNarrow, gbuffer_kernel<false, false>);
    go(kWide, gbuffer_kernel<false, true>);
    go(kTwoLevel, gbuffer_kernel<true, true>);
    return st;
}

// Job k's G-buffer and its visibility in one launch (frame_kernel): the
// visibility job must read the G-buffer job's own pos and nz, at its size,
// through the same hierarchy.
dhr_status frame_jobs(dhr_ctx* ctx, const dhr_gbuffer_job* gj, const dhr_trace_job* tj, uint32_t n, dhr_stream stream,
                      const char* what) {
    std::vector<FrameDesc> descs(n);
    std::vector<uint32_t> tiles(n);
    for (uint32_t k = 0; k < n; ++k) {
        dhr_status st = gbuf_desc_of(ctx, gj[k], k, what, &descs[k].g);
        if (st != DHR_OK) return st;
        st = trace_desc_of(ctx, tj[k], k, nullptr, what, &descs[k].t);
        if (st != DHR_OK) return st;
        if (tj[k].bvh != gj[k].bvh || tj[k].params.W != gj[k].W || tj[k].params.H != gj[k].H ||
            tj[k].pos != gj[k].pos || tj[k].nz != gj[k].nz)
            return set_error(ctx, DHR_ERR_INVALID_ARG,
                             "%s: job %u: visibility must read the G-buffer's own pos and nz (same bvh and size)",
                             what, k);
        tiles[k] = tiles_of(gj[k].W, gj[k].H);
    }
    std::vector<Hier> h(n);
    for (uint32_t k = 0; k < n; ++k) h[k] = hier_of(ctx, gj[k].bvh);
    DeviceGuard g(ctx->device);
    const Groups<FrameDesc> G(descs, tiles, h);
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(ctx->trace_counters);
    if (cnt && !G.d[kTwoLevel].empty())
        return set_error(ctx, DHR_ERR_UNSUPPORTED, "%s: work counters cover single-level hierarchies only", what);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    dhr_status st = DHR_OK;
    auto go = [&](Hier k, auto kernel) {
        if (st == DHR_OK && !G.d[k].empty())
            st = launch_batches<FrameDesc, kFrameMaxB>(ctx, G.d[k], G.t[k], kernel, kBlock, s, what, cnt);
    };
    if (cnt) {
        go(kNarrow, frame_kernel<true, false, false>);
        go(kWide, frame_kernel<true, false, true>);
    } else {
        go(kNarrow, frame_kernel<false, false, false>);
        go(kWide, frame_kernel<false, false, true>);
    }
    go(kTwoLevel, frame_kernel<false, true, true>);
    return st;
}

}  // namespace
}  // namespace dhr

extern "C" {

dhr_status dhr_trace_visibility(dhr_ctx* ctx, const dhr_bvh* bvh, const dhr_trace_params* params, const float* pos,
                                const float* nz, uint8_t* ao_count, uint8_t* shadow_count, uint64_t* debug_ray_bits,
                                dhr_stream stream) {
    if (!ctx) return DHR_ERR_INVALID_ARG;
    if (!params) return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_trace_visibility: params is NULL");
    dhr_trace_job job{bvh, *params, pos, nz, ao_count, shadow_count};
    const uint64_t* bits[1] = {debug_ray_bits};
    return dhr::trace_jobs(ctx, &job, 1, bits, stream, "dhr_trace_visibility");
}

dhr_status dhr_trace_visibility_batch(dhr_ctx* ctx, const dhr_trace_job* jobs, uint32_t n_jobs, dhr_stream stream) {
    if (!ctx) return DHR_ERR_INVALID_ARG;
    if (!jobs && n_jobs) return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_trace_visibility_batch: jobs is NULL");
    return dhr::trace_jobs(ctx, jobs, n_jobs, nullptr, stream, "dhr_trace_visibility_batch");
}

dhr_status dhr_gbuffer(dhr_ctx* ctx, const dhr_bvh* bvh, const dhr_camera* cur, const dhr_camera* prev, uint32_t W,
                       uint32_t H, float* pos, float* nz, float* dz, float* mv, dhr_stream stream) {
    if (!ctx) return DHR_ERR_INVALID_ARG;
    if (!cur) return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_gbuffer: camera is NULL");
    dhr_gbuffer_job job;
    std::memset(&job, 0, sizeof job);
    job.bvh = bvh;
    job.cur = *cur;
    if (prev) job.prev = *prev;
    job.has_prev = prev != nullptr;
    job.W = W;
    job.H = H;
    job.pos = pos;
    job.nz = nz;
    job.dz = dz;
    job.mv = mv;
    return dhr::gbuffer_jobs(ctx, &job, 1, stream, "dhr_gbuffer");
}

dhr_status dhr_gbuffer_batch(dhr_ctx* ctx, const dhr_gbuffer_job* jobs, uint32_t n_jobs, dhr_stream stream) {
    if (!ctx) return DHR_ERR_INVALID_ARG;
    if (!jobs && n_jobs) return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_gbuffer_batch: jobs is NULL");
    return dhr::gbuffer_jobs(ctx, jobs, n_jobs, stream, "dhr_gbuffer_batch");
}

dhr_status dhr_gbuffer_trace(dhr_ctx* ctx, const dhr_bvh* bvh, const dhr_camera* cur, const dhr_camera* prev,
                             uint32_t W, uint32_t H, const dhr_trace_params* params, float* pos, float* nz, float* dz,
                             float* mv, uint8_t* ao_count, uint8_t* shadow_count, dhr_stream stream) {
    if (!ctx) return DHR_ERR_INVALID_ARG;
    if (!cur || !params) return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_gbuffer_trace: camera or params is NULL");
    dhr_gbuffer_job g;
    std::memset(&g, 0, sizeof g);
    g.bvh = bvh;
    g.cur = *cur;
    if (prev) g.prev = *prev;
    g.has_prev = prev != nullptr;
    g.W = W;
    g.H = H;
    g.pos = pos;
    g.nz = nz;
    g.dz = dz;
    g.mv = mv;
    dhr_trace_job t{bvh, *params, pos, nz, ao_count, shadow_count};
    return dhr::frame_jobs(ctx, &g, &t, 1, stream, "dhr_gbuffer_trace");
}

dhr_status dhr_gbuffer_trace_batch(dhr_ctx* ctx, const dhr_gbuffer_job* gbuffer_jobs, const dhr_trace_job* trace_jobs,
                                   uint32_t n_jobs, dhr_stream stream) {
    if (!ctx) return DHR_ERR_INVALID_ARG;
    if ((!gbuffer_jobs || !trace_jobs) && n_jobs)
        return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_gbuffer_trace_batch: jobs is NULL");
    return dhr::frame_jobs(ctx, gbuffer_jobs, trace_jobs, n_jobs, stream, "dhr_gbuffer_trace_batch");
}

dhr_status dhr_philox4x32_10(dhr_ctx* ctx, uint32_t k0, uint32_t k1, const uint32_t* ctr, uint32_t* out, uint64_t n,
                             dhr_stream stream) {
    if (!ctx) return DHR_ERR_INVALID_ARG;
    if (n == 0) return DHR_OK;
    if (!ctr || !out || !dhr::aligned16(ctr) || !dhr::aligned16(out) || n > (1ull << 36))
        return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_philox4x32_10: bad buffers or size");
    dhr::DeviceGuard g(ctx->device);
    const uint32_t blocks = (uint32_t)((n + 255) / 256);
    hipLaunchKernelGGL(dhr::philox_kernel, dim3(blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), k0, k1,
                       reinterpret_cast<const uint4*>(ctr), reinterpret_cast<uint4*>(out), n);
    return dhr::check_launch(ctx, "dhr_philox4x32_10");
}

dhr_status dhr_set_trace_counters(dhr_ctx* ctx, uint64_t* counters) {
    if (!ctx) return DHR_ERR_INVALID_ARG;
    if (counters && !dhr::aligned8(counters))
        return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_set_trace_counters: misaligned buffer");
    ctx->trace_counters = counters;
    return DHR_OK;
}

}  // extern "C"
