// Modified SVGF forward (Section 3.3): temporal accumulation, variance
// estimate and the iterated a-trous levels.  One lane per pixel, 16 x 16
// pixel workgroups; every pass covers a ragged batch of frames in one launch.
#include <cmath>
#include <cstring>
#include <vector>

#include "svgf_common.h"

namespace dhr {
namespace {

// History tap consistency: the normal test and the distance of the tap's
// world position from the current tangent plane, in pixel footprints.  The
// decision is discrete, so its arithmetic is pinned to fp32 in this order.
__device__ __forceinline__ bool tap_consistent(float3 n, float3 p, float z, float4 m, float4 pp, float cos_min,
                                               float plane_px, float pix) {
#pragma clang fp contract(off)
    const float dn = __builtin_fmaf(n.x, m.x, __builtin_fmaf(n.y, m.y, n.z * m.z));
    if (!(dn >= cos_min)) return false;
    const float dx = pp.x - p.x;
    const float dy = pp.y - p.y;
    const float dzz = pp.z - p.z;
    const float dpl = fabsf(__builtin_fmaf(n.x, dx, __builtin_fmaf(n.y, dy, n.z * dzz)));
    const float thr = (plane_px * pix) * z;
    return dpl <= thr;
}

__global__ __launch_bounds__(kSvgfBlock) void temporal_kernel(const SvgfBatch B, const SvgfK P) {
    const int j = find_job(B.tile0, (int)B.n, blockIdx.x);
    const SvgfDesc& D = B.d[j];
    uint32_t x, y;
    tile_xy(blockIdx.x - B.tile0[j], D.tiles_x, x, y);
    if (x >= D.W || y >= D.H) return;
    const size_t i = (size_t)y * D.W + x;
    const float4 n4 = D.nz[i];
    if (!(n4.w > 0.0f)) {
        D.hist_out[i] = make_float4(1.0f, 1.0f, 1.0f, 0.0f);
        return;
    }
    // The blend and the moving averages run in FP64 and are rounded once to
    // the fp32 history: the variance downstream is a difference of moments
    // whose square root amplifies any rounding left in them.
    const double xs = (double)D.ao[i] / (double)D.n_ao;
    const float4 p4 = D.pos[i];
    const float2 mv = D.mv[i];
    bool any = false;
    double wsum = 0.0, c = 0.0, m1 = 0.0, m2 = 0.0;
    float hmax = 0.0f;
    if (D.hist_in && isfinite(mv.x) && isfinite(mv.y)) {
        const float flx = floorf(mv.x), fly = floorf(mv.y);
        const float fx = mv.x - flx, fy = mv.y - fly;
        const float X0 = (float)x + flx, Y0 = (float)y + fly;
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (k == 1 ? !(fx > 0.0f) : !(fx < 1.0f)) continue;
                if (jj == 1 ? !(fy > 0.0f) : !(fy < 1.0f)) continue;
                const float tx = X0 + (float)k, ty = Y0 + (float)jj;
                if (!(tx >= 0.0f && tx < (float)D.W && ty >= 0.0f && ty < (float)D.H)) continue;
                const size_t q = (size_t)ty * D.W + (size_t)tx;
                const float4 pn = D.prev_nz[q];
                if (!(pn.w > 0.0f)) continue;
                const float4 hq = D.hist_in[q];
                if (!(hq.w > 0.0f)) continue;
                const float4 pp = D.prev_pos[q];
                if (P.use_obj && fbits(pp.w) != fbits(p4.w)) continue;
                if (!tap_consistent(f3(n4), f3(p4), n4.w, pn, pp, P.cos_min, P.plane_px, D.pix)) continue;
                const double b = (k ? (double)fx : 1.0 - (double)fx) * (jj ? (double)fy : 1.0 - (double)fy);
                any = true;
                wsum += b;
                c = fma(b, (double)hq.x, c);
                m1 = fma(b, (double)hq.y, m1);
                m2 = fma(b, (double)hq.z, m2);
                hmax = fmaxf(hmax, hq.w);
            }
        }
    }
    float4 h;
    if (any) {
        c /= wsum;
        m1 /= wsum;
        m2 /= wsum;
        const double hl = fmin((double)hmax + 1.0, (double)P.cap);
        const double a = fmax((double)P.alpha, 1.0 / hl);
        const double am = fmax((double)P.alpha_m, 1.0 / hl);
        h = make_float4((float)fma(a, xs - c, c), (float)fma(am, xs - m1, m1), (float)fma(am, xs * xs - m2, m2),
                        (float)hl);
    } else {
        h = make_float4((float)xs, (float)xs, (float)(xs * xs), 1.0f);
    }
    D.hist_out[i] = h;
}

__global__ __launch_bounds__(kSvgfBlock) void variance_kernel(const SvgfBatch B, const SvgfK P) {
    const int j = find_job(B.tile0, (int)B.n, blockIdx.x);
    const SvgfDesc& D = B.d[j];
    uint32_t x, y;
    tile_xy(blockIdx.x - B.tile0[j], D.tiles_x, x, y);
    if (x >= D.W || y >= D.H) return;
    const size_t i = (size_t)y * D.W + x;
    float2* dst = level_buf(D, 0);
    const float4 n4 = D.nz[i];
    if (!(n4.w > 0.0f)) {
        dst[i] = make_float2(1.0f, 0.0f);
        return;
    }
    const float4 h = D.hist_out[i];
    float var;
    if (h.w >= (float)P.var_min_h) {
        // difference of the stored moments, exact in FP64, rounded once
        var = (float)fmax(0.0, (double)h.z - (double)h.y * (double)h.y);
    } else {
        // pooled moments of the valid neighbours, depth/normal weights of level 0;
        // one pass with FP64 sums: var = sum w (mu2 - mu1^2) / sum w + (sum w mu1^2 / sum w - mbar^2)
        const int R = (int)P.R;
        const float2 dzp = D.dz[i];
        const float3 np = f3(n4);
        const float eps_zp = P.eps_z * n4.w;
        double sw = 0.0, s1 = 0.0, s11 = 0.0, s2 = 0.0;
        for (int b = -R; b <= R; ++b) {
            const int qy = (int)y + b;
            if (qy < 0 || qy >= (int)D.H) continue;
            for (int a = -R; a <= R; ++a) {
                const int qx = (int)x + a;
                if (qx < 0 || qx >= (int)D.W) continue;
                const size_t q = (size_t)qy * D.W + qx;
                const float4 nq = D.nz[q];
                if (!(nq.w > 0.0f)) continue;
                double w = 1.0;
                if (a != 0 || b != 0)
                    w = (double)fused_weight(depth_coef(dzp, a, b, 1, P.sz[0], eps_zp), 0.0f, n4.w, 0.0f, np, P.sn[0],
                                             nq, 0.0f);
                const float4 hq = D.hist_out[q];
                const double m1 = (double)hq.y;
                sw += w;
                s1 = fma(w, m1, s1);
                s11 = fma(w * m1, m1, s11);
                s2 = fma(w, (double)hq.z - m1 * m1, s2);
            }
        }
        const double mbar = s1 / sw;
        var = (float)fmax(0.0, s2 / sw + fmax(0.0, s11 / sw - mbar * mbar));
    }
    dst[i] = make_float2(h.x, var);
}

// A-trous level at a large stride: every tap read from global memory (each
// tap of a wave is a contiguous row segment, so loads stay coalesced; LDS
// sub-image tiles would touch one cache line per pixel at these strides).
template <int LEVEL>
__global__ __launch_bounds__(kSvgfBlock) void atrous_direct_kernel(const SvgfBatch B, const SvgfK P) {
    constexpr int s = 1 << LEVEL;
    const int j = find_job(B.tile0, (int)B.n, blockIdx.x);
    const SvgfDesc& D = B.d[j];
    uint32_t ux, uy;
    tile_xy(blockIdx.x - B.tile0[j], D.tiles_x, ux, uy);
    if (ux >= D.W || uy >= D.H) return;
    const int x = (int)ux, y = (int)uy, W = (int)D.W, H = (int)D.H;
    const size_t i = (size_t)y * W + x;
    const bool last = LEVEL + 1 == (int)P.levels;
    const float2* __restrict__ src = level_buf(D, LEVEL);
    const float4* __restrict__ nzb = D.nz;
    const float4 n4 = nzb[i];
    if (!(n4.w > 0.0f)) {
        if (last)
            D.out[i] = 1.0f;
        else
            level_buf(D, LEVEL + 1)[i] = make_float2(1.0f, 0.0f);
        return;
    }
    float G = 0.0f, sk = 0.0f;
#pragma unroll
    for (int b = -1; b <= 1; ++b)
#pragma unroll
        for (int a = -1; a <= 1; ++a) {
            const int qx = x + a, qy = y + b;
            if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
            const size_t q = (size_t)qy * W + qx;
            if (!(nzb[q].w > 0.0f)) continue;
            const float k = k3(a) * k3(b);
            G = fmaf(k, src[q].y, G);
            sk += k;
        }
    const float g = sqrtf(G / sk);
    const float ke = kNegLog2e / fmaf(P.sl[LEVEL], g, P.eps_l);
    const float2 cvp = src[i];
    const float2 dzp = D.dz[i];
    const float3 np = f3(n4);
    const float sz = P.sz[LEVEL], sn = P.sn[LEVEL], eps_zp = P.eps_z * n4.w;
    float Dn = 0.140625f, Sc = 0.0f, Sv = 0.140625f * 0.140625f * cvp.y;
#pragma unroll
    for (int tp = 0; tp < 12; ++tp) {
        const int a = (tp + 13) % 5 - 2, b = (tp + 13) / 5 - 2;
        const float kz = depth_coef(dzp, a, b, s, sz, eps_zp);
        const float h = b3(a) * b3(b);
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int qx = x + (m ? -s * a : s * a), qy = y + (m ? -s * b : s * b);
            if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
            const size_t q = (size_t)qy * W + qx;
            const float4 nq = nzb[q];
            if (!(nq.w > 0.0f)) continue;
            const float2 cvq = src[q];
            const float hw = h * fused_weight(kz, ke, n4.w, cvp.x, np, sn, nq, cvq.x);
            Dn += hw;
            Sc = fmaf(hw, cvq.x - cvp.x, Sc);
            Sv = fmaf(hw * hw, cvq.y, Sv);
        }
    }
    const float inv = 1.0f / Dn;
    const float cn = fmaf(Sc, inv, cvp.x);
    const float vn = Sv * inv * inv;
    if (last)
        D.out[i] = cn;
    else
        level_buf(D, LEVEL + 1)[i] = make_float2(cn, vn);
    if (LEVEL == (int)P.fb_level && D.hist_out) reinterpret_cast<float*>(D.hist_out)[4 * i] = cn;
}

// A-trous level LEVEL (stride s = 2^LEVEL).  The pixels congruent to
// (ox, oy) mod s form a sub-image on which the dilated 5x5 stencil is dense:
// a workgroup owns a 16 x 16 block of one sub-image and stages its 20 x 20
// neighbourhood (geometry and (c, var)) in LDS once, so the 25 taps read LDS
// instead of global memory.  Tile t of a frame: super-tile t / s^2 (16s x 16s
// image pixels), sub-image t % s^2.
template <int LEVEL>
__global__ __launch_bounds__(kSvgfBlock) void atrous_kernel(const SvgfBatch B, const SvgfK P) {
    constexpr int s = 1 << LEVEL;
    constexpr int T = kSvgfTile, TW = kSvgfTile + 4;
    __shared__ float4 s_nz[TW * TW];
    __shared__ float2 s_cv[TW * TW];
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int j = find_job(B.tile0, (int)B.n, lb);
    const SvgfDesc& D = B.d[j];
    const int t = (int)(lb - B.tile0[j]);
    const int W = (int)D.W, H = (int)D.H;
    const int nsx = (W + T * s - 1) / (T * s);
    const int sub = t % (s * s), st = t / (s * s);
    const int bx = (st % nsx) * T * s + sub % s, by = (st / nsx) * T * s + sub / s;
    const float2* __restrict__ src = level_buf(D, LEVEL);
    for (int e = threadIdx.x; e < TW * TW; e += kSvgfBlock) {
        const int qx = bx + s * (e % TW - 2), qy = by + s * (e / TW - 2);
        float4 nq = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        float2 cq = make_float2(0.0f, 0.0f);
        if (qx >= 0 && qx < W && qy >= 0 && qy < H) {
            const size_t q = (size_t)qy * W + qx;
            nq = D.nz[q];
            cq = src[q];
        }
        s_nz[e] = nq;
        s_cv[e] = cq;
    }
    __syncthreads();
    const int li = threadIdx.x % T, lj = threadIdx.x / T;
    const int x = bx + s * li, y = by + s * lj;
    if (x >= W || y >= H) return;
    const size_t i = (size_t)y * W + x;
    const int c = (lj + 2) * TW + (li + 2);
    const bool last = LEVEL + 1 == (int)P.levels;
    const float4 n4 = s_nz[c];
    if (!(n4.w > 0.0f)) {
        if (last)
            D.out[i] = 1.0f;
        else
            level_buf(D, LEVEL + 1)[i] = make_float2(1.0f, 0.0f);
        return;
    }
    // 3x3 prefilter of the variance (stride 1: in the tile only at level 0)
    float G = 0.0f, sk = 0.0f;
#pragma unroll
    for (int b = -1; b <= 1; ++b)
#pragma unroll
        for (int a = -1; a <= 1; ++a) {
            const float k = k3(a) * k3(b);
            if (LEVEL == 0) {
                const int e = c + b * TW + a;
                if (!(s_nz[e].w > 0.0f)) continue;
                G = fmaf(k, s_cv[e].y, G);
            } else {
                const int qx = x + a, qy = y + b;
                if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
                const size_t q = (size_t)qy * W + qx;
                if (!(D.nz[q].w > 0.0f)) continue;
                G = fmaf(k, src[q].y, G);
            }
            sk += k;
        }
    const float g = sqrtf(G / sk);
    const float ke = kNegLog2e / fmaf(P.sl[LEVEL], g, P.eps_l);
    const float2 cvp = s_cv[c];
    const float2 dzp = D.dz[i];
    const float3 np = f3(n4);
    const float sz = P.sz[LEVEL], sn = P.sn[LEVEL], eps_zp = P.eps_z * n4.w;
    // centre tap: w = 1
    float Dn = 0.140625f, Sc = 0.0f, Sv = 0.140625f * 0.140625f * cvp.y;
#pragma unroll
    for (int tp = 0; tp < 12; ++tp) {
        // the 12 taps after (0, 0) in raster order, and their mirrors
        const int a = (tp + 13) % 5 - 2, b = (tp + 13) / 5 - 2;
        const float kz = depth_coef(dzp, a, b, s, sz, eps_zp);
        const float h = b3(a) * b3(b);
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int e = m ? c - b * TW - a : c + b * TW + a;
            const float4 nq = s_nz[e];
            const float2 cvq = s_cv[e];
            const float w = fused_weight(kz, ke, n4.w, cvp.x, np, sn, nq, cvq.x);
            const float hw = nq.w > 0.0f ? h * w : 0.0f;
            Dn += hw;
            Sc = fmaf(hw, cvq.x - cvp.x, Sc);
            Sv = fmaf(hw * hw, cvq.y, Sv);
        }
    }
    // deviation form: exact where every tap equals the centre (a constant
    // region stays on the |c_p - c_q| kink instead of drifting by an ulp)
    const float inv = 1.0f / Dn;
    const float cn = fmaf(Sc, inv, cvp.x);
    const float vn = Sv * inv * inv;
    if (last)
        D.out[i] = cn;
    else
        level_buf(D, LEVEL + 1)[i] = make_float2(cn, vn);
    if (LEVEL == (int)P.fb_level && D.hist_out) reinterpret_cast<float*>(D.hist_out)[4 * i] = cn;
}

// Levels 0-2 use LDS sub-image tiles, larger strides read taps directly.
constexpr uint32_t kTiledLevels = 3;

void launch_atrous(uint32_t level, dim3 grid, hipStream_t s, const SvgfBatch& B, const SvgfK& K) {
    switch (level) {
        case 0: hipLaunchKernelGGL(atrous_kernel<0>, grid, dim3(kSvgfBlock), 0, s, B, K); break;
        case 1: hipLaunchKernelGGL(atrous_kernel<1>, grid, dim3(kSvgfBlock), 0, s, B, K); break;
        case 2: hipLaunchKernelGGL(atrous_kernel<2>, grid, dim3(kSvgfBlock), 0, s, B, K); break;
        case 3: hipLaunchKernelGGL(atrous_direct_kernel<3>, grid, dim3(kSvgfBlock), 0, s, B, K); break;
        case 4: hipLaunchKernelGGL(atrous_direct_kernel<4>, grid, dim3(kSvgfBlock), 0, s, B, K); break;
        case 5: hipLaunchKernelGGL(atrous_direct_kernel<5>, grid, dim3(kSvgfBlock), 0, s, B, K); break;
        case 6: hipLaunchKernelGGL(atrous_direct_kernel<6>, grid, dim3(kSvgfBlock), 0, s, B, K); break;
        default: hipLaunchKernelGGL(atrous_direct_kernel<7>, grid, dim3(kSvgfBlock), 0, s, B, K); break;
    }
}

// ------------------------------------------------------------------ host side

dhr_status check_params(dhr_ctx* ctx, const dhr_svgf_params* p, const char* what) {
    if (!p) return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: params is NULL", what);
    if (p->levels < 1 || p->levels > DHR_MAX_LEVELS)
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: levels = %u outside 1..8", what, p->levels);
    for (uint32_t l = 0; l < p->levels; ++l) {
        if (!(p->sigma_z[l] > 0.0f) || !(p->sigma_l[l] > 0.0f) || !(p->sigma_n[l] >= 0.0f) ||
            std::isnan(p->sigma_z[l]) || std::isnan(p->sigma_l[l]) || !std::isfinite(p->sigma_n[l]))
            return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: level %u: sigma_z, sigma_l must be > 0 and sigma_n >= 0",
                             what, l);
    }
    if (!(p->alpha > 0.0f && p->alpha <= 1.0f) || !(p->alpha_moments > 0.0f && p->alpha_moments <= 1.0f))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: alpha outside (0, 1]", what);
    if (!(p->eps_z_rel > 0.0f) || !(p->eps_l > 0.0f) || !std::isfinite(p->eps_z_rel) || !std::isfinite(p->eps_l))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: eps_z_rel and eps_l must be positive", what);
    if (p->fallback_radius > 3) return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: fallback_radius > 3", what);
    if (p->feedback_level >= p->levels) return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: feedback_level >= levels", what);
    if (!(p->history_cap >= 1.0f) || !std::isfinite(p->history_cap))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: history_cap < 1", what);
    if (!std::isfinite(p->cos_normal_min) || !std::isfinite(p->plane_px))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: non-finite threshold", what);
    return DHR_OK;
}

SvgfK kparams(const dhr_svgf_params* p) {
    SvgfK k;
    std::memset(&k, 0, sizeof k);
    k.levels = p->levels;
    k.alpha = p->alpha;
    k.alpha_m = p->alpha_moments;
    for (int l = 0; l < DHR_MAX_LEVELS; ++l) {
        k.sz[l] = p->sigma_z[l];
        k.sn[l] = p->sigma_n[l];
        k.sl[l] = p->sigma_l[l];
    }
    k.eps_z = p->eps_z_rel;
    k.eps_l = p->eps_l;
    k.cos_min = p->cos_normal_min;
    k.plane_px = p->plane_px;
    k.use_obj = p->use_obj_id ? 1u : 0u;
    k.var_min_h = p->var_min_history;
    k.R = p->fallback_radius;
    k.fb_level = p->feedback_level;
    k.cap = p->history_cap;
    return k;
}

uint32_t svgf_tiles_x(uint32_t W) { return (W + kSvgfTile - 1) / kSvgfTile; }
uint32_t svgf_tiles(uint32_t W, uint32_t H) { return svgf_tiles_x(W) * ((H + kSvgfTile - 1) / kSvgfTile); }

bool sz_ok(uint32_t W, uint32_t H) { return W >= 1 && H >= 1 && W <= DHR_MAX_SIDE && H <= DHR_MAX_SIDE; }

// Tiles of an a-trous level: super-tiles of 16s x 16s pixels, s^2 sub-tiles each.
uint32_t atrous_tiles(uint32_t W, uint32_t H, uint32_t level) {
    if (level >= kTiledLevels) return svgf_tiles(W, H);
    const uint32_t s = 1u << level, span = kSvgfTile * s;
    return ((W + span - 1) / span) * ((H + span - 1) / span) * s * s;
}

// The batch of descriptors [b, b + n) with the tile prefix of `tiles(W, H)`.
template <class TF>
SvgfBatch make_batch(const std::vector<SvgfDesc>& descs, size_t b, size_t n, TF tiles) {
    SvgfBatch B;
    std::memset(&B, 0, sizeof B);
    B.n = (uint32_t)n;
    uint64_t acc = 0;
    for (size_t k = 0; k < n; ++k) {
        B.tile0[k] = (uint32_t)acc;
        B.d[k] = descs[b + k];
        acc += tiles(descs[b + k].W, descs[b + k].H);
    }
    B.tile0[n] = (uint32_t)acc;
    return B;
}

// Launches the passes over all descriptors in chunks of kSvgfMaxB: `pixel`
// passes on 16 x 16 tiles, then `levels` a-trous levels.
template <class F>
dhr_status for_chunks(dhr_ctx* ctx, const std::vector<SvgfDesc>& descs, const char* what, uint32_t levels,
                      hipStream_t s, const SvgfK& K, F pixel_passes) {
    for (size_t b = 0; b < descs.size(); b += kSvgfMaxB) {
        const size_t n = std::min<size_t>(kSvgfMaxB, descs.size() - b);
        const SvgfBatch B = make_batch(descs, b, n, svgf_tiles);
        pixel_passes(B, dim3(B.tile0[n]));
        for (uint32_t l = 0; l < levels; ++l) {
            const SvgfBatch Bl = make_batch(descs, b, n, [l](uint32_t W, uint32_t H) { return atrous_tiles(W, H, l); });
            launch_atrous(l, dim3(Bl.tile0[n]), s, Bl, K);
        }
        dhr_status st = check_launch(ctx, what);
        if (st != DHR_OK) return st;
    }
    return DHR_OK;
}

}  // namespace

// also used by the adjoint
dhr_status svgf_check_params(dhr_ctx* ctx, const dhr_svgf_params* p, const char* what) {
    return check_params(ctx, p, what);
}

}  // namespace dhr

extern "C" {

uint64_t dhr_svgf_workspace_bytes(uint32_t W, uint32_t H, const dhr_svgf_params* params, int which) {
    const uint64_t HW = (uint64_t)W * H;
    const uint32_t L = params ? params->levels : 5;
    if (which == 0) return 2 * HW * 8;
    // adjoint: per-pixel coefficients (float4), two (c, v) adjoint buffers,
    // prefilter/centre terms (float4), and per-tile sigma partials (3 doubles
    // per level and tile)
    const uint64_t tiles = (uint64_t)((W + dhr::kSvgfTile - 1) / dhr::kSvgfTile) * ((H + dhr::kSvgfTile - 1) / dhr::kSvgfTile);
    return HW * 16 + 2 * HW * 8 + HW * 16 + (uint64_t)L * tiles * 24;
}

dhr_status dhr_svgf_filter(dhr_ctx* ctx, const dhr_svgf_params* params, const dhr_svgf_frame* frames,
                           uint32_t n_frames, dhr_stream stream) {
    using namespace dhr;
    if (!ctx) return DHR_ERR_INVALID_ARG;
    dhr_status st = check_params(ctx, params, "dhr_svgf_filter");
    if (st != DHR_OK) return st;
    if (n_frames && !frames) return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_svgf_filter: frames is NULL");
    std::vector<SvgfDesc> descs(n_frames);
    for (uint32_t k = 0; k < n_frames; ++k) {
        const dhr_svgf_frame& F = frames[k];
        if (!sz_ok(F.W, F.H)) return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_svgf_filter: frame %u: bad size", k);
        if (F.n_ao == 0) return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_svgf_filter: frame %u: n_ao == 0", k);
        if (!F.ao_count || !F.pos || !F.nz || !F.dz || !F.mv || !F.hist_out || !F.out || (!F.save && !F.work))
            return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_svgf_filter: frame %u: missing buffer", k);
        if (F.hist_in && (!F.prev_pos || !F.prev_nz))
            return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_svgf_filter: frame %u: hist_in needs prev_pos/prev_nz", k);
        if (F.hist_in && F.hist_in == F.hist_out)
            return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_svgf_filter: frame %u: hist_out aliases hist_in", k);
        if (!aligned16(F.pos) || !aligned16(F.nz) || !aligned16(F.hist_out) || !aligned8(F.dz) || !aligned8(F.mv) ||
            (F.hist_in && (!aligned16(F.hist_in) || !aligned16(F.prev_pos) || !aligned16(F.prev_nz))) ||
            (F.save && !aligned8(F.save)) || (F.work && !aligned8(F.work)))
            return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_svgf_filter: frame %u: misaligned buffer", k);
        if (!(F.pix > 0.0f) || !std::isfinite(F.pix))
            return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_svgf_filter: frame %u: pix must be positive", k);
        SvgfDesc& d = descs[k];
        std::memset(&d, 0, sizeof d);
        d.W = F.W;
        d.H = F.H;
        d.n_ao = F.n_ao;
        d.tiles_x = svgf_tiles_x(F.W);
        d.ao = F.ao_count;
        d.pos = reinterpret_cast<const float4*>(F.pos);
        d.nz = reinterpret_cast<const float4*>(F.nz);
        d.dz = reinterpret_cast<const float2*>(F.dz);
        d.mv = reinterpret_cast<const float2*>(F.mv);
        d.prev_pos = reinterpret_cast<const float4*>(F.prev_pos);
        d.prev_nz = reinterpret_cast<const float4*>(F.prev_nz);
        d.hist_in = reinterpret_cast<const float4*>(F.hist_in);
        d.hist_out = reinterpret_cast<float4*>(F.hist_out);
        d.out = F.out;
        d.save = reinterpret_cast<float2*>(F.save);
        d.work = reinterpret_cast<float2*>(F.work);
        d.pix = F.pix;
    }
    DeviceGuard g(ctx->device);
    const SvgfK K = kparams(params);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    st = for_chunks(ctx, descs, "dhr_svgf_filter", K.levels, s, K, [&](const SvgfBatch& B, dim3 grid) {
        hipLaunchKernelGGL(temporal_kernel, grid, dim3(kSvgfBlock), 0, s, B, K);
        hipLaunchKernelGGL(variance_kernel, grid, dim3(kSvgfBlock), 0, s, B, K);
    });
    return st;
}

dhr_status dhr_svgf_spatial_forward(dhr_ctx* ctx, const dhr_svgf_params* params, const dhr_svgf_spatial_frame* frames,
                                    uint32_t n_frames, dhr_stream stream) {
    using namespace dhr;
    if (!ctx) return DHR_ERR_INVALID_ARG;
    dhr_status st = check_params(ctx, params, "dhr_svgf_spatial_forward");
    if (st != DHR_OK) return st;
    if (n_frames && !frames) return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_svgf_spatial_forward: frames is NULL");
    std::vector<SvgfDesc> descs(n_frames);
    DeviceGuard g(ctx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    for (uint32_t k = 0; k < n_frames; ++k) {
        const dhr_svgf_spatial_frame& F = frames[k];
        if (!sz_ok(F.W, F.H)) return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_svgf_spatial_forward: frame %u: bad size", k);
        if (!F.cv_in || !F.nz || !F.dz || !F.out || (!F.save && !F.work))
            return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_svgf_spatial_forward: frame %u: missing buffer", k);
        if (!aligned8(F.cv_in) || !aligned16(F.nz) || !aligned8(F.dz) || (F.save && !aligned8(F.save)) ||
            (F.work && !aligned8(F.work)))
            return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_svgf_spatial_forward: frame %u: misaligned buffer", k);
        SvgfDesc& d = descs[k];
        std::memset(&d, 0, sizeof d);
        d.W = F.W;
        d.H = F.H;
        d.tiles_x = svgf_tiles_x(F.W);
        d.nz = reinterpret_cast<const float4*>(F.nz);
        d.dz = reinterpret_cast<const float2*>(F.dz);
        d.out = F.out;
        d.save = reinterpret_cast<float2*>(F.save);
        d.work = reinterpret_cast<float2*>(F.work);
        if (F.save) {
            if (F.save != F.cv_in &&
                hipMemcpyAsync(F.save, F.cv_in, (size_t)F.W * F.H * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return set_error(ctx, DHR_ERR_DEVICE, "dhr_svgf_spatial_forward: copy failed");
        } else {
            d.b0 = reinterpret_cast<const float2*>(F.cv_in);
        }
    }
    const SvgfK K = kparams(params);
    return for_chunks(ctx, descs, "dhr_svgf_spatial_forward", K.levels, s, K, [](const SvgfBatch&, dim3) {});
}

}  // extern "C"
