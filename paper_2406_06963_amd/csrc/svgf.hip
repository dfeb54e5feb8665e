// Modified SVGF forward (Section 3.3): temporal accumulation, variance
// estimate and the iterated a-trous levels.  One lane per pixel, 16 x 16
// pixel workgroups; every pass covers a ragged batch of frames in one launch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
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

// The accumulated history of one pixel (valid, index i); see temporal_kernel.
__device__ __forceinline__ float4 accumulate(const SvgfDesc& D, const SvgfK& P, uint32_t x, uint32_t y, size_t i,
                                             float4 n4) {
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
        // the four bilinear taps' data are fetched up front (a tap that is
        // inactive or outside the frame reads the pixel itself and is
        // discarded), so the loads overlap instead of following the tests
        float4 pn[4], hq[4], pp[4];
        bool act[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = t & 1, jj = t >> 1;
            const float tx = X0 + (float)k, ty = Y0 + (float)jj;
            act[t] = (k == 1 ? fx > 0.0f : fx < 1.0f) && (jj == 1 ? fy > 0.0f : fy < 1.0f) && tx >= 0.0f &&
                     tx < (float)D.W && ty >= 0.0f && ty < (float)D.H;
            const size_t q = act[t] ? (size_t)ty * D.W + (size_t)tx : i;
            pn[t] = D.prev_nz[q];
            hq[t] = D.hist_in[q];
            pp[t] = D.prev_pos[q];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = t & 1, jj = t >> 1;
            if (!act[t] || !(pn[t].w > 0.0f) || !(hq[t].w > 0.0f)) continue;
            if (P.use_obj && fbits(pp[t].w) != fbits(p4.w)) continue;
            if (!tap_consistent(f3(n4), f3(p4), n4.w, pn[t], pp[t], P.cos_min, P.plane_px, D.pix)) continue;
            const double b = (k ? (double)fx : 1.0 - (double)fx) * (jj ? (double)fy : 1.0 - (double)fy);
            any = true;
            wsum += b;
            c = fma(b, (double)hq[t].x, c);
            m1 = fma(b, (double)hq[t].y, m1);
            m2 = fma(b, (double)hq[t].z, m2);
            hmax = fmaxf(hmax, hq[t].w);
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
    return h;
}

// Temporal accumulation, and the level-0 input (c, var) of every pixel whose
// variance needs no neighbours: invalid pixels, and valid ones with a history
// of at least var_min_history frames (variance = difference of the stored
// moments).  Each tile records whether it holds a pixel of shorter history;
// only those tiles run the spatial fallback (variance_kernel).
__global__ __launch_bounds__(kSvgfBlock) void temporal_kernel(const SvgfBatch B, const SvgfK P) {
    const int j = find_job(B.tile0, (int)B.n, blockIdx.x);
    const SvgfDesc& D = B.d[j];
    const uint32_t t = blockIdx.x - B.tile0[j];
    uint32_t x, y;
    tile_xy(t, D.tiles_x, x, y);
    bool fallback = false;
    if (x < D.W && y < D.H) {
        const size_t i = (size_t)y * D.W + x;
        const float4 n4 = D.nz[i];
        float2* dst = level_buf(D, 0);
        if (!(n4.w > 0.0f)) {
            D.hist_out[i] = make_float4(1.0f, 1.0f, 1.0f, 0.0f);
            dst[i] = make_float2(1.0f, 0.0f);
        } else {
            const float4 h = accumulate(D, P, x, y, i, n4);
            D.hist_out[i] = h;
            fallback = !(h.w >= (float)P.var_min_h);
            // difference of the stored moments, exact in FP64, rounded once
            if (!fallback) dst[i] = make_float2(h.x, (float)fmax(0.0, (double)h.z - (double)h.y * (double)h.y));
        }
    }
    const int any = __syncthreads_or(fallback);
    if (threadIdx.x == 0) D.fb[t] = any ? 1u : 0u;
}

// Variance of level 0 for the pixels of short history (the others were
// written by temporal_kernel): only tiles that hold one do any work; they
// stage the moments and geometry of their 16 x 16 tile plus a 3-pixel rim in
// LDS for the spatial fallback.
constexpr int kVarRim = 3;

// R = fallback radius (0..3): the (2R + 1)^2 taps are unrolled, so their LDS
// reads and weights overlap instead of waiting tap by tap.
template <int R>
__global__ __launch_bounds__(kSvgfBlock) void variance_kernel(const SvgfBatch B, const SvgfK P) {
    constexpr int TW = kSvgfTile + 2 * kVarRim;
    __shared__ float4 s_nz[TW * TW];  // zero for invalid or outside pixels
    __shared__ float2 s_m[TW * TW];   // stored moments (m1, m2)
    const int j = find_job(B.tile0, (int)B.n, blockIdx.x);
    const SvgfDesc& D = B.d[j];
    const uint32_t t = blockIdx.x - B.tile0[j];
    if (D.fb[t] == 0u) return;  // the whole workgroup: no pixel of short history
    uint32_t x, y;
    tile_xy(t, D.tiles_x, x, y);
    const int W = (int)D.W, H = (int)D.H;
    const bool inside = x < D.W && y < D.H;
    const size_t i = inside ? (size_t)y * D.W + x : 0;
    const float4 n4 = D.nz[i];
    const float4 h = D.hist_out[i];
    const bool valid = inside && n4.w > 0.0f;
    const bool fallback = valid && !(h.w >= (float)P.var_min_h);
    if (__syncthreads_or(fallback)) {
        const int bx = (int)x - (int)(threadIdx.x % kSvgfTile) - kVarRim;
        const int by = (int)y - (int)(threadIdx.x / kSvgfTile) - kVarRim;
        stage_tile<TW * TW>(
            [&](int e) {
                const int qx = bx + e % TW, qy = by + e / TW;
                Staged r{make_float4(0.0f, 0.0f, 0.0f, 0.0f), make_float2(0.0f, 0.0f)};
                if (qx >= 0 && qx < W && qy >= 0 && qy < H) {
                    const size_t q = (size_t)qy * W + qx;
                    const float4 hq = D.hist_out[q];
                    r.nz = D.nz[q];
                    r.cv = make_float2(hq.y, hq.z);
                }
                return r;
            },
            [&](int e, const Staged& r) {
                const bool ok = r.nz.w > 0.0f;
                s_nz[e] = ok ? r.nz : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                s_m[e] = r.cv;
            });
        __syncthreads();
    }
    if (!fallback) return;
    float2* dst = level_buf(D, 0);
    float var;
    {
        // pooled moments of the valid neighbours, depth/normal weights of level 0;
        // one pass with FP64 sums: var = sum w (mu2 - mu1^2) / sum w + (sum w mu1^2 / sum w - mbar^2)
        const float2 dzp = D.dz[i];
        const float3 np = f3(n4);
        const float eps_zp = P.eps_z * n4.w;
        const int c = (int)(threadIdx.x / kSvgfTile + kVarRim) * TW + (int)(threadIdx.x % kSvgfTile) + kVarRim;
        // kz of the taps after the centre in raster order; a tap and its
        // mirror (-a, -b) have the same |a dz/dx + b dz/dy|, hence the same kz
        constexpr int K = 2 * R + 1, centre = (K * K - 1) / 2;
        float kzh[centre > 0 ? centre : 1];
#pragma unroll
        for (int t = 0; t < centre; ++t)
            kzh[t] = depth_coef(dzp, (centre + 1 + t) % K - R, (centre + 1 + t) / K - R, 1, P.sz[0], eps_zp);
        double sw = 0.0, s1 = 0.0, s11 = 0.0, s2 = 0.0;
#pragma unroll
        for (int b = -R; b <= R; ++b) {
#pragma unroll
            for (int a = -R; a <= R; ++a) {
                const int idx = (b + R) * K + a + R;
                const int e = c + b * TW + a;
                // an invalid or outside neighbour was staged with a zero
                // normal: its weight is exactly 0 and the sums stay unchanged
                const double w = idx == centre
                                     ? 1.0
                                     : (double)fused_weight(idx > centre ? kzh[idx - centre - 1] : kzh[centre - 1 - idx],
                                                            0.0f, n4.w, 0.0f, np, P.sn[0], s_nz[e], 0.0f);
                const double m1 = (double)s_m[e].x;
                sw += w;
                s1 = fma(w, m1, s1);
                s11 = fma(w * m1, m1, s11);
                s2 = fma(w, (double)s_m[e].y - m1 * m1, s2);
            }
        }
        const double mbar = s1 / sw;
        var = (float)fmax(0.0, s2 / sw + fmax(0.0, s11 / sw - mbar * mbar));
    }
    dst[i] = make_float2(h.x, var);
}

// Prefilter of level `level` (used for levels read directly): for every pixel, ke from the 3x3 blur of
// its input variance.  A workgroup covers 64 x 16 pixels (4 rows per lane)
// and stages their 66 x 18 neighbourhood in LDS.  The previous level marked
// invalid pixels with kNoVar.  Writes D.ke.
constexpr int kPreTX = 64, kPreTY = 16;

uint32_t prefilter_tiles(uint32_t W, uint32_t H) {
    return ((W + kPreTX - 1) / kPreTX) * ((H + kPreTY - 1) / kPreTY);
}

__global__ __launch_bounds__(kSvgfBlock) void prefilter_kernel(const SvgfBatch B, const SvgfK P, uint32_t level) {
    constexpr int CW = kPreTX + 2, CH = kPreTY + 2, RPL = kPreTY * kPreTX / kSvgfBlock;
    __shared__ float s_v[CW * CH];
    const int j = find_job(B.tile0, (int)B.n, blockIdx.x);
    const SvgfDesc& D = B.d[j];
    const int t = (int)(blockIdx.x - B.tile0[j]);
    const int W = (int)D.W, H = (int)D.H;
    const int ntx = (W + kPreTX - 1) / kPreTX;
    const int bx = (t % ntx) * kPreTX - 1, by = (t / ntx) * kPreTY - 1;
    const float2* __restrict__ src = level_buf(D, level);
    stage_tile<CW * CH>(
        [&](int e) {
            const int qx = bx + e % CW, qy = by + e / CW;
            return (qx >= 0 && qx < W && qy >= 0 && qy < H) ? src[(size_t)qy * W + qx].y : kNoVar;
        },
        [&](int e, float v) { s_v[e] = v; });
    __syncthreads();
    const int li = threadIdx.x % kPreTX, lj = (threadIdx.x / kPreTX) * RPL;
    const int x = bx + 1 + li;
    if (x >= W) return;
    const float sl = P.sl[level], eps_l = P.eps_l;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int y = by + 1 + lj + r;
        if (y >= H) return;
        float G = 0.0f, sk = 0.0f;
#pragma unroll
        for (int b = -1; b <= 1; ++b)
#pragma unroll
            for (int a = -1; a <= 1; ++a) {
                const float v = s_v[(lj + r + 1 + b) * CW + li + 1 + a];
                if (!has_var(v)) continue;
                const float k = k3(a) * k3(b);
                G = fmaf(k, v, G);
                sk += k;
            }
        D.ke[(size_t)y * W + x] = sk > 0.0f ? ke_of(G, sk, sl, eps_l) : 0.0f;
    }
}

// A-trous level at a large stride: every tap read from global memory (each
// tap of a wave is a contiguous row segment, so loads stay coalesced; LDS
// sub-image tiles would touch one cache line per pixel at these strides).
template <int LEVEL, int KR>
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
            level_buf(D, LEVEL + 1)[i] = make_float2(1.0f, kNoVar);
        return;
    }
    const float ke = D.ke[i];
    const float2 cvp = src[i];
    const float2 dzp = D.dz[i];
    const float3 np = f3(n4);
    const float sz = P.sz[LEVEL], sn = P.sn[LEVEL], eps_zp = P.eps_z * n4.w;
    float Dn = centre_h<KR>, Sc = 0.0f, Sv = centre_h<KR> * centre_h<KR> * cvp.y;
#pragma unroll
    for (int tp = 0; tp < half_taps<KR>; ++tp) {
        int a, b;
        tap_ab<KR>(tp, a, b);
        const float kz = depth_coef(dzp, a, b, s, sz, eps_zp);
        const float h = hk<KR>(a) * hk<KR>(b);
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

// A-trous level LEVEL (stride s = 2^LEVEL; used for level 0).  The pixels
// congruent to (ox, oy) mod s form a sub-image on which the dilated stencil
// (5x5, or 3x3 for KR = 1) is dense:
// a workgroup owns a 16 x 16 block of one sub-image and stages its 20 x 20 (18 x 18)
// neighbourhood (geometry and (c, var)) in LDS once, so the 25 taps read LDS
// instead of global memory.  Tile t of a frame: super-tile t / s^2 (16s x 16s
// image pixels), sub-image t % s^2.
template <int LEVEL, int KR>
__global__ __launch_bounds__(kSvgfBlock) void atrous_kernel(const SvgfBatch B, const SvgfK P) {
    constexpr int s = 1 << LEVEL;
    constexpr int T = kSvgfTile, TW = kSvgfTile + 2 * KR;
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
    stage_tile<TW * TW>(
        [&](int e) {
            const int qx = bx + s * (e % TW - KR), qy = by + s * (e / TW - KR);
            return load_staged(D.nz, src, qx, qy, W, H);
        },
        [&](int e, const Staged& r) {
            const bool ok = r.nz.w > 0.0f;
            s_nz[e] = ok ? r.nz : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            s_cv[e] = ok ? r.cv : make_float2(0.0f, 0.0f);
        });
    __syncthreads();
    const int li = threadIdx.x % T, lj = threadIdx.x / T;
    const int x = bx + s * li, y = by + s * lj;
    if (x >= W || y >= H) return;
    const size_t i = (size_t)y * W + x;
    const int c = (lj + KR) * TW + (li + KR);
    const bool last = LEVEL + 1 == (int)P.levels;
    const float4 n4 = s_nz[c];
    if (!(n4.w > 0.0f)) {
        if (last)
            D.out[i] = 1.0f;
        else
            level_buf(D, LEVEL + 1)[i] = make_float2(1.0f, kNoVar);
        return;
    }
    // 3x3 prefilter of the variance: from the tile at level 0 (stride 1),
    // from the prefilter pass at the other levels (invalid pixels were staged
    // with z = 0)
    float ke;
    if (LEVEL == 0) {
        float G = 0.0f, sk = 0.0f;
#pragma unroll
        for (int b = -1; b <= 1; ++b)
#pragma unroll
            for (int a = -1; a <= 1; ++a) {
                const int e = c + b * TW + a;
                const float k = k3(a) * k3(b);
                G = fmaf(k, s_cv[e].y, G);  // zero on invalid pixels
                sk += s_nz[e].w > 0.0f ? k : 0.0f;
            }
        ke = ke_of(G, sk, P.sl[LEVEL], P.eps_l);
    } else {
        ke = D.ke[i];
    }
    const float2 cvp = s_cv[c];
    const float2 dzp = D.dz[i];
    const float3 np = f3(n4);
    const float sz = P.sz[LEVEL], sn = P.sn[LEVEL], eps_zp = P.eps_z * n4.w;
    // centre tap: w = 1
    float Dn = centre_h<KR>, Sc = 0.0f, Sv = centre_h<KR> * centre_h<KR> * cvp.y;
#pragma unroll
    for (int tp = 0; tp < half_taps<KR>; ++tp) {
        // the taps after (0, 0) in raster order, and their mirrors
        int a, b;
        tap_ab<KR>(tp, a, b);
        const float kz = depth_coef(dzp, a, b, s, sz, eps_zp);
        const float lh = lhk<KR>(a) + lhk<KR>(b);
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int e = m ? c - b * TW - a : c + b * TW + a;
            accumulate_tap(lh, kz, ke, n4.w, cvp.x, np, sn, s_nz[e], s_cv[e], Dn, Sc, Sv);
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

// A-trous level LEVEL >= 1 (stride s = 2^LEVEL) on row classes: a workgroup
// owns 64 consecutive pixels of 4 rows that are s apart (rows congruent mod
// s), so every tap of the dilated 5x5 stencil falls on 8 staged rows of
// 64 + 4s consecutive pixels (3x3 stencil, KR = 1: 6 rows of 64 + 2s).  Staging reads whole row segments (coalesced at
// any stride) and each staged pixel serves up to 20 taps from LDS.  Tile t of
// a frame: column block t % tx, then row class, then block of 4s rows.
template <int LEVEL, int KR>
__global__ __launch_bounds__(kSvgfBlock) void atrous_rows_kernel(const SvgfBatch B, const SvgfK P) {
    constexpr int s = 1 << LEVEL;
    constexpr int CW = kRowsTX + 2 * KR * s, CH = kRowsTY + 2 * KR, GW = kRowsTX + 2;
    __shared__ float4 s_nz[CH * CW];
    __shared__ float2 s_cv[CH * CW];
    __shared__ float s_g[kRowsTY * 2 * GW];  // variance of the rows above and below each output row
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int j = find_job(B.tile0, (int)B.n, lb);
    const SvgfDesc& D = B.d[j];
    const int t = (int)(lb - B.tile0[j]);
    const int W = (int)D.W, H = (int)D.H;
    const int ntx = (W + kRowsTX - 1) / kRowsTX;
    const int X = t % ntx, rest = t / ntx;
    const int x0 = X * kRowsTX, y0 = (rest / s) * (kRowsTY * s) + rest % s;
    const float2* __restrict__ src = level_buf(D, LEVEL);
    stage_tile<CH * CW>(
        [&](int e) {
            const int qx = x0 - KR * s + e % CW, qy = y0 + s * (e / CW - KR);
            return load_staged(D.nz, src, qx, qy, W, H);
        },
        [&](int e, const Staged& r) {
            const bool ok = r.nz.w > 0.0f;
            s_nz[e] = ok ? r.nz : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            s_cv[e] = ok ? r.cv : make_float2(0.0f, 0.0f);
        });
    // the 3x3 variance prefilter needs the rows next to each output row (the
    // previous level marked invalid pixels with kNoVar)
    stage_tile<kRowsTY * 2 * GW>(
        [&](int e) {
            const int qx = x0 - 1 + e % GW, qy = y0 + s * (e / (2 * GW)) + ((e / GW) % 2 ? 1 : -1);
            const float v = src[clamped_index(qx, qy, W, H)].y;
            return inside(qx, qy, W, H) ? v : kNoVar;
        },
        [&](int e, float v) { s_g[e] = v; });
    __syncthreads();
    const int li = threadIdx.x % kRowsTX, lj = threadIdx.x / kRowsTX;
    const int x = x0 + li, y = y0 + s * lj;
    if (x >= W || y >= H) return;
    const size_t i = (size_t)y * W + x;
    const int c = (lj + KR) * CW + KR * s + li;
    const bool last = LEVEL + 1 == (int)P.levels;
    const float4 n4 = s_nz[c];
    if (!(n4.w > 0.0f)) {
        if (last)
            D.out[i] = 1.0f;
        else
            level_buf(D, LEVEL + 1)[i] = make_float2(1.0f, kNoVar);
        return;
    }
    float G = 0.0f, sk = 0.0f;
#pragma unroll
    for (int b = -1; b <= 1; ++b)
#pragma unroll
        for (int a = -1; a <= 1; ++a) {
            float v;
            if (b == 0)
                v = s_nz[c + a].w > 0.0f ? s_cv[c + a].y : kNoVar;
            else
                v = s_g[(2 * lj + (b > 0)) * GW + li + 1 + a];
            if (!has_var(v)) continue;
            const float k = k3(a) * k3(b);
            G = fmaf(k, v, G);
            sk += k;
        }
    const float ke = ke_of(G, sk, P.sl[LEVEL], P.eps_l);
    const float2 cvp = s_cv[c];
    const float2 dzp = D.dz[i];
    const float3 np = f3(n4);
    const float sz = P.sz[LEVEL], sn = P.sn[LEVEL], eps_zp = P.eps_z * n4.w;
    float Dn = centre_h<KR>, Sc = 0.0f, Sv = centre_h<KR> * centre_h<KR> * cvp.y;
#pragma unroll
    for (int tp = 0; tp < half_taps<KR>; ++tp) {
        int a, b;
        tap_ab<KR>(tp, a, b);
        const float kz = depth_coef(dzp, a, b, s, sz, eps_zp);
        const float lh = lhk<KR>(a) + lhk<KR>(b);
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int e = m ? c - b * CW - s * a : c + b * CW + s * a;
            accumulate_tap(lh, kz, ke, n4.w, cvp.x, np, sn, s_nz[e], s_cv[e], Dn, Sc, Sv);
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

// Level 0 uses dense 16 x 16 tiles (its variance prefilter comes from the
// same tile), levels 1-5 row classes, deeper levels read taps directly.
constexpr uint32_t kRowsMaxLevel = 5;

template <int KR>
void launch_atrous_r(uint32_t level, dim3 grid, hipStream_t s, const SvgfBatch& B, const SvgfK& K) {
    switch (level) {
        case 0: hipLaunchKernelGGL((atrous_kernel<0, KR>), grid, dim3(kSvgfBlock), 0, s, B, K); break;
        case 1: hipLaunchKernelGGL((atrous_rows_kernel<1, KR>), grid, dim3(kSvgfBlock), 0, s, B, K); break;
        case 2: hipLaunchKernelGGL((atrous_rows_kernel<2, KR>), grid, dim3(kSvgfBlock), 0, s, B, K); break;
        case 3: hipLaunchKernelGGL((atrous_rows_kernel<3, KR>), grid, dim3(kSvgfBlock), 0, s, B, K); break;
        case 4: hipLaunchKernelGGL((atrous_rows_kernel<4, KR>), grid, dim3(kSvgfBlock), 0, s, B, K); break;
        case 5: hipLaunchKernelGGL((atrous_rows_kernel<5, KR>), grid, dim3(kSvgfBlock), 0, s, B, K); break;
        case 6: hipLaunchKernelGGL((atrous_direct_kernel<6, KR>), grid, dim3(kSvgfBlock), 0, s, B, K); break;
        default: hipLaunchKernelGGL((atrous_direct_kernel<7, KR>), grid, dim3(kSvgfBlock), 0, s, B, K); break;
    }
}

void launch_atrous(uint32_t level, dim3 grid, hipStream_t s, const SvgfBatch& B, const SvgfK& K) {
    if (K.kw == 3)
        launch_atrous_r<1>(level, grid, s, B, K);
    else
        launch_atrous_r<2>(level, grid, s, B, K);
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
    if (p->kernel_width != 3 && p->kernel_width != 5)
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: kernel_width = %u is neither 3 nor 5", what, p->kernel_width);
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
        // sigma_n = 0 (weight 1 for every n_p . n_q > 0) as the smallest
        // normal float: same weights, and the tap loop's exponent stays -inf
        // (weight 0) where n_p . n_q = 0
        k.sn[l] = std::max(p->sigma_n[l], std::numeric_limits<float>::min());
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
    k.kw = p->kernel_width;
    return k;
}

uint32_t svgf_tiles_x(uint32_t W) { return (W + kSvgfTile - 1) / kSvgfTile; }
uint32_t svgf_tiles(uint32_t W, uint32_t H) { return svgf_tiles_x(W) * ((H + kSvgfTile - 1) / kSvgfTile); }

bool sz_ok(uint32_t W, uint32_t H) { return W >= 1 && H >= 1 && W <= DHR_MAX_SIDE && H <= DHR_MAX_SIDE; }

// Tiles of an a-trous level: super-tiles of 16s x 16s pixels, s^2 sub-tiles each.
uint32_t atrous_tiles(uint32_t W, uint32_t H, uint32_t level) {
    if (level >= 1 && level <= kRowsMaxLevel) return rows_tiles(W, H, (int)level);
    return svgf_tiles(W, H);
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
        const SvgfBatch Bp = make_batch(descs, b, n, prefilter_tiles);
        pixel_passes(B, dim3(B.tile0[n]));
        for (uint32_t l = 0; l < levels; ++l) {
            if (l > kRowsMaxLevel)
                hipLaunchKernelGGL(prefilter_kernel, dim3(Bp.tile0[n]), dim3(kSvgfBlock), 0, s, Bp, K, l);
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
    if (which == 0) return 2 * HW * 8 + HW * 4 + (uint64_t)dhr::svgf_tiles(W, H) * 4;  // (c, var) ping-pong, ke,
                                                                                     // tile fallback flags
    // adjoint: per-pixel coefficients (float4), two (c, v) adjoint buffers,
    // prefilter/centre terms (float4), and per-workgroup sigma partials (3
    // doubles per level and workgroup)
    uint64_t tiles = 0;
    for (uint32_t l = 0; l < L && l < DHR_MAX_LEVELS; ++l) tiles += dhr::adjoint_tiles(W, H, l);
    return HW * 16 + 2 * HW * 8 + HW * 16 + tiles * 24;
}

}  // extern "C"

namespace dhr {
namespace {

// The filter of dhr_svgf_filter and dhr_svgf_filter_noalloc.  With
// `scratch` NULL every frame brings its own work buffer; otherwise the
// frames' work buffers are consecutive 256-byte-aligned slices of
// `scratch` (of `scratch_bytes` bytes) and their own `work` must be NULL.
dhr_status filter_impl(dhr_ctx* ctx, const dhr_svgf_params* params, const dhr_svgf_frame* frames, uint32_t n_frames,
                       dhr_stream stream, char* scratch, uint64_t scratch_bytes, const char* what) {
    dhr_status st = check_params(ctx, params, what);
    if (st != DHR_OK) return st;
    if (n_frames && !frames) return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: frames is NULL", what);
    std::vector<SvgfDesc> descs(n_frames);
    uint64_t used = 0;
    for (uint32_t k = 0; k < n_frames; ++k) {
        const dhr_svgf_frame& F = frames[k];
        if (!sz_ok(F.W, F.H)) return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: frame %u: bad size", what, k);
        if (F.n_ao == 0) return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: frame %u: n_ao == 0", what, k);
        if (!F.ao_count || !F.pos || !F.nz || !F.dz || !F.mv || !F.hist_out || !F.out || (!scratch && !F.work))
            return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: frame %u: missing buffer", what, k);
        if (scratch && F.work)
            return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: frame %u: work must be NULL (the library's scratch is used)",
                             what, k);
        if (F.hist_in && (!F.prev_pos || !F.prev_nz))
            return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: frame %u: hist_in needs prev_pos/prev_nz", what, k);
        if (F.hist_in && F.hist_in == F.hist_out)
            return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: frame %u: hist_out aliases hist_in", what, k);
        if (!aligned16(F.pos) || !aligned16(F.nz) || !aligned16(F.hist_out) || !aligned8(F.dz) || !aligned8(F.mv) ||
            (F.hist_in && (!aligned16(F.hist_in) || !aligned16(F.prev_pos) || !aligned16(F.prev_nz))) ||
            (F.save && !aligned8(F.save)) || (F.work && !aligned8(F.work)))
            return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: frame %u: misaligned buffer", what, k);
        if (!(F.pix > 0.0f) || !std::isfinite(F.pix))
            return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: frame %u: pix must be positive", what, k);
        float* work = F.work;
        if (scratch) {
            const uint64_t need = (dhr_svgf_workspace_bytes(F.W, F.H, params, 0) + 255) & ~uint64_t(255);
            if (used + need > scratch_bytes)
                return set_error(ctx, DHR_ERR_INVALID_ARG,
                                 "%s: the frames need more than the %llu bytes of scratch (%llu through frame %u)", what,
                                 (unsigned long long)scratch_bytes, (unsigned long long)(used + need), k);
            work = reinterpret_cast<float*>(scratch + used);
            used += need;
        }
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
        d.work = reinterpret_cast<float2*>(work);
        d.ke = work + (size_t)F.W * F.H * 4;
        d.fb = reinterpret_cast<uint32_t*>(work) + (size_t)F.W * F.H * 5;
        d.pix = F.pix;
    }
    DeviceGuard g(ctx->device);
    const SvgfK K = kparams(params);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    st = for_chunks(ctx, descs, what, K.levels, s, K, [&](const SvgfBatch& B, dim3 grid) {
        hipLaunchKernelGGL(temporal_kernel, grid, dim3(kSvgfBlock), 0, s, B, K);
        switch (K.R) {
            case 0: hipLaunchKernelGGL(variance_kernel<0>, grid, dim3(kSvgfBlock), 0, s, B, K); break;
            case 1: hipLaunchKernelGGL(variance_kernel<1>, grid, dim3(kSvgfBlock), 0, s, B, K); break;
            case 2: hipLaunchKernelGGL(variance_kernel<2>, grid, dim3(kSvgfBlock), 0, s, B, K); break;
            default: hipLaunchKernelGGL(variance_kernel<3>, grid, dim3(kSvgfBlock), 0, s, B, K); break;
        }
    });
    return st;
}

// Scratch of dhr_svgf_filter_noalloc: one array per device, held while the
// library is loaded.  Host code never passes `scratch` itself to a kernel or
// a copy (on the host it names a stand-in, not device memory); it uses the
// device address that svgf_scratch_init looked up for each device.
constexpr uint64_t kNoAllocScratchBytes = DHR_SVGF_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// Looks up the device address of `scratch` on the context's device, once per
// device, with that device current (called by dhr_create).
dhr_status svgf_scratch_init(dhr_ctx* ctx) {
    if (ctx->device < 0 || ctx->device >= kMaxDevices)
        return set_error(ctx, DHR_ERR_UNSUPPORTED, "dhr_create: device %d beyond %d", ctx->device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[ctx->device]) {
        DeviceGuard g(ctx->device);
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(ctx, DHR_ERR_DEVICE, "dhr_create: no address for the filter's scratch: %s",
                             hipGetErrorString(e));
        g_scratch_ptr[ctx->device] = p;
    }
    ctx->scratch = g_scratch_ptr[ctx->device];
    return DHR_OK;
}

}  // namespace dhr

extern "C" {

dhr_status dhr_svgf_filter(dhr_ctx* ctx, const dhr_svgf_params* params, const dhr_svgf_frame* frames,
                           uint32_t n_frames, dhr_stream stream) {
    if (!ctx) return DHR_ERR_INVALID_ARG;
    return dhr::filter_impl(ctx, params, frames, n_frames, stream, nullptr, 0, "dhr_svgf_filter");
}

dhr_status dhr_svgf_filter_noalloc(dhr_ctx* ctx, const dhr_svgf_params* params, const dhr_svgf_frame* frames,
                                   uint32_t n_frames, dhr_stream stream) {
    if (!ctx) return DHR_ERR_INVALID_ARG;
    if (!ctx->scratch) return dhr::set_error(ctx, DHR_ERR_DEVICE, "dhr_svgf_filter_noalloc: no scratch on this device");
    return dhr::filter_impl(ctx, params, frames, n_frames, stream, static_cast<char*>(ctx->scratch),
                            dhr::kNoAllocScratchBytes, "dhr_svgf_filter_noalloc");
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
        if (!F.cv_in || !F.nz || !F.dz || !F.out || !F.work)
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
        d.ke = reinterpret_cast<float*>(F.work) + (size_t)F.W * F.H * 4;
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
