// Adjoint of the spatial filter stack (the a-trous levels of Section 3.3 with
// their variance prefilter): gradients of a loss with respect to the input AO
// value c, the input variance v and the per-level sigma_z, sigma_n, sigma_l.
//
// For one level with c'_p = sum_q h w_pq c_q / D_p, v'_p = sum_q h^2 w_pq^2
// v_q / D_p^2 and incoming adjoints (a_p, b_p) of (c'_p, v'_p), write A = a/D,
// B = b/D^2, K = 2 B v' D.  The adjoint of a tap weight is
//     wbar_pq = h (A_p (c_q - c'_p) - K_p) + 2 B_p h^2 w_pq v_q,
// the direct terms are dc_q += A_p h w, dv_q += B_p h^2 w^2, and the weight
// chain rule reaches c_p, c_q (through w_l), the prefiltered deviation g_p and
// the sigmas.  Pass A runs per centre pixel p (coefficients, the centre-role
// terms, g's adjoint, sigma partials); pass B runs per neighbour q and gathers
// over p = q - s (a, b): no atomics, so results are deterministic.  Sigma
// partials are summed per tile in FP64 and reduced in a fixed order.
#include <cmath>
#include <cstring>
#include <vector>

#include "svgf_common.h"

namespace dhr {

dhr_status svgf_check_params(dhr_ctx* ctx, const dhr_svgf_params* p, const char* what);

namespace {

struct BwdDesc {
    uint32_t W, H, tiles_x, tiles;
    const float2* save;     // [levels][HW]
    const float4* nz;
    const float2* dz;
    const float* grad_out;  // [HW]
    float2* grad_cv;        // [HW]
    float2* g0;             // adjoint ping-pong [HW] x 2
    float2* g1;
    float4* coef;           // [HW] (A, B, c', 1 / E)
    float4* aux;            // [HW] (prefilter adjoint / sk, centre-role dc, K, 0)
    double* part;           // [sum over levels of the level's workgroups][3]
    uint32_t part_off[DHR_MAX_LEVELS + 1];  // first workgroup of each level in part
};
constexpr int kBwdMaxB = 24;
using BwdBatch = Batch<BwdDesc, kBwdMaxB>;
static_assert(sizeof(BwdBatch) <= 4000, "kernel arguments too large");

__device__ __forceinline__ float2* adj_out(const BwdDesc& D, uint32_t l, uint32_t L) {
    return l == 0 ? D.grad_cv : (((L - 1 - l) & 1u) ? D.g1 : D.g0);
}

__device__ __forceinline__ float sgn(float v) { return v > 0.0f ? 1.0f : (v < 0.0f ? -1.0f : 0.0f); }

__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < kSvgfBlock / 64; ++k) s += red[k];
    return s;
}

// Pass A on 16 x 16 tiles with taps read from global memory (deep levels).
__global__ __launch_bounds__(kSvgfBlock) void adjoint_a_direct(const BwdBatch Bt, const SvgfK P, uint32_t level) {
    __shared__ double red[kSvgfBlock / 64];
    const int j = find_job(Bt.tile0, (int)Bt.n, blockIdx.x);
    const BwdDesc& D = Bt.d[j];
    const uint32_t tile = blockIdx.x - Bt.tile0[j];
    uint32_t x, y;
    tile_xy(tile, D.tiles_x, x, y);
    const uint32_t L = P.levels;
    const int W = (int)D.W, H = (int)D.H, s = 1 << level;
    float s_z = 0.0f, s_n = 0.0f, s_l = 0.0f;
    if (x < D.W && y < D.H) {
        const size_t i = (size_t)y * W + x;
        const float2* cv = D.save + (size_t)level * W * H;
        const float4 n4 = D.nz[i];
        if (!(n4.w > 0.0f)) {
            D.coef[i] = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
            D.aux[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        } else {
            float ab, bb;
            if (level + 1 == L) {
                ab = D.grad_out[i];
                bb = 0.0f;
            } else {
                const float2 g = adj_out(D, level + 1, L)[i];
                ab = g.x;
                bb = g.y;
            }
            float G = 0.0f, sk = 0.0f;
#pragma unroll
            for (int b = -1; b <= 1; ++b)
#pragma unroll
                for (int a = -1; a <= 1; ++a) {
                    const int qx = (int)x + a, qy = (int)y + b;
                    if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
                    const size_t q = (size_t)qy * W + qx;
                    if (!(D.nz[q].w > 0.0f)) continue;
                    const float k = k3(a) * k3(b);
                    G = fmaf(k, cv[q].y, G);
                    sk += k;
                }
            const float g = sqrtf(G / sk);
            const float sl = P.sl[level], sz = P.sz[level], sn = P.sn[level];
            const float E = fmaf(sl, g, P.eps_l);
            const float iE = 1.0f / E;
            const float ke = kNegLog2e * iE;
            const float2 cvp = cv[i];
            const float2 dzp = D.dz[i];
            const float3 np = f3(n4);
            const float eps_zp = P.eps_z * n4.w;
            // sweep 1: tap weights (kept), normaliser and the level's outputs
            float wv[25];
            float Dn = 0.0f, Sc = 0.0f, Sv = 0.0f;
#pragma unroll
            for (int t = 0; t < 25; ++t) {
                const int a = t % 5 - 2, b = t / 5 - 2;
                wv[t] = -1.0f;
                const int qx = (int)x + s * a, qy = (int)y + s * b;
                if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
                const size_t q = (size_t)qy * W + qx;
                const float4 nq = D.nz[q];
                if (!(nq.w > 0.0f)) continue;
                const float2 c2 = cv[q];
                const float w = (a == 0 && b == 0)
                                    ? 1.0f
                                    : fused_weight(depth_coef(dzp, a, b, s, sz, eps_zp), ke, n4.w, cvp.x, np, sn, nq, c2.x);
                wv[t] = w;
                const float hw = b3(a) * b3(b) * w;
                Dn += hw;
                Sc = fmaf(hw, c2.x - cvp.x, Sc);
                Sv = fmaf(hw * hw, c2.y, Sv);
            }
            const float iD = 1.0f / Dn;
            const float cpr = fmaf(Sc, iD, cvp.x), vpr = Sv * iD * iD;
            const float A = ab * iD, Bc = bb * iD * iD;
            const float K2 = 2.0f * Bc * vpr * Dn;
            float cbar_c = 0.0f, gbar = 0.0f;
            const float iE2 = iE * iE;
            // sweep 2: weight adjoints, the centre-role terms and the sigma partials
#pragma unroll
            for (int t = 0; t < 25; ++t) {
                const int a = t % 5 - 2, b = t / 5 - 2;
                const float w = wv[t];
                if (w < 0.0f || (a == 0 && b == 0)) continue;
                const size_t q = (size_t)((int)y + s * b) * W + (size_t)((int)x + s * a);
                const float4 nq = D.nz[q];
                const float2 c2 = cv[q];
                const float h = b3(a) * b3(b);
                const float wbar = h * (A * (c2.x - cpr) - K2) + 2.0f * Bc * h * h * w * c2.y;
                const float dc = cvp.x - c2.x;
                const float ww = wbar * w;
                cbar_c -= ww * sgn(dc) * iE;
                gbar = fmaf(ww * fabsf(dc), sl * iE2, gbar);
                s_l = fmaf(ww * fabsf(dc), g * iE2, s_l);
                const float S = tap_span(dzp, a, b, s);
                const float iF = hw_rcp(fmaf(sz, S, eps_zp));
                s_z = fmaf(ww * fabsf(n4.w - nq.w), S * iF * iF, s_z);
                const float xn = fminf(dot3(np, f3(nq)), 1.0f);
                if (w > 0.0f && xn > 0.0f) s_n = fmaf(ww, hw_log2(xn) * 0.6931471805599453f, s_n);
            }
            const float Gb = g > 0.0f ? gbar / (2.0f * g) / sk : 0.0f;
            D.coef[i] = make_float4(A, Bc, cpr, iE);
            D.aux[i] = make_float4(Gb, cbar_c, K2, 0.0f);
        }
    }
    const double tz = block_sum((double)s_z, red);
    const double tn = block_sum((double)s_n, red);
    const double tl = block_sum((double)s_l, red);
    if (threadIdx.x == 0) {
        double* o = D.part + ((size_t)D.part_off[level] + tile) * 3;
        o[0] = tz;
        o[1] = tn;
        o[2] = tl;
    }
}

// Pass B on 16 x 16 tiles with taps read from global memory (deep levels).
__global__ __launch_bounds__(kSvgfBlock) void adjoint_b_direct(const BwdBatch Bt, const SvgfK P, uint32_t level) {
    const int j = find_job(Bt.tile0, (int)Bt.n, blockIdx.x);
    const BwdDesc& D = Bt.d[j];
    uint32_t x, y;
    tile_xy(blockIdx.x - Bt.tile0[j], D.tiles_x, x, y);
    if (x >= D.W || y >= D.H) return;
    const uint32_t L = P.levels;
    const int W = (int)D.W, H = (int)D.H, s = 1 << level;
    const size_t i = (size_t)y * W + x;
    float2* out = adj_out(D, level, L);
    const float4 n4 = D.nz[i];
    if (!(n4.w > 0.0f)) {
        out[i] = make_float2(0.0f, 0.0f);
        return;
    }
    const float2* cv = D.save + (size_t)level * W * H;
    const float2 cvq = cv[i];
    const float sz = P.sz[level], sn = P.sn[level];
    float acc_c = D.aux[i].y, acc_v = 0.0f;
#pragma unroll
    for (int b = -2; b <= 2; ++b) {
        const int py = (int)y - s * b;
        if (py < 0 || py >= H) continue;
#pragma unroll
        for (int a = -2; a <= 2; ++a) {
            const int px = (int)x - s * a;
            if (px < 0 || px >= W) continue;
            const size_t p = (size_t)py * W + px;
            const float4 np4 = D.nz[p];
            if (!(np4.w > 0.0f)) continue;
            const float4 cf = D.coef[p];
            const float h = b3(a) * b3(b);
            const float Kp = D.aux[p].z;
            if (a == 0 && b == 0) {
                acc_c = fmaf(cf.x, h, acc_c);
                acc_v = fmaf(cf.y, h * h, acc_v);
                continue;
            }
            const float cp = cv[p].x;
            const float iE = cf.w;
            const float w = fused_weight(depth_coef(D.dz[p], a, b, s, sz, P.eps_z * np4.w), kNegLog2e * iE, np4.w, cp,
                                         f3(np4), sn, n4, cvq.x);
            const float wbar = h * (cf.x * (cvq.x - cf.z) - Kp) + 2.0f * cf.y * h * h * w * cvq.y;
            acc_c += cf.x * h * w + wbar * w * sgn(cp - cvq.x) * iE;
            acc_v = fmaf(cf.y * h * h, w * w, acc_v);
        }
    }
    // adjoint of the 3x3 prefilter: v_q feeds g of every valid neighbour
#pragma unroll
    for (int b = -1; b <= 1; ++b)
#pragma unroll
        for (int a = -1; a <= 1; ++a) {
            const int rx = (int)x + a, ry = (int)y + b;
            if (rx < 0 || rx >= W || ry < 0 || ry >= H) continue;
            const size_t r = (size_t)ry * W + rx;
            if (!(D.nz[r].w > 0.0f)) continue;
            acc_v = fmaf(D.aux[r].x, k3(a) * k3(b), acc_v);
        }
    out[i] = make_float2(acc_c, acc_v);
}

// The same two passes on row-class tiles (levels up to kAdjRowsMax): the
// taps' geometry and inputs are staged in LDS once per workgroup, as in the
// forward levels.  Taps outside the frame or on invalid pixels are staged
// with a zero normal (their weight is zero) and, in pass B, 1/E = 1 (every
// term stays finite and vanishes).
template <int LEVEL>
__global__ __launch_bounds__(kSvgfBlock) void adjoint_a_rows(const BwdBatch Bt, const SvgfK P) {
    constexpr int s = 1 << LEVEL;
    constexpr int CW = kRowsTX + 4 * s, CH = kRowsTY + 4, GW = kRowsTX + 2;
    __shared__ float4 s_nz[CH * CW];
    __shared__ float2 s_cv[CH * CW];
    __shared__ float s_g[kRowsTY * 2 * GW];  // variance of the rows next to each output row
    __shared__ double red[kSvgfBlock / 64];
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int j = find_job(Bt.tile0, (int)Bt.n, lb);
    const BwdDesc& D = Bt.d[j];
    const int t = (int)(lb - Bt.tile0[j]);
    const int W = (int)D.W, H = (int)D.H;
    const int ntx = (W + kRowsTX - 1) / kRowsTX;
    const int X = t % ntx, rest = t / ntx;
    const int x0 = X * kRowsTX, y0 = (rest / s) * (kRowsTY * s) + rest % s;
    const float2* cv = D.save + (size_t)LEVEL * W * H;
    stage_tile<CH * CW>(
        [&](int e) {
            const int qx = x0 - 2 * s + e % CW, qy = y0 + s * (e / CW - 2);
            return load_staged(D.nz, cv, qx, qy, W, H);
        },
        [&](int e, const Staged& r) {
            const bool ok = r.nz.w > 0.0f;
            s_nz[e] = ok ? r.nz : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            s_cv[e] = ok ? r.cv : make_float2(0.0f, 0.0f);
        });
    stage_tile<kRowsTY * 2 * GW>(
        [&](int e) {
            const int qx = x0 - 1 + e % GW, qy = y0 + s * (e / (2 * GW)) + ((e / GW) % 2 ? 1 : -1);
            const size_t q = clamped_index(qx, qy, W, H);
            const float vq = cv[q].y;
            return inside(qx, qy, W, H) && D.nz[q].w > 0.0f ? vq : kNoVar;
        },
        [&](int e, float v) { s_g[e] = v; });
    __syncthreads();
    const int li = threadIdx.x % kRowsTX, lj = threadIdx.x / kRowsTX;
    const int x = x0 + li, y = y0 + s * lj;
    const int c = (lj + 2) * CW + 2 * s + li;
    float s_z = 0.0f, s_n = 0.0f, s_l = 0.0f;
    if (x < W && y < H) {
        const size_t i = (size_t)y * W + x;
        const float4 n4 = s_nz[c];
        if (!(n4.w > 0.0f)) {
            D.coef[i] = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
            D.aux[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        } else {
            const uint32_t L = P.levels;
            float ab, bb;
            if (LEVEL + 1 == (int)L) {
                ab = D.grad_out[i];
                bb = 0.0f;
            } else {
                const float2 g = adj_out(D, LEVEL + 1, L)[i];
                ab = g.x;
                bb = g.y;
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
            const float g = sqrtf(G / sk);
            const float sl = P.sl[LEVEL], sz = P.sz[LEVEL], sn = P.sn[LEVEL];
            const float E = fmaf(sl, g, P.eps_l);
            const float iE = 1.0f / E;
            const float ke = kNegLog2e * iE;
            const float2 cvp = s_cv[c];
            const float2 dzp = D.dz[i];
            const float3 np = f3(n4);
            const float eps_zp = P.eps_z * n4.w;
            // One sweep over the taps.  The weight adjoint of tap t is
            //   ww_t = wbar_t w_t = A al_t - (A d + K) be_t + 2 B ga_t
            // with be_t = h w, al_t = be_t (c_q - c_p), ga_t = be_t^2 v_q and
            // d = c' - c_p, so each sum over taps of ww_t phi_t (phi: the
            // sign and size of c_p - c_q, the depth term's sigma factor, the
            // normal term's log) is a combination of three sums that need
            // neither A, K nor c' yet: every weight is formed once.  A tap
            // and its mirror (-a, -b) share the depth reciprocal.  One pair
            // row per iteration (unrolling all taps would hoist their LDS
            // reads and hold them all in registers).
            const float h0 = b3(0) * b3(0);
            float Dn = h0, Sc = 0.0f, Sv = h0 * h0 * cvp.y;
            float pa[4] = {0.0f, 0.0f, 0.0f, 0.0f}, pb[4] = {0.0f, 0.0f, 0.0f, 0.0f},
                  pg[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
            for (int b = 0; b <= 2; ++b)
#pragma unroll
            for (int a = -2; a <= 2; ++a) {
                if (b == 0 && a <= 0) continue;  // row 0: the taps right of the centre; their mirrors below
                const float S = tap_span(dzp, a, b, s);
                const float iF = hw_rcp(fmaf(sz, S, eps_zp));
                const float kz = kNegLog2e * iF, fz = S * iF * iF;
                const float h = b3(a) * b3(b);
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    const int e = m ? c - b * CW - s * a : c + b * CW + s * a;
                    const float4 nq = s_nz[e];
                    const float2 c2 = s_cv[e];
                    const float xn = fminf(dot3(np, f3(nq)), 1.0f);
                    const float lx = hw_log2(xn);
                    const float adz = fabsf(n4.w - nq.w);
                    const float dc = cvp.x - c2.x;
                    const float ew = fmaf(kz, adz, fmaf(ke, fabsf(dc), sn * lx));
                    const float w = xn > 0.0f ? hw_exp2(ew) : 0.0f;
                    const float be = h * w, al = -be * dc, ga = be * be * c2.y;
                    Dn += be;
                    Sc += al;
                    Sv += ga;
                    const float phi[4] = {sgn(dc), fabsf(dc), adz * fz, w > 0.0f && xn > 0.0f ? lx : 0.0f};
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        pa[k] = fmaf(al, phi[k], pa[k]);
                        pb[k] = fmaf(be, phi[k], pb[k]);
                        pg[k] = fmaf(ga, phi[k], pg[k]);
                    }
                }
            }
            const float iD = 1.0f / Dn;
            const float dlt = Sc * iD, cpr = cvp.x + dlt, vpr = Sv * iD * iD;
            const float A = ab * iD, Bc = bb * iD * iD;
            const float K2 = 2.0f * Bc * vpr * Dn;
            const float mu = fmaf(A, dlt, K2), B2 = 2.0f * Bc;
            float sum[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) sum[k] = fmaf(A, pa[k], fmaf(-mu, pb[k], B2 * pg[k]));
            const float iE2 = iE * iE;
            const float cbar_c = -sum[0] * iE;
            const float gbar = sum[1] * (sl * iE2);
            s_l += sum[1] * (g * iE2);
            s_z += sum[2];
            s_n += sum[3] * 0.6931471805599453f;
            const float Gb = g > 0.0f ? gbar / (2.0f * g) / sk : 0.0f;
            D.coef[i] = make_float4(A, Bc, cpr, iE);
            D.aux[i] = make_float4(Gb, cbar_c, K2, 0.0f);
        }
    }
    const double tz = block_sum((double)s_z, red);
    const double tn = block_sum((double)s_n, red);
    const double tl = block_sum((double)s_l, red);
    if (threadIdx.x == 0) {
        double* o = D.part + ((size_t)D.part_off[LEVEL] + t) * 3;
        o[0] = tz;
        o[1] = tn;
        o[2] = tl;
    }
}

// Pass B staging: a centre pixel p's geometry, its coefficients (A, B, c', 1/E)
// and (c_p, K_p, dz_p).
struct StagedP {
    float4 nz, cf, ck;
};

template <int LEVEL>
__global__ __launch_bounds__(kSvgfBlock) void adjoint_b_rows(const BwdBatch Bt, const SvgfK P) {
    constexpr int s = 1 << LEVEL;
    constexpr int CW = kRowsTX + 4 * s, CH = kRowsTY + 4, GW = kRowsTX + 2;
    __shared__ float4 s_nz[CH * CW];
    __shared__ float4 s_cf[CH * CW];
    __shared__ float4 s_ck[CH * CW];         // (c_p, K_p, dz_p.x, dz_p.y)
    __shared__ float s_gb[kRowsTY * 3 * GW];  // prefilter adjoint of the rows around each output row
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int j = find_job(Bt.tile0, (int)Bt.n, lb);
    const BwdDesc& D = Bt.d[j];
    const int t = (int)(lb - Bt.tile0[j]);
    const int W = (int)D.W, H = (int)D.H;
    const int ntx = (W + kRowsTX - 1) / kRowsTX;
    const int X = t % ntx, rest = t / ntx;
    const int x0 = X * kRowsTX, y0 = (rest / s) * (kRowsTY * s) + rest % s;
    const float2* cv = D.save + (size_t)LEVEL * W * H;
    stage_tile<CH * CW>(
        [&](int e) {
            // outside the frame: the nearest pixel's records, marked invalid
            // (depth 0), which the store replaces by the neutral ones
            const int px = x0 - 2 * s + e % CW, py = y0 + s * (e / CW - 2);
            const size_t p = clamped_index(px, py, W, H);
            const float2 dz = D.dz[p];
            StagedP r{D.nz[p], D.coef[p], make_float4(cv[p].x, D.aux[p].z, dz.x, dz.y)};
            if (!inside(px, py, W, H)) r.nz.w = 0.0f;
            return r;
        },
        [&](int e, const StagedP& r) {
            const bool ok = r.nz.w > 0.0f;
            s_nz[e] = ok ? r.nz : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            s_cf[e] = ok ? r.cf : make_float4(0.0f, 0.0f, 0.0f, 1.0f);
            s_ck[e] = ok ? r.ck : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        });
    stage_tile<kRowsTY * 3 * GW>(
        [&](int e) {
            const int rx = x0 - 1 + e % GW, ry = y0 + s * (e / (3 * GW)) + (e / GW) % 3 - 1;
            const float v = D.aux[clamped_index(rx, ry, W, H)].x;
            return inside(rx, ry, W, H) ? v : 0.0f;
        },
        [&](int e, float v) { s_gb[e] = v; });
    __syncthreads();
    const int li = threadIdx.x % kRowsTX, lj = threadIdx.x / kRowsTX;
    const int x = x0 + li, y = y0 + s * lj;
    if (x >= W || y >= H) return;
    const uint32_t L = P.levels;
    const size_t i = (size_t)y * W + x;
    float2* out = adj_out(D, LEVEL, L);
    const int c = (lj + 2) * CW + 2 * s + li;
    const float4 n4 = s_nz[c];
    if (!(n4.w > 0.0f)) {
        out[i] = make_float2(0.0f, 0.0f);
        return;
    }
    const float2 cvq = cv[i];
    const float sz = P.sz[LEVEL], sn = P.sn[LEVEL];
    float acc_c = D.aux[i].y, acc_v = 0.0f;
#pragma unroll
    for (int b = -2; b <= 2; ++b) {
#pragma unroll
        for (int a = -2; a <= 2; ++a) {
            // centre pixel p = q - s (a, b), whose tap (a, b) is this pixel
            const int e = c - b * CW - s * a;
            const float4 cf = s_cf[e];
            const float h = b3(a) * b3(b);
            if (a == 0 && b == 0) {
                acc_c = fmaf(cf.x, h, acc_c);
                acc_v = fmaf(cf.y, h * h, acc_v);
                continue;
            }
            const float4 np4 = s_nz[e];
            const float4 ck = s_ck[e];
            const float cp = ck.x, Kp = ck.y;
            const float iE = cf.w;
            const float w = fused_weight(depth_coef(make_float2(ck.z, ck.w), a, b, s, sz, P.eps_z * np4.w),
                                         kNegLog2e * iE, np4.w, cp, f3(np4), sn, n4, cvq.x);
            const float wbar = h * (cf.x * (cvq.x - cf.z) - Kp) + 2.0f * cf.y * h * h * w * cvq.y;
            acc_c += cf.x * h * w + wbar * w * sgn(cp - cvq.x) * iE;
            acc_v = fmaf(cf.y * h * h, w * w, acc_v);
        }
    }
    // adjoint of the 3x3 prefilter: v_q feeds g of every valid neighbour
    // (invalid neighbours carry a zero prefilter adjoint)
#pragma unroll
    for (int b = -1; b <= 1; ++b)
#pragma unroll
        for (int a = -1; a <= 1; ++a) acc_v = fmaf(s_gb[(3 * lj + b + 1) * GW + li + 1 + a], k3(a) * k3(b), acc_v);
    out[i] = make_float2(acc_c, acc_v);
}

// grad_sigma[fam * L + l] = sum over frames and workgroup partials, in a
// fixed order: lane t of the block keeps four independent sums (partials t,
// t + 1024, t + 2048, t + 3072 of each stride of 4096) so that four loads are
// in flight per lane.
constexpr int kReduceBlock = 1024;

__global__ __launch_bounds__(kReduceBlock) void sigma_reduce_kernel(const BwdBatch Bt, uint32_t L, float* grad_sigma,
                                                                    int accumulate) {
    __shared__ double red[kReduceBlock / 64];
    const uint32_t o = blockIdx.x;  // fam * L + l
    const uint32_t fam = o / L, l = o % L;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (uint32_t f = 0; f < Bt.n; ++f) {
        const BwdDesc& D = Bt.d[f];
        const double* p = D.part + (size_t)D.part_off[l] * 3 + fam;
        const uint32_t nt = D.part_off[l + 1] - D.part_off[l];
        for (uint32_t t = threadIdx.x; t < nt; t += 4 * kReduceBlock) {
            a0 += p[(size_t)t * 3];
            if (t + kReduceBlock < nt) a1 += p[(size_t)(t + kReduceBlock) * 3];
            if (t + 2 * kReduceBlock < nt) a2 += p[(size_t)(t + 2 * kReduceBlock) * 3];
            if (t + 3 * kReduceBlock < nt) a3 += p[(size_t)(t + 3 * kReduceBlock) * 3];
        }
    }
    double acc = (a0 + a1) + (a2 + a3);
#pragma unroll
    for (int k = 32; k > 0; k >>= 1) acc += __shfl_xor(acc, k, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int k = 0; k < kReduceBlock / 64; ++k) tot += red[k];
        grad_sigma[o] = accumulate ? (float)((double)grad_sigma[o] + tot) : (float)tot;
    }
}

__global__ void zero_kernel(float* p, uint32_t n) {
    for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) p[k] = 0.0f;
}

void launch_adjoint_rows(uint32_t level, dim3 grid, hipStream_t s, const BwdBatch& B, const SvgfK& K) {
    switch (level) {
        case 0:
            hipLaunchKernelGGL(adjoint_a_rows<0>, grid, dim3(kSvgfBlock), 0, s, B, K);
            hipLaunchKernelGGL(adjoint_b_rows<0>, grid, dim3(kSvgfBlock), 0, s, B, K);
            break;
        case 1:
            hipLaunchKernelGGL(adjoint_a_rows<1>, grid, dim3(kSvgfBlock), 0, s, B, K);
            hipLaunchKernelGGL(adjoint_b_rows<1>, grid, dim3(kSvgfBlock), 0, s, B, K);
            break;
        case 2:
            hipLaunchKernelGGL(adjoint_a_rows<2>, grid, dim3(kSvgfBlock), 0, s, B, K);
            hipLaunchKernelGGL(adjoint_b_rows<2>, grid, dim3(kSvgfBlock), 0, s, B, K);
            break;
        case 3:
            hipLaunchKernelGGL(adjoint_a_rows<3>, grid, dim3(kSvgfBlock), 0, s, B, K);
            hipLaunchKernelGGL(adjoint_b_rows<3>, grid, dim3(kSvgfBlock), 0, s, B, K);
            break;
        default:
            hipLaunchKernelGGL(adjoint_a_rows<4>, grid, dim3(kSvgfBlock), 0, s, B, K);
            hipLaunchKernelGGL(adjoint_b_rows<4>, grid, dim3(kSvgfBlock), 0, s, B, K);
            break;
    }
}

}  // namespace
}  // namespace dhr

extern "C" {

dhr_status dhr_svgf_backward(dhr_ctx* ctx, const dhr_svgf_params* params, const dhr_svgf_bwd_frame* frames,
                             uint32_t n_frames, float* grad_sigma, dhr_stream stream) {
    using namespace dhr;
    if (!ctx) return DHR_ERR_INVALID_ARG;
    dhr_status st = svgf_check_params(ctx, params, "dhr_svgf_backward");
    if (st != DHR_OK) return st;
    if (params->kernel_width != 5)
        return set_error(ctx, DHR_ERR_UNSUPPORTED, "dhr_svgf_backward: the adjoint takes kernel_width 5 only");
    if (!grad_sigma || (n_frames && !frames))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_svgf_backward: null pointer");
    const uint32_t L = params->levels;
    std::vector<BwdDesc> descs(n_frames);
    for (uint32_t k = 0; k < n_frames; ++k) {
        const dhr_svgf_bwd_frame& F = frames[k];
        if (F.W < 1 || F.H < 1 || F.W > DHR_MAX_SIDE || F.H > DHR_MAX_SIDE)
            return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_svgf_backward: frame %u: bad size", k);
        if (!F.save || !F.nz || !F.dz || !F.grad_out || !F.grad_cv || !F.work)
            return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_svgf_backward: frame %u: missing buffer", k);
        if (!aligned8(F.save) || !aligned16(F.nz) || !aligned8(F.dz) || !aligned8(F.grad_cv) || !aligned16(F.work))
            return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_svgf_backward: frame %u: misaligned buffer", k);
        const size_t HW = (size_t)F.W * F.H;
        BwdDesc& d = descs[k];
        std::memset(&d, 0, sizeof d);
        d.W = F.W;
        d.H = F.H;
        d.tiles_x = (F.W + kSvgfTile - 1) / kSvgfTile;
        d.tiles = d.tiles_x * ((F.H + kSvgfTile - 1) / kSvgfTile);
        d.save = reinterpret_cast<const float2*>(F.save);
        d.nz = reinterpret_cast<const float4*>(F.nz);
        d.dz = reinterpret_cast<const float2*>(F.dz);
        d.grad_out = F.grad_out;
        d.grad_cv = reinterpret_cast<float2*>(F.grad_cv);
        char* w = reinterpret_cast<char*>(F.work);
        d.coef = reinterpret_cast<float4*>(w);
        d.g0 = reinterpret_cast<float2*>(w + HW * 16);
        d.g1 = reinterpret_cast<float2*>(w + HW * 24);
        d.aux = reinterpret_cast<float4*>(w + HW * 32);
        d.part = reinterpret_cast<double*>(w + HW * 48);
        uint32_t acc = 0;
        for (uint32_t l = 0; l <= DHR_MAX_LEVELS; ++l) {
            d.part_off[l] = acc;
            if (l < L) acc += adjoint_tiles(F.W, F.H, l);
        }
    }
    DeviceGuard g(ctx->device);
    const SvgfK K = [&] {
        SvgfK k;
        std::memset(&k, 0, sizeof k);
        k.levels = L;
        for (int l = 0; l < DHR_MAX_LEVELS; ++l) {
            k.sz[l] = params->sigma_z[l];
            k.sn[l] = params->sigma_n[l];
            k.sl[l] = params->sigma_l[l];
        }
        k.eps_z = params->eps_z_rel;
        k.eps_l = params->eps_l;
        return k;
    }();
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (n_frames == 0) {
        // a fill kernel rather than a memset node, so the call can be captured in a graph
        hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s, grad_sigma, 3 * L);
        return check_launch(ctx, "dhr_svgf_backward");
    }
    for (size_t b0 = 0; b0 < descs.size(); b0 += kBwdMaxB) {
        BwdBatch B;
        std::memset(&B, 0, sizeof B);
        const size_t n = std::min<size_t>(kBwdMaxB, descs.size() - b0);
        B.n = (uint32_t)n;
        for (size_t k = 0; k < n; ++k) B.d[k] = descs[b0 + k];
        for (int l = (int)L - 1; l >= 0; --l) {
            // workgroup prefix of this level's tiling
            uint64_t tot = 0;
            for (size_t k = 0; k < n; ++k) {
                B.tile0[k] = (uint32_t)tot;
                tot += adjoint_tiles(descs[b0 + k].W, descs[b0 + k].H, (uint32_t)l);
            }
            B.tile0[n] = (uint32_t)tot;
            if (tot > 0x7FFFFFFFull) return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_svgf_backward: batch too large");
            if (l <= (int)kAdjRowsMax) {
                launch_adjoint_rows((uint32_t)l, dim3((uint32_t)tot), s, B, K);
            } else {
                hipLaunchKernelGGL(adjoint_a_direct, dim3((uint32_t)tot), dim3(kSvgfBlock), 0, s, B, K, (uint32_t)l);
                hipLaunchKernelGGL(adjoint_b_direct, dim3((uint32_t)tot), dim3(kSvgfBlock), 0, s, B, K, (uint32_t)l);
            }
        }
        hipLaunchKernelGGL(sigma_reduce_kernel, dim3(3 * L), dim3(kReduceBlock), 0, s, B, L, grad_sigma, b0 > 0 ? 1 : 0);
        st = check_launch(ctx, "dhr_svgf_backward");
        if (st != DHR_OK) return st;
    }
    return DHR_OK;
}

}  // extern "C"
