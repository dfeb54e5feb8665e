// Pinhole camera of the G-buffer passes and the texel a primary hit writes
// (Section 2.2: world-space position per pixel; Section 3.3: motion vectors
// back-project a pixel into the previous frame).  Shared by the ray-traced
// and the rasterised G-buffer, so both write identical texels for the same
// hit.
#pragma once

#include <cmath>

#include "device.h"
#include "internal.h"

// Operations round separately unless an fmaf is written (both G-buffer
// kernels inline these functions and must agree bit for bit).
#pragma clang fp contract(off)

namespace dhr {

struct CamD {
    float eye[3], fwd[3], right[3], up[3];
    float tx, ty;  // tan(fov/2) * aspect, tan(fov/2)
    float kx, ky;  // 2 tx / W, 2 ty / H: image-plane step per pixel
};

// Orthonormal frame of a look-at camera (up hint +y), computed in double on
// the host and rounded once.  False for a degenerate camera.
inline bool make_cam(const dhr_camera& c, uint32_t W, uint32_t H, CamD* out) {
    double e[3], f[3];
    for (int k = 0; k < 3; ++k) {
        e[k] = c.eye[k];
        f[k] = (double)c.target[k] - (double)c.eye[k];
    }
    double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(fl > 0.0) || !std::isfinite(fl) || !(c.fov_y > 0.0f) || !(c.fov_y < 3.14f)) return false;
    for (double& v : f) v /= fl;
    double r[3] = {f[1] * 0.0 - f[2] * 1.0, f[2] * 0.0 - f[0] * 0.0, f[0] * 1.0 - f[1] * 0.0};  // fwd x (0,1,0)
    double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(rl > 1e-9)) return false;
    for (double& v : r) v /= rl;
    double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
    for (int k = 0; k < 3; ++k) {
        out->eye[k] = (float)e[k];
        out->fwd[k] = (float)f[k];
        out->right[k] = (float)r[k];
        out->up[k] = (float)u[k];
    }
    const double th = std::tan(0.5 * (double)c.fov_y);
    out->tx = (float)(th * (double)W / (double)H);
    out->ty = (float)th;
    out->kx = (float)(2.0 * th / (double)H);  // 2 tx / W
    out->ky = (float)(2.0 * th / (double)H);
    return true;
}

// Unit direction of the ray through image point (px, py) (pixel centres at
// x + 0.5, y + 0.5): image-plane offsets px kx - tx and ty - py ky, then a
// hardware reciprocal square root (about 1 ulp) normalises.
__device__ __forceinline__ float3 cam_dir(const CamD& c, float px, float py) {
    const float sx = fmaf(px, c.kx, -c.tx);
    const float sy = fmaf(-py, c.ky, c.ty);
    const float3 d = f3(fmaf(c.up[0], sy, fmaf(c.right[0], sx, c.fwd[0])),
                        fmaf(c.up[1], sy, fmaf(c.right[1], sx, c.fwd[1])),
                        fmaf(c.up[2], sy, fmaf(c.right[2], sx, c.fwd[2])));
    return d * __builtin_amdgcn_rsqf(dot3(d, d));
}

// G-buffer texel of pixel (x, y) whose ray d from the eye hits the triangle
// record `rec` (v0 + original index, e1 + object id, e2) at t, or nothing
// (rec NULL): position + object id, viewer-facing unit normal + view depth,
// the depth of the hit plane through the next pixel to the right and below
// (1e20 where that ray misses the plane), and the motion to the previous
// frame's pixel (NaN when the point is behind the previous camera).
__device__ __forceinline__ void gbuffer_texel(const CamD& C, const CamD& Q, bool has_prev, uint32_t W, uint32_t H,
                                              uint32_t x, uint32_t y, float3 d, const float4* rec, float t,
                                              float4& pos_out, float4& nz_out, float2& dz_out, float2& mv_out) {
    if (!rec) {
        pos_out = make_float4(0.0f, 0.0f, 0.0f, __uint_as_float(DHR_MISS_ID));
        nz_out = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        dz_out = make_float2(0.0f, 0.0f);
        mv_out = make_float2(0.0f, 0.0f);
        return;
    }
    const float3 eye = f3(C.eye[0], C.eye[1], C.eye[2]);
    const float3 fwd = f3(C.fwd[0], C.fwd[1], C.fwd[2]);
    const float4 v0 = rec[0];
    const float4 e1 = rec[1];
    const float4 e2 = rec[2];
    const float3 P = f3(fmaf(d.x, t, eye.x), fmaf(d.y, t, eye.y), fmaf(d.z, t, eye.z));
    float3 nrm = normalize3(cross3(f3(e1), f3(e2)));
    if (dot3(nrm, d) > 0.0f) nrm = nrm * -1.0f;
    const float z = t * dot3(d, fwd);
    pos_out = make_float4(P.x, P.y, P.z, e1.w);
    nz_out = make_float4(nrm.x, nrm.y, nrm.z, z);
    float dzv[2];
    const float pd = dot3(f3(v0) - eye, nrm);
    for (int k = 0; k < 2; ++k) {
        const float3 d1 = cam_dir(C, x + 0.5f + (k == 0), y + 0.5f + (k == 1));
        const float den = dot3(d1, nrm);
        float out = 1e20f;
        if (den != 0.0f) {
            const float t1 = pd / den;
            if (t1 > 0.0f) out = fmaf(t1, dot3(d1, fwd), -z);
        }
        dzv[k] = out;
    }
    dz_out = make_float2(dzv[0], dzv[1]);
    float2 mv = make_float2(__builtin_nanf(""), __builtin_nanf(""));
    if (has_prev) {
        const float3 v = P - f3(Q.eye[0], Q.eye[1], Q.eye[2]);
        const float zc = dot3(v, f3(Q.fwd[0], Q.fwd[1], Q.fwd[2]));
        if (zc > 0.0f) {
            const float xc = dot3(v, f3(Q.right[0], Q.right[1], Q.right[2])) / zc;
            const float yc = dot3(v, f3(Q.up[0], Q.up[1], Q.up[2])) / zc;
            const float px = (xc / Q.tx + 1.0f) * 0.5f * (float)W;
            const float py = (1.0f - yc / Q.ty) * 0.5f * (float)H;
            mv = make_float2(px - (x + 0.5f), py - (y + 0.5f));
        }
    }
    mv_out = mv;
}

}  // namespace dhr

#pragma clang fp contract(fast)
