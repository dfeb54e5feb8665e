// Oracle (test infrastructure only): G-buffer of primary rays and the
// stochastic visibility rays (ambient occlusion and soft shadows).
//
// Paper references:
//  * Section 2.2: a shadow ray from each pixel's world-space position towards
//    every light; Section 3.1: the ray direction is drawn at random inside the
//    cone subtended by the light, with the light distance kept.
//  * Section 3.2, eqs. (1)-(3): N cosine-weighted hemisphere rays of length r;
//    a ray is unoccluded iff it meets nothing closer than r; the pixel stores
//    N_unoccluded as one byte (N <= 255).
//  * Section 3.3: the G-buffer holds motion vectors that back-project the
//    pixel's world position into the previous frame.
#include <algorithm>

#include "orc.h"
#include "orc_common.h"

namespace orc {
namespace {

const float kDzSentinel = 1e20f;   // plane not seen at the neighbouring pixel
const uint32_t kMissId = 0xFFFFFFFFu;

struct Cam {
    V3 eye, fwd, right, up;
    double tan_half, aspect;
    int W, H;
};

Cam make_cam(const orc_camera& c, int W, int H) {
    Cam k;
    k.eye = V3{c.eye[0], c.eye[1], c.eye[2]};
    V3 tgt{c.target[0], c.target[1], c.target[2]};
    k.fwd = normalize(tgt - k.eye);
    k.right = normalize(cross(k.fwd, V3{0.0, 1.0, 0.0}));
    k.up = cross(k.right, k.fwd);
    k.tan_half = std::tan(0.5 * c.fov_y);
    k.aspect = (double)W / (double)H;
    k.W = W;
    k.H = H;
    return k;
}

// Direction through the continuous pixel position (px, py); pixel centres are
// at integer + 0.5, row 0 at the top.
V3 pixel_dir(const Cam& c, double px, double py) {
    double sx = (2.0 * px / c.W - 1.0) * c.tan_half * c.aspect;
    double sy = (1.0 - 2.0 * py / c.H) * c.tan_half;
    return normalize(c.fwd + c.right * sx + c.up * sy);
}

bool project(const Cam& c, const V3& P, double* px, double* py) {
    V3 v = P - c.eye;
    double zc = dot(v, c.fwd);
    if (!(zc > 0.0)) return false;
    double xc = dot(v, c.right) / zc;
    double yc = dot(v, c.up) / zc;
    *px = (xc / (c.tan_half * c.aspect) + 1.0) * 0.5 * c.W;
    *py = (1.0 - yc / c.tan_half) * 0.5 * c.H;
    return true;
}

float id_bits(uint32_t id) {
    float f;
    std::memcpy(&f, &id, 4);
    return f;
}

}  // namespace
}  // namespace orc

extern "C" {

void orc_gbuffer(const orc_scene* sc, const orc_camera* cur, const orc_camera* prev, int W, int H,
                 float* pos, float* nz, float* dz, float* mv) {
    using namespace orc;
    const Cam cam = make_cam(*cur, W, H);
    Cam pcam;
    if (prev) pcam = make_cam(*prev, W, H);
    const float fnan = std::numeric_limits<float>::quiet_NaN();
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const int64_t i = (int64_t)y * W + x;
            V3 d = pixel_dir(cam, x + 0.5, y + 0.5);
            double t;
            const Tri* tri;
            closest_bvh(sc->s, cam.eye, d, &t, &tri);
            if (!tri) {
                pos[4 * i] = pos[4 * i + 1] = pos[4 * i + 2] = 0.0f;
                pos[4 * i + 3] = id_bits(kMissId);
                nz[4 * i] = nz[4 * i + 1] = nz[4 * i + 2] = nz[4 * i + 3] = 0.0f;
                dz[2 * i] = dz[2 * i + 1] = 0.0f;
                mv[2 * i] = mv[2 * i + 1] = 0.0f;
                continue;
            }
            V3 P = cam.eye + d * t;
            V3 n = normalize(cross(tri->v1 - tri->v0, tri->v2 - tri->v0));
            if (dot(n, d) > 0.0) n = n * -1.0;
            double z = t * dot(d, cam.fwd);
            pos[4 * i] = (float)P.x;
            pos[4 * i + 1] = (float)P.y;
            pos[4 * i + 2] = (float)P.z;
            pos[4 * i + 3] = id_bits(tri->obj);
            nz[4 * i] = (float)n.x;
            nz[4 * i + 1] = (float)n.y;
            nz[4 * i + 2] = (float)n.z;
            nz[4 * i + 3] = (float)z;
            // depth of the hit triangle's plane seen through pixel +x and +y
            for (int k = 0; k < 2; ++k) {
                V3 d1 = pixel_dir(cam, x + 0.5 + (k == 0), y + 0.5 + (k == 1));
                double den = dot(d1, n);
                float out = kDzSentinel;
                if (den != 0.0) {
                    double t1 = dot(tri->v0 - cam.eye, n) / den;
                    if (t1 > 0.0) out = (float)(t1 * dot(d1, cam.fwd) - z);
                }
                dz[2 * i + k] = out;
            }
            double px, py;
            if (prev && project(pcam, P, &px, &py)) {
                mv[2 * i] = (float)(px - (x + 0.5));
                mv[2 * i + 1] = (float)(py - (y + 0.5));
            } else {
                mv[2 * i] = mv[2 * i + 1] = fnan;
            }
        }
    }
}

void orc_trace(const orc_scene* sc, const orc_trace_params* P, const float* pos, const float* nz,
               const int64_t* pix_list, int64_t n_pix, uint8_t* ao_count, uint8_t* shadow_count,
               uint64_t* ray_bits) {
    using namespace orc;
    const int64_t HW = (int64_t)P->W * P->H;
    const int64_t count = pix_list ? n_pix : HW;
    const int streams = 1 + P->n_lights;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < count; ++j) {
        const int64_t i = pix_list ? pix_list[j] : j;
        const uint32_t x = (uint32_t)(i % P->W), y = (uint32_t)(i / P->W);
        uint64_t bits[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        const bool valid = nz[4 * i + 3] > 0.0f;
        int ao_unocc = 0;
        int sh_unocc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (!valid) {
            ao_unocc = P->n_ao;
            for (int s = 0; s < P->n_ao && s < 64; ++s) bits[0] |= 1ull << s;
            for (int l = 0; l < P->n_lights; ++l) {
                sh_unocc[l] = P->n_shadow;
                for (int s = 0; s < P->n_shadow && s < 64; ++s) bits[1 + l] |= 1ull << s;
            }
        } else {
            V3 p{pos[4 * i], pos[4 * i + 1], pos[4 * i + 2]};
            V3 n = normalize(V3{nz[4 * i], nz[4 * i + 1], nz[4 * i + 2]});
            double eps = P->eps_origin_abs;
            if (!(eps > 0.0)) {
                double m = std::max({std::fabs(p.x), std::fabs(p.y), std::fabs(p.z)});
                eps = std::max(1e-3 * P->ao_radius, std::ldexp(m, -17));
            }
            V3 o = p + n * eps;
            // ambient occlusion: eqs. (2)-(3)
            for (int s = 0; s < P->n_ao; ++s) {
                double u0, u1;
                ray_uniforms(P->seed, P->client_id, x, y, P->frame, 0, P->ao_sample_offset + s, &u0, &u1);
                V3 w = sample_cosine(n, u0, u1);
                bool occ = anyhit_bvh(sc->s, o, w, P->ao_radius);
                if (!occ) {
                    ++ao_unocc;
                    if (s < 64) bits[0] |= 1ull << s;
                }
            }
            // soft shadows: Section 3.1
            for (int l = 0; l < P->n_lights; ++l) {
                const orc_light& L = P->lights[l];
                for (int s = 0; s < P->n_shadow; ++s) {
                    double u0, u1;
                    ray_uniforms(P->seed, P->client_id, x, y, P->frame, 1 + l, s, &u0, &u1);
                    bool occ;
                    if (L.kind == 0) {
                        V3 axis = normalize(V3{L.vec[0], L.vec[1], L.vec[2]});
                        V3 w = sample_cone(axis, L.one_minus_cos, u0, u1);
                        occ = dot(n, w) <= 0.0 ? true : anyhit_bvh(sc->s, o, w, kInf);
                    } else {
                        V3 C{L.vec[0], L.vec[1], L.vec[2]};
                        V3 D = C - o;
                        double dist = length(D);
                        if (dist <= L.radius) {
                            occ = false;
                        } else {
                            V3 axis = D * (1.0 / dist);
                            double q = (L.radius / dist) * (L.radius / dist);
                            double k = q / (1.0 + std::sqrt(1.0 - q));
                            V3 w = sample_cone(axis, k, u0, u1);
                            if (dot(n, w) <= 0.0) {
                                occ = true;
                            } else {
                                double b = dot(w, D);
                                double c = dist * dist - L.radius * L.radius;
                                double disc = std::max(b * b - c, 0.0);
                                double tl = b - std::sqrt(disc);
                                occ = anyhit_bvh(sc->s, o, w, tl);
                            }
                        }
                    }
                    if (!occ) {
                        ++sh_unocc[l];
                        if (s < 64) bits[1 + l] |= 1ull << s;
                    }
                }
            }
        }
        ao_count[j] = (uint8_t)ao_unocc;
        for (int l = 0; l < P->n_lights; ++l) shadow_count[(int64_t)l * count + j] = (uint8_t)sh_unocc[l];
        if (ray_bits)
            for (int st = 0; st < streams; ++st) ray_bits[(int64_t)st * count + j] = bits[st];
    }
}

}  // extern "C"
