/*
 * CPU oracle of the DHR+S server hot path (arxiv 2406.06963): TEST
 * INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product path never
 * links, loads or calls it, and it shares no code, header or constant table
 * with the HIP library.
 *
 * Plain, slow, obviously correct: FP64 arithmetic, loops in the order the
 * method is described, OpenMP only across independent pixels.  Inputs are the
 * same fp32 buffers the GPU path reads; outputs are FP64.
 *
 * Where a floating-point comparison decides a discrete outcome inside the
 * temporal filter (normal and plane-distance consistency of a history tap),
 * the decision is taken in fp32 with an operation order fixed by this file,
 * so that both implementations take the same decision; everything else is
 * FP64.
 *
 * Layouts (row-major pixel index i = y*W + x, row 0 at the top):
 *   pos  float[HW][4]  world position xyz, w = object id bits (0xFFFFFFFF = miss)
 *   nz   float[HW][4]  unit geometric normal facing the viewer, w = view depth
 *                      (> 0 iff the pixel is valid)
 *   dz   float[HW][2]  depth of the hit plane at pixel +x / +y minus depth
 *   mv   float[HW][2]  motion to the history camera, in pixels
 *   hist float[HW][4]  (c, mu1, mu2, history length)
 *
 * The history is an fp32 buffer: the temporal step rounds its result to fp32
 * once when it stores it (returned here as FP64 values that are exactly
 * representable in fp32), and the variance estimate reads the stored values.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double eye[3]; double target[3]; double fov_y; } orc_camera;

typedef struct {
    int32_t kind;          /* 0 directional, 1 sphere */
    double vec[3];         /* unit direction towards the light, or sphere centre */
    double one_minus_cos;  /* directional: 1 - cos(cone half-angle) */
    double radius;         /* sphere radius */
} orc_light;

typedef struct {
    int32_t W, H;
    uint32_t frame, client_id, seed;
    int32_t n_ao; uint32_t ao_sample_offset; double ao_radius;
    int32_t n_shadow, n_lights;
    orc_light lights[8];
    double eps_origin_abs;  /* 0 => max(1e-3 * ao_radius, 2^-17 * |p|_inf) */
} orc_trace_params;

typedef struct {
    int32_t levels;
    double alpha, alpha_moments;
    double sigma_z[8], sigma_n[8], sigma_l[8];
    double eps_z_rel, eps_l;
    float cos_normal_min, plane_px;   /* decision thresholds (fp32 decisions) */
    int32_t use_obj_id, var_min_history, fallback_radius, feedback_level;
    double history_cap;
    int32_t kernel_width;   /* 5: B3 spline taps; 3: (1,2,1)/4 taps */
} orc_svgf_params;

/* ---- counter-based RNG: Philox4x32-10 (Salmon et al., SC'11) ---- */
void orc_philox4x32_10(uint32_t k0, uint32_t k1, const uint32_t* ctr, uint32_t* out, int64_t n);

/* ---- samplers (unit vectors, FP64) ---- */
void orc_sample_cosine(const double* n, const double* u, double* out, int64_t count);
void orc_sample_cone(const double* axis, double one_minus_cos, const double* u, double* out, int64_t count);

/* ---- scene: own median-split BVH over fp32 triangles [T][3][3] ---- */
typedef struct orc_scene orc_scene;
orc_scene* orc_scene_create(const float* tris, const uint32_t* obj_id, int64_t T);
void orc_scene_destroy(orc_scene*);
int orc_scene_depth(const orc_scene*);

/* any-hit of n rays (o[3], d[3], tmax) against the BVH and by brute force;
 * hit_bvh / hit_brute: 0/1 per ray. */
void orc_anyhit(const orc_scene*, const double* o, const double* d, const double* tmax,
                int64_t n, uint8_t* hit_bvh, uint8_t* hit_brute);
/* closest hit: t (inf on miss) and original triangle index (-1 on miss). */
void orc_closest(const orc_scene*, const double* o, const double* d, int64_t n,
                 double* t, int64_t* tri, int use_brute);

/* ---- G-buffer of primary rays (fp32 outputs, rounded once) ---- */
void orc_gbuffer(const orc_scene*, const orc_camera* cur, const orc_camera* prev /*NULL*/,
                 int W, int H, float* pos, float* nz, float* dz, float* mv);

/* ---- visibility rays ----
 * ao_count [HW], shadow_count [n_lights][HW]; ray_bits NULL or
 * [1 + n_lights][HW] (bit s set iff sample s is unoccluded, needs n <= 64).
 * pix_list NULL => all pixels; else n_pix pixel indices (outputs indexed by
 * position in the list). */
void orc_trace(const orc_scene*, const orc_trace_params*, const float* pos, const float* nz,
               const int64_t* pix_list, int64_t n_pix,
               uint8_t* ao_count, uint8_t* shadow_count, uint64_t* ray_bits);

/* ---- SVGF forward ---- */
void orc_svgf_temporal(const orc_svgf_params*, int W, int H, int n_ao, const uint8_t* ao_count,
                       const float* pos, const float* nz, const float* mv,
                       const float* prev_pos, const float* prev_nz, const float* hist_in,
                       float pix, double* hist_out);
void orc_svgf_variance(const orc_svgf_params*, int W, int H, const double* hist,
                       const float* nz, const float* dz, double* cv);
void orc_svgf_atrous(const orc_svgf_params*, int W, int H, int level, const double* cv_in,
                     const float* nz, const float* dz, double* cv_out);
/* full frame: temporal -> variance -> levels, level feedback into hist_out.c;
 * cv0 (NULL or [HW][2]) receives the variance-pass output, save (NULL or
 * [levels][HW][2]) each level's input. */
void orc_svgf_filter(const orc_svgf_params*, int W, int H, int n_ao, const uint8_t* ao_count,
                     const float* pos, const float* nz, const float* dz, const float* mv,
                     const float* prev_pos, const float* prev_nz, const float* hist_in,
                     float pix, double* hist_out, double* out, double* cv0, double* save);

/* spatial stack only (differentiable part): cv_in [HW][2] -> out [HW] */
void orc_svgf_spatial(const orc_svgf_params*, int W, int H, const double* cv_in,
                      const float* nz, const float* dz, double* out, double* save);
/* vector-Jacobian product of the spatial stack: grad_out [HW] ->
 * grad_cv [HW][2], grad_sigma [3][levels] (z, n, l) */
void orc_svgf_spatial_vjp(const orc_svgf_params*, int W, int H, const double* cv_in,
                          const float* nz, const float* dz, const double* grad_out,
                          double* grad_cv, double* grad_sigma);
/* Jacobian-vector product by forward-mode dual numbers (independent of the
 * VJP): tangents dcv [HW][2] and dsigma [3][levels] -> dout [HW] */
void orc_svgf_spatial_jvp(const orc_svgf_params*, int W, int H, const double* cv_in,
                          const float* nz, const float* dz, const double* dcv,
                          const double* dsigma, double* dout);

/* ---- wire form of a served frame ---- */
/* q = floor(255 * clamp(x, 0, 1) + 1/2) in fp32; NaN and negatives give 0 */
void orc_quantize_u8(const float* x, uint8_t* q, int64_t n);
/* bit l of mask[i] = 2 * shadow_count[l][i] >= n_shadow (light l visible) */
void orc_light_mask(const uint8_t* shadow_count, int n_lights, int n_shadow, int64_t hw, uint8_t* mask);

int orc_num_threads(void);
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
