/*
 * dhr.h — C ABI of the DHR+S server hot path on MI355X (gfx950).
 *
 * Method: Tan, Low, Chow, Teo, Bhojan, "DHR+S: distributed hybrid rendering
 * with realistic real-time shadows for interactive thin client metaverse and
 * game applications" (arxiv 2406.06963).  The server traces, per pixel,
 * ambient-occlusion rays (Section 3.2, eqs. (1)-(3)) and soft-shadow rays
 * (Section 3.1) through a bounding-volume hierarchy (Section 3.2), and
 * reconstructs the noisy AO with a modified spatiotemporal variance-guided
 * filter (Section 3.3).
 *
 * Conventions shared by every call
 * --------------------------------
 * Pixel index i = y*W + x, row 0 at the top, pixel centres at (x+0.5, y+0.5).
 * Per-pixel device buffers (caller-owned, 16-byte aligned):
 *   pos   float[HW][4]  world position xyz; w holds the object id's bits
 *                       (DHR_MISS_ID where the primary ray missed)
 *   nz    float[HW][4]  unit geometric normal facing the viewer; w = view-space
 *                       depth z.  A pixel is VALID iff nz.w > 0.
 *   dz    float[HW][2]  depth of the hit triangle's plane seen through pixel
 *                       (x+1, y) and (x, y+1), minus z (1e20 when that plane is
 *                       not in front of the camera there)
 *   mv    float[HW][2]  motion into the history camera in pixels: the pixel's
 *                       world position lands at (x + 0.5 + mv.x, y + 0.5 + mv.y)
 *   hist  float[HW][4]  SVGF history (c, mu1, mu2, history length)
 * Every call is asynchronous on the given stream (a hipStream_t; NULL = the
 * legacy null stream) unless stated otherwise.  No call keeps a caller pointer
 * beyond the work it enqueues.  Calls never throw; on DHR_ERR_INVALID_ARG
 * nothing is launched and dhr_last_error() says why.  Asynchronous device
 * faults surface at the next call or at dhr_sync() as DHR_ERR_DEVICE.  A
 * context is not thread-safe; distinct contexts are independent.  The library
 * keeps no per-call scratch: every buffer a call needs is passed in, so calls
 * on different streams of one context may overlap.
 */
#ifndef DHR_H
#define DHR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dhr_status {
    DHR_OK = 0,
    DHR_ERR_INVALID_ARG = 1,
    DHR_ERR_OOM = 2,
    DHR_ERR_DEVICE = 3,
    DHR_ERR_UNSUPPORTED = 4
} dhr_status;

typedef struct dhr_ctx dhr_ctx;
typedef struct dhr_bvh dhr_bvh;
typedef void* dhr_stream; /* hipStream_t */

#define DHR_MAX_LIGHTS 8
#define DHR_MAX_LEVELS 8
#define DHR_MAX_SIDE 16384
#define DHR_MISS_ID 0xFFFFFFFFu

/* ------------------------------------------------------------------------
 * Context
 * ------------------------------------------------------------------------ */

/* Creates a context bound to HIP device `device`.  *out receives the handle
 * (library-owned; free with dhr_destroy).  DHR_ERR_DEVICE if the device is
 * absent, DHR_ERR_UNSUPPORTED if it is not gfx950.
 * Traversal addresses a single-level tree's records by 32-bit byte offsets
 * when its node and triangle counts are both at most 2^26, by 64-bit offsets
 * otherwise; the environment variable DHR_WIDE_RECORDS=1, read here, makes
 * this context use 64-bit offsets for every tree (same results, for
 * testing that path on small scenes). */
dhr_status dhr_create(int device, dhr_ctx** out);
void dhr_destroy(dhr_ctx* ctx);
/* Message of the last failing call on this context ("" if none).  The string
 * is owned by the context and valid until its next call. */
const char* dhr_last_error(const dhr_ctx* ctx);
/* Waits for the stream; reports an earlier asynchronous fault as
 * DHR_ERR_DEVICE. */
dhr_status dhr_sync(dhr_ctx* ctx, dhr_stream stream);
const char* dhr_version(void);

/* ------------------------------------------------------------------------
 * Bounding-volume hierarchy (Section 3.2: objects are grouped hierarchically
 * in bounding volumes so that a ray missing a volume skips its content; short
 * rays descend less deep).
 * ------------------------------------------------------------------------ */

typedef struct {
    uint32_t max_leaf;   /* triangles per leaf, 1..8 (default 4)               */
    uint32_t max_depth;  /* 8..32 (default 32); subtrees switch to median splits
                            so the limit holds (the traversal stack holds 64) */
    uint32_t sah_bins;   /* binned-SAH bins, 4..64 (default 64)                */
    uint32_t threads;    /* host build threads, 0 = hardware concurrency       */
} dhr_bvh_opts;

typedef struct {
    uint64_t n_nodes, n_tris, device_bytes;
    uint32_t depth, max_leaf_size;
    double sah_cost, build_ms;
} dhr_bvh_info;

/* Builds a binned-SAH BVH over T world-space triangles and uploads it to the
 * context's device.  SYNCHRONOUS.
 *   tris    host float[T][3][3] (vertex, xyz), not retained
 *   obj_id  host uint32[T] or NULL (then the triangle index is the id); the id
 *           DHR_MISS_ID is reserved
 *   opts    NULL = defaults
 *   out     receives the library-owned handle; free with dhr_bvh_destroy
 * Errors: INVALID_ARG (T == 0, T > 2^28, non-finite vertex, bad opts),
 * OOM (device allocation failed). */
dhr_status dhr_build_bvh(dhr_ctx* ctx, const float* tris, const uint32_t* obj_id, uint32_t T,
                         const dhr_bvh_opts* opts, dhr_bvh** out);
/* Builds the BVH on the device from device-resident triangles: a linear BVH
 * over the Morton codes of the triangle centroids (Karras, HPG 2012) whose
 * subtrees of at most four triangles become leaves, in the node layout
 * dhr_build_bvh produces (info.depth counts the levels before that
 * collapse, an upper bound), so every call
 * taking a dhr_bvh accepts it and every query gives the same result as with
 * any other valid hierarchy over the same triangles.  Its tree is of lower
 * quality than the SAH build (traversal is slower) but it builds in
 * milliseconds with the scene already in HBM, and it can be refitted.
 *   tris    device float[T][3][3] (finite, 4-byte aligned; not retained)
 *   obj_id  device uint32[T] or NULL (then the triangle index is the id)
 *   out     receives the handle; free with dhr_bvh_destroy
 * The kernels run on `stream`; the call waits for them (it reads back where
 * each depth level starts) before returning.  Errors: INVALID_ARG (T == 0 or > 2^28, null or
 * misaligned pointer), OOM, DEVICE, UNSUPPORTED (a path longer than the
 * traversal stack; cannot happen for 30-bit codes, checked anyway). */
dhr_status dhr_build_bvh_device(dhr_ctx* ctx, const float* tris, const uint32_t* obj_id, uint32_t T, dhr_bvh** out,
                                dhr_stream stream);

/* Two-level hierarchy for instanced geometry (the large terrain workload
 * places thousands of copies of one box): a top level over the instances'
 * world boxes, bottom level 0 over the base geometry, bottom level 1 over
 * one mesh that every instance places with its own transform.  Rays enter
 * the mesh's hierarchy transformed into its space (direction not
 * renormalised, so t is shared), and every query answers as on the
 * flattened scene: base triangles first (index i), then instance k's copy
 * of mesh triangle j (index n_base + k n_mesh + j) for ties.  Host build,
 * synchronous, like dhr_build_bvh (whose options apply to all three levels).
 *   base_tris  host float[n_base][3][3]; base_obj host uint32[n_base] or NULL
 *   mesh_tris  host float[n_mesh][3][3] in the mesh's own space
 *   xforms     host float[n_inst][12]: row-major 3x4 object-to-world [A | t]
 *              (A invertible)
 *   inst_obj   host uint32[n_inst] object id of each instance, or NULL (then k)
 * Accepted by dhr_gbuffer(_batch) and dhr_trace_visibility(_batch); not by
 * dhr_gbuffer_raster, dhr_refit_bvh, dhr_bvh_export or the work counters
 * (UNSUPPORTED).  Errors: INVALID_ARG (null pointer, a count of 0 or beyond
 * 2^28 base / 2^20 mesh / 2^24 instances, non-finite or singular transform,
 * the reserved object id), OOM. */
dhr_status dhr_build_bvh_instanced(dhr_ctx* ctx, const float* base_tris, const uint32_t* base_obj, uint32_t n_base,
                                   const float* mesh_tris, uint32_t n_mesh, const float* xforms,
                                   const uint32_t* inst_obj, uint32_t n_inst, const dhr_bvh_opts* opts, dhr_bvh** out);

/* Refit of a device-built BVH after its triangles moved: same count, same
 * order, same object ids.  Triangle records and boxes are recomputed from
 * `tris` (device float[T][3][3]) and the topology is kept, so queries stay
 * exact while traversal slows as the motion departs from the built layout.
 * Asynchronous on `stream`; must not overlap work that reads the BVH.
 * Errors: INVALID_ARG (null, misaligned, or a BVH built on the host). */
dhr_status dhr_refit_bvh(dhr_ctx* ctx, dhr_bvh* bvh, const float* tris, dhr_stream stream);

dhr_status dhr_bvh_get_info(const dhr_bvh* bvh, dhr_bvh_info* info);
/* Copies the device records (to inspect, cache or serialise a hierarchy):
 *   nodes  device buffer of info.n_nodes * 64 bytes: per node the x and y
 *          slabs of child 0 (lo.x, hi.x, lo.y, hi.y), the same of child 1,
 *          the z slabs of both (lo0, hi0, lo1, hi1) and the child references
 *          (int: node index >= 0, leaf ~(first << 3 | count - 1)); node 0 is
 *          the root
 *   tris   device buffer of info.n_tris * 48 bytes in leaf order: v0 + input
 *          index (bits), e1 + object id (bits), e2
 * Asynchronous on `stream`.  Errors: INVALID_ARG (null pointer). */
dhr_status dhr_bvh_export(dhr_ctx* ctx, const dhr_bvh* bvh, float* nodes, float* tris, dhr_stream stream);
/* Frees the BVH's device memory (waits for work using it).  Valid before or
 * after the context that built it has been destroyed. */
void dhr_bvh_destroy(dhr_bvh* bvh);

/* ------------------------------------------------------------------------
 * G-buffer by primary rays (Section 2.2: world-space position per pixel;
 * Section 3.3: motion vectors in the G-buffer back-project the pixel into the
 * previous frame).  The paper rasterises this on the client's side; here it
 * is the closest hit of the ray through each pixel centre (ties: lowest
 * triangle index).
 * ------------------------------------------------------------------------ */

/* Pinhole camera: fwd = normalize(target - eye), right = normalize(fwd x +y),
 * up = right x fwd; fov_y is the vertical field of view in radians; the
 * aspect ratio is W/H. */
typedef struct {
    float eye[3];
    float target[3];
    float fov_y;
} dhr_camera;

/* Writes pos, nz, dz, mv (layouts above) for a W x H image.  prev = NULL
 * writes NaN motion.  Missed pixels: pos = (0,0,0,DHR_MISS_ID), nz = dz = mv
 * = 0.  Errors: INVALID_ARG (null/misaligned buffers, W or H outside
 * 1..16384, degenerate camera). */
dhr_status dhr_gbuffer(dhr_ctx* ctx, const dhr_bvh* bvh, const dhr_camera* cur, const dhr_camera* prev,
                       uint32_t W, uint32_t H, float* pos, float* nz, float* dz, float* mv,
                       dhr_stream stream);

/* ------------------------------------------------------------------------
 * Stochastic visibility (Section 3.1 soft shadows, Section 3.2 AO).
 * ------------------------------------------------------------------------ */

/* kind 0: directional light; vec = unit direction towards it, one_minus_cos =
 * 1 - cos(cone half-angle) (computed by the caller, e.g. 2 sin^2(theta/2));
 * the shadow ray is unbounded.  kind 1: sphere light; vec = centre, radius =
 * R; the cone is the sphere's solid angle seen from the ray origin and the
 * ray ends where it enters the sphere (the ray's length is kept, Section 3.1);
 * points within R of the centre see the light. */
typedef struct {
    uint32_t kind;
    float vec[3];
    float one_minus_cos;
    float radius;
} dhr_light;

/* Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key (seed,
 * client_id) and counter (x, y, frame, stream << 16 | sample); stream 0 is AO
 * (sample = ao_sample_offset + s), stream 1 + i is light i (sample = s).
 * u0, u1 = (r0 >> 8) 2^-24, (r1 >> 8) 2^-24.
 * AO ray: cosine-weighted about the normal (Malley), length ao_radius;
 * unoccluded iff nothing is hit at 0 < t < ao_radius (eq. (3)).
 * Shadow ray: uniform in the light's cone (solid angle); a direction with
 * n . w <= 0 is occluded without tracing.
 * Origin o = p + eps n, eps = eps_origin_abs if > 0, else
 * max(1e-3 ao_radius, 2^-17 max|p_k|). */
typedef struct {
    uint32_t W, H, frame, client_id, seed;
    uint32_t n_ao;             /* 0..255: rays per pixel; the count fits a byte (Section 3.2) */
    uint32_t ao_sample_offset; /* ao_sample_offset + n_ao <= 65536 */
    float ao_radius;           /* r > 0 when n_ao > 0 */
    uint32_t n_shadow;         /* 0..255 rays per light per pixel */
    uint32_t n_lights;         /* 0..8 */
    dhr_light lights[DHR_MAX_LIGHTS];
    float eps_origin_abs;
} dhr_trace_params;

/* Traces every pixel of a W x H G-buffer.
 *   pos, nz          device, layouts above (invalid pixels count as fully
 *                    visible: ao = n_ao, shadow = n_shadow)
 *   ao_count         device uint8[HW]: N_unoccluded of eq. (3)
 *   shadow_count     device uint8[n_lights][HW]: unoccluded shadow rays per
 *                    light; with n_shadow = 1 the bits (light i -> bit i) form
 *                    the paper's visibility bitmask (Fig. 1).  May be NULL
 *                    when n_lights == 0.
 *   debug_ray_bits   NULL, or device uint64[1 + n_lights][HW]: bit s set iff
 *                    sample s of that stream is unoccluded (needs n <= 64)
 * Errors: INVALID_ARG (n_ao > 255, n_shadow > 255, n_lights > 8, bad light,
 * ao_radius <= 0 with n_ao > 0, sample range, buffers). */
dhr_status dhr_trace_visibility(dhr_ctx* ctx, const dhr_bvh* bvh, const dhr_trace_params* params,
                                const float* pos, const float* nz, uint8_t* ao_count,
                                uint8_t* shadow_count, uint64_t* debug_ray_bits, dhr_stream stream);

/* Ragged batches for serving: one launch per pass covers every job, each
 * with its own scene, size, camera and buffers (a batch of one is the plain
 * call).  Results are identical to the per-job calls. */
typedef struct {
    const dhr_bvh* bvh;
    dhr_camera cur, prev;
    uint32_t has_prev;
    uint32_t W, H;
    float *pos, *nz, *dz, *mv;
} dhr_gbuffer_job;
dhr_status dhr_gbuffer_batch(dhr_ctx* ctx, const dhr_gbuffer_job* jobs, uint32_t n_jobs, dhr_stream stream);

/* The same G-buffer by rasterisation (Section 2.2: the server rasterises
 * its G-buffer and traces visibility from it).  Each triangle proposes the
 * pixels of its conservative screen box (clipped to the camera's near side,
 * grown by half a pixel; triangles whose plane passes within about 1e-5 of
 * the eye coordinates' scale propose the whole frame), each candidate is
 * decided by the ray-triangle test of the traversal, and a pixel keeps the
 * minimum of (t, input index): the texels equal dhr_gbuffer's on the same
 * triangles bit for bit, with any BVH from either builder (its triangle
 * records are read, not its nodes).
 *   work        device scratch of dhr_gbuffer_raster_workspace_bytes(W, H,
 *               n_tris) bytes, 16-byte aligned (per-pixel keys, the list of
 *               large triangles, their 8x8 tiles); calls that overlap need
 *               disjoint work
 *   work_bytes  its size
 * Asynchronous on `stream`.  Errors: INVALID_ARG (null, misaligned or short
 * buffer, bad size, degenerate camera, foreign BVH). */
uint64_t dhr_gbuffer_raster_workspace_bytes(uint32_t W, uint32_t H, uint32_t n_tris);
dhr_status dhr_gbuffer_raster(dhr_ctx* ctx, const dhr_bvh* bvh, const dhr_camera* cur, const dhr_camera* prev,
                              uint32_t W, uint32_t H, float* pos, float* nz, float* dz, float* mv, void* work,
                              uint64_t work_bytes, dhr_stream stream);

typedef struct {
    const dhr_bvh* bvh;
    dhr_trace_params params;
    const float *pos, *nz;
    uint8_t *ao_count, *shadow_count;
} dhr_trace_job;
dhr_status dhr_trace_visibility_batch(dhr_ctx* ctx, const dhr_trace_job* jobs, uint32_t n_jobs,
                                      dhr_stream stream);

/* G-buffer and visibility of a frame in one launch (Section 2.2: the server
 * renders the G-buffer and traces the frame's visibility rays from it;
 * Sections 3.1 and 3.2 for the rays).  Writes exactly what dhr_gbuffer
 * followed by dhr_trace_visibility (debug_ray_bits NULL) writes, with the
 * same arguments, byte for byte; each 16 x 8 pixel block's visibility rays
 * start as soon as its own texels exist, so the few blocks whose primary
 * rays take long walks (grazing views) overlap other blocks' work instead of
 * leaving the device idle behind them.  params->W, H must equal W, H.
 * While work counters are set (dhr_set_trace_counters) the counts cover the
 * primary rays (one per pixel) and the visibility rays.
 * Errors: as the two calls. */
dhr_status dhr_gbuffer_trace(dhr_ctx* ctx, const dhr_bvh* bvh, const dhr_camera* cur, const dhr_camera* prev,
                             uint32_t W, uint32_t H, const dhr_trace_params* params, float* pos, float* nz, float* dz,
                             float* mv, uint8_t* ao_count, uint8_t* shadow_count, dhr_stream stream);
/* The batched form: job k of each array describes one frame; trace_jobs[k]
 * must name gbuffer_jobs[k]'s bvh, size, pos and nz (INVALID_ARG otherwise).
 * Results are identical to the per-job calls. */
dhr_status dhr_gbuffer_trace_batch(dhr_ctx* ctx, const dhr_gbuffer_job* gbuffer_jobs, const dhr_trace_job* trace_jobs,
                                   uint32_t n_jobs, dhr_stream stream);

/* ------------------------------------------------------------------------
 * Modified SVGF (Section 3.3).
 *
 * Temporal: for a valid pixel with x_s = ao_count / n_ao, the history is read
 * at the 2x2 pixels around (x + mv.x, y + mv.y) with bilinear weights (taps
 * of zero weight ignored).  A tap is used iff it is in the image, was valid
 * with history length > 0, has the same object id (use_obj_id), its normal
 * n_q satisfies n . n_q >= cos_normal_min, and |n . (p_q - p)| <=
 * plane_px * pix * z (these two tests are evaluated in fp32 as
 * fmaf(a.x,b.x, fmaf(a.y,b.y, a.z*b.z)) so the decision is reproducible).
 * With usable taps: c, mu1, mu2 are the renormalised bilinear blend, h' =
 * min(1 + max tap length, history_cap), a = max(alpha, 1/h'), am =
 * max(alpha_moments, 1/h'), c' = c + a (x_s - c), mu1' = mu1 + am (x_s - mu1),
 * mu2' = mu2 + am (x_s^2 - mu2).  Otherwise a reset: h' = 1, c' = mu1' =
 * x_s, mu2' = x_s^2.
 * Variance: h' >= var_min_history: max(0, mu2' - mu1'^2) (one fma); else
 * the weighted variance of the pooled moments of the (2R+1)^2 valid
 * neighbours, R = fallback_radius, weights w_z w_n of level 0.
 * A-trous level l (stride s = 2^l): g = sqrt of the 3x3 (1,2,1)/4 blur of
 * the variance over valid pixels; 5x5 taps q = p + s (a, b), h = B3(a) B3(b)
 * with B3 = (1,4,6,4,1)/16 (kernel_width 3: 3x3 taps, h = K(a) K(b) with
 * K = (1,2,1)/4); w = 1 at the centre, else
 *   w_z = exp(-|z_p - z_q| / (sigma_z |s (a dz.x + b dz.y)| + eps_z_rel z_p))
 *   w_n = max(0, min(1, n_p . n_q))^sigma_n   (0 when the dot is <= 0)
 *   w_l = exp(-|c_p - c_q| / (sigma_l g + eps_l))
 * c' = sum h w c / sum h w, v' = sum h^2 w^2 v / (sum h w)^2 over valid
 * in-image taps.  The output of level feedback_level becomes hist_out.c.
 * Invalid pixels: hist_out = (1,1,1,0), out = 1, never a tap or neighbour.
 * ------------------------------------------------------------------------ */

typedef struct {
    uint32_t levels;          /* 1..8 (5) */
    float alpha;              /* (0.2) */
    float alpha_moments;      /* (0.2) */
    float sigma_z[DHR_MAX_LEVELS]; /* > 0 (1) */
    float sigma_n[DHR_MAX_LEVELS]; /* >= 0 (128) */
    float sigma_l[DHR_MAX_LEVELS]; /* > 0 (4) */
    float eps_z_rel;          /* (1e-4) */
    float eps_l;              /* (1e-4) */
    float cos_normal_min;     /* (0.9) */
    float plane_px;           /* (4) */
    uint32_t use_obj_id;      /* (1) */
    uint32_t var_min_history; /* (4) */
    uint32_t fallback_radius; /* 0..3 (3) */
    uint32_t feedback_level;  /* < levels (0) */
    float history_cap;        /* >= 1 (255) */
    uint32_t kernel_width;    /* 5: B3 spline taps (default); 3: (1,2,1)/4 taps,
                                 the lighter variant (one level of a smaller
                                 kernel, Section 3.3's outlook); the adjoint
                                 takes 5 only */
} dhr_svgf_params;

/* Fills the defaults above. */
void dhr_svgf_default_params(dhr_svgf_params* p);

typedef struct {
    uint32_t W, H, n_ao;        /* n_ao >= 1: the denominator of x_s */
    const uint8_t* ao_count;    /* device uint8[HW] */
    const float *pos, *nz, *dz, *mv;
    const float *prev_pos, *prev_nz, *hist_in; /* previous frame; hist_in NULL = no history */
    float* hist_out;            /* device float[HW][4]; must not alias hist_in */
    float* out;                 /* device float[HW]: filtered AO */
    float* save;                /* NULL or device float[levels][HW][2]: the input
                                   (c, var) of every level, for dhr_svgf_backward
                                   (levels >= 1 hold var = -3e38 on invalid pixels) */
    float* work;                /* device scratch of dhr_svgf_workspace_bytes(W,H,p,0)
                                   bytes (16-byte aligned) */
    float pix;                  /* 2 tan(fov_y / 2) / H of the current camera */
} dhr_svgf_frame;

/* Temporal -> variance -> levels for n_frames frames (a ragged batch; one
 * launch per pass).  Errors: INVALID_ARG (bad params, n_ao == 0, buffers,
 * hist_out aliasing hist_in). */
dhr_status dhr_svgf_filter(dhr_ctx* ctx, const dhr_svgf_params* params, const dhr_svgf_frame* frames,
                           uint32_t n_frames, dhr_stream stream);

/* For callers that cannot allocate device memory or pass a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): dhr_svgf_filter with every frame's scratch taken from a
 * library-owned device array of DHR_SVGF_NOALLOC_SCRATCH_BYTES bytes per GPU
 * (allocated when the library is loaded, held until the process ends).  The
 * frames are as for dhr_svgf_filter except that `work` must be NULL; frame k
 * uses dhr_svgf_workspace_bytes(W,H,p,0) bytes rounded up to 256.  The call
 * allocates nothing.  Every call on one GPU shares that GPU's array (nothing
 * in it needs to start at zero; it keeps the last call's contents): calls
 * that overlap on one GPU -- on different streams, or from different
 * contexts -- race and give undefined results.  Errors: as dhr_svgf_filter,
 * plus INVALID_ARG when work is not NULL or the frames need more than
 * DHR_SVGF_NOALLOC_SCRATCH_BYTES (one 1920 x 1080 frame needs 41.5 MB). */
#define DHR_SVGF_NOALLOC_SCRATCH_BYTES (64ull << 20)
dhr_status dhr_svgf_filter_noalloc(dhr_ctx* ctx, const dhr_svgf_params* params, const dhr_svgf_frame* frames,
                                   uint32_t n_frames, dhr_stream stream);

/* Differentiable part alone: the a-trous levels applied to given (c, var). */
typedef struct {
    uint32_t W, H;
    const float* cv_in;         /* device float[HW][2] */
    const float *nz, *dz;
    float* out;                 /* device float[HW] */
    float* save;                /* NULL or device float[levels][HW][2] */
    float* work;                /* device scratch of dhr_svgf_workspace_bytes(W,H,p,0)
                                   bytes (16-byte aligned) */
} dhr_svgf_spatial_frame;
dhr_status dhr_svgf_spatial_forward(dhr_ctx* ctx, const dhr_svgf_params* params,
                                    const dhr_svgf_spatial_frame* frames, uint32_t n_frames,
                                    dhr_stream stream);

/* Vector-Jacobian product of the spatial stack (levels and variance
 * prefilter) for a loss L of the output:
 *   grad_out  device float[HW] = dL/d out
 *   grad_cv   device float[HW][2] receives dL/d (c_in, var_in)
 *   grad_sigma device float[3][levels] receives dL/d (sigma_z, sigma_n,
 *             sigma_l), summed over all frames (overwritten; deterministic)
 * Kinks take the subgradient 0.  No gradient flows into z, normals or the
 * history.  work: dhr_svgf_workspace_bytes(W,H,p,1) bytes per frame.
 * Errors: INVALID_ARG (bad params, sizes or buffers), UNSUPPORTED
 * (kernel_width 3: the adjoint covers the 5x5 kernel only). */
typedef struct {
    uint32_t W, H;
    const float* save;          /* from the forward call with the same params */
    const float *nz, *dz;
    const float* grad_out;
    float* grad_cv;
    float* work;
} dhr_svgf_bwd_frame;
dhr_status dhr_svgf_backward(dhr_ctx* ctx, const dhr_svgf_params* params, const dhr_svgf_bwd_frame* frames,
                             uint32_t n_frames, float* grad_sigma, dhr_stream stream);

/* Scratch bytes one frame needs: which = 0 forward (filter / spatial), 1
 * backward.  Frames of one call need disjoint work buffers; a buffer may be
 * reused by a later call on the same stream. */
uint64_t dhr_svgf_workspace_bytes(uint32_t W, uint32_t H, const dhr_svgf_params* params, int which);

/* Instrumentation for measurement: while `counters` (device uint64[4], or
 * NULL to switch off) is set, dhr_trace_visibility(_batch) and
 * dhr_gbuffer_trace(_batch) on this context run a counting variant of their
 * kernel that adds (rays traced, interior-node visits, leaf visits, triangle
 * tests) into it; single-level hierarchies only (UNSUPPORTED otherwise).
 * Results are unchanged; the counting variant is slower and is never the
 * timed one. */
dhr_status dhr_set_trace_counters(dhr_ctx* ctx, uint64_t* counters);

/* ------------------------------------------------------------------------
 * Wire form of a served frame (Section 3.2: the AO a client receives is one
 * byte per pixel; Section 3.1, Fig. 1: one visibility bit per light).
 *   value  device float[n] (e.g. the filtered AO) or NULL -> q device
 *          uint8[n]: q = floor(255 * clamp(x, 0, 1) + 1/2), evaluated in fp32
 *          without fused multiply-add; NaN gives 0
 *   shadow_count device uint8[n_lights][n] (the trace output) or NULL ->
 *          mask device uint8[n]: bit l set iff 2 * count_l >= n_shadow (light
 *          l reached by at least half of its rays; with one ray per light,
 *          that ray), light 0 = least significant bit
 * Errors: INVALID_ARG (an input without its output, n_lights outside 1..8 or
 * n_shadow == 0 with shadow_count, n > 2^36).
 * ------------------------------------------------------------------------ */
dhr_status dhr_encode_frame(dhr_ctx* ctx, const float* value, uint8_t* q, const uint8_t* shadow_count,
                            uint32_t n_lights, uint32_t n_shadow, uint8_t* mask, uint64_t n, dhr_stream stream);

/* ------------------------------------------------------------------------
 * The random-number generator alone (ray generation uses it in-kernel):
 * n counters (device uint32[n][4]) under key (k0, k1) -> device
 * uint32[n][4].
 * ------------------------------------------------------------------------ */
dhr_status dhr_philox4x32_10(dhr_ctx* ctx, uint32_t k0, uint32_t k1, const uint32_t* ctr, uint32_t* out,
                             uint64_t n, dhr_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* DHR_H */
