// Context, error reporting and parameter helpers of the C ABI.
#include <cstdlib>
#include <cstring>

#include "internal.h"

namespace dhr {

dhr_status set_error(dhr_ctx* ctx, dhr_status st, const char* fmt, ...) {
    if (!ctx) return st;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
    return st;
}

dhr_status check_launch(dhr_ctx* ctx, const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(ctx, DHR_ERR_DEVICE, "%s: launch failed: %s", what, hipGetErrorString(e));
    return DHR_OK;
}

}  // namespace dhr

extern "C" {

const char* dhr_version(void) { return "dhr 0.1 (gfx950)"; }

dhr_status dhr_create(int device, dhr_ctx** out) {
    if (!out) return DHR_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return DHR_ERR_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return DHR_ERR_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return DHR_ERR_UNSUPPORTED;
    dhr_ctx* c = new dhr_ctx;
    c->device = device;
    c->n_cu = prop.multiProcessorCount;
    const char* wide = std::getenv("DHR_WIDE_RECORDS");
    c->wide_records = wide && wide[0] == '1';
    const dhr_status st = dhr::svgf_scratch_init(c);
    if (st != DHR_OK) {
        std::fprintf(stderr, "%s\n", c->err.c_str());
        delete c;
        return st;
    }
    *out = c;
    return DHR_OK;
}

void dhr_destroy(dhr_ctx* ctx) { delete ctx; }

const char* dhr_last_error(const dhr_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

dhr_status dhr_sync(dhr_ctx* ctx, dhr_stream stream) {
    if (!ctx) return DHR_ERR_INVALID_ARG;
    dhr::DeviceGuard g(ctx->device);
    hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return dhr::set_error(ctx, DHR_ERR_DEVICE, "dhr_sync: %s", hipGetErrorString(e));
    return DHR_OK;
}

void dhr_svgf_default_params(dhr_svgf_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->levels = 5;
    p->alpha = 0.2f;
    p->alpha_moments = 0.2f;
    for (int l = 0; l < DHR_MAX_LEVELS; ++l) {
        p->sigma_z[l] = 1.0f;
        p->sigma_n[l] = 128.0f;
        p->sigma_l[l] = 4.0f;
    }
    p->eps_z_rel = 1e-4f;
    p->eps_l = 1e-4f;
    p->cos_normal_min = 0.9f;
    p->plane_px = 4.0f;
    p->use_obj_id = 1;
    p->var_min_history = 4;
    p->fallback_radius = 3;
    p->feedback_level = 0;
    p->history_cap = 255.0f;
    p->kernel_width = 5;
}

}  // extern "C"
