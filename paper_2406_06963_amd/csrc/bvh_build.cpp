// Host BVH builder: binned surface-area heuristic (Wald, "On fast
// construction of SAH-based bounding volume hierarchies", 2007), with the
// tree depth capped so that device traversal stacks have a fixed size, then
// flattened into the device layout (child boxes stored in the parent, leaves
// as triangle ranges).  The paper relies on the driver's hierarchy
// (Section 3.2); this is the library's own.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <future>
#include <limits>
#include <memory>
#include <thread>
#include <vector>

#include "internal.h"

namespace dhr {
namespace {

constexpr float kInf = std::numeric_limits<float>::infinity();

struct Box {
    float lo[3] = {kInf, kInf, kInf};
    float hi[3] = {-kInf, -kInf, -kInf};
    void grow(const Box& b) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], b.lo[k]);
            hi[k] = std::max(hi[k], b.hi[k]);
        }
    }
    void grow(const float* p) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], p[k]);
            hi[k] = std::max(hi[k], p[k]);
        }
    }
    double area() const {
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = std::max(0.0, (double)hi[k] - (double)lo[k]);
        return 2.0 * (d[0] * d[1] + d[1] * d[2] + d[2] * d[0]);
    }
};

struct Prim {
    Box b;
    float c[3];
    uint32_t idx;
};

struct BNode {
    Box box;
    std::unique_ptr<BNode> kid[2];
    uint32_t first = 0, count = 0;  // leaf when count > 0
};

uint32_t ceil_log2(uint64_t v) {
    uint32_t r = 0;
    while ((1ull << r) < v) ++r;
    return r;
}

class Builder {
   public:
    Builder(std::vector<Prim>& prims, const dhr_bvh_opts& o) : prims_(prims), o_(o) {
        threads_left_ = (int)(o.threads ? o.threads : std::max(1u, std::thread::hardware_concurrency())) - 1;
    }

    std::unique_ptr<BNode> build(uint32_t b, uint32_t e, uint32_t depth) {
        auto node = std::make_unique<BNode>();
        Box cb;
        for (uint32_t i = b; i < e; ++i) {
            node->box.grow(prims_[i].b);
            cb.grow(prims_[i].c);
        }
        const uint32_t n = e - b;
        if (n <= o_.max_leaf) {
            node->first = b;
            node->count = n;
            return node;
        }
        const uint32_t need = ceil_log2((n + o_.max_leaf - 1) / o_.max_leaf);
        uint32_t mid = 0;
        if (depth + need < o_.max_depth) mid = sah_split(b, e, cb);
        if (mid <= b || mid >= e) mid = median_split(b, e, cb);
        if (n > 32768 && threads_left_.fetch_sub(1) > 0) {
            auto fut = std::async(std::launch::async, [&, b, mid, depth] { return build(b, mid, depth + 1); });
            node->kid[1] = build(mid, e, depth + 1);
            node->kid[0] = fut.get();
            threads_left_.fetch_add(1);
        } else {
            node->kid[0] = build(b, mid, depth + 1);
            node->kid[1] = build(mid, e, depth + 1);
        }
        return node;
    }

   private:
    // Object median on the widest centroid axis (ties broken by index).
    uint32_t median_split(uint32_t b, uint32_t e, const Box& cb) {
        int axis = 0;
        float best = -1.0f;
        for (int k = 0; k < 3; ++k)
            if (cb.hi[k] - cb.lo[k] > best) best = cb.hi[k] - cb.lo[k], axis = k;
        uint32_t mid = b + (e - b) / 2;
        std::nth_element(prims_.begin() + b, prims_.begin() + mid, prims_.begin() + e,
                         [axis](const Prim& x, const Prim& y) {
                             return x.c[axis] < y.c[axis] || (x.c[axis] == y.c[axis] && x.idx < y.idx);
                         });
        return mid;
    }

    // Binned SAH: cost(split) = A_L N_L + A_R N_R over bin boundaries.
    uint32_t sah_split(uint32_t b, uint32_t e, const Box& cb) {
        const uint32_t K = o_.sah_bins;
        double best_cost = std::numeric_limits<double>::infinity();
        int best_axis = -1;
        uint32_t best_bin = 0;
        std::vector<Box> bins(K);
        std::vector<uint32_t> cnt(K);
        std::vector<double> rarea(K);
        std::vector<uint32_t> rcnt(K);
        for (int axis = 0; axis < 3; ++axis) {
            const float lo = cb.lo[axis], ext = cb.hi[axis] - cb.lo[axis];
            if (!(ext > 0.0f)) continue;
            const float scale = (float)K / ext;
            std::fill(bins.begin(), bins.end(), Box());
            std::fill(cnt.begin(), cnt.end(), 0u);
            for (uint32_t i = b; i < e; ++i) {
                uint32_t k = std::min(K - 1, (uint32_t)((prims_[i].c[axis] - lo) * scale));
                bins[k].grow(prims_[i].b);
                ++cnt[k];
            }
            Box acc;
            uint32_t c = 0;
            for (int k = (int)K - 1; k > 0; --k) {
                acc.grow(bins[k]);
                c += cnt[k];
                rarea[k] = acc.area();
                rcnt[k] = c;
            }
            acc = Box();
            c = 0;
            for (uint32_t k = 0; k + 1 < K; ++k) {
                acc.grow(bins[k]);
                c += cnt[k];
                if (c == 0 || rcnt[k + 1] == 0) continue;
                double cost = acc.area() * c + rarea[k + 1] * rcnt[k + 1];
                if (cost < best_cost) best_cost = cost, best_axis = axis, best_bin = k;
            }
        }
        if (best_axis < 0) return b;  // every centroid coincides: caller takes the median
        const float lo = cb.lo[best_axis], scale = (float)K / (cb.hi[best_axis] - cb.lo[best_axis]);
        auto it = std::partition(prims_.begin() + b, prims_.begin() + e, [&](const Prim& p) {
            return std::min(K - 1, (uint32_t)((p.c[best_axis] - lo) * scale)) <= best_bin;
        });
        return (uint32_t)(it - prims_.begin());
    }

    std::vector<Prim>& prims_;
    const dhr_bvh_opts& o_;
    std::atomic<int> threads_left_{0};
};

struct Flattener {
    std::vector<float4> out;  // 4 per node
    float pad = 0.0f;
    uint32_t depth = 0, max_leaf = 0;
    double sah = 0.0, root_area = 1.0;

    static int leaf_ref(uint32_t first, uint32_t count) {
        return ~(int)((first << kLeafCountBits) | (count - 1));
    }

    int ref_of(const BNode* n, uint32_t d) {
        if (n->count > 0) {
            depth = std::max(depth, d);
            max_leaf = std::max(max_leaf, n->count);
            sah += n->box.area() / root_area * n->count;
            return leaf_ref(n->first, n->count);
        }
        return emit(n, d);
    }

    // Writes an internal node; returns its index.
    int emit(const BNode* n, uint32_t d) {
        const int id = (int)(out.size() / 4);
        out.resize(out.size() + 4);
        sah += n->box.area() / root_area;  // traversal step
        const Box* kb[2];
        Box empty;
        empty.lo[0] = empty.lo[1] = empty.lo[2] = 1e30f;
        empty.hi[0] = empty.hi[1] = empty.hi[2] = -1e30f;
        int ref[2];
        for (int k = 0; k < 2; ++k) {
            if (n->kid[k]) {
                kb[k] = &n->kid[k]->box;
                ref[k] = ref_of(n->kid[k].get(), d + 1);
            } else {
                kb[k] = &empty;
                ref[k] = -1;
            }
        }
        float lo[2][3], hi[2][3];
        for (int k = 0; k < 2; ++k)
            for (int a = 0; a < 3; ++a) {
                bool real = n->kid[k] != nullptr;
                lo[k][a] = real ? kb[k]->lo[a] - pad : kb[k]->lo[a];
                hi[k][a] = real ? kb[k]->hi[a] + pad : kb[k]->hi[a];
            }
        float4* o = &out[4 * id];
        o[0] = make_float4(lo[0][0], hi[0][0], lo[0][1], hi[0][1]);
        o[1] = make_float4(lo[1][0], hi[1][0], lo[1][1], hi[1][1]);
        o[2] = make_float4(lo[0][2], hi[0][2], lo[1][2], hi[1][2]);
        int4 r = make_int4(ref[0], ref[1], 0, 0);
        std::memcpy(&o[3], &r, 16);
        return id;
    }
};

}  // namespace

bool build_host_bvh(const float* tris, const uint32_t* obj_id, uint32_t T, const dhr_bvh_opts& o, HostBvh* out) {
    std::vector<Prim> prims(T);
    float maxabs = 0.0f;
    for (uint32_t i = 0; i < T; ++i) {
        Prim& p = prims[i];
        const float* v = tris + 9ull * i;
        for (int k = 0; k < 9; ++k) {
            if (!std::isfinite(v[k])) {
                out->error = "non-finite vertex coordinate in triangle " + std::to_string(i);
                return false;
            }
            maxabs = std::max(maxabs, std::fabs(v[k]));
        }
        p.b.grow(v);
        p.b.grow(v + 3);
        p.b.grow(v + 6);
        for (int k = 0; k < 3; ++k) p.c[k] = 0.5f * (p.b.lo[k] + p.b.hi[k]);
        p.idx = i;
    }
    Builder builder(prims, o);
    std::unique_ptr<BNode> root = builder.build(0, T, 0);

    Flattener fl;
    // Boxes grow outward by 2^-20 of the scene's largest coordinate so that
    // rounding in the fp32 slab test can never reject a box that holds a hit.
    fl.pad = std::ldexp(std::max(maxabs, 1e-6f), -20);
    fl.root_area = std::max(root->box.area(), 1e-30);
    if (root->count > 0) {
        // a single leaf: wrap it in an internal root whose second child is empty
        auto wrap = std::make_unique<BNode>();
        wrap->box = root->box;
        wrap->kid[0] = std::move(root);
        root = std::move(wrap);
    }
    fl.emit(root.get(), 0);

    out->n_nodes = fl.out.size() / 4;
    out->depth = fl.depth;
    out->max_leaf_size = fl.max_leaf;
    out->sah_cost = fl.sah;
    out->nodes = (float4*)std::malloc(fl.out.size() * sizeof(float4));
    out->tris = (float4*)std::malloc(3ull * T * sizeof(float4));
    if (!out->nodes || !out->tris) {
        std::free(out->nodes);
        std::free(out->tris);
        out->nodes = out->tris = nullptr;
        out->error = "host allocation failed";
        return false;
    }
    std::memcpy(out->nodes, fl.out.data(), fl.out.size() * sizeof(float4));
    for (uint32_t i = 0; i < T; ++i) {
        const uint32_t src = prims[i].idx;
        const float* v = tris + 9ull * src;
        uint32_t oid = obj_id ? obj_id[src] : src;
        float fidx, foid;
        std::memcpy(&fidx, &src, 4);
        std::memcpy(&foid, &oid, 4);
        out->tris[3ull * i + 0] = make_float4(v[0], v[1], v[2], fidx);
        out->tris[3ull * i + 1] = make_float4(v[3] - v[0], v[4] - v[1], v[5] - v[2], foid);
        out->tris[3ull * i + 2] = make_float4(v[6] - v[0], v[7] - v[1], v[8] - v[2], 0.0f);
    }
    return true;
}

}  // namespace dhr

extern "C" {

dhr_status dhr_build_bvh(dhr_ctx* ctx, const float* tris, const uint32_t* obj_id, uint32_t T,
                         const dhr_bvh_opts* opts, dhr_bvh** out) {
    if (!ctx) return DHR_ERR_INVALID_ARG;
    if (!tris || !out) return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_build_bvh: null pointer");
    *out = nullptr;
    if (T == 0 || T > (1u << 28))
        return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_build_bvh: T = %u outside 1..2^28", T);
    dhr_bvh_opts o{4, 32, 16, 0};
    if (opts) o = *opts;
    if (o.max_leaf == 0) o.max_leaf = 4;
    if (o.max_depth == 0) o.max_depth = 32;
    if (o.sah_bins == 0) o.sah_bins = 64;
    if (o.max_leaf > 8 || o.max_depth < 8 || o.max_depth > 32 || o.sah_bins < 4 || o.sah_bins > 64)
        return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_build_bvh: options out of range");
    if ((uint64_t)(T + o.max_leaf - 1) / o.max_leaf > (1ull << o.max_depth))
        return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_build_bvh: max_depth too small for T");
    if (obj_id)
        for (uint32_t i = 0; i < T; ++i)
            if (obj_id[i] == DHR_MISS_ID)
                return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_build_bvh: object id 0xFFFFFFFF is reserved");

    auto t0 = std::chrono::steady_clock::now();
    dhr::HostBvh hb;
    if (!dhr::build_host_bvh(tris, obj_id, T, o, &hb))
        return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_build_bvh: %s", hb.error.c_str());

    dhr::DeviceGuard g(ctx->device);
    dhr_bvh* b = new dhr_bvh;
    b->ctx = ctx;
    b->device = ctx->device;
    const size_t nb = hb.n_nodes * 4 * sizeof(float4), tb = 3ull * T * sizeof(float4), rb = 4ull * T;
    if (hipMalloc(&b->nodes, nb) != hipSuccess || hipMalloc(&b->tris, tb) != hipSuccess ||
        hipMalloc(&b->rec_of, rb) != hipSuccess) {
        if (b->nodes) (void)hipFree(b->nodes);
        if (b->tris) (void)hipFree(b->tris);
        delete b;
        std::free(hb.nodes);
        std::free(hb.tris);
        (void)hipGetLastError();
        return dhr::set_error(ctx, DHR_ERR_OOM, "dhr_build_bvh: device allocation of %zu bytes failed", nb + tb + rb);
    }
    // inverse of the leaf order (the input index sits in v0.w of each record)
    std::vector<uint32_t> rec_of(T);
    for (uint32_t k = 0; k < T; ++k) {
        uint32_t orig;
        std::memcpy(&orig, &hb.tris[3ull * k].w, 4);
        rec_of[orig] = k;
    }
    hipError_t e1 = hipMemcpy(b->nodes, hb.nodes, nb, hipMemcpyHostToDevice);
    hipError_t e2 = hipMemcpy(b->tris, hb.tris, tb, hipMemcpyHostToDevice);
    if (e2 == hipSuccess) e2 = hipMemcpy(b->rec_of, rec_of.data(), rb, hipMemcpyHostToDevice);
    std::free(hb.nodes);
    std::free(hb.tris);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        (void)hipFree(b->nodes);
        (void)hipFree(b->tris);
        (void)hipFree(b->rec_of);
        delete b;
        return dhr::set_error(ctx, DHR_ERR_DEVICE, "dhr_build_bvh: upload failed: %s",
                              hipGetErrorString(e1 != hipSuccess ? e1 : e2));
    }
    b->info.n_nodes = hb.n_nodes;
    b->info.n_tris = T;
    b->info.device_bytes = nb + tb + rb;
    b->info.depth = hb.depth;
    b->info.max_leaf_size = hb.max_leaf_size;
    b->info.sah_cost = hb.sah_cost;
    b->info.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = b;
    return DHR_OK;
}

dhr_status dhr_build_bvh_instanced(dhr_ctx* ctx, const float* base_tris, const uint32_t* base_obj, uint32_t n_base,
                                   const float* mesh_tris, uint32_t n_mesh, const float* xforms,
                                   const uint32_t* inst_obj, uint32_t n_inst, const dhr_bvh_opts* opts, dhr_bvh** out) {
    using namespace dhr;
    if (!ctx) return DHR_ERR_INVALID_ARG;
    const char* what = "dhr_build_bvh_instanced";
    if (!base_tris || !mesh_tris || !xforms || !out) return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: null pointer", what);
    *out = nullptr;
    if (n_base == 0 || n_mesh == 0 || n_inst == 0 || n_base > (1u << 28) || n_mesh > (1u << 20) ||
        n_inst > (1u << 24) || (uint64_t)n_base + (uint64_t)n_inst * n_mesh > 0x7FFFFFFFull)
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: counts outside the supported range", what);
    dhr_bvh_opts o{4, 32, 16, 0};
    if (opts) o = *opts;
    if (o.max_leaf == 0) o.max_leaf = 4;
    if (o.max_depth == 0) o.max_depth = 32;
    if (o.sah_bins == 0) o.sah_bins = 64;
    if (o.max_leaf > 8 || o.max_depth < 8 || o.max_depth > 32 || o.sah_bins < 4 || o.sah_bins > 64)
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: options out of range", what);
    for (uint32_t n : {n_base, n_inst + 1})
        if ((uint64_t)(n + o.max_leaf - 1) / o.max_leaf > (1ull << o.max_depth))
            return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: max_depth too small", what);
    if (base_obj)
        for (uint32_t i = 0; i < n_base; ++i)
            if (base_obj[i] == DHR_MISS_ID)
                return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: object id 0xFFFFFFFF is reserved", what);
    if (inst_obj)
        for (uint32_t k = 0; k < n_inst; ++k)
            if (inst_obj[k] == DHR_MISS_ID)
                return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: object id 0xFFFFFFFF is reserved", what);
    const auto t0 = std::chrono::steady_clock::now();
    // instance transforms: object-to-world M = [A | t], world-to-object [A^-1 | -A^-1 t] (double)
    std::vector<double> inv(12ull * n_inst);
    for (uint32_t k = 0; k < n_inst; ++k) {
        const float* m = xforms + 12ull * k;
        for (int q = 0; q < 12; ++q)
            if (!std::isfinite(m[q])) return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: transform %u not finite", what, k);
        const double a = m[0], b = m[1], c = m[2], d = m[4], e = m[5], f = m[6], g = m[8], h = m[9], i = m[10];
        const double det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
        const double scale = std::max({std::fabs(a), std::fabs(b), std::fabs(c), std::fabs(d), std::fabs(e),
                                       std::fabs(f), std::fabs(g), std::fabs(h), std::fabs(i)});
        if (!(std::fabs(det) > 1e-12 * scale * scale * scale))
            return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: transform %u is singular", what, k);
        const double r[9] = {(e * i - f * h) / det, (c * h - b * i) / det, (b * f - c * e) / det,
                             (f * g - d * i) / det, (a * i - c * g) / det, (c * d - a * f) / det,
                             (d * h - e * g) / det, (b * g - a * h) / det, (a * e - b * d) / det};
        double* w = inv.data() + 12ull * k;
        for (int row = 0; row < 3; ++row) {
            for (int col = 0; col < 3; ++col) w[4 * row + col] = r[3 * row + col];
            w[4 * row + 3] = -(r[3 * row] * m[3] + r[3 * row + 1] * m[7] + r[3 * row + 2] * m[11]);
        }
    }
    HostBvh hb[3];  // base, mesh, top
    if (!build_host_bvh(base_tris, base_obj, n_base, o, &hb[0]))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: base geometry: %s", what, hb[0].error.c_str());
    auto free_host = [&] {
        for (HostBvh& h : hb) {
            std::free(h.nodes);
            std::free(h.tris);
            h.nodes = h.tris = nullptr;
        }
    };
    if (!build_host_bvh(mesh_tris, nullptr, n_mesh, o, &hb[1])) {
        free_host();
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: mesh: %s", what, hb[1].error.c_str());
    }
    // world boxes of the items (0: base geometry, 1 + k: instance k) as
    // degenerate triangles (lo, hi, lo) spanning them, rounded outward
    const uint32_t n_items = n_inst + 1;
    std::vector<float> boxes(9ull * n_items);
    auto put_box = [&](uint32_t item, const double* lo, const double* hi) {
        float* bx = boxes.data() + 9ull * item;
        for (int q = 0; q < 3; ++q) {
            float l = (float)lo[q], h = (float)hi[q];
            if ((double)l > lo[q]) l = std::nextafter(l, -INFINITY);
            if ((double)h < hi[q]) h = std::nextafter(h, INFINITY);
            bx[q] = l;
            bx[3 + q] = h;
            bx[6 + q] = l;
        }
    };
    {
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (uint64_t v = 0; v < 3ull * n_base; ++v)
            for (int q = 0; q < 3; ++q) {
                lo[q] = std::min(lo[q], (double)base_tris[3 * v + q]);
                hi[q] = std::max(hi[q], (double)base_tris[3 * v + q]);
            }
        put_box(0, lo, hi);
    }
    for (uint32_t k = 0; k < n_inst; ++k) {
        const float* m = xforms + 12ull * k;
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (uint64_t v = 0; v < 3ull * n_mesh; ++v) {
            const float* p = mesh_tris + 3 * v;
            for (int q = 0; q < 3; ++q) {
                const double w = (double)m[4 * q] * p[0] + (double)m[4 * q + 1] * p[1] + (double)m[4 * q + 2] * p[2] +
                                 (double)m[4 * q + 3];
                lo[q] = std::min(lo[q], w);
                hi[q] = std::max(hi[q], w);
            }
        }
        put_box(1 + k, lo, hi);
    }
    if (!build_host_bvh(boxes.data(), nullptr, n_items, o, &hb[2])) {
        free_host();
        return set_error(ctx, DHR_ERR_INVALID_ARG, "%s: top level: %s", what, hb[2].error.c_str());
    }
    // instance records in the top level's leaf order
    std::vector<float4> rec(8ull * n_items);
    for (uint32_t pos = 0; pos < n_items; ++pos) {
        uint32_t item;
        std::memcpy(&item, &hb[2].tris[3ull * pos].w, 4);
        float4* R = rec.data() + 8ull * pos;
        double wi[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0}, fw[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
        uint32_t info[4] = {0u, DHR_MISS_ID, 0u, 0u};
        if (item > 0) {
            const uint32_t k = item - 1;
            for (int q = 0; q < 12; ++q) {
                wi[q] = inv[12ull * k + q];
                fw[q] = xforms[12ull * k + q];
            }
            info[0] = 1u;
            info[1] = inst_obj ? inst_obj[k] : k;
            info[2] = n_base + k * n_mesh;
        }
        for (int row = 0; row < 3; ++row) {
            R[row] = make_float4((float)wi[4 * row], (float)wi[4 * row + 1], (float)wi[4 * row + 2], (float)wi[4 * row + 3]);
            R[3 + row] = make_float4((float)fw[4 * row], (float)fw[4 * row + 1], (float)fw[4 * row + 2],
                                     (float)fw[4 * row + 3]);
        }
        float fi[4];
        std::memcpy(fi, info, 16);
        R[6] = make_float4(fi[0], fi[1], fi[2], fi[3]);
        R[7] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    // device: nodes [top | base | mesh], triangles [base | mesh], instances, description
    DeviceGuard g(ctx->device);
    const uint64_t nn[3] = {hb[2].n_nodes, hb[0].n_nodes, hb[1].n_nodes};
    const uint64_t node_bytes = 64ull * (nn[0] + nn[1] + nn[2]), tri_bytes = 48ull * (n_base + n_mesh),
                   inst_bytes = 128ull * n_items;
    dhr_bvh* b = new dhr_bvh;
    b->ctx = ctx;
    b->device = ctx->device;
    bool ok = hipMalloc(&b->nodes, node_bytes) == hipSuccess && hipMalloc(&b->tris, tri_bytes) == hipSuccess &&
              hipMalloc(&b->inst, inst_bytes) == hipSuccess && hipMalloc(&b->tl, sizeof(TwoLevelHost)) == hipSuccess;
    if (ok) {
        TwoLevelHost tl;
        tl.inst = b->inst;
        tl.nodes[0] = b->nodes + 4 * nn[0];
        tl.nodes[1] = b->nodes + 4 * (nn[0] + nn[1]);
        tl.tris[0] = b->tris;
        tl.tris[1] = b->tris + 3ull * n_base;
        ok = hipMemcpy(b->nodes, hb[2].nodes, 64ull * nn[0], hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(b->nodes + 4 * nn[0], hb[0].nodes, 64ull * nn[1], hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(b->nodes + 4 * (nn[0] + nn[1]), hb[1].nodes, 64ull * nn[2], hipMemcpyHostToDevice) ==
                 hipSuccess &&
             hipMemcpy(b->tris, hb[0].tris, 48ull * n_base, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(b->tris + 3ull * n_base, hb[1].tris, 48ull * n_mesh, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(b->inst, rec.data(), inst_bytes, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(b->tl, &tl, sizeof tl, hipMemcpyHostToDevice) == hipSuccess;
    }
    const uint32_t depth = hb[2].depth + std::max(hb[0].depth, hb[1].depth);
    const uint32_t max_leaf = std::max({hb[0].max_leaf_size, hb[1].max_leaf_size, hb[2].max_leaf_size});
    free_host();
    if (!ok) {
        (void)hipGetLastError();
        dhr_bvh_destroy(b);
        return set_error(ctx, DHR_ERR_OOM, "%s: device allocation or upload failed", what);
    }
    b->info.n_nodes = nn[0] + nn[1] + nn[2];
    b->info.n_tris = n_base + n_mesh;
    b->info.device_bytes = node_bytes + tri_bytes + inst_bytes;
    b->info.depth = depth;
    b->info.max_leaf_size = max_leaf;
    b->info.sah_cost = 0.0;
    b->info.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = b;
    return DHR_OK;
}

dhr_status dhr_bvh_export(dhr_ctx* ctx, const dhr_bvh* bvh, float* nodes, float* tris, dhr_stream stream) {
    if (!ctx) return DHR_ERR_INVALID_ARG;
    if (!bvh || !nodes || !tris) return dhr::set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_bvh_export: null pointer");
    if (bvh->tl) return dhr::set_error(ctx, DHR_ERR_UNSUPPORTED, "dhr_bvh_export: a two-level hierarchy");
    dhr::DeviceGuard g(bvh->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(nodes, bvh->nodes, bvh->info.n_nodes * 64, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(tris, bvh->tris, bvh->info.n_tris * 48, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return dhr::set_error(ctx, DHR_ERR_DEVICE, "dhr_bvh_export: copy failed");
    return DHR_OK;
}

dhr_status dhr_bvh_get_info(const dhr_bvh* bvh, dhr_bvh_info* info) {
    if (!bvh || !info) return DHR_ERR_INVALID_ARG;
    *info = bvh->info;
    return DHR_OK;
}

void dhr_bvh_destroy(dhr_bvh* bvh) {
    if (!bvh) return;
    dhr::DeviceGuard g(bvh->device);
    for (void* p : {(void*)bvh->nodes, (void*)bvh->tris, (void*)bvh->rec_of, (void*)bvh->child, (void*)bvh->range,
                    (void*)bvh->parent,
                    (void*)bvh->box, (void*)bvh->by_depth, (void*)bvh->bounds, bvh->tl, (void*)bvh->inst})
        if (p) (void)hipFree(p);
    delete bvh;
}

}  // extern "C"
