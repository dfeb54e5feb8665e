// Device BVH build and refit: a linear BVH over the Morton codes of the
// triangle centroids (Karras, "Maximizing parallelism in the construction of
// BVHs, octrees, and k-d trees", HPG 2012), built where the scene lives so a
// dynamic scene does not cross PCIe every frame (Section 3.2 relies on the
// driver's hierarchy; this one is the library's own).  Subtrees of at most
// four triangles (consecutive in Morton order) become leaves; the nodes take
// the layout the traversal reads (two child boxes in the parent, padded by
// 2^-20 of the scene's largest coordinate).  A refit keeps
// the topology and recomputes triangles and boxes from new vertices.
//
// Depth: a node's common-prefix length (30 code bits, then 32 index bits for
// equal codes, so at most 63) grows strictly from parent to child, so no path
// holds more than 64 interior nodes and the traversal's 64-entry stack
// always suffices.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstring>
#include <utility>
#include <vector>

#include "device.h"
#include "internal.h"

namespace dhr {
namespace {

constexpr int kB = 256;

// ---- scene bounds: centroid box and the largest absolute coordinate ----
// partial[b] = (lo x, lo y, lo z, hi x, hi y, hi z, max |coord|)
__global__ __launch_bounds__(kB) void bounds_kernel(const float* __restrict__ tris, uint32_t T, float* partial) {
    __shared__ float red[7][kB];
    float v[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0f};
    for (uint32_t t = blockIdx.x * kB + threadIdx.x; t < T; t += gridDim.x * kB) {
        const float* p = tris + 9ull * t;
        for (int a = 0; a < 3; ++a) {
            const float lo = fminf(fminf(p[a], p[3 + a]), p[6 + a]), hi = fmaxf(fmaxf(p[a], p[3 + a]), p[6 + a]);
            const float c = 0.5f * (lo + hi);
            v[a] = fminf(v[a], c);
            v[3 + a] = fmaxf(v[3 + a], c);
            v[6] = fmaxf(v[6], fmaxf(fabsf(lo), fabsf(hi)));
        }
    }
    for (int k = 0; k < 7; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = kB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 7; ++k) {
                const float o = red[k][threadIdx.x + s];
                red[k][threadIdx.x] = (k < 3) ? fminf(red[k][threadIdx.x], o) : fmaxf(red[k][threadIdx.x], o);
            }
        __syncthreads();
    }
    if (threadIdx.x < 7) partial[7 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// One workgroup of kB lanes: lane t folds partials t, t + kB, ... (all
// seven components), then a tree over the lanes in LDS.  Min and max are
// exact, so the result does not depend on the order.
__global__ __launch_bounds__(kB) void bounds_final_kernel(float* partial, uint32_t nb) {
    __shared__ float red[7][kB];
    float v[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0f};
    for (uint32_t b = threadIdx.x; b < nb; b += kB)
        for (int k = 0; k < 7; ++k) {
            const float o = partial[7 * b + k];
            v[k] = (k < 3) ? fminf(v[k], o) : fmaxf(v[k], o);
        }
    for (int k = 0; k < 7; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int h = kB / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 7; ++k) {
                const float o = red[k][threadIdx.x + h];
                red[k][threadIdx.x] = (k < 3) ? fminf(red[k][threadIdx.x], o) : fmaxf(red[k][threadIdx.x], o);
            }
        __syncthreads();
    }
    if (threadIdx.x < 7) partial[threadIdx.x] = red[threadIdx.x][0];  // the result lands in partial[0..6]
}

// ---- Morton codes of the centroids, 10 bits per axis ----
__device__ __forceinline__ uint32_t spread10(uint32_t v) {
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ __launch_bounds__(kB) void morton_kernel(const float* __restrict__ tris, uint32_t T,
                                                    const float* __restrict__ b, uint32_t* key, uint32_t* val) {
    const uint32_t t = blockIdx.x * kB + threadIdx.x;
    if (t >= T) return;
    const float* p = tris + 9ull * t;
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
        const float lo = fminf(fminf(p[a], p[3 + a]), p[6 + a]), hi = fmaxf(fmaxf(p[a], p[3 + a]), p[6 + a]);
        const float c = 0.5f * (lo + hi);
        const float ext = b[3 + a] - b[a];
        const float u = ext > 0.0f ? (c - b[a]) / ext : 0.0f;
        q[a] = (uint32_t)fminf(fmaxf(u * 1024.0f, 0.0f), 1023.0f);
    }
    key[t] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    val[t] = t;
}

// ---- hierarchy over the sorted codes ----
// common-prefix length of sorted entries i and j (-1 outside), index bits
// breaking ties between equal codes
__device__ __forceinline__ int prefix(const uint32_t* __restrict__ key, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    const uint32_t a = key[i], b = key[j];
    if (a != b) return __clz(a ^ b);
    return 32 + __clz((uint32_t)i ^ (uint32_t)j);
}

// child references: internal node c >= 0, leaf k as ~k; parent[T - 1 + k] of
// leaf k; range[i] = the sorted positions [lo, hi] node i covers
__global__ __launch_bounds__(kB) void karras_kernel(const uint32_t* __restrict__ key, int n, int2* child,
                                                    int* parent, int2* range) {
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (prefix(key, n, i, i + 1) - prefix(key, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = prefix(key, n, i, i - d);
    int lmax = 2;
    while (prefix(key, n, i, i + lmax * d) > dmin) lmax *= 2;
    int l = 0;
    for (int t = lmax / 2; t >= 1; t /= 2)
        if (prefix(key, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = prefix(key, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (prefix(key, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int g = i + s * d + min(d, 0);
    const int lo = min(i, j), hi = max(i, j);
    const int c0 = (lo == g) ? ~g : g;
    const int c1 = (hi == g + 1) ? ~(g + 1) : g + 1;
    child[i] = make_int2(c0, c1);
    range[i] = make_int2(lo, hi);
    parent[c0 >= 0 ? c0 : (n - 1) + ~c0] = i;
    parent[c1 >= 0 ? c1 : (n - 1) + ~c1] = i;
    if (i == 0) parent[0] = -1;
}

// ---- leaves: triangle records in sorted order and their boxes ----
__global__ __launch_bounds__(kB) void leaves_kernel(const float* __restrict__ tris, const uint32_t* __restrict__ obj,
                                                    const uint32_t* __restrict__ order, uint32_t T, float4* tri_out,
                                                    float* box, uint32_t* rec_of) {
    const uint32_t k = blockIdx.x * kB + threadIdx.x;
    if (k >= T) return;
    if (order) rec_of[order[k]] = k;
    // build: sorted position k holds input triangle order[k]; refit (order
    // NULL): the current record holds the input index and the object id
    const uint32_t src = order ? order[k] : __float_as_uint(tri_out[3ull * k].w);
    const float* v = tris + 9ull * src;
    const uint32_t oid = order ? (obj ? obj[src] : src) : __float_as_uint(tri_out[3ull * k + 1].w);
    tri_out[3ull * k + 0] = make_float4(v[0], v[1], v[2], __uint_as_float(src));
    tri_out[3ull * k + 1] = make_float4(v[3] - v[0], v[4] - v[1], v[5] - v[2], __uint_as_float(oid));
    tri_out[3ull * k + 2] = make_float4(v[6] - v[0], v[7] - v[1], v[8] - v[2], 0.0f);
    float* b = box + 6ull * ((T - 1) + k);
    for (int a = 0; a < 3; ++a) {
        b[a] = fminf(fminf(v[a], v[3 + a]), v[6 + a]);
        b[3 + a] = fmaxf(fmaxf(v[a], v[3 + a]), v[6 + a]);
    }
}

// ---- internal boxes bottom-up, one level per launch: the launches order the
// levels, so no fences or arrival counters are needed (device-scope fences
// would write back every XCD's L2) ----
// sort key of internal node i: 63 - its depth (root 0), found by walking
// the parent links (at most 63 of them), so the deepest level sorts first
__global__ __launch_bounds__(kB) void depth_kernel(const int* __restrict__ parent, uint32_t NI, uint32_t* key) {
    const uint32_t i = blockIdx.x * kB + threadIdx.x;
    if (i >= NI) return;
    uint32_t d = 0;
    for (int n = parent[i]; n >= 0 && d < 63; n = parent[n]) ++d;
    key[i] = 63u - d;
}

// start[key] = first sorted position holding that key
__global__ __launch_bounds__(kB) void level_start_kernel(const uint32_t* __restrict__ key, uint32_t n,
                                                         uint32_t* start) {
    const uint32_t k = blockIdx.x * kB + threadIdx.x;
    if (k < n && (k == 0 || key[k] != key[k - 1])) start[key[k]] = k;
}

__global__ __launch_bounds__(kB) void merge_kernel(const uint32_t* __restrict__ nodes, uint32_t n,
                                                   const int2* __restrict__ child, uint32_t T, float* box) {
    const uint32_t k = blockIdx.x * kB + threadIdx.x;
    if (k >= n) return;
    const uint32_t node = nodes[k];
    const int2 c = child[node];
    const uint32_t a = c.x >= 0 ? (uint32_t)c.x : (T - 1) + ~c.x;
    const uint32_t b = c.y >= 0 ? (uint32_t)c.y : (T - 1) + ~c.y;
    for (int q = 0; q < 3; ++q) {
        box[6ull * node + q] = fminf(box[6ull * a + q], box[6ull * b + q]);
        box[6ull * node + 3 + q] = fmaxf(box[6ull * a + 3 + q], box[6ull * b + 3 + q]);
    }
}

// ---- node records in the traversal's layout ----
// A subtree of at most kLeafMax triangles (consecutive in sorted order)
// becomes one leaf of its parent; the nodes inside it are left unreferenced.
constexpr int kLeafMax = 4;

__global__ __launch_bounds__(kB) void emit_kernel(const int2* __restrict__ child, const int2* __restrict__ range,
                                                  const float* __restrict__ box, uint32_t T,
                                                  const float* __restrict__ bounds, float4* nodes) {
    const uint32_t i = blockIdx.x * kB + threadIdx.x;
    if (i >= T - 1) return;
    const float pad = ldexpf(fmaxf(bounds[6], 1e-6f), -20);
    const int2 c = child[i];
    float lo[2][3], hi[2][3];
    int ref[2];
    for (int s = 0; s < 2; ++s) {
        const int r = s ? c.y : c.x;
        const uint32_t n = r >= 0 ? (uint32_t)r : (T - 1) + ~r;
        for (int a = 0; a < 3; ++a) {
            lo[s][a] = box[6ull * n + a] - pad;
            hi[s][a] = box[6ull * n + 3 + a] + pad;
        }
        if (r < 0) {
            ref[s] = ~(int)((uint32_t)~r << kLeafCountBits);  // leaf of one triangle
        } else {
            const int2 rg = range[r];
            const int cnt = rg.y - rg.x + 1;
            ref[s] = cnt <= kLeafMax ? ~(int)(((uint32_t)rg.x << kLeafCountBits) | (uint32_t)(cnt - 1)) : r;
        }
    }
    float4* o = nodes + 4ull * i;
    o[0] = make_float4(lo[0][0], hi[0][0], lo[0][1], hi[0][1]);
    o[1] = make_float4(lo[1][0], hi[1][0], lo[1][1], hi[1][1]);
    o[2] = make_float4(lo[0][2], hi[0][2], lo[1][2], hi[1][2]);
    o[3] = __builtin_bit_cast(float4, make_int4(ref[0], ref[1], 0, 0));
}

// A single triangle: a root whose first child is the leaf and whose second
// child is empty (an inverted box no ray enters).
__global__ void single_root_kernel(const float* __restrict__ tris, const float* __restrict__ bounds, float4* nodes) {
    const float pad = ldexpf(fmaxf(bounds[6], 1e-6f), -20);
    float lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = fminf(fminf(tris[a], tris[3 + a]), tris[6 + a]) - pad;
        hi[a] = fmaxf(fmaxf(tris[a], tris[3 + a]), tris[6 + a]) + pad;
    }
    nodes[0] = make_float4(lo[0], hi[0], lo[1], hi[1]);
    nodes[1] = make_float4(1e30f, -1e30f, 1e30f, -1e30f);
    nodes[2] = make_float4(lo[2], hi[2], 1e30f, -1e30f);
    nodes[3] = __builtin_bit_cast(float4, make_int4(~0, -1, 0, 0));
}

__global__ void iota_kernel(uint32_t* v, uint32_t n) {
    const uint32_t i = blockIdx.x * kB + threadIdx.x;
    if (i < n) v[i] = i;
}

uint32_t blocks(uint64_t n) { return (uint32_t)((n + kB - 1) / kB); }

// Bounds, triangle records and boxes for the current vertices, then the node
// records.  `order[k]` is the input index of sorted triangle k.
dhr_status fill(dhr_ctx* ctx, dhr_bvh* b, const float* tris, const uint32_t* obj, const uint32_t* order,
                hipStream_t s, const char* what) {
    const uint32_t T = b->n_tris;
    const uint32_t nb = std::min<uint32_t>(blocks(T), 1024);
    hipLaunchKernelGGL(bounds_kernel, dim3(nb), dim3(kB), 0, s, tris, T, b->bounds);
    hipLaunchKernelGGL(bounds_final_kernel, dim3(1), dim3(kB), 0, s, b->bounds, nb);
    if (T == 1) {
        hipLaunchKernelGGL(leaves_kernel, dim3(1), dim3(kB), 0, s, tris, obj, order, T, b->tris, b->box, b->rec_of);
        hipLaunchKernelGGL(single_root_kernel, dim3(1), dim3(1), 0, s, tris, b->bounds, b->nodes);
        return check_launch(ctx, what);
    }
    hipLaunchKernelGGL(leaves_kernel, dim3(blocks(T)), dim3(kB), 0, s, tris, obj, order, T, b->tris, b->box, b->rec_of);
    for (size_t l = 0; l + 1 < b->level_off.size(); ++l) {
        const uint32_t o = b->level_off[l], n = b->level_off[l + 1] - o;
        if (n) hipLaunchKernelGGL(merge_kernel, dim3(blocks(n)), dim3(kB), 0, s, b->by_depth + o, n, b->child, T, b->box);
    }
    hipLaunchKernelGGL(emit_kernel, dim3(blocks(T - 1)), dim3(kB), 0, s, b->child, b->range, b->box, T, b->bounds,
                       b->nodes);
    return check_launch(ctx, what);
}

void release(dhr_bvh* b) {
    for (void* p : {(void*)b->nodes, (void*)b->tris, (void*)b->rec_of, (void*)b->child, (void*)b->range,
                    (void*)b->parent, (void*)b->box, (void*)b->by_depth, (void*)b->bounds})
        if (p) (void)hipFree(p);
    delete b;
}

}  // namespace
}  // namespace dhr

extern "C" {

dhr_status dhr_build_bvh_device(dhr_ctx* ctx, const float* tris, const uint32_t* obj_id, uint32_t T, dhr_bvh** out,
                                dhr_stream stream) {
    using namespace dhr;
    if (!ctx) return DHR_ERR_INVALID_ARG;
    if (!tris || !out) return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_build_bvh_device: null pointer");
    *out = nullptr;
    if (T == 0 || T > (1u << 28))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_build_bvh_device: T = %u outside 1..2^28", T);
    if ((reinterpret_cast<uintptr_t>(tris) & 3) || (obj_id && (reinterpret_cast<uintptr_t>(obj_id) & 3)))
        return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_build_bvh_device: misaligned buffer");
    DeviceGuard g(ctx->device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    dhr_bvh* b = new dhr_bvh;
    b->ctx = ctx;
    b->device = ctx->device;
    b->n_tris = T;
    const uint64_t NI = T > 1 ? T - 1 : 1;  // internal nodes (a lone triangle gets a root)
    uint32_t *key = nullptr, *key2 = nullptr, *val = nullptr, *order = nullptr;
    void* tmp = nullptr;
    size_t tmp_bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, key, key2, val, order, (int)T, 0, 30, s);
    size_t tmp_depth = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_depth, key, key2, val, order, (int)NI, 0, 6, s);
    tmp_bytes = std::max(tmp_bytes, tmp_depth);
    bool ok = hipMalloc(&b->nodes, NI * 64) == hipSuccess && hipMalloc(&b->tris, 48ull * T) == hipSuccess &&
              hipMalloc(&b->rec_of, 4ull * T) == hipSuccess &&
              hipMalloc(&b->child, sizeof(int2) * NI) == hipSuccess && hipMalloc(&b->range, sizeof(int2) * NI) == hipSuccess &&
              hipMalloc(&b->parent, sizeof(int) * (NI + T)) == hipSuccess &&
              hipMalloc(&b->box, 24ull * (NI + T)) == hipSuccess && hipMalloc(&b->by_depth, 4ull * NI) == hipSuccess &&
              hipMalloc(&b->bounds, 4ull * 7 * 1024) == hipSuccess && hipMalloc(&key, 4ull * T) == hipSuccess &&
              hipMalloc(&key2, 4ull * T) == hipSuccess && hipMalloc(&val, 4ull * std::max<uint64_t>(T, 64)) == hipSuccess &&
              hipMalloc(&order, 4ull * T) == hipSuccess && hipMalloc(&tmp, std::max<size_t>(tmp_bytes, 16)) == hipSuccess;
    auto cleanup = [&] {
        for (void* p : {(void*)key, (void*)key2, (void*)val, (void*)tmp}) if (p) (void)hipFree(p);
    };
    if (!ok) {
        (void)hipGetLastError();
        if (order) (void)hipFree(order);
        cleanup();
        release(b);
        return set_error(ctx, DHR_ERR_OOM, "dhr_build_bvh_device: device allocation failed");
    }
    const auto t0 = std::chrono::steady_clock::now();
    dhr_status st = DHR_OK;
    const uint32_t nb = std::min<uint32_t>(blocks(T), 1024);
    hipLaunchKernelGGL(bounds_kernel, dim3(nb), dim3(kB), 0, s, tris, T, b->bounds);
    hipLaunchKernelGGL(bounds_final_kernel, dim3(1), dim3(kB), 0, s, b->bounds, nb);
    if (T > 1) {
        hipLaunchKernelGGL(morton_kernel, dim3(blocks(T)), dim3(kB), 0, s, tris, T, b->bounds, key, val);
        if (hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, key, key2, val, order, (int)T, 0, 30, s) != hipSuccess)
            st = set_error(ctx, DHR_ERR_DEVICE, "dhr_build_bvh_device: sort failed");
        if (st == DHR_OK) {
            hipLaunchKernelGGL(karras_kernel, dim3(blocks(T - 1)), dim3(kB), 0, s, key2, (int)T, b->child, b->parent,
                               b->range);
            // internal nodes grouped by depth, deepest first, for the
            // level-by-level box pass
            hipLaunchKernelGGL(depth_kernel, dim3(blocks(NI)), dim3(kB), 0, s, b->parent, (uint32_t)NI, key);
            hipLaunchKernelGGL(iota_kernel, dim3(blocks(NI)), dim3(kB), 0, s, val, (uint32_t)NI);
            if (hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, key, key2, val, b->by_depth, (int)NI, 0, 6, s) !=
                hipSuccess)
                st = set_error(ctx, DHR_ERR_DEVICE, "dhr_build_bvh_device: sort failed");
        }
        uint32_t start[64];
        if (st == DHR_OK) {
            if (hipMemsetAsync(val, 0xFF, sizeof(start), s) != hipSuccess)
                st = set_error(ctx, DHR_ERR_DEVICE, "dhr_build_bvh_device: clearing level starts failed");
            else
                hipLaunchKernelGGL(level_start_kernel, dim3(blocks(NI)), dim3(kB), 0, s, key2, (uint32_t)NI, val);
        }
        if (st == DHR_OK && (hipMemcpyAsync(start, val, sizeof(start), hipMemcpyDeviceToHost, s) != hipSuccess ||
                             hipStreamSynchronize(s) != hipSuccess))
            st = set_error(ctx, DHR_ERR_DEVICE, "dhr_build_bvh_device: %s", hipGetErrorString(hipGetLastError()));
        if (st == DHR_OK) {
            for (int k = 0; k < 64; ++k)
                if (start[k] != 0xFFFFFFFFu) b->level_off.push_back(start[k]);
            b->level_off.push_back((uint32_t)NI);
        }
    } else {
        hipLaunchKernelGGL(iota_kernel, dim3(1), dim3(kB), 0, s, order, 1u);
    }
    if (st == DHR_OK) st = check_launch(ctx, "dhr_build_bvh_device");
    if (st == DHR_OK) st = fill(ctx, b, tris, obj_id, order, s, "dhr_build_bvh_device");
    // the sorted order is kept in the triangles' w (original index); the
    // refit reads it from there
    if (st == DHR_OK && hipStreamSynchronize(s) != hipSuccess)
        st = set_error(ctx, DHR_ERR_DEVICE, "dhr_build_bvh_device: %s", hipGetErrorString(hipGetLastError()));
    (void)hipFree(order);
    cleanup();
    if (st != DHR_OK) {
        release(b);
        return st;
    }
    // levels of internal nodes, then one of leaves (the deepest internal
    // node's children are leaves)
    const uint32_t depth = T > 1 ? (uint32_t)b->level_off.size() : 2u;
    b->info.n_nodes = NI;
    b->info.n_tris = T;
    b->info.device_bytes = NI * 64 + 52ull * T;
    b->info.depth = depth;
    b->info.max_leaf_size = T > 1 ? (uint32_t)std::min<uint32_t>(T, kLeafMax) : 1u;
    b->info.sah_cost = 0.0;
    b->info.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (depth - 1 > (uint32_t)kStack) {  // interior nodes on the longest path
        release(b);
        return set_error(ctx, DHR_ERR_UNSUPPORTED, "dhr_build_bvh_device: depth %u beyond the traversal stack", depth);
    }
    *out = b;
    return DHR_OK;
}

dhr_status dhr_refit_bvh(dhr_ctx* ctx, dhr_bvh* bvh, const float* tris, dhr_stream stream) {
    using namespace dhr;
    if (!ctx) return DHR_ERR_INVALID_ARG;
    if (!bvh || !tris || bvh->ctx != ctx) return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_refit_bvh: bad argument");
    if (!bvh->box) return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_refit_bvh: the BVH was not built on the device");
    if (reinterpret_cast<uintptr_t>(tris) & 3) return set_error(ctx, DHR_ERR_INVALID_ARG, "dhr_refit_bvh: misaligned");
    DeviceGuard g(ctx->device);
    return fill(ctx, bvh, tris, nullptr, nullptr, reinterpret_cast<hipStream_t>(stream), "dhr_refit_bvh");
}

}  // extern "C"
