// Library-internal declarations shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/dhr.h"

struct dhr_ctx {
    int device = 0;
    int n_cu = 0;
    std::string err;
    uint64_t* trace_counters = nullptr;  // instrumentation (dhr_set_trace_counters)
    void* scratch = nullptr;             // device address of this device's filter scratch (dhr_svgf_filter_noalloc)
    bool wide_records = false;           // DHR_WIDE_RECORDS=1: 64-bit record addressing for every tree
};

// Device-resident BVH.  Node: 4 x 16 bytes (two child boxes + child refs);
// triangle: 3 x 16 bytes (v0 + original index, e1 + object id, e2).
struct dhr_bvh {
    dhr_ctx* ctx = nullptr;  // identity only: never dereferenced after creation
    int device = 0;
    float4* nodes = nullptr;
    float4* tris = nullptr;
    uint32_t* rec_of = nullptr;  // [T]: leaf-order record of each input triangle
    // two-level hierarchies (dhr_build_bvh_instanced): `nodes` starts with the
    // top level; `tl` is the device description of instances and bottom levels
    void* tl = nullptr;
    float4* inst = nullptr;
    dhr_bvh_info info{};
    // topology kept by the device build for refits (NULL for host builds):
    // children of each internal node, parents of internal nodes and leaves,
    // per-node boxes and arrival counters of the bottom-up pass
    int2* child = nullptr;
    int2* range = nullptr;        // [T - 1]: sorted triangle positions under each internal node
    int* parent = nullptr;        // [T - 1] internal, then [T] leaves
    float* box = nullptr;         // [T - 1 + T][6]
    uint32_t* by_depth = nullptr; // internal nodes ordered by depth, deepest level first
    float* bounds = nullptr;      // reduction scratch
    uint32_t n_tris = 0;
    std::vector<uint32_t> level_off;  // by_depth ranges of the levels, deepest first
};

namespace dhr {

// The "leaf" child reference: ~(first << 3 | (count - 1)), always < 0.
constexpr int kLeafCountBits = 3;

dhr_status set_error(dhr_ctx* ctx, dhr_status st, const char* fmt, ...);

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
inline bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

// Makes the context's device current for the scope of an entry point.
class DeviceGuard {
   public:
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
        if (prev_ != dev) (void)hipSetDevice(dev);
        dev_ = dev;
    }
    ~DeviceGuard() {
        if (prev_ >= 0 && prev_ != dev_) (void)hipSetDevice(prev_);
    }

   private:
    int prev_ = -1, dev_ = 0;
};

// Checks the launch(es) just enqueued.
dhr_status check_launch(dhr_ctx* ctx, const char* what);

// Sets ctx->scratch to the device address of the no-alloc filter's scratch on
// ctx->device (looked up once per device).
dhr_status svgf_scratch_init(dhr_ctx* ctx);

// Host image of the device description of a two-level hierarchy (the
// layout of the kernels' TwoLevel: instance records, then the node and
// triangle arrays of bottom levels 0 and 1).
struct TwoLevelHost {
    const float4* inst;
    const float4* nodes[2];
    const float4* tris[2];
};

// Host-side BVH build into flat arrays ready for upload.
struct HostBvh {
    std::string error;
    uint64_t n_nodes = 0;
    uint32_t depth = 0, max_leaf_size = 0;
    double sah_cost = 0.0;
    float4* nodes = nullptr;  // n_nodes * 4 float4 (malloc'd)
    float4* tris = nullptr;   // T * 3 float4 (malloc'd)
};
bool build_host_bvh(const float* tris, const uint32_t* obj_id, uint32_t T, const dhr_bvh_opts& opts,
                    HostBvh* out);

}  // namespace dhr
