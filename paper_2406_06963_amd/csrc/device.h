// Device helpers: vector math, the counter-based RNG, direction samplers,
// BVH traversal and the ragged-batch tile mapping shared by every kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dhr {

// ---------------------------------------------------------------- float3 math
__device__ __forceinline__ float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
__device__ __forceinline__ float3 f3(float4 v) { return make_float3(v.x, v.y, v.z); }
__device__ __forceinline__ float3 operator+(float3 a, float3 b) { return f3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 operator-(float3 a, float3 b) { return f3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 operator*(float3 a, float s) { return f3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return f3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float3 normalize3(float3 a) { return a * (1.0f / sqrtf(dot3(a, a))); }

__device__ __forceinline__ uint32_t fbits(float f) { return __float_as_uint(f); }

// ---------------------------------------------------------------- RNG
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// multiply/xor S-box over a 4x32-bit counter, key bumped by the Weyl
// constants of the golden ratio and sqrt(3)-1 between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Two uniforms in [0,1) with 24 random bits each, exact in fp32.
__device__ __forceinline__ float2 ray_uniforms(uint32_t seed, uint32_t client, uint32_t x, uint32_t y, uint32_t frame,
                                               uint32_t stream, uint32_t sample) {
    const uint4 r = philox4x32_10(make_uint4(x, y, frame, (stream << 16) | sample), seed, client);
    return make_float2((float)(r.x >> 8) * 0x1p-24f, (float)(r.y >> 8) * 0x1p-24f);
}

// Orthonormal basis around unit n (Duff et al., JCGT 2017, branchless Frisvad).
__device__ __forceinline__ void onb(float3 n, float3& b1, float3& b2) {
    const float s = copysignf(1.0f, n.z);
    const float a = -1.0f / (s + n.z);
    const float b = n.x * n.y * a;
    b1 = f3(1.0f + s * n.x * n.x * a, s * b, -s * n.x);
    b2 = f3(b, s + n.y * n.y * a, -n.y);
}

// Cosine-weighted direction about n: Malley's method (uniform disk point
// lifted to the hemisphere).
__device__ __forceinline__ float3 sample_cosine(float3 n, float u0, float u1) {
    float sp, cp;
    sincospif(2.0f * u1, &sp, &cp);
    const float rho = sqrtf(u0);
    float3 b1, b2;
    onb(n, b1, b2);
    return b1 * (rho * cp) + b2 * (rho * sp) + n * sqrtf(1.0f - u0);
}

// Uniform direction in the cone about `axis` with 1 - cos(theta_max) = k.
__device__ __forceinline__ float3 sample_cone(float3 axis, float k, float u0, float u1) {
    const float s = u0 * k;
    const float ct = 1.0f - s;
    const float st = sqrtf(s * (2.0f - s));
    float sp, cp;
    sincospif(2.0f * u1, &sp, &cp);
    float3 b1, b2;
    onb(axis, b1, b2);
    return b1 * (st * cp) + b2 * (st * sp) + axis * ct;
}

// ---------------------------------------------------------------- batches
// Every kernel covers a ragged batch of jobs with one launch.  Job j owns the
// global tiles [tile0[j], tile0[j+1]); a workgroup finds its job by a scan
// over the (uniform, kernel-argument) prefix.
template <class D, int MAXB>
struct Batch {
    uint32_t n;
    uint32_t tile0[MAXB + 1];
    D d[MAXB];
};

__device__ __forceinline__ int find_job(const uint32_t* tile0, int n, uint32_t t) {
    int j = 0;
    while (j + 1 < n && t >= tile0[j + 1]) ++j;
    return j;
}

// ---------------------------------------------------------------- traversal
constexpr int kStack = 32;  // the builder caps the depth at 32

struct Ray {
    float3 o, d;
    float tmax;
};

__device__ __forceinline__ float3 safe_inv(float3 d) {
    const float e = 1e-20f;
    return f3(1.0f / (fabsf(d.x) > e ? d.x : copysignf(e, d.x)), 1.0f / (fabsf(d.y) > e ? d.y : copysignf(e, d.y)),
              1.0f / (fabsf(d.z) > e ? d.z : copysignf(e, d.z)));
}

// Slab test of both child boxes of a node against [0, tmax].
__device__ __forceinline__ void node_test(const float4* __restrict__ nodes, int node, float3 id, float3 ood,
                                          float tmax, bool& h0, bool& h1, float& tn0, float& tn1, int& c0, int& c1) {
    const float4 a = nodes[4 * node + 0];
    const float4 b = nodes[4 * node + 1];
    const float4 c = nodes[4 * node + 2];
    const int4 ch = __builtin_bit_cast(int4, nodes[4 * node + 3]);
    const float ax0 = fmaf(a.x, id.x, -ood.x), ax1 = fmaf(a.y, id.x, -ood.x);
    const float ay0 = fmaf(a.z, id.y, -ood.y), ay1 = fmaf(a.w, id.y, -ood.y);
    const float az0 = fmaf(c.x, id.z, -ood.z), az1 = fmaf(c.y, id.z, -ood.z);
    const float bx0 = fmaf(b.x, id.x, -ood.x), bx1 = fmaf(b.y, id.x, -ood.x);
    const float by0 = fmaf(b.z, id.y, -ood.y), by1 = fmaf(b.w, id.y, -ood.y);
    const float bz0 = fmaf(c.z, id.z, -ood.z), bz1 = fmaf(c.w, id.z, -ood.z);
    const float a_in = fmaxf(fmaxf(fminf(ax0, ax1), fminf(ay0, ay1)), fmaxf(fminf(az0, az1), 0.0f));
    const float a_out = fminf(fminf(fmaxf(ax0, ax1), fmaxf(ay0, ay1)), fminf(fmaxf(az0, az1), tmax));
    const float b_in = fmaxf(fmaxf(fminf(bx0, bx1), fminf(by0, by1)), fmaxf(fminf(bz0, bz1), 0.0f));
    const float b_out = fminf(fminf(fmaxf(bx0, bx1), fmaxf(by0, by1)), fminf(fmaxf(bz0, bz1), tmax));
    h0 = a_in <= a_out;
    h1 = b_in <= b_out;
    tn0 = a_in;
    tn1 = b_in;
    c0 = ch.x;
    c1 = ch.y;
}

// Moller-Trumbore in fp32 (two-sided, edges inclusive); returns t or NaN/inf
// outside.
__device__ __forceinline__ float tri_t(const float4* __restrict__ tris, int i, float3 o, float3 d) {
    const float4 v0 = tris[3 * i + 0];
    const float4 e1 = tris[3 * i + 1];
    const float4 e2 = tris[3 * i + 2];
    const float3 E1 = f3(e1), E2 = f3(e2);
    const float3 p = cross3(d, E2);
    const float det = dot3(E1, p);
    const float inv = 1.0f / det;
    const float3 tv = o - f3(v0);
    const float u = dot3(tv, p) * inv;
    const float3 q = cross3(tv, E1);
    const float v = dot3(d, q) * inv;
    const float t = dot3(E2, q) * inv;
    const bool inside = (u >= 0.0f) & (v >= 0.0f) & (u + v <= 1.0f);
    return inside ? t : __builtin_nanf("");
}

__device__ __forceinline__ void leaf_range(int ref, int& first, int& count) {
    const int l = ~ref;
    first = l >> 3;
    count = (l & 7) + 1;
}

// Traversal work counters of one lane (only the counting kernel variant keeps them).
struct TravCount {
    uint32_t nodes = 0, leaves = 0, tris = 0;
};

// Traversal in the while-while form with leaf postponing: a lane that reaches
// a leaf keeps it aside and goes on descending, and the wave only switches to
// triangle tests once every lane holds a leaf (or has nothing left), so the
// two kinds of work do not interleave within a wave.  The stack lives in LDS
// (`stk`: this lane's column, row stride `stride`); the builder caps the depth
// at kStack, and at most one entry is pushed per interior node on the path.
constexpr int kDone = 0x7FFFFFFF;  // empty stack

// Any hit at 0 < t < tmax.  With COUNT the lane's work is tallied in `cnt`.
template <bool COUNT = false>
__device__ __forceinline__ bool any_hit(const float4* __restrict__ nodes, const float4* __restrict__ tris,
                                        const Ray& r, int* stk, int stride, TravCount* cnt = nullptr) {
    const float3 id = safe_inv(r.d);
    const float3 ood = f3(r.o.x * id.x, r.o.y * id.y, r.o.z * id.z);
    int sp = 0;
    int node = 0;   // interior index >= 0, leaf ref < 0, kDone
    int leaf = 0;   // postponed leaf ref (< 0) or none (>= 0)
    while (node != kDone || leaf < 0) {
        while (node >= 0 && node != kDone) {
            bool h0, h1;
            float t0, t1;
            int c0, c1;
            if (COUNT) ++cnt->nodes;
            node_test(nodes, node, id, ood, r.tmax, h0, h1, t0, t1, c0, c1);
            if (h0 && h1) {
                const bool first0 = t0 <= t1;
                stk[sp * stride] = first0 ? c1 : c0;
                ++sp;
                node = first0 ? c0 : c1;
            } else if (h0 || h1) {
                node = h0 ? c0 : c1;
            } else {
                node = sp ? stk[--sp * stride] : kDone;
            }
            if (node < 0 && leaf >= 0) {
                leaf = node;
                node = sp ? stk[--sp * stride] : kDone;
            }
            if (!__any(leaf >= 0)) break;
        }
        while (leaf < 0) {
            int first, count;
            leaf_range(leaf, first, count);
            if (COUNT) ++cnt->leaves;
            for (int k = 0; k < count; ++k) {
                if (COUNT) ++cnt->tris;
                const float t = tri_t(tris, first + k, r.o, r.d);
                if (t > 0.0f && t < r.tmax) return true;
            }
            leaf = node;
            if (node < 0) node = sp ? stk[--sp * stride] : kDone;
        }
    }
    return false;
}

// Closest hit at t > 0 (ties: lowest original triangle index).  Returns the
// position of the triangle in leaf order, or -1.
__device__ __forceinline__ int closest_hit(const float4* __restrict__ nodes, const float4* __restrict__ tris,
                                           float3 o, float3 d, float& tbest, int* stk, int stride) {
    const float3 id = safe_inv(d);
    const float3 ood = f3(o.x * id.x, o.y * id.y, o.z * id.z);
    int sp = 0;
    int node = 0;
    int leaf = 0;
    int best = -1;
    uint32_t best_orig = 0xFFFFFFFFu;
    tbest = __builtin_inff();
    while (node != kDone || leaf < 0) {
        while (node >= 0 && node != kDone) {
            bool h0, h1;
            float t0, t1;
            int c0, c1;
            node_test(nodes, node, id, ood, tbest, h0, h1, t0, t1, c0, c1);
            if (h0 && h1) {
                const bool first0 = t0 <= t1;
                stk[sp * stride] = first0 ? c1 : c0;
                ++sp;
                node = first0 ? c0 : c1;
            } else if (h0 || h1) {
                node = h0 ? c0 : c1;
            } else {
                node = sp ? stk[--sp * stride] : kDone;
            }
            if (node < 0 && leaf >= 0) {
                leaf = node;
                node = sp ? stk[--sp * stride] : kDone;
            }
            if (!__any(leaf >= 0)) break;
        }
        while (leaf < 0) {
            int first, count;
            leaf_range(leaf, first, count);
            for (int k = 0; k < count; ++k) {
                const float t = tri_t(tris, first + k, o, d);
                if (t > 0.0f && t <= tbest) {
                    const uint32_t orig = fbits(tris[3 * (first + k)].w);
                    if (t < tbest || orig < best_orig) {
                        tbest = t;
                        best = first + k;
                        best_orig = orig;
                    }
                }
            }
            leaf = node;
            if (node < 0) node = sp ? stk[--sp * stride] : kDone;
        }
    }
    return best;
}

}  // namespace dhr
