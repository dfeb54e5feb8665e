// Device helpers: vector math, the counter-based RNG, direction samplers,
// BVH traversal and the ragged-batch tile mapping shared by every kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

// Every helper below rounds each operation on its own unless an fmaf is
// written out: the rasterised and the ray-traced G-buffer inline the same
// helpers into different kernels and must produce the same bits, which
// contraction chosen per inlining context would not guarantee.  The build's
// setting is restored at the end of the header.
#pragma clang fp contract(off)

namespace dhr {

// ---------------------------------------------------------------- float3 math
__device__ __forceinline__ float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
__device__ __forceinline__ float3 f3(float4 v) { return make_float3(v.x, v.y, v.z); }
__device__ __forceinline__ float3 operator+(float3 a, float3 b) { return f3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 operator-(float3 a, float3 b) { return f3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 operator*(float3 a, float s) { return f3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ float dot3(float3 a, float3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return f3(fmaf(a.y, b.z, -(a.z * b.y)), fmaf(a.z, b.x, -(a.x * b.z)), fmaf(a.x, b.y, -(a.y * b.x)));
}
__device__ __forceinline__ float3 normalize3(float3 a) { return a * (1.0f / sqrtf(dot3(a, a))); }

__device__ __forceinline__ uint32_t fbits(float f) { return __float_as_uint(f); }

// ---------------------------------------------------------------- RNG
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// multiply/xor S-box over a 4x32-bit counter, key bumped by the Weyl
// constants of the golden ratio and sqrt(3)-1 between rounds.  Each product
// is taken as one 32 x 32 -> 64-bit multiply (one v_mad_u64_u32 for both
// halves instead of a low and a high multiply, both quarter rate).
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
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
// Traversal stack depth: at most one entry is pushed per interior node on the
// current path.  The host builder caps the depth at 32; device-built trees
// have at most 64 interior nodes on a path (their common-prefix lengths grow
// strictly from 0 to at most 63).
constexpr int kStack = 64;

struct Ray {
    float3 o, d;
    float tmax;
};

// Inverse direction for the slab tests, components clamped away from zero
// (|1/d| <= 1e20).  The hardware reciprocal (about 1 ulp) instead of a
// correctly rounded division: it only sets where the box tests prune, and
// the same value serves every plane of a ray, so the test stays monotone in
// the plane.
__device__ __forceinline__ float3 safe_inv(float3 d) {
    const float e = 1e-20f;
    return f3(__builtin_amdgcn_rcpf(fabsf(d.x) > e ? d.x : copysignf(e, d.x)),
              __builtin_amdgcn_rcpf(fabsf(d.y) > e ? d.y : copysignf(e, d.y)),
              __builtin_amdgcn_rcpf(fabsf(d.z) > e ? d.z : copysignf(e, d.z)));
}

// A node: the two child boxes (x and y slabs of child 0, of child 1, then the
// z slabs of both) and the two child references.
struct NodeRec {
    float4 a, b, c, ch;
};

// Records are read at wave-uniform indices through the constant address
// space (the tree is read-only while kernels run): one scalar load per wave
// instead of a vector load per lane.
typedef float vf4 __attribute__((ext_vector_type(4)));
using cvf4 = const __attribute__((address_space(4))) vf4;

__device__ __forceinline__ float4 ld_const(const float4* base, int i) {
    const vf4 v = ((cvf4*)base)[i];
    return make_float4(v.x, v.y, v.z, v.w);
}

// Record addressing.  Narrow (WIDE = false): the record's byte offset as a
// 32-bit value, which the scalar load takes as its SGPR offset, so a node
// step spends one shift instead of 64-bit address arithmetic on the scalar
// unit (the walk's other bottleneck beside VALU issue).  It needs each array
// under 4 GB: trees_narrow() on the host.  Wide: 64-bit offsets, any size.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* at_byte(const float4* base, uint32_t off) {
    return (const __attribute__((address_space(4))) T*)((const __attribute__((address_space(4))) char*)base + off);
}
__device__ __forceinline__ float4 f4of(vf4 v) { return make_float4(v.x, v.y, v.z, v.w); }

template <bool WIDE>
__device__ __forceinline__ NodeRec load_node_uniform(const float4* __restrict__ nodes, int node) {
    if (WIDE)
        return NodeRec{ld_const(nodes, 4 * node), ld_const(nodes, 4 * node + 1), ld_const(nodes, 4 * node + 2),
                       ld_const(nodes, 4 * node + 3)};
    const __attribute__((address_space(4))) vf4* p = at_byte<vf4>(nodes, (uint32_t)node << 6);
    return NodeRec{f4of(p[0]), f4of(p[1]), f4of(p[2]), f4of(p[3])};
}

// Slab test of both child boxes of a node against [0, tmax]: per axis the
// entry plane is the min and the exit plane the max of the two plane
// distances.  (Picking the planes once per wave where every lane's direction
// has the same signs saves the min and max, but the pick costs a vector move
// and select per plane, or scalar-unit work that the loop's control flow
// already keeps busy; both measured slower.)
// Returns each child's entry and exit distance (entry clamped to 0); the
// child is hit where entry <= min(exit, tmax).
//
// OCT >= 0: every live lane's direction has the sign pattern OCT (bit k set:
// axis k negative), so the entry plane of each axis is known at compile time
// (the lower plane for a positive direction, the upper for a negative one)
// and the min / max pairs drop out: 23 VALU per node instead of 35.  The
// plane distances are fma(plane, 1/d, -o/d), monotone in the plane, so the
// picked plane is the one the min / max would pick, bit for bit.  Lanes
// whose signs differ may only be dead ones (tmax < 0: an entry >= 0 never
// passes entry <= tmax).
template <int OCT = -1>
__device__ __forceinline__ void box_test(const NodeRec& n, float3 id, float3 ood, float& a_in, float& a_out,
                                         float& b_in, float& b_out, int& c0, int& c1) {
    const float4 a = n.a, b = n.b, c = n.c;
    const int4 ch = __builtin_bit_cast(int4, n.ch);
    const float ax0 = fmaf(a.x, id.x, -ood.x), ax1 = fmaf(a.y, id.x, -ood.x);
    const float ay0 = fmaf(a.z, id.y, -ood.y), ay1 = fmaf(a.w, id.y, -ood.y);
    const float az0 = fmaf(c.x, id.z, -ood.z), az1 = fmaf(c.y, id.z, -ood.z);
    const float bx0 = fmaf(b.x, id.x, -ood.x), bx1 = fmaf(b.y, id.x, -ood.x);
    const float by0 = fmaf(b.z, id.y, -ood.y), by1 = fmaf(b.w, id.y, -ood.y);
    const float bz0 = fmaf(c.z, id.z, -ood.z), bz1 = fmaf(c.w, id.z, -ood.z);
    if constexpr (OCT < 0) {
        a_in = fmaxf(fmaxf(fminf(ax0, ax1), fminf(ay0, ay1)), fmaxf(fminf(az0, az1), 0.0f));
        a_out = fminf(fminf(fmaxf(ax0, ax1), fmaxf(ay0, ay1)), fmaxf(az0, az1));
        b_in = fmaxf(fmaxf(fminf(bx0, bx1), fminf(by0, by1)), fmaxf(fminf(bz0, bz1), 0.0f));
        b_out = fminf(fminf(fmaxf(bx0, bx1), fmaxf(by0, by1)), fmaxf(bz0, bz1));
    } else {
        constexpr bool nx = OCT & 1, ny = OCT & 2, nz = OCT & 4;
        a_in = fmaxf(fmaxf(nx ? ax1 : ax0, ny ? ay1 : ay0), fmaxf(nz ? az1 : az0, 0.0f));
        a_out = fminf(fminf(nx ? ax0 : ax1, ny ? ay0 : ay1), nz ? az0 : az1);
        b_in = fmaxf(fmaxf(nx ? bx1 : bx0, ny ? by1 : by0), fmaxf(nz ? bz1 : bz0, 0.0f));
        b_out = fminf(fminf(nx ? bx0 : bx1, ny ? by0 : by1), nz ? bz0 : bz1);
    }
    c0 = ch.x;
    c1 = ch.y;
}

// The sign pattern shared by the live lanes' directions (bit k: axis k
// negative, as the sign of the clamped inverse), or -1 if they differ.
__device__ __forceinline__ int wave_octant(float3 id, bool live) {
    const uint64_t L = __ballot(live);
    const uint64_t sx = __ballot(live && id.x < 0.0f), sy = __ballot(live && id.y < 0.0f),
                   sz = __ballot(live && id.z < 0.0f);
    if ((sx != 0 && sx != L) || (sy != 0 && sy != L) || (sz != 0 && sz != L)) return -1;
    return (sx ? 1 : 0) | (sy ? 2 : 0) | (sz ? 4 : 0);
}

// Moller-Trumbore in fp32 (two-sided, edges inclusive) of the triangle
// (v0, e1, e2); returns t or NaN/inf outside.
__device__ __forceinline__ float tri_t_rec(float4 v0, float4 e1, float4 e2, float3 o, float3 d) {
    const float3 E1 = f3(e1), E2 = f3(e2);
    const float3 p = cross3(d, E2);
    const float det = dot3(E1, p);
    const float inv = __builtin_amdgcn_rcpf(det);
    const float3 tv = o - f3(v0);
    const float u = dot3(tv, p) * inv;
    const float3 q = cross3(tv, E1);
    const float v = dot3(d, q) * inv;
    const float t = dot3(E2, q) * inv;
    const bool inside = (u >= 0.0f) & (v >= 0.0f) & (u + v <= 1.0f);
    return inside ? t : __builtin_nanf("");
}

// Triangle i read at a wave-uniform index (scalar loads).
__device__ __forceinline__ float tri_t_uniform(const float4* __restrict__ tris, int i, float3 o, float3 d,
                                               uint32_t* orig = nullptr) {
    const float4 v0 = ld_const(tris, 3 * i);
    if (orig) *orig = fbits(v0.w);
    return tri_t_rec(v0, ld_const(tris, 3 * i + 1), ld_const(tris, 3 * i + 2), o, d);
}

// A triangle record (v0 + original index, e1 + object id, e2).
struct TriRec {
    float4 v0, e1, e2;
};
template <bool WIDE>
__device__ __forceinline__ TriRec load_tri_uniform(const float4* __restrict__ tris, int i) {
    if (WIDE) return TriRec{ld_const(tris, 3 * i), ld_const(tris, 3 * i + 1), ld_const(tris, 3 * i + 2)};
    const __attribute__((address_space(4))) vf4* p = at_byte<vf4>(tris, (uint32_t)i * 48u);
    return TriRec{f4of(p[0]), f4of(p[1]), f4of(p[2])};
}

// Whether the ray hits triangle (v0, e1, e2) at 0 < t < tmax: the
// Moller-Trumbore tests with the barycentrics and t left unnormalised
// (multiplied by det, signed by det), so no division is needed.
struct TriTest {
    float U, V, T, ad;
};
__device__ __forceinline__ TriTest tri_test_rec(const TriRec& r, float3 o, float3 d) {
    const float4 v0 = r.v0, e1 = r.e1, e2 = r.e2;
    const float3 E1 = f3(e1), E2 = f3(e2);
    const float3 p = cross3(d, E2);
    const float det = dot3(E1, p);
    const float3 tv = o - f3(v0);
    const float3 q = cross3(tv, E1);
    const uint32_t sgn = fbits(det) & 0x80000000u;
    return TriTest{__uint_as_float(fbits(dot3(tv, p)) ^ sgn), __uint_as_float(fbits(dot3(d, q)) ^ sgn),
                   __uint_as_float(fbits(dot3(E2, q)) ^ sgn), fabsf(det)};
}
__device__ __forceinline__ bool tri_hits_rec(const TriRec& r, float3 o, float3 d, float tmax) {
    const TriTest h = tri_test_rec(r, o, d);
    return (h.U >= 0.0f) & (h.V >= 0.0f) & (h.U + h.V <= h.ad) & (h.T > 0.0f) & (h.T < tmax * h.ad);
}
// The same test for the whole wave as a lane mask, each compare's own
// ballot combined on the scalar unit (no per-lane flag to materialise).
__device__ __forceinline__ uint64_t tri_hit_mask(const TriRec& r, float3 o, float3 d, float tmax) {
    const TriTest h = tri_test_rec(r, o, d);
    return __builtin_amdgcn_ballot_w64(h.U >= 0.0f) & __builtin_amdgcn_ballot_w64(h.V >= 0.0f) &
           __builtin_amdgcn_ballot_w64(h.U + h.V <= h.ad) & __builtin_amdgcn_ballot_w64(h.T > 0.0f) &
           __builtin_amdgcn_ballot_w64(h.T < tmax * h.ad);
}

template <bool WIDE>
__device__ __forceinline__ bool tri_hits_uniform(const float4* __restrict__ tris, int i, float3 o, float3 d,
                                                 float tmax) {
    return tri_hits_rec(load_tri_uniform<WIDE>(tris, i), o, d, tmax);
}

// Two consecutive records i, i + 1 (96 bytes) as one 64- and one 32-byte
// scalar load, so both are in flight before either is tested.
typedef float vf16 __attribute__((ext_vector_type(16)));
typedef float vf8 __attribute__((ext_vector_type(8)));
template <bool WIDE>
__device__ __forceinline__ void load_tri_pair_uniform(const float4* __restrict__ tris, int i, TriRec& a, TriRec& b) {
    const vf16 p = WIDE ? *(const __attribute__((address_space(4))) vf16*)(tris + 3 * i)
                        : *at_byte<vf16>(tris, (uint32_t)i * 48u);
    const vf8 q = WIDE ? *(const __attribute__((address_space(4))) vf8*)(tris + 3 * i + 4)
                       : *at_byte<vf8>(tris, (uint32_t)i * 48u + 64u);
    a = TriRec{make_float4(p[0], p[1], p[2], p[3]), make_float4(p[4], p[5], p[6], p[7]),
               make_float4(p[8], p[9], p[10], p[11])};
    b = TriRec{make_float4(p[12], p[13], p[14], p[15]), make_float4(q[0], q[1], q[2], q[3]),
               make_float4(q[4], q[5], q[6], q[7])};
}

// The triangles [first, first + count) of a leaf two at a time: a pair's
// records arrive by one request, so a leaf pays one load latency per pair
// instead of one per triangle; an odd last triangle is loaded alone (the
// record after it may lie beyond the array).  test(rec, index) is called in
// index order.
template <bool WIDE, class Test>
__device__ __forceinline__ void leaf_pairs(const float4* __restrict__ tris, int first, int count, Test test) {
    int k = 0;
    for (; k + 1 < count; k += 2) {
        TriRec a, b;
        load_tri_pair_uniform<WIDE>(tris, first + k, a, b);
        test(a, first + k);
        test(b, first + k + 1);
    }
    if (k < count) test(load_tri_uniform<WIDE>(tris, first + k), first + k);
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

constexpr int kDone = 0x7FFFFFFF;  // empty stack

// ---------------------------------------------------------------- traversal
// The whole wave walks one path through the tree: the union of its lanes'
// paths (rays of a wave come from an 8 x 8 pixel square, so they share most
// of it).  A child is entered when any lane's ray hits its box, the nearer
// child first by majority vote of the lanes that hit both.  Node and
// triangle records are read once per wave at a uniform address (scalar
// loads), and the stack is one LDS column per wave (`wstk`,
// kStack entries: no path holds more than kStack interior nodes and at most one entry
// is pushed per level).  Child boxes lie inside the parent's box and the slab
// test is monotone in the planes, so a lane visits every node its own ray
// hits: each lane's result is that of a traversal of its own ray.  Lanes
// without work pass tmax < 0, which misses every box.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// visit_leaf(first, count) tests a leaf's triangles for every lane; done()
// is true once no lane needs more of the walk; tmax is read at every node.
// With COUNT, `cnt` tallies the work of this lane's own ray: the nodes and
// leaves whose boxes it hits (a bit stack beside the wave's stack records
// whether it hit each pushed child) and the triangles of those leaves.
template <bool COUNT, int OCT, bool WIDE, class Leaf, class Done>
__device__ __forceinline__ void packet_walk(const float4* __restrict__ nodes, float3 id, float3 ood,
                                            const float& tmax, bool live, int* wstk, Leaf visit_leaf, Done done,
                                            TravCount* cnt) {
    int sp = 0, node = 0;
    bool in = live;          // COUNT: this lane's ray hits the current node
    uint64_t in_stack = 0;   // COUNT: the same for every stack entry (up to 64)
    while (true) {
        if (node >= 0) {
            float t0, x0, t1, x1;
            int c0, c1;
            if (COUNT && in) ++cnt->nodes;
            box_test<OCT>(load_node_uniform<WIDE>(nodes, node), id, ood, t0, x0, t1, x1, c0, c1);
            c0 = uniform(c0);
            c1 = uniform(c1);
            // hit masks: entry <= min(exit, tmax), one compare per child (the
            // distances are never NaN: the inverse direction is clamped to 1e20)
            const uint64_t m0 = __ballot(t0 <= fminf(x0, tmax));
            const uint64_t m1 = __ballot(t1 <= fminf(x1, tmax));
            const bool h0 = COUNT && (t0 <= x0) && (t0 <= tmax), h1 = COUNT && (t1 <= x1) && (t1 <= tmax);
            // Each branch below tests one scalar comparison made just before
            // it: booleans combined with others would be kept as lane masks,
            // at several scalar instructions per node.
            if ((m0 | m1) == 0) {  // neither child: the next stack entry
                if (sp == 0) return;
                node = uniform(wstk[--sp]);
                if (COUNT) in = (in_stack >> sp) & 1ull;
                continue;
            }
            if (m1 == 0) {
                if (COUNT) in = h0;
                node = c0;
                continue;
            }
            if (m0 == 0) {
                if (COUNT) in = h1;
                node = c1;
                continue;
            }
            // both children: the nearer one of the majority of the lanes that
            // hit both goes first
            const uint64_t both = m0 & m1, f0 = both & __ballot(t0 <= t1);
            if (2 * __popcll(f0) >= __popcll(both)) {
                if (COUNT) {
                    in_stack = (in_stack & ~(1ull << sp)) | (h1 ? 1ull << sp : 0ull);
                    in = h0;
                }
                wstk[sp++] = c1;
                node = c0;
            } else {
                if (COUNT) {
                    in_stack = (in_stack & ~(1ull << sp)) | (h0 ? 1ull << sp : 0ull);
                    in = h1;
                }
                wstk[sp++] = c0;
                node = c1;
            }
            continue;
        }
        int first, count;
        leaf_range(node, first, count);
        if (COUNT && in) {
            ++cnt->leaves;
            cnt->tris += count;
        }
        visit_leaf(first, count);
        if (done()) return;
        if (sp == 0) return;
        node = uniform(wstk[--sp]);
        if (COUNT) in = (in_stack >> sp) & 1ull;
    }
}

// packet_walk with the box test specialised for the wave's direction signs
// when the live lanes share them (shadow rays towards one light, most
// primary-ray waves), the generic one otherwise (ambient-occlusion rays).
template <bool COUNT, bool WIDE, class Leaf, class Done>
__device__ __forceinline__ void walk(const float4* __restrict__ nodes, float3 id, float3 ood, const float& tmax,
                                     bool live, int* wstk, Leaf leaf, Done done, TravCount* cnt) {
    switch (wave_octant(id, live)) {
        case 0: packet_walk<COUNT, 0, WIDE>(nodes, id, ood, tmax, live, wstk, leaf, done, cnt); break;
        case 1: packet_walk<COUNT, 1, WIDE>(nodes, id, ood, tmax, live, wstk, leaf, done, cnt); break;
        case 2: packet_walk<COUNT, 2, WIDE>(nodes, id, ood, tmax, live, wstk, leaf, done, cnt); break;
        case 3: packet_walk<COUNT, 3, WIDE>(nodes, id, ood, tmax, live, wstk, leaf, done, cnt); break;
        case 4: packet_walk<COUNT, 4, WIDE>(nodes, id, ood, tmax, live, wstk, leaf, done, cnt); break;
        case 5: packet_walk<COUNT, 5, WIDE>(nodes, id, ood, tmax, live, wstk, leaf, done, cnt); break;
        case 6: packet_walk<COUNT, 6, WIDE>(nodes, id, ood, tmax, live, wstk, leaf, done, cnt); break;
        case 7: packet_walk<COUNT, 7, WIDE>(nodes, id, ood, tmax, live, wstk, leaf, done, cnt); break;
        default: packet_walk<COUNT, -1, WIDE>(nodes, id, ood, tmax, live, wstk, leaf, done, cnt); break;
    }
}

// Any hit at 0 < t < r.tmax for the lanes with `live`; the others return false.
template <bool COUNT, bool WIDE>
__device__ __forceinline__ bool any_hit(const float4* __restrict__ nodes, const float4* __restrict__ tris, const Ray& r,
                                        bool live, int* wstk, TravCount* cnt = nullptr) {
    const uint64_t lives = __ballot(live);
    if (lives == 0) return false;
    const float3 id = safe_inv(r.d);
    const float3 ood = f3(r.o.x * id.x, r.o.y * id.y, r.o.z * id.z);
    float tmax = live ? r.tmax : -1.0f;
    // Lanes whose ray has hit, as a wave mask on the scalar unit; a lane's
    // tmax drops to -1 (it leaves the walk) after the leaf of its hit, so
    // it may test that leaf's later triangles to no effect.  (One triangle
    // at a time: loading pairs here, as closest_hit does, measured slower on
    // the visibility rays.)
    uint64_t hits = 0;
    auto leaf = [&](int first, int count) {
        for (int k = 0; k < count; ++k)
            hits |= tri_hit_mask(load_tri_uniform<WIDE>(tris, first + k), r.o, r.d, tmax);  // not lanes with tmax < 0
        tmax = __builtin_amdgcn_inverse_ballot_w64(hits) ? -1.0f : tmax;
    };
    auto done = [&] { return (lives & ~hits) == 0; };
    walk<COUNT, WIDE>(nodes, id, ood, tmax, live, wstk, leaf, done, cnt);
    return __builtin_amdgcn_inverse_ballot_w64(hits);
}

// Closest hit at t > 0 (ties: lowest original triangle index) for the lanes
// with `live`; returns the position in leaf order, or -1.  COUNT: as for
// any_hit.
template <bool COUNT, bool WIDE>
__device__ __forceinline__ int closest_hit(const float4* __restrict__ nodes, const float4* __restrict__ tris, float3 o,
                                           float3 d, bool live, float& tbest, int* wstk, TravCount* cnt = nullptr) {
    const float3 id = safe_inv(d);
    const float3 ood = f3(o.x * id.x, o.y * id.y, o.z * id.z);
    int best = -1;
    uint32_t best_orig = 0xFFFFFFFFu;
    tbest = live ? __builtin_inff() : -1.0f;
    auto leaf = [&](int first, int count) {
        leaf_pairs<WIDE>(tris, first, count, [&](const TriRec& rec, int k) {
            const uint32_t orig = fbits(rec.v0.w);
            const float t = tri_t_rec(rec.v0, rec.e1, rec.e2, o, d);
            const bool take = (t > 0.0f) & (t <= tbest) & ((t < tbest) | (orig < best_orig));
            tbest = take ? t : tbest;
            best = take ? k : best;
            best_orig = take ? orig : best_orig;
        });
    };
    auto done = [] { return false; };
    walk<COUNT, WIDE>(nodes, id, ood, tbest, live, wstk, leaf, done, cnt);
    if (!live) tbest = __builtin_inff();
    return best;
}

// ---------------------------------------------------------------- two levels
// A top-level hierarchy over instances: its leaves index instance records of
// kInstStride float4 (world-to-object rows 0-2, object-to-world rows 3-5,
// (bottom level as bits, object id override bits (0xFFFFFFFF: keep the
// triangle's), first global triangle index as bits, 0), padding).  Bottom
// level 0 holds the base geometry, 1 the shared mesh.  Rays enter a bottom
// level transformed, direction not renormalised, so t is the same in both
// spaces.  The global index of a mesh triangle (ties of the closest hit) is
// the instance's first index plus its index in the mesh, as in the
// flattened scene.
struct TwoLevel {
    const float4* inst;
    const float4* nodes[2];
    const float4* tris[2];
};
constexpr int kInstStride = 8;
// (selects rather than indexes, so the description stays in registers)
__device__ __forceinline__ const float4* bottom_nodes(const TwoLevel& L, int b) { return b ? L.nodes[1] : L.nodes[0]; }
__device__ __forceinline__ const float4* bottom_tris(const TwoLevel& L, int b) { return b ? L.tris[1] : L.tris[0]; }

__device__ __forceinline__ float3 xf_point(float4 r0, float4 r1, float4 r2, float3 p) {
    return f3(fmaf(r0.x, p.x, fmaf(r0.y, p.y, fmaf(r0.z, p.z, r0.w))),
              fmaf(r1.x, p.x, fmaf(r1.y, p.y, fmaf(r1.z, p.z, r1.w))),
              fmaf(r2.x, p.x, fmaf(r2.y, p.y, fmaf(r2.z, p.z, r2.w))));
}
__device__ __forceinline__ float3 xf_dir(float4 r0, float4 r1, float4 r2, float3 v) {
    return f3(fmaf(r0.x, v.x, fmaf(r0.y, v.y, r0.z * v.z)), fmaf(r1.x, v.x, fmaf(r1.y, v.y, r1.z * v.z)),
              fmaf(r2.x, v.x, fmaf(r2.y, v.y, r2.z * v.z)));
}

// Walks bottom level b for the ray (o, d) in its space; `leaf(first, count)`
// as in packet_walk.  The live lanes are those with tmax >= 0.  Two-level
// walks address records wide, whatever the size of their arrays.
template <class Leaf, class Done>
__device__ __forceinline__ void walk_bottom(const float4* __restrict__ nodes, float3 o, float3 d, const float& tmax,
                                            int* wstk, Leaf leaf, Done done) {
    const float3 id = safe_inv(d);
    const float3 ood = f3(o.x * id.x, o.y * id.y, o.z * id.z);
    const bool live = tmax >= 0.0f;
    packet_walk<false, -1, true>(nodes, id, ood, tmax, live, wstk, leaf, done, nullptr);
}

// any_hit through a two-level hierarchy (`top` its top-level nodes); wstk2
// is the wave's stack for the bottom levels.
__device__ __forceinline__ bool any_hit_2l(const float4* __restrict__ top, const TwoLevel& L, const Ray& r, bool live,
                                           int* wstk, int* wstk2) {
    if (__ballot(live) == 0) return false;
    const float3 id = safe_inv(r.d);
    const float3 ood = f3(r.o.x * id.x, r.o.y * id.y, r.o.z * id.z);
    float tmax = live ? r.tmax : -1.0f;
    bool hit = false;
    auto done = [&] { return __ballot(tmax >= 0.0f) == 0; };
    auto top_leaf = [&](int first, int count) {
        for (int k = 0; k < count && !done(); ++k) {
            const float4* I = L.inst + kInstStride * (first + k);
            const float4 m0 = ld_const(I, 0), m1 = ld_const(I, 1), m2 = ld_const(I, 2);
            const int b = (int)fbits(ld_const(I, 6).x);
            const float3 o = xf_point(m0, m1, m2, r.o), d = xf_dir(m0, m1, m2, r.d);
            const float4* tb = bottom_tris(L, b);
            auto leaf = [&](int f, int c) {
                for (int j = 0; j < c; ++j)
                    if (tri_hits_uniform<true>(tb, f + j, o, d, tmax)) {  // false for finished lanes
                        hit = true;
                        tmax = -1.0f;
                    }
            };
            walk_bottom(bottom_nodes(L, b), o, d, tmax, wstk2, leaf, done);
        }
    };
    packet_walk<false, -1, true>(top, id, ood, tmax, live, wstk, top_leaf, done, nullptr);
    return hit;
}

// closest_hit through a two-level hierarchy: the instance and the triangle
// (position in its bottom level's leaf order) of the hit, or inst = -1.
__device__ __forceinline__ void closest_hit_2l(const float4* __restrict__ top, const TwoLevel& L, float3 o, float3 d,
                                               bool live, float& tbest, int& inst, int& tri, int* wstk, int* wstk2) {
    const float3 id = safe_inv(d);
    const float3 ood = f3(o.x * id.x, o.y * id.y, o.z * id.z);
    inst = -1;
    tri = -1;
    uint32_t best_glob = 0xFFFFFFFFu;
    tbest = live ? __builtin_inff() : -1.0f;
    auto done = [] { return false; };
    auto top_leaf = [&](int first, int count) {
        for (int k = 0; k < count; ++k) {
            const float4* I = L.inst + kInstStride * (first + k);
            const float4 m0 = ld_const(I, 0), m1 = ld_const(I, 1), m2 = ld_const(I, 2), info = ld_const(I, 6);
            const int b = (int)fbits(info.x);
            const uint32_t g0 = fbits(info.z);
            const float3 oo = xf_point(m0, m1, m2, o), dd = xf_dir(m0, m1, m2, d);
            const float4* tb = bottom_tris(L, b);
            auto leaf = [&](int f, int c) {
                for (int j = 0; j < c; ++j) {
                    uint32_t orig;
                    const float t = tri_t_uniform(tb, f + j, oo, dd, &orig);
                    const uint32_t g = g0 + orig;
                    if (t > 0.0f && t <= tbest && (t < tbest || g < best_glob)) {
                        tbest = t;
                        inst = first + k;
                        tri = f + j;
                        best_glob = g;
                    }
                }
            };
            walk_bottom(bottom_nodes(L, b), oo, dd, tbest, wstk2, leaf, done);
        }
    };
    packet_walk<false, -1, true>(top, id, ood, tbest, live, wstk, top_leaf, done, nullptr);
    if (!live) tbest = __builtin_inff();
}

}  // namespace dhr

#pragma clang fp contract(fast)
