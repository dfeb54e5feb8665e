// Oracle-internal helpers (test infrastructure only): FP64 vectors, the
// oracle's own BVH and the shared declarations between its source files.
#ifndef ORC_COMMON_H
#define ORC_COMMON_H
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

namespace orc {

struct V3 {
    double x, y, z;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double length(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 normalize(V3 a) { return a * (1.0 / length(a)); }
inline double comp(V3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

const double kInf = std::numeric_limits<double>::infinity();

// ---- rng / samplers (orc_rng.cpp) ----
void philox(uint32_t k0, uint32_t k1, const uint32_t ctr[4], uint32_t out[4]);
void ray_uniforms(uint32_t seed, uint32_t client, uint32_t x, uint32_t y, uint32_t frame,
                  uint32_t stream, uint32_t sample, double* u0, double* u1);
void onb(const V3& n, V3* b1, V3* b2);
V3 sample_cosine(const V3& n, double u0, double u1);
V3 sample_cone(const V3& axis, double k, double u0, double u1);

// ---- scene and BVH (orc_geom.cpp) ----
struct Tri {
    V3 v0, v1, v2;
    uint32_t obj;
    int64_t index;   // original index
};

struct Node {
    V3 lo, hi;
    int64_t left = -1, right = -1;   // children (internal)
    int64_t first = 0, count = 0;    // triangle range (leaf when count > 0)
};

struct Scene {
    std::vector<Tri> tris;           // in BVH order
    std::vector<Tri> original;       // in input order (brute force)
    std::vector<Node> nodes;
    int depth = 0;
};

// Moller-Trumbore (1997): hit distance t of the ray o + t d with the
// two-sided triangle, or NaN when the ray is parallel to its plane or the hit
// point lies outside the triangle (edges inclusive).  t may be <= 0.
double intersect(const Tri& tri, const V3& o, const V3& d);
bool anyhit_bvh(const Scene& s, const V3& o, const V3& d, double tmax);
bool anyhit_brute(const Scene& s, const V3& o, const V3& d, double tmax);
// closest hit with t > 0, ties broken by the smallest original index
void closest_bvh(const Scene& s, const V3& o, const V3& d, double* t, const Tri** tri);
void closest_brute(const Scene& s, const V3& o, const V3& d, double* t, const Tri** tri);

}  // namespace orc

struct orc_scene {
    orc::Scene s;
};

#endif
