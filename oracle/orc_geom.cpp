// Oracle (test infrastructure only): ray-triangle intersection, the oracle's
// own object-median BVH, and brute force over all triangles.
//
// The bounding-volume hierarchy is only an accelerator (Section 3.2 of the
// paper groups objects hierarchically so that a ray that misses a volume skips
// everything inside it); the plain definition of visibility is brute force:
// a ray is occluded iff some triangle is hit at 0 < t < tmax.  The BVH here is
// deliberately simple (split at the object median of the longest centroid
// axis) and is pinned against brute force by the test suite.
#include <omp.h>

#include <algorithm>

#include "orc.h"
#include "orc_common.h"

namespace orc {

double intersect(const Tri& tri, const V3& o, const V3& d) {
    const double nan = std::numeric_limits<double>::quiet_NaN();
    V3 e1 = tri.v1 - tri.v0;
    V3 e2 = tri.v2 - tri.v0;
    V3 p = cross(d, e2);
    double det = dot(e1, p);
    // A ray parallel to the triangle's plane does not hit it.  In FP64 a ray
    // lying in the plane yields |det| ~ 1e-17 of its scale and then u, v and t
    // are rounding noise, so "parallel" is |det| <= 1e-12 |e1| |e2| |d|.
    if (!(std::fabs(det) > 1e-12 * length(e1) * length(e2) * length(d))) return nan;
    double inv = 1.0 / det;
    V3 tv = o - tri.v0;
    double u = dot(tv, p) * inv;
    if (u < 0.0 || u > 1.0) return nan;
    V3 q = cross(tv, e1);
    double v = dot(d, q) * inv;
    if (v < 0.0 || u + v > 1.0) return nan;
    return dot(e2, q) * inv;
}

namespace {

void tri_bounds(const Tri& t, V3* lo, V3* hi) {
    lo->x = std::min({t.v0.x, t.v1.x, t.v2.x});
    lo->y = std::min({t.v0.y, t.v1.y, t.v2.y});
    lo->z = std::min({t.v0.z, t.v1.z, t.v2.z});
    hi->x = std::max({t.v0.x, t.v1.x, t.v2.x});
    hi->y = std::max({t.v0.y, t.v1.y, t.v2.y});
    hi->z = std::max({t.v0.z, t.v1.z, t.v2.z});
}

V3 centroid(const Tri& t) { return (t.v0 + t.v1 + t.v2) * (1.0 / 3.0); }

int64_t build(Scene& s, int64_t first, int64_t count, int depth) {
    int64_t id = (int64_t)s.nodes.size();
    s.nodes.push_back(Node{});
    s.depth = std::max(s.depth, depth);
    V3 lo{kInf, kInf, kInf}, hi{-kInf, -kInf, -kInf};
    V3 clo{kInf, kInf, kInf}, chi{-kInf, -kInf, -kInf};
    for (int64_t i = first; i < first + count; ++i) {
        V3 a, b;
        tri_bounds(s.tris[i], &a, &b);
        lo = V3{std::min(lo.x, a.x), std::min(lo.y, a.y), std::min(lo.z, a.z)};
        hi = V3{std::max(hi.x, b.x), std::max(hi.y, b.y), std::max(hi.z, b.z)};
        V3 c = centroid(s.tris[i]);
        clo = V3{std::min(clo.x, c.x), std::min(clo.y, c.y), std::min(clo.z, c.z)};
        chi = V3{std::max(chi.x, c.x), std::max(chi.y, c.y), std::max(chi.z, c.z)};
    }
    s.nodes[id].lo = lo;
    s.nodes[id].hi = hi;
    if (count <= 4) {
        s.nodes[id].first = first;
        s.nodes[id].count = count;
        return id;
    }
    V3 ext = chi - clo;
    int axis = (ext.x >= ext.y && ext.x >= ext.z) ? 0 : (ext.y >= ext.z ? 1 : 2);
    int64_t mid = first + count / 2;
    std::nth_element(s.tris.begin() + first, s.tris.begin() + mid, s.tris.begin() + first + count,
                     [axis](const Tri& a, const Tri& b) {
                         double ca = comp(centroid(a), axis), cb = comp(centroid(b), axis);
                         return ca < cb || (ca == cb && a.index < b.index);
                     });
    int64_t l = build(s, first, mid - first, depth + 1);
    int64_t r = build(s, mid, first + count - mid, depth + 1);
    s.nodes[id].left = l;
    s.nodes[id].right = r;
    return id;
}

// Conservative slab test of the segment [0, tmax]: boxes are padded so that
// rounding in the slab arithmetic can never reject a box holding a hit.
bool hit_box(const Node& nd, const V3& o, const V3& d, double tmax) {
    double t0 = 0.0, t1 = tmax;
    for (int k = 0; k < 3; ++k) {
        double lo = comp(nd.lo, k), hi = comp(nd.hi, k);
        double pad = 1e-9 * (1.0 + std::max(std::fabs(lo), std::fabs(hi)));
        lo -= pad;
        hi += pad;
        double ok = comp(o, k), dk = comp(d, k);
        if (dk == 0.0) {
            if (ok < lo || ok > hi) return false;
            continue;
        }
        double ta = (lo - ok) / dk, tb = (hi - ok) / dk;
        if (ta > tb) std::swap(ta, tb);
        t0 = std::max(t0, ta);
        t1 = std::min(t1, tb);
        if (t0 > t1) return false;
    }
    return true;
}

}  // namespace

bool anyhit_brute(const Scene& s, const V3& o, const V3& d, double tmax) {
    for (const Tri& t : s.original) {
        double th = intersect(t, o, d);
        if (th > 0.0 && th < tmax) return true;
    }
    return false;
}

bool anyhit_bvh(const Scene& s, const V3& o, const V3& d, double tmax) {
    if (s.nodes.empty()) return false;
    std::vector<int64_t> stack{0};
    while (!stack.empty()) {
        const Node& nd = s.nodes[stack.back()];
        stack.pop_back();
        if (!hit_box(nd, o, d, tmax)) continue;
        if (nd.count > 0) {
            for (int64_t i = nd.first; i < nd.first + nd.count; ++i) {
                double th = intersect(s.tris[i], o, d);
                if (th > 0.0 && th < tmax) return true;
            }
        } else {
            stack.push_back(nd.left);
            stack.push_back(nd.right);
        }
    }
    return false;
}

namespace {
void consider(const Tri& t, const V3& o, const V3& d, double* best, const Tri** bt) {
    double th = intersect(t, o, d);
    if (!(th > 0.0)) return;
    if (th < *best || (th == *best && *bt && t.index < (*bt)->index)) {
        *best = th;
        *bt = &t;
    }
}
}  // namespace

void closest_brute(const Scene& s, const V3& o, const V3& d, double* t, const Tri** tri) {
    double best = kInf;
    const Tri* bt = nullptr;
    for (const Tri& tr : s.original) consider(tr, o, d, &best, &bt);
    *t = best;
    *tri = bt;
}

void closest_bvh(const Scene& s, const V3& o, const V3& d, double* t, const Tri** tri) {
    double best = kInf;
    const Tri* bt = nullptr;
    if (!s.nodes.empty()) {
        std::vector<int64_t> stack{0};
        while (!stack.empty()) {
            const Node& nd = s.nodes[stack.back()];
            stack.pop_back();
            if (!hit_box(nd, o, d, best)) continue;
            if (nd.count > 0) {
                for (int64_t i = nd.first; i < nd.first + nd.count; ++i)
                    consider(s.tris[i], o, d, &best, &bt);
            } else {
                stack.push_back(nd.left);
                stack.push_back(nd.right);
            }
        }
    }
    *t = best;
    *tri = bt;
}

}  // namespace orc

extern "C" {

orc_scene* orc_scene_create(const float* tris, const uint32_t* obj_id, int64_t T) {
    orc_scene* sc = new orc_scene;
    orc::Scene& s = sc->s;
    s.tris.resize(T);
    for (int64_t i = 0; i < T; ++i) {
        const float* p = tris + 9 * i;
        orc::Tri& t = s.tris[i];
        t.v0 = orc::V3{p[0], p[1], p[2]};
        t.v1 = orc::V3{p[3], p[4], p[5]};
        t.v2 = orc::V3{p[6], p[7], p[8]};
        t.obj = obj_id ? obj_id[i] : (uint32_t)i;
        t.index = i;
    }
    s.original = s.tris;
    if (T > 0) orc::build(s, 0, T, 0);
    return sc;
}

void orc_scene_destroy(orc_scene* s) { delete s; }

int orc_scene_depth(const orc_scene* s) { return s->s.depth; }

void orc_anyhit(const orc_scene* sc, const double* o, const double* d, const double* tmax,
                int64_t n, uint8_t* hit_bvh, uint8_t* hit_brute) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        orc::V3 oo{o[3 * i], o[3 * i + 1], o[3 * i + 2]};
        orc::V3 dd{d[3 * i], d[3 * i + 1], d[3 * i + 2]};
        if (hit_bvh) hit_bvh[i] = orc::anyhit_bvh(sc->s, oo, dd, tmax[i]);
        if (hit_brute) hit_brute[i] = orc::anyhit_brute(sc->s, oo, dd, tmax[i]);
    }
}

void orc_closest(const orc_scene* sc, const double* o, const double* d, int64_t n, double* t,
                 int64_t* tri, int use_brute) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        orc::V3 oo{o[3 * i], o[3 * i + 1], o[3 * i + 2]};
        orc::V3 dd{d[3 * i], d[3 * i + 1], d[3 * i + 2]};
        const orc::Tri* bt;
        if (use_brute)
            orc::closest_brute(sc->s, oo, dd, &t[i], &bt);
        else
            orc::closest_bvh(sc->s, oo, dd, &t[i], &bt);
        tri[i] = bt ? bt->index : -1;
    }
}

int orc_num_threads(void) { return omp_get_max_threads(); }

void orc_set_num_threads(int n) { omp_set_num_threads(n); }

}  // extern "C"
