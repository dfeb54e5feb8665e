// Oracle-internal (test infrastructure only): edge-stopping weights of the
// spatial filter, written once as templates over the scalar type so that the
// same definitions serve FP64 evaluation and forward-mode dual numbers.
//
// Paper, Section 3.3: the filter weights neighbours by differences in depth
// and surface normal (the modification for ambient occlusion) and iterates
// the spatial kernel, each pass refining the previous one.  The kernel shape
// (5x5 B3 spline at stride 2^level), the 3x3 variance prefilter and the
// luminance-like stopping term on the AO value follow SVGF (Schied et al.
// 2017, reference [23] of the paper).
#ifndef ORC_FILTER_H
#define ORC_FILTER_H
#include <cmath>

#include "orc.h"

namespace orc {

// 1-D taps of the B3 spline: (1, 4, 6, 4, 1) / 16; prefilter: (1, 2, 1) / 4.
const double kH1[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
const double kK1[3] = {0.25, 0.5, 0.25};

// The a-trous kernel: radius 2 with B3 taps (kernel_width 5), or radius 1
// with (1, 2, 1) / 4 taps (kernel_width 3: the lighter variant, one smaller
// kernel, that Section 3.3 anticipates).
inline int kernel_radius(const orc_svgf_params& P) { return P.kernel_width == 3 ? 1 : 2; }
inline double kernel_tap(int R, int a) { return R == 2 ? kH1[a + 2] : kK1[a + 1]; }

// ---- forward-mode dual numbers (value, tangent) ----
struct Dual {
    double v, d;
    Dual() : v(0), d(0) {}
    Dual(double a) : v(a), d(0) {}
    Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual dexp(Dual a) { double e = std::exp(a.v); return {e, e * a.d}; }
inline Dual dsqrt(Dual a) { double s = std::sqrt(a.v); return {s, s > 0.0 ? a.d / (2.0 * s) : 0.0}; }
// |a| with derivative sign(a), sign(0) = 0
inline Dual dabs(Dual a) { return a.v > 0.0 ? a : (a.v < 0.0 ? -a : Dual(0.0, 0.0)); }
inline double val(Dual a) { return a.v; }

inline double dexp(double a) { return std::exp(a); }
inline double dsqrt(double a) { return std::sqrt(a); }
inline double dabs(double a) { return std::fabs(a); }
inline double val(double a) { return a; }

// depth stopping: exp(-|z_p - z_q| / (sigma_z |s (a dzx + b dzy)| + eps_z z_p))
template <class T>
T weight_z(double zp, double zq, double dzx, double dzy, int a, int b, int s, T sigma_z,
           double eps_z_rel) {
    double S = std::fabs((double)s * ((double)a * dzx + (double)b * dzy));
    T F = sigma_z * T(S) + T(eps_z_rel * zp);
    return dexp(-(T(std::fabs(zp - zq)) / F));
}

// normal stopping: max(0, min(1, n_p . n_q)) ^ sigma_n, zero when the dot is <= 0
template <class T>
T weight_n(const float* np, const float* nq, T sigma_n) {
    double x = (double)np[0] * nq[0] + (double)np[1] * nq[1] + (double)np[2] * nq[2];
    if (x > 1.0) x = 1.0;
    if (!(x > 0.0)) return T(0.0);
    return dexp(sigma_n * T(std::log(x)));
}

// AO-value stopping: exp(-|c_p - c_q| / (sigma_l g + eps_l))
template <class T>
T weight_l(T cp, T cq, T g, T sigma_l, double eps_l) {
    return dexp(-(dabs(cp - cq) / (sigma_l * g + T(eps_l))));
}

inline bool valid_px(const float* nz, int64_t i) { return nz[4 * i + 3] > 0.0f; }

// One a-trous level (stride 2^level) over a whole image.  cv: [HW][2] (c, var).
template <class T>
void atrous_level(const orc_svgf_params& P, int W, int H, int level, const T* cv, const float* nz,
                  const float* dz, T sz, T sn, T sl, T* out) {
    const int s = 1 << level;
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const int64_t p = (int64_t)y * W + x;
            if (!valid_px(nz, p)) {
                out[2 * p] = T(1.0);
                out[2 * p + 1] = T(0.0);
                continue;
            }
            // 3x3 Gaussian prefilter of the variance for the stopping term
            T G(0.0);
            double sk = 0.0;
            for (int b = -1; b <= 1; ++b)
                for (int a = -1; a <= 1; ++a) {
                    int qx = x + a, qy = y + b;
                    if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
                    int64_t q = (int64_t)qy * W + qx;
                    if (!valid_px(nz, q)) continue;
                    double k = kK1[a + 1] * kK1[b + 1];
                    G += T(k) * cv[2 * q + 1];
                    sk += k;
                }
            T g = dsqrt(G / T(sk));
            T cp = cv[2 * p];
            T D(0.0), Sc(0.0), Sv(0.0);
            const int R = kernel_radius(P);
            for (int b = -R; b <= R; ++b)
                for (int a = -R; a <= R; ++a) {
                    int qx = x + s * a, qy = y + s * b;
                    if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
                    int64_t q = (int64_t)qy * W + qx;
                    if (!valid_px(nz, q)) continue;
                    double h = kernel_tap(R, a) * kernel_tap(R, b);
                    T w(1.0);
                    if (a != 0 || b != 0) {
                        w = weight_z(nz[4 * p + 3], nz[4 * q + 3], dz[2 * p], dz[2 * p + 1], a, b, s, sz, P.eps_z_rel) *
                            weight_n(nz + 4 * p, nz + 4 * q, sn) * weight_l(cp, cv[2 * q], g, sl, P.eps_l);
                    }
                    T hw = T(h) * w;
                    D += hw;
                    Sc += hw * cv[2 * q];
                    Sv += hw * hw * cv[2 * q + 1];
                }
            out[2 * p] = Sc / D;
            out[2 * p + 1] = Sv / (D * D);
        }
    }
}

}  // namespace orc
#endif
