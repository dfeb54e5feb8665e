// Oracle (test infrastructure only): the modified SVGF forward pass.
//
// Paper, Section 3.3:
//  * temporal: an exponential moving average accumulates samples over frames;
//  * motion vectors back-project the pixel into the previous frame, and
//    history samples inconsistent in depth, normal or mesh id are discarded;
//  * without usable history the variance comes from a larger spatial kernel
//    until enough history has accumulated;
//  * the variance drives the weights of an iterated spatial kernel;
//  * for ambient occlusion the weights use depth and normal differences.
// Constants, kernel shapes and the ordering of steps the paper leaves open
// follow SVGF (reference [23] of the paper); each such reading is listed in
// the design notes of the repository.
#include <algorithm>
#include <vector>

#include "orc.h"
#include "orc_common.h"
#include "orc_filter.h"

namespace {

uint32_t bits_of(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}

// Consistency of one history tap, decided in fp32 with a fixed operation
// order (the decision is discrete, so both implementations must take it in
// the same precision): normal agreement and distance of the previous world
// position from the current pixel's tangent plane, in pixel footprints.
bool tap_consistent(const orc_svgf_params& P, const float* n, const float* p, float z, const float* m,
                    const float* pp, float pix) {
    float dn = fmaf(n[0], m[0], fmaf(n[1], m[1], n[2] * m[2]));
    if (!(dn >= P.cos_normal_min)) return false;
    float dx = pp[0] - p[0];
    float dy = pp[1] - p[1];
    float dzz = pp[2] - p[2];
    float dpl = fabsf(fmaf(n[0], dx, fmaf(n[1], dy, n[2] * dzz)));
    float thr = (P.plane_px * pix) * z;
    return dpl <= thr;
}

template <class T>
void spatial_stack(const orc_svgf_params& P, int W, int H, const T* cv_in, const float* nz, const float* dz,
                   const T* sig /* [3][8] z,n,l */, T* out, T* save) {
    const int64_t HW = (int64_t)W * H;
    std::vector<T> a(cv_in, cv_in + 2 * HW), b(2 * HW);
    for (int l = 0; l < P.levels; ++l) {
        if (save) std::copy(a.begin(), a.end(), save + (int64_t)l * 2 * HW);
        orc::atrous_level<T>(P, W, H, l, a.data(), nz, dz, sig[l], sig[8 + l], sig[16 + l], b.data());
        std::swap(a, b);
    }
    for (int64_t i = 0; i < HW; ++i) out[i] = orc::valid_px(nz, i) ? a[2 * i] : T(1.0);
}

}  // namespace

extern "C" {

void orc_svgf_temporal(const orc_svgf_params* P, int W, int H, int n_ao, const uint8_t* ao_count,
                       const float* pos, const float* nz, const float* mv, const float* prev_pos,
                       const float* prev_nz, const float* hist_in, float pix, double* hist_out) {
    const bool have_hist = hist_in && prev_pos && prev_nz;
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const int64_t i = (int64_t)y * W + x;
            double* ho = hist_out + 4 * i;
            if (!orc::valid_px(nz, i)) {
                ho[0] = ho[1] = ho[2] = 1.0;
                ho[3] = 0.0;
                continue;
            }
            const double xs = (double)ao_count[i] / (double)n_ao;
            bool any = false;
            double wsum = 0.0, c = 0.0, m1 = 0.0, m2 = 0.0, hmax = 0.0;
            const float mvx = mv[2 * i], mvy = mv[2 * i + 1];
            if (have_hist && std::isfinite(mvx) && std::isfinite(mvy)) {
                // bilinear taps around the back-projected position.  The
                // fraction is rounded to fp32 (the motion vector's own
                // precision) and a tap takes part iff its bilinear factor is
                // nonzero: tap 0 iff f < 1, tap 1 iff f > 0.
                const double flx = std::floor((double)mvx), fly = std::floor((double)mvy);
                const double fx = (double)(float)((double)mvx - flx), fy = (double)(float)((double)mvy - fly);
                const double X0 = x + flx, Y0 = y + fly;
                for (int j = 0; j < 2; ++j)
                    for (int k = 0; k < 2; ++k) {
                        if ((k == 1 && !(fx > 0.0)) || (k == 0 && !(fx < 1.0))) continue;
                        if ((j == 1 && !(fy > 0.0)) || (j == 0 && !(fy < 1.0))) continue;
                        const double tx = X0 + k, ty = Y0 + j;
                        if (tx < 0.0 || tx >= W || ty < 0.0 || ty >= H) continue;
                        const int64_t q = (int64_t)ty * W + (int64_t)tx;
                        if (!orc::valid_px(prev_nz, q)) continue;
                        if (!(hist_in[4 * q + 3] > 0.0f)) continue;
                        if (P->use_obj_id && bits_of(prev_pos[4 * q + 3]) != bits_of(pos[4 * i + 3])) continue;
                        if (!tap_consistent(*P, nz + 4 * i, pos + 4 * i, nz[4 * i + 3], prev_nz + 4 * q,
                                            prev_pos + 4 * q, pix))
                            continue;
                        const double b = (k ? fx : 1.0 - fx) * (j ? fy : 1.0 - fy);
                        any = true;
                        wsum += b;
                        c += b * hist_in[4 * q];
                        m1 += b * hist_in[4 * q + 1];
                        m2 += b * hist_in[4 * q + 2];
                        hmax = std::max(hmax, (double)hist_in[4 * q + 3]);
                    }
            }
            if (any) {
                c /= wsum;
                m1 /= wsum;
                m2 /= wsum;
                const double h = std::min(hmax + 1.0, P->history_cap);
                const double a = std::max(P->alpha, 1.0 / h);
                const double am = std::max(P->alpha_moments, 1.0 / h);
                ho[0] = c + a * (xs - c);
                ho[1] = m1 + am * (xs - m1);
                ho[2] = m2 + am * (xs * xs - m2);
                ho[3] = h;
            } else {
                ho[0] = xs;
                ho[1] = xs;
                ho[2] = xs * xs;
                ho[3] = 1.0;
            }
            // the history buffer holds fp32: the step's result is stored once,
            // rounded to fp32, and everything downstream reads the stored value
            for (int k = 0; k < 4; ++k) ho[k] = (double)(float)ho[k];
        }
    }
}

void orc_svgf_variance(const orc_svgf_params* P, int W, int H, const double* hist, const float* nz,
                       const float* dz, double* cv) {
    const int R = P->fallback_radius;
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const int64_t p = (int64_t)y * W + x;
            if (!orc::valid_px(nz, p)) {
                cv[2 * p] = 1.0;
                cv[2 * p + 1] = 0.0;
                continue;
            }
            const double* hp = hist + 4 * p;
            double var;
            if (hp[3] >= P->var_min_history) {
                var = std::max(0.0, hp[2] - hp[1] * hp[1]);
            } else {
                // spatial estimate from neighbours' moments, depth/normal weights
                double sw = 0.0, s1 = 0.0, s2 = 0.0;
                for (int b = -R; b <= R; ++b)
                    for (int a = -R; a <= R; ++a) {
                        int qx = x + a, qy = y + b;
                        if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
                        int64_t q = (int64_t)qy * W + qx;
                        if (!orc::valid_px(nz, q)) continue;
                        double w = 1.0;
                        if (a != 0 || b != 0)
                            w = orc::weight_z<double>(nz[4 * p + 3], nz[4 * q + 3], dz[2 * p], dz[2 * p + 1], a, b, 1,
                                                      P->sigma_z[0], P->eps_z_rel) *
                                orc::weight_n<double>(nz + 4 * p, nz + 4 * q, P->sigma_n[0]);
                        const double* hq = hist + 4 * q;
                        sw += w;
                        s1 += w * hq[1];
                        s2 += w * (hq[2] - hq[1] * hq[1]);
                    }
                const double mbar = s1 / sw;
                double s3 = 0.0;
                for (int b = -R; b <= R; ++b)
                    for (int a = -R; a <= R; ++a) {
                        int qx = x + a, qy = y + b;
                        if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
                        int64_t q = (int64_t)qy * W + qx;
                        if (!orc::valid_px(nz, q)) continue;
                        double w = 1.0;
                        if (a != 0 || b != 0)
                            w = orc::weight_z<double>(nz[4 * p + 3], nz[4 * q + 3], dz[2 * p], dz[2 * p + 1], a, b, 1,
                                                      P->sigma_z[0], P->eps_z_rel) *
                                orc::weight_n<double>(nz + 4 * p, nz + 4 * q, P->sigma_n[0]);
                        const double d = hist[4 * q + 1] - mbar;
                        s3 += w * d * d;
                    }
                var = std::max(0.0, s2 / sw + s3 / sw);
            }
            cv[2 * p] = hp[0];
            cv[2 * p + 1] = var;
        }
    }
}

void orc_svgf_atrous(const orc_svgf_params* P, int W, int H, int level, const double* cv_in,
                     const float* nz, const float* dz, double* cv_out) {
    orc::atrous_level<double>(*P, W, H, level, cv_in, nz, dz, P->sigma_z[level], P->sigma_n[level],
                              P->sigma_l[level], cv_out);
}

void orc_svgf_filter(const orc_svgf_params* P, int W, int H, int n_ao, const uint8_t* ao_count,
                     const float* pos, const float* nz, const float* dz, const float* mv, const float* prev_pos,
                     const float* prev_nz, const float* hist_in, float pix, double* hist_out, double* out,
                     double* cv0, double* save) {
    const int64_t HW = (int64_t)W * H;
    orc_svgf_temporal(P, W, H, n_ao, ao_count, pos, nz, mv, prev_pos, prev_nz, hist_in, pix, hist_out);
    std::vector<double> a(2 * HW), b(2 * HW);
    orc_svgf_variance(P, W, H, hist_out, nz, dz, a.data());
    if (cv0) std::copy(a.begin(), a.end(), cv0);
    for (int l = 0; l < P->levels; ++l) {
        if (save) std::copy(a.begin(), a.end(), save + (int64_t)l * 2 * HW);
        orc_svgf_atrous(P, W, H, l, a.data(), nz, dz, b.data());
        std::swap(a, b);
        if (l == P->feedback_level)
            for (int64_t i = 0; i < HW; ++i)
                if (orc::valid_px(nz, i)) hist_out[4 * i] = (double)(float)a[2 * i];
    }
    for (int64_t i = 0; i < HW; ++i) out[i] = orc::valid_px(nz, i) ? a[2 * i] : 1.0;
}

void orc_svgf_spatial(const orc_svgf_params* P, int W, int H, const double* cv_in, const float* nz,
                      const float* dz, double* out, double* save) {
    double sig[24] = {0};
    for (int l = 0; l < 8; ++l) {
        sig[l] = P->sigma_z[l];
        sig[8 + l] = P->sigma_n[l];
        sig[16 + l] = P->sigma_l[l];
    }
    spatial_stack<double>(*P, W, H, cv_in, nz, dz, sig, out, save);
}

void orc_svgf_spatial_jvp(const orc_svgf_params* P, int W, int H, const double* cv_in, const float* nz,
                          const float* dz, const double* dcv, const double* dsigma, double* dout) {
    const int64_t HW = (int64_t)W * H;
    const int L = P->levels;
    std::vector<orc::Dual> cv(2 * HW), out(HW);
    for (int64_t i = 0; i < 2 * HW; ++i) cv[i] = orc::Dual(cv_in[i], dcv[i]);
    orc::Dual sig[24];
    for (int l = 0; l < 8; ++l) {
        sig[l] = orc::Dual(P->sigma_z[l], l < L ? dsigma[l] : 0.0);
        sig[8 + l] = orc::Dual(P->sigma_n[l], l < L ? dsigma[L + l] : 0.0);
        sig[16 + l] = orc::Dual(P->sigma_l[l], l < L ? dsigma[2 * L + l] : 0.0);
    }
    spatial_stack<orc::Dual>(*P, W, H, cv.data(), nz, dz, sig, out.data(), nullptr);
    for (int64_t i = 0; i < HW; ++i) dout[i] = out[i].d;
}

}  // extern "C"
