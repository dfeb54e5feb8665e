// Oracle (test infrastructure only): vector-Jacobian product of the spatial
// filter stack (the a-trous levels with their variance prefilter) with respect
// to the input AO value c, the input variance v and the per-level
// edge-stopping parameters sigma_z, sigma_n, sigma_l.
//
// Written in scatter form straight from the chain rule of one level
//     c'_p = sum_q h w_pq c_q / D_p,   v'_p = sum_q h^2 w_pq^2 v_q / D_p^2,
//     D_p  = sum_q h w_pq,             w_pq = w_z w_n w_l (centre tap w = 1),
//     w_l  = exp(-|c_p - c_q| / (sigma_l g_p + eps_l)),  g_p = sqrt(prefilter(v)_p),
// walking the levels in reverse and scattering every partial derivative to
// the pixel it belongs to.  Kinks take the subgradient 0 (sign(0) = 0, the
// square root at 0, ln of a zero weight).  Serial and FP64.
#include <algorithm>
#include <vector>

#include "orc.h"
#include "orc_common.h"
#include "orc_filter.h"

extern "C" {

void orc_svgf_spatial_vjp(const orc_svgf_params* P, int W, int H, const double* cv_in, const float* nz,
                          const float* dz, const double* grad_out, double* grad_cv, double* grad_sigma) {
    using orc::kK1;
    const int R = orc::kernel_radius(*P), KW = 2 * R + 1;
    const int64_t HW = (int64_t)W * H;
    const int L = P->levels;
    // forward, keeping every level's input
    std::vector<std::vector<double>> lv(L + 1, std::vector<double>(2 * HW));
    std::copy(cv_in, cv_in + 2 * HW, lv[0].begin());
    for (int l = 0; l < L; ++l)
        orc_svgf_atrous(P, W, H, l, lv[l].data(), nz, dz, lv[l + 1].data());

    std::vector<double> abar(HW, 0.0), bbar(HW, 0.0);   // d loss / d (c', v') of the current level
    for (int64_t i = 0; i < HW; ++i) abar[i] = orc::valid_px(nz, i) ? grad_out[i] : 0.0;
    for (int k = 0; k < 3 * L; ++k) grad_sigma[k] = 0.0;

    for (int l = L - 1; l >= 0; --l) {
        const int s = 1 << l;
        const double sz = P->sigma_z[l], sn = P->sigma_n[l], sl = P->sigma_l[l];
        const std::vector<double>& cv = lv[l];
        std::vector<double> cbar(HW, 0.0), vbar(HW, 0.0);
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                const int64_t p = (int64_t)y * W + x;
                if (!orc::valid_px(nz, p)) continue;
                const double ab = abar[p], bb = bbar[p];
                // prefilter
                double G = 0.0, sk = 0.0;
                for (int b = -1; b <= 1; ++b)
                    for (int a = -1; a <= 1; ++a) {
                        int qx = x + a, qy = y + b;
                        if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
                        int64_t q = (int64_t)qy * W + qx;
                        if (!orc::valid_px(nz, q)) continue;
                        G += kK1[a + 1] * kK1[b + 1] * cv[2 * q + 1];
                        sk += kK1[a + 1] * kK1[b + 1];
                    }
                const double g = std::sqrt(G / sk);
                const double E = sl * g + P->eps_l;
                const double cp = cv[2 * p];
                // weights and normaliser
                double D = 0.0, Sc = 0.0, Sv = 0.0;
                double wt[25];
                for (int b = -R; b <= R; ++b)
                    for (int a = -R; a <= R; ++a) {
                        int t = (b + R) * KW + (a + R);
                        wt[t] = -1.0;
                        int qx = x + s * a, qy = y + s * b;
                        if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
                        int64_t q = (int64_t)qy * W + qx;
                        if (!orc::valid_px(nz, q)) continue;
                        double w = 1.0;
                        if (a != 0 || b != 0)
                            w = orc::weight_z<double>(nz[4 * p + 3], nz[4 * q + 3], dz[2 * p], dz[2 * p + 1], a, b, s,
                                                      sz, P->eps_z_rel) *
                                orc::weight_n<double>(nz + 4 * p, nz + 4 * q, sn) *
                                orc::weight_l<double>(cp, cv[2 * q], g, sl, P->eps_l);
                        wt[t] = w;
                        double h = orc::kernel_tap(R, a) * orc::kernel_tap(R, b);
                        D += h * w;
                        Sc += h * w * cv[2 * q];
                        Sv += h * h * w * w * cv[2 * q + 1];
                    }
                const double cpr = Sc / D, vpr = Sv / (D * D);
                double gbar = 0.0;
                for (int b = -R; b <= R; ++b)
                    for (int a = -R; a <= R; ++a) {
                        int t = (b + R) * KW + (a + R);
                        const double w = wt[t];
                        if (w < 0.0) continue;
                        int64_t q = (int64_t)(y + s * b) * W + (x + s * a);
                        const double h = orc::kernel_tap(R, a) * orc::kernel_tap(R, b);
                        const double cq = cv[2 * q], vq = cv[2 * q + 1];
                        // direct dependence of c' on c_q and of v' on v_q
                        cbar[q] += ab * h * w / D;
                        vbar[q] += bb * h * h * w * w / (D * D);
                        if (a == 0 && b == 0) continue;   // centre weight is the constant 1
                        // adjoint of the weight w_pq
                        const double wbar = ab * h * (cq - cpr) / D + bb * (2.0 * h * h * w * vq / (D * D) - 2.0 * vpr * h / D);
                        // AO-value term w_l
                        const double dc = cp - cq;
                        const double sg = dc > 0.0 ? 1.0 : (dc < 0.0 ? -1.0 : 0.0);
                        cbar[p] += -wbar * w * sg / E;
                        cbar[q] += wbar * w * sg / E;
                        gbar += wbar * w * std::fabs(dc) * sl / (E * E);
                        grad_sigma[2 * L + l] += wbar * w * std::fabs(dc) * g / (E * E);
                        // depth term w_z
                        const double Sd = std::fabs((double)s * ((double)a * dz[2 * p] + (double)b * dz[2 * p + 1]));
                        const double F = sz * Sd + P->eps_z_rel * nz[4 * p + 3];
                        grad_sigma[l] += wbar * w * std::fabs((double)nz[4 * p + 3] - (double)nz[4 * q + 3]) * Sd / (F * F);
                        // normal term w_n
                        double xn = (double)nz[4 * p] * nz[4 * q] + (double)nz[4 * p + 1] * nz[4 * q + 1] +
                                    (double)nz[4 * p + 2] * nz[4 * q + 2];
                        if (xn > 1.0) xn = 1.0;
                        if (w > 0.0 && xn > 0.0) grad_sigma[L + l] += wbar * w * std::log(xn);
                    }
                // prefilter: g = sqrt(G), G = sum_r K_r v_r / sum_r K_r
                if (g > 0.0) {
                    const double Gbar = gbar / (2.0 * g);
                    for (int b = -1; b <= 1; ++b)
                        for (int a = -1; a <= 1; ++a) {
                            int qx = x + a, qy = y + b;
                            if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
                            int64_t q = (int64_t)qy * W + qx;
                            if (!orc::valid_px(nz, q)) continue;
                            vbar[q] += Gbar * kK1[a + 1] * kK1[b + 1] / sk;
                        }
                }
            }
        abar.swap(cbar);
        bbar.swap(vbar);
    }
    for (int64_t i = 0; i < HW; ++i) {
        grad_cv[2 * i] = abar[i];
        grad_cv[2 * i + 1] = bbar[i];
    }
}

}  // extern "C"
