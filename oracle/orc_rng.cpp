// Oracle (test infrastructure only): counter-based RNG and direction samplers.
//
// Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw, "Parallel
// random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of a multiply-based
// S-box over a 4x32-bit counter under a 2x32-bit key, with the key bumped by
// Weyl-sequence constants between rounds.  The paper under test only says that
// directions are "random" (Section 3.1) and that AO rays are drawn at random
// (Section 3.3); the counter layout (x, y, frame, stream<<16 | sample) and the
// key (seed, client) are this implementation's reading.
#include "orc.h"
#include "orc_common.h"

namespace {

// Multipliers and Weyl key increments of Philox4x32 (SC'11, Section 4).
const uint32_t kM0 = 0xD2511F53u;
const uint32_t kM1 = 0xCD9E8D57u;
const uint32_t kW0 = 0x9E3779B9u;   // golden ratio
const uint32_t kW1 = 0xBB67AE85u;   // sqrt(3) - 1

void philox_round(uint32_t c[4], const uint32_t k[2]) {
    uint64_t p0 = (uint64_t)kM0 * c[0];
    uint64_t p1 = (uint64_t)kM1 * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

}  // namespace

namespace orc {

void philox(uint32_t k0, uint32_t k1, const uint32_t ctr[4], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {k0, k1};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k[0] += kW0; k[1] += kW1; }
        philox_round(c, k);
    }
    for (int i = 0; i < 4; ++i) out[i] = c[i];
}

// Two uniforms in [0,1) from one Philox block: the top 24 bits of words 0 and
// 1, scaled by 2^-24 (exact in fp32 and FP64).
void ray_uniforms(uint32_t seed, uint32_t client, uint32_t x, uint32_t y, uint32_t frame,
                  uint32_t stream, uint32_t sample, double* u0, double* u1) {
    uint32_t ctr[4] = {x, y, frame, (stream << 16) | sample};
    uint32_t r[4];
    philox(seed, client, ctr, r);
    *u0 = (double)(r[0] >> 8) * 0x1p-24;
    *u1 = (double)(r[1] >> 8) * 0x1p-24;
}

// Orthonormal basis around a unit vector n: the revised Frisvad construction
// (Duff, Burgess, Christensen, Hery, Kensler, Liani, Villemin, JCGT 2017).
void onb(const V3& n, V3* b1, V3* b2) {
    double s = std::copysign(1.0, n.z);
    double a = -1.0 / (s + n.z);
    double b = n.x * n.y * a;
    *b1 = V3{1.0 + s * n.x * n.x * a, s * b, -s * n.x};
    *b2 = V3{b, s + n.y * n.y * a, -n.y};
}

// Cosine-weighted hemisphere about n by Malley's method: a uniform point of
// the unit disk lifted onto the hemisphere.
V3 sample_cosine(const V3& n, double u0, double u1) {
    double rho = std::sqrt(u0);
    double phi = 2.0 * M_PI * u1;
    double lx = rho * std::cos(phi), ly = rho * std::sin(phi), lz = std::sqrt(1.0 - u0);
    V3 b1, b2;
    onb(n, &b1, &b2);
    return b1 * lx + b2 * ly + n * lz;
}

// Uniform in solid angle inside the cone about `axis` with 1 - cos(theta_max)
// = k: cos(theta) = 1 - u0 k, written with s = u0 k so that sin(theta) =
// sqrt(s (2 - s)) stays accurate for narrow cones.
V3 sample_cone(const V3& axis, double k, double u0, double u1) {
    double s = u0 * k;
    double ct = 1.0 - s;
    double st = std::sqrt(s * (2.0 - s));
    double phi = 2.0 * M_PI * u1;
    V3 b1, b2;
    onb(axis, &b1, &b2);
    return b1 * (st * std::cos(phi)) + b2 * (st * std::sin(phi)) + axis * ct;
}

}  // namespace orc

extern "C" {

void orc_philox4x32_10(uint32_t k0, uint32_t k1, const uint32_t* ctr, uint32_t* out, int64_t n) {
    for (int64_t i = 0; i < n; ++i) orc::philox(k0, k1, ctr + 4 * i, out + 4 * i);
}

void orc_sample_cosine(const double* n, const double* u, double* out, int64_t count) {
    for (int64_t i = 0; i < count; ++i) {
        orc::V3 nn = orc::normalize(orc::V3{n[3 * i], n[3 * i + 1], n[3 * i + 2]});
        orc::V3 d = orc::sample_cosine(nn, u[2 * i], u[2 * i + 1]);
        out[3 * i] = d.x; out[3 * i + 1] = d.y; out[3 * i + 2] = d.z;
    }
}

void orc_sample_cone(const double* axis, double k, const double* u, double* out, int64_t count) {
    orc::V3 a = orc::normalize(orc::V3{axis[0], axis[1], axis[2]});
    for (int64_t i = 0; i < count; ++i) {
        orc::V3 d = orc::sample_cone(a, k, u[2 * i], u[2 * i + 1]);
        out[3 * i] = d.x; out[3 * i + 1] = d.y; out[3 * i + 2] = d.z;
    }
}

}  // extern "C"
