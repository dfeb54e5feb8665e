// Wire form of a served frame (oracle): the AO a client receives is one byte
// per pixel (Section 3.2: N_unoccluded fits 8 bits), and the per-light
// visibility is a bitmask (Section 3.1, Fig. 1: bit i = light i visible).
//
// Quantising a filtered value is a discrete decision taken from a float, so
// it is made in fp32, in the order written here (this file is compiled
// without floating-point contraction): q = floor(255 * clamp(x, 0, 1) + 1/2).
#include <cmath>

#include "orc.h"

extern "C" {

void orc_quantize_u8(const float* x, uint8_t* q, int64_t n) {
    for (int64_t i = 0; i < n; ++i) {
        float v = x[i];
        if (!(v > 0.0f)) v = 0.0f;  // negative values and NaN
        if (v > 1.0f) v = 1.0f;
        const float s = 255.0f * v;
        q[i] = (uint8_t)std::floor(s + 0.5f);
    }
}

void orc_light_mask(const uint8_t* shadow_count, int n_lights, int n_shadow, int64_t hw, uint8_t* mask) {
    for (int64_t i = 0; i < hw; ++i) {
        uint8_t m = 0;
        for (int l = 0; l < n_lights; ++l) {
            // a light counts as visible when at least half of its rays reach it
            // (with one ray per light: that ray)
            if (2 * (int)shadow_count[(int64_t)l * hw + i] >= n_shadow) m |= (uint8_t)(1u << l);
        }
        mask[i] = m;
    }
}

}  // extern "C"
