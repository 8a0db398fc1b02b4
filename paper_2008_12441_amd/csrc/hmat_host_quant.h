// Host-side quantisation to the 16-bit storage forms (bit-defined), shared by
// the H-matrix and H^2 host sources.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

namespace hmat {

// ---------------------------------------------------------------------------
// FP16 quantisation (host, bit-defined): power-of-two scale per stored array,
// s = 2^(ceil(log2 amax) - 15), q = round-to-nearest-even(v / s) in IEEE half.
// |v / s| <= 2^15 < 65504, and q * s reproduces the stored value exactly.
// ---------------------------------------------------------------------------
inline uint16_t f32_to_f16_rne(float v) {
    uint32_t x;
    std::memcpy(&x, &v, 4);
    const uint32_t sign = (x >> 16) & 0x8000u;
    const uint32_t ax = x & 0x7fffffffu;
    if (ax >= 0x7f800000u) return (uint16_t)(sign | (ax > 0x7f800000u ? 0x7e00u : 0x7c00u));
    if (ax >= 0x477ff000u) return (uint16_t)(sign | 0x7c00u);  // rounds to infinity
    if (ax < 0x38800000u) {                                    // half subnormal range
        const float f = std::fabs(v) * 16777216.0f;            // exact: units of 2^-24
        return (uint16_t)(sign | (uint32_t)std::nearbyint(f));
    }
    const uint32_t mant = ax & 0x7fffffu;
    const uint32_t exp = (ax >> 23) - 127 + 15;
    uint32_t h = (exp << 10) | (mant >> 13);
    const uint32_t rem = mant & 0x1fffu;
    if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) h += 1;
    return (uint16_t)(sign | h);
}

// FP32 -> BF16, round to nearest even (NaN stays NaN).
inline uint16_t f32_to_bf16_rne(float v) {
    uint32_t x;
    std::memcpy(&x, &v, 4);
    if ((x & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((x >> 16) | 0x40u);
    const uint32_t lsb = (x >> 16) & 1u;
    x += 0x7fffu + lsb;
    return (uint16_t)(x >> 16);
}

// 16-bit code of v in the storage form: FP16 of v * inv (inv = 1 / scale, a
// power of two, so the product is exact) or BF16 of v.
inline uint16_t quant16(float v, float inv, bool bf16) {
    return bf16 ? f32_to_bf16_rne(v) : f32_to_f16_rne(v * inv);
}

inline float pow2_scale_f16(float amax) {
    if (!(amax > 0.0f)) return 1.0f;
    int e = 0;
    const float m = std::frexp(amax, &e);  // amax = m 2^e, m in [0.5, 1)
    const int c = (m == 0.5f) ? e - 1 : e; // ceil(log2 amax)
    return std::ldexp(1.0f, std::max(c - 15, -126));
}

// Largest |v| of a column-major array (rows x cols, ld); clears *finite when
// an entry is not finite.
inline float col_major_amax(const float *a, int64_t rows, int64_t cols, int64_t ld, bool *finite) {
    float m = 0.0f;
    for (int64_t j = 0; j < cols; ++j)
        for (int64_t i = 0; i < rows; ++i) {
            const float v = a[i + j * ld];
            if (!std::isfinite(v)) *finite = false;
            m = std::max(m, std::fabs(v));
        }
    return m;
}

}  // namespace hmat
