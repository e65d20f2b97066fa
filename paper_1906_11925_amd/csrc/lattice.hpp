// Lattice velocity sets and storage codecs for the GPU path.
//
// D3Q19 is the paper's lattice (Section 2, Figure 1); D3Q15 is the second one.
// Ordering: 0 = rest, then opposite pairs (2k-1, 2k), so opp(i) = i + 1 for odd
// i and i - 1 for even i > 0.  Weights: D3Q15 rest 2/9, faces 1/9, corners 1/72;
// D3Q19 rest 1/3, faces 1/18, edges 1/36.
//
// Populations are stored as deviations from the rest equilibrium, d_i = f_i - w_i
// (the rest state is exactly zero).  16-bit storage multiplies d_i by a power of
// two close to 1/w_i before rounding (an exact scaling that keeps small
// deviations out of the FP16 subnormal range); FP32 storage is unscaled.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hlb {

enum Storage { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };

template <int Q>
struct Lat;

template <>
struct Lat<15> {
    static constexpr int q = 15;
    static constexpr int cx[15] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
    static constexpr int cy[15] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1};
    static constexpr int cz[15] = {0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1};
    static constexpr float w[15] = {2.f / 9, 1.f / 9, 1.f / 9, 1.f / 9, 1.f / 9, 1.f / 9, 1.f / 9,
                                    1.f / 72, 1.f / 72, 1.f / 72, 1.f / 72, 1.f / 72, 1.f / 72,
                                    1.f / 72, 1.f / 72};
    static constexpr double wd[15] = {2.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                      1.0 / 9, 1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72,
                                      1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72};
    static constexpr float scale[15] = {4.f, 8.f, 8.f, 8.f, 8.f, 8.f, 8.f,
                                        64.f, 64.f, 64.f, 64.f, 64.f, 64.f, 64.f, 64.f};
    static constexpr float iscale[15] = {0.25f, 0.125f, 0.125f, 0.125f, 0.125f, 0.125f,
                                         0.125f, 0.015625f, 0.015625f, 0.015625f, 0.015625f,
                                         0.015625f, 0.015625f, 0.015625f, 0.015625f};
};

template <>
struct Lat<19> {
    static constexpr int q = 19;
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr float w[19] = {1.f / 3, 1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18,
                                    1.f / 18, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36,
                                    1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36,
                                    1.f / 36};
    static constexpr double wd[19] = {1.0 / 3, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                      1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                      1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                      1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    static constexpr float scale[19] = {4.f, 16.f, 16.f, 16.f, 16.f, 16.f, 16.f,
                                        32.f, 32.f, 32.f, 32.f, 32.f, 32.f,
                                        32.f, 32.f, 32.f, 32.f, 32.f, 32.f};
    static constexpr float iscale[19] = {0.25f, 0.0625f, 0.0625f, 0.0625f, 0.0625f, 0.0625f,
                                         0.0625f, 0.03125f, 0.03125f, 0.03125f, 0.03125f,
                                         0.03125f, 0.03125f, 0.03125f, 0.03125f, 0.03125f,
                                         0.03125f, 0.03125f, 0.03125f};
};

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// ---------------------------------------------------------------------------
// storage codecs: element type and FP32 <-> stored conversion
// ---------------------------------------------------------------------------
template <int ST>
struct Store;

template <>
struct Store<ST_F32> {
    using T = float;
    __device__ static inline float dec(T v) { return v; }
    __device__ static inline T enc(float x) { return x; }
};

template <>
struct Store<ST_F16> {
    using T = _Float16;  // conversion from float rounds to nearest even
    __device__ static inline float dec(T v) { return (float)v; }
    __device__ static inline T enc(float x) { return (T)x; }
};

template <>
struct Store<ST_BF16> {
    using T = uint16_t;  // raw bfloat16 bits
    __device__ static inline float dec(T v) { return __uint_as_float(((uint32_t)v) << 16); }
    // round to nearest even on the upper 16 bits; NaN stays a quiet NaN
    __device__ static inline T enc(float x) {
        uint32_t b = __float_as_uint(x);
        if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) return (T)((b >> 16) | 0x40u);
        b += 0x7fffu + ((b >> 16) & 1u);
        return (T)(b >> 16);
    }
};

// decode/encode with the optional per-direction power-of-two scale
template <int Q, int ST, bool SCALED>
struct Codec {
    using S = Store<ST>;
    using T = typename S::T;
    __device__ static inline float dec(int i, T v) {
        float x = S::dec(v);
        if constexpr (SCALED && ST != ST_F32) x *= Lat<Q>::iscale[i];
        return x;
    }
    __device__ static inline T enc(int i, float x) {
        if constexpr (SCALED && ST != ST_F32) x *= Lat<Q>::scale[i];
        return S::enc(x);
    }
};

}  // namespace hlb
