// Device helpers shared by the forward and adjoint kernels: template dispatch,
// tiled indexing, table decoding, moments, equilibrium and iolet time series.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "lattice.hpp"

namespace hlb {

template <int Q_, int ST_, bool SC_>
struct Tag {
    static constexpr int Q = Q_;
    static constexpr int ST = ST_;
    static constexpr bool SC = SC_;
};

template <class F>
inline hipError_t dispatch(int q, int st, bool scaled, F&& f) {
    if (q == 15) {
        if (st == ST_F32) return f(Tag<15, ST_F32, false>{});
        if (st == ST_F16) return scaled ? f(Tag<15, ST_F16, true>{}) : f(Tag<15, ST_F16, false>{});
        if (st == ST_BF16) return scaled ? f(Tag<15, ST_BF16, true>{}) : f(Tag<15, ST_BF16, false>{});
    } else if (q == 19) {
        if (st == ST_F32) return f(Tag<19, ST_F32, false>{});
        if (st == ST_F16) return scaled ? f(Tag<19, ST_F16, true>{}) : f(Tag<19, ST_F16, false>{});
        if (st == ST_BF16) return scaled ? f(Tag<19, ST_BF16, true>{}) : f(Tag<19, ST_BF16, false>{});
    }
    return hipErrorInvalidValue;
}

// element (direction i, site s) of a tiled array with R rows per tile
template <int R>
__device__ inline int64_t tix(int i, int32_t s) {
    return ((int64_t)(s >> kTileShift) * R + i) * kTile + (s & (kTile - 1));
}

// decode a table entry j for direction i of site s: (source direction, source site).
// A wall link (bit 31 set) reads the opposite population of the site itself; its
// low 15 bits hold the interpolated-wall fraction (0: halfway bounce-back).
__device__ inline void link_src(int i, int32_t j, int32_t s, int& dir, int32_t& site) {
    const bool wall = j < 0;
    dir = wall ? opp(i) : i;
    site = wall ? s : j;
}

// Interpolated (BFL, linear) walls on gathered pre-collision deviations d: for a
// wall link i with fraction q = code / 2^15 (o = opp(i), d[i] holding A[o][s]):
//   q <  1/2: d_i = 2q A[o][s] + (1 - 2q) A[o][s + c_i]   (the value pulled for o,
//             when link o is a fluid link; halfway bounce-back otherwise)
//   q >= 1/2: d_i = A[o][s] / (2q) + (2q - 1)/(2q) A[i][s]
// The weights sum to one, so the rule applies to deviations unchanged.
template <int Q, int ST, bool SC>
__device__ inline void apply_bfl(const typename Store<ST>::T* __restrict__ A, int32_t s, int32_t n,
                                 const int32_t (&j)[Q], float (&d)[Q]) {
    using C = Codec<Q, ST, SC>;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int32_t code = j[i] & 0x7fff;
        if (j[i] < 0 && code != 0) {
            const int o = opp(i);
            const float q = (float)code * (1.0f / 32768.0f);
            const float bb = d[i];
            if (q < 0.5f) {
                if (j[o] >= 0 && j[o] < n) d[i] = 2.0f * q * bb + (1.0f - 2.0f * q) * d[o];
            } else {
                const float own = C::dec(i, A[tix<Q>(i, s)]);
                d[i] = bb / (2.0f * q) + (2.0f * q - 1.0f) / (2.0f * q) * own;
            }
        }
    }
}

template <bool NT, class T>
__device__ inline T ld_maybe_nt(const T* p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// Links j[1..Q-1] of site s (decoded form).  Wave form: all 64 lanes of the
// wavefront call it for the sites of one tile (lane = s & 63), lanes past n
// included, because the compact decoding exchanges the tile's source list
// between lanes.  Split into the loads (load_codes) and the decoding
// (decode_codes) so that a caller can issue the loads of the next tile early.
template <int Q, bool NT>
__device__ inline void load_codes(const Table& tb, int32_t s, uint32_t (&c)[Q], int32_t& e0,
                                  int32_t& e1) {
    if (tb.t16 == nullptr) {
#pragma unroll
        for (int i = 1; i < Q; ++i) c[i] = (uint32_t)ld_maybe_nt<NT>(tb.t32 + tix<Q - 1>(i - 1, s));
        e0 = e1 = 0;
        return;
    }
    const int32_t T = s >> kTileShift;
    const int32_t off = tb.toff[T];
    const int32_t cnt = tb.toff[T + 1] - off;
    const int lane = s & (kTile - 1);
    e0 = lane < cnt ? tb.tlist[off + lane] : 0;
    e1 = lane + kTile < cnt ? tb.tlist[off + kTile + lane] : 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) c[i] = ld_maybe_nt<NT>(tb.t16 + tix<Q - 1>(i - 1, s));
}

template <int Q>
__device__ inline void decode_codes(const Table& tb, int32_t s, const uint32_t (&c)[Q], int32_t e0,
                                    int32_t e1, int32_t (&j)[Q]) {
    if (tb.t16 == nullptr) {
#pragma unroll
        for (int i = 1; i < Q; ++i) j[i] = (int32_t)c[i];
        return;
    }
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int slot = (int)((c[i] >> kTileShift) & 0x1ffu);
        const int32_t a = __shfl(e0, slot & (kTile - 1), kTile);
        const int32_t b = __shfl(e1, slot & (kTile - 1), kTile);
        const int32_t tile = slot < kTile ? a : b;
        j[i] = (c[i] & 0x8000u) ? (int32_t)(0x80000000u | (c[i] & 0x7fffu))
                                : ((tile << kTileShift) | (int32_t)(c[i] & (kTile - 1)));
    }
}

template <int Q, bool NT>
__device__ inline void links_wave(const Table& tb, int32_t s, int32_t (&j)[Q]) {
    uint32_t c[Q];
    int32_t e0, e1;
    load_codes<Q, NT>(tb, s, c, e0, e1);
    decode_codes<Q>(tb, s, c, e0, e1, j);
}

// One link of an arbitrary site (no lane exchange).
template <int Q>
__device__ inline int32_t link_one(const Table& tb, int32_t s, int i) {
    if (tb.t16 == nullptr) return tb.t32[tix<Q - 1>(i - 1, s)];
    const uint32_t c = tb.t16[tix<Q - 1>(i - 1, s)];
    if (c & 0x8000u) return (int32_t)(0x80000000u | (c & 0x7fffu));
    const int32_t tile = tb.tlist[tb.toff[s >> kTileShift] + (int)((c >> kTileShift) & 0x1ffu)];
    return (tile << kTileShift) | (int32_t)(c & (kTile - 1));
}

// moments of FP32 deviations: drho = sum d, m = sum c d (constant-folded per lattice)
template <int Q>
__device__ inline void moments(const float (&d)[Q], float& drho, float& mx, float& my, float& mz) {
    using Lt = Lat<Q>;
    drho = d[0];
    mx = my = mz = 0.f;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        drho += d[i];
        if (Lt::cx[i] > 0) mx += d[i];
        if (Lt::cx[i] < 0) mx -= d[i];
        if (Lt::cy[i] > 0) my += d[i];
        if (Lt::cy[i] < 0) my -= d[i];
        if (Lt::cz[i] > 0) mz += d[i];
        if (Lt::cz[i] < 0) mz -= d[i];
    }
}

// equilibrium deviations deq_i = f_i^eq(rho, u) - w_i for all i (pairs share the
// even part of the quadratic)
template <int Q>
__device__ inline void eq_dev(float drho, float rho, float ux, float uy, float uz,
                              float (&deq)[Q]) {
    using Lt = Lat<Q>;
    const float usq15 = 1.5f * (ux * ux + uy * uy + uz * uz);
    deq[0] = Lt::w[0] * (drho - rho * usq15);
#pragma unroll
    for (int k = 1; k < Q; k += 2) {
        const float cu = (float)Lt::cx[k] * ux + (float)Lt::cy[k] * uy + (float)Lt::cz[k] * uz;
        const float sym = Lt::w[k] * (drho + rho * (4.5f * cu * cu - usq15));
        const float asym = Lt::w[k] * rho * 3.0f * cu;
        deq[k] = sym + asym;
        deq[k + 1] = sym - asym;
    }
}

__device__ inline double iolet_value(const DevIolet& io, const double* harm, double t) {
    double v = io.mean;
    for (int h = 1; h <= io.n_harm; ++h) {
        const double ph = fmod((double)h * t, io.period) / io.period;  // in [0, 1)
        double sv, cv;
        sincospi(2.0 * ph, &sv, &cv);
        v += harm[io.harm_off + h - 1] * cv + harm[io.harm_off + io.n_harm + h - 1] * sv;
    }
    return v;
}

}  // namespace hlb
