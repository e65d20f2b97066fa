// HIP kernels of the sparse lattice-Boltzmann step for gfx950 (MI355X).
//
// The time step (paper Section 2: propagation and collision on a sparse lattice
// of fluid sites) is one fused kernel per step: every thread owns one fluid site,
// pulls its populations through the int32 neighbour table (wall links point at
// the opposite population of the same site, iolet links at a ghost slot filled
// just before by the ghost-fill kernel), applies the LBGK collision in FP32 and
// writes the post-collision populations with coalesced stores.  The work is a
// gather/scatter stencil at ~1.3 flop per byte, bound by HBM bandwidth, so there
// is no matrix-core work and no LDS staging: the kernel is written for wide
// memory-level parallelism (all table and population loads of a thread issued
// before any arithmetic) and for L2 locality (Morton-ordered sites, blocks
// mapped to XCDs in contiguous ranges).
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
static hipError_t dispatch(int q, int st, bool scaled, F&& f) {
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

// ---------------------------------------------------------------------------
// fused pull stream + LBGK collide
// ---------------------------------------------------------------------------
template <int Q, int ST, bool SC, bool BRINK>
__global__ __launch_bounds__(kBlock) void k_stream_collide(
    const typename Store<ST>::T* __restrict__ src, typename Store<ST>::T* __restrict__ dst,
    const int32_t* __restrict__ tbl, int32_t n, int64_t pitch, int64_t tpitch, int32_t per_xcd,
    float omega, const float* __restrict__ alpha) {
    using C = Codec<Q, ST, SC>;
    // consecutive block ids are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous range of sites so that neighbour gathers hit its own L2
    int32_t b = blockIdx.x;
    if (per_xcd > 0) b = (b & 7) * per_xcd + (b >> 3);
    const int32_t s = b * kBlock + (int32_t)threadIdx.x;
    if (s >= n) return;

    int32_t j[Q];
#pragma unroll
    for (int i = 1; i < Q; ++i) j[i] = tbl[(int64_t)(i - 1) * tpitch + s];
    float d[Q];
    d[0] = C::dec(0, src[s]);
#pragma unroll
    for (int i = 1; i < Q; ++i) d[i] = C::dec(i, src[(int64_t)i * pitch + j[i]]);

    float drho, mx, my, mz;
    moments<Q>(d, drho, mx, my, mz);
    const float rho = 1.0f + drho;
    const float ir = 1.0f / rho;
    float ux = mx * ir, uy = my * ir, uz = mz * ir;
    if constexpr (BRINK) {
        const float a = 1.0f - alpha[s];
        ux *= a;
        uy *= a;
        uz *= a;
    }
    float deq[Q];
    eq_dev<Q>(drho, rho, ux, uy, uz, deq);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float v = d[i] - omega * (d[i] - deq[i]);
        dst[(int64_t)i * pitch + s] = C::enc(i, v);
    }
}

// ---------------------------------------------------------------------------
// iolet ghost fill: the incoming population of every iolet link for this step
// ---------------------------------------------------------------------------
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

template <int Q, int ST, bool SC>
__global__ __launch_bounds__(kBlock) void k_ghost_fill(typename Store<ST>::T* __restrict__ A,
                                                        Ghosts G, int32_t n, int64_t pitch,
                                                        double t) {
    using C = Codec<Q, ST, SC>;
    using Lt = Lat<Q>;
    const int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (l >= G.count) return;
    const int32_t s = G.site[l];
    const int i = G.dir[l];
    const DevIolet io = G.iolets[G.iolet[l]];
    const double v = iolet_value(io, G.harm, t);
    float g;
    if (io.kind == 0) {
        // equilibrium at the iolet density with the site's own (lagged) velocity
        float d[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) d[k] = C::dec(k, A[(int64_t)k * pitch + s]);
        float drho, mx, my, mz;
        moments<Q>(d, drho, mx, my, mz);
        const float ir = 1.0f / (1.0f + drho);
        const float ux = mx * ir, uy = my * ir, uz = mz * ir;
        const float cu = (float)Lt::cx[i] * ux + (float)Lt::cy[i] * uy + (float)Lt::cz[i] * uz;
        const float usq = ux * ux + uy * uy + uz * uz;
        const float rk = (float)v, rk1 = (float)(v - 1.0);
        g = Lt::w[i] * (rk1 + rk * (3.0f * cu + 4.5f * cu * cu - 1.5f * usq));
    } else {
        // Ladd moving-wall bounce-back
        const int o = opp(i);
        g = C::dec(o, A[(int64_t)o * pitch + s]) + G.coef[l] * (float)v;
    }
    A[(int64_t)i * pitch + n + l] = C::enc(i, g);
}

// ---------------------------------------------------------------------------
// observables: pressure deviation, velocity, wall shear stress
// ---------------------------------------------------------------------------
template <int Q, int ST, bool SC>
__global__ __launch_bounds__(kBlock) void k_observables(
    const typename Store<ST>::T* __restrict__ A, const int32_t* __restrict__ tbl, int32_t n,
    int64_t pitch, int64_t tpitch, int32_t streamed, float omega, const int32_t* __restrict__ perm,
    const float* __restrict__ normal, float* __restrict__ p, float* __restrict__ u,
    float* __restrict__ wss) {
    using C = Codec<Q, ST, SC>;
    using Lt = Lat<Q>;
    const int32_t s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    float d[Q];
    d[0] = C::dec(0, A[s]);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int32_t j = streamed ? tbl[(int64_t)(i - 1) * tpitch + s] : s;
        d[i] = C::dec(i, A[(int64_t)i * pitch + j]);
    }
    float drho, mx, my, mz;
    moments<Q>(d, drho, mx, my, mz);
    const float rho = 1.0f + drho;
    const float ir = 1.0f / rho;
    const float ux = mx * ir, uy = my * ir, uz = mz * ir;
    const int32_t o = perm ? perm[s] : s;
    if (p) p[o] = drho * (1.0f / 3.0f);
    if (u) {
        u[3 * (int64_t)o + 0] = ux;
        u[3 * (int64_t)o + 1] = uy;
        u[3 * (int64_t)o + 2] = uz;
    }
    if (!wss) return;
    const float nx = normal[s], ny = normal[n + s], nz = normal[2 * (int64_t)n + s];
    if (nx == 0.f && ny == 0.f && nz == 0.f) {
        wss[o] = 0.f;
        return;
    }
    float deq[Q];
    eq_dev<Q>(drho, rho, ux, uy, uz, deq);
    float pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const float e = d[i] - deq[i];
        const float cx = Lt::cx[i], cy = Lt::cy[i], cz = Lt::cz[i];
        if (Lt::cx[i]) pxx += e;
        if (Lt::cy[i]) pyy += e;
        if (Lt::cz[i]) pzz += e;
        if (Lt::cx[i] && Lt::cy[i]) pxy += cx * cy * e;
        if (Lt::cx[i] && Lt::cz[i]) pxz += cx * cz * e;
        if (Lt::cy[i] && Lt::cz[i]) pyz += cy * cz * e;
    }
    const float k = -(1.0f - 0.5f * omega);
    const float sx = k * (pxx * nx + pxy * ny + pxz * nz);
    const float sy = k * (pxy * nx + pyy * ny + pyz * nz);
    const float sz = k * (pxz * nx + pyz * ny + pzz * nz);
    const float nsn = sx * nx + sy * ny + sz * nz;
    const float tx = sx - nsn * nx, ty = sy - nsn * ny, tz = sz - nsn * nz;
    wss[o] = sqrtf(tx * tx + ty * ty + tz * tz);
}

// ---------------------------------------------------------------------------
// FP64 totals (mass, momentum) with a deterministic two-pass reduction
// ---------------------------------------------------------------------------
constexpr int kTotBlocks = 1024;

int64_t totals_parts(int64_t n) {
    int64_t nb = (n + kBlock - 1) / kBlock;
    return nb < 1 ? 1 : (nb > kTotBlocks ? kTotBlocks : nb);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int Q, int ST, bool SC>
__global__ __launch_bounds__(kBlock) void k_totals(const typename Store<ST>::T* __restrict__ A,
                                                    int32_t n, int64_t pitch,
                                                    double* __restrict__ partial,
                                                    int32_t* __restrict__ flag) {
    using C = Codec<Q, ST, SC>;
    using Lt = Lat<Q>;
    double acc[4] = {0, 0, 0, 0};
    bool bad = false;
    for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * kBlock) {
        double r = 0, x = 0, y = 0, z = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double v = C::dec(i, A[(int64_t)i * pitch + s]);
            r += v;
            x += Lt::cx[i] * v;
            y += Lt::cy[i] * v;
            z += Lt::cz[i] * v;
        }
        bad |= !(isfinite(r) && isfinite(x) && isfinite(y) && isfinite(z));
        acc[0] += r;
        acc[1] += x;
        acc[2] += y;
        acc[3] += z;
    }
    if (bad) flag[0] = 1;
    __shared__ double red[4][kBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double v = wave_sum(acc[c]);
        if (lane == 0) red[c][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double v = 0;
        for (int w = 0; w < kBlock / 64; ++w) v += red[threadIdx.x][w];
        partial[(int64_t)blockIdx.x * 4 + threadIdx.x] = v;
    }
}

__global__ __launch_bounds__(kBlock) void k_totals_final(const double* __restrict__ partial,
                                                          int32_t nparts, double n_sites,
                                                          double* __restrict__ out) {
    __shared__ double red[4][kBlock / 64];
    double acc[4] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < nparts; b += kBlock)
        for (int c = 0; c < 4; ++c) acc[c] += partial[(int64_t)b * 4 + c];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int c = 0; c < 4; ++c) {
        const double v = wave_sum(acc[c]);
        if (lane == 0) red[c][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double v = 0;
        for (int w = 0; w < kBlock / 64; ++w) v += red[threadIdx.x][w];
        out[threadIdx.x] = threadIdx.x == 0 ? n_sites + v : v;
    }
}

// ---------------------------------------------------------------------------
// state transfer between the internal (Morton, pitched) and caller layouts
// ---------------------------------------------------------------------------
template <int Q, int ST, bool SC>
__global__ __launch_bounds__(kBlock) void k_state(typename Store<ST>::T* __restrict__ A,
                                                   void* __restrict__ ext,
                                                   const int32_t* __restrict__ perm, int32_t n,
                                                   int64_t pitch, int mode) {
    using C = Codec<Q, ST, SC>;
    using T = typename Store<ST>::T;
    const int32_t s = blockIdx.x * kBlock + threadIdx.x;
    const int i = blockIdx.y;
    if (s >= n) return;
    const int64_t e = (int64_t)i * n + (perm ? perm[s] : s);
    const int64_t a = (int64_t)i * pitch + s;
    switch (mode) {
        case 0: static_cast<T*>(ext)[e] = A[a]; break;
        case 1: A[a] = static_cast<const T*>(ext)[e]; break;
        case 2: static_cast<float*>(ext)[e] = C::dec(i, A[a]); break;
        default: A[a] = C::enc(i, static_cast<const float*>(ext)[e]); break;
    }
}

__global__ __launch_bounds__(kBlock) void k_zero(uint32_t* __restrict__ p, int64_t words) {
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < words;
         k += (int64_t)gridDim.x * kBlock)
        p[k] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_copy(const uint4* __restrict__ src,
                                                  uint4* __restrict__ dst, int64_t n16) {
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n16;
         k += (int64_t)gridDim.x * kBlock)
        dst[k] = src[k];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

static inline size_t elem_size(int st) { return st == ST_F32 ? 4 : 2; }

hipError_t launch_ghost_fill(const Layout& L, const Ghosts& G, void* A, int64_t t,
                             hipStream_t s) {
    if (G.count == 0) return hipSuccess;
    return dispatch(L.q, L.storage, L.scaled, [&](auto tag) {
        using Tg = decltype(tag);
        using T = typename Store<Tg::ST>::T;
        k_ghost_fill<Tg::Q, Tg::ST, Tg::SC><<<blocks_for(G.count), kBlock, 0, s>>>(
            static_cast<T*>(A), G, (int32_t)L.n, L.pitch, (double)t);
        return hipGetLastError();
    });
}

hipError_t launch_stream_collide(const Layout& L, const void* src, void* dst, float omega,
                                 const float* alpha, bool xcd_remap, hipStream_t s) {
    if (L.n == 0) return hipSuccess;
    const int64_t nb = (L.n + kBlock - 1) / kBlock;
    int32_t per = 0;
    int64_t grid = nb;
    if (xcd_remap) {
        per = (int32_t)((nb + 7) / 8);
        grid = (int64_t)per * 8;
    }
    return dispatch(L.q, L.storage, L.scaled, [&](auto tag) {
        using Tg = decltype(tag);
        using T = typename Store<Tg::ST>::T;
        if (alpha)
            k_stream_collide<Tg::Q, Tg::ST, Tg::SC, true><<<(unsigned)grid, kBlock, 0, s>>>(
                static_cast<const T*>(src), static_cast<T*>(dst), L.tbl, (int32_t)L.n, L.pitch,
                L.tpitch, per, omega, alpha);
        else
            k_stream_collide<Tg::Q, Tg::ST, Tg::SC, false><<<(unsigned)grid, kBlock, 0, s>>>(
                static_cast<const T*>(src), static_cast<T*>(dst), L.tbl, (int32_t)L.n, L.pitch,
                L.tpitch, per, omega, nullptr);
        return hipGetLastError();
    });
}

hipError_t launch_observables(const Layout& L, const void* A, int streamed, float omega,
                              const int32_t* perm, const float* normal, float* p, float* u,
                              float* wss, hipStream_t s) {
    if (L.n == 0) return hipSuccess;
    return dispatch(L.q, L.storage, L.scaled, [&](auto tag) {
        using Tg = decltype(tag);
        using T = typename Store<Tg::ST>::T;
        k_observables<Tg::Q, Tg::ST, Tg::SC><<<blocks_for(L.n), kBlock, 0, s>>>(
            static_cast<const T*>(A), L.tbl, (int32_t)L.n, L.pitch, L.tpitch, streamed, omega,
            perm, normal, p, u, wss);
        return hipGetLastError();
    });
}

hipError_t launch_totals(const Layout& L, const void* A, double* partial, int64_t nparts,
                         double* out, int32_t* flag, hipStream_t s) {
    hipError_t e = dispatch(L.q, L.storage, L.scaled, [&](auto tag) {
        using Tg = decltype(tag);
        using T = typename Store<Tg::ST>::T;
        k_totals<Tg::Q, Tg::ST, Tg::SC><<<(unsigned)nparts, kBlock, 0, s>>>(
            static_cast<const T*>(A), (int32_t)L.n, L.pitch, partial, flag);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    k_totals_final<<<1, kBlock, 0, s>>>(partial, (int32_t)nparts, (double)L.n, out);
    return hipGetLastError();
}

hipError_t launch_state(const Layout& L, void* A, void* ext, const int32_t* perm, int mode,
                        hipStream_t s) {
    if (L.n == 0) return hipSuccess;
    return dispatch(L.q, L.storage, L.scaled, [&](auto tag) {
        using Tg = decltype(tag);
        using T = typename Store<Tg::ST>::T;
        dim3 grid(blocks_for(L.n), (unsigned)Tg::Q);
        k_state<Tg::Q, Tg::ST, Tg::SC><<<grid, kBlock, 0, s>>>(static_cast<T*>(A), ext, perm,
                                                                (int32_t)L.n, L.pitch, mode);
        return hipGetLastError();
    });
}

hipError_t launch_zero(const Layout& L, void* A, hipStream_t s) {
    const int64_t bytes = (int64_t)L.q * L.pitch * (int64_t)elem_size(L.storage);
    const int64_t words = bytes / 4;
    int64_t nb = (words + kBlock - 1) / kBlock;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    k_zero<<<(unsigned)nb, kBlock, 0, s>>>(static_cast<uint32_t*>(A), words);
    return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, int64_t bytes, hipStream_t s) {
    const int64_t n16 = bytes / 16;
    int64_t nb = (n16 + kBlock - 1) / kBlock;
    if (nb > 65536) nb = 65536;
    if (nb < 1) nb = 1;
    k_copy<<<(unsigned)nb, kBlock, 0, s>>>(static_cast<const uint4*>(src), static_cast<uint4*>(dst),
                                           n16);
    return hipGetLastError();
}

}  // namespace hlb
