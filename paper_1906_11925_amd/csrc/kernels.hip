// HIP kernels of the sparse lattice-Boltzmann step for gfx950 (MI355X).
//
// The time step (paper Section 2: propagation and collision on a sparse lattice
// of fluid sites) is one fused kernel per step: every thread owns one fluid site,
// pulls its populations from the upstream sites its links name, applies the LBGK
// collision in FP32 and stores the post-collision populations.  A wall link names
// the site itself with the top bit set and reads its opposite population; an
// iolet link names a ghost slot.  The kernel's epilogue writes the ghost slots of
// the next step from the freshly stored populations of the sites that own iolet
// links, so the separate ghost-fill kernel runs only for a state that did not come
// out of the step (after create or a restore).
//
// Links are found in one of three forms (see Table in kernels.hpp):
//  * the int32 neighbour table;
//  * the compact 16-bit table, whose codes name a slot in the tile's short list of
//    source tiles (exchanged between lanes with ds_bpermute) and a lane;
//  * two-level block addressing (4x4x4 blocks with fluid bitmaps): each 256-thread
//    workgroup stages the block records its four tiles need into LDS with one
//    coalesced load and decodes every link from LDS.
// The work is a gather stencil at ~1.3 flop per byte, memory-bound (in practice by
// the rate of requests from L1 to L2 that the gathers issue), so there is no
// matrix-core work.  With FP32 storage and block addressing, workgroups of 4 or 8
// tiles first copy their own tiles' populations into LDS, by loads that write LDS
// directly, and pulls from inside the workgroup read LDS: fewer L1 misses reach
// L2.  A variant of the step also stores the pulled populations, for the reverse
// sweep over a recorded trajectory.
//
// Memory layout: sites are Morton-ordered and grouped in tiles of 64, the width of
// a wavefront.  Populations are stored [tile][direction][64] and the tables
// [tile][direction-1][64], so one wavefront's stores of all directions and its
// table loads each cover one contiguous block (3.75 KB and 3.5 KB for D3Q15 in
// FP32) instead of 2Q separate address streams; every per-direction access of a
// wavefront is a 256-byte (FP32) or 128-byte (16-bit) aligned chunk.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "kernels.hpp"
#include "lattice.hpp"
#include "lbdev.hpp"
#include "step.hpp"

namespace hlb {

template <int Q, int ST, bool SC, bool BRINK, bool BFL, bool FOUT>
__global__ __launch_bounds__(kScBlock) void k_stream_collide(
    const typename Store<ST>::T* __restrict__ src, typename Store<ST>::T* __restrict__ dst,
    Table tb, int32_t n, int32_t xcd_group, float omega, const float* __restrict__ alpha, Ghosts G,
    int64_t t_next, typename Store<ST>::T* __restrict__ fout) {
    __shared__ StageLds lds;
    stream_collide_group<Q, ST, SC, BRINK, BFL, FOUT>(src, dst, tb, n,
                                                      xcd_block((int32_t)blockIdx.x, xcd_group),
                                                      omega, alpha, G, t_next, lds, fout);
}

// workgroups of W tiles with their own populations staged in LDS (block addressing);
// DMA: the copy writes LDS directly (FP32); FOUT: also store the pulled populations
template <int Q, int ST, bool SC, bool BRINK, int W, bool DMA, bool FOUT>
__global__ __launch_bounds__(W * kTile) void k_stream_collide_staged(
    const typename Store<ST>::T* __restrict__ src, typename Store<ST>::T* __restrict__ dst,
    Table tb, int32_t n, int32_t tiles_alloc, int32_t xcd_group, float omega,
    const float* __restrict__ alpha, Ghosts G, int64_t t_next,
    typename Store<ST>::T* __restrict__ fout) {
    __shared__ __attribute__((aligned(16))) typename Store<ST>::T pops[W][Q][kTile];
    __shared__ StageLds lds[W / 4];
    const int32_t w = xcd_block((int32_t)blockIdx.x, xcd_group);
    stream_collide_staged<Q, ST, SC, BRINK, W, DMA, FOUT>(src, dst, tb, n, tiles_alloc, w * W,
                                                          omega, alpha, G, t_next, pops, lds, fout);
}

// ---------------------------------------------------------------------------
// iolet ghost fill: the incoming population of every iolet link for this step
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_iolet_series(const DevIolet* __restrict__ iolets,
                                                          const double* __restrict__ harm,
                                                          int32_t n_iolets, int64_t t0,
                                                          int64_t count, double* __restrict__ vals,
                                                          double* __restrict__ basis,
                                                          int32_t basis_stride) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= count * n_iolets) return;
    const int64_t m = e / n_iolets;
    const int k = (int)(e % n_iolets);
    const DevIolet io = iolets[k];
    const double t = (double)(t0 + m);
    vals[e] = iolet_value(io, harm, t);
    if (basis && io.kind == 1) {
        double* b = basis + e * basis_stride;
        for (int h = 1; h <= io.n_harm; ++h) {
            const double ph = fmod((double)h * t, io.period) / io.period;  // in [0, 1)
            double sv, cv;
            sincospi(2.0 * ph, &sv, &cv);
            b[2 * (h - 1)] = cv;
            b[2 * (h - 1) + 1] = sv;
        }
    }
}

template <int Q, int ST, bool SC>
__global__ __launch_bounds__(kBlock) void k_ghost_fill(typename Store<ST>::T* __restrict__ A,
                                                        Ghosts G, int32_t n, int64_t t) {
    using C = Codec<Q, ST, SC>;
    const int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (l >= G.count) return;
    const int32_t s = G.site[l];
    const int i = G.dir[l];
    // pressure: equilibrium at the iolet density with the site's own (lagged)
    // velocity; velocity: Ladd moving-wall bounce-back
    float vs[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) vs[k] = C::dec(k, A[tix<Q>(k, s)]);
    A[tix<Q>(i, ghost_slot(G, n, l))] = C::enc(i, ghost_value<Q>(G, l, i, vs, t));
}

// ---------------------------------------------------------------------------
// observables: pressure deviation, velocity, wall shear stress
// ---------------------------------------------------------------------------
template <int Q, int ST, bool SC>
__global__ __launch_bounds__(kBlock) void k_observables(
    const typename Store<ST>::T* __restrict__ A, Table tb, int32_t n,
    int32_t streamed, float omega, const int32_t* __restrict__ perm,
    const float* __restrict__ normal, float* __restrict__ p, float* __restrict__ u,
    float* __restrict__ wss) {
    using C = Codec<Q, ST, SC>;
    using Lt = Lat<Q>;
    static_assert(kBlock == 4 * kTile, "a workgroup covers one group of four tiles");
    __shared__ StageLds lds;
    const int32_t g = blockIdx.x;
    const int32_t s = g * kBlock + threadIdx.x;
    const bool live = (s & ~(kTile - 1)) < n;
    int32_t j[Q];
    if (streamed) links_group<Q, false>(tb, g, s, live, lds, j);
    if (!live || s >= n) return;
    float d[Q];
    d[0] = C::dec(0, A[tix<Q>(0, s)]);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        int dir = i;
        int32_t site = s;
        if (streamed) link_src(i, j[i], s, dir, site);
        d[i] = C::dec(i, A[tix<Q>(dir, site)]);
    }
    if (streamed) apply_bfl<Q, ST, SC>(A, s, n, j, d);
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
                                                    int32_t n, double* __restrict__ partial,
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
            const double v = C::dec(i, A[tix<Q>(i, (int32_t)s)]);
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
// state transfer between the internal (Morton, tiled) and caller layouts
// ---------------------------------------------------------------------------
template <int Q, int ST, bool SC>
__global__ __launch_bounds__(kBlock) void k_state(typename Store<ST>::T* __restrict__ A,
                                                   void* __restrict__ ext,
                                                   const int32_t* __restrict__ perm, int32_t n,
                                                   int mode) {
    using C = Codec<Q, ST, SC>;
    using T = typename Store<ST>::T;
    const int32_t s = blockIdx.x * kBlock + threadIdx.x;
    const int i = blockIdx.y;
    if (s >= n) return;
    const int64_t e = (int64_t)i * n + (perm ? perm[s] : s);
    const int64_t a = tix<Q>(i, s);
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
            static_cast<T*>(A), G, (int32_t)L.n, t);
        return hipGetLastError();
    });
}

template <int W>
static hipError_t launch_staged(const Layout& L, const Ghosts& G, const void* src, void* dst,
                                float omega, const float* alpha, int xcd_group, int64_t t_next,
                                void* fout, hipStream_t s) {
    const int64_t tiles = (L.n + kTile - 1) / kTile;
    const int64_t nb = (tiles + W - 1) / W;
    // the same number of tiles per XCD chunk as the four-tile workgroups
    const int32_t per = xcd_group > 0 ? std::max(1, xcd_group * 4 / W) : 0;
    int64_t grid = nb;
    if (per > 0) grid = ((nb + 8 * per - 1) / (8 * per)) * (8 * per);
    const int32_t tiles_alloc = (int32_t)(L.slots / kTile);
    return dispatch(L.q, L.storage, L.scaled, [&](auto tag) {
        using Tg = decltype(tag);
        using T = typename Store<Tg::ST>::T;
        auto go = [&](auto kernel) {
            kernel<<<(unsigned)grid, W * kTile, 0, s>>>(static_cast<const T*>(src),
                                                        static_cast<T*>(dst), L.tb, (int32_t)L.n,
                                                        tiles_alloc, per, omega, alpha, G, t_next,
                                                        static_cast<T*>(fout));
            return hipGetLastError();
        };
        // the direct-to-LDS copy exists for FP32 rows only, and so does the store of
        // the pulled populations (the recording forward)
        if constexpr (Tg::ST == ST_F32) {
            if (fout)
                return L.lds_dma
                           ? (alpha ? go(k_stream_collide_staged<Tg::Q, Tg::ST, Tg::SC, true, W, true, true>)
                                    : go(k_stream_collide_staged<Tg::Q, Tg::ST, Tg::SC, false, W, true, true>))
                           : (alpha ? go(k_stream_collide_staged<Tg::Q, Tg::ST, Tg::SC, true, W, false, true>)
                                    : go(k_stream_collide_staged<Tg::Q, Tg::ST, Tg::SC, false, W, false, true>));
            if (L.lds_dma)
                return alpha ? go(k_stream_collide_staged<Tg::Q, Tg::ST, Tg::SC, true, W, true, false>)
                             : go(k_stream_collide_staged<Tg::Q, Tg::ST, Tg::SC, false, W, true, false>);
        }
        if (fout) return hipErrorInvalidValue;
        return alpha ? go(k_stream_collide_staged<Tg::Q, Tg::ST, Tg::SC, true, W, false, false>)
                     : go(k_stream_collide_staged<Tg::Q, Tg::ST, Tg::SC, false, W, false, false>);
    });
}

hipError_t launch_stream_collide(const Layout& L, const Ghosts& G, const void* src, void* dst,
                                 float omega, const float* alpha, int xcd_group, int64_t t_next,
                                 hipStream_t s, void* fout) {
    if (L.n == 0) return hipSuccess;
    if (fout && L.bfl) return hipErrorInvalidValue;  // interpolated values are not stored values
    if (L.stage_tiles > 0 && L.tb.grp && !L.bfl) {
        if (L.stage_tiles == 4) return launch_staged<4>(L, G, src, dst, omega, alpha, xcd_group, t_next, fout, s);
        if (L.stage_tiles == 8) return launch_staged<8>(L, G, src, dst, omega, alpha, xcd_group, t_next, fout, s);
        if (L.stage_tiles == 16) return launch_staged<16>(L, G, src, dst, omega, alpha, xcd_group, t_next, fout, s);
    }
    int64_t nb = (L.n + kScBlock - 1) / kScBlock;
    const int32_t per = xcd_group > 0 ? xcd_group : 0;
    int64_t grid = nb;
    if (per > 0) grid = ((nb + 8 * per - 1) / (8 * per)) * (8 * per);
    return dispatch(L.q, L.storage, L.scaled, [&](auto tag) {
        using Tg = decltype(tag);
        using T = typename Store<Tg::ST>::T;
        auto go = [&](auto kernel, const float* a) {
            kernel<<<(unsigned)grid, kScBlock, 0, s>>>(static_cast<const T*>(src),
                                                       static_cast<T*>(dst), L.tb, (int32_t)L.n,
                                                       per, omega, a, G, t_next,
                                                       static_cast<T*>(fout));
        };
        if (fout) {  // the recording forward: FP32 storage, halfway walls
            if constexpr (Tg::ST == ST_F32) {
                alpha ? go(k_stream_collide<Tg::Q, Tg::ST, Tg::SC, true, false, true>, alpha)
                      : go(k_stream_collide<Tg::Q, Tg::ST, Tg::SC, false, false, true>, nullptr);
                return hipGetLastError();
            }
            return hipErrorInvalidValue;
        }
        if (alpha)
            L.bfl ? go(k_stream_collide<Tg::Q, Tg::ST, Tg::SC, true, true, false>, alpha)
                  : go(k_stream_collide<Tg::Q, Tg::ST, Tg::SC, true, false, false>, alpha);
        else
            L.bfl ? go(k_stream_collide<Tg::Q, Tg::ST, Tg::SC, false, true, false>, nullptr)
                  : go(k_stream_collide<Tg::Q, Tg::ST, Tg::SC, false, false, false>, nullptr);
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
            static_cast<const T*>(A), L.tb, (int32_t)L.n, streamed, omega, perm, normal, p, u,
            wss);
        return hipGetLastError();
    });
}

hipError_t launch_totals(const Layout& L, const void* A, double* partial, int64_t nparts,
                         double* out, int32_t* flag, hipStream_t s) {
    hipError_t e = dispatch(L.q, L.storage, L.scaled, [&](auto tag) {
        using Tg = decltype(tag);
        using T = typename Store<Tg::ST>::T;
        k_totals<Tg::Q, Tg::ST, Tg::SC><<<(unsigned)nparts, kBlock, 0, s>>>(
            static_cast<const T*>(A), (int32_t)L.n, partial, flag);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    k_totals_final<<<1, kBlock, 0, s>>>(partial, (int32_t)nparts, (double)L.n, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// totals without any allocation: the reduction's partial sums live in a
// file-scope device array, one copy per GPU
// ---------------------------------------------------------------------------
constexpr int kScratchDoubles = kTotBlocks * 4 + 2;  // partial sums, then the flag word
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each GPU

// The device address of this GPU's `scratch` (the host-side name is only a
// stand-in), looked up once per device with that device current.
static hipError_t scratch_address(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

int64_t totals_scratch_parts() { return kTotBlocks; }

hipError_t launch_totals_noalloc(const Layout& L, const void* A, double* out, hipStream_t s) {
    const int64_t nparts = totals_parts(L.n);
    if (nparts > kTotBlocks) return hipErrorInvalidValue;
    double* sp = nullptr;
    hipError_t e = scratch_address(&sp);
    if (e != hipSuccess) return e;
    int32_t* flag = reinterpret_cast<int32_t*>(sp + (int64_t)kTotBlocks * 4);
    return launch_totals(L, A, sp, nparts, out, flag, s);
}

hipError_t launch_state(const Layout& L, void* A, void* ext, const int32_t* perm, int mode,
                        hipStream_t s) {
    if (L.n == 0) return hipSuccess;
    return dispatch(L.q, L.storage, L.scaled, [&](auto tag) {
        using Tg = decltype(tag);
        using T = typename Store<Tg::ST>::T;
        dim3 grid(blocks_for(L.n), (unsigned)Tg::Q);
        k_state<Tg::Q, Tg::ST, Tg::SC><<<grid, kBlock, 0, s>>>(static_cast<T*>(A), ext, perm,
                                                                (int32_t)L.n, mode);
        return hipGetLastError();
    });
}

hipError_t launch_zero(const Layout& L, void* A, hipStream_t s) {
    const int64_t bytes = (int64_t)L.q * L.slots * (int64_t)elem_size(L.storage);
    const int64_t words = bytes / 4;
    int64_t nb = (words + kBlock - 1) / kBlock;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    k_zero<<<(unsigned)nb, kBlock, 0, s>>>(static_cast<uint32_t*>(A), words);
    return hipGetLastError();
}

bool ghosts_fused() { return HLB_FUSE_GHOSTS != 0; }

hipError_t launch_iolet_series(const DevIolet* iolets, const double* harm, int32_t n_iolets,
                               int64_t t0, int64_t count, double* vals, double* basis,
                               int32_t basis_stride, hipStream_t s) {
    if (n_iolets == 0 || count <= 0) return hipSuccess;
    k_iolet_series<<<blocks_for(count * n_iolets), kBlock, 0, s>>>(iolets, harm, n_iolets, t0,
                                                                   count, vals, basis, basis_stride);
    return hipGetLastError();
}

hipError_t launch_zero_words(void* p, int64_t words, hipStream_t s) {
    if (words <= 0) return hipSuccess;
    int64_t nb = (words + kBlock - 1) / kBlock;
    if (nb > 4096) nb = 4096;
    k_zero<<<(unsigned)nb, kBlock, 0, s>>>(static_cast<uint32_t*>(p), words);
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
