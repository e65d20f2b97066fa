// The fused pull-stream + LBGK-collide step of one site and one workgroup, shared
// by the step kernel and the adjoint's recompute.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "lattice.hpp"
#include "lbdev.hpp"

namespace hlb {

// ---------------------------------------------------------------------------
// fused pull stream + LBGK collide
// ---------------------------------------------------------------------------
// Build-time tuning knobs (every variant computes the same result):
//   HLB_NT_STORE  nontemporal stores of the post-collision populations
//   HLB_NT_TABLE  nontemporal loads of the neighbour table
#ifndef HLB_NT_STORE
#define HLB_NT_STORE 1
#endif
#ifndef HLB_NT_TABLE
#define HLB_NT_TABLE 1
#endif
// One workgroup covers one group of four tiles (the unit of the staged block
// records).  Groups of 8 or 16 tiles per workgroup (more neighbours sharing one
// L1) measured no faster with the explicit tables.
constexpr int kScBlock = 4 * kTile;

template <class T>
__device__ inline void st_pop(T* p, T v) {
#if HLB_NT_STORE
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

// Incoming population of iolet link l (direction i) of a site whose stored
// populations decode to vs, at time t (the definition the ghost-fill kernel applies).
// Both the step kernel's epilogue and the ghost-fill kernel inline it; without
// contraction every product and sum rounds on its own in both, so a state
// restored from a checkpoint gets the same ghost values, bit for bit, as the
// step that produced it (the moment sums it calls multiply only by 0 and +-1,
// which is exact either way).
template <int Q>
__device__ inline float ghost_value(const Ghosts& G, int64_t l, int i, const float (&vs)[Q],
                                    int64_t t) {
#pragma clang fp contract(off)
    using Lt = Lat<Q>;
    const int k = G.iolet[l];
    const double v = G.vals[(t - G.vals_t0) * G.n_iolets + k];
    if (G.iolets[k].kind == 0) {
        float drho, mx, my, mz;
        moments<Q>(vs, drho, mx, my, mz);
        const float ir = 1.0f / (1.0f + drho);
        const float ux = mx * ir, uy = my * ir, uz = mz * ir;
        const float cu = (float)Lt::cx[i] * ux + (float)Lt::cy[i] * uy + (float)Lt::cz[i] * uz;
        const float usq = ux * ux + uy * uy + uz * uz;
        const float rk = (float)v, rk1 = (float)(v - 1.0);
        return Lt::w[i] * (rk1 + rk * (3.0f * cu + 4.5f * cu * cu - 1.5f * usq));
    }
    return vs[opp(i)] + G.coef[l] * (float)v;
}

// With HLB_FUSE_GHOSTS, a site that owns iolet links also writes the incoming
// populations of those links for the next step (time t_next) into dst's ghost
// slots, from its freshly stored populations; the separate ghost fill is then
// only needed for a state that did not come out of this kernel.
#ifndef HLB_FUSE_GHOSTS
#define HLB_FUSE_GHOSTS 1
#endif

// The pulled (pre-collision) deviations of one site and what the epilogue needs
// about its iolet links.
template <int Q>
struct Pulled {
    float d[Q];
    uint32_t gmask;  // directions of the site's iolet links (fused ghost epilogue)
    int64_t gl;      // the first of those links
};

// Pull the populations of site s whose links are decoded in j.
template <int Q, int ST, bool SC, bool BFL>
__device__ inline void site_pull(const typename Store<ST>::T* __restrict__ src, int32_t n,
                                 const Ghosts& G, int32_t s, const int32_t (&j)[Q], Pulled<Q>& P) {
    using C = Codec<Q, ST, SC>;
    P.d[0] = C::dec(0, src[tix<Q>(0, s)]);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        int dir;
        int32_t site;
        link_src(i, j[i], s, dir, site);
        P.d[i] = C::dec(i, src[tix<Q>(dir, site)]);
    }
    if constexpr (BFL) apply_bfl<Q, ST, SC>(src, s, n, j, P.d);
    P.gmask = 0;
    P.gl = -1;
#if HLB_FUSE_GHOSTS
    // directions of the site's iolet links and the first of those links (they are
    // consecutive in the link list, in direction order), for the epilogue
    int32_t top = j[1];  // walls are negative, sites below n, ghost slots from n
#pragma unroll
    for (int i = 2; i < Q; ++i) top = max(top, j[i]);
    if (top >= n) {
#pragma unroll
        for (int i = 1; i < Q; ++i)
            if (j[i] >= n) {
                if (P.gl < 0) P.gl = ghost_link<Q>(G, n, j[i], i);
                P.gmask |= 1u << i;
            }
    }
#else
    (void)G;
#endif
}

// Collide the pulled populations of site s and store them (and, with the fused
// ghost epilogue, the incoming populations of its iolet links for time t_next).
// FOUT: also store the pulled populations themselves into fout, in the site's own
// slots, for the reverse sweep (exact: each is a stored value decoded; halfway
// walls only).
template <int Q, int ST, bool SC, bool BRINK, bool FOUT = false>
__device__ inline void site_collide_store(typename Store<ST>::T* __restrict__ dst, int32_t n,
                                          float omega, const float* __restrict__ alpha,
                                          const Ghosts& G, int64_t t_next, int32_t s,
                                          const Pulled<Q>& P,
                                          typename Store<ST>::T* __restrict__ fout) {
    using C = Codec<Q, ST, SC>;
    const float(&d)[Q] = P.d;
    if constexpr (FOUT) {
#pragma unroll
        for (int i = 0; i < Q; ++i) st_pop(fout + tix<Q>(i, s), C::enc(i, d[i]));
    } else {
        (void)fout;
    }
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
    float vs[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const typename Store<ST>::T e = C::enc(i, d[i] - omega * (d[i] - deq[i]));
        st_pop(dst + tix<Q>(i, s), e);
        vs[i] = C::dec(i, e);
    }
#if HLB_FUSE_GHOSTS
    // The iolet links of a site are consecutive in the link list, in direction
    // order.  With one slot per link (table encodings) the first one is the
    // smallest ghost slot the site pulls from; with shared ghost cells (block
    // addressing) it is found through the cell's link list.
    if (P.gmask) {
        int64_t gl = P.gl;
#pragma unroll
        for (int i = 1; i < Q; ++i)
            if (P.gmask & (1u << i)) {
                dst[tix<Q>(i, ghost_slot(G, n, gl))] = C::enc(i, ghost_value<Q>(G, gl, i, vs, t_next));
                ++gl;
            }
    }
#else
    (void)vs;
    (void)G;
    (void)t_next;
    (void)n;
#endif
}

// Pull, collide and store one site whose links are decoded in j.
template <int Q, int ST, bool SC, bool BRINK, bool BFL, bool FOUT = false>
__device__ inline void site_update(const typename Store<ST>::T* __restrict__ src,
                                   typename Store<ST>::T* __restrict__ dst, int32_t n, float omega,
                                   const float* __restrict__ alpha, const Ghosts& G,
                                   int64_t t_next, int32_t s, const int32_t (&j)[Q],
                                   typename Store<ST>::T* __restrict__ fout) {
    Pulled<Q> P;
    site_pull<Q, ST, SC, BFL>(src, n, G, s, j, P);
    site_collide_store<Q, ST, SC, BRINK, FOUT>(dst, n, omega, alpha, G, t_next, s, P, fout);
}

// Block ids are dealt round-robin to the 8 XCDs (each with its own L2).  With
// xcd_group = G > 0, every XCD takes G consecutive blocks of a window of 8G
// blocks, so neighbouring sites share an L2 while all XCDs still sweep the
// Morton order together (and share the last-level cache).
__device__ inline int32_t xcd_block(int32_t b, int32_t xcd_group) {
    if (xcd_group > 0) {
        const int32_t w = 8 * xcd_group;
        b = (b / w) * w + (b & 7) * xcd_group + (b >> 3) % xcd_group;
    }
    return b;
}

// One workgroup (group g of four tiles) of the fused step.  Every thread of the
// workgroup calls it.  FOUT: also store the pulled populations into fout.
template <int Q, int ST, bool SC, bool BRINK, bool BFL, bool FOUT = false>
__device__ inline void stream_collide_group(const typename Store<ST>::T* __restrict__ src,
                                            typename Store<ST>::T* __restrict__ dst,
                                            const Table& tb, int32_t n, int32_t g, float omega,
                                            const float* __restrict__ alpha, const Ghosts& G,
                                            int64_t t_next, StageLds& lds,
                                            typename Store<ST>::T* __restrict__ fout = nullptr) {
    if (g * kScBlock >= n) return;  // the whole workgroup lies past the end
    const int32_t s = g * kScBlock + (int32_t)threadIdx.x;
    const bool live = (s & ~(kTile - 1)) < n;  // the wavefront's tile has sites
    // all link decoding, then all population gathers, before any arithmetic
    int32_t j[Q];
    links_group<Q, HLB_NT_TABLE != 0>(tb, g, s, live, lds, j);
    if (!live || s >= n) return;
    site_update<Q, ST, SC, BRINK, BFL, FOUT>(src, dst, n, omega, alpha, G, t_next, s, j, fout);
}

// Links of the sites of a workgroup of W tiles (W a multiple of 4) from the
// staged records of its W/4 groups: every thread takes its share of its group's
// blob, one barrier, then every wavefront decodes its tile.  Groups whose records
// did not fit decode from the global records.  Every thread calls it.
template <int Q, int W, bool WAIT_VM = false>
__device__ inline void links_tiles(const Table& tb, int32_t T0, int32_t n, StageLds (&lds)[W / 4],
                                   int32_t (&j)[Q]) {
    const int wave = (int)threadIdx.x >> kTileShift;
    const int32_t g = (T0 >> 2) + (wave >> 2);  // this thread's group of four tiles
    const int32_t s = (T0 << kTileShift) + (int32_t)threadIdx.x;
    const bool live = (s & ~(kTile - 1)) < n;
    StageHdr h{0, 0, 0};
    if (((int64_t)g << 8) < n) {
        h = stage_header(tb, g);
        // the group's 256 threads fetch its blob (thread index within the group)
        const int32_t t = (int32_t)threadIdx.x & (kScBlock - 1);
        if (h.nown > 0) {
            const int row_chunks = (h.nown * kRowBytes + 15) >> 4;
            if (t < row_chunks + h.nrec)
                lds[wave >> 2].chunk[t < row_chunks ? t : kStageRowChunks + t - row_chunks] =
                    tb.gblob[h.off + t];
        }
    }
    // WAIT_VM: the caller issued loads that write LDS directly; they count as vector
    // memory operations, so wait for every one of them before the barrier
    if constexpr (WAIT_VM) __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (!live) return;
    if (h.nown > 0)
        decode_staged<Q>(tb, h.nown, s, lds[wave >> 2], j);
    else
        links_blocks_wave<Q>(tb, s, j);
}

// The fused step for a workgroup of W consecutive tiles (64 W threads) that first
// copies its own tiles' populations into LDS with coalesced loads: a link whose
// upstream site (or ghost slot) lies in those tiles reads LDS, any other reads
// global memory, so each wavefront's gathers touch only the lines of tiles outside
// the workgroup.  Block addressing, halfway walls.  Every thread calls it.  With DMA
// (FP32 storage) the copy uses loads that write LDS directly; pops must then be
// 16-byte aligned.
template <int Q, int ST, bool SC, bool BRINK, int W, bool DMA = false, bool FOUT = false>
__device__ inline void stream_collide_staged(const typename Store<ST>::T* __restrict__ src,
                                             typename Store<ST>::T* __restrict__ dst,
                                             const Table& tb, int32_t n, int32_t tiles_alloc,
                                             int32_t T0, float omega,
                                             const float* __restrict__ alpha, const Ghosts& G,
                                             int64_t t_next,
                                             typename Store<ST>::T (&pops)[W][Q][kTile],
                                             StageLds (&lds)[W / 4],
                                             typename Store<ST>::T* __restrict__ fout = nullptr) {
    using T = typename Store<ST>::T;
    using C = Codec<Q, ST, SC>;
    if (((int64_t)T0 << kTileShift) >= n) return;
    const int wave = (int)threadIdx.x >> kTileShift, lane = (int)threadIdx.x & (kTile - 1);
    const int32_t staged = min(W, tiles_alloc - T0);  // tiles of the array in this workgroup
    constexpr bool kDma = DMA && sizeof(T) == 4;
    if (wave < staged) {
        if constexpr (kDma) {
            // A tile's Q rows are one contiguous block, in memory as in LDS: copy it
            // with 16 bytes per lane per load, written straight into LDS (no
            // registers, no LDS store instructions).  The barrier in links_tiles
            // waits for these loads.
            constexpr int kBytes = Q * kTile * 4;
            const char* g = reinterpret_cast<const char*>(src + (int64_t)(T0 + wave) * (Q * kTile));
            char* l = reinterpret_cast<char*>(&pops[wave][0][0]);
#pragma unroll
            for (int c = 0; c < (kBytes + 1023) / 1024; ++c)
                if (c * 1024 + lane * 16 < kBytes)
                    __builtin_amdgcn_global_load_lds(g + c * 1024 + lane * 16, l + c * 1024, 16, 0, 0);
        } else {
            const int32_t s = ((T0 + wave) << kTileShift) + lane;
#pragma unroll
            for (int i = 0; i < Q; ++i) pops[wave][i][lane] = src[tix<Q>(i, s)];
        }
    }
    int32_t j[Q];
    links_tiles<Q, W, kDma>(tb, T0, n, lds, j);  // holds the barrier after the staging
    const int32_t s = (T0 << kTileShift) + (int32_t)threadIdx.x;
    if (s >= n) return;
    const int32_t lo = T0 << kTileShift;
    const uint32_t span = (uint32_t)staged << kTileShift;
    Pulled<Q> P;
    P.d[0] = C::dec(0, pops[wave][0][lane]);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        int dir;
        int32_t site;
        link_src(i, j[i], s, dir, site);
        const uint32_t r = (uint32_t)(site - lo);
        const T v = r < span ? pops[r >> kTileShift][dir][r & (kTile - 1)] : src[tix<Q>(dir, site)];
        P.d[i] = C::dec(i, v);
    }
    P.gmask = 0;
    P.gl = -1;
#if HLB_FUSE_GHOSTS
    int32_t top = j[1];
#pragma unroll
    for (int i = 2; i < Q; ++i) top = max(top, j[i]);
    if (top >= n) {
#pragma unroll
        for (int i = 1; i < Q; ++i)
            if (j[i] >= n) {
                if (P.gl < 0) P.gl = ghost_link<Q>(G, n, j[i], i);
                P.gmask |= 1u << i;
            }
    }
#endif
    site_collide_store<Q, ST, SC, BRINK, FOUT>(dst, n, omega, alpha, G, t_next, s, P, fout);
}

}  // namespace hlb
