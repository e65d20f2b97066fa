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

// ---- two-level block addressing -------------------------------------------
__device__ inline uint64_t block_mask(const BlockRec& r) {
    return ((uint64_t)r.mask_hi << 32) | (uint64_t)r.mask_lo;
}

// position of the set bit of rank r (counted from 0) of m; the result stays in
// [0, 63] for any m and r
__device__ inline int select_bit(uint64_t m, int r) {
    uint32_t x = (uint32_t)m;
    int p = 0;
    int c = __popc(x);
    if (r >= c) {
        r -= c;
        x = (uint32_t)(m >> 32);
        p = 32;
    }
    c = __popc(x & 0xffffu);
    if (r >= c) {
        r -= c;
        x >>= 16;
        p += 16;
    }
    c = __popc(x & 0xffu);
    if (r >= c) {
        r -= c;
        x >>= 8;
        p += 8;
    }
    c = __popc(x & 0xfu);
    if (r >= c) {
        r -= c;
        x >>= 4;
        p += 4;
    }
    c = __popc(x & 0x3u);
    if (r >= c) {
        r -= c;
        x >>= 2;
        p += 2;
    }
    if (r >= (int)(x & 1u)) p += 1;
    return p;
}

// 6-bit Morton position of local coordinates (x, y, z) in [0, 4)^3
__device__ inline int block_pos(int x, int y, int z) {
    return (x & 1) | ((y & 1) << 1) | ((z & 1) << 2) | ((x & 2) << 2) | ((y & 2) << 3) |
           ((z & 2) << 4);
}

// Links j[1..Q-1] of the site at local coordinates (bx, by, bz) of block bl.
template <int Q>
__device__ inline void block_links(const Table& tb, int32_t bl, int bx, int by, int bz,
                                   int32_t (&j)[Q]) {
    using Lt = Lat<Q>;
    const int32_t* nb = tb.bnbr + (int64_t)bl * 27;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int ux = bx - Lt::cx[i], uy = by - Lt::cy[i], uz = bz - Lt::cz[i];  // in [-1, 4]
        const int d = ((ux >> 2) + 1) + 3 * ((uy >> 2) + 1) + 9 * ((uz >> 2) + 1);
        const int32_t b2 = nb[d];
        int32_t v = (int32_t)0x80000000u;  // wall
        if (b2 >= 0) {
            const BlockRec r = tb.brec[b2];
            const uint64_t m = block_mask(r);
            const int p = block_pos(ux & 3, uy & 3, uz & 3);
            const uint64_t below = (1ull << p) - 1ull;
            if ((m >> p) & 1ull) {
                v = r.off + __popcll(m & below);
            } else if (r.goff >= 0) {
                const uint64_t g = tb.gmask[b2];
                if ((g >> p) & 1ull) v = tb.n + r.goff + __popcll(g & below);
            }
        }
        j[i] = v;
    }
}

// the site's block bl (given a first guess b0 <= bl) and its local coordinates
__device__ inline void block_site(const Table& tb, int32_t s, int32_t bl, int& bx, int& by,
                                  int& bz) {
    const BlockRec r = tb.brec[bl];
    const int p = select_bit(block_mask(r), s - r.off);
    bx = (p & 1) | ((p >> 2) & 2);
    by = ((p >> 1) & 1) | ((p >> 3) & 2);
    bz = ((p >> 2) & 1) | ((p >> 4) & 2);
}

// Wave form: the blocks that the tile's sites fall into are found with
// wave-uniform loads of their first-site offsets.
template <int Q>
__device__ inline void links_blocks_wave(const Table& tb, int32_t s, int32_t (&j)[Q]) {
    const int32_t T = __builtin_amdgcn_readfirstlane(s >> kTileShift);
    const int32_t end = (T + 1) << kTileShift;
    const int32_t b0 = tb.tblock[T];
    int32_t bl = b0;
    for (int32_t b = b0 + 1; b < tb.nfluid; ++b) {
        const int32_t o = tb.brec[b].off;
        if (o >= end) break;
        if (s >= o) bl = b;
    }
    int bx, by, bz;
    block_site(tb, s, bl, bx, by, bz);
    block_links<Q>(tb, bl, bx, by, bz, j);
}

// LDS of one workgroup for the staged block records
struct StageLds {
    uint4 chunk[kStageChunks];
};

// A group's staged blob: where it starts and how many own blocks and records it
// holds (nown = 0: the group's records did not fit and its links decode from the
// global records).  Uniform over the workgroup.
struct StageHdr {
    int32_t off;
    int nown, nrec;
};

// The group entries never change during a launch: read them through the constant
// address space, so that they come in through the scalar cache even after the
// kernel has stored populations (a vector load would have to wait for those
// stores before its value could be used).
__device__ inline StageHdr stage_header(const Table& tb, int32_t g) {
    const __attribute__((address_space(4))) int32_t* grp =
        (const __attribute__((address_space(4))) int32_t*)tb.grp;
    const int32_t cnt = grp[2 * g + 1];
    return StageHdr{grp[2 * g], cnt & 0xffff, cnt >> 16};
}

// One thread's share of staging a blob: at most one 16-byte chunk and its LDS slot
// (-1: none).  Fetching and committing are separate so that a workgroup can load
// the next group's blob while it works on the current one.
struct StageChunk {
    uint4 v;
    int dst;
};

__device__ inline StageChunk stage_fetch(const Table& tb, const StageHdr& h) {
    StageChunk c;
    c.dst = -1;
    c.v = make_uint4(0u, 0u, 0u, 0u);
    if (h.nown == 0) return c;
    const int row_chunks = (h.nown * kRowBytes + 15) >> 4;
    const int t = (int)threadIdx.x;
    if (t < row_chunks + h.nrec) {
        c.v = tb.gblob[h.off + t];
        c.dst = t < row_chunks ? t : kStageRowChunks + t - row_chunks;
    }
    return c;
}

__device__ inline void stage_commit(const StageChunk& c, StageLds& lds) {
    if (c.dst >= 0) lds.chunk[c.dst] = c.v;
}

// Links of site s from its group's staged blob in LDS (nown > 0 own blocks).  All
// lanes of the wavefront call it (the own-block search is wave-uniform in its
// bounds).  Per link: the row byte names the neighbour block's staged record; a
// fluid position ranks in its mask; any other position is a wall unless the block
// has ghost cells and the position is one (global ghost masks; rare, only next to
// iolet planes).
template <int Q>
__device__ inline void decode_staged(const Table& tb, int nown, int32_t s, const StageLds& lds,
                                     int32_t (&j)[Q]) {
    using Lt = Lat<Q>;
    const uint8_t* rows = reinterpret_cast<const uint8_t*>(lds.chunk);
    const BlockRec* recs = reinterpret_cast<const BlockRec*>(lds.chunk + kStageRowChunks);
    // own block: the last one whose first site is at or before s (offsets ascend;
    // only blocks starting inside this wavefront's tile can change the answer)
    const int32_t last = __builtin_amdgcn_readfirstlane(s | (kTile - 1));
    int k = 0;
    for (int q = 1; q < nown; ++q) {
        const int32_t o = recs[q].off;
        if (o > last) break;
        if (s >= o) k = q;
    }
    const BlockRec own = recs[k];
    const int p = select_bit(block_mask(own), s - own.off);
    const int bx = (p & 1) | ((p >> 2) & 2);
    const int by = ((p >> 1) & 1) | ((p >> 3) & 2);
    const int bz = ((p >> 2) & 1) | ((p >> 4) & 2);
    const uint8_t* row = rows + k * kRowBytes;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int ux = bx - Lt::cx[i], uy = by - Lt::cy[i], uz = bz - Lt::cz[i];  // in [-1, 4]
        const int d = ((ux >> 2) + 1) + 3 * ((uy >> 2) + 1) + 9 * ((uz >> 2) + 1);
        const int pp = block_pos(ux & 3, uy & 3, uz & 3);
        const BlockRec r = recs[row[d]];
        const uint32_t sh = (uint32_t)pp & 31u;
        const bool upper = pp >= 32;
        const uint32_t w = upper ? r.mask_hi : r.mask_lo;
        const int rank = __popc(w & ((1u << sh) - 1u)) + (upper ? __popc(r.mask_lo) : 0);
        const bool fluid = (w >> sh) & 1u;
        int32_t v = fluid ? r.off + rank : (int32_t)0x80000000u;
        if (!fluid && r.goff >= 0) {
            const int32_t b2 = r.goff;
            const uint64_t gm = tb.gmask[b2];
            if ((gm >> pp) & 1ull)
                v = tb.n + tb.brec[b2].goff + __popcll(gm & ((1ull << pp) - 1ull));
        }
        j[i] = v;
    }
}

// Links of the sites of one 256-thread workgroup (group g = four consecutive
// tiles) from the group's staged block records.  Every thread of the workgroup
// calls it (it holds a barrier); `live`: the thread's wavefront has sites.
template <int Q>
__device__ inline void links_blocks_group(const Table& tb, int32_t g, int32_t s, bool live,
                                          StageLds& lds, int32_t (&j)[Q]) {
    const StageHdr h = stage_header(tb, g);
    if (h.nown == 0) {  // the group's records did not fit: global records
        if (live) links_blocks_wave<Q>(tb, s, j);
        return;
    }
    stage_commit(stage_fetch(tb, h), lds);
    __syncthreads();
    if (live) decode_staged<Q>(tb, h.nown, s, lds, j);
}

// Links of site s in a kernel whose 256-thread workgroups each cover one group g
// of four consecutive tiles (s = 256 g + thread).  Every thread of the workgroup
// calls it; `live`: the thread's wavefront has sites (the others only help stage).
template <int Q, bool NT>
__device__ inline void links_group(const Table& tb, int32_t g, int32_t s, bool live,
                                   StageLds& lds, int32_t (&j)[Q]);

// Wave form of the link decode (all lanes of a wavefront call it); block
// addressing decodes from the global records here (see links_group).
template <int Q, bool NT>
__device__ inline void links_wave(const Table& tb, int32_t s, int32_t (&j)[Q]) {
    if (tb.brec) {
        links_blocks_wave<Q>(tb, s, j);
        return;
    }
    uint32_t c[Q];
    int32_t e0, e1;
    load_codes<Q, NT>(tb, s, c, e0, e1);
    decode_codes<Q>(tb, s, c, e0, e1, j);
}

template <int Q, bool NT>
__device__ inline void links_group(const Table& tb, int32_t g, int32_t s, bool live,
                                   StageLds& lds, int32_t (&j)[Q]) {
    if (tb.grp) {
        links_blocks_group<Q>(tb, g, s, live, lds, j);
        return;
    }
    if (live) links_wave<Q, NT>(tb, s, j);
}

// All links of an arbitrary site (no lane exchange; any lane may call it).
template <int Q>
__device__ inline void links_site(const Table& tb, int32_t s, int32_t (&j)[Q]) {
    if (tb.brec) {
        int32_t bl = tb.tblock[s >> kTileShift];
        while (bl + 1 < tb.nfluid && tb.brec[bl + 1].off <= s) ++bl;
        int bx, by, bz;
        block_site(tb, s, bl, bx, by, bz);
        block_links<Q>(tb, bl, bx, by, bz, j);
        return;
    }
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (tb.t16 == nullptr) {
            j[i] = tb.t32[tix<Q - 1>(i - 1, s)];
            continue;
        }
        const uint32_t c = tb.t16[tix<Q - 1>(i - 1, s)];
        if (c & 0x8000u) {
            j[i] = (int32_t)(0x80000000u | (c & 0x7fffu));
        } else {
            const int32_t tile =
                tb.tlist[tb.toff[s >> kTileShift] + (int)((c >> kTileShift) & 0x1ffu)];
            j[i] = (tile << kTileShift) | (int32_t)(c & (kTile - 1));
        }
    }
}

// slot holding the incoming population of iolet link l
__device__ inline int32_t ghost_slot(const Ghosts& G, int32_t n, int64_t l) {
    return G.slot ? G.slot[l] : n + (int32_t)l;
}

// iolet link that pulls direction i from ghost slot `slot`
template <int Q>
__device__ inline int64_t ghost_link(const Ghosts& G, int32_t n, int32_t slot, int i) {
    return G.slot ? (int64_t)G.cell_link[(int64_t)(slot - n) * Q + i] : (int64_t)(slot - n);
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
