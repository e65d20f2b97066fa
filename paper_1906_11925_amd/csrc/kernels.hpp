// Internal launch interface between the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hlb {

constexpr int kBlock = 256;  // threads per block (4 wavefronts of 64)
constexpr int kTile = 64;    // sites per tile of the [tile][direction][64] layouts
constexpr int kTileShift = 6;

// Device copy of an iolet descriptor; harmonics live in a separate double array.
struct DevIolet {
    int32_t kind;      // 0 pressure, 1 velocity
    int32_t n_harm;
    int32_t harm_off;  // offset of cos (then sin) coefficients in the harmonic array
    int32_t pad;
    double mean;
    double period;
};

// One 4x4x4 block of the lattice in block addressing.  Positions inside a block
// are 6-bit Morton codes p (bits x0 y0 z0 x1 y1 z1), the order of the sites.
struct BlockRec {
    uint32_t mask_lo, mask_hi;  // fluid positions
    int32_t off;                // site index of the block's first fluid site
    int32_t goff;               // ghost index of its first ghost cell, -1: none
};

// How a site's links are found.  Decoded, a link names the source site (>= 0),
// bit 31 set for a wall link (the kernel then reads the opposite population of
// the site itself; the low 15 bits hold the interpolated-wall fraction, 0 for
// halfway bounce-back), or a ghost slot >= n holding the incoming population of
// an iolet link.  Three encodings:
//  * t32: neighbour table [ceil(n/64)][q-1][64] of those int32 values;
//  * t16 (compact): the same table in 16 bits: bit 15 = wall (bits 0..14 the
//    fraction); else bits 6..14 = slot in the tile's list of source tiles
//    tlist[toff[T] .. toff[T+1]) (at most 128 entries) and bits 0..5 = lane
//    within the source tile, source site = tlist[toff[T] + slot] * 64 + lane;
//  * brec (two-level block addressing, no per-link data): the lattice is cut into
//    4x4x4 blocks; a block record holds its fluid mask and first site index, so
//    the site at position p of block b is brec[b].off + popcount(mask below p).
//    bnbr[b][27] lists the ids of the 27 blocks around block b (index
//    (dx+1) + 3 (dy+1) + 9 (dz+1), -1 where no block exists, 13 = b itself);
//    tblock[T] is the block of the first site of tile T.  Positions past an iolet
//    plane that some link pulls from are ghost cells: gmask[b] marks them and the
//    g-th cell (block order, then position) holds its populations in slot n + g.
//    Blocks nfluid.. hold ghost cells only.  A position that is neither fluid nor
//    a ghost cell is a wall (halfway bounce-back).
//
//    For a fast decode every group of four tiles (256 sites, one workgroup) has a
//    staged copy of the records it needs, loaded into LDS with one coalesced read
//    per workgroup: grp[2g] = offset of group g's blob in 16-byte units, grp[2g+1]
//    = nown | nrec << 16 (nown = 0: the group uses the global records).  The blob
//    holds nown rows of kRowBytes bytes (the group's own blocks, consecutive ids
//    from the block of its first site; row k, byte d = index into the blob's
//    records of neighbour d of own block k; where no block exists it names an
//    empty record (no fluid, no ghost cells)), padded to 16 bytes,
//    then nrec BlockRecs whose first nown are the own blocks in order; in these
//    copies goff holds the block's id when it has ghost cells (-1 otherwise).
struct Table {
    const int32_t* t32;
    const uint16_t* t16;
    const int32_t* toff;
    const int32_t* tlist;
    const BlockRec* brec;
    const uint64_t* gmask;
    const int32_t* bnbr;
    const int32_t* tblock;
    const uint4* gblob;
    const int32_t* grp;
    int32_t nfluid;  // blocks holding fluid sites
    int32_t nblocks;
    int32_t n;       // fluid sites (the first ghost slot)
};

// capacity of a group's staged blob (groups beyond it use the global records)
constexpr int kRowBytes = 28;
constexpr int kStageRows = 24;
constexpr int kStageRowChunks = (kStageRows * kRowBytes + 15) / 16;
constexpr int kStageRecs = 160;
constexpr int kStageChunks = kStageRowChunks + kStageRecs;  // <= threads per workgroup

// Layout of one handle's device data, shared by all launches.  Populations are
// stored [slots/64][q][64] (sites, then ghost slots, Morton order).
struct Layout {
    int q;
    int storage;
    bool scaled;
    int64_t n;      // fluid sites
    int64_t slots;  // site + ghost slots per direction, a multiple of 64
    Table tb;
    bool bfl;       // some wall links carry an interpolated-wall fraction
    // with block addressing and halfway walls: workgroups of this many tiles (4, 8
    // or 16) copy their own populations into LDS first (0: four tiles, no copy)
    int stage_tiles;
    // FP32 staging copies with loads that write LDS directly
    bool lds_dma;
};

// Iolet links, sorted by site then direction.  Link l's incoming population lives
// in direction dir[l] of slot slot[l] (null: slot n + l, one slot per link, the
// table encodings; block addressing shares one ghost cell among the links that
// pull from the same position).
struct Ghosts {
    int64_t count;
    const int32_t* slot;
    const int32_t* cell_link;  // with shared ghost cells: [cells][q] link pulling (cell, i), or -1
    const int32_t* site;   // Morton site index of each iolet link
    const uint8_t* dir;    // direction of the link
    const uint8_t* iolet;  // iolet id
    const float* coef;     // 6 w_i (c_i . e_k) W_s for velocity links, else 0
    const DevIolet* iolets;
    const double* harm;
    const double* vals;    // iolet values per step: vals[(t - vals_t0) * n_iolets + k]
    int64_t vals_t0;
    int32_t n_iolets;
    // Fourier basis of velocity iolets per step (adjoint only, else null):
    // basis[((t - vals_t0) * n_iolets + k) * basis_stride + 2 (h - 1) + {0, 1}] =
    // cos, sin of 2 pi h t / period_k for h = 1 .. n_harm_k
    const double* basis;
    int32_t basis_stride;
};

// vals[m * n_iolets + k] = value of iolet k at time t0 + m, for m < count; with
// basis != null also the Fourier basis of velocity iolets (layout as Ghosts::basis)
hipError_t launch_iolet_series(const DevIolet* iolets, const double* harm, int32_t n_iolets,
                               int64_t t0, int64_t count, double* vals, double* basis,
                               int32_t basis_stride, hipStream_t s);

hipError_t launch_ghost_fill(const Layout& L, const Ghosts& G, void* A, int64_t t,
                             hipStream_t s);

// xcd_group: consecutive workgroups per XCD in the workgroup-to-tile mapping (0:
// identity).  When ghosts_fused(), the kernel also fills dst's ghost slots for
// time t_next.  fout (optional, same layout and storage as dst; FP32 storage and
// halfway walls only, else hipErrorInvalidValue): also receives the step's
// pre-collision populations f, for the reverse sweep.
hipError_t launch_stream_collide(const Layout& L, const Ghosts& G, const void* src, void* dst,
                                 float omega, const float* alpha, int xcd_group, int64_t t_next,
                                 hipStream_t s, void* fout = nullptr);
bool ghosts_fused();

// streamed != 0: gather pre-collision populations from `A` (the previous buffer,
// ghosts included); 0: use the populations of `A` in place.
hipError_t launch_observables(const Layout& L, const void* A, int streamed, float omega,
                              const int32_t* perm, const float* normal, float* p, float* u,
                              float* wss, hipStream_t s);

// FP64 totals of the stored state into out[4]; sets *flag = 1 on a non-finite value.
hipError_t launch_totals(const Layout& L, const void* A, double* partial, int64_t nparts,
                         double* out, int32_t* flag, hipStream_t s);
int64_t totals_parts(int64_t n);

// The same totals with the partial sums in a per-GPU static scratch array of
// totals_scratch_parts() blocks (no allocation, no synchronisation); `out` is a
// device double[4].  Calls that overlap on one GPU share the array.
hipError_t launch_totals_noalloc(const Layout& L, const void* A, double* out, hipStream_t s);
int64_t totals_scratch_parts();

// mode 0: raw get, 1: raw set, 2: decoded get (float), 3: decoded set (float)
hipError_t launch_state(const Layout& L, void* A, void* ext, const int32_t* perm, int mode,
                        hipStream_t s);

// fill every population of A (all directions, sites and ghosts) with deviation 0
hipError_t launch_zero(const Layout& L, void* A, hipStream_t s);

hipError_t launch_copy(void* dst, const void* src, int64_t bytes, hipStream_t s);

// fill `words` 32-bit words with zero
hipError_t launch_zero_words(void* p, int64_t words, hipStream_t s);

}  // namespace hlb
