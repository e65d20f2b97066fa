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

// Neighbour table, [ceil(n/64)][q-1][64].  Decoded, a link names the source
// site (>= 0), the site itself with bit 31 set for a bounce-back wall link, or
// n + l for ghost slot l.  Two encodings:
//  * t32: that int32 value directly;
//  * t16 (compact): bit 15 = wall; bits 6..14 = slot in the tile's list of source
//    tiles tlist[toff[T] .. toff[T+1]) (at most 128 entries); bits 0..5 = lane
//    within the source tile.  Source site = tlist[toff[T] + slot] * 64 + lane.
struct Table {
    const int32_t* t32;
    const uint16_t* t16;
    const int32_t* toff;
    const int32_t* tlist;
};

// Layout of one handle's device data, shared by all launches.  Populations are
// stored [slots/64][q][64] (sites, then ghost slots, Morton order).
struct Layout {
    int q;
    int storage;
    bool scaled;
    int64_t n;      // fluid sites
    int64_t slots;  // site + ghost slots per direction, a multiple of 64
    Table tb;
};

struct Ghosts {
    int64_t count;
    const int32_t* site;   // Morton site index of each iolet link
    const uint8_t* dir;    // direction of the link
    const uint8_t* iolet;  // iolet id
    const float* coef;     // 6 w_i (c_i . e_k) W_s for velocity links, else 0
    const DevIolet* iolets;
    const double* harm;
    const double* vals;    // iolet values per step: vals[(t - vals_t0) * n_iolets + k]
    int64_t vals_t0;
    int32_t n_iolets;
};

// vals[m * n_iolets + k] = value of iolet k at time t0 + m, for m < count
hipError_t launch_iolet_series(const DevIolet* iolets, const double* harm, int32_t n_iolets,
                               int64_t t0, int64_t count, double* vals, hipStream_t s);

hipError_t launch_ghost_fill(const Layout& L, const Ghosts& G, void* A, int64_t t,
                             hipStream_t s);

// xcd_group: consecutive blocks per XCD in the block-to-tile mapping (0: identity).
// When ghosts_fused(), the kernel also fills dst's ghost slots for time t_next.
hipError_t launch_stream_collide(const Layout& L, const Ghosts& G, const void* src, void* dst,
                                 float omega, const float* alpha, int xcd_group, int64_t t_next,
                                 hipStream_t s);
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

// mode 0: raw get, 1: raw set, 2: decoded get (float), 3: decoded set (float)
hipError_t launch_state(const Layout& L, void* A, void* ext, const int32_t* perm, int mode,
                        hipStream_t s);

// fill every population of A (all directions, sites and ghosts) with deviation 0
hipError_t launch_zero(const Layout& L, void* A, hipStream_t s);

hipError_t launch_copy(void* dst, const void* src, int64_t bytes, hipStream_t s);

// fill `words` 32-bit words with zero
hipError_t launch_zero_words(void* p, int64_t words, hipStream_t s);

}  // namespace hlb
