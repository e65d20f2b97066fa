// Internal launch interface of the volume renderer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace hlb {

// Block map of the rendered volume: grid[(gx * gdim[1] + gy) * gdim[2] + gz] is the
// record index of block (blo + g), or -1 where no site lies; rec[k] holds that
// block's fluid mask and first site; values holds one value per site (site order).
// near[(hx * (gdim[1] + 1) + hy) * (gdim[2] + 1) + hz] is nonzero when a block among
// (blo - 1 + h) + {0, 1}^3 holds a site: the blocks a trilinear sample whose base
// voxel lies in block blo - 1 + h can reach.
struct RenderVolume {
    const int32_t* grid;
    const BlockRec* rec;
    const float* values;
    const uint8_t* near;
    int32_t blo[3];
    int32_t gdim[3];
};

// Fixed-point view (2^20 units per lattice spacing), as in hemelb_view_t.
struct RenderView {
    int64_t origin[3];
    int64_t right[3];
    int64_t up[3];
    int64_t dir[3];
    int64_t dir_right[3], dir_up[3];  // ray (i, j) steps dir + i dir_right + j dir_up
    int32_t width, height, steps;
    float scale, offset;
    int32_t filter;  // 0: nearest voxel, 1: trilinear
};

// image [height][width][4] of the volume seen through view v; lut: device [256][4]
hipError_t launch_render(const RenderVolume& V, const RenderView& v, const float* lut, float* image,
                         hipStream_t s);

// out[m] = in[perm[m]] (perm null: identity), m < n
hipError_t launch_permute(const float* in, const int32_t* perm, int64_t n, float* out,
                          hipStream_t s);

}  // namespace hlb
