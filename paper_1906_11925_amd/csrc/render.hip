// In-situ direct volume rendering of a lattice property by ray marching
// (paper Section 3.C.2: voxels sampled from a volume, viewing parameters and a
// transfer-function look-up table with steerable scale and offset).
//
// One thread per ray.  Sample positions are fixed-point integers (2^20 units per
// lattice spacing), so every ray visits exactly the voxels the definition names.
// Two sampling rules: the nearest voxel, or trilinear filtering as a texture unit
// does it (8-bit fractional weights, empty voxels zero); the trilinear weights
// are integers summing to 2^24 and each corner's product with its FP32 value is
// exact in FP64, so the filtered value is the same however the sum is evaluated
// (in corner order here).
// The volume is the sparse site list itself: a dense map of 4x4x4 blocks over the
// sites' bounding box gives each block's record (fluid mask, first site index),
// and a voxel's site is the block's first site plus the number of fluid positions
// before it.  A sample that falls in an empty block (or outside the map) jumps to
// the first sample past that block: exact integer arithmetic, so no contributing
// sample is ever skipped.  The work per sample is a few dependent loads from a
// small map (cache resident), so the kernel is bound by latency, not by HBM.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "lbdev.hpp"
#include "render.hpp"

namespace hlb {

constexpr int kRayTile = 16;  // rays per workgroup: 16 x 16
constexpr int64_t kFix = 1 << 20;

__device__ inline int64_t ceil_div_pos(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Value of the site at voxel x, if there is one.
__device__ inline bool voxel_value(const RenderVolume& V, const int64_t (&x)[3], float& val) {
    int64_t g[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g[a] = (x[a] >> 2) - V.blo[a];
        if (g[a] < 0 || g[a] >= V.gdim[a]) return false;
    }
    const int32_t blk = V.grid[(g[0] * V.gdim[1] + g[1]) * V.gdim[2] + g[2]];
    if (blk < 0) return false;
    const BlockRec r = V.rec[blk];
    const int p = block_pos((int)(x[0] & 3), (int)(x[1] & 3), (int)(x[2] & 3));
    const uint64_t m = block_mask(r);
    if (!((m >> p) & 1ull)) return false;
    val = V.values[r.off + __popcll(m & ((1ull << p) - 1ull))];
    return true;
}

// Composite one sample of value val.
__device__ inline void composite(const RenderView& v, const float4* __restrict__ lut, float val,
                                 float& c0, float& c1, float& c2, float& A) {
    const float t = (val - v.offset) * v.scale;
    const float f = floorf(t * 256.0f);
    const int e = f >= 255.0f ? 255 : (f > 0.0f ? (int)f : 0);
    const float4 rgba = lut[e];
    const float w = (1.0f - A) * rgba.w;
    c0 += w * rgba.x;
    c1 += w * rgba.y;
    c2 += w * rgba.z;
    A += w;
}

template <bool TRI>
__global__ __launch_bounds__(kRayTile* kRayTile) void k_render(RenderVolume V, RenderView v,
                                                                 const float4* __restrict__ lut,
                                                                 float4* __restrict__ image) {
    const int32_t i = (int32_t)(blockIdx.x * kRayTile + threadIdx.x % kRayTile);
    const int32_t j = (int32_t)(blockIdx.y * kRayTile + threadIdx.x / kRayTile);
    if (i >= v.width || j >= v.height) return;
    int64_t P0[3], D[3];  // start and step of ray (i, j)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        P0[a] = v.origin[a] + (int64_t)i * v.right[a] + (int64_t)j * v.up[a];
        D[a] = v.dir[a] + (int64_t)i * v.dir_right[a] + (int64_t)j * v.dir_up[a];
    }

    // samples that can reach a site: on each axis P must lie in
    // [4 lo FIX - FIX/2, 4 (lo + dim) FIX - FIX/2) for the nearest voxel, and in
    // [(4 lo - 1) FIX, 4 (lo + dim) FIX) for trilinear (base voxel or the next one
    // inside the map's box)
    int64_t k0 = 0, k1 = v.steps;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t lo = TRI ? (4 * (int64_t)V.blo[a] - 1) * kFix : 4 * (int64_t)V.blo[a] * kFix - kFix / 2;
        const int64_t hi = TRI ? 4 * ((int64_t)V.blo[a] + V.gdim[a]) * kFix
                               : 4 * ((int64_t)V.blo[a] + V.gdim[a]) * kFix - kFix / 2;  // exclusive
        const int64_t d = D[a];
        if (d == 0) {
            if (P0[a] < lo || P0[a] >= hi) k1 = 0;
        } else if (d > 0) {
            if (P0[a] < lo) k0 = max(k0, ceil_div_pos(lo - P0[a], d));
            k1 = P0[a] >= hi ? 0 : min(k1, ceil_div_pos(hi - P0[a], d));
        } else {
            if (P0[a] >= hi) k0 = max(k0, ceil_div_pos(P0[a] - (hi - 1), -d));
            k1 = P0[a] < lo ? 0 : min(k1, ceil_div_pos(P0[a] - (lo - 1), -d));
        }
    }

    float c0 = 0.f, c1 = 0.f, c2 = 0.f, A = 0.f;
    int64_t k = k0;
    if constexpr (TRI) {
        const int64_t nd1 = V.gdim[1] + 1, nd2 = V.gdim[2] + 1;
        while (k < k1) {
            int64_t b[3], B[3];
            int fr[3];
            bool in = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int64_t P = P0[a] + k * D[a];
                b[a] = P >> 20;                               // base voxel (floor)
                fr[a] = (int)((P - b[a] * kFix) >> 12);        // 8-bit fraction
                B[a] = b[a] >> 2;
                const int64_t h = B[a] - V.blo[a] + 1;
                in = in && h >= 0 && h <= V.gdim[a];
            }
            const bool reach =
                in && V.near[((B[0] - V.blo[0] + 1) * nd1 + (B[1] - V.blo[1] + 1)) * nd2 +
                             (B[2] - V.blo[2] + 1)] != 0;
            if (!reach) {
                // no corner of any sample whose base voxel lies in block B is a site:
                // jump to the first sample whose base voxel leaves B
                int64_t next = k1;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int64_t d = D[a];
                    if (d > 0)
                        next = min(next, ceil_div_pos((4 * B[a] + 4) * kFix - P0[a], d));
                    else if (d < 0)
                        next = min(next, ceil_div_pos(P0[a] - (4 * B[a] * kFix - 1), -d));
                }
                k = max(k + 1, next);
                continue;
            }
            double acc = 0.0;
            bool hit = false;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int64_t x[3] = {b[0] + (c & 1), b[1] + ((c >> 1) & 1), b[2] + ((c >> 2) & 1)};
                const int32_t W = ((c & 1) ? fr[0] : 256 - fr[0]) *
                                  (((c >> 1) & 1) ? fr[1] : 256 - fr[1]) *
                                  (((c >> 2) & 1) ? fr[2] : 256 - fr[2]);
                float val;
                if (W > 0 && voxel_value(V, x, val)) {
                    acc += (double)W * (double)val;  // exact product
                    hit = true;
                }
            }
            if (hit) composite(v, lut, (float)(acc * 0x1p-24), c0, c1, c2, A);
            ++k;
        }
        image[(int64_t)j * v.width + i] = make_float4(c0, c1, c2, A);
        return;
    }
    while (k < k1) {
        int64_t x[3], b[3];
        bool in = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            x[a] = (P0[a] + k * D[a] + kFix / 2) >> 20;  // nearest voxel (floor)
            b[a] = x[a] >> 2;
            const int64_t g = b[a] - V.blo[a];
            in = in && g >= 0 && g < V.gdim[a];
        }
        int32_t blk = -1;
        if (in)
            blk = V.grid[((b[0] - V.blo[0]) * V.gdim[1] + (b[1] - V.blo[1])) * V.gdim[2] +
                         (b[2] - V.blo[2])];
        if (blk < 0) {
            // empty block: jump to the first sample outside it on some axis
            int64_t next = k1;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int64_t d = D[a];
                if (d > 0) {
                    const int64_t e = (4 * b[a] + 4) * kFix - kFix / 2;
                    next = min(next, ceil_div_pos(e - P0[a], d));
                } else if (d < 0) {
                    const int64_t e = 4 * b[a] * kFix - kFix / 2 - 1;
                    next = min(next, ceil_div_pos(P0[a] - e, -d));
                }
            }
            k = max(k + 1, next);
            continue;
        }
        const BlockRec r = V.rec[blk];
        const int p = block_pos((int)(x[0] & 3), (int)(x[1] & 3), (int)(x[2] & 3));
        const uint64_t m = block_mask(r);
        if ((m >> p) & 1ull)
            composite(v, lut, V.values[r.off + __popcll(m & ((1ull << p) - 1ull))], c0, c1, c2, A);
        ++k;
    }
    image[(int64_t)j * v.width + i] = make_float4(c0, c1, c2, A);
}

__global__ __launch_bounds__(kBlock) void k_permute(const float* __restrict__ in,
                                                     const int32_t* __restrict__ perm, int64_t n,
                                                     float* __restrict__ out) {
    const int64_t m = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (m >= n) return;
    out[m] = in[perm ? perm[m] : m];
}

hipError_t launch_render(const RenderVolume& V, const RenderView& v, const float* lut, float* image,
                         hipStream_t s) {
    if (v.width <= 0 || v.height <= 0) return hipSuccess;
    const dim3 grid((unsigned)((v.width + kRayTile - 1) / kRayTile),
                    (unsigned)((v.height + kRayTile - 1) / kRayTile));
    if (v.filter == 1)
        k_render<true><<<grid, kRayTile * kRayTile, 0, s>>>(
            V, v, reinterpret_cast<const float4*>(lut), reinterpret_cast<float4*>(image));
    else
        k_render<false><<<grid, kRayTile * kRayTile, 0, s>>>(
            V, v, reinterpret_cast<const float4*>(lut), reinterpret_cast<float4*>(image));
    return hipGetLastError();
}

hipError_t launch_permute(const float* in, const int32_t* perm, int64_t n, float* out,
                          hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_permute<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(in, perm, n, out);
    return hipGetLastError();
}

}  // namespace hlb
