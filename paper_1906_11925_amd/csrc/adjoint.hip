// Discrete adjoint of the sparse LBGK step, and the objective it differentiates.
//
// Objective (over a window W of steps; step t maps A_t to A_{t+1} through the
// pre-collision populations f_t):
//   J = sum_{t in W} (Q(t) - Q*)^2 + lam * mean_{t in W} mean_{s in D} WSS_s(f_t),
//   Q(t) = sum over the outlet's iolet links (s, i) of A_t[opp(i)][s] - f_t[i][s].
//
// The reverse sweep runs in pull form, one thread per site, and each kernel writes
// only the rows of its own sites:
//  * the stream transpose: population k of site s was read in the forward by the
//    link opp(k) of s pulling the other way (from the site s + c_k), by s itself
//    across a wall (bounce-back), or, across an iolet, by nobody; so
//    dJ/dA_t[k][s] gathers fhat_t = dJ/df_t along the site's own decoded links,
//    with the direction reversed.  The forward's table validation guarantees that
//    links pair up this way.
//  * at a site with iolet links the same thread turns the adjoints of the values
//    those links pulled (the incoming iolet populations) into their sources: the
//    Ladd term sends its adjoint to the site's opposite population and (times its
//    coefficient and the tabulated Fourier basis) to the inlet coefficients; the
//    pressure equilibrium sends it to all of the site's own populations through
//    u(A_t[:, s]); the outlet flux term of the objective enters here too.
//  * the transposed collision Jacobian at the taped state of the previous step,
//      fhat_j = (1 - omega) g_j + omega (a + c_j . b),
//      a = sum_i g_i dfeq_i/drho, b = sum_i g_i dfeq_i/dm  (Brinkman-aware),
//    plus the wall-shear objective term, and dJ/dalpha_s accumulated in FP64.
// The first two are the transpose of step t + 1 and the third that of step t, so one
// kernel covers parts of two steps: fhat_{t+1} -> fhat_t.  A segment starts from
// ghat (its first kernel skips the gather) and ends with a kernel that applies the
// stream transpose alone, so the sweep holds dJ/dA_t between segments.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "adjoint.hpp"
#include "kernels.hpp"
#include "lattice.hpp"
#include "lbdev.hpp"
#include "step.hpp"

namespace hlb {

constexpr int kObjParts = 256;  // most blocks of the objective's partial sums

// pre-collision populations (deviations) of site s from a state with filled
// ghosts, given its decoded links j
template <int Q, int ST, bool SC>
__device__ inline void gather_pre(const typename Store<ST>::T* __restrict__ A, int32_t s,
                                  int32_t n, float (&d)[Q], int32_t (&j)[Q]) {
    using C = Codec<Q, ST, SC>;
    j[0] = s;
    d[0] = C::dec(0, A[tix<Q>(0, s)]);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        int dir;
        int32_t site;
        link_src(i, j[i], s, dir, site);
        d[i] = C::dec(i, A[tix<Q>(dir, site)]);
    }
    apply_bfl<Q, ST, SC>(A, s, n, j, d);
}

// traction tangential to the wall, t = sigma n - (n.sigma n) n, with
// sigma = -(1 - omega/2) sum_i c_i c_i (f_i - f_i^eq(rho, u))
template <int Q>
__device__ inline void shear(const float (&d)[Q], float drho, float ux, float uy, float uz,
                             float omega, float nx, float ny, float nz, float& tx, float& ty,
                             float& tz) {
    using Lt = Lat<Q>;
    float deq[Q];
    eq_dev<Q>(drho, 1.0f + drho, ux, uy, uz, deq);
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
    tx = sx - nsn * nx;
    ty = sy - nsn * ny;
    tz = sz - nsn * nz;
}

__device__ inline double block_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double r = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += red[w];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// forward objective terms of one step: Q(t) and sum over D of WSS(f_t).  Each
// block sums a fixed share of the outlet links and dome sites (a grid-stride
// loop, then a fixed reduction tree) into part[2 b], part[2 b + 1]; a second
// kernel adds the partials in block order, so the result is deterministic.
// ---------------------------------------------------------------------------
template <int Q, int ST, bool SC>
__global__ __launch_bounds__(kBlock) void k_objective(
    const typename Store<ST>::T* __restrict__ A, Table tb, int32_t n,
    Ghosts G, const int32_t* __restrict__ out_links, int32_t n_out,
    const int32_t* __restrict__ dome, int32_t n_dome, const float* __restrict__ normal,
    float omega, double* __restrict__ part) {
    using C = Codec<Q, ST, SC>;
    __shared__ double red[kBlock / 64];
    double q = 0.0, w = 0.0;
    const int64_t items = (int64_t)n_out + n_dome;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < items;
         k += (int64_t)gridDim.x * kBlock) {
        if (k < n_out) {
            const int32_t l = out_links[k];
            const int32_t s = G.site[l];
            const int i = G.dir[l];
            const int o = opp(i);
            q += (double)C::dec(o, A[tix<Q>(o, s)]) -
                 (double)C::dec(i, A[tix<Q>(i, ghost_slot(G, n, l))]);
        } else {
            const int32_t s = dome[k - n_out];
            float d[Q];
            int32_t j[Q];
            links_site<Q>(tb, s, j);
            gather_pre<Q, ST, SC>(A, s, n, d, j);
            float drho, mx, my, mz;
            moments<Q>(d, drho, mx, my, mz);
            const float ir = 1.0f / (1.0f + drho);
            float tx, ty, tz;
            shear<Q>(d, drho, mx * ir, my * ir, mz * ir, omega, normal[s], normal[n + s],
                     normal[2 * (int64_t)n + s], tx, ty, tz);
            w += sqrtf(tx * tx + ty * ty + tz * tz);
        }
    }
    const double qs = block_sum(q, red);
    const double ws = block_sum(w, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = qs;
        part[2 * blockIdx.x + 1] = ws;
    }
}

// one wavefront: lane k adds partials k, k + 64, ... in order, then a fixed
// butterfly over the lanes
__global__ __launch_bounds__(64) void k_objective_final(const double* __restrict__ part,
                                                        int32_t nparts, double* __restrict__ q_out,
                                                        double* __restrict__ w_out) {
    double q = 0.0, w = 0.0;
    for (int32_t b = (int32_t)threadIdx.x; b < nparts; b += 64) {
        q += part[2 * b];
        w += part[2 * b + 1];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        q += __shfl_xor(q, off, 64);
        w += __shfl_xor(w, off, 64);
    }
    if (threadIdx.x == 0) {
        *q_out = q;
        *w_out = w;
    }
}

// ---------------------------------------------------------------------------
// iolet terms of the stream transpose (called by the site's own thread)
// ---------------------------------------------------------------------------
// Adds to g the adjoint that the values pulled by the iolet links of site s (at
// the step whose ghosts were filled from A) send to the site's own populations of
// A, and accumulates the inlet-coefficient adjoints.  fh: dJ/df of that step.
template <int Q, int ST, bool SC>
__device__ inline void iolet_terms(const typename Store<ST>::T* __restrict__ A, int32_t s,
                                   const int32_t (&j)[Q], const float* __restrict__ fh,
                                   const Ghosts& G, const IoletAdj& I, int64_t kis, int32_t n,
                                   float (&g)[Q]) {
    using C = Codec<Q, ST, SC>;
    using Lt = Lat<Q>;
    float d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = C::dec(i, A[tix<Q>(i, s)]);
    float drho, mx, my, mz;
    moments<Q>(d, drho, mx, my, mz);
    const float rA = 1.0f + drho;
    const float ir = 1.0f / rA;
    const float ux = mx * ir, uy = my * ir, uz = mz * ir;
    const double qbar = I.q_index >= 0 ? 2.0 * (I.q_tape[I.q_index] - I.q_target) : 0.0;
    float acc[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) acc[i] = 0.f;
    // the site's iolet links are consecutive in the link list, in direction order
    int64_t l = I.S.lo[kis];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (j[i] < n) continue;
        const int o = opp(i);
        const int kio = G.iolet[l];
        const DevIolet io = G.iolets[kio];
        const int64_t step = ((int64_t)I.t - G.vals_t0) * G.n_iolets + kio;
        float gh = fh[tix<Q>(i, s)];  // adjoint of the incoming value the link pulled
        if (kio == I.outlet && I.q_index >= 0) {
            gh -= (float)qbar;
            acc[o] += (float)qbar;
        }
        if (io.kind == 1) {
            acc[o] += gh;
            // d value / d(mean, cos_h, sin_h), with the basis tabulated for this step
            const double c = (double)gh * (double)G.coef[l];
            double* th = I.theta_acc + l * I.nbasis;
            const double* bs = G.basis + step * G.basis_stride;
            th[0] += c;
            for (int h = 1; h <= io.n_harm; ++h) {
                th[h] += c * bs[2 * (h - 1)];
                th[io.n_harm + h] += c * bs[2 * (h - 1) + 1];
            }
        } else {
            const float rk = (float)G.vals[step];
            const float cix = Lt::cx[i], ciy = Lt::cy[i], ciz = Lt::cz[i];
            const float cu = cix * ux + ciy * uy + ciz * uz;
            const float sc = Lt::w[i] * rk;
            const float gx = sc * (3.0f * cix + 9.0f * cu * cix - 3.0f * ux);
            const float gy = sc * (3.0f * ciy + 9.0f * cu * ciy - 3.0f * uy);
            const float gz = sc * (3.0f * ciz + 9.0f * cu * ciz - 3.0f * uz);
            const float gi = gh * ir;
#pragma unroll
            for (int jd = 0; jd < Q; ++jd)
                acc[jd] += gi * ((Lt::cx[jd] - ux) * gx + (Lt::cy[jd] - uy) * gy + (Lt::cz[jd] - uz) * gz);
        }
        ++l;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) g[i] += acc[i];
}

// ---------------------------------------------------------------------------
// one reverse kernel (group grp of four tiles; every thread of the workgroup
// calls it).  A: taped state of the collision step (ADJ_OWN, ADJ_PULL), whose
// pre-collision populations f_t the kernel re-gathers, unless F (uniform) holds
// them already, as the recording forward stored them in the sites' own slots; Ai:
// taped state of the stream step (ADJ_PULL, ADJ_FINAL).
// ---------------------------------------------------------------------------
template <int Q, int ST, bool SC, bool BRINK, int MODE>
__device__ inline void adj_group(
    const typename Store<ST>::T* __restrict__ A, const typename Store<ST>::T* __restrict__ F,
    const typename Store<ST>::T* __restrict__ Ai,
    const float* __restrict__ gin, float* __restrict__ gout, const Table& tb, int32_t n,
    float omega, const float* __restrict__ alpha, double* __restrict__ alpha_hat,
    const float* __restrict__ wss_w, const float* __restrict__ normal, const Ghosts& G,
    const IoletAdj& I, int32_t grp, StageLds& lds) {
    using Lt = Lat<Q>;
    static_assert(kBlock == 4 * kTile, "a workgroup covers one group of four tiles");
    if ((int64_t)grp * kBlock >= n) return;  // the whole workgroup lies past the end
    const int32_t s = grp * kBlock + threadIdx.x;
    const bool live = (s & ~(kTile - 1)) < n;
    const bool mine = live && s < n;
    float g[Q];
    // per-site inputs that do not depend on the links: issue their loads before the
    // link decode so the two latencies overlap
    if constexpr (MODE == ADJ_OWN) {
#pragma unroll
        for (int i = 0; i < Q; ++i) g[i] = mine ? gin[tix<Q>(i, s)] : 0.f;
    }
    const float keep = BRINK && mine && MODE != ADJ_FINAL ? 1.0f - alpha[s] : 1.0f;
    const float ws = wss_w && mine && MODE != ADJ_FINAL ? wss_w[s] : 0.f;
    int32_t j[Q];
    links_group<Q, false>(tb, grp, s, live, lds, j);
    if (!mine) return;
    if constexpr (MODE != ADJ_OWN) {
        // stream transpose: the link i of s pulled population i from j[i], so the
        // population opp(i) of s went to j[i] (its link i pulled the other way), or
        // was bounced back into the site's own direction i, or left through an iolet
        g[0] = gin[tix<Q>(0, s)];
        int32_t top = j[1];  // walls are negative, sites below n, ghost slots from n
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int o = opp(i);
            top = max(top, j[i]);
            g[o] = j[i] >= n ? 0.f : gin[j[i] < 0 ? tix<Q>(i, s) : tix<Q>(o, j[i])];
        }
        if (top >= n) {
            int64_t l = -1;
#pragma unroll
            for (int i = 1; i < Q; ++i)
                if (l < 0 && j[i] >= n) l = ghost_link<Q>(G, n, j[i], i);
            iolet_terms<Q, ST, SC>(Ai, s, j, gin, G, I, I.link_is[l], n, g);
        }
    }
    if constexpr (MODE == ADJ_FINAL) {
#pragma unroll
        for (int i = 0; i < Q; ++i) gout[tix<Q>(i, s)] = g[i];
        return;
    } else {
        using C = Codec<Q, ST, SC>;
        float d[Q];
        if (F) {
#pragma unroll
            for (int i = 0; i < Q; ++i) d[i] = C::dec(i, F[tix<Q>(i, s)]);
        } else {
            gather_pre<Q, ST, SC>(A, s, n, d, j);
        }
        float drho, mx, my, mz;
        moments<Q>(d, drho, mx, my, mz);
        const float rho = 1.0f + drho;
        const float ir = 1.0f / rho;
        const float ux = mx * ir, uy = my * ir, uz = mz * ir;
        const float bx = keep * ux, by = keep * uy, bz = keep * uz;
        const float ub2 = bx * bx + by * by + bz * bz;
        const float ubu = bx * ux + by * uy + bz * uz;
        // a = sum g_i dfeq_i/drho,  b = sum g_i dfeq_i/dm,  alpha term
        float a = 0.f, b0 = 0.f, b1 = 0.f, b2 = 0.f, ga = 0.f;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const float cx = Lt::cx[i], cy = Lt::cy[i], cz = Lt::cz[i];
            const float cub = cx * bx + cy * by + cz * bz;
            const float cu = cx * ux + cy * uy + cz * uz;
            const float wg = Lt::w[i] * g[i];
            a += wg * (1.0f - 4.5f * cub * cub + 1.5f * ub2);
            const float t = wg * (3.0f + 9.0f * cub);
            b0 += t * cx - 3.0f * wg * bx;
            b1 += t * cy - 3.0f * wg * by;
            b2 += t * cz - 3.0f * wg * bz;
            if constexpr (BRINK) ga += wg * (3.0f * cu + 9.0f * cub * cu - 3.0f * ubu);
        }
        b0 *= keep;
        b1 *= keep;
        b2 *= keep;
        if constexpr (BRINK) alpha_hat[s] += (double)(-omega * rho * ga);

        float fh[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i)
            fh[i] = (1.0f - omega) * g[i] +
                    omega * (a + (float)Lt::cx[i] * b0 + (float)Lt::cy[i] * b1 + (float)Lt::cz[i] * b2);

        // wall-shear objective: dWSS/df_j = -(1 - omega/2) (t^.(c_j - u)) (n.(c_j - u))
        if (ws != 0.f) {
            const float nx = normal[s], ny = normal[n + s], nz = normal[2 * (int64_t)n + s];
            float tx, ty, tz;
            shear<Q>(d, drho, ux, uy, uz, omega, nx, ny, nz, tx, ty, tz);
            const float tn = sqrtf(tx * tx + ty * ty + tz * tz);
            if (tn > 0.f) {
                const float it = 1.0f / tn;
                tx *= it;
                ty *= it;
                tz *= it;
                const float kk = -(1.0f - 0.5f * omega) * ws;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const float ex = Lt::cx[i] - ux, ey = Lt::cy[i] - uy, ez = Lt::cz[i] - uz;
                    fh[i] += kk * (tx * ex + ty * ey + tz * ez) * (nx * ex + ny * ey + nz * ez);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) gout[tix<Q>(i, s)] = fh[i];
    }
}

template <int Q, int ST, bool SC, bool BRINK, int MODE>
__global__ __launch_bounds__(kBlock) void k_adj_step(
    const typename Store<ST>::T* __restrict__ A, const typename Store<ST>::T* __restrict__ F,
    const typename Store<ST>::T* __restrict__ Ai,
    const float* __restrict__ gin, float* __restrict__ gout, Table tb, int32_t n,
    int32_t xcd_group, float omega, const float* __restrict__ alpha,
    double* __restrict__ alpha_hat, const float* __restrict__ wss_w,
    const float* __restrict__ normal, Ghosts G, IoletAdj I) {
    __shared__ StageLds lds;
    adj_group<Q, ST, SC, BRINK, MODE>(A, F, Ai, gin, gout, tb, n, omega, alpha, alpha_hat, wss_w,
                                      normal, G, I, xcd_block((int32_t)blockIdx.x, xcd_group),
                                      lds);
}

// A reverse step of one segment (blocks below nb, a multiple of 8 xcd_group) and a
// recompute step of the next earlier segment (the other blocks) in one launch: the
// two touch disjoint buffers, and for a lattice too small to fill the GPU each half
// runs beside the other instead of after it.  The longer reverse half is
// dispatched first, so the recompute workgroups fill the compute units as they
// drain.  With SREC (FP32 storage, block addressing, halfway walls) the recompute
// half is the forward step that first copies its four tiles' populations into LDS.
template <int Q, int ST, bool SC, bool BRINK, int MODE, bool SREC>
__global__ __launch_bounds__(kBlock) void k_adj_dual(
    const typename Store<ST>::T* __restrict__ src, typename Store<ST>::T* __restrict__ dst,
    Ghosts Gf, int64_t t_next, int32_t nb, const typename Store<ST>::T* __restrict__ A,
    const typename Store<ST>::T* __restrict__ Ai, const float* __restrict__ gin,
    float* __restrict__ gout, Table tb, int32_t n, int32_t tiles_alloc, int32_t xcd_group,
    float omega, const float* __restrict__ alpha, double* __restrict__ alpha_hat,
    const float* __restrict__ wss_w, const float* __restrict__ normal, Ghosts G, IoletAdj I) {
    __shared__ StageLds lds[1];
    const int32_t b = (int32_t)blockIdx.x;
    if (b < nb) {
        adj_group<Q, ST, SC, BRINK, MODE>(A, nullptr, Ai, gin, gout, tb, n, omega, alpha,
                                          alpha_hat, wss_w, normal, G, I, xcd_block(b, xcd_group),
                                          lds[0]);
        return;
    }
    const int32_t g = xcd_block(b - nb, xcd_group);
    if constexpr (SREC) {
        __shared__ __attribute__((aligned(16))) typename Store<ST>::T pops[4][Q][kTile];
        stream_collide_staged<Q, ST, SC, BRINK, 4, true>(src, dst, tb, n, tiles_alloc, 4 * g,
                                                         omega, alpha, Gf, t_next, pops, lds);
    } else {
        stream_collide_group<Q, ST, SC, BRINK, false>(src, dst, tb, n, g, omega, alpha, Gf, t_next,
                                                      lds[0]);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

int32_t objective_parts(int64_t items) {
    return (int32_t)std::min<int64_t>(kObjParts, std::max<int64_t>(1, (items + kBlock - 1) / kBlock));
}

hipError_t launch_objective(const Layout& L, const Ghosts& G, const void* A, const Objective& O,
                            const float* normal, float omega, double* part, double* q_out,
                            double* w_out, hipStream_t s) {
    const int32_t parts = objective_parts((int64_t)O.n_out + O.n_dome);
    hipError_t e = dispatch(L.q, L.storage, L.scaled, [&](auto tag) {
        using Tg = decltype(tag);
        using T = typename Store<Tg::ST>::T;
        k_objective<Tg::Q, Tg::ST, Tg::SC><<<(unsigned)parts, kBlock, 0, s>>>(
            static_cast<const T*>(A), L.tb, (int32_t)L.n, G, O.out_links, O.n_out, O.dome,
            O.n_dome, normal, omega, part);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    k_objective_final<<<1, 64, 0, s>>>(part, parts, q_out, w_out);
    return hipGetLastError();
}

// grid of four-tile workgroups, padded to whole XCD windows
static int64_t adj_grid(int64_t n, int xcd_group) {
    const int64_t nb = (int64_t)blocks(n);
    return xcd_group > 0 ? ((nb + 8 * xcd_group - 1) / (8 * xcd_group)) * (8 * xcd_group) : nb;
}

// the kernel for one (mode, Brinkman) choice, as a function of the dispatch tag
template <int MODE, bool BRINK, typename Tg>
static hipError_t adj_step_mode(const Layout& L, const Ghosts& G, const IoletAdj& I,
                                const void* A, const void* F, const void* Ai, const float* gin, float* gout,
                                float omega, const float* alpha, double* alpha_hat,
                                const float* wss_w, const float* normal, int xcd_group,
                                hipStream_t s) {
    using T = typename Store<Tg::ST>::T;
    k_adj_step<Tg::Q, Tg::ST, Tg::SC, BRINK, MODE>
        <<<(unsigned)adj_grid(L.n, xcd_group), kBlock, 0, s>>>(
            static_cast<const T*>(A), static_cast<const T*>(F), static_cast<const T*>(Ai), gin, gout,
            L.tb, (int32_t)L.n, xcd_group, omega, alpha, alpha_hat, wss_w, normal, G, I);
    return hipGetLastError();
}

template <int MODE, typename Tg>
static hipError_t adj_step_brink(const Layout& L, const Ghosts& G, const IoletAdj& I,
                                 const void* A, const void* F, const void* Ai, const float* gin, float* gout,
                                 float omega, const float* alpha, double* alpha_hat,
                                 const float* wss_w, const float* normal, int xcd_group,
                                 hipStream_t s) {
    if (alpha && MODE != ADJ_FINAL)
        return adj_step_mode<MODE, true, Tg>(L, G, I, A, F, Ai, gin, gout, omega, alpha, alpha_hat,
                                             wss_w, normal, xcd_group, s);
    return adj_step_mode<MODE, false, Tg>(L, G, I, A, F, Ai, gin, gout, omega, nullptr, alpha_hat,
                                          wss_w, normal, xcd_group, s);
}

hipError_t launch_adj_step(const Layout& L, const Ghosts& G, const IoletAdj& I, int mode,
                           const void* A, const void* F, const void* Ai, const float* gin, float* gout,
                           float omega, const float* alpha, double* alpha_hat,
                           const float* wss_w, const float* normal, int xcd_group,
                           hipStream_t s) {
    if (L.n == 0) return hipSuccess;
    return dispatch(L.q, L.storage, L.scaled, [&](auto tag) {
        using Tg = decltype(tag);
        switch (mode) {
            case ADJ_OWN:
                return adj_step_brink<ADJ_OWN, Tg>(L, G, I, A, F, Ai, gin, gout, omega, alpha,
                                                   alpha_hat, wss_w, normal, xcd_group, s);
            case ADJ_PULL:
                return adj_step_brink<ADJ_PULL, Tg>(L, G, I, A, F, Ai, gin, gout, omega, alpha,
                                                    alpha_hat, wss_w, normal, xcd_group, s);
            case ADJ_FINAL:
                return adj_step_brink<ADJ_FINAL, Tg>(L, G, I, A, F, Ai, gin, gout, omega, nullptr,
                                                     nullptr, nullptr, normal, xcd_group, s);
        }
        return hipErrorInvalidValue;
    });
}

template <int MODE, bool BRINK, bool SREC, typename Tg>
static hipError_t adj_dual_mode(const Layout& L, const Ghosts& Gf, const void* src, void* dst,
                                int64_t t_next, const Ghosts& G, const IoletAdj& I,
                                const void* A, const void* Ai, const float* gin, float* gout,
                                float omega, const float* alpha, double* alpha_hat,
                                const float* wss_w, const float* normal, int xcd_group,
                                hipStream_t s) {
    using T = typename Store<Tg::ST>::T;
    const int64_t nb = adj_grid(L.n, xcd_group);
    k_adj_dual<Tg::Q, Tg::ST, Tg::SC, BRINK, MODE, SREC><<<(unsigned)(2 * nb), kBlock, 0, s>>>(
        static_cast<const T*>(src), static_cast<T*>(dst), Gf, t_next, (int32_t)nb,
        static_cast<const T*>(A), static_cast<const T*>(Ai), gin, gout, L.tb, (int32_t)L.n,
        (int32_t)(L.slots / kTile), xcd_group, omega, alpha, alpha_hat, wss_w, normal, G, I);
    return hipGetLastError();
}

template <int MODE, typename Tg>
static hipError_t adj_dual_brink(const Layout& L, const Ghosts& Gf, const void* src, void* dst,
                                 int64_t t_next, const Ghosts& G, const IoletAdj& I,
                                 const void* A, const void* Ai, const float* gin, float* gout,
                                 float omega, const float* alpha, double* alpha_hat,
                                 const float* wss_w, const float* normal, int xcd_group,
                                 hipStream_t s) {
    // the recompute half stages its populations where the forward step would
    const bool srec = Tg::ST == ST_F32 && L.stage_tiles > 0 && L.tb.grp && !L.bfl;
    if (alpha)
        return srec ? adj_dual_mode<MODE, true, true, Tg>(L, Gf, src, dst, t_next, G, I, A, Ai,
                                                          gin, gout, omega, alpha, alpha_hat,
                                                          wss_w, normal, xcd_group, s)
                    : adj_dual_mode<MODE, true, false, Tg>(L, Gf, src, dst, t_next, G, I, A, Ai,
                                                           gin, gout, omega, alpha, alpha_hat,
                                                           wss_w, normal, xcd_group, s);
    return srec ? adj_dual_mode<MODE, false, true, Tg>(L, Gf, src, dst, t_next, G, I, A, Ai, gin,
                                                       gout, omega, nullptr, alpha_hat, wss_w,
                                                       normal, xcd_group, s)
                : adj_dual_mode<MODE, false, false, Tg>(L, Gf, src, dst, t_next, G, I, A, Ai, gin,
                                                        gout, omega, nullptr, alpha_hat, wss_w,
                                                        normal, xcd_group, s);
}

hipError_t launch_adj_dual(const Layout& L, const Ghosts& Gf, const void* src, void* dst,
                           int64_t t_next, const Ghosts& G, const IoletAdj& I, int mode,
                           const void* A, const void* Ai, const float* gin, float* gout,
                           float omega, const float* alpha, double* alpha_hat,
                           const float* wss_w, const float* normal, int xcd_group,
                           hipStream_t s) {
    if (L.n == 0) return hipSuccess;
    if (mode != ADJ_OWN && mode != ADJ_PULL) return hipErrorInvalidValue;
    return dispatch(L.q, L.storage, L.scaled, [&](auto tag) {
        using Tg = decltype(tag);
        return mode == ADJ_OWN
                   ? adj_dual_brink<ADJ_OWN, Tg>(L, Gf, src, dst, t_next, G, I, A, Ai, gin, gout,
                                                 omega, alpha, alpha_hat, wss_w, normal, xcd_group, s)
                   : adj_dual_brink<ADJ_PULL, Tg>(L, Gf, src, dst, t_next, G, I, A, Ai, gin, gout,
                                                  omega, alpha, alpha_hat, wss_w, normal, xcd_group,
                                                  s);
    });
}

}  // namespace hlb
