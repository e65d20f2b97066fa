// Internal launch interface of the objective and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace hlb {

// device lists of the objective: the outlet's ghost links and the dome sites
struct Objective {
    const int32_t* out_links;  // ghost-link indices belonging to the outlet iolet
    int32_t n_out;
    const int32_t* dome;       // Morton indices of dome sites with a wall normal
    int32_t n_dome;
};

// sites that own iolet links, with their (contiguous) ghost-link ranges
struct IoletSites {
    int64_t count;
    const int32_t* site;
    const int32_t* lo;
    const int32_t* hi;
};

// Q(t) and the sum of WSS over the dome for the step whose pre-collision state
// (ghosts filled) is A; deterministic two-pass reduction through `part`, which
// holds 2 * objective_parts(n_out + n_dome) doubles.
int32_t objective_parts(int64_t items);
hipError_t launch_objective(const Layout& L, const Ghosts& G, const void* A, const Objective& O,
                            const float* normal, float omega, double* part, double* q_out,
                            double* w_out, hipStream_t s);

// The iolet part of one reverse step t.
struct IoletAdj {
    IoletSites S;           // sites with iolet links, sorted by site
    const int32_t* link_is; // entry in S of the site of each iolet link
    float* pend;            // [S.count][q]: adjoint pending for the sites' own populations
    double t;               // boundary time of the step
    int32_t outlet;         // iolet of the flux objective
    const double* q_tape;   // Q(t) of the window steps
    int64_t q_index;        // index of Q(t) in q_tape, or -1 outside the window
    double q_target;
    double* theta_acc;      // FP64 inlet-coefficient adjoints per link, nbasis each
    int32_t nbasis;
};

// One reverse step t: gin = dJ/dA_{t+1} -> gout = dJ/dA_t (FP32, tiled), accumulating
// dJ/dalpha (FP64 per site) and the inlet-coefficient adjoints (FP64 per link);
// wss_w: per-site weight of the wall-shear term, or null outside the window.  What
// the iolet sites send to their own populations stays in I.pend until the next
// reverse step reads it, or launch_adj_flush adds it to gout.
hipError_t launch_adj_step(const Layout& L, const Ghosts& G, const IoletAdj& I, const void* A,
                           const float* gin, float* gout, float omega, const float* alpha,
                           double* alpha_hat, const float* wss_w, const float* normal,
                           hipStream_t s);
hipError_t launch_adj_flush(int q, float* gout, const IoletAdj& I, hipStream_t s);

// One launch of two independent steps: the recompute step src -> dst at t_next
// (ghosts Gf) and the reverse step of launch_adj_step (no interpolated walls).
hipError_t launch_adj_dual(const Layout& L, const Ghosts& Gf, const void* src, void* dst,
                           int64_t t_next, const Ghosts& G, const IoletAdj& I, const void* A,
                           const float* gin, float* gout, float omega, const float* alpha,
                           double* alpha_hat, const float* wss_w, const float* normal,
                           hipStream_t s);

}  // namespace hlb
