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

// The iolet terms of the stream transpose at step t (the step whose ghost values
// are differentiated).
struct IoletAdj {
    IoletSites S;           // sites with iolet links, sorted by site
    const int32_t* link_is; // entry in S of the site of each iolet link
    double t;               // boundary time of the step
    int32_t outlet;         // iolet of the flux objective
    const double* q_tape;   // Q(t) of the window steps
    int64_t q_index;        // index of Q(t) in q_tape, or -1 outside the window
    double q_target;
    double* theta_acc;      // FP64 inlet-coefficient adjoints per link, nbasis each
    int32_t nbasis;
};

// The reverse sweep in pull form.  Between kernels of one segment the sweep holds
// fhat_t = dJ/df_t, the adjoint of the pre-collision populations; at segment ends
// it holds ghat_t = dJ/dA_t.  Every kernel writes only its own sites' rows
// (coalesced), so nothing is scattered and nothing waits for another thread.
//   ADJ_OWN   ghat_{t+1} (gin, own rows) -> fhat_t: the transposed collision of step
//             t at the taped state A (= A_t), the wall-shear term, dJ/dalpha.  F
//             (optional): the pre-collision populations f_t in the sites' own slots,
//             as the recording forward stored them; then A is not read.
//   ADJ_PULL  fhat_{t+1} (gin) -> fhat_t: first ghat_{t+1} by the stream transpose
//             of step t + 1 (population k of site s was read by the link of the
//             site s + c_k, i.e. by the link opp(k) of s pulling the other way, by
//             s itself across a wall, or by nobody across an iolet) plus the iolet
//             terms of step t + 1 at the taped state Ai (= A_{t+1}, ghosts and
//             I for time t + 1), then as ADJ_OWN.
//   ADJ_FINAL fhat_t (gin) -> ghat_t (gout): the stream transpose of step t alone,
//             iolet terms at Ai (= A_t).
enum AdjMode { ADJ_OWN = 0, ADJ_PULL = 1, ADJ_FINAL = 2 };

// wss_w: per-site weight of the wall-shear term of step t, or null outside the
// window; xcd_group: the workgroup-to-XCD grouping of the forward step.
hipError_t launch_adj_step(const Layout& L, const Ghosts& G, const IoletAdj& I, int mode,
                           const void* A, const void* F, const void* Ai, const float* gin,
                           float* gout, float omega, const float* alpha, double* alpha_hat,
                           const float* wss_w, const float* normal, int xcd_group,
                           hipStream_t s);

// One launch of two independent steps: the recompute step src -> dst at t_next
// (ghosts Gf) and a reverse step of launch_adj_step in mode ADJ_OWN or ADJ_PULL (no
// interpolated walls).
hipError_t launch_adj_dual(const Layout& L, const Ghosts& Gf, const void* src, void* dst,
                           int64_t t_next, const Ghosts& G, const IoletAdj& I, int mode,
                           const void* A, const void* Ai, const float* gin, float* gout,
                           float omega, const float* alpha, double* alpha_hat,
                           const float* wss_w, const float* normal, int xcd_group,
                           hipStream_t s);

}  // namespace hlb
