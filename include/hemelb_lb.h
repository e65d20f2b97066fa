/*
 * hemelb_lb.h - C ABI of the sparse lattice-Boltzmann time step on MI355X (gfx950).
 *
 * The method (paper Section 2, "HemeLB model"): a lattice Boltzmann solver on a
 * sparse lattice of fluid sites; each site holds one population per discrete
 * lattice vector (D3Q19 in the paper, D3Q15 also supported), evolved by
 * propagation (streaming) and collision steps, with Ladd velocity iolets at
 * inlets and, in the experiments (Section 4), simple bounce-back at walls.
 * Throughput is counted as in Table 3: site updates per second = fluid sites x
 * steps / wall time.
 *
 * One step, as this library computes it, for every fluid site s and lattice
 * direction i (upstream point y = x_s - c_i):
 *   f_i(s) = A[i][y]                                   y fluid
 *          = A[opp(i)][s]                              y wall (halfway bounce-back;
 *                                                      interpolated with wall_q)
 *          = f_i^eq(rho_k(t), u_s)                     y past pressure iolet k,
 *                                                      u_s = velocity of A[:][s]
 *          = A[opp(i)][s] + 6 w_i (c_i . e_k) U_k(t) W_s   y past velocity iolet k (Ladd)
 *   rho = sum f, u = sum c f / rho,
 *   f^eq_i(rho,u) = w_i rho (1 + 3 c_i.u + 4.5 (c_i.u)^2 - 1.5 u.u),
 *   A'[i][s] = f_i - (f_i - f^eq_i(rho, (1 - alpha_s) u)) / tau.
 * Step n (n = 1, 2, ...) uses boundary time t = n - 1.  The initial state is the
 * rest equilibrium A = w_i.
 *
 * Lattice ordering (shared convention): index 0 is the rest vector, then
 * opposite pairs (2k-1, 2k).
 *   D3Q15: (+-1,0,0) (0,+-1,0) (0,0,+-1) +-(1,1,1) +-(1,1,-1) +-(1,-1,1) +-(-1,1,1)
 *   D3Q19: (+-1,0,0) (0,+-1,0) (0,0,+-1) +-(1,1,0) +-(1,-1,0) +-(1,0,1) +-(1,0,-1)
 *          +-(0,1,1) +-(0,1,-1)
 * where "+-v" lists v then -v.
 *
 * Conventions for every call:
 *   - return 0 on success, a negative HEMELB_E* code on failure; the calling
 *     thread's message is available from hemelb_lb_last_error();
 *   - "host" pointers are read (or written) before the call returns and stay
 *     owned by the caller; "device" pointers are caller-owned device memory on
 *     the handle's GPU, accessed asynchronously on the handle's stream;
 *   - a handle is not thread-safe; separate handles are independent.
 */
#ifndef HEMELB_LB_H
#define HEMELB_LB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hemelb_lb* hemelb_lb_t;

/* error codes */
#define HEMELB_OK 0
#define HEMELB_EINVAL (-1)     /* invalid argument; nothing was done */
#define HEMELB_ENOMEM (-2)     /* device or host allocation failed */
#define HEMELB_EDEVICE (-3)    /* HIP runtime error (message holds the HIP string) */
#define HEMELB_EDIVERGED (-4)  /* a divergence check found a non-finite density/momentum */
#define HEMELB_EORDER (-5)     /* call out of order (e.g. adjoint without a forward tape) */
#define HEMELB_ECANCELLED (-6) /* hemelb_lb_cancel() stopped a step request */

/* population storage (the collision always computes in FP32) */
#define HEMELB_STORE_F32 0  /* FP32 deviations f_i - w_i */
#define HEMELB_STORE_F16 1  /* FP16 deviations, round-to-nearest-even */
#define HEMELB_STORE_BF16 2 /* BF16 deviations, round-to-nearest-even */

/* desc.flags */
#define HEMELB_FLAG_NO_SCALE 1 /* 16-bit storage: omit the per-direction power-of-two scale */
/* How the kernels find a site's upstream neighbours (at most one of these).  With
 * none, block addressing where it applies, else the 16-bit table (which falls back
 * to int32 where it must):
 *   BLOCKS   two-level block addressing (the paper's decomposition of the lattice
 *            into blocks, Section 2 and Table 2): 4x4x4 blocks, each with a fluid
 *            bitmap, its first site index and the ids of its 26 neighbour blocks;
 *            no per-link data.  Applies when coords are given, wall_q is NULL and
 *            every link of nbr is the one the sites' positions imply (fluid links
 *            join sites one lattice vector apart, iolet links of one upstream
 *            position name the same iolet, no periodic wrap); EINVAL otherwise.
 *   TABLE16  explicit neighbour table in 16 bits per link against per-tile lists
 *            of source tiles (falls back to TABLE32 where a tile draws on more
 *            than 128 source tiles)
 *   TABLE32  explicit int32 neighbour table */
#define HEMELB_FLAG_BLOCKS 2
#define HEMELB_FLAG_TABLE16 4
#define HEMELB_FLAG_TABLE32 8

/* hemelb_lb_info_t.addressing */
#define HEMELB_ADDR_TABLE32 0
#define HEMELB_ADDR_TABLE16 1
#define HEMELB_ADDR_BLOCKS 2

/* iolet kinds */
#define HEMELB_IOLET_PRESSURE 0
#define HEMELB_IOLET_VELOCITY 1

/* upstream codes in the neighbour table */
#define HEMELB_LINK_WALL (-1)           /* halfway bounce-back */
#define HEMELB_LINK_IOLET(k) (-2 - (k)) /* upstream point lies past iolet k */

/*
 * Inlet/outlet ("iolet", paper Section 2 and Section 3.B: Ladd velocity iolets,
 * with a velocity weights file and a time-dependent inlet velocity, Figure 6).
 * The imposed value at boundary time t is
 *   v(t) = mean + sum_{h=1..n_harm} cos_k[h-1] cos(2 pi h t / period)
 *                                 + sin_k[h-1] sin(2 pi h t / period)
 * and is a density (PRESSURE) or a speed along the unit vector `direction`
 * (VELOCITY; the inward normal of an inlet, or a wall's tangential direction).
 * cos_k / sin_k are host arrays of n_harm doubles (may be NULL when n_harm = 0).
 */
typedef struct {
    int32_t kind;
    double direction[3];
    double mean;
    int32_t n_harm;
    const double* cos_k;
    const double* sin_k;
    double period;
} hemelb_iolet_t;

/*
 * Problem description (paper Section 2: a sparse lattice of fluid sites and its
 * boundary conditions; Table 1 / Section 4: step length, voxel size and
 * viscosity fix the relaxation time tau; Table 2: site counts).
 * All arrays are host memory, copied during hemelb_lb_create.
 *   lattice      15 or 19
 *   storage      HEMELB_STORE_*
 *   flags        HEMELB_FLAG_*
 *   n_sites      N >= 0 fluid sites (N + ghost links must stay below 2^30)
 *   coords       int32 [N][3] site coordinates in [0, 2^21), or NULL.  When given,
 *                sites are processed in Morton (Z-order, x lowest bit) order and the
 *                wall normals can be derived; results still come back in caller order.
 *   nbr          int32 [N][lattice]: nbr[s][i] = upstream code of direction i at
 *                site s: a site index (>= 0), HEMELB_LINK_WALL, or HEMELB_LINK_IOLET(k).
 *                Column 0 (rest) is ignored.  Fluid links must be reciprocal:
 *                nbr[nbr[s][i]][opp(i)] == s.
 *   tau          relaxation time, > 0.5; +infinity is accepted (no collision: a step
 *                is then a pure permutation of the populations)
 *   n_iolets, iolets
 *   site_weight  double [N] inlet profile weight W_s, or NULL (all 1)
 *   wall_normal  float [N][3] wall normals for the wall shear stress, or NULL
 *                (normalize(sum of c_i over wall links i))
 *   alpha        float [N] Brinkman damping in [0, 1], or NULL (0)
 *   stream       hipStream_t for all work of the handle, or NULL (default stream)
 *   wall_q       float [N][lattice], or NULL for halfway bounce-back everywhere: for
 *                every wall link (nbr[s][i] == HEMELB_LINK_WALL) the fraction q in
 *                (0, 1] of the way from the site to its upstream point at which the
 *                wall lies (other entries ignored).  Wall links then use the
 *                interpolated bounce-back of Bouzidi, Firdaouss and Lallemand (the
 *                BFL wall boundary of Section 3.B, linear variant); q is rounded to a
 *                multiple of 2^-15.  Not supported by the adjoint calls.
 */
typedef struct {
    int32_t lattice;
    int32_t storage;
    int32_t flags;
    int64_t n_sites;
    const int32_t* coords;
    const int32_t* nbr;
    double tau;
    int32_t n_iolets;
    const hemelb_iolet_t* iolets;
    const double* site_weight;
    const float* wall_normal;
    const float* alpha;
    void* stream;
    const float* wall_q;
} hemelb_lb_desc_t;

typedef struct {
    int64_t n_sites;     /* N */
    int64_t n_ghosts;    /* iolet links (one incoming population each) */
    int64_t pitch;       /* slots per direction: sites, then ghost slots (one per iolet
                            link, or one per upstream position with block addressing),
                            in whole 64-site tiles */
    int64_t time;        /* completed steps (boundary time of the next step) */
    int32_t lattice;
    int32_t storage;
    double bytes_per_update;  /* algorithmic HBM bytes of one site update: populations read
                                 and written once plus the addressing data (neighbour
                                 table, or block records) read once */
    int64_t device_bytes;     /* device memory held by the handle */
    int32_t addressing;       /* HEMELB_ADDR_* in use */
} hemelb_lb_info_t;

/*
 * Neighbour table from a voxel label grid (host only, no device work).
 * Implements the upstream classification of pull streaming (Section 2): for each
 * fluid site x and direction i, the point x - c_i is a fluid site, a wall, or lies
 * past an iolet.
 *   labels    uint8 [(X+2)][(Y+2)][(Z+2)], point (x,y,z) at [x+1][y+1][z+1];
 *             0 solid, 1 fluid (only inside the box), 2+k past iolet k
 *   shape     {X, Y, Z}, each >= 1
 *   periodic  {px, py, pz}: nonzero wraps that axis (its padding is unused)
 *   lattice   15 or 19
 *   n_sites   out: number of fluid sites N
 *   coords    out (host, may be NULL): int32 [N][3], lexicographic order (x slowest)
 *   nbr       out (host, may be NULL): int32 [N][lattice] upstream codes as above
 * Call with coords = nbr = NULL to obtain N, then again with arrays of that size.
 * Errors: EINVAL for bad shape/lattice or labels > 2+254; ENOMEM.
 */
int hemelb_lb_links(const uint8_t* labels, const int32_t shape[3], const int32_t periodic[3],
                    int32_t lattice, int64_t* n_sites, int32_t* coords, int32_t* nbr);

/*
 * Create a handle: validate (no device work on failure), Morton-order the sites,
 * build the device neighbour table, allocate ping-pong population buffers and
 * set the rest equilibrium at time 0.
 * Errors: EINVAL (message names the first offending site/direction), ENOMEM, EDEVICE.
 *
 * Launch-shape settings, read from the environment when a handle is created (none
 * changes any result bit; each exists to compare kernel forms):
 *   HEMELB_XCD_GROUP=G     consecutive workgroups given to one XCD (default 16; 0
 *                          leaves the hardware's round-robin)
 *   HEMELB_STAGE_TILES=W   tiles per workgroup that copy their own populations into
 *                          LDS first: 4, 8 or 16, anything else none (default, with
 *                          block addressing: FP32 8 for D3Q15 from 4M sites, else 4;
 *                          none below 256 four-tile groups or with 16-bit storage)
 *   HEMELB_LDS_DMA=0       make that copy go through registers instead of loads
 *                          that write LDS directly
 *   HEMELB_VERBOSE=1       print the time of each setup phase to stderr
 */
int hemelb_lb_create(hemelb_lb_t* out, const hemelb_lb_desc_t* desc);

/* Release all device memory of the handle (after finishing its queued work). */
int hemelb_lb_destroy(hemelb_lb_t h);

/*
 * Enqueue n >= 0 time steps (Section 2: propagation + collision; Table 3 counts
 * these as site updates) on the handle's stream and return without waiting.
 * Each step is one fused stream+collide launch, whose epilogue also writes the
 * incoming iolet populations of the next step; a separate ghost fill runs only
 * before the first step after create, set_state or set_deviations.  Once per
 * 1024 steps a small kernel tabulates the iolet time series.
 * Errors: EINVAL (n < 0), EORDER (past the end of a record), ECANCELLED, EDEVICE.
 */
int hemelb_lb_step(hemelb_lb_t h, int64_t n);

/*
 * Wait for the handle's queued work; with checks on, reports EDIVERGED if a check
 * (or a hemelb_lb_totals call) has met a non-finite value since the state was last
 * set.  The report repeats on every sync until set_state / set_deviations installs
 * a new state, which clears it.
 */
int hemelb_lb_sync(hemelb_lb_t h);

/* Run a divergence check (non-finite density or momentum) every `every` steps (0: off). */
int hemelb_lb_set_check(hemelb_lb_t h, int64_t every);

/* Ask a running hemelb_lb_step() on another thread to stop between steps. */
int hemelb_lb_cancel(hemelb_lb_t h);

/* Use another stream for subsequent work (hipStream_t, NULL = default). */
int hemelb_lb_set_stream(hemelb_lb_t h, void* stream);

/*
 * Observables of the current time (the lattice properties that Section 3.C.2
 * computes and caches for output), from the pre-collision populations of the last step (from the
 * stored populations when no step has run since create/set_state):
 *   p    float [N] device, pressure deviation (rho - 1) / 3 from the reference
 *        density 1 (lattice units; p = rho/3 minus 1/3, kept as a deviation so
 *        that FP32 does not round it away), or NULL
 *   u    float [N][3] device, velocity, or NULL
 *   wss  float [N] device, wall shear stress |sigma n - (n.sigma n) n| with
 *        sigma = -(1 - 1/(2 tau)) sum_i c_i c_i (f_i - f_i^eq); 0 at sites without
 *        a wall link, or NULL
 * Caller site order.  Asynchronous on the handle's stream.
 */
int hemelb_lb_observables(hemelb_lb_t h, float* p, float* u, float* wss);

/*
 * Totals of the stored populations in FP64: out[0] = total mass sum_s rho_s,
 * out[1..3] = total momentum.  host `out`; waits for the stream.
 */
int hemelb_lb_totals(hemelb_lb_t h, double out[4]);

/*
 * hemelb_lb_totals for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * FP64 totals, bit for bit, written to device memory `out` (double[4], caller-owned)
 * asynchronously on the handle's stream, with no synchronisation and no allocation.
 * The reduction's partial sums live in a static device array of 1024 x 4 doubles,
 * one per GPU, held until the process ends; the first call on a GPU looks up its
 * address.  Every call on a GPU shares that array: calls that overlap on one GPU
 * (other streams or threads) race and their results are undefined.  Any lattice
 * size fits (the reduction uses at most 1024 blocks); EINVAL otherwise.  A
 * non-finite state shows as non-finite totals; the divergence flag is not touched.
 */
int hemelb_lb_totals_noalloc(hemelb_lb_t h, double* out);

/*
 * Stored populations in the storage format (checkpoint / resume):
 *   dst/src  device, [lattice][N] in caller order; element type float (F32) or
 *            16-bit (F16/BF16); value = (f_i - w_i) * scale_i, where scale_i is a
 *            power of two (1 for F32 and with HEMELB_FLAG_NO_SCALE; see DESIGN).
 *   t        out/in: completed steps.  set_state resets the "last step" of the
 *            observables to the given state.
 */
int hemelb_lb_get_state(hemelb_lb_t h, void* dst, int64_t* t);
int hemelb_lb_set_state(hemelb_lb_t h, const void* src, int64_t t);

/* Decoded FP32 deviations f_i - w_i, device [lattice][N] in caller order. */
int hemelb_lb_get_deviations(hemelb_lb_t h, float* dst);
int hemelb_lb_set_deviations(hemelb_lb_t h, const float* src, int64_t t);

/* Sizes, time and byte counts of a handle (host `info`). */
int hemelb_lb_info(hemelb_lb_t h, hemelb_lb_info_t* info);

/*
 * Plan without a device: validate `d` exactly as hemelb_lb_create does and report
 * the layout it would build (host `info`: n_sites, n_ghosts, pitch, addressing,
 * bytes_per_update, and device_bytes = the device memory create would allocate;
 * time is 0).  Runs on the host only, so it also serves to size a run before a
 * GPU is at hand.  Errors: those of hemelb_lb_create's validation (EINVAL, with
 * the same messages), ENOMEM.
 */
int hemelb_lb_plan(const hemelb_lb_desc_t* d, hemelb_lb_info_t* info);

/*
 * Kernel timing with HIP events recorded on the handle's stream around every
 * fused stream+collide launch of subsequent steps (capacity: max_launches; 0
 * turns timing off).  hemelb_lb_kernel_time waits and returns the summed
 * milliseconds and the number of timed launches (host pointers).
 */
int hemelb_lb_kernel_timing(hemelb_lb_t h, int64_t max_launches);
int hemelb_lb_kernel_time(hemelb_lb_t h, double* ms, int64_t* launches);

/*
 * In-situ direct volume rendering of a lattice property by ray marching (the
 * visualization of Section 3.C.2: voxels sampled from a volume, viewing
 * parameters and a transfer-function look-up table with steerable scale and
 * offset).  The volume holds one value per fluid site at the site's integer
 * coordinates (voxel centres); all other points are empty.
 *
 * A view gives fixed-point integer vectors, HEMELB_VIEW_FIX units per lattice
 * spacing: ray (i, j), 0 <= i < width, 0 <= j < height, starts at
 * P0 = origin + i * right + j * up and samples P_k = P0 + k * D, k = 0 .. steps-1,
 * with D = dir + i * dir_right + j * dir_up (dir_right = dir_up = 0: an
 * orthographic view; right = up = 0: a pinhole view from the eye at origin).
 * With filter HEMELB_FILTER_NEAREST a sample takes the nearest voxel,
 * x = floor((P_k + FIX/2) / FIX) per axis, and contributes if x is a fluid site,
 * with its value v.  With HEMELB_FILTER_TRILINEAR it filters as a 3D texture
 * does: base voxel b = floor(P_k / FIX), 8-bit fraction a = floor((P_k - b FIX) /
 * 2^12) per axis; corner b + c, c in {0,1}^3, weighs W_c = prod (c ? a : 256 - a)
 * (integers summing to 2^24) and holds the site's value or 0 where there is no
 * site; v = (float)(sum_c W_c v_c / 2^24), summed in FP64 in corner order c = x +
 * 2y + 4z (each product is exact; zero-weight corners are not read).  The sample
 * contributes if a corner of non-zero weight is a site.  A contributing sample
 * of value v: t = (v - offset) * scale (FP32), table entry
 * e = clamp(floor(256 t), 0, 255) (0 for a NaN), (r, g, b, a) = lut[e] (straight
 * alpha), composited front to back in FP32: C += (1 - A) a (r, g, b),
 * A += (1 - A) a.  Samples that can reach no site are skipped (whole 4x4x4
 * blocks at a time).
 *   values  device float [N], one per site in caller order
 *   view    host; lut: host float [256][4]
 *   image   device float [height][width][4] = (C, A), written on the handle's stream
 * Errors: EINVAL if the handle was created without coords, for a NULL pointer,
 * width or height outside [1, 16384], steps outside [0, 2^24], an unknown filter
 * or a non-finite scale or offset; ENOMEM; EDEVICE.  The first call builds the
 * block maps of the volume (device memory: about 5 bytes per 4x4x4 block of the
 * sites' bounding box).
 */
#define HEMELB_VIEW_FIX (1 << 20)
#define HEMELB_FILTER_NEAREST 0
#define HEMELB_FILTER_TRILINEAR 1
typedef struct {
    int64_t origin[3];
    int64_t right[3];
    int64_t up[3];
    int64_t dir[3];
    int32_t width;
    int32_t height;
    int32_t steps;
    float scale;
    float offset;
    const float* lut;
    int32_t filter; /* HEMELB_FILTER_NEAREST or HEMELB_FILTER_TRILINEAR */
    int64_t dir_right[3];
    int64_t dir_up[3];
} hemelb_view_t;

int hemelb_lb_render(hemelb_lb_t h, const float* values, const hemelb_view_t* view, float* image);

/*
 * Plain device copy of `bytes` (multiple of 16, 16-byte aligned device pointers)
 * on `stream`: the practical bandwidth ceiling and a counter calibration for
 * the stream+collide kernel.  Errors: EINVAL, EDEVICE.
 */
int hemelb_copy_probe(void* dst, const void* src, int64_t bytes, void* stream);

/*
 * Differentiation of the time step.  The paper's step (Section 2) is the map
 * A_t -> A_{t+1} defined at the top of this header; these calls run its exact
 * discrete adjoint (reverse mode, FP32 adjoint populations, FP64 accumulation of
 * parameter gradients) for the objective
 *   J = sum_{t0<=t<t1} (Q(t) - q_target)^2 + lam * mean_t mean_{s in D} WSS_s(t),
 * where Q(t) = sum over the links (s, i) of iolet `outlet` of A_t[opp(i)][s] - f_i(s)
 * is the mass leaving through that iolet during step t and WSS is the wall
 * shear stress of hemelb_lb_observables (Section 3.C.2's lattice properties)
 * at the dome sites D (sites with a wall normal among those marked in `dome`).
 * Parameters: the Fourier coefficients of every velocity iolet and the per-site
 * Brinkman field alpha.
 *   outlet    iolet id
 *   q_target  Q*
 *   dome      host uint8 [N] caller order (nonzero: in D), or NULL (no shear term)
 *   lam       weight of the shear term
 *   t0, t1    window of steps, 0 <= t0 <= t1
 */
typedef struct {
    int32_t outlet;
    double q_target;
    const uint8_t* dome;
    double lam;
    int64_t t0, t1;
} hemelb_objective_t;

/*
 * Replace the time series of iolet k (inlet velocity waveform, Section 3.B /
 * Figure 6).  kind, n_harm and direction must equal those given at create.
 * Waits for the handle's stream.  Errors: EINVAL.
 */
int hemelb_lb_set_iolet(hemelb_lb_t h, int32_t k, const hemelb_iolet_t* io);

/* Replace the Brinkman field: host float [N] in [0, 1], caller order, or NULL for none. */
int hemelb_lb_set_alpha(hemelb_lb_t h, const float* alpha);

/*
 * Set (or clear, obj = NULL) the objective.  Subsequent steps inside the window
 * record Q(t) and the dome shear on the device.  Clearing or replacing it ends
 * any adjoint run.  Errors: EINVAL.
 */
int hemelb_lb_set_objective(hemelb_lb_t h, const hemelb_objective_t* obj);

/*
 * J and its two terms (host doubles, any may be NULL), after the forward run has
 * passed the window end; hemelb_lb_objective_flux copies Q(t) for the window's
 * t1 - t0 steps to host `q`.  Waits.  Errors: EORDER.
 */
int hemelb_lb_objective_value(hemelb_lb_t h, double* J, double* flux_term, double* wss_term);
int hemelb_lb_objective_flux(hemelb_lb_t h, double* q);

/*
 * Start the reverse sweep at the handle's current time T (the end of the forward
 * run): dJ/dA_T = 0, gradients zero.  max_segment bounds the steps of one
 * recompute segment (the tape holds max_segment + 1 population buffers).
 * Errors: EORDER (no objective), EINVAL, ENOMEM.
 */
int hemelb_lb_adjoint_begin(hemelb_lb_t h, int64_t max_segment);

/*
 * One checkpoint segment, processed backwards: restore `checkpoint` (device,
 * raw state of hemelb_lb_get_state taken at time t0), recompute steps
 * t0 .. t0+steps-1 onto the tape, then run their adjoint steps in reverse.
 * Segments must be called in reverse order so that t0 + steps equals the time
 * reached by the previous segment (T for the first).  Asynchronous.
 * Errors: EORDER, EINVAL.
 */
int hemelb_lb_adjoint_segment(hemelb_lb_t h, const void* checkpoint, int64_t t0, int64_t steps);

/*
 * The whole reverse sweep over nseg segments given in forward order (host arrays:
 * checkpoints[k] is the device raw state at time t0[k], segment k covers steps
 * t0[k] .. t0[k]+steps[k]-1, consecutive segments join and the last ends at the
 * time the sweep has reached).  The result is that of calling
 * hemelb_lb_adjoint_segment for k = nseg-1 .. 0, bit for bit; each adjoint step
 * of segment k runs in one launch with a recompute step of segment k-1 (a second
 * tape, allocated on first use), so the sweep takes about one launch per time
 * step instead of two.  Asynchronous on the handle's stream.
 * Errors: EORDER, EINVAL, ENOMEM.
 */
int hemelb_lb_adjoint_run(hemelb_lb_t h, const void* const* checkpoints, const int64_t* t0,
                          const int64_t* steps, int64_t nseg);

/*
 * Store-all checkpointing, for problems whose whole trajectory fits in device
 * memory (each state is q * pitch * sizeof(storage) bytes).  hemelb_lb_record
 * allocates max_steps + 1 population buffers and copies the current state (time
 * t0) into the first; each following step writes its new state into the next
 * buffer instead of the handle's own, so the trajectory t0 .. t0 + max_steps
 * stays on the device.  With FP32 storage and halfway walls it also allocates,
 * when device memory allows, max_steps more buffers, into which each recorded step
 * stores its pre-collision populations, so that the reverse sweep reads them
 * instead of re-gathering them (4000 steps of the 199k-site half aneurysm in FP32:
 * 96 GB in all); otherwise, and with 16-bit storage, only the states are kept, with
 * the same results.  Every other call works as before; a
 * hemelb_lb_step request that would go past the record (nothing is done) and
 * hemelb_lb_set_state / _set_deviations during it return EORDER.
 * hemelb_lb_adjoint_recorded runs the reverse sweep (after hemelb_lb_adjoint_begin)
 * from the time the sweep has reached back to t0 over the recorded states, with
 * no recomputation; the result equals that of the checkpointed calls bit for
 * bit.  hemelb_lb_record_end copies the current and previous state back into the
 * handle's own buffers and frees the record (no-op when not recording; waits).
 * Errors: EINVAL, EORDER, ENOMEM, EDEVICE.
 */
int hemelb_lb_record(hemelb_lb_t h, int64_t max_steps);
int hemelb_lb_adjoint_recorded(hemelb_lb_t h);
int hemelb_lb_record_end(hemelb_lb_t h);

/*
 * Gradients accumulated so far (waits).  dtheta: host doubles, for every velocity
 * iolet in id order its 1 + 2 n_harm derivatives (mean, cos_1..n, sin_1..n);
 * dalpha: host doubles [N] caller order.  Either may be NULL.  Errors: EORDER.
 */
int hemelb_lb_adjoint_grads(hemelb_lb_t h, double* dtheta, double* dalpha);

/* Current adjoint populations dJ/dA_t (device float [lattice][N], caller order). */
int hemelb_lb_get_adjoint(hemelb_lb_t h, float* dst);

/* Thread-local message of the last failure; static text for a code. */
const char* hemelb_lb_last_error(void);
const char* hemelb_lb_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* HEMELB_LB_H */
