// Host side of the C ABI: validation, Morton ordering, device neighbour table,
// ghost (iolet link) lists, memory management and the per-step launch loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/hemelb_lb.h"
#include "adjoint.hpp"
#include "kernels.hpp"
#include "render.hpp"
#include <rocprofiler-sdk-roctx/roctx.h>

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory)
        return fail(HEMELB_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(HEMELB_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                                   \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return hip_fail(_e, what);      \
    } while (0)

// host copies of the lattice vectors (same ordering as the device tables)
struct HostLat {
    int q;
    int c[19][3];
    double w[19];
};

HostLat host_lattice(int q) {
    HostLat L{};
    L.q = q;
    static const int faces[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    static const int corners[4][3] = {{1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {-1, 1, 1}};
    static const int edges[6][3] = {{1, 1, 0}, {1, -1, 0}, {1, 0, 1},
                                    {1, 0, -1}, {0, 1, 1}, {0, 1, -1}};
    int k = 1;
    auto add = [&](const int* v, double w) {
        for (int a = 0; a < 3; ++a) {
            L.c[k][a] = v[a];
            L.c[k + 1][a] = -v[a];
        }
        L.w[k] = L.w[k + 1] = w;
        k += 2;
    };
    if (q == 15) {
        L.w[0] = 2.0 / 9.0;
        for (auto& f : faces) add(f, 1.0 / 9.0);
        for (auto& c : corners) add(c, 1.0 / 72.0);
    } else {
        L.w[0] = 1.0 / 3.0;
        for (auto& f : faces) add(f, 1.0 / 18.0);
        for (auto& e : edges) add(e, 1.0 / 36.0);
    }
    return L;
}

inline int opp_dir(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// wall fraction q in (0, 1] -> multiple of 2^-15 in [1, 32767] (0 is reserved for
// halfway bounce-back)
inline uint32_t wall_code(float q) {
    long k = lroundf(q * 32768.0f);
    if (k < 1) k = 1;
    if (k > 32767) k = 32767;
    return (uint32_t)k;
}

inline uint64_t spread3(uint64_t v) {  // 21 bits -> every third bit
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

inline uint64_t morton(int32_t x, int32_t y, int32_t z) {
    return spread3((uint64_t)x) | (spread3((uint64_t)y) << 1) | (spread3((uint64_t)z) << 2);
}

// Setup progress on stderr, one line per phase, when HEMELB_VERBOSE is set in the
// environment (planning a lattice of several hundred million sites takes minutes).
struct Progress {
    using clock = std::chrono::steady_clock;
    bool on = std::getenv("HEMELB_VERBOSE") != nullptr;
    clock::time_point t0 = clock::now(), last = t0;
    void operator()(const char* phase) {
        if (!on) return;
        const clock::time_point t = clock::now();
        std::fprintf(stderr, "[hemelb] %-30s %7.2f s  (%.1f s in all)\n", phase,
                     std::chrono::duration<double>(t - last).count(),
                     std::chrono::duration<double>(t - t0).count());
        std::fflush(stderr);
        last = t;
    }
};

unsigned worker_count() { return std::max(1u, std::min(16u, std::thread::hardware_concurrency())); }

// Run task(0) .. task(count - 1), each on its own thread except task 0, which
// runs on the caller's.  A task that cannot get a thread runs on the caller's
// thread too.  Every thread is joined before the first exception a task threw is
// rethrown, so no exception leaves a thread or a joinable std::thread behind.
template <class Task>
void run_tasks(unsigned count, Task&& task) {
    std::vector<std::exception_ptr> err(count);
    auto run = [&](unsigned k) {
        try {
            task(k);
        } catch (...) {
            err[k] = std::current_exception();
        }
    };
    std::vector<std::thread> th;
    for (unsigned k = 1; k < count; ++k) {
        bool started = false;
        try {
            th.emplace_back(run, k);
            started = true;
        } catch (...) {
        }
        if (!started) run(k);
    }
    if (count > 0) run(0);
    for (auto& x : th) x.join();
    for (auto& e : err)
        if (e) std::rethrow_exception(e);
}

// f(a, b) over contiguous chunks [a, b) of [0, n), in parallel for large n
template <class F>
void parallel_for(int64_t n, F&& f) {
    const unsigned nt = n < 100000 ? 1u : worker_count();
    run_tasks(nt, [&](unsigned t) { f(n * t / nt, n * (t + 1) / nt); });
}

// Sort v by `less`: chunks sorted in parallel, then merged pairwise in parallel.
template <class T, class Less>
void parallel_sort(std::vector<T>& v, Less less) {
    const int64_t n = (int64_t)v.size();
    const unsigned nt = worker_count();
    if (n < 1000000 || nt == 1) {
        std::sort(v.begin(), v.end(), less);
        return;
    }
    std::vector<int64_t> cut(nt + 1);
    for (unsigned t = 0; t <= nt; ++t) cut[t] = n * t / nt;
    run_tasks(nt, [&](unsigned t) { std::sort(v.begin() + cut[t], v.begin() + cut[t + 1], less); });
    for (size_t w = 1; w < nt; w *= 2) {
        const unsigned pairs = (unsigned)((nt - w + 2 * w - 1) / (2 * w));  // a = 0, 2w, .. with a + w < nt
        run_tasks(pairs, [&](unsigned k) {
            const size_t a = 2 * w * k;
            const int64_t lo = cut[a], mid = cut[a + w], hi = cut[std::min<size_t>(a + 2 * w, nt)];
            std::inplace_merge(v.begin() + lo, v.begin() + mid, v.begin() + hi, less);
        });
    }
}

// Host-side C++ exceptions (an allocation or a thread start failing) become error
// codes: none may cross the C ABI.
template <class F>
int no_throw(F&& f) {
    try {
        return f();
    } catch (const std::bad_alloc&) {
        return fail(HEMELB_ENOMEM, "host memory allocation failed");
    } catch (const std::exception& e) {
        return fail(HEMELB_EDEVICE, "host error: %s", e.what());
    }
}

}  // namespace

struct hemelb_lb {
    int q = 15, storage = 0, flags = 0;
    bool scaled = false;
    int64_t n = 0, nghost = 0, slots = 0, ttiles = 0;
    double tau = 0;
    float omega = 0;
    hipStream_t stream = nullptr;
    int device = 0;

    void* A[2] = {nullptr, nullptr};
    int cur = 0;  // A[cur] holds the current post-collision state
    bool bfl = false;           // interpolated walls present
    int32_t* tbl = nullptr;     // int32 table (when the compact one does not apply)
    uint16_t* t16 = nullptr;    // compact table
    int32_t* toff = nullptr;
    int32_t* tlist = nullptr;
    int64_t tlist_len = 0;
    hlb::BlockRec* brec = nullptr;  // block addressing
    uint64_t* gmask = nullptr;
    int32_t* bnbr = nullptr;
    int32_t* tblock = nullptr;
    int32_t nfluid = 0, nblocks = 0;
    int addressing = HEMELB_ADDR_TABLE32;
    int32_t* g_slot = nullptr;  // ghost slot of each iolet link (block addressing)
    int32_t* g_cell_link = nullptr;  // [cells][q]: iolet link pulling (cell, i), or -1
    uint32_t* gblob = nullptr;  // staged block records per 4-tile group
    int32_t* grp = nullptr;
    int64_t blob_words = 0;
    int32_t* g_site = nullptr;
    uint8_t* g_dir = nullptr;
    uint8_t* g_iolet = nullptr;
    float* g_coef = nullptr;
    hlb::DevIolet* d_iolets = nullptr;
    double* d_harm = nullptr;
    int32_t n_iolets = 0;
    double* d_vals = nullptr;  // iolet values for a batch of steps
    int64_t vals_cap = 0;      // steps the buffer holds
    int64_t vals_t0 = 0;
    int32_t basis_stride = 0;   // Fourier basis doubles per (step, iolet): 2 x the most harmonics
    int32_t* perm = nullptr;  // Morton index -> caller index (null: identity)
    float* normal = nullptr;  // [3][n] Morton order
    float* alpha = nullptr;
    double* partial = nullptr;
    double* tot = nullptr;
    int32_t* flag = nullptr;
    int64_t nparts = 1;

    int64_t t = 0;
    bool streamed = false;
    bool ghosts_ready = false;  // A[cur]'s ghost slots hold the incoming values for time t
    int xcd_group = 16;  // consecutive workgroups per XCD (measured best at 8-16)
    // stream-collide workgroups that copy their own tiles' populations into LDS
    // (block addressing only; the copy keeps the in-group pulls off the L1, which
    // then holds the other tiles' lines).  FP32 storage: 8 tiles for D3Q15 lattices
    // of 4M sites or more, else 4; none for lattices of fewer than 256 four-tile
    // groups (too few workgroups to hide the copy) and none with 16-bit storage
    // (slower)
    int stage_tiles = 0;
    // the FP32 staging copy uses loads that write LDS directly
    bool lds_dma = true;
    int64_t check_every = 0;
    std::atomic<bool> cancel{false};

    std::vector<hipEvent_t> ev;
    int64_t ev_cap = 0, ev_used = 0;

    int64_t device_bytes = 0;

    // volume rendering: block map of the sites (built on the first render call)
    std::vector<int32_t> h_coords;  // [n][3] site coordinates in Morton order (when given)
    int32_t* r_grid = nullptr;
    uint8_t* r_near = nullptr;
    hlb::BlockRec* r_rec = nullptr;
    float* r_vals = nullptr;
    float* r_lut = nullptr;
    int32_t r_blo[3] = {0, 0, 0}, r_gdim[3] = {0, 0, 0};
    bool r_ready = false;

    // host copies kept for runtime updates and the adjoint
    std::vector<int32_t> order;     // Morton index -> caller index
    std::vector<int32_t> h_gsite;   // ghost link -> Morton site
    std::vector<uint8_t> h_gdir, h_giol;
    std::vector<uint8_t> has_normal;  // per Morton site
    struct HostIolet {
        int kind, n_harm, harm_off;
        double dir[3];
    };
    std::vector<HostIolet> h_iolets;
    std::vector<double> h_harm;

    // objective (outlet flux + dome wall shear over a window of steps)
    bool obj_set = false;
    int32_t obj_outlet = -1;
    double q_target = 0, lam = 0;
    int64_t w0 = 0, w1 = 0, n_dome = 0;
    int32_t* d_out_links = nullptr;
    int32_t n_out = 0;
    int32_t* d_dome = nullptr;
    float* d_wss_w = nullptr;
    double* d_qtape = nullptr;
    double* d_wtape = nullptr;
    double* d_opart = nullptr;  // partial sums of the objective's blocks
    int64_t obj_bytes = 0;      // device bytes of the objective's arrays

    // adjoint
    std::vector<void*> tape;  // K+1 population buffers of a recompute segment
    std::vector<void*> tape2;  // a second tape: recompute one segment while reversing another
    // recorded trajectory: rec[m] holds the state at time rec_t0 + m; while recording,
    // A[] point into rec and the handle's own population buffers wait in A_own.  With
    // FP32 storage (halfway walls) frec[m] holds the pre-collision populations of step
    // rec_t0 + m, which the reverse sweep then reads in place instead of re-gathering.
    std::vector<void*> rec, frec;
    int64_t rec_t0 = -1;
    void* A_own[2] = {nullptr, nullptr};
    struct Series {            // iolet values and Fourier basis of one segment
        double* vals = nullptr;
        double* basis = nullptr;
        int64_t cap = 0, t0 = 0;
        int32_t stride = 0;    // basis doubles per (step, iolet) the buffer was sized for
    } series[2];
    float* ghat[2] = {nullptr, nullptr};
    int gcur = 0;
    double* alpha_hat = nullptr;
    double* theta_acc = nullptr;
    int32_t nbasis = 1;
    int32_t* is_link = nullptr;  // entry of each iolet link's site among the iolet sites
    int32_t* is_site = nullptr;
    int32_t* is_lo = nullptr;
    int32_t* is_hi = nullptr;
    int64_t n_is = 0;
    int64_t adj_t = -1;

    hlb::Layout layout() const {
        return hlb::Layout{q, storage, scaled, n, slots,
                           hlb::Table{tbl, t16, toff, tlist, brec, gmask, bnbr, tblock,
                                      reinterpret_cast<const uint4*>(gblob), grp, nfluid, nblocks,
                                      (int32_t)n},
                           bfl, stage_tiles, lds_dma};
    }
    hlb::Ghosts ghosts() const {
        return hlb::Ghosts{nghost,  g_slot,   g_cell_link, g_site,  g_dir,   g_iolet,
                           g_coef,  d_iolets, d_harm,      d_vals,  vals_t0, n_iolets,
                           nullptr, basis_stride};
    }
    size_t elem() const { return storage == HEMELB_STORE_F32 ? 4 : 2; }
    // algorithmic HBM bytes of one site update: populations read and written once,
    // plus the addressing data read once (the neighbour table and the compact
    // table's per-tile lists, or the block records, neighbour-block ids and per-tile
    // first blocks)
    double addr_bytes = 0;  // addressing data one step reads (see HostPlan)
    double bytes_per_update() const {
        return 2.0 * q * (double)elem() + (n > 0 ? addr_bytes / (double)n : 0.0);
    }
};

namespace {

template <class T>
int dev_alloc(hemelb_lb* h, T** p, size_t count, const char* what) {
    *p = nullptr;
    if (count == 0) return HEMELB_OK;
    void* q = nullptr;
    const size_t bytes = count * sizeof(T);
    HIP_TRY(hipMalloc(&q, bytes), what);
    *p = static_cast<T*>(q);
    h->device_bytes += (int64_t)bytes;
    return HEMELB_OK;
}

template <class T>
int dev_upload(hemelb_lb* h, T** p, const std::vector<T>& v, const char* what) {
    int rc = dev_alloc(h, p, v.size(), what);
    if (rc) return rc;
    if (!v.empty()) HIP_TRY(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), what);
    return HEMELB_OK;
}

void release(hemelb_lb* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    if (h->rec_t0 >= 0) {  // A[] alias recorded buffers, freed below
        h->A[0] = h->A_own[0];
        h->A[1] = h->A_own[1];
    }
    for (void* p : h->rec)
        if (p) (void)hipFree(p);
    for (void* p : h->frec)
        if (p) (void)hipFree(p);
    void* ptrs[] = {h->A[0],      h->A[1],      h->tbl,        h->g_site,    h->g_dir,
                    h->t16,       h->toff,      h->tlist,      h->brec,      h->gmask,
                    h->bnbr,      h->tblock,    h->g_slot,     h->gblob,     h->grp,
                    h->g_cell_link, h->is_link,
                    h->g_iolet,   h->g_coef,    h->d_iolets,   h->d_harm,    h->perm,
                    h->normal,    h->alpha,     h->partial,    h->tot,       h->flag,
                    h->d_out_links, h->d_dome,  h->d_wss_w,    h->d_qtape,   h->d_wtape,
                    h->d_opart,
                    h->ghat[0],   h->ghat[1],   h->alpha_hat,  h->theta_acc, h->is_site,
                    h->r_grid,    h->r_near,     h->r_rec,     h->r_vals,    h->r_lut,
                    h->is_lo,     h->is_hi,     h->d_vals};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (void* p : h->tape)
        if (p) (void)hipFree(p);
    for (void* p : h->tape2)
        if (p) (void)hipFree(p);
    for (auto& sr : h->series) {
        if (sr.vals) (void)hipFree(sr.vals);
        if (sr.basis) (void)hipFree(sr.basis);
    }
    for (auto e : h->ev) (void)hipEventDestroy(e);
    delete h;
}

int validate(const hemelb_lb_desc_t* d) {
    if (!d) return fail(HEMELB_EINVAL, "desc is NULL");
    if (d->lattice != 15 && d->lattice != 19)
        return fail(HEMELB_EINVAL, "lattice must be 15 or 19 (got %d)", d->lattice);
    if (d->storage < HEMELB_STORE_F32 || d->storage > HEMELB_STORE_BF16)
        return fail(HEMELB_EINVAL, "unknown storage %d", d->storage);
    const int32_t known = HEMELB_FLAG_NO_SCALE | HEMELB_FLAG_BLOCKS | HEMELB_FLAG_TABLE16 |
                          HEMELB_FLAG_TABLE32;
    if (d->flags & ~known) return fail(HEMELB_EINVAL, "unknown flags 0x%x", d->flags);
    const int32_t addr = d->flags & (HEMELB_FLAG_BLOCKS | HEMELB_FLAG_TABLE16 | HEMELB_FLAG_TABLE32);
    if (addr & (addr - 1))
        return fail(HEMELB_EINVAL, "at most one of the BLOCKS, TABLE16 and TABLE32 flags");
    if (d->n_sites < 0) return fail(HEMELB_EINVAL, "n_sites < 0");
    if (d->n_sites >= (int64_t)1 << 30) return fail(HEMELB_EINVAL, "n_sites must be below 2^30");
    if (!(d->tau > 0.5)) return fail(HEMELB_EINVAL, "tau must exceed 1/2 (got %g)", d->tau);
    if (d->n_iolets < 0 || d->n_iolets > 254) return fail(HEMELB_EINVAL, "n_iolets out of range");
    if (d->n_iolets > 0 && !d->iolets) return fail(HEMELB_EINVAL, "iolets is NULL");
    for (int k = 0; k < d->n_iolets; ++k) {
        const hemelb_iolet_t& io = d->iolets[k];
        if (io.kind != HEMELB_IOLET_PRESSURE && io.kind != HEMELB_IOLET_VELOCITY)
            return fail(HEMELB_EINVAL, "iolet %d: unknown kind %d", k, io.kind);
        if (io.n_harm < 0 || io.n_harm > 64) return fail(HEMELB_EINVAL, "iolet %d: n_harm", k);
        if (io.n_harm > 0 && (!io.cos_k || !io.sin_k || !(io.period > 0)))
            return fail(HEMELB_EINVAL, "iolet %d: harmonics need cos_k, sin_k and period > 0", k);
        if (!std::isfinite(io.mean)) return fail(HEMELB_EINVAL, "iolet %d: mean not finite", k);
        for (int h = 0; h < io.n_harm; ++h)
            if (!std::isfinite(io.cos_k[h]) || !std::isfinite(io.sin_k[h]))
                return fail(HEMELB_EINVAL, "iolet %d: harmonic %d not finite", k, h);
        if (io.kind == HEMELB_IOLET_VELOCITY)
            for (int a = 0; a < 3; ++a)
                if (!std::isfinite(io.direction[a]))
                    return fail(HEMELB_EINVAL, "iolet %d: direction not finite", k);
    }
    const int64_t n = d->n_sites;
    const int q = d->lattice;
    if (n == 0) return HEMELB_OK;
    if (!d->nbr) return fail(HEMELB_EINVAL, "nbr is NULL");
    const int32_t* nb = d->nbr;
    // find the first site with a bad link in parallel; the loop below then names it
    std::atomic<int64_t> first{n};
    parallel_for(n, [&](int64_t a, int64_t b) {
        for (int64_t s = a; s < b && s < first.load(std::memory_order_relaxed); ++s)
            for (int i = 1; i < q; ++i) {
                const int32_t v = nb[s * q + i];
                const bool bad = v >= 0 ? (v >= n || nb[(int64_t)v * q + opp_dir(i)] != s)
                                        : (v != HEMELB_LINK_WALL && (-2 - v < 0 || -2 - v >= d->n_iolets));
                if (bad) {
                    int64_t cur = first.load();
                    while (s < cur && !first.compare_exchange_weak(cur, s)) {
                    }
                    return;
                }
            }
    });
    for (int64_t s = first.load(); s < n; ++s)
        for (int i = 1; i < q; ++i) {
            const int32_t v = nb[s * q + i];
            if (v >= 0) {
                if (v >= n) return fail(HEMELB_EINVAL, "nbr[%lld][%d] = %d out of range", (long long)s, i, v);
                if (nb[(int64_t)v * q + opp_dir(i)] != s)
                    return fail(HEMELB_EINVAL,
                                "link (%lld, %d) not reciprocal: nbr[%d][%d] != %lld",
                                (long long)s, i, v, opp_dir(i), (long long)s);
            } else if (v != HEMELB_LINK_WALL) {
                const int k = -2 - v;
                if (k < 0 || k >= d->n_iolets)
                    return fail(HEMELB_EINVAL, "nbr[%lld][%d] = %d: no such iolet", (long long)s, i, v);
            }
        }
    if (d->coords)
        for (int64_t s = 0; s < n; ++s)
            for (int a = 0; a < 3; ++a) {
                const int32_t c = d->coords[s * 3 + a];
                if (c < 0 || c >= (1 << 21))
                    return fail(HEMELB_EINVAL, "coords[%lld][%d] = %d outside [0, 2^21)", (long long)s, a, c);
            }
    if (d->site_weight)
        for (int64_t s = 0; s < n; ++s)
            if (!std::isfinite(d->site_weight[s]))
                return fail(HEMELB_EINVAL, "site_weight[%lld] not finite", (long long)s);
    if (d->alpha)
        for (int64_t s = 0; s < n; ++s)
            if (!(d->alpha[s] >= 0.f && d->alpha[s] <= 1.f))
                return fail(HEMELB_EINVAL, "alpha[%lld] outside [0, 1]", (long long)s);
    if (d->wall_normal)
        for (int64_t s = 0; s < 3 * n; ++s)
            if (!std::isfinite(d->wall_normal[s]))
                return fail(HEMELB_EINVAL, "wall_normal[%lld] not finite", (long long)(s / 3));
    if (d->wall_q)
        for (int64_t s = 0; s < n; ++s)
            for (int i = 1; i < q; ++i)
                if (nb[s * q + i] == HEMELB_LINK_WALL) {
                    const float v = d->wall_q[s * q + i];
                    if (!(v > 0.f && v <= 1.f))
                        return fail(HEMELB_EINVAL, "wall_q[%lld][%d] = %g outside (0, 1]",
                                    (long long)s, i, (double)v);
                }
    return HEMELB_OK;
}

// Two-level block addressing (the lattice cut into 4x4x4 blocks).  Built from the
// Morton-ordered sites; applies only when every link of the caller's table is the
// one the sites' positions imply, which is checked link by link.
struct BlockPlan {
    std::vector<hlb::BlockRec> rec;  // fluid blocks in site order, then ghost-only blocks
    std::vector<uint64_t> gmask;
    std::vector<int32_t> nbr;        // [nfluid][27]
    std::vector<int32_t> tblock;     // block of the first site of each tile
    std::vector<int32_t> gslot;      // ghost slot of each iolet link
    std::vector<int32_t> cell_link;  // [cells][q]: iolet link pulling (cell, i), or -1
    std::vector<uint32_t> blob;      // staged records of every 4-tile group (16-byte units)
    std::vector<int32_t> grp;        // per group: blob offset, nown | nrec << 16
    double fallback_bytes = 0;       // global records read by groups whose blob would not fit
    int32_t nfluid = 0;
    int64_t ncells = 0;
    std::string why;                 // reason it does not apply
};

inline int block_pos(int x, int y, int z) {
    return (x & 1) | ((y & 1) << 1) | ((z & 1) << 2) | ((x & 2) << 2) | ((y & 2) << 3) |
           ((z & 2) << 4);
}

inline uint64_t block_key(int64_t bx, int64_t by, int64_t bz) {  // each in [-1, 2^21)
    return ((uint64_t)(bx + 1) << 42) | ((uint64_t)(by + 1) << 21) | (uint64_t)(bz + 1);
}

inline uint64_t rec_mask(const hlb::BlockRec& r) {
    return ((uint64_t)r.mask_hi << 32) | (uint64_t)r.mask_lo;
}

// order: Morton index -> caller index; inv: its inverse; gbase[m]: first iolet link
// of Morton site m; gsite/gdir/giol: the iolet links (site, direction, iolet)
bool build_blocks(const hemelb_lb_desc_t* d, const HostLat& lat, const std::vector<int32_t>& order,
                  const std::vector<int32_t>& inv, const std::vector<int64_t>& gbase,
                  const std::vector<int32_t>& gsite, const std::vector<uint8_t>& gdir,
                  const std::vector<uint8_t>& giol, int64_t ttiles, BlockPlan& P) {
    const int q = d->lattice;
    const int64_t n = d->n_sites;
    const int64_t ng = (int64_t)gsite.size();
    auto X = [&](int64_t m, int a) -> int64_t { return d->coords[3 * (int64_t)order[m] + a]; };
    std::unordered_map<uint64_t, int32_t> id;
    id.reserve((size_t)(n / 16 + ng + 16));
    std::vector<int64_t> bc;  // block coordinates, 3 per block
    std::vector<int32_t> site_block(n);
    uint64_t last = ~0ull;
    for (int64_t m = 0; m < n; ++m) {
        const int64_t x = X(m, 0), y = X(m, 1), z = X(m, 2);
        const uint64_t k = block_key(x >> 2, y >> 2, z >> 2);
        if (k != last) {
            // Morton order keeps each block's sites together
            if (!id.emplace(k, (int32_t)P.rec.size()).second) {
                P.why = "internal: sites of a block are not contiguous";
                return false;
            }
            P.rec.push_back(hlb::BlockRec{0u, 0u, (int32_t)m, -1});
            bc.insert(bc.end(), {x >> 2, y >> 2, z >> 2});
            last = k;
        }
        const int p = block_pos((int)(x & 3), (int)(y & 3), (int)(z & 3));
        if (p < 32)
            P.rec.back().mask_lo |= 1u << p;
        else
            P.rec.back().mask_hi |= 1u << (p - 32);
        site_block[m] = (int32_t)P.rec.size() - 1;
    }
    P.nfluid = (int32_t)P.rec.size();

    // ghost cells: the positions past iolet planes that iolet links pull from
    struct Cell {
        int32_t block, pos, iolet;
        int64_t link;
    };
    std::vector<Cell> cells((size_t)ng);
    for (int64_t l = 0; l < ng; ++l) {
        const int i = gdir[l];
        const int64_t m = gsite[l];
        const int64_t x = X(m, 0) - lat.c[i][0], y = X(m, 1) - lat.c[i][1], z = X(m, 2) - lat.c[i][2];
        const uint64_t k = block_key(x >> 2, y >> 2, z >> 2);
        auto it = id.find(k);
        int32_t b;
        if (it == id.end()) {
            b = (int32_t)P.rec.size();
            id.emplace(k, b);
            P.rec.push_back(hlb::BlockRec{0u, 0u, (int32_t)n, -1});
            bc.insert(bc.end(), {x >> 2, y >> 2, z >> 2});
        } else {
            b = it->second;
        }
        const int p = block_pos((int)(x & 3), (int)(y & 3), (int)(z & 3));
        if ((rec_mask(P.rec[b]) >> p) & 1ull) {
            P.why = "an iolet link pulls from the position of a fluid site";
            return false;
        }
        cells[l] = Cell{b, p, giol[l], l};
    }
    std::sort(cells.begin(), cells.end(), [](const Cell& a, const Cell& b) {
        return a.block < b.block || (a.block == b.block && a.pos < b.pos);
    });
    P.gmask.assign(P.rec.size(), 0ull);
    P.gslot.assign((size_t)ng, 0);
    int64_t g = -1;
    for (size_t e = 0; e < cells.size(); ++e) {
        const Cell& c = cells[e];
        if (e == 0 || c.block != cells[e - 1].block || c.pos != cells[e - 1].pos) {
            ++g;
            if (P.rec[c.block].goff < 0) P.rec[c.block].goff = (int32_t)g;
            P.gmask[c.block] |= 1ull << c.pos;
        } else if (c.iolet != cells[e - 1].iolet) {
            P.why = "one position past an iolet plane is named with two iolet ids";
            return false;
        }
        P.gslot[c.link] = (int32_t)(n + g);
    }
    P.ncells = g + 1;
    P.cell_link.assign((size_t)std::max<int64_t>(1, P.ncells) * q, -1);
    for (int64_t l = 0; l < ng; ++l)
        P.cell_link[(size_t)(P.gslot[l] - n) * q + gdir[l]] = (int32_t)l;

    // the 27 blocks around every fluid block
    P.nbr.assign((size_t)P.nfluid * 27, -1);
    parallel_for(P.nfluid, [&](int64_t a, int64_t b) {
        for (int64_t k = a; k < b; ++k)
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        auto it = id.find(block_key(bc[3 * k] + dx, bc[3 * k + 1] + dy,
                                                    bc[3 * k + 2] + dz));
                        if (it != id.end())
                            P.nbr[(size_t)k * 27 + (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)] = it->second;
                    }
    });

    // every link must decode to what the caller's table says
    std::atomic<int64_t> bad{-1};
    parallel_for(n, [&](int64_t a, int64_t b) {
        for (int64_t m = a; m < b && bad.load(std::memory_order_relaxed) < 0; ++m) {
            const int64_t s = order[m];
            const int32_t bl = site_block[m];
            const int bx = (int)(X(m, 0) & 3), by = (int)(X(m, 1) & 3), bz = (int)(X(m, 2) & 3);
            int64_t gl = gbase[m];
            for (int i = 1; i < q; ++i) {
                const int32_t v = d->nbr[s * q + i];
                int32_t want;
                if (v >= 0)
                    want = inv[v];
                else if (v == HEMELB_LINK_WALL)
                    want = (int32_t)0x80000000u;
                else
                    want = P.gslot[gl++];
                const int ux = bx - lat.c[i][0], uy = by - lat.c[i][1], uz = bz - lat.c[i][2];
                const int dd = ((ux >> 2) + 1) + 3 * ((uy >> 2) + 1) + 9 * ((uz >> 2) + 1);
                const int32_t b2 = P.nbr[(size_t)bl * 27 + dd];
                int32_t got = (int32_t)0x80000000u;
                if (b2 >= 0) {
                    const uint64_t mk = rec_mask(P.rec[b2]);
                    const int p = block_pos(ux & 3, uy & 3, uz & 3);
                    const uint64_t below = (1ull << p) - 1ull;
                    if ((mk >> p) & 1ull)
                        got = P.rec[b2].off + __builtin_popcountll(mk & below);
                    else if ((P.gmask[b2] >> p) & 1ull)
                        got = (int32_t)n + P.rec[b2].goff + __builtin_popcountll(P.gmask[b2] & below);
                }
                if (got != want) {
                    int64_t none = -1;
                    bad.compare_exchange_strong(none, s * q + i);
                    break;
                }
            }
        }
    });
    if (bad.load() >= 0) {
        char buf[160];
        snprintf(buf, sizeof buf,
                 "link (site %lld, direction %d) is not the one the site positions imply",
                 (long long)(bad.load() / q), (int)(bad.load() % q));
        P.why = buf;
        return false;
    }
    P.tblock.assign((size_t)ttiles, 0);
    for (int64_t T = 0; T < ttiles; ++T) P.tblock[T] = site_block[std::min(T * hlb::kTile, n - 1)];

    // staged records of each group of four tiles (one 256-thread workgroup)
    const int64_t groups = (ttiles + 3) / 4;
    P.grp.assign((size_t)groups * 2, 0);
    std::vector<int32_t> recs;
    std::vector<uint8_t> rows;
    for (int64_t g = 0; g < groups; ++g) {
        const int64_t s0 = g * 4 * hlb::kTile, s1 = std::min(s0 + 4 * hlb::kTile, n) - 1;
        const int32_t b_lo = site_block[s0], b_hi = site_block[s1];
        const int nown = b_hi - b_lo + 1;
        P.grp[2 * g] = (int32_t)(P.blob.size() / 4);
        // a group left at nown = 0 reads, per own block, its record, neighbour ids and the
        // neighbours' records
        const double global_bytes = (double)nown * (sizeof(hlb::BlockRec) + 27 * 4 + 8);
        if (nown > hlb::kStageRows) {
            P.fallback_bytes += global_bytes;
            continue;
        }
        recs.clear();
        for (int32_t b = b_lo; b <= b_hi; ++b) recs.push_back(b);
        rows.assign((size_t)nown * hlb::kRowBytes, 0xff);
        bool fits = true;
        for (int k = 0; k < nown && fits; ++k)
            for (int dd = 0; dd < 27; ++dd) {
                const int32_t nb = P.nbr[(size_t)(b_lo + k) * 27 + dd];  // -1: the empty record
                int idx = (int)(std::find(recs.begin(), recs.end(), nb) - recs.begin());
                if (idx == (int)recs.size()) {
                    if ((int)recs.size() == hlb::kStageRecs) {
                        fits = false;
                        break;
                    }
                    recs.push_back(nb);
                }
                rows[(size_t)k * hlb::kRowBytes + dd] = (uint8_t)idx;
            }
        if (!fits) {
            P.fallback_bytes += global_bytes;
            continue;
        }
        const size_t row_words = (size_t)((nown * hlb::kRowBytes + 15) / 16) * 4;
        const size_t at = P.blob.size();
        P.blob.resize(at + row_words + recs.size() * 4, 0);
        std::memcpy(&P.blob[at], rows.data(), rows.size());
        for (size_t r = 0; r < recs.size(); ++r) {
            hlb::BlockRec c{0u, 0u, 0, -1};  // no block there: no fluid, no ghost cells
            if (recs[r] >= 0) {
                c = P.rec[recs[r]];
                c.goff = c.goff >= 0 ? recs[r] : -1;  // staged copies name ghost blocks by id
            }
            std::memcpy(&P.blob[at + row_words + 4 * r], &c, sizeof c);
        }
        P.grp[2 * g + 1] = nown | (int32_t)(recs.size() << 16);
    }
    if (P.blob.empty()) P.blob.assign(4, 0);

    // the staged copies must decode every link as the caller's table says (the
    // same steps the kernels take, on the host)
    parallel_for(n, [&](int64_t a, int64_t b) {
        for (int64_t m = a; m < b && bad.load(std::memory_order_relaxed) < 0; ++m) {
            const int64_t g = m / (4 * hlb::kTile);
            const int nown = P.grp[2 * g + 1] & 0xffff;
            if (nown == 0) continue;
            const uint8_t* bytes = reinterpret_cast<const uint8_t*>(&P.blob[4 * (size_t)P.grp[2 * g]]);
            const hlb::BlockRec* recs =
                reinterpret_cast<const hlb::BlockRec*>(bytes + 16 * ((nown * hlb::kRowBytes + 15) / 16));
            int k = 0;
            for (int qq = 1; qq < nown; ++qq)
                if (m >= recs[qq].off) k = qq;
            const uint64_t om = rec_mask(recs[k]);
            int rank = (int)(m - recs[k].off), p = 0;
            for (; p < 64; ++p)
                if (((om >> p) & 1ull) && rank-- == 0) break;
            const int bx = (p & 1) | ((p >> 2) & 2), by = ((p >> 1) & 1) | ((p >> 3) & 2),
                      bz = ((p >> 2) & 1) | ((p >> 4) & 2);
            const int64_t s = order[m];
            int64_t gl = gbase[m];
            for (int i = 1; i < q; ++i) {
                const int32_t v = d->nbr[s * q + i];
                const int32_t want = v >= 0 ? inv[v]
                                   : v == HEMELB_LINK_WALL ? (int32_t)0x80000000u : P.gslot[gl++];
                const int ux = bx - lat.c[i][0], uy = by - lat.c[i][1], uz = bz - lat.c[i][2];
                const int dd = ((ux >> 2) + 1) + 3 * ((uy >> 2) + 1) + 9 * ((uz >> 2) + 1);
                const hlb::BlockRec& r = recs[bytes[k * hlb::kRowBytes + dd]];
                const int pp = block_pos(ux & 3, uy & 3, uz & 3);
                const uint64_t mk = rec_mask(r), below = (1ull << pp) - 1ull;
                int32_t got = (int32_t)0x80000000u;
                if ((mk >> pp) & 1ull)
                    got = r.off + __builtin_popcountll(mk & below);
                else if (r.goff >= 0 && ((P.gmask[r.goff] >> pp) & 1ull))
                    got = (int32_t)n + P.rec[r.goff].goff + __builtin_popcountll(P.gmask[r.goff] & below);
                if (got != want) {
                    int64_t none = -1;
                    bad.compare_exchange_strong(none, s * q + i);
                    break;
                }
            }
        }
    });
    if (bad.load() >= 0) {
        P.why = "internal: a staged block record decodes a link wrongly";
        return false;
    }
    return true;
}

// iolet values for times t0 .. t0 + count - 1 into the handle's table
int fill_series(hemelb_lb* h, int64_t t0, int64_t count) {
    if (h->n_iolets == 0) return HEMELB_OK;
    if (count > h->vals_cap) {
        HIP_TRY(hipStreamSynchronize(h->stream), "sync");
        if (h->d_vals) {
            (void)hipFree(h->d_vals);
            h->device_bytes -= h->vals_cap * h->n_iolets * (int64_t)sizeof(double);
            h->d_vals = nullptr;
        }
        const int64_t cap = std::max<int64_t>(count, 1025);
        int rc = dev_alloc(h, &h->d_vals, (size_t)(cap * h->n_iolets), "iolet values");
        if (rc) return rc;
        h->vals_cap = cap;
    }
    HIP_TRY(hlb::launch_iolet_series(h->d_iolets, h->d_harm, h->n_iolets, t0, count, h->d_vals,
                                     nullptr, 0, h->stream),
            "iolet series");
    h->vals_t0 = t0;
    return HEMELB_OK;
}

int do_step(hemelb_lb* h) {
    const hlb::Layout L = h->layout();
    void* fout = nullptr;
    if (h->rec_t0 >= 0) {  // recording: the new state goes to the next recorded buffer
        const int64_t m = h->t - h->rec_t0;
        if (m + 1 >= (int64_t)h->rec.size())
            return fail(HEMELB_EORDER, "the record holds %lld steps; end it before stepping on",
                        (long long)h->rec.size() - 1);
        h->A[h->cur ^ 1] = h->rec[m + 1];
        if (m < (int64_t)h->frec.size()) fout = h->frec[m];
    }
    void* src = h->A[h->cur];
    void* dst = h->A[h->cur ^ 1];
    if (!h->ghosts_ready)
        HIP_TRY(hlb::launch_ghost_fill(L, h->ghosts(), src, h->t, h->stream), "ghost fill");
    if (h->obj_set && h->t >= h->w0 && h->t < h->w1) {
        const hlb::Objective O{h->d_out_links, h->n_out, h->d_dome, (int32_t)h->n_dome};
        HIP_TRY(hlb::launch_objective(L, h->ghosts(), src, O, h->normal, h->omega, h->d_opart,
                                      h->d_qtape + (h->t - h->w0), h->d_wtape + (h->t - h->w0),
                                      h->stream),
                "objective");
    }
    const bool timed = h->ev_used + 2 <= (int64_t)h->ev.size() && h->ev_cap > 0;
    if (timed) HIP_TRY(hipEventRecord(h->ev[h->ev_used], h->stream), "event");
    HIP_TRY(hlb::launch_stream_collide(L, h->ghosts(), src, dst, h->omega, h->alpha, h->xcd_group,
                                       h->t + 1, h->stream, fout),
            "stream collide");
    if (timed) {
        HIP_TRY(hipEventRecord(h->ev[h->ev_used + 1], h->stream), "event");
        h->ev_used += 2;
    }
    h->cur ^= 1;
    h->t += 1;
    h->streamed = true;
    h->ghosts_ready = hlb::ghosts_fused();
    if (h->check_every > 0 && h->t % h->check_every == 0)
        HIP_TRY(hlb::launch_totals(L, h->A[h->cur], h->partial, h->nparts, h->tot, h->flag,
                                   h->stream),
                "divergence check");
    return HEMELB_OK;
}

int check_flag(hemelb_lb* h) {
    int32_t f = 0;
    HIP_TRY(hipMemcpy(&f, h->flag, sizeof f, hipMemcpyDeviceToHost), "flag readback");
    if (f) return fail(HEMELB_EDIVERGED, "non-finite density or momentum detected");
    return HEMELB_OK;
}

// Everything create builds on the host before any device work.
struct HostPlan {
    int64_t n = 0, nghost = 0, slots = 0, ttiles = 0;
    std::vector<int32_t> order, inv;  // Morton index -> caller index, and back
    std::vector<int32_t> gsite;       // iolet links in Morton site order, direction ascending
    std::vector<uint8_t> gdir, giol;
    std::vector<float> gcoef;
    int addressing = HEMELB_ADDR_TABLE32;
    BlockPlan bp;                     // block addressing
    std::vector<int32_t> tbl;         // int32 table
    std::vector<uint16_t> t16;        // compact table
    std::vector<int32_t> toff, tlist;
    std::vector<float> nrm;           // wall normals [3][n], Morton order
    std::vector<hlb::DevIolet> dio;
    std::vector<double> harm;
    std::vector<float> alpha;
    std::vector<int32_t> perm;
    double addr_bytes = 0;  // addressing data one step reads: the table, or the staged
                            // block records and group entries (plus global records of
                            // groups whose staged copy would not fit) and tile blocks
};

// Validate d and build the host side of its layout (no device work).
int make_plan(const hemelb_lb_desc_t* d, HostPlan& P, Progress& prog) {
    int rc = validate(d);
    if (rc) return rc;
    prog("validate");
    const int q = d->lattice;
    const int64_t n = d->n_sites;
    P.n = n;
    const HostLat lat = host_lattice(q);

    // Morton order: order[m] = caller index of the m-th site
    P.order.resize(n);
    P.inv.resize(n);
    std::iota(P.order.begin(), P.order.end(), 0);
    if (d->coords && n > 0) {
        struct KI {
            uint64_t key;
            int32_t idx;
        };
        std::vector<KI> ki(n);
        parallel_for(n, [&](int64_t a, int64_t b) {
            for (int64_t s = a; s < b; ++s) {
                const int32_t* c = d->coords + 3 * s;
                ki[s] = KI{morton(c[0], c[1], c[2]), (int32_t)s};
            }
        });
        parallel_sort(ki, [](const KI& a, const KI& b) {
            return a.key < b.key || (a.key == b.key && a.idx < b.idx);
        });
        for (int64_t m = 0; m < n; ++m) P.order[m] = ki[m].idx;
        for (int64_t m = 1; m < n; ++m)
            if (ki[m].key == ki[m - 1].key)
                return fail(HEMELB_EINVAL, "duplicate coordinates at sites %d and %d",
                            ki[m - 1].idx, ki[m].idx);
    }
    for (int64_t m = 0; m < n; ++m) P.inv[P.order[m]] = (int32_t)m;
    prog("site order");

    // iolet links in Morton site order, direction ascending
    for (int64_t m = 0; m < n; ++m) {
        const int64_t s = P.order[m];
        for (int i = 1; i < q; ++i) {
            const int32_t v = d->nbr[s * q + i];
            if (v <= -2) {
                const int k = -2 - v;
                P.gsite.push_back((int32_t)m);
                P.gdir.push_back((uint8_t)i);
                P.giol.push_back((uint8_t)k);
                double coef = 0.0;
                const hemelb_iolet_t& io = d->iolets[k];
                if (io.kind == HEMELB_IOLET_VELOCITY) {
                    const double W = d->site_weight ? d->site_weight[s] : 1.0;
                    const double ce = lat.c[i][0] * io.direction[0] + lat.c[i][1] * io.direction[1] +
                                      lat.c[i][2] * io.direction[2];
                    coef = 6.0 * lat.w[i] * ce * W;
                }
                P.gcoef.push_back((float)coef);
            }
        }
    }
    P.nghost = (int64_t)P.gsite.size();
    if (n + P.nghost >= ((int64_t)1 << 30))
        return fail(HEMELB_EINVAL, "sites + iolet links must stay below 2^30");
    P.ttiles = std::max<int64_t>(1, (n + hlb::kTile - 1) / hlb::kTile);
    std::vector<int64_t> gbase(n + 1, 0);  // first iolet link of each Morton site
    for (int64_t l = 0; l < P.nghost; ++l) gbase[P.gsite[l] + 1]++;
    for (int64_t m = 0; m < n; ++m) gbase[m + 1] += gbase[m];
    prog("iolet links");

    // addressing: asked for, or by default block addressing where it applies and the
    // explicit table otherwise (on the 53M-site tree blocks are the faster form in
    // every storage; on the 5.6M-site tree the table is 2% faster with FP32 storage)
    bool blocks = false;
    const bool try_blocks = (d->flags & HEMELB_FLAG_BLOCKS) ||
                            !(d->flags & (HEMELB_FLAG_TABLE16 | HEMELB_FLAG_TABLE32));
    if (try_blocks && n > 0) {
        if (!d->coords)
            P.bp.why = "it needs site coordinates";
        else if (d->wall_q)
            P.bp.why = "interpolated walls need the neighbour table";
        else
            blocks = build_blocks(d, lat, P.order, P.inv, gbase, P.gsite, P.gdir, P.giol, P.ttiles,
                                  P.bp);
    }
    if (try_blocks && n > 0) prog("block addressing");
    if ((d->flags & HEMELB_FLAG_BLOCKS) && n > 0 && !blocks)
        return fail(HEMELB_EINVAL, "block addressing does not apply: %s", P.bp.why.c_str());
    const int64_t ghost_slots = blocks ? P.bp.ncells : P.nghost;
    P.slots = std::max<int64_t>(hlb::kTile, ((n + ghost_slots + hlb::kTile - 1) / hlb::kTile) * hlb::kTile);

    if (blocks) {
        P.addressing = HEMELB_ADDR_BLOCKS;
        P.addr_bytes = 4.0 * (double)(P.bp.blob.size() + P.bp.grp.size()) + P.bp.fallback_bytes;
    } else {
        // pull table [tile][q-1][64]: fluid -> Morton index of the upstream site;
        // wall -> bit 31 set (read the opposite direction of the same site) with the
        // interpolated-wall fraction in units of 2^-15 in the low bits (0: halfway);
        // iolet -> ghost slot n + l
        std::vector<int32_t> tbl((size_t)P.ttiles * (q - 1) * hlb::kTile, 0);
        parallel_for(n, [&](int64_t a, int64_t b) {
            for (int64_t m = a; m < b; ++m) {
                const int64_t s = P.order[m];
                int64_t g = gbase[m];
                for (int i = 1; i < q; ++i) {
                    const int32_t v = d->nbr[s * q + i];
                    uint32_t e;
                    if (v >= 0)
                        e = (uint32_t)P.inv[v];
                    else if (v == HEMELB_LINK_WALL)
                        e = 0x80000000u | (d->wall_q ? wall_code(d->wall_q[s * q + i]) : 0u);
                    else
                        e = (uint32_t)(n + (g++));
                    const size_t at = ((size_t)(m / hlb::kTile) * (q - 1) + (i - 1)) * hlb::kTile +
                                      (size_t)(m % hlb::kTile);
                    tbl[at] = (int32_t)e;
                }
            }
        });
        prog("neighbour table");
        // compact form: 16-bit codes against a per-tile list of source tiles.  Tiles
        // are independent: codes and list lengths first, then the lists at their offsets.
        bool compact = !(d->flags & HEMELB_FLAG_TABLE32);
        if (compact) {
            const size_t per = (size_t)(q - 1) * hlb::kTile;
            // sorted distinct source tiles of tile T
            auto sources = [&](int64_t T, std::vector<int32_t>& tiles) {
                tiles.clear();
                const size_t base = (size_t)T * per;
                for (size_t e = 0; e < per; ++e) {
                    const int32_t v = tbl[base + e];
                    if (v >= 0) tiles.push_back(v >> hlb::kTileShift);
                }
                std::sort(tiles.begin(), tiles.end());
                tiles.erase(std::unique(tiles.begin(), tiles.end()), tiles.end());
            };
            P.t16.assign(tbl.size(), 0);
            std::vector<int64_t> count((size_t)P.ttiles, 0);
            std::atomic<bool> fits{true};
            parallel_for(P.ttiles, [&](int64_t a, int64_t b) {
                std::vector<int32_t> tiles;
                for (int64_t T = a; T < b && fits.load(std::memory_order_relaxed); ++T) {
                    sources(T, tiles);
                    if (tiles.size() > 2 * (size_t)hlb::kTile) {
                        fits = false;
                        break;
                    }
                    count[T] = (int64_t)tiles.size();
                    const size_t base = (size_t)T * per;
                    for (size_t e = 0; e < per; ++e) {
                        const int32_t v = tbl[base + e];
                        uint16_t c;
                        if (v < 0) {
                            c = (uint16_t)(0x8000u | ((uint32_t)v & 0x7fffu));
                        } else {
                            const int32_t slot =
                                (int32_t)(std::lower_bound(tiles.begin(), tiles.end(),
                                                           v >> hlb::kTileShift) -
                                          tiles.begin());
                            c = (uint16_t)((slot << hlb::kTileShift) | (v & (hlb::kTile - 1)));
                        }
                        P.t16[base + e] = c;
                    }
                }
            });
            compact = fits.load();
            if (compact) {
                P.toff.assign((size_t)P.ttiles + 1, 0);
                int64_t total = 0;
                for (int64_t T = 0; T < P.ttiles; ++T) {
                    P.toff[T] = (int32_t)total;
                    total += count[T];
                }
                P.toff[P.ttiles] = (int32_t)total;
                P.tlist.assign((size_t)total, 0);
                parallel_for(P.ttiles, [&](int64_t a, int64_t b) {
                    std::vector<int32_t> tiles;
                    for (int64_t T = a; T < b; ++T) {
                        sources(T, tiles);
                        std::copy(tiles.begin(), tiles.end(), P.tlist.begin() + P.toff[T]);
                    }
                });
            }
        }
        if (compact) {
            if (P.tlist.empty()) P.tlist.push_back(0);
            P.addressing = HEMELB_ADDR_TABLE16;
            P.addr_bytes = 2.0 * (q - 1) * (double)n + 4.0 * (double)(P.toff.size() + P.tlist.size());
        } else {
            P.t16.clear();
            P.toff.clear();
            P.tlist.clear();
            P.tbl = std::move(tbl);
            P.addr_bytes = 4.0 * (q - 1) * (double)n;
        }
        prog("compact table");
    }

    // wall normals [3][n] in Morton order
    P.nrm.assign((size_t)3 * n, 0.f);
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        for (int64_t m = lo; m < hi; ++m) {
            const int64_t s = P.order[m];
            double v[3] = {0, 0, 0};
            if (d->wall_normal) {
                for (int a = 0; a < 3; ++a) v[a] = d->wall_normal[3 * s + a];
            } else {
                for (int i = 1; i < q; ++i)
                    if (d->nbr[s * q + i] == HEMELB_LINK_WALL)
                        for (int a = 0; a < 3; ++a) v[a] += lat.c[i][a];
            }
            const double nn = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            if (nn > 0)
                for (int a = 0; a < 3; ++a) P.nrm[(size_t)a * n + m] = (float)(v[a] / nn);
        }
    });

    // iolet descriptors and harmonics
    P.dio.resize(d->n_iolets);
    for (int k = 0; k < d->n_iolets; ++k) {
        const hemelb_iolet_t& io = d->iolets[k];
        P.dio[k].kind = io.kind == HEMELB_IOLET_PRESSURE ? 0 : 1;
        P.dio[k].n_harm = io.n_harm;
        P.dio[k].harm_off = (int32_t)P.harm.size();
        P.dio[k].pad = 0;
        P.dio[k].mean = io.mean;
        P.dio[k].period = io.n_harm > 0 ? io.period : 1.0;
        for (int hh = 0; hh < io.n_harm; ++hh) P.harm.push_back(io.cos_k[hh]);
        for (int hh = 0; hh < io.n_harm; ++hh) P.harm.push_back(io.sin_k[hh]);
    }
    if (d->coords) P.perm = P.order;
    if (d->alpha) {
        P.alpha.resize(n);
        for (int64_t m = 0; m < n; ++m) P.alpha[m] = d->alpha[P.order[m]];
    }
    prog("normals and site data");
    return HEMELB_OK;
}

// Device bytes of the arrays create allocates for plan P (population buffers,
// addressing data, ghost lists, normals, alpha, permutation, reductions).
int64_t planned_device_bytes(const HostPlan& P, int q, size_t elem) {
    int64_t b = 2 * (int64_t)q * P.slots * (int64_t)elem;
    b += (int64_t)(P.bp.rec.size() * sizeof(hlb::BlockRec) + P.bp.gmask.size() * 8 +
                   P.bp.nbr.size() * 4 + P.bp.tblock.size() * 4 + P.bp.gslot.size() * 4 +
                   P.bp.blob.size() * 4 + P.bp.grp.size() * 4 + P.bp.cell_link.size() * 4);
    b += (int64_t)(P.tbl.size() * 4 + P.t16.size() * 2 + P.toff.size() * 4 + P.tlist.size() * 4);
    b += (int64_t)(P.gsite.size() * 4 + P.gdir.size() + P.giol.size() + P.gcoef.size() * 4);
    b += (int64_t)(P.dio.size() * sizeof(hlb::DevIolet) + P.harm.size() * 8);
    b += (int64_t)(P.perm.size() * 4 + P.nrm.size() * 4 + P.alpha.size() * 4);
    b += hlb::totals_parts(P.n) * 4 * 8 + 4 * 8 + 4;
    return b;
}

// block map of the sites for the renderer
int build_render_volume(hemelb_lb_t h) {
    const int64_t n = h->n;
    std::vector<hlb::BlockRec> rec;
    std::vector<int32_t> bc;  // block coordinates, 3 per record
    int64_t lo[3] = {0, 0, 0}, hi[3] = {-1, -1, -1};
    uint64_t last = ~0ull;
    for (int64_t m = 0; m < n; ++m) {
        const int32_t* c = &h->h_coords[3 * m];
        const uint64_t k = block_key(c[0] >> 2, c[1] >> 2, c[2] >> 2);
        if (k != last) {
            rec.push_back(hlb::BlockRec{0u, 0u, (int32_t)m, -1});
            for (int a = 0; a < 3; ++a) {
                const int32_t b = c[a] >> 2;
                bc.push_back(b);
                if (rec.size() == 1 || b < lo[a]) lo[a] = b;
                if (rec.size() == 1 || b > hi[a]) hi[a] = b;
            }
            last = k;
        }
        const int p = block_pos(c[0] & 3, c[1] & 3, c[2] & 3);
        if (p < 32)
            rec.back().mask_lo |= 1u << p;
        else
            rec.back().mask_hi |= 1u << (p - 32);
    }
    int64_t cells = 1;
    for (int a = 0; a < 3; ++a) {
        h->r_blo[a] = (int32_t)lo[a];
        h->r_gdim[a] = (int32_t)(hi[a] - lo[a] + 1);
        cells *= std::max<int64_t>(0, h->r_gdim[a]);
    }
    if (cells > ((int64_t)1 << 31))
        return fail(HEMELB_ENOMEM, "the sites' bounding box holds %lld blocks (at most 2^31)",
                    (long long)cells);
    std::vector<int32_t> grid((size_t)cells, -1);
    for (size_t k = 0; k < rec.size(); ++k) {
        const int64_t gx = bc[3 * k] - lo[0], gy = bc[3 * k + 1] - lo[1], gz = bc[3 * k + 2] - lo[2];
        grid[(size_t)((gx * h->r_gdim[1] + gy) * h->r_gdim[2] + gz)] = (int32_t)k;
    }
    // blocks within reach of a trilinear sample: near[B'] for B' = blo - 1 + h,
    // h in [0, gdim] per axis, marks whether a block of B' + {0, 1}^3 holds a site
    const int64_t nd[3] = {h->r_gdim[0] + 1, h->r_gdim[1] + 1, h->r_gdim[2] + 1};
    std::vector<uint8_t> near((size_t)(nd[0] * nd[1] * nd[2]), 0);
    for (size_t k = 0; k < rec.size(); ++k) {
        const int64_t g[3] = {bc[3 * k] - lo[0], bc[3 * k + 1] - lo[1], bc[3 * k + 2] - lo[2]};
        for (int c = 0; c < 8; ++c) {  // block g is reached from h = g + 1 - c
            const int64_t x = g[0] + 1 - (c & 1), y = g[1] + 1 - ((c >> 1) & 1),
                          z = g[2] + 1 - ((c >> 2) & 1);
            near[(size_t)((x * nd[1] + y) * nd[2] + z)] = 1;
        }
    }
    int rc;
    if ((rc = dev_upload(h, &h->r_grid, grid, "render block map"))) return rc;
    if ((rc = dev_upload(h, &h->r_near, near, "render reach map"))) return rc;
    if ((rc = dev_upload(h, &h->r_rec, rec, "render block records"))) return rc;
    if ((rc = dev_alloc(h, &h->r_vals, (size_t)std::max<int64_t>(n, 1), "render values"))) return rc;
    if ((rc = dev_alloc(h, &h->r_lut, 256 * 4, "render table"))) return rc;
    h->r_ready = true;
    return HEMELB_OK;
}

// iolet values (and the Fourier basis of velocity iolets) for times t0 .. t0 + count
// - 1 into the series buffers `sr`, on `stream`
int fill_segment_series(hemelb_lb* h, hemelb_lb::Series& sr, int64_t t0, int64_t count,
                        hipStream_t stream) {
    if (h->n_iolets == 0) return HEMELB_OK;
    if (count > sr.cap || h->basis_stride > sr.stride) {
        HIP_TRY(hipDeviceSynchronize(), "sync");  // no queued work may still use the buffers
        if (sr.vals) (void)hipFree(sr.vals);
        if (sr.basis) (void)hipFree(sr.basis);
        h->device_bytes -= sr.cap * h->n_iolets * (1 + sr.stride) * (int64_t)sizeof(double);
        sr.vals = sr.basis = nullptr;
        sr.cap = 0;
        sr.stride = 0;
        int rc = dev_alloc(h, &sr.vals, (size_t)(count * h->n_iolets), "segment iolet values");
        if (rc) return rc;
        if (h->basis_stride > 0 &&
            (rc = dev_alloc(h, &sr.basis, (size_t)(count * h->n_iolets * h->basis_stride),
                            "segment iolet basis")))
            return rc;
        sr.cap = count;
        sr.stride = h->basis_stride;
    }
    HIP_TRY(hlb::launch_iolet_series(h->d_iolets, h->d_harm, h->n_iolets, t0, count, sr.vals,
                                     sr.basis, h->basis_stride, stream),
            "iolet series");
    sr.t0 = t0;
    return HEMELB_OK;
}

hlb::Ghosts segment_ghosts(const hemelb_lb* h, const hemelb_lb::Series& sr) {
    hlb::Ghosts G = h->ghosts();
    G.vals = sr.vals;
    G.vals_t0 = sr.t0;
    G.basis = sr.basis;
    return G;
}

// restore `checkpoint` into tape[0] for a recompute from time t0 (series for
// `steps` steps)
int begin_recompute(hemelb_lb* h, std::vector<void*>& tape, hemelb_lb::Series& sr,
                    const void* checkpoint, int64_t t0, int64_t steps, hipStream_t stream) {
    int rc = fill_segment_series(h, sr, t0, steps + 1, stream);
    if (rc) return rc;
    HIP_TRY(hlb::launch_state(h->layout(), tape[0], const_cast<void*>(checkpoint), h->perm, 1,
                              stream),
            "checkpoint restore");
    return HEMELB_OK;
}

// recompute step m of the segment starting at t0: tape[m] -> tape[m + 1]
int recompute_step(hemelb_lb* h, std::vector<void*>& tape, const hemelb_lb::Series& sr, int64_t t0,
                   int64_t m, hipStream_t stream) {
    const hlb::Layout L = h->layout();
    const hlb::Ghosts G = segment_ghosts(h, sr);
    if (m == 0 || !hlb::ghosts_fused())
        HIP_TRY(hlb::launch_ghost_fill(L, G, tape[m], t0 + m, stream), "recompute ghosts");
    HIP_TRY(hlb::launch_stream_collide(L, G, tape[m], tape[m + 1], h->omega, h->alpha, h->xcd_group,
                                       t0 + m + 1, stream),
            "recompute");
    return HEMELB_OK;
}

// iolet terms of the reverse step at time t
hlb::IoletAdj iolet_adj(const hemelb_lb* h, int64_t t) {
    const hlb::IoletSites S{h->n_is, h->is_site, h->is_lo, h->is_hi};
    const bool inw = t >= h->w0 && t < h->w1;
    return hlb::IoletAdj{S,          h->is_link,        (double)t,     h->obj_outlet,
                         h->d_qtape, inw ? t - h->w0 : -1, h->q_target, h->theta_acc, h->nbasis};
}

// objective weights of the reverse step at time t (null outside the window)
const float* wss_weights(const hemelb_lb* h, int64_t t) {
    return t >= h->w0 && t < h->w1 ? h->d_wss_w : nullptr;
}

// Reverse kernel of step t0 + m of a segment of `steps` steps (tape[m] = A_{t0+m};
// ftape, if given, holds the steps' pre-collision populations): the segment's last
// step starts from dJ/dA_{t0+steps}, the others from the fhat of the step after.
int reverse_mode(int64_t m, int64_t steps) { return m == steps - 1 ? hlb::ADJ_OWN : hlb::ADJ_PULL; }

int reverse_step(hemelb_lb* h, std::vector<void*>& tape, const std::vector<void*>* ftape,
                 const hemelb_lb::Series& sr, int64_t t0, int64_t m, int64_t steps,
                 hipStream_t stream) {
    const int64_t t = t0 + m;
    const int mode = reverse_mode(m, steps);
    const void* F = ftape ? (*ftape)[m] : nullptr;
    HIP_TRY(hlb::launch_adj_step(h->layout(), segment_ghosts(h, sr), iolet_adj(h, t + 1), mode,
                                 tape[m], F, tape[m + 1], h->ghat[h->gcur], h->ghat[h->gcur ^ 1],
                                 h->omega, h->alpha, h->alpha_hat, wss_weights(h, t), h->normal,
                                 h->xcd_group, stream),
            "adjoint step");
    h->gcur ^= 1;
    return HEMELB_OK;
}

// recompute step mf of the segment at tf0 (tape tf, series sf) and reverse step
// mr of the segment at tr0 of nr_steps steps (tape tr, series sr) in one launch
int dual_step(hemelb_lb* h, std::vector<void*>& tf, const hemelb_lb::Series& sf, int64_t tf0,
              int64_t mf, std::vector<void*>& tr, const hemelb_lb::Series& sr, int64_t tr0,
              int64_t mr, int64_t nr_steps, hipStream_t stream) {
    const hlb::Layout L = h->layout();
    const hlb::Ghosts Gf = segment_ghosts(h, sf);
    if (mf == 0 || !hlb::ghosts_fused())
        HIP_TRY(hlb::launch_ghost_fill(L, Gf, tf[mf], tf0 + mf, stream), "recompute ghosts");
    const int64_t t = tr0 + mr;
    HIP_TRY(hlb::launch_adj_dual(L, Gf, tf[mf], tf[mf + 1], tf0 + mf + 1, segment_ghosts(h, sr),
                                 iolet_adj(h, t + 1), reverse_mode(mr, nr_steps), tr[mr],
                                 tr[mr + 1], h->ghat[h->gcur], h->ghat[h->gcur ^ 1], h->omega,
                                 h->alpha, h->alpha_hat, wss_weights(h, t), h->normal,
                                 h->xcd_group, stream),
            "adjoint dual step");
    h->gcur ^= 1;
    return HEMELB_OK;
}

// end of a segment at t0 (tape[0] = A_t0): the stream transpose of step t0 alone,
// fhat_t0 -> dJ/dA_t0
int end_reverse(hemelb_lb* h, std::vector<void*>& tape, const hemelb_lb::Series& sr, int64_t t0,
                hipStream_t stream) {
    HIP_TRY(hlb::launch_adj_step(h->layout(), segment_ghosts(h, sr), iolet_adj(h, t0),
                                 hlb::ADJ_FINAL, nullptr, nullptr, tape[0], h->ghat[h->gcur],
                                 h->ghat[h->gcur ^ 1], h->omega, nullptr, nullptr, nullptr,
                                 h->normal, h->xcd_group, stream),
            "adjoint segment end");
    h->gcur ^= 1;
    return HEMELB_OK;
}

}  // namespace

// A named range on the profiler's timeline (rocprofv3 --marker-trace) around one
// entry point, so a trace shows which call issued which kernels.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

extern "C" {

const char* hemelb_lb_last_error(void) { return g_err.c_str(); }

const char* hemelb_lb_strerror(int code) {
    switch (code) {
        case HEMELB_OK: return "success";
        case HEMELB_EINVAL: return "invalid argument";
        case HEMELB_ENOMEM: return "out of memory";
        case HEMELB_EDEVICE: return "device error";
        case HEMELB_EDIVERGED: return "simulation diverged";
        case HEMELB_EORDER: return "call out of order";
        case HEMELB_ECANCELLED: return "cancelled";
        default: return "unknown error";
    }
}

static int links_impl(const uint8_t* labels, const int32_t shape[3], const int32_t periodic[3],
                    int32_t lattice, int64_t* n_sites, int32_t* coords, int32_t* nbr) {
    if (!labels || !shape || !n_sites) return fail(HEMELB_EINVAL, "NULL argument");
    if (lattice != 15 && lattice != 19) return fail(HEMELB_EINVAL, "lattice must be 15 or 19");
    const int64_t X = shape[0], Y = shape[1], Z = shape[2];
    if (X < 1 || Y < 1 || Z < 1 || X >= (1 << 21) || Y >= (1 << 21) || Z >= (1 << 21))
        return fail(HEMELB_EINVAL, "bad shape");
    const bool per[3] = {periodic && periodic[0] != 0, periodic && periodic[1] != 0,
                         periodic && periodic[2] != 0};
    const int64_t PY = Y + 2, PZ = Z + 2;
    auto lab = [&](int64_t x, int64_t y, int64_t z) -> uint8_t {
        return labels[((x + 1) * PY + (y + 1)) * PZ + (z + 1)];
    };
    // per-row fluid bitmaps with per-word prefix counts (rank queries)
    const int64_t rows = X * Y, wpr = (Z + 63) / 64;
    std::vector<uint64_t> bits;
    std::vector<uint32_t> wpre;
    std::vector<int64_t> row_start;
    try {
        bits.assign((size_t)(rows * wpr), 0);
        wpre.assign((size_t)(rows * wpr), 0);
        row_start.assign((size_t)rows + 1, 0);
    } catch (const std::bad_alloc&) {
        return fail(HEMELB_ENOMEM, "link builder: host allocation failed");
    }
    std::vector<int64_t> row_cnt(rows, 0);
    parallel_for(rows, [&](int64_t a, int64_t b) {
        for (int64_t r = a; r < b; ++r) {
            const int64_t x = r / Y, y = r % Y;
            uint32_t cnt = 0;
            for (int64_t w = 0; w < wpr; ++w) {
                uint64_t m = 0;
                for (int64_t z = w * 64; z < std::min(Z, w * 64 + 64); ++z) {
                    const uint8_t v = lab(x, y, z);
                    if (v == 1) m |= 1ull << (z - w * 64);
                }
                bits[r * wpr + w] = m;
                wpre[r * wpr + w] = cnt;
                cnt += (uint32_t)__builtin_popcountll(m);
            }
            row_cnt[r] = cnt;
        }
    });
    for (int64_t r = 0; r < rows; ++r) row_start[r + 1] = row_start[r] + row_cnt[r];
    const int64_t n = row_start[rows];
    *n_sites = n;
    if (!coords && !nbr) return HEMELB_OK;
    const HostLat L = host_lattice(lattice);
    const int q = lattice;
    auto rank = [&](int64_t x, int64_t y, int64_t z) -> int64_t {
        const int64_t r = x * Y + y, w = z >> 6;
        const uint64_t m = bits[r * wpr + w] & ((1ull << (z & 63)) - 1ull);
        return row_start[r] + wpre[r * wpr + w] + __builtin_popcountll(m);
    };
    parallel_for(rows, [&](int64_t a, int64_t b) {
        for (int64_t r = a; r < b; ++r) {
            const int64_t x = r / Y, y = r % Y;
            int64_t s = row_start[r];
            for (int64_t w = 0; w < wpr; ++w) {
                uint64_t m = bits[r * wpr + w];
                while (m) {
                    const int64_t z = w * 64 + __builtin_ctzll(m);
                    m &= m - 1;
                    if (coords) {
                        coords[s * 3 + 0] = (int32_t)x;
                        coords[s * 3 + 1] = (int32_t)y;
                        coords[s * 3 + 2] = (int32_t)z;
                    }
                    if (nbr) {
                        nbr[s * q] = (int32_t)s;
                        for (int i = 1; i < q; ++i) {
                            int64_t p[3] = {x - L.c[i][0], y - L.c[i][1], z - L.c[i][2]};
                            const int64_t dim[3] = {X, Y, Z};
                            for (int ax = 0; ax < 3; ++ax)
                                if (per[ax]) p[ax] = ((p[ax] % dim[ax]) + dim[ax]) % dim[ax];
                            const uint8_t v = lab(p[0], p[1], p[2]);
                            int32_t code;
                            const bool inside = p[0] >= 0 && p[0] < X && p[1] >= 0 && p[1] < Y &&
                                                p[2] >= 0 && p[2] < Z;
                            if (v == 1 && inside)
                                code = (int32_t)rank(p[0], p[1], p[2]);
                            else if (v >= 2)
                                code = -(int32_t)v;  // -2 - (v - 2)
                            else
                                code = HEMELB_LINK_WALL;
                            nbr[s * q + i] = code;
                        }
                    }
                    ++s;
                }
            }
        }
    });
    return HEMELB_OK;
}

int hemelb_lb_links(const uint8_t* labels, const int32_t shape[3], const int32_t periodic[3],
                    int32_t lattice, int64_t* n_sites, int32_t* coords, int32_t* nbr) {
    const Range range("hemelb_lb_links");
    return no_throw([&] { return links_impl(labels, shape, periodic, lattice, n_sites, coords, nbr); });
}

static int plan_impl(const hemelb_lb_desc_t* d, hemelb_lb_info_t* info) {
    if (!info) return fail(HEMELB_EINVAL, "info is NULL");
    HostPlan P;
    Progress prog;
    int rc = make_plan(d, P, prog);
    if (rc) return rc;
    const size_t elem = d->storage == HEMELB_STORE_F32 ? 4 : 2;
    info->n_sites = P.n;
    info->n_ghosts = P.nghost;
    info->pitch = P.slots;
    info->time = 0;
    info->lattice = d->lattice;
    info->storage = d->storage;
    info->bytes_per_update =
        2.0 * d->lattice * (double)elem + (P.n > 0 ? P.addr_bytes / (double)P.n : 0.0);
    info->device_bytes = planned_device_bytes(P, d->lattice, elem);
    info->addressing = P.addressing;
    return HEMELB_OK;
}

int hemelb_lb_plan(const hemelb_lb_desc_t* d, hemelb_lb_info_t* info) {
    const Range range("hemelb_lb_plan");
    return no_throw([&] { return plan_impl(d, info); });
}

// Fill a new handle from plan P: everything of hemelb_lb_create after the handle
// exists.  On failure h has been released.
static int init_handle(hemelb_lb* h, hemelb_lb_t* out, const hemelb_lb_desc_t* d, HostPlan& P,
                       Progress& prog) {
    h->q = d->lattice;
    h->storage = d->storage;
    h->flags = d->flags;
    h->scaled = d->storage != HEMELB_STORE_F32 && !(d->flags & HEMELB_FLAG_NO_SCALE);
    h->bfl = d->wall_q != nullptr;
    h->n = d->n_sites;
    h->tau = d->tau;
    h->omega = std::isinf(d->tau) ? 0.0f : (float)(1.0 / d->tau);
    h->stream = static_cast<hipStream_t>(d->stream);
    if (const char* e = getenv("HEMELB_XCD_GROUP")) h->xcd_group = std::max(0, atoi(e));
    h->stage_tiles = 0;
    if (h->storage == HEMELB_STORE_F32 && (d->n_sites + 255) / 256 >= 256)
        h->stage_tiles = h->q == 15 && d->n_sites >= ((int64_t)1 << 22) ? 8 : 4;
    if (const char* e = getenv("HEMELB_STAGE_TILES")) {
        const int v = atoi(e);
        h->stage_tiles = (v == 4 || v == 8 || v == 16) ? v : 0;
    }
    if (const char* e = getenv("HEMELB_LDS_DMA")) h->lds_dma = atoi(e) != 0;
    (void)hipGetDevice(&h->device);
    const int q = h->q;
    const int64_t n = h->n;
    h->nghost = P.nghost;
    h->slots = P.slots;
    h->ttiles = P.ttiles;
    h->addressing = P.addressing;
    h->addr_bytes = P.addr_bytes;
    h->has_normal.assign(n, 0);
    for (int64_t m = 0; m < n; ++m)
        h->has_normal[m] = (P.nrm[m] != 0.f || P.nrm[(size_t)n + m] != 0.f ||
                            P.nrm[2 * (size_t)n + m] != 0.f);
    for (int k = 0; k < d->n_iolets; ++k) {
        const hemelb_iolet_t& io = d->iolets[k];
        hemelb_lb::HostIolet hi{io.kind, io.n_harm, P.dio[k].harm_off,
                                {io.direction[0], io.direction[1], io.direction[2]}};
        h->h_iolets.push_back(hi);
    }
    h->h_harm = P.harm;
    h->n_iolets = d->n_iolets;
    if (d->coords) {
        h->h_coords.resize((size_t)3 * n);
        for (int64_t m = 0; m < n; ++m)
            for (int a = 0; a < 3; ++a) h->h_coords[3 * m + a] = d->coords[3 * (int64_t)P.order[m] + a];
    }

#define TRY(x)              \
    do {                    \
        int _r = (x);       \
        if (_r) {           \
            release(h);     \
            return _r;      \
        }                   \
    } while (0)
    const size_t popbytes = (size_t)q * h->slots * h->elem();
    for (int b = 0; b < 2; ++b) {
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, popbytes);
        if (e != hipSuccess) {
            release(h);
            return hip_fail(e, "population buffer");
        }
        h->A[b] = p;
        h->device_bytes += (int64_t)popbytes;
    }
    if (P.addressing == HEMELB_ADDR_BLOCKS) {
        h->nfluid = P.bp.nfluid;
        h->nblocks = (int32_t)P.bp.rec.size();
        TRY(dev_upload(h, &h->brec, P.bp.rec, "block records"));
        TRY(dev_upload(h, &h->gmask, P.bp.gmask, "ghost masks"));
        TRY(dev_upload(h, &h->bnbr, P.bp.nbr, "neighbour blocks"));
        TRY(dev_upload(h, &h->tblock, P.bp.tblock, "tile blocks"));
        TRY(dev_upload(h, &h->g_slot, P.bp.gslot, "ghost slots"));
        TRY(dev_upload(h, &h->g_cell_link, P.bp.cell_link, "ghost cell links"));
        TRY(dev_upload(h, &h->gblob, P.bp.blob, "staged block records"));
        TRY(dev_upload(h, &h->grp, P.bp.grp, "staged block groups"));
        h->blob_words = (int64_t)P.bp.blob.size();
    } else if (P.addressing == HEMELB_ADDR_TABLE16) {
        TRY(dev_upload(h, &h->t16, P.t16, "compact table"));
        TRY(dev_upload(h, &h->toff, P.toff, "table tile offsets"));
        TRY(dev_upload(h, &h->tlist, P.tlist, "table tile lists"));
        h->tlist_len = (int64_t)P.tlist.size();
    } else {
        TRY(dev_upload(h, &h->tbl, P.tbl, "neighbour table"));
    }
    TRY(dev_upload(h, &h->g_site, P.gsite, "ghost sites"));
    TRY(dev_upload(h, &h->g_dir, P.gdir, "ghost dirs"));
    TRY(dev_upload(h, &h->g_iolet, P.giol, "ghost iolets"));
    TRY(dev_upload(h, &h->g_coef, P.gcoef, "ghost coefs"));
    TRY(dev_upload(h, &h->d_iolets, P.dio, "iolets"));
    TRY(dev_upload(h, &h->d_harm, P.harm, "harmonics"));
    TRY(dev_upload(h, &h->perm, P.perm, "permutation"));
    TRY(dev_upload(h, &h->normal, P.nrm, "normals"));
    TRY(dev_upload(h, &h->alpha, P.alpha, "alpha"));
    h->nparts = hlb::totals_parts(n);
    TRY(dev_alloc(h, &h->partial, (size_t)h->nparts * 4, "partials"));
    TRY(dev_alloc(h, &h->tot, 4, "totals"));
    TRY(dev_alloc(h, &h->flag, 1, "flag"));
    {
        const int32_t z = 0;
        hipError_t e = hipMemcpy(h->flag, &z, sizeof z, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            release(h);
            return hip_fail(e, "flag init");
        }
    }
    const hlb::Layout L = h->layout();
    for (int b = 0; b < 2; ++b) {
        hipError_t e = hlb::launch_zero(L, h->A[b], h->stream);
        if (e != hipSuccess) {
            release(h);
            return hip_fail(e, "initial state");
        }
    }
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        release(h);
        return hip_fail(e, "create sync");
    }
#undef TRY
    prog("device upload");
    h->order = std::move(P.order);
    h->h_gsite = std::move(P.gsite);
    h->h_gdir = std::move(P.gdir);
    h->h_giol = std::move(P.giol);
    *out = h;
    return HEMELB_OK;
}

static int create_impl(hemelb_lb_t* out, const hemelb_lb_desc_t* d) {
    if (!out) return fail(HEMELB_EINVAL, "out is NULL");
    *out = nullptr;
    HostPlan P;
    Progress prog;
    int rc = make_plan(d, P, prog);
    if (rc) return rc;
    hemelb_lb* h = new (std::nothrow) hemelb_lb();
    if (!h) return fail(HEMELB_ENOMEM, "handle allocation failed");
    try {
        return init_handle(h, out, d, P, prog);
    } catch (...) {
        release(h);  // a host allocation failed part way: no handle escapes
        throw;
    }
}

int hemelb_lb_create(hemelb_lb_t* out, const hemelb_lb_desc_t* d) {
    const Range range("hemelb_lb_create");
    return no_throw([&] { return create_impl(out, d); });
}

int hemelb_lb_destroy(hemelb_lb_t h) {
    const Range range("hemelb_lb_destroy");
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    release(h);
    return HEMELB_OK;
}

int hemelb_lb_step(hemelb_lb_t h, int64_t n) {
    const Range range("hemelb_lb_step");
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    if (n < 0) return fail(HEMELB_EINVAL, "negative step count");
    if (h->rec_t0 >= 0 && h->t + n > h->rec_t0 + (int64_t)h->rec.size() - 1)
        return fail(HEMELB_EORDER, "the record ends at step %lld; %lld steps from %lld go past it",
                    (long long)(h->rec_t0 + (int64_t)h->rec.size() - 1), (long long)n,
                    (long long)h->t);
    HIP_TRY(hipSetDevice(h->device), "set device");
    constexpr int64_t kBatch = 1024;  // steps per table of iolet values
    for (int64_t k = 0; k < n; ++k) {
        if (h->cancel.exchange(false))
            return fail(HEMELB_ECANCELLED, "cancelled after %lld of %lld steps", (long long)k,
                        (long long)n);
        int rc;
        if (k % kBatch == 0 && (rc = fill_series(h, h->t, std::min(kBatch, n - k) + 1))) return rc;
        rc = do_step(h);
        if (rc) return rc;
    }
    return HEMELB_OK;
}

int hemelb_lb_sync(hemelb_lb_t h) {
    const Range range("hemelb_lb_sync");
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    HIP_TRY(hipStreamSynchronize(h->stream), "sync");
    if (h->check_every > 0) return check_flag(h);
    return HEMELB_OK;
}

int hemelb_lb_set_check(hemelb_lb_t h, int64_t every) {
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    if (every < 0) return fail(HEMELB_EINVAL, "negative check interval");
    h->check_every = every;
    return HEMELB_OK;
}

int hemelb_lb_cancel(hemelb_lb_t h) {
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    h->cancel = true;
    return HEMELB_OK;
}

int hemelb_lb_set_stream(hemelb_lb_t h, void* stream) {
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    h->stream = static_cast<hipStream_t>(stream);
    return HEMELB_OK;
}

int hemelb_lb_observables(hemelb_lb_t h, float* p, float* u, float* wss) {
    const Range range("hemelb_lb_observables");
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    const void* A = h->streamed ? h->A[h->cur ^ 1] : h->A[h->cur];
    HIP_TRY(hlb::launch_observables(h->layout(), A, h->streamed ? 1 : 0, h->omega, h->perm,
                                    h->normal, p, u, wss, h->stream),
            "observables");
    return HEMELB_OK;
}

int hemelb_lb_totals(hemelb_lb_t h, double out[4]) {
    const Range range("hemelb_lb_totals");
    if (!h || !out) return fail(HEMELB_EINVAL, "NULL argument");
    HIP_TRY(hlb::launch_totals(h->layout(), h->A[h->cur], h->partial, h->nparts, h->tot, h->flag,
                               h->stream),
            "totals");
    HIP_TRY(hipMemcpyAsync(out, h->tot, 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream),
            "totals readback");
    HIP_TRY(hipStreamSynchronize(h->stream), "totals sync");
    return HEMELB_OK;
}

int hemelb_lb_totals_noalloc(hemelb_lb_t h, double* out) {
    const Range range("hemelb_lb_totals_noalloc");
    if (!h || !out) return fail(HEMELB_EINVAL, "NULL argument");
    if (hlb::totals_parts(h->n) > hlb::totals_scratch_parts())
        return fail(HEMELB_EINVAL, "%lld reduction blocks exceed the scratch of %lld",
                    (long long)hlb::totals_parts(h->n), (long long)hlb::totals_scratch_parts());
    HIP_TRY(hipSetDevice(h->device), "set device");
    HIP_TRY(hlb::launch_totals_noalloc(h->layout(), h->A[h->cur], out, h->stream), "totals");
    return HEMELB_OK;
}

static int state_io(hemelb_lb_t h, void* ext, int mode) {
    HIP_TRY(hlb::launch_state(h->layout(), h->A[h->cur], ext, h->perm, mode, h->stream), "state");
    // a state written by the caller starts a new history: a divergence seen
    // before it no longer applies (a fill kernel, not a memset, so that a
    // captured graph replays it)
    if (mode == 1 || mode == 3)
        HIP_TRY(hlb::launch_zero_words(h->flag, 1, h->stream), "divergence flag reset");
    return HEMELB_OK;
}

int hemelb_lb_get_state(hemelb_lb_t h, void* dst, int64_t* t) {
    const Range range("hemelb_lb_get_state");
    if (!h || (!dst && h->n > 0)) return fail(HEMELB_EINVAL, "NULL argument");
    if (t) *t = h->t;
    return state_io(h, dst, 0);
}

int hemelb_lb_set_state(hemelb_lb_t h, const void* src, int64_t t) {
    const Range range("hemelb_lb_set_state");
    if (!h || (!src && h->n > 0)) return fail(HEMELB_EINVAL, "NULL argument");
    if (t < 0) return fail(HEMELB_EINVAL, "negative time");
    if (h->rec_t0 >= 0) return fail(HEMELB_EORDER, "a trajectory is being recorded");
    h->t = t;
    h->streamed = false;
    h->ghosts_ready = false;
    return state_io(h, const_cast<void*>(src), 1);
}

int hemelb_lb_get_deviations(hemelb_lb_t h, float* dst) {
    const Range range("hemelb_lb_get_deviations");
    if (!h || (!dst && h->n > 0)) return fail(HEMELB_EINVAL, "NULL argument");
    return state_io(h, dst, 2);
}

int hemelb_lb_set_deviations(hemelb_lb_t h, const float* src, int64_t t) {
    const Range range("hemelb_lb_set_deviations");
    if (!h || (!src && h->n > 0)) return fail(HEMELB_EINVAL, "NULL argument");
    if (t < 0) return fail(HEMELB_EINVAL, "negative time");
    if (h->rec_t0 >= 0) return fail(HEMELB_EORDER, "a trajectory is being recorded");
    h->t = t;
    h->streamed = false;
    h->ghosts_ready = false;
    return state_io(h, const_cast<float*>(src), 3);
}

int hemelb_lb_info(hemelb_lb_t h, hemelb_lb_info_t* info) {
    if (!h || !info) return fail(HEMELB_EINVAL, "NULL argument");
    info->n_sites = h->n;
    info->n_ghosts = h->nghost;
    info->pitch = h->slots;
    info->time = h->t;
    info->lattice = h->q;
    info->storage = h->storage;
    info->bytes_per_update = h->bytes_per_update();
    info->device_bytes = h->device_bytes;
    info->addressing = h->addressing;
    return HEMELB_OK;
}

int hemelb_lb_kernel_timing(hemelb_lb_t h, int64_t max_launches) {
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    if (max_launches < 0) return fail(HEMELB_EINVAL, "negative capacity");
    HIP_TRY(hipStreamSynchronize(h->stream), "timing sync");
    while ((int64_t)h->ev.size() < 2 * max_launches) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e), "event create");
        h->ev.push_back(e);
    }
    h->ev_cap = max_launches;
    h->ev_used = 0;
    return HEMELB_OK;
}

int hemelb_lb_kernel_time(hemelb_lb_t h, double* ms, int64_t* launches) {
    if (!h || !ms || !launches) return fail(HEMELB_EINVAL, "NULL argument");
    HIP_TRY(hipStreamSynchronize(h->stream), "timing sync");
    double tot = 0;
    for (int64_t k = 0; k + 1 < h->ev_used; k += 2) {
        float t = 0;
        HIP_TRY(hipEventElapsedTime(&t, h->ev[k], h->ev[k + 1]), "elapsed");
        tot += t;
    }
    *ms = tot;
    *launches = h->ev_used / 2;
    return HEMELB_OK;
}

static int render_impl(hemelb_lb_t h, const float* values, const hemelb_view_t* view, float* image) {
    if (!h || !view || !image || !view->lut || (!values && h->n > 0))
        return fail(HEMELB_EINVAL, "NULL argument");
    if (h->n > 0 && h->h_coords.empty())
        return fail(HEMELB_EINVAL, "rendering needs the site coordinates (create with coords)");
    if (view->width < 1 || view->width > 16384 || view->height < 1 || view->height > 16384)
        return fail(HEMELB_EINVAL, "image size %d x %d outside [1, 16384]", view->width,
                    view->height);
    if (view->steps < 0 || view->steps > (1 << 24))
        return fail(HEMELB_EINVAL, "steps %d outside [0, 2^24]", view->steps);
    if (!std::isfinite(view->scale) || !std::isfinite(view->offset))
        return fail(HEMELB_EINVAL, "transfer scale and offset must be finite");
    if (view->filter != HEMELB_FILTER_NEAREST && view->filter != HEMELB_FILTER_TRILINEAR)
        return fail(HEMELB_EINVAL, "unknown filter %d", view->filter);
    for (int a = 0; a < 3; ++a)
        for (const int64_t v : {view->origin[a], view->right[a], view->up[a], view->dir[a],
                                view->dir_right[a], view->dir_up[a]})
            if (v > ((int64_t)1 << 46) || v < -((int64_t)1 << 46))
                return fail(HEMELB_EINVAL, "view vector component beyond 2^46 fixed-point units");
    HIP_TRY(hipSetDevice(h->device), "set device");
    int rc;
    if (!h->r_ready && (rc = build_render_volume(h))) return rc;
    HIP_TRY(hlb::launch_permute(values, h->perm, h->n, h->r_vals, h->stream), "render values");
    HIP_TRY(hipMemcpyAsync(h->r_lut, view->lut, 256 * 4 * sizeof(float), hipMemcpyHostToDevice,
                           h->stream),
            "render table");
    hlb::RenderVolume V{h->r_grid,
                        h->r_rec,
                        h->r_vals,
                        h->r_near,
                        {h->r_blo[0], h->r_blo[1], h->r_blo[2]},
                        {h->r_gdim[0], h->r_gdim[1], h->r_gdim[2]}};
    hlb::RenderView v{};
    for (int a = 0; a < 3; ++a) {
        v.origin[a] = view->origin[a];
        v.right[a] = view->right[a];
        v.up[a] = view->up[a];
        v.dir[a] = view->dir[a];
        v.dir_right[a] = view->dir_right[a];
        v.dir_up[a] = view->dir_up[a];
    }
    v.width = view->width;
    v.height = view->height;
    v.steps = view->steps;
    v.scale = view->scale;
    v.offset = view->offset;
    v.filter = view->filter;
    HIP_TRY(hlb::launch_render(V, v, h->r_lut, image, h->stream), "render");
    return HEMELB_OK;
}

int hemelb_lb_render(hemelb_lb_t h, const float* values, const hemelb_view_t* view, float* image) {
    const Range range("hemelb_lb_render");
    return no_throw([&] { return render_impl(h, values, view, image); });
}

int hemelb_copy_probe(void* dst, const void* src, int64_t bytes, void* stream) {
    if (!dst || !src || bytes <= 0 || (bytes % 16) || ((uintptr_t)dst % 16) || ((uintptr_t)src % 16))
        return fail(HEMELB_EINVAL, "copy probe needs 16-byte aligned pointers and size");
    HIP_TRY(hlb::launch_copy(dst, src, bytes, static_cast<hipStream_t>(stream)), "copy probe");
    return HEMELB_OK;
}

static int set_iolet_impl(hemelb_lb_t h, int32_t k, const hemelb_iolet_t* io) {
    if (!h || !io) return fail(HEMELB_EINVAL, "NULL argument");
    if (k < 0 || k >= (int32_t)h->h_iolets.size()) return fail(HEMELB_EINVAL, "no iolet %d", k);
    hemelb_lb::HostIolet& hi = h->h_iolets[k];
    if (io->kind != hi.kind || io->n_harm != hi.n_harm)
        return fail(HEMELB_EINVAL, "iolet %d: kind and number of harmonics are fixed at create", k);
    if (io->n_harm > 0 && (!io->cos_k || !io->sin_k || !(io->period > 0)))
        return fail(HEMELB_EINVAL, "iolet %d: harmonics need cos_k, sin_k and period > 0", k);
    if (!std::isfinite(io->mean)) return fail(HEMELB_EINVAL, "iolet %d: mean not finite", k);
    for (int a = 0; a < 3; ++a)
        if (io->kind == HEMELB_IOLET_VELOCITY && io->direction[a] != hi.dir[a])
            return fail(HEMELB_EINVAL, "iolet %d: direction is fixed at create", k);
    for (int m = 0; m < io->n_harm; ++m) {
        if (!std::isfinite(io->cos_k[m]) || !std::isfinite(io->sin_k[m]))
            return fail(HEMELB_EINVAL, "iolet %d: harmonic %d not finite", k, m);
        h->h_harm[hi.harm_off + m] = io->cos_k[m];
        h->h_harm[hi.harm_off + io->n_harm + m] = io->sin_k[m];
    }
    hlb::DevIolet dv{hi.kind == HEMELB_IOLET_PRESSURE ? 0 : 1, hi.n_harm, hi.harm_off, 0, io->mean,
                     io->n_harm > 0 ? io->period : 1.0};
    HIP_TRY(hipStreamSynchronize(h->stream), "sync");
    h->ghosts_ready = false;
    HIP_TRY(hipMemcpy(h->d_iolets + k, &dv, sizeof dv, hipMemcpyHostToDevice), "iolet upload");
    if (!h->h_harm.empty())
        HIP_TRY(hipMemcpy(h->d_harm, h->h_harm.data(), h->h_harm.size() * sizeof(double),
                          hipMemcpyHostToDevice),
                "harmonics upload");
    return HEMELB_OK;
}

int hemelb_lb_set_iolet(hemelb_lb_t h, int32_t k, const hemelb_iolet_t* io) {
    const Range range("hemelb_lb_set_iolet");
    return no_throw([&] { return set_iolet_impl(h, k, io); });
}

static int set_alpha_impl(hemelb_lb_t h, const float* alpha) {
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    HIP_TRY(hipStreamSynchronize(h->stream), "sync");
    if (!alpha) {
        if (h->alpha) {
            (void)hipFree(h->alpha);
            h->device_bytes -= h->n * (int64_t)sizeof(float);
            h->alpha = nullptr;
        }
        return HEMELB_OK;
    }
    for (int64_t s = 0; s < h->n; ++s)
        if (!(alpha[s] >= 0.f && alpha[s] <= 1.f))
            return fail(HEMELB_EINVAL, "alpha[%lld] outside [0, 1]", (long long)s);
    if (h->n == 0) return HEMELB_OK;
    std::vector<float> a(h->n);
    for (int64_t m = 0; m < h->n; ++m) a[m] = alpha[h->order[m]];
    if (!h->alpha) {
        int rc = dev_alloc(h, &h->alpha, (size_t)h->n, "alpha");
        if (rc) return rc;
    }
    HIP_TRY(hipMemcpy(h->alpha, a.data(), a.size() * sizeof(float), hipMemcpyHostToDevice),
            "alpha upload");
    return HEMELB_OK;
}

int hemelb_lb_set_alpha(hemelb_lb_t h, const float* alpha) {
    const Range range("hemelb_lb_set_alpha");
    return no_throw([&] { return set_alpha_impl(h, alpha); });
}

static int set_objective_impl(hemelb_lb_t h, const hemelb_objective_t* obj) {
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    HIP_TRY(hipStreamSynchronize(h->stream), "sync");
    for (void** p : {(void**)&h->d_out_links, (void**)&h->d_dome, (void**)&h->d_wss_w,
                     (void**)&h->d_qtape, (void**)&h->d_wtape, (void**)&h->d_opart})
        if (*p) {
            (void)hipFree(*p);
            *p = nullptr;
        }
    h->device_bytes -= h->obj_bytes;
    h->obj_bytes = 0;
    h->obj_set = false;
    h->adj_t = -1;
    if (!obj) return HEMELB_OK;
    if (obj->outlet < 0 || obj->outlet >= (int32_t)h->h_iolets.size())
        return fail(HEMELB_EINVAL, "objective outlet %d is not an iolet", obj->outlet);
    if (obj->t0 < 0 || obj->t1 < obj->t0) return fail(HEMELB_EINVAL, "bad objective window");
    if (!std::isfinite(obj->q_target) || !std::isfinite(obj->lam))
        return fail(HEMELB_EINVAL, "objective constants must be finite");
    std::vector<int32_t> outl, dome;
    for (int64_t l = 0; l < h->nghost; ++l)
        if (h->h_giol[l] == obj->outlet) outl.push_back((int32_t)l);
    std::vector<float> w;
    if (obj->dome) {
        for (int64_t m = 0; m < h->n; ++m)
            if (obj->dome[h->order[m]] && h->has_normal[m]) dome.push_back((int32_t)m);
        const int64_t W = obj->t1 - obj->t0;
        if (!dome.empty() && W > 0) {
            w.assign(h->n, 0.f);
            const double wt = obj->lam / ((double)W * (double)dome.size());
            for (int32_t m : dome) w[m] = (float)wt;
        }
    }
    const size_t nw = (size_t)std::max<int64_t>(1, obj->t1 - obj->t0);
    int rc;
    const int64_t before = h->device_bytes;
    if ((rc = dev_upload(h, &h->d_out_links, outl, "objective links"))) return rc;
    if ((rc = dev_upload(h, &h->d_dome, dome, "objective dome"))) return rc;
    if ((rc = dev_upload(h, &h->d_wss_w, w, "objective weights"))) return rc;
    std::vector<double> zeros(nw, 0.0);
    const std::vector<double> parts(
        2 * (size_t)hlb::objective_parts((int64_t)outl.size() + (int64_t)dome.size()), 0.0);
    if ((rc = dev_upload(h, &h->d_opart, parts, "objective partials"))) return rc;
    if ((rc = dev_upload(h, &h->d_qtape, zeros, "flux tape"))) return rc;
    if ((rc = dev_upload(h, &h->d_wtape, zeros, "shear tape"))) return rc;
    h->obj_bytes = h->device_bytes - before;
    h->n_out = (int32_t)outl.size();
    h->n_dome = (int64_t)dome.size();
    h->obj_outlet = obj->outlet;
    h->q_target = obj->q_target;
    h->lam = obj->lam;
    h->w0 = obj->t0;
    h->w1 = obj->t1;
    h->obj_set = true;
    return HEMELB_OK;
}

int hemelb_lb_set_objective(hemelb_lb_t h, const hemelb_objective_t* obj) {
    const Range range("hemelb_lb_set_objective");
    return no_throw([&] { return set_objective_impl(h, obj); });
}

int hemelb_lb_objective_value(hemelb_lb_t h, double* J, double* flux_term, double* wss_term) {
    const Range range("hemelb_lb_objective_value");
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    if (!h->obj_set) return fail(HEMELB_EORDER, "no objective set");
    if (h->t < h->w1)
        return fail(HEMELB_EORDER, "the forward run (t = %lld) has not reached the window end %lld",
                    (long long)h->t, (long long)h->w1);
    HIP_TRY(hipStreamSynchronize(h->stream), "sync");
    const int64_t W = h->w1 - h->w0;
    std::vector<double> q(std::max<int64_t>(W, 1)), w(std::max<int64_t>(W, 1));
    HIP_TRY(hipMemcpy(q.data(), h->d_qtape, q.size() * sizeof(double), hipMemcpyDeviceToHost), "tape");
    HIP_TRY(hipMemcpy(w.data(), h->d_wtape, w.size() * sizeof(double), hipMemcpyDeviceToHost), "tape");
    double fl = 0, ws = 0;
    for (int64_t k = 0; k < W; ++k) {
        fl += (q[k] - h->q_target) * (q[k] - h->q_target);
        ws += w[k];
    }
    if (W > 0 && h->n_dome > 0) ws *= h->lam / ((double)W * (double)h->n_dome);
    else ws = 0;
    if (J) *J = fl + ws;
    if (flux_term) *flux_term = fl;
    if (wss_term) *wss_term = ws;
    return HEMELB_OK;
}

int hemelb_lb_objective_flux(hemelb_lb_t h, double* q) {
    const Range range("hemelb_lb_objective_flux");
    if (!h || !q) return fail(HEMELB_EINVAL, "NULL argument");
    if (!h->obj_set) return fail(HEMELB_EORDER, "no objective set");
    HIP_TRY(hipStreamSynchronize(h->stream), "sync");
    const int64_t W = h->w1 - h->w0;
    if (W > 0)
        HIP_TRY(hipMemcpy(q, h->d_qtape, W * sizeof(double), hipMemcpyDeviceToHost), "tape");
    return HEMELB_OK;
}

static int adjoint_begin_impl(hemelb_lb_t h, int64_t max_segment) {
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    if (!h->obj_set) return fail(HEMELB_EORDER, "set an objective and run the forward first");
    if (h->bfl)
        return fail(HEMELB_EINVAL, "the adjoint covers halfway bounce-back walls only (no wall_q)");
    if (max_segment < 1) return fail(HEMELB_EINVAL, "max_segment must be >= 1");
    HIP_TRY(hipSetDevice(h->device), "set device");
    const size_t popbytes = (size_t)h->q * h->slots * h->elem();
    while ((int64_t)h->tape.size() < max_segment + 1) {
        void* p = nullptr;
        HIP_TRY(hipMalloc(&p, popbytes), "adjoint tape");
        h->tape.push_back(p);
        h->device_bytes += (int64_t)popbytes;
    }
    const size_t gcount = (size_t)h->q * h->slots;
    int rc;
    for (int b = 0; b < 2; ++b)
        if (!h->ghat[b] && (rc = dev_alloc(h, &h->ghat[b], gcount, "adjoint state"))) return rc;
    if (!h->alpha_hat && h->n > 0 && (rc = dev_alloc(h, &h->alpha_hat, (size_t)h->n, "alpha adjoint")))
        return rc;
    int32_t hmax = 0;
    for (auto& io : h->h_iolets)
        if (io.kind == HEMELB_IOLET_VELOCITY) hmax = std::max(hmax, io.n_harm);
    h->nbasis = 1 + 2 * hmax;
    h->basis_stride = 2 * hmax;
    if (!h->theta_acc && h->nghost > 0 &&
        (rc = dev_alloc(h, &h->theta_acc, (size_t)h->nghost * h->nbasis, "theta adjoint")))
        return rc;
    if (!h->is_site && h->nghost > 0) {
        std::vector<int32_t> st, lo, hi;
        for (int64_t l = 0; l < h->nghost;) {
            int64_t e = l;
            while (e < h->nghost && h->h_gsite[e] == h->h_gsite[l]) ++e;
            st.push_back(h->h_gsite[l]);
            lo.push_back((int32_t)l);
            hi.push_back((int32_t)e);
            l = e;
        }
        std::vector<int32_t> of_link((size_t)h->nghost);
        for (size_t k = 0; k < st.size(); ++k)
            for (int32_t l = lo[k]; l < hi[k]; ++l) of_link[l] = (int32_t)k;
        if ((rc = dev_upload(h, &h->is_link, of_link, "iolet link sites"))) return rc;
        if ((rc = dev_upload(h, &h->is_site, st, "iolet sites"))) return rc;
        if ((rc = dev_upload(h, &h->is_lo, lo, "iolet sites"))) return rc;
        if ((rc = dev_upload(h, &h->is_hi, hi, "iolet sites"))) return rc;
        h->n_is = (int64_t)st.size();
    }
    h->gcur = 0;
    hlb::Layout Lg = h->layout();
    Lg.storage = HEMELB_STORE_F32;
    HIP_TRY(hlb::launch_zero(Lg, h->ghat[0], h->stream), "adjoint zero");
    if (h->alpha_hat) HIP_TRY(hlb::launch_zero_words(h->alpha_hat, 2 * h->n, h->stream), "zero");
    if (h->theta_acc)
        HIP_TRY(hlb::launch_zero_words(h->theta_acc, 2 * h->nghost * h->nbasis, h->stream), "zero");
    h->adj_t = h->t;
    return HEMELB_OK;
}

int hemelb_lb_adjoint_begin(hemelb_lb_t h, int64_t max_segment) {
    const Range range("hemelb_lb_adjoint_begin");
    return no_throw([&] { return adjoint_begin_impl(h, max_segment); });
}

static int adjoint_segment_impl(hemelb_lb_t h, const void* checkpoint, int64_t t0, int64_t steps) {
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    if (h->adj_t < 0) return fail(HEMELB_EORDER, "call hemelb_lb_adjoint_begin first");
    if (steps < 1 || steps + 1 > (int64_t)h->tape.size())
        return fail(HEMELB_EINVAL, "segment of %lld steps exceeds the tape (%lld)", (long long)steps,
                    (long long)h->tape.size() - 1);
    if (t0 < 0 || t0 + steps != h->adj_t)
        return fail(HEMELB_EORDER, "segments must run backwards: expected one ending at %lld",
                    (long long)h->adj_t);
    if (!checkpoint && h->n > 0) return fail(HEMELB_EINVAL, "checkpoint is NULL");
    HIP_TRY(hipSetDevice(h->device), "set device");
    h->ghosts_ready = false;
    int rc = begin_recompute(h, h->tape, h->series[0], checkpoint, t0, steps, h->stream);
    for (int64_t m = 0; m < steps && !rc; ++m) rc = recompute_step(h, h->tape, h->series[0], t0, m, h->stream);
    for (int64_t m = steps - 1; m >= 0 && !rc; --m)
        rc = reverse_step(h, h->tape, nullptr, h->series[0], t0, m, steps, h->stream);
    if (!rc) rc = end_reverse(h, h->tape, h->series[0], t0, h->stream);
    if (rc) return rc;
    h->adj_t = t0;
    return HEMELB_OK;
}

int hemelb_lb_adjoint_segment(hemelb_lb_t h, const void* checkpoint, int64_t t0, int64_t steps) {
    const Range range("hemelb_lb_adjoint_segment");
    return no_throw([&] { return adjoint_segment_impl(h, checkpoint, t0, steps); });
}

static int adjoint_run_impl(hemelb_lb_t h, const void* const* checkpoints, const int64_t* t0,
                          const int64_t* steps, int64_t nseg) {
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    if (h->adj_t < 0) return fail(HEMELB_EORDER, "call hemelb_lb_adjoint_begin first");
    if (nseg < 0 || (nseg > 0 && (!checkpoints || !t0 || !steps)))
        return fail(HEMELB_EINVAL, "NULL segment arrays");
    if (nseg == 0) return HEMELB_OK;
    for (int64_t k = 0; k < nseg; ++k) {
        if (steps[k] < 1 || steps[k] + 1 > (int64_t)h->tape.size())
            return fail(HEMELB_EINVAL, "segment %lld of %lld steps exceeds the tape (%lld)",
                        (long long)k, (long long)steps[k], (long long)h->tape.size() - 1);
        if (!checkpoints[k] && h->n > 0) return fail(HEMELB_EINVAL, "checkpoint %lld is NULL", (long long)k);
        const int64_t end = k + 1 < nseg ? t0[k + 1] : h->adj_t;
        if (t0[k] < 0 || t0[k] + steps[k] != end)
            return fail(HEMELB_EORDER, "segment %lld must end where the next one starts (%lld)",
                        (long long)k, (long long)end);
    }
    HIP_TRY(hipSetDevice(h->device), "set device");
    h->ghosts_ready = false;
    const size_t popbytes = (size_t)h->q * h->slots * h->elem();
    while (h->tape2.size() < h->tape.size()) {
        void* p = nullptr;
        HIP_TRY(hipMalloc(&p, popbytes), "adjoint tape");
        h->tape2.push_back(p);
        h->device_bytes += (int64_t)popbytes;
    }
    std::vector<void*>* tapes[2] = {&h->tape, &h->tape2};
    // Segment k is recomputed into tape (nseg - 1 - k) & 1.  The reverse steps of
    // segment k pair with the recompute steps of segment k - 1 (the other tape and
    // series buffer): each pair is one launch, so a lattice too small to fill the
    // GPU keeps it busy with both, at half the launches.  One stream orders
    // everything, so results are those of the segments run one after another.
    int rc = begin_recompute(h, *tapes[0], h->series[0], checkpoints[nseg - 1], t0[nseg - 1],
                             steps[nseg - 1], h->stream);
    for (int64_t m = 0; m < steps[nseg - 1] && !rc; ++m)
        rc = recompute_step(h, *tapes[0], h->series[0], t0[nseg - 1], m, h->stream);
    if (rc) return rc;
    for (int64_t i = 0; i < nseg; ++i) {
        const int64_t k = nseg - 1 - i;
        const int b = (int)(i & 1), nb = b ^ 1;
        std::vector<void*>& tr = *tapes[b];
        std::vector<void*>& tf = *tapes[nb];
        const int64_t nr = k > 0 ? steps[k - 1] : 0;
        if (k > 0 && (rc = begin_recompute(h, tf, h->series[nb], checkpoints[k - 1], t0[k - 1],
                                           nr, h->stream)))
            return rc;
        for (int64_t m = 0; m < std::max(steps[k], nr); ++m) {
            const int64_t mr = steps[k] - 1 - m;
            if (m < steps[k] && m < nr)
                rc = dual_step(h, tf, h->series[nb], t0[k - 1], m, tr, h->series[b], t0[k], mr,
                               steps[k], h->stream);
            else if (m < steps[k])
                rc = reverse_step(h, tr, nullptr, h->series[b], t0[k], mr, steps[k], h->stream);
            else
                rc = recompute_step(h, tf, h->series[nb], t0[k - 1], m, h->stream);
            if (rc) return rc;
        }
        if ((rc = end_reverse(h, tr, h->series[b], t0[k], h->stream))) return rc;
    }
    h->adj_t = t0[0];
    return HEMELB_OK;
}

int hemelb_lb_adjoint_run(hemelb_lb_t h, const void* const* checkpoints, const int64_t* t0,
                          const int64_t* steps, int64_t nseg) {
    const Range range("hemelb_lb_adjoint_run");
    return no_throw([&] { return adjoint_run_impl(h, checkpoints, t0, steps, nseg); });
}

static int record_impl(hemelb_lb_t h, int64_t max_steps) {
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    if (max_steps < 1) return fail(HEMELB_EINVAL, "max_steps must be >= 1");
    if (h->rec_t0 >= 0) return fail(HEMELB_EORDER, "a trajectory is already being recorded");
    HIP_TRY(hipSetDevice(h->device), "set device");
    const size_t popbytes = (size_t)h->q * h->slots * h->elem();
    // max_steps + 1 states and, with FP32 storage and halfway walls, the pre-collision
    // populations of each recorded step when memory allows (with 16-bit storage the
    // reverse step's re-gather is as fast as reading them, so they are not kept)
    std::vector<void*> rec, frec;
    for (int64_t m = 0; m <= max_steps; ++m) {
        void* p = nullptr;
        const hipError_t e = hipMalloc(&p, popbytes);
        if (e != hipSuccess) {
            for (void* x : rec) (void)hipFree(x);
            return hip_fail(e, "trajectory record");
        }
        rec.push_back(p);
    }
    if (h->storage == HEMELB_STORE_F32 && !h->bfl) {
        for (int64_t m = 0; m < max_steps; ++m) {
            void* p = nullptr;
            if (hipMalloc(&p, popbytes) != hipSuccess) {  // states only: the reverse re-gathers
                (void)hipGetLastError();                  // leave no error for later calls
                for (void* x : frec) (void)hipFree(x);
                frec.clear();
                break;
            }
            frec.push_back(p);
        }
    }
    // the current state (with its ghost slots) starts the record
    HIP_TRY(hipMemcpyAsync(rec[0], h->A[h->cur], popbytes, hipMemcpyDeviceToDevice, h->stream),
            "record start");
    h->rec = std::move(rec);
    h->frec = std::move(frec);
    h->device_bytes += (int64_t)(popbytes * (h->rec.size() + h->frec.size()));
    h->A_own[0] = h->A[0];
    h->A_own[1] = h->A[1];
    h->A[h->cur] = h->rec[0];
    h->rec_t0 = h->t;
    return HEMELB_OK;
}

int hemelb_lb_record(hemelb_lb_t h, int64_t max_steps) {
    const Range range("hemelb_lb_record");
    return no_throw([&] { return record_impl(h, max_steps); });
}

int hemelb_lb_record_end(hemelb_lb_t h) {
    const Range range("hemelb_lb_record_end");
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    if (h->rec_t0 < 0) return HEMELB_OK;
    HIP_TRY(hipSetDevice(h->device), "set device");
    const size_t popbytes = (size_t)h->q * h->slots * h->elem();
    // the current and the previous state (observables re-gather the latter) move
    // back into the handle's own buffers
    for (int b = 0; b < 2; ++b)
        if (h->A[b] != h->A_own[b])
            HIP_TRY(hipMemcpyAsync(h->A_own[b], h->A[b], popbytes, hipMemcpyDeviceToDevice,
                                   h->stream),
                    "record end");
    HIP_TRY(hipStreamSynchronize(h->stream), "sync");
    h->A[0] = h->A_own[0];
    h->A[1] = h->A_own[1];
    for (void* p : h->rec) (void)hipFree(p);
    for (void* p : h->frec) (void)hipFree(p);
    h->device_bytes -= (int64_t)(popbytes * (h->rec.size() + h->frec.size()));
    h->rec.clear();
    h->frec.clear();
    h->rec_t0 = -1;
    return HEMELB_OK;
}

static int adjoint_recorded_impl(hemelb_lb_t h) {
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    if (h->adj_t < 0) return fail(HEMELB_EORDER, "call hemelb_lb_adjoint_begin first");
    if (h->rec_t0 < 0) return fail(HEMELB_EORDER, "no trajectory is being recorded");
    const int64_t steps = h->adj_t - h->rec_t0;
    if (steps < 1 || h->adj_t > h->t)
        return fail(HEMELB_EORDER, "the reverse sweep is at %lld; the record covers %lld .. %lld",
                    (long long)h->adj_t, (long long)h->rec_t0, (long long)h->t);
    HIP_TRY(hipSetDevice(h->device), "set device");
    h->ghosts_ready = false;
    int rc = fill_segment_series(h, h->series[0], h->rec_t0, steps + 1, h->stream);
    for (int64_t m = steps - 1; m >= 0 && !rc; --m)
        rc = reverse_step(h, h->rec, h->frec.empty() ? nullptr : &h->frec, h->series[0],
                          h->rec_t0, m, steps, h->stream);
    if (!rc) rc = end_reverse(h, h->rec, h->series[0], h->rec_t0, h->stream);
    if (rc) return rc;
    h->adj_t = h->rec_t0;
    return HEMELB_OK;
}

int hemelb_lb_adjoint_recorded(hemelb_lb_t h) {
    const Range range("hemelb_lb_adjoint_recorded");
    return no_throw([&] { return adjoint_recorded_impl(h); });
}

static int adjoint_grads_impl(hemelb_lb_t h, double* dtheta, double* dalpha) {
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    if (h->adj_t < 0) return fail(HEMELB_EORDER, "no adjoint run");
    HIP_TRY(hipStreamSynchronize(h->stream), "sync");
    if (dalpha) {
        std::vector<double> a(h->n, 0.0);
        if (h->n > 0)
            HIP_TRY(hipMemcpy(a.data(), h->alpha_hat, h->n * sizeof(double), hipMemcpyDeviceToHost),
                    "alpha adjoint");
        for (int64_t m = 0; m < h->n; ++m) dalpha[h->order[m]] = a[m];
    }
    if (dtheta) {
        std::vector<double> acc((size_t)h->nghost * h->nbasis, 0.0);
        if (!acc.empty())
            HIP_TRY(hipMemcpy(acc.data(), h->theta_acc, acc.size() * sizeof(double),
                              hipMemcpyDeviceToHost),
                    "theta adjoint");
        size_t off = 0;
        for (size_t k = 0; k < h->h_iolets.size(); ++k) {
            const auto& io = h->h_iolets[k];
            if (io.kind != HEMELB_IOLET_VELOCITY) continue;
            const int B = 1 + 2 * io.n_harm;
            for (int b = 0; b < B; ++b) dtheta[off + b] = 0.0;
            for (int64_t l = 0; l < h->nghost; ++l)
                if (h->h_giol[l] == k)
                    for (int b = 0; b < B; ++b) dtheta[off + b] += acc[(size_t)l * h->nbasis + b];
            off += B;
        }
    }
    return HEMELB_OK;
}

int hemelb_lb_adjoint_grads(hemelb_lb_t h, double* dtheta, double* dalpha) {
    const Range range("hemelb_lb_adjoint_grads");
    return no_throw([&] { return adjoint_grads_impl(h, dtheta, dalpha); });
}

static int get_adjoint_impl(hemelb_lb_t h, float* dst) {
    if (!h || (!dst && h->n > 0)) return fail(HEMELB_EINVAL, "NULL argument");
    if (h->adj_t < 0) return fail(HEMELB_EORDER, "no adjoint run");
    hlb::Layout Lg = h->layout();
    Lg.storage = HEMELB_STORE_F32;
    Lg.scaled = false;
    HIP_TRY(hlb::launch_state(Lg, h->ghat[h->gcur], dst, h->perm, 0, h->stream), "adjoint get");
    return HEMELB_OK;
}

int hemelb_lb_get_adjoint(hemelb_lb_t h, float* dst) {
    const Range range("hemelb_lb_get_adjoint");
    return no_throw([&] { return get_adjoint_impl(h, dst); });
}

}  // extern "C"
