// Host side of the C ABI: validation, Morton ordering, device neighbour table,
// ghost (iolet link) lists, memory management and the per-step launch loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hemelb_lb.h"
#include "kernels.hpp"

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

template <class F>
void parallel_for(int64_t n, F&& f) {
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 100000) nt = 1;
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t) {
        const int64_t a = n * t / nt, b = n * (t + 1) / nt;
        if (nt == 1) {
            f(a, b);
            return;
        }
        th.emplace_back([=, &f] { f(a, b); });
    }
    for (auto& x : th) x.join();
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
    int32_t* tbl = nullptr;
    int32_t* g_site = nullptr;
    uint8_t* g_dir = nullptr;
    uint8_t* g_iolet = nullptr;
    float* g_coef = nullptr;
    hlb::DevIolet* d_iolets = nullptr;
    double* d_harm = nullptr;
    int32_t* perm = nullptr;  // Morton index -> caller index (null: identity)
    float* normal = nullptr;  // [3][n] Morton order
    float* alpha = nullptr;
    double* partial = nullptr;
    double* tot = nullptr;
    int32_t* flag = nullptr;
    int64_t nparts = 1;

    int64_t t = 0;
    bool streamed = false;
    int xcd_group = 16;  // consecutive 256-site blocks per XCD (measured best at 8-16)
    int64_t check_every = 0;
    std::atomic<bool> cancel{false};

    std::vector<hipEvent_t> ev;
    int64_t ev_cap = 0, ev_used = 0;

    int64_t device_bytes = 0;

    hlb::Layout layout() const {
        return hlb::Layout{q, storage, scaled, n, slots, tbl};
    }
    hlb::Ghosts ghosts() const {
        return hlb::Ghosts{nghost, g_site, g_dir, g_iolet, g_coef, d_iolets, d_harm};
    }
    size_t elem() const { return storage == HEMELB_STORE_F32 ? 4 : 2; }
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
    if (h->stream || true) (void)hipStreamSynchronize(h->stream);
    void* ptrs[] = {h->A[0], h->A[1], h->tbl, h->g_site, h->g_dir, h->g_iolet, h->g_coef,
                    h->d_iolets, h->d_harm, h->perm, h->normal, h->alpha, h->partial, h->tot,
                    h->flag};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (auto e : h->ev) (void)hipEventDestroy(e);
    delete h;
}

int validate(const hemelb_lb_desc_t* d) {
    if (!d) return fail(HEMELB_EINVAL, "desc is NULL");
    if (d->lattice != 15 && d->lattice != 19)
        return fail(HEMELB_EINVAL, "lattice must be 15 or 19 (got %d)", d->lattice);
    if (d->storage < HEMELB_STORE_F32 || d->storage > HEMELB_STORE_BF16)
        return fail(HEMELB_EINVAL, "unknown storage %d", d->storage);
    if (d->flags & ~HEMELB_FLAG_NO_SCALE) return fail(HEMELB_EINVAL, "unknown flags 0x%x", d->flags);
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
    for (int64_t s = 0; s < n; ++s)
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
    return HEMELB_OK;
}

int do_step(hemelb_lb* h) {
    const hlb::Layout L = h->layout();
    void* src = h->A[h->cur];
    void* dst = h->A[h->cur ^ 1];
    HIP_TRY(hlb::launch_ghost_fill(L, h->ghosts(), src, h->t, h->stream), "ghost fill");
    const bool timed = h->ev_used + 2 <= (int64_t)h->ev.size() && h->ev_cap > 0;
    if (timed) HIP_TRY(hipEventRecord(h->ev[h->ev_used], h->stream), "event");
    HIP_TRY(hlb::launch_stream_collide(L, src, dst, h->omega, h->alpha, h->xcd_group, h->stream),
            "stream collide");
    if (timed) {
        HIP_TRY(hipEventRecord(h->ev[h->ev_used + 1], h->stream), "event");
        h->ev_used += 2;
    }
    h->cur ^= 1;
    h->t += 1;
    h->streamed = true;
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

}  // namespace

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

int hemelb_lb_links(const uint8_t* labels, const int32_t shape[3], const int32_t periodic[3],
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

int hemelb_lb_create(hemelb_lb_t* out, const hemelb_lb_desc_t* d) {
    if (!out) return fail(HEMELB_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(d);
    if (rc) return rc;
    hemelb_lb* h = new (std::nothrow) hemelb_lb();
    if (!h) return fail(HEMELB_ENOMEM, "handle allocation failed");
    h->q = d->lattice;
    h->storage = d->storage;
    h->flags = d->flags;
    h->scaled = d->storage != HEMELB_STORE_F32 && !(d->flags & HEMELB_FLAG_NO_SCALE);
    h->n = d->n_sites;
    h->tau = d->tau;
    h->omega = std::isinf(d->tau) ? 0.0f : (float)(1.0 / d->tau);
    h->stream = static_cast<hipStream_t>(d->stream);
    if (const char* e = getenv("HEMELB_XCD_GROUP")) h->xcd_group = std::max(0, atoi(e));
    (void)hipGetDevice(&h->device);
    const int q = h->q;
    const int64_t n = h->n;
    const HostLat lat = host_lattice(q);

    // Morton order: order[m] = caller index of the m-th site
    std::vector<int32_t> order(n), inv(n);
    std::iota(order.begin(), order.end(), 0);
    if (d->coords && n > 0) {
        struct KI {
            uint64_t key;
            int32_t idx;
        };
        std::vector<KI> ki(n);
        parallel_for(n, [&](int64_t a, int64_t b) {
            for (int64_t s = a; s < b; ++s)
                ki[s] = KI{morton(d->coords[3 * s], d->coords[3 * s + 1], d->coords[3 * s + 2]),
                           (int32_t)s};
        });
        std::sort(ki.begin(), ki.end(), [](const KI& a, const KI& b) {
            return a.key < b.key || (a.key == b.key && a.idx < b.idx);
        });
        for (int64_t m = 0; m < n; ++m) order[m] = ki[m].idx;
        for (int64_t m = 1; m < n; ++m)
            if (ki[m].key == ki[m - 1].key) {
                delete h;
                return fail(HEMELB_EINVAL, "duplicate coordinates at sites %d and %d",
                            ki[m - 1].idx, ki[m].idx);
            }
    }
    for (int64_t m = 0; m < n; ++m) inv[order[m]] = (int32_t)m;

    // ghost links in Morton site order, direction ascending
    std::vector<int32_t> gsite;
    std::vector<uint8_t> gdir, giol;
    std::vector<float> gcoef;
    for (int64_t m = 0; m < n; ++m) {
        const int64_t s = order[m];
        for (int i = 1; i < q; ++i) {
            const int32_t v = d->nbr[s * q + i];
            if (v <= -2) {
                const int k = -2 - v;
                gsite.push_back((int32_t)m);
                gdir.push_back((uint8_t)i);
                giol.push_back((uint8_t)k);
                double coef = 0.0;
                const hemelb_iolet_t& io = d->iolets[k];
                if (io.kind == HEMELB_IOLET_VELOCITY) {
                    const double W = d->site_weight ? d->site_weight[s] : 1.0;
                    const double ce = lat.c[i][0] * io.direction[0] + lat.c[i][1] * io.direction[1] +
                                      lat.c[i][2] * io.direction[2];
                    coef = 6.0 * lat.w[i] * ce * W;
                }
                gcoef.push_back((float)coef);
            }
        }
    }
    h->nghost = (int64_t)gsite.size();
    if (n + h->nghost >= ((int64_t)1 << 30)) {
        delete h;
        return fail(HEMELB_EINVAL, "sites + iolet links must stay below 2^30");
    }
    h->slots = ((n + h->nghost + hlb::kTile - 1) / hlb::kTile) * hlb::kTile;
    if (h->slots == 0) h->slots = hlb::kTile;
    h->ttiles = (n + hlb::kTile - 1) / hlb::kTile;
    if (h->ttiles == 0) h->ttiles = 1;

    // internal pull table [tile][q-1][64]: fluid -> Morton index of the upstream
    // site; wall -> own index with bit 31 set (read the opposite direction of the
    // same site); iolet -> ghost slot n + l
    std::vector<int32_t> tbl((size_t)h->ttiles * (q - 1) * hlb::kTile, 0);
    {
        std::vector<int64_t> gbase(n + 1, 0);
        for (int64_t l = 0; l < h->nghost; ++l) gbase[gsite[l] + 1]++;
        for (int64_t m = 0; m < n; ++m) gbase[m + 1] += gbase[m];
        for (int64_t m = 0; m < n; ++m) {
            const int64_t s = order[m];
            int64_t g = gbase[m];
            for (int i = 1; i < q; ++i) {
                const int32_t v = d->nbr[s * q + i];
                uint32_t e;
                if (v >= 0)
                    e = (uint32_t)inv[v];
                else if (v == HEMELB_LINK_WALL)
                    e = (uint32_t)m | 0x80000000u;
                else
                    e = (uint32_t)(n + (g++));
                const size_t at = ((size_t)(m / hlb::kTile) * (q - 1) + (i - 1)) * hlb::kTile +
                                  (size_t)(m % hlb::kTile);
                tbl[at] = (int32_t)e;
            }
        }
    }

    // wall normals [3][n] in Morton order
    std::vector<float> nrm((size_t)3 * n, 0.f);
    for (int64_t m = 0; m < n; ++m) {
        const int64_t s = order[m];
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
            for (int a = 0; a < 3; ++a) nrm[(size_t)a * n + m] = (float)(v[a] / nn);
    }

    // iolet descriptors and harmonics
    std::vector<hlb::DevIolet> dio(d->n_iolets);
    std::vector<double> harm;
    for (int k = 0; k < d->n_iolets; ++k) {
        const hemelb_iolet_t& io = d->iolets[k];
        dio[k].kind = io.kind == HEMELB_IOLET_PRESSURE ? 0 : 1;
        dio[k].n_harm = io.n_harm;
        dio[k].harm_off = (int32_t)harm.size();
        dio[k].pad = 0;
        dio[k].mean = io.mean;
        dio[k].period = io.n_harm > 0 ? io.period : 1.0;
        for (int hh = 0; hh < io.n_harm; ++hh) harm.push_back(io.cos_k[hh]);
        for (int hh = 0; hh < io.n_harm; ++hh) harm.push_back(io.sin_k[hh]);
    }

    std::vector<int32_t> perm;
    if (d->coords) perm = order;
    std::vector<float> alpha;
    if (d->alpha) {
        alpha.resize(n);
        for (int64_t m = 0; m < n; ++m) alpha[m] = d->alpha[order[m]];
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
    TRY(dev_upload(h, &h->tbl, tbl, "neighbour table"));
    TRY(dev_upload(h, &h->g_site, gsite, "ghost sites"));
    TRY(dev_upload(h, &h->g_dir, gdir, "ghost dirs"));
    TRY(dev_upload(h, &h->g_iolet, giol, "ghost iolets"));
    TRY(dev_upload(h, &h->g_coef, gcoef, "ghost coefs"));
    TRY(dev_upload(h, &h->d_iolets, dio, "iolets"));
    TRY(dev_upload(h, &h->d_harm, harm, "harmonics"));
    TRY(dev_upload(h, &h->perm, perm, "permutation"));
    TRY(dev_upload(h, &h->normal, nrm, "normals"));
    TRY(dev_upload(h, &h->alpha, alpha, "alpha"));
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
    *out = h;
    return HEMELB_OK;
}

int hemelb_lb_destroy(hemelb_lb_t h) {
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    release(h);
    return HEMELB_OK;
}

int hemelb_lb_step(hemelb_lb_t h, int64_t n) {
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    if (n < 0) return fail(HEMELB_EINVAL, "negative step count");
    HIP_TRY(hipSetDevice(h->device), "set device");
    for (int64_t k = 0; k < n; ++k) {
        if (h->cancel.exchange(false))
            return fail(HEMELB_ECANCELLED, "cancelled after %lld of %lld steps", (long long)k,
                        (long long)n);
        int rc = do_step(h);
        if (rc) return rc;
    }
    return HEMELB_OK;
}

int hemelb_lb_sync(hemelb_lb_t h) {
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
    if (!h) return fail(HEMELB_EINVAL, "NULL handle");
    const void* A = h->streamed ? h->A[h->cur ^ 1] : h->A[h->cur];
    HIP_TRY(hlb::launch_observables(h->layout(), A, h->streamed ? 1 : 0, h->omega, h->perm,
                                    h->normal, p, u, wss, h->stream),
            "observables");
    return HEMELB_OK;
}

int hemelb_lb_totals(hemelb_lb_t h, double out[4]) {
    if (!h || !out) return fail(HEMELB_EINVAL, "NULL argument");
    HIP_TRY(hlb::launch_totals(h->layout(), h->A[h->cur], h->partial, h->nparts, h->tot, h->flag,
                               h->stream),
            "totals");
    HIP_TRY(hipMemcpyAsync(out, h->tot, 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream),
            "totals readback");
    HIP_TRY(hipStreamSynchronize(h->stream), "totals sync");
    return HEMELB_OK;
}

static int state_io(hemelb_lb_t h, void* ext, int mode) {
    HIP_TRY(hlb::launch_state(h->layout(), h->A[h->cur], ext, h->perm, mode, h->stream), "state");
    return HEMELB_OK;
}

int hemelb_lb_get_state(hemelb_lb_t h, void* dst, int64_t* t) {
    if (!h || (!dst && h->n > 0)) return fail(HEMELB_EINVAL, "NULL argument");
    if (t) *t = h->t;
    return state_io(h, dst, 0);
}

int hemelb_lb_set_state(hemelb_lb_t h, const void* src, int64_t t) {
    if (!h || (!src && h->n > 0)) return fail(HEMELB_EINVAL, "NULL argument");
    if (t < 0) return fail(HEMELB_EINVAL, "negative time");
    h->t = t;
    h->streamed = false;
    return state_io(h, const_cast<void*>(src), 1);
}

int hemelb_lb_get_deviations(hemelb_lb_t h, float* dst) {
    if (!h || (!dst && h->n > 0)) return fail(HEMELB_EINVAL, "NULL argument");
    return state_io(h, dst, 2);
}

int hemelb_lb_set_deviations(hemelb_lb_t h, const float* src, int64_t t) {
    if (!h || (!src && h->n > 0)) return fail(HEMELB_EINVAL, "NULL argument");
    if (t < 0) return fail(HEMELB_EINVAL, "negative time");
    h->t = t;
    h->streamed = false;
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
    info->bytes_per_update = (int64_t)(2 * h->q * h->elem() + 4 * (h->q - 1));
    info->device_bytes = h->device_bytes;
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

int hemelb_copy_probe(void* dst, const void* src, int64_t bytes, void* stream) {
    if (!dst || !src || bytes <= 0 || (bytes % 16) || ((uintptr_t)dst % 16) || ((uintptr_t)src % 16))
        return fail(HEMELB_EINVAL, "copy probe needs 16-byte aligned pointers and size");
    HIP_TRY(hlb::launch_copy(dst, src, bytes, static_cast<hipStream_t>(stream)), "copy probe");
    return HEMELB_OK;
}

}  // extern "C"
