// Host-only driver of the library's planner, built with sanitizers by the test
// that runs it (no GPU is touched): reads a padded voxel label grid, builds the
// site list and upstream codes (hemelb_lb_links), then validates and plans every
// addressing form for both storages (hemelb_lb_plan), and prints one line per plan.
//
// Input file (little-endian): int32 X, Y, Z, px, py, pz, lattice, n_iolets; per
// iolet int32 kind and double direction[3], mean; then (X+2)(Y+2)(Z+2) uint8 labels.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hemelb_lb.h"

static bool read_all(FILE* f, void* p, size_t bytes) { return fread(p, 1, bytes, f) == bytes; }

int main(int argc, char** argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s labels.bin\n", argv[0]);
        return 2;
    }
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t hdr[8];
    if (!read_all(f, hdr, sizeof hdr)) return 2;
    const int32_t shape[3] = {hdr[0], hdr[1], hdr[2]};
    const int32_t periodic[3] = {hdr[3], hdr[4], hdr[5]};
    const int32_t q = hdr[6], nio = hdr[7];
    std::vector<hemelb_iolet_t> io((size_t)(nio > 0 ? nio : 1));
    for (int k = 0; k < nio; ++k) {
        int32_t kind;
        double v[4];
        if (!read_all(f, &kind, sizeof kind) || !read_all(f, v, sizeof v)) return 2;
        io[k] = hemelb_iolet_t{kind, {v[0], v[1], v[2]}, v[3], 0, nullptr, nullptr, 1.0};
    }
    const size_t cells = (size_t)(shape[0] + 2) * (shape[1] + 2) * (shape[2] + 2);
    std::vector<uint8_t> labels(cells);
    if (!read_all(f, labels.data(), cells)) return 2;
    fclose(f);

    int64_t n = 0;
    if (hemelb_lb_links(labels.data(), shape, periodic, q, &n, nullptr, nullptr)) {
        fprintf(stderr, "links: %s\n", hemelb_lb_last_error());
        return 1;
    }
    std::vector<int32_t> coords((size_t)n * 3), nbr((size_t)n * q);
    if (hemelb_lb_links(labels.data(), shape, periodic, q, &n, coords.data(), nbr.data())) {
        fprintf(stderr, "links: %s\n", hemelb_lb_last_error());
        return 1;
    }
    printf("sites %lld\n", (long long)n);
    const int32_t forms[3] = {HEMELB_FLAG_TABLE32, HEMELB_FLAG_TABLE16, HEMELB_FLAG_BLOCKS};
    for (int32_t st : {HEMELB_STORE_F32, HEMELB_STORE_F16}) {
        for (int32_t flag : forms) {
            hemelb_lb_desc_t d{};
            d.lattice = q;
            d.storage = st;
            d.flags = flag;
            d.n_sites = n;
            d.coords = coords.data();
            d.nbr = nbr.data();
            d.tau = 0.6;
            d.n_iolets = nio;
            d.iolets = io.data();
            hemelb_lb_info_t info{};
            const int rc = hemelb_lb_plan(&d, &info);
            printf("plan storage %d flag %d rc %d addressing %d ghosts %lld pitch %lld bpu %.6f "
                   "device %lld\n",
                   st, flag, rc, info.addressing, (long long)info.n_ghosts, (long long)info.pitch,
                   info.bytes_per_update, (long long)info.device_bytes);
        }
    }
    // a validation failure (a broken reciprocal link) must be reported, not crash
    if (n > 1) {
        std::vector<int32_t> bad = nbr;
        for (int64_t s = 0; s < n; ++s)
            for (int i = 1; i < q; ++i)
                if (bad[(size_t)s * q + i] >= 0) {
                    bad[(size_t)s * q + i] = (int32_t)((bad[(size_t)s * q + i] + 1) % n);
                    s = n;
                    break;
                }
        hemelb_lb_desc_t d{};
        d.lattice = q;
        d.storage = HEMELB_STORE_F32;
        d.n_sites = n;
        d.coords = coords.data();
        d.nbr = bad.data();
        d.tau = 0.6;
        d.n_iolets = nio;
        d.iolets = io.data();
        hemelb_lb_info_t info{};
        printf("broken rc %d\n", hemelb_lb_plan(&d, &info));
    }
    return 0;
}
