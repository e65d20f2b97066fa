// Stand-ins for the library's kernel launchers, for host-only sanitizer builds of
// the planner: they let host.cpp link without any device code.  Every one
// reports that no device is present; the planner calls none of them.
#include "../../paper_1906_11925_amd/csrc/adjoint.hpp"
#include "../../paper_1906_11925_amd/csrc/kernels.hpp"
#include "../../paper_1906_11925_amd/csrc/render.hpp"

namespace hlb {

hipError_t launch_iolet_series(const DevIolet*, const double*, int32_t, int64_t, int64_t, double*,
                               double*, int32_t, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_ghost_fill(const Layout&, const Ghosts&, void*, int64_t, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_stream_collide(const Layout&, const Ghosts&, const void*, void*, float,
                                 const float*, int, int64_t, hipStream_t, void*) {
    return hipErrorNoDevice;
}
bool ghosts_fused() { return true; }
hipError_t launch_observables(const Layout&, const void*, int, float, const int32_t*,
                              const float*, float*, float*, float*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_totals(const Layout&, const void*, double*, int64_t, double*, int32_t*,
                         hipStream_t) {
    return hipErrorNoDevice;
}
// the planner sizes the totals' partial sums with this; same count as the kernels' file
int64_t totals_parts(int64_t n) {
    const int64_t nb = (n + kBlock - 1) / kBlock;
    return nb < 1 ? 1 : (nb > 1024 ? 1024 : nb);
}
hipError_t launch_totals_noalloc(const Layout&, const void*, double*, hipStream_t) {
    return hipErrorNoDevice;
}
int64_t totals_scratch_parts() { return 1024; }
hipError_t launch_state(const Layout&, void*, void*, const int32_t*, int, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_zero(const Layout&, void*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_copy(void*, const void*, int64_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_zero_words(void*, int64_t, hipStream_t) { return hipErrorNoDevice; }
int32_t objective_parts(int64_t) { return 1; }
hipError_t launch_objective(const Layout&, const Ghosts&, const void*, const Objective&,
                            const float*, float, double*, double*, double*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_adj_step(const Layout&, const Ghosts&, const IoletAdj&, int, const void*,
                           const void*, const void*, const float*, float*, float, const float*,
                           double*, const float*, const float*, int, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_adj_dual(const Layout&, const Ghosts&, const void*, void*, int64_t,
                           const Ghosts&, const IoletAdj&, int, const void*, const void*,
                           const float*, float*, float, const float*, double*, const float*,
                           const float*, int, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_render(const RenderVolume&, const RenderView&, const float*, float*,
                         hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_permute(const float*, const int32_t*, int64_t, float*, hipStream_t) {
    return hipErrorNoDevice;
}

}  // namespace hlb
