// Batched solves: many right-hand sides / many shifts (placeholder until the
// multi-RHS Dslash lands).
#include "cg_internal.hpp"

namespace hisq {
size_t cg_multi_workspace_bytes(const Geom &g, int nrhs, int mode)
{
    (void)g; (void)nrhs; (void)mode;
    return 0;
}
}  // namespace hisq

using namespace hisq;

extern "C" int cg_solve_multi(int nrhs, const double *masses, double tol, int mode, const void *fat, const void *lng,
                              const void *fat_lo, const void *lng_lo, const void *b, void *x, const int dims[4],
                              const hisq_cg_opts *opts, void *workspace, size_t ws_bytes, hisq_cg_stats *stats,
                              void *stream)
{
    (void)nrhs; (void)masses; (void)tol; (void)mode; (void)fat; (void)lng; (void)fat_lo; (void)lng_lo; (void)b;
    (void)x; (void)dims; (void)opts; (void)workspace; (void)ws_bytes; (void)stats; (void)stream;
    return fail(HISQ_EINVAL, "cg_solve_multi: not built yet");
}
