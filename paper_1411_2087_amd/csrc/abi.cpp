// Error reporting, geometry validation and small ABI queries of libhisq.so.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "hisq_common.hpp"

namespace hisq {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    return HISQ_EHIP;
}

int make_geom(const int dims[4], Geom &g)
{
    if (!dims) return fail(HISQ_EINVAL, "dims is NULL");
    long long V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (dims[mu] < 4 || (dims[mu] & 1))
            return fail(HISQ_EDIMS, "every lattice extent must be even and >= 4 (dims[" + std::to_string(mu) +
                                        "] = " + std::to_string(dims[mu]) + ")");
        g.L[mu] = dims[mu];
        V *= dims[mu];
    }
    if (V / 2 > (1LL << 30)) return fail(HISQ_EDIMS, "lattice too large (Vh must fit in 2^30)");
    g.Lxh = dims[0] / 2;
    g.Vh = (int)(V / 2);
    g.ntiles = (g.Vh + TILE - 1) / TILE;
    g.sy = g.Lxh;
    g.sz = g.Lxh * dims[1];
    g.st = g.Lxh * dims[1] * dims[2];
    g.oP = g.otb = g.ozb = g.ontb = 0;
    return HISQ_OK;
}

static int block_of(int L)
{
    for (int b : { 8, 6, 4, 2 })
        if (L % b == 0) return b;
    return 1;
}

static bool blocked_order(Geom &g, int tb, int zb)
{
    if ((g.Lxh * g.L[1]) % TILE) return false;
    if (tb <= 0) tb = block_of(g.L[3]);
    if (zb <= 0) zb = block_of(g.L[2]);
    if (g.L[3] % tb || g.L[2] % zb) return false;
    g.oP = g.Lxh * g.L[1] / TILE;
    g.otb = tb;
    g.ozb = zb;
    g.ontb = g.L[3] / g.otb;
    return true;
}

bool blocked_order(Geom &g) { return blocked_order(g, 0, 0); }

void apply_order(Geom &g, int order)
{
    switch (order) {
    case 1: blocked_order(g, 0, 0); break;
    case 2: blocked_order(g, 8, g.L[2]); break;
    case 3: blocked_order(g, 4, g.L[2]); break;
    case 4: blocked_order(g, 2, g.L[2]); break;
    case 5: blocked_order(g, 8, 16); break;
    default: break;
    }
}

}  // namespace hisq

extern "C" const char *hisq_last_error(void) { return hisq::g_last_error.c_str(); }

extern "C" const char *hisq_version(void) { return "hisq-mi355x 0.1 (gfx950)"; }
