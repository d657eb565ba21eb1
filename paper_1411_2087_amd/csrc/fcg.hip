// Flexible CG on A x = b (even sites, FP64) preconditioned by the
// gauge-covariant network K (net.hip), with plain FP64 CG as the fallback.
//
// Notay's flexible CG with one stored direction, in the Polak-Ribiere form
// of the direction update (Golub & Ye 1999), which tolerates a preconditioner
// that is only approximately symmetric (K runs in FP32 features with BF16
// channel mixing):
//     z_k = K(r_k)
//     beta_k = Re<z_k, r_k - r_{k-1}> / Re<z_{k-1}, r_{k-1}>   (beta_0 = 0)
//     p_k = z_k + beta_k p_{k-1}
//     alpha_k = Re<z_k, r_k> / Re<p_k, A p_k>
//     x += alpha_k p_k,  r -= alpha_k A p_k
// If Re<z, r> <= 0 or Re<p, A p> <= 0 (K not positive on r), or the lowest
// residual has not halved over a window of FCG_WINDOW iterations, the solve
// hands x to plain FP64 CG.  The final residual b - A x is recomputed in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "cg_internal.hpp"

namespace hisq {

int net_prep_dispatch(const Geom &g, const void *W, int C, void *acts, int batch, hipStream_t s);
int net_layers_dispatch(const Geom &g, const void *fat, const void *W, int C, void *acts, int batch, hipStream_t s);
void net_acts_io(void *acts, const Geom &g, int C, int batch, void **in_full, void **out_full);
size_t net_act_bytes_g(const Geom &g, int C, int batch);
int cg_plain_f64(double mass, double tol, const void *fat, const void *lng, const void *b, void *x, const Geom &g,
                 const hisq_cg_opts &o, void *ws, size_t ws_bytes, hisq_cg_stats &stats, hipStream_t s);
size_t cg_workspace_bytes(const Geom &g, int mode);

struct FState {
    SolverFlags flags;  // done: converged or handed to the fallback
    int iter;
    int fallback;       // 1: K not positive on r / A-product <= 0 ; 2: too slow (progress rule)
    int window_start;   // iteration at which the current progress window opened
    double m4, bb, stop2, rr, best_rr, zr, zr_old, zrp, pAp, alpha, beta, rr_true;
    double rr_window;   // lowest |r|^2 when the window opened
};
// progress rule: over every FCG_WINDOW iterations the lowest |r| reached must
// fall below half the lowest before the window (|r|^2 / 4), otherwise the
// preconditioner is not paying for itself and plain CG takes over.  The rule
// watches the lowest |r|, not the current one: flexible CG minimises the
// A-norm of the error, and |r| rises for tens of iterations at a time (with a
// trained network at m = 0.005 it stays above its first value for ~100
// iterations, the FP64 oracle's flexible CG included); plain CG at such
// masses needs ~400 iterations per decade.
constexpr int FCG_WINDOW = 1000;

constexpr int F_NT = 256;
constexpr int F_U = 4;

static int f_blocks(long long n) { return (int)std::max<long long>(1, (n + F_NT * F_U - 1) / (F_NT * F_U)); }

__device__ __forceinline__ long long f_index(int j) { return ((long long)blockIdx.x * F_U + j) * F_NT + threadIdx.x; }

// r32 = float(r)
__global__ __launch_bounds__(F_NT) void k_f_tofloat(const double2 *__restrict__ r, float2 *__restrict__ r32,
                                                    long long n, const FState *st)
{
    if (st->flags.done) return;
#pragma unroll
    for (int j = 0; j < F_U; ++j) {
        const long long i = f_index(j);
        if (i < n) r32[i] = make_float2((float)r[i].x, (float)r[i].y);
    }
}

// z = double(z32); partials of Re<z, r> and Re<z, r_prev>
__global__ __launch_bounds__(F_NT) void k_f_z(const float2 *__restrict__ z32, double2 *__restrict__ z,
                                              const double2 *__restrict__ r, const double2 *__restrict__ rp,
                                              long long n, double *partials, const FState *st)
{
    if (st->flags.done) return;
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int j = 0; j < F_U; ++j) {
        const long long i = f_index(j);
        if (i < n) {
            const double2 zv = make_double2(z32[i].x, z32[i].y);
            z[i] = zv;
            const double2 rv = r[i], pv = rp[i];
            a = fma(zv.x, rv.x, fma(zv.y, rv.y, a));
            b = fma(zv.x, pv.x, fma(zv.y, pv.y, b));
        }
    }
    __shared__ double lds[2 * (F_NT / 64)];
    block_sum2<F_NT>(a, b, lds);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = a;
        partials[2 * blockIdx.x + 1] = b;
    }
}

// p = z + beta p
__global__ __launch_bounds__(F_NT) void k_f_p(double2 *__restrict__ p, const double2 *__restrict__ z, long long n,
                                              const FState *st)
{
    if (st->flags.done) return;
    const double be = st->beta;
#pragma unroll
    for (int j = 0; j < F_U; ++j) {
        const long long i = f_index(j);
        if (i < n) {
            double2 pv = p[i];
            const double2 zv = z[i];
            pv.x = fma(be, pv.x, zv.x);
            pv.y = fma(be, pv.y, zv.y);
            p[i] = pv;
        }
    }
}

// Ap = m4 p - D_eo t ; partials of Re<p, Ap>
__global__ __launch_bounds__(256) HISQ_WAVES(8) void k_f_ap(Geom g, const char *__restrict__ fat,
                                                         const char *__restrict__ lng, const double2 *__restrict__ t,
                                                         const double2 *__restrict__ p, double2 *__restrict__ ap,
                                                         int nblocks, double *partials, const FState *st)
{
    if (st->flags.done) return;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    if (blk >= nblocks) return;
    const int tile = blk * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63, h = tile * TILE + lane;
    double s = 0.0;
    if (tile < g.ntiles) {
        const int hc = h < g.Vh ? h : g.Vh - 1;
        double acc[6];
        dslash_site<PF64>(g, fat, lng, t, 0, tile, lane, hc, acc);
        if (h < g.Vh) {
            const double m = st->m4;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double2 pv = p[(size_t)h * 3 + c];
                double2 v;
                v.x = fma(m, pv.x, -acc[2 * c]);
                v.y = fma(m, pv.y, -acc[2 * c + 1]);
                ap[(size_t)h * 3 + c] = v;
                s = fma(pv.x, v.x, fma(pv.y, v.y, s));
            }
        }
    }
    block_partial<256>(s, partials, blk);
}

// x += alpha p ; r_prev = r ; r -= alpha Ap ; r32 = float(r) ; partials of |r|^2
__global__ __launch_bounds__(F_NT) void k_f_upd(double2 *__restrict__ x, double2 *__restrict__ r,
                                                double2 *__restrict__ rp, const double2 *__restrict__ p,
                                                const double2 *__restrict__ ap, float2 *__restrict__ r32, long long n,
                                                double *partials, const FState *st)
{
    if (st->flags.done) return;
    const double al = st->alpha;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < F_U; ++j) {
        const long long i = f_index(j);
        if (i < n) {
            double2 xv = x[i], rv = r[i];
            const double2 pv = p[i], av = ap[i];
            rp[i] = rv;
            xv.x = fma(al, pv.x, xv.x);
            xv.y = fma(al, pv.y, xv.y);
            rv.x = fma(-al, av.x, rv.x);
            rv.y = fma(-al, av.y, rv.y);
            x[i] = xv;
            r[i] = rv;
            r32[i] = make_float2((float)rv.x, (float)rv.y);  // the next application's network input
            s = fma(rv.x, rv.x, fma(rv.y, rv.y, s));
        }
    }
    block_partial<F_NT>(s, partials, blockIdx.x);
}

// r = b - (m4 x - D_eo t) ; partials of |r|^2   (init, final check)
__global__ __launch_bounds__(256) HISQ_WAVES(8) void k_f_resid(Geom g, const char *__restrict__ fat,
                                                            const char *__restrict__ lng,
                                                            const double2 *__restrict__ t,
                                                            const double2 *__restrict__ x,
                                                            const double2 *__restrict__ b, double2 *__restrict__ r,
                                                            double2 *__restrict__ rp, int nblocks, double *partials,
                                                            const FState *st)
{
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    if (blk >= nblocks) return;
    const int tile = blk * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63, h = tile * TILE + lane;
    double s = 0.0;
    if (tile < g.ntiles) {
        const int hc = h < g.Vh ? h : g.Vh - 1;
        double acc[6];
        dslash_site<PF64>(g, fat, lng, t, 0, tile, lane, hc, acc);
        if (h < g.Vh) {
            const double m = st->m4;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const size_t i = (size_t)h * 3 + c;
                const double2 xv = x[i], bv = b[i];
                double2 v;
                v.x = bv.x - fma(m, xv.x, -acc[2 * c]);
                v.y = bv.y - fma(m, xv.y, -acc[2 * c + 1]);
                r[i] = v;
                if (rp) rp[i] = v;
                s = fma(v.x, v.x, fma(v.y, v.y, s));
            }
        }
    }
    block_partial<256>(s, partials, blk);
}

enum { FF_BB = 0, FF_INIT = 1, FF_Z = 2, FF_PAP = 3, FF_UPD = 4, FF_TRUE = 5 };

__global__ __launch_bounds__(256) void k_f_fin(const double *__restrict__ partials, int nb, int pairs, FState *st,
                                               int mode)
{
    if (st->flags.done && (mode == FF_Z || mode == FF_PAP || mode == FF_UPD)) return;
    __shared__ double lds[2 * 4];
    double acc[2] = { 0.0, 0.0 };
    if (pairs) strided_sums<256, 2, 4>(partials, nb, acc);
    else strided_sums<256, 1, 8>(partials, nb, acc);
    double a = acc[0], b = acc[1];
    block_sum2<256>(a, b, lds);
    if (threadIdx.x) return;
    switch (mode) {
    case FF_BB: st->bb = a; st->stop2 = st->stop2 * a; break;  // stop2 holds tol^2 until here
    case FF_INIT:
        st->rr = st->best_rr = st->rr_true = st->rr_window = a;
        st->window_start = 0;
        st->flags.done = a <= st->stop2;
        break;
    case FF_Z:
        st->zrp = b;
        if (!(a > 0.0) || !isfinite(a)) { st->fallback = 1; st->flags.done = 1; break; }
        st->beta = st->iter == 0 ? 0.0 : (a - b) / st->zr_old;
        st->zr = a;
        break;
    case FF_PAP:
        st->pAp = a;
        if (!(a > 0.0) || !isfinite(a)) { st->fallback = 1; st->flags.done = 1; break; }
        st->alpha = st->zr / a;
        break;
    case FF_UPD:
        st->iter += 1;
        st->rr = a;
        st->zr_old = st->zr;
        if (!isfinite(a)) { st->fallback = 1; st->flags.done = 1; break; }
        if (a <= st->stop2) { st->flags.done = 1; break; }
        if (a < st->best_rr) st->best_rr = a;
        if (st->iter - st->window_start >= FCG_WINDOW) {
            // the lowest |r| of the window must be below half the lowest before it
            if (st->best_rr > 0.25 * st->rr_window) { st->fallback = 2; st->flags.done = 1; break; }
            st->rr_window = st->best_rr;
            st->window_start = st->iter;
        }
        break;
    case FF_TRUE: st->rr_true = a; break;
    }
}

__global__ void k_f_init(FState *st, double tol2, double m4)
{
    if (threadIdx.x || blockIdx.x) return;
    st->flags.done = 0;
    st->flags.reliable = 0;
    st->iter = st->fallback = st->window_start = 0;
    st->rr_window = 0.0;
    st->m4 = m4;
    st->stop2 = tol2;
    st->bb = st->rr = st->best_rr = st->zr = st->zr_old = st->zrp = st->pAp = st->alpha = st->beta = st->rr_true = 0.0;
}

// partials of |b|^2
__global__ __launch_bounds__(F_NT) void k_f_norm(const double2 *__restrict__ b, long long n, double *partials)
{
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < F_U; ++j) {
        const long long i = f_index(j);
        if (i < n) s = fma(b[i].x, b[i].x, fma(b[i].y, b[i].y, s));
    }
    block_partial<F_NT>(s, partials, blockIdx.x);
}

static size_t a256f(size_t v) { return (v + 255) & ~(size_t)255; }
static_assert(sizeof(FState) <= PIN_SLOT_BYTES, "FState does not fit its pinned slot");

// Byte model of one flexible-CG iteration.  The network on the full lattice
// (V = 2 Vh sites): per layer the fat links (each matrix serves two sites, so
// four per site at 72 bytes) and the input and output features (24 bytes per
// channel); the embedding and extraction of the even vector.  Per even site:
// two FP64 Dslash link streams and 20 FP64-vector equivalents of streams
// (r to FP32, z from FP32 with the two dot products, p, the two Dslash
// sources and outputs, A p, x, r, r_prev).
static double fcg_iter_bytes(const Geom &g, int C)
{
    const double layers = 4 * 4 * 72.0 + 24.0 * ((1 + C) + 2 * (C + C) + (C + 1));
    const double net = layers * 2 * g.Vh + (24.0 + 2 * 24.0 + 2 * 24.0 + 24.0) * g.Vh;
    return net + (2 * link_bytes_site(HISQ_F64) + 20 * 48.0) * g.Vh;
}

size_t fcg_ws_bytes(const Geom &g, int C)
{
    const size_t v64 = a256f((size_t)g.Vh * 3 * 16);
    const size_t nparts = std::max<size_t>((size_t)(g.ntiles + 3) / 4, 2 * (size_t)f_blocks((long long)g.Vh * 3)) + 64;
    const size_t own = a256f(sizeof(FState)) + a256f(nparts * sizeof(double)) + 7 * v64 +
                       a256f(net_act_bytes_g(g, C, 1));
    return std::max(own, cg_workspace_bytes(g, HISQ_CG_PLAIN_F64));
}

static int fcg_impl(double mass, double tol, const void *fat, const void *lng, const void *fat32, const void *W,
                    int C, const void *b, void *x, const Geom &g, const hisq_cg_opts &o, void *ws, size_t ws_bytes,
                    hisq_cg_stats &stats, hipStream_t s)
{
    char *p = (char *)ws;
    auto take = [&](size_t n) { void *r = p; p += a256f(n); return r; };
    const size_t v64 = (size_t)g.Vh * 3 * 16, v32 = (size_t)g.Vh * 3 * 8;
    const long long n = (long long)g.Vh * 3;
    const int nbf = f_blocks(n), nbd = (g.ntiles + 3) / 4;
    const size_t nparts = std::max<size_t>((size_t)nbd, 2 * (size_t)nbf) + 64;
    FState *st = (FState *)take(sizeof(FState));
    double *part = (double *)take(nparts * sizeof(double));
    double2 *r = (double2 *)take(v64), *rp = (double2 *)take(v64), *z = (double2 *)take(v64),
            *pv = (double2 *)take(v64), *ap = (double2 *)take(v64), *t = (double2 *)take(v64);
    take(v64);
    void *acts = take(net_act_bytes_g(g, C, 1));
    // the network's input slot takes float(r) on the even sites (its odd half stays zero) and its output slot's
    // even half is z: no embedding or extraction per application
    void *in_full = nullptr, *out_full = nullptr;
    net_acts_io(acts, g, C, 1, &in_full, &out_full);
    float2 *r32 = (float2 *)in_full;
    const float2 *z32 = (const float2 *)out_full;
    FState *hs = (FState *)pinned_slot(PIN_FCG);
    if (!hs) return fail(HISQ_EHIP, "fcg_solve: pinned state allocation failed");
    const dim3 gb(nbf), gd(xcd_grid(nbd));
    auto t0 = std::chrono::steady_clock::now();
    hipLaunchKernelGGL(k_f_init, dim3(1), dim3(1), 0, s, st, tol * tol, 4.0 * mass * mass);
    HISQ_HIP(hipMemsetAsync(r32 + (size_t)g.Vh * 3, 0, v32, s));  // the odd half of the network's input
    if (net_prep_dispatch(g, W, C, acts, 1, s)) return HISQ_EHIP;
    hipLaunchKernelGGL(k_f_norm, gb, dim3(F_NT), 0, s, (const double2 *)b, n, part);
    hipLaunchKernelGGL(k_f_fin, dim3(1), dim3(256), 0, s, (const double *)part, nbf, 0, st, (int)FF_BB);
    // r = r_prev = b - A x0
    HISQ_HIP(launch_dslash<PF64>(g, fat, lng, x, t, 1, s));
    hipLaunchKernelGGL(k_f_resid, gd, dim3(256), 0, s, g, (const char *)fat, (const char *)lng, (const double2 *)t,
                       (const double2 *)x, (const double2 *)b, r, rp, nbd, part, (const FState *)st);
    hipLaunchKernelGGL(k_f_fin, dim3(1), dim3(256), 0, s, (const double *)part, nbd, 0, st, (int)FF_INIT);
    // the first network input; later ones come from k_f_upd
    hipLaunchKernelGGL(k_f_tofloat, gb, dim3(F_NT), 0, s, (const double2 *)r, r32, n, (const FState *)st);
    HISQ_HIP(hipGetLastError());
    HISQ_HIP(hipMemcpyAsync(hs, st, sizeof(FState), hipMemcpyDeviceToHost, s));
    HISQ_HIP(hipStreamSynchronize(s));
    if (hs->bb == 0.0) {
        HISQ_HIP(hipMemsetAsync(x, 0, v64, s));
        HISQ_HIP(hipStreamSynchronize(s));
        stats.iters = 0;
        stats.true_resid = 0.0;
        stats.status = HISQ_OK;
        stats.time_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return HISQ_OK;
    }
    auto iter = [&](hipStream_t q) -> hipError_t {
        int rc = net_layers_dispatch(g, fat32, W, C, acts, 1, q);
        if (rc) return hipErrorUnknown;
        hipLaunchKernelGGL(k_f_z, gb, dim3(F_NT), 0, q, z32, z, (const double2 *)r, (const double2 *)rp,
                           n, part, (const FState *)st);
        hipLaunchKernelGGL(k_f_fin, dim3(1), dim3(256), 0, q, (const double *)part, nbf, 1, st, (int)FF_Z);
        hipLaunchKernelGGL(k_f_p, gb, dim3(F_NT), 0, q, pv, (const double2 *)z, n, (const FState *)st);
        hipError_t e = launch_dslash<PF64>(g, fat, lng, pv, t, 1, q, &st->flags, GATE_NOT_DONE);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_f_ap, gd, dim3(256), 0, q, g, (const char *)fat, (const char *)lng, (const double2 *)t,
                           (const double2 *)pv, ap, nbd, part, (const FState *)st);
        hipLaunchKernelGGL(k_f_fin, dim3(1), dim3(256), 0, q, (const double *)part, nbd, 0, st, (int)FF_PAP);
        hipLaunchKernelGGL(k_f_upd, gb, dim3(F_NT), 0, q, (double2 *)x, r, rp, (const double2 *)pv, (const double2 *)ap,
                           r32, n, part, (const FState *)st);
        hipLaunchKernelGGL(k_f_fin, dim3(1), dim3(256), 0, q, (const double *)part, nbf, 0, st, (int)FF_UPD);
        return hipGetLastError();
    };
    // K iterations per host check, replayed as a graph
    int rc = HISQ_OK;
    {
        hipGraphExec_t exec = nullptr;
        hipGraph_t graph = nullptr;
        const int K = std::max(1, o.check_every);
        if (o.use_graph) {
            hipStream_t cs = capture_stream();
            if (!cs) return fail(HISQ_EHIP, "fcg_solve: cannot create capture stream");
            HISQ_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            hipError_t e = hipSuccess;
            for (int k = 0; k < K && e == hipSuccess; ++k) e = iter(cs);
            hipGraph_t gtmp = nullptr;
            hipError_t e2 = hipStreamEndCapture(cs, &gtmp);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (gtmp) hipGraphDestroy(gtmp);
                return hip_fail(e != hipSuccess ? e : e2, "fcg_solve: capture");
            }
            graph = gtmp;
            HISQ_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        }
        int queued = 0;
        while (!hs->flags.done && queued < o.max_iter) {
            const int k = std::min(K, o.max_iter - queued);
            hipError_t e = hipSuccess;
            if (exec && k == K) e = hipGraphLaunch(exec, s);
            else for (int i = 0; i < k && e == hipSuccess; ++i) e = iter(s);
            if (e == hipSuccess) e = hipMemcpyAsync(hs, st, sizeof(FState), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) { rc = hip_fail(e, "fcg_solve: iteration"); break; }
            queued += k;
        }
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        if (rc) return rc;
    }
    const int fcg_iters = hs->iter;
    const int fell_back = hs->fallback;
    stats.iters = fcg_iters;
    stats.iter_resid = std::sqrt(hs->rr / hs->bb);
    stats.bytes_moved = (fcg_iters * fcg_iter_bytes(g, C) + 2 * (2 * link_bytes_site(HISQ_F64) + 6 * 48.0) * g.Vh);
    stats.fallback_used = 0;
    stats.fallback_iters = 0;
    if (fell_back || !(hs->rr <= hs->stop2)) {
        // true residual first: stop if already converged, else continue with plain CG from x
        HISQ_HIP(launch_dslash<PF64>(g, fat, lng, x, t, 1, s));
        hipLaunchKernelGGL(k_f_resid, gd, dim3(256), 0, s, g, (const char *)fat, (const char *)lng, (const double2 *)t,
                           (const double2 *)x, (const double2 *)b, r, (double2 *)nullptr, nbd, part, (const FState *)st);
        hipLaunchKernelGGL(k_f_fin, dim3(1), dim3(256), 0, s, (const double *)part, nbd, 0, st, (int)FF_TRUE);
        HISQ_HIP(hipMemcpyAsync(hs, st, sizeof(FState), hipMemcpyDeviceToHost, s));
        HISQ_HIP(hipStreamSynchronize(s));
        if (!(hs->rr_true <= hs->stop2) && fcg_iters < o.max_iter) {
            hisq_cg_opts o2 = o;
            o2.max_iter = std::max(1, o.max_iter - fcg_iters);
            hisq_cg_stats s2;
            std::memset(&s2, 0, sizeof s2);
            const int rc2 = cg_plain_f64(mass, tol, fat, lng, b, x, g, o2, ws, ws_bytes, s2, s);
            stats.fallback_used = fell_back ? fell_back : 3;
            stats.fallback_iters = s2.iters;
            stats.iters = fcg_iters + s2.iters;
            stats.true_resid = s2.true_resid;
            stats.iter_resid = s2.iter_resid;
            stats.bytes_moved += s2.bytes_moved;
            stats.status = rc2;
            stats.time_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            return rc2;
        }
    } else {
        HISQ_HIP(launch_dslash<PF64>(g, fat, lng, x, t, 1, s));
        hipLaunchKernelGGL(k_f_resid, gd, dim3(256), 0, s, g, (const char *)fat, (const char *)lng, (const double2 *)t,
                           (const double2 *)x, (const double2 *)b, r, (double2 *)nullptr, nbd, part, (const FState *)st);
        hipLaunchKernelGGL(k_f_fin, dim3(1), dim3(256), 0, s, (const double *)part, nbd, 0, st, (int)FF_TRUE);
        HISQ_HIP(hipMemcpyAsync(hs, st, sizeof(FState), hipMemcpyDeviceToHost, s));
        HISQ_HIP(hipStreamSynchronize(s));
        if (!(hs->rr_true <= hs->stop2)) {
            // recursion said converged, the true residual disagrees: finish with plain CG
            hisq_cg_opts o2 = o;
            o2.max_iter = std::max(1, o.max_iter - fcg_iters);
            hisq_cg_stats s2;
            std::memset(&s2, 0, sizeof s2);
            const int rc2 = cg_plain_f64(mass, tol, fat, lng, b, x, g, o2, ws, ws_bytes, s2, s);
            stats.fallback_used = 3;
            stats.fallback_iters = s2.iters;
            stats.iters = fcg_iters + s2.iters;
            stats.true_resid = s2.true_resid;
            stats.iter_resid = s2.iter_resid;
            stats.bytes_moved += s2.bytes_moved;
            stats.status = rc2;
            stats.time_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            return rc2;
        }
    }
    stats.true_resid = std::sqrt(hs->rr_true / hs->bb);
    stats.status = stats.true_resid <= tol ? HISQ_OK : HISQ_ENOCONV;
    stats.time_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats.status) return fail(stats.status, "fcg_solve: not converged within max_iter");
    return HISQ_OK;
}

}  // namespace hisq

using namespace hisq;

extern "C" int fcg_solve(double mass, double tol, const void *fat, const void *lng, const void *fat32,
                         const void *weights, int channels, const void *b, void *x, const int dims[4],
                         const hisq_cg_opts *opts, void *workspace, size_t ws_bytes, hisq_cg_stats *stats,
                         void *stream)
{
    hisq_cg_stats local;
    hisq_cg_stats &st = stats ? *stats : local;
    std::memset(&st, 0, sizeof(st));
    Geom g;
    int rc = make_geom(dims, g);
    if (rc) return st.status = rc;
    if (channels != 4 && channels != 8 && channels != 16)
        return st.status = fail(HISQ_EINVAL, "fcg_solve: channels must be 4, 8 or 16");
    if (!fat || !lng || !fat32 || !weights || !b || !x) return st.status = fail(HISQ_EINVAL, "fcg_solve: NULL pointer");
    if (b == x) return st.status = fail(HISQ_EALIAS, "fcg_solve: b and x alias");
    if (!(tol > 0) || !(mass >= 0)) return st.status = fail(HISQ_EINVAL, "fcg_solve: need tol > 0 and mass >= 0");
    if (!workspace || ws_bytes < fcg_ws_bytes(g, channels))
        return st.status = fail(HISQ_EWORKSPACE, "fcg_solve: workspace NULL or smaller than hisq_workspace_bytes()");
    if (!aligned16({fat, lng, fat32, weights, b, x, workspace}))
        return st.status = fail(HISQ_EINVAL, "fcg_solve: device pointers must be 16-byte aligned");
    hisq_cg_opts o = resolve_opts(opts, g);
    if (!opts || opts->check_every <= 0) o.check_every = 10;
    hipStream_t s = (hipStream_t)stream;
    HISQ_HIP(hipStreamSynchronize(s));
    rc = fcg_impl(mass, tol, fat, lng, fat32, weights, channels, b, x, g, o, workspace, ws_bytes, st, s);
    st.status = rc;
    return rc;
}
