// Even-odd conjugate gradient on A = 4 m^2 - D_eo D_oe (Sec. 3 CG driven by
// the Dslash; Sec. 4 even-odd preconditioning), plain FP64 and mixed
// precision with reliable updates.
//
// Everything stays on the GPU: alpha, beta and the residual norms live in a
// device-resident state block, every dot product is a deterministic
// two-stage reduction (wave64 butterfly -> per-workgroup partial -> a
// one-workgroup finaliser kernel sums the partials in a fixed order and
// updates the scalars), and kernels read the
// state's `done` flag so iterations queued past convergence cost one launch
// each and change nothing.  The host only looks at the state every
// `check_every` iterations; those iterations are replayed as one captured
// HIP graph.
//
// Per iteration (plain FP64):
//   t  = D_oe p ; |t|^2                                 (Dslash + norm epilogue)
//   pAp = 4m^2 |p|^2 + |t|^2 ; alpha                    (D_eo = -D_oe^dag, so
//                                                        <p, A p> needs no second pass)
//   x += alpha p ; r -= alpha (4m^2 p - D_eo t) ; |r|^2 (Dslash + update epilogue:
//                                                        A p never goes to memory)
//   beta ; p = r + beta p ; |p|^2                       (one BLAS pass)
// Mixed precision (Sleijpen & van der Vorst 1996 reliable updates, in the
// form used for lattice QCD by Clark et al. 2010): the same iteration on FP32
// vectors with FP32 or FP16+scale links and FP64 dot accumulation; when
// |r_inner| < delta * max|r_inner| since the last update (or the inner
// residual meets tol) the FP64 solution absorbs x_inner, the true residual
// b - A x is recomputed with the FP64 operator and the inner residual is
// replaced by it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "cg_internal.hpp"

namespace hisq {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ double2 cv(double2 v) { return v; }
__device__ __forceinline__ double2 cv_d(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ double2 cv_d(double2 v) { return v; }

template <class T> struct VecT;
template <> struct VecT<double2> { using real = double; };
template <> struct VecT<float2> { using real = float; };

// ------------------------------------------------------------------ finalisers
enum {
    FIN_BB = 0,           // bb = v ; stop2 = tol2 * bb
    FIN_PAP = 1,          // pAp = v ; alpha or breakdown
    FIN_UPD_PLAIN = 2,    // rr_new = v ; iter++ ; converged? ; beta ; rr
    FIN_UPD_MIXED = 3,    // as above, deciding reliable updates
    FIN_INIT_PLAIN = 4,   // rr = rr_true = v ; done = v <= stop2
    FIN_TRUE = 5,         // rr_true = v
    FIN_RELIABLE = 6,     // rr_true = v ; beta = v / rr ; rr = maxrr = v ; reliable = 0 ; done?
    FIN_INIT_MIXED = 7,   // rr = maxrr = rr_true = v ; done = v <= stop2
};

__device__ __forceinline__ void finalize(CGState *st, int mode, double v)
{
    switch (mode) {
    case FIN_BB:
        st->bb = v;
        st->stop2 = st->tol2 * v;
        break;
    case FIN_PAP:
        st->pAp = v;
        if (!(v > 0.0) || !isfinite(v)) {
            st->flags.done = CG_BREAKDOWN;
        } else {
            st->alpha = st->rr / v;
        }
        break;
    case FIN_UPD_PLAIN:
        st->rr_new = v;
        st->iter += 1;
        if (!isfinite(v)) {
            st->flags.done = CG_BREAKDOWN;
        } else if (v <= st->stop2) {
            st->flags.done = CG_CONVERGED;
            st->rr = v;
        } else {
            st->beta = v / st->rr;
            st->rr = v;
        }
        break;
    case FIN_UPD_MIXED:
        st->rr_new = v;
        st->iter += 1;
        if (!isfinite(v)) {
            st->flags.done = CG_BREAKDOWN;
        } else if (v <= st->stop2 || v < st->delta2 * st->maxrr) {
            st->flags.reliable = 1;
        } else {
            st->maxrr = fmax(st->maxrr, v);
            st->beta = v / st->rr;
            st->rr = v;
            // the inner solve has gone ten times as long as its first cycle without a reliable update
            if (st->first_gap > 0 && st->iter - st->last_upd > 10 * st->first_gap + 1000) st->flags.done = CG_STALLED;
        }
        break;
    case FIN_INIT_PLAIN:
        st->rr = v;
        st->rr_true = v;
        st->flags.done = (v <= st->stop2) ? CG_CONVERGED : 0;
        break;
    case FIN_TRUE:
        st->rr_true = v;
        break;
    case FIN_RELIABLE: {
        const int gap = st->iter - st->last_upd;
        if (st->first_gap == 0) st->first_gap = gap > 0 ? gap : 1;
        // poor: the true residual fell by less than sqrt(delta) since the last
        // update (an update fires after a fall by delta in the iterated residual),
        // or did not halve when delta is small
        st->poor = (v > fmax(0.25, sqrt(st->delta2)) * st->rr_upd) ? st->poor + 1 : 0;
        st->rr_upd = v;
        st->last_upd = st->iter;
        st->rr_true = v;
        st->nupdates += 1;
        st->beta = v / st->rr;
        st->rr = v;
        st->maxrr = v;
        st->flags.reliable = 0;
        if (!isfinite(v)) st->flags.done = CG_BREAKDOWN;
        else if (v <= st->stop2) st->flags.done = CG_CONVERGED;
        else if (st->poor >= 2) st->flags.done = CG_STALLED;  // the inner operator is too far from A
        break;
    }
    case FIN_INIT_MIXED:
        st->rr = v;
        st->maxrr = v;
        st->rr_true = v;
        st->rr_upd = v;
        st->last_upd = 0;
        st->first_gap = 0;
        st->poor = 0;
        st->flags.reliable = 0;
        st->flags.done = (v <= st->stop2) ? CG_CONVERGED : 0;
        break;
    }
}

// ------------------------------------------------------------------ BLAS kernels
// Streaming vector kernels: each thread owns BL_U entries spaced BL_NT apart
// (every load instruction of a wavefront is one contiguous span), issues all
// its loads before any arithmetic, and the grid covers the vector once.
// Every vector a solver kernel writes is stored nontemporally: a Dslash
// whose source was written through the caches runs measurably slower than
// one whose source was streamed out.
constexpr int BL_NT = 256;
constexpr int BL_U = 4;

int blas_blocks(long long n)
{
    long long nb = (n + (long long)BL_NT * BL_U - 1) / ((long long)BL_NT * BL_U);
    return (int)(nb > 0 ? nb : 1);
}

__device__ __forceinline__ long long bl_index(int j) { return ((long long)blockIdx.x * BL_U + j) * BL_NT + threadIdx.x; }

// Partials of Re<x, y> (or |x|^2) over n complex entries.
template <class T>
__global__ __launch_bounds__(BL_NT) void k_dot_state(const T *__restrict__ x, const T *__restrict__ y, long long n,
                                                     double *partials)
{
    T a[BL_U], b[BL_U];
#pragma unroll
    for (int j = 0; j < BL_U; ++j) {
        const long long i = bl_index(j);
        if (i < n) { a[j] = x[i]; b[j] = y[i]; }
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < BL_U; ++j) {
        if (bl_index(j) < n) {
            double2 u = cv_d(a[j]), v = cv_d(b[j]);
            s = fma(u.x, v.x, s);
            s = fma(u.y, v.y, s);
        }
    }
    block_partial<BL_NT>(s, partials, blockIdx.x);
}

// p = r + beta p ; partials of |p|^2 (the first half of the next <p, A p>)
template <class T>
__global__ __launch_bounds__(BL_NT) void k_cg_p_norm(T *__restrict__ p, const T *__restrict__ r, long long n,
                                                     double *partials, const CGState *st)
{
    if (paused(st->flags)) return;
    using R = typename VecT<T>::real;
    const R beta = (R)st->beta;
    T pv[BL_U], rv[BL_U];
#pragma unroll
    for (int j = 0; j < BL_U; ++j) {
        const long long i = bl_index(j);
        if (i < n) { pv[j] = p[i]; rv[j] = r[i]; }
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < BL_U; ++j) {
        const long long i = bl_index(j);
        if (i < n) {
            pv[j].x = fma(beta, pv[j].x, rv[j].x);
            pv[j].y = fma(beta, pv[j].y, rv[j].y);
            ntstore(pv[j], p + i);
            s = fma((double)pv[j].x, (double)pv[j].x, s);
            s = fma((double)pv[j].y, (double)pv[j].y, s);
        }
    }
    block_partial<BL_NT>(s, partials, blockIdx.x);
}

// x64 += xs ; xs = 0   (reliable update)
__global__ __launch_bounds__(BL_NT) void k_accum(double2 *__restrict__ x, float2 *__restrict__ xs, long long n,
                                                 const CGState *st)
{
    if (st->flags.done || !st->flags.reliable) return;
    float2 v[BL_U];
    double2 a[BL_U];
#pragma unroll
    for (int j = 0; j < BL_U; ++j) {
        const long long i = bl_index(j);
        if (i < n) { v[j] = xs[i]; a[j] = x[i]; }
    }
#pragma unroll
    for (int j = 0; j < BL_U; ++j) {
        const long long i = bl_index(j);
        if (i < n) {
            a[j].x += (double)v[j].x;
            a[j].y += (double)v[j].y;
            ntstore(a[j], x + i);
            ntstore(make_float2(0.f, 0.f), xs + i);
        }
    }
}

// Second stage of every reduction: one block sums the partials in a fixed
// order and applies finaliser `mode` to the state.  It is gated like the
// kernel that produced the partials, so a skipped producer is a no-op here.
constexpr int FIN_NT = 256;
__global__ __launch_bounds__(FIN_NT) void k_finalize(const double *__restrict__ partials, int n, CGState *st, int mode,
                                                     int gate)
{
    if (solver_gate_closed(&st->flags, gate)) return;  // first: queued past a pause, the kernel costs ~1 us
    double acc[1] = { 0.0 };
    strided_sums<FIN_NT, 1, 8>(partials, n, acc);
    __shared__ double lds[FIN_NT / 64];
    const double v = block_sum<FIN_NT>(acc[0], lds);
    if (threadIdx.x == 0) finalize(st, mode, v);
}

// pAp = m4 |p|^2 + |D_oe p|^2 from the partials of k_cg_p_norm (or k_dot_state)
// and of k_cg_Dp, then alpha (FIN_PAP).
__global__ __launch_bounds__(FIN_NT) void k_finalize_pap(const double *__restrict__ part_p, int np,
                                                         const double *__restrict__ part_t, int nt, CGState *st)
{
    if (paused(st->flags)) return;
    double ap[1] = { 0.0 }, at[1] = { 0.0 };
    strided_sums<FIN_NT, 1, 8>(part_p, np, ap);
    strided_sums<FIN_NT, 1, 8>(part_t, nt, at);
    __shared__ double lds[FIN_NT / 64];
    const double pp = block_sum<FIN_NT>(ap[0], lds);
    const double tt = block_sum<FIN_NT>(at[0], lds);
    if (threadIdx.x == 0) finalize(st, FIN_PAP, fma(st->m4, pp, tt));
}

__global__ void k_state_init(CGState *st, double tol2, double delta2, double m4)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->flags.done = 0;
        st->flags.reliable = 0;
        st->iter = 0;
        st->nupdates = 0;
        st->tol2 = tol2;
        st->delta2 = delta2;
        st->m4 = m4;
        st->rr = st->rr_new = st->rr_true = st->maxrr = 0.0;
        st->alpha = st->beta = st->pAp = 0.0;
    }
}

__global__ void k_force_reliable(CGState *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0 && !st->flags.done) st->flags.reliable = 1;
}

__global__ void k_clear_done(CGState *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) st->flags.done = 0;
}

// ------------------------------------------------------------------ Dslash-fused kernels
// Waves per SIMD the fused kernels ask for and terms of the 16 unrolled
// together, per link storage (measured with the mixed solves at 32^4):
//   FP64 forms        5 waves, 2 terms: a wave has two directions' link loads
//                     in flight (their best Dslash launch shape)
//   I16S, FP32 two-row 4 waves, 4 terms (2-3 % faster solves than 8 / 1)
//   FP32, FP16S       8 waves, 1 term
template <class P> constexpr bool cg_wide()
{
    return P::prec == HISQ_I16S || P::prec == HISQ_F32C || P::prec == HISQ_I16SC;
}
template <class P> constexpr int cg_waves()
{
    return (P::prec == HISQ_F64 || P::prec == HISQ_F64C) ? 5 : (cg_wide<P>() ? 4 : 8);
}
template <class P> constexpr int cg_unroll()
{
    return (P::prec == HISQ_F64 || P::prec == HISQ_F64C) ? 2 : (cg_wide<P>() ? 4 : 1);
}

// t = D_oe p on the odd sites ; partials of |t|^2
template <class P, int NT, int W>
__global__ __launch_bounds__(NT) HISQ_WAVES(W) void k_cg_Dp(Geom g, const char *__restrict__ fat,
                                                            const char *__restrict__ lng,
                                                            const typename P::cvec *__restrict__ p,
                                                            typename P::cvec *__restrict__ t, int nblocks,
                                                            double *partials, const CGState *st)
{
    if (paused(st->flags)) return;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    if (blk >= nblocks) return;
    const int k = blk * (NT / TILE) + (threadIdx.x >> 6);
    const int tile = k < g.ntiles ? tile_of(g, k) : 0;
    const int lane = threadIdx.x & 63;
    const int h = tile * TILE + lane;
    double s = 0.0;
    if (k < g.ntiles) {
        const int hc = h < g.Vh ? h : g.Vh - 1;
        typename P::real acc[6];
        dslash_site<P, cg_unroll<P>()>(g, fat, lng, p, 1, tile, lane, hc, acc);
        if (h < g.Vh) {
            typename P::cvec *o = t + (size_t)h * 3;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                typename P::cvec v;
                v.x = acc[2 * c];
                v.y = acc[2 * c + 1];
                ntstore(v, o + c);
                s = fma((double)v.x, (double)v.x, s);
                s = fma((double)v.y, (double)v.y, s);
            }
        }
    }
    block_partial<NT>(s, partials, blk);
}

// A p = m4 p - D_eo t in registers ; x += alpha p ; r -= alpha A p ; partials of |r|^2
template <class P, int NT, int W>
__global__ __launch_bounds__(NT) HISQ_WAVES(W) void k_cg_Ap_upd(Geom g, const char *__restrict__ fat,
                                                                const char *__restrict__ lng,
                                                                const typename P::cvec *__restrict__ t,
                                                                const typename P::cvec *__restrict__ p,
                                                                typename P::cvec *__restrict__ x,
                                                                typename P::cvec *__restrict__ r, int nblocks,
                                                                double *partials, const CGState *st)
{
    if (paused(st->flags)) return;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    if (blk >= nblocks) return;
    const int k = blk * (NT / TILE) + (threadIdx.x >> 6);
    const int tile = k < g.ntiles ? tile_of(g, k) : 0;
    const int lane = threadIdx.x & 63;
    const int h = tile * TILE + lane;
    double s = 0.0;
    if (k < g.ntiles) {
        const int hc = h < g.Vh ? h : g.Vh - 1;
        typename P::real acc[6];
        dslash_site<P, cg_unroll<P>()>(g, fat, lng, t, 0, tile, lane, hc, acc);
        if (h < g.Vh) {
            using R = typename P::real;
            const R m = (R)st->m4, a = (R)st->alpha;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const size_t i = (size_t)h * 3 + c;
                const typename P::cvec pv = p[i];
                // x and r are streamed (read once, written once per iteration): in FP64 streaming loads keep
                // them from evicting the gathered t and the p that the next Dslash gathers (48^3x96: 2663 ->
                // 2615 us per launch)
                typename P::cvec xv, rv;
                if constexpr (sizeof(typename P::real) == 8) {
                    xv = ntload(x + i);
                    rv = ntload(r + i);
                } else {
                    xv = x[i];
                    rv = r[i];
                }
                const R apx = fma(m, pv.x, -acc[2 * c]), apy = fma(m, pv.y, -acc[2 * c + 1]);
                xv.x = fma(a, pv.x, xv.x);
                xv.y = fma(a, pv.y, xv.y);
                rv.x = fma(-a, apx, rv.x);
                rv.y = fma(-a, apy, rv.y);
                ntstore(xv, x + i);
                ntstore(rv, r + i);
                s = fma((double)rv.x, (double)rv.x, s);
                s = fma((double)rv.y, (double)rv.y, s);
            }
        }
    }
    block_partial<NT>(s, partials, blk);
}

// r = b - (m4 x - D_eo t) in FP64 ; optional copies ; partials of |r|^2
template <class PH, int NT>
__global__ __launch_bounds__(NT) HISQ_WAVES(cg_waves<PH>()) void k_resid(Geom g, const char *__restrict__ fat, const char *__restrict__ lng,
                                              const double2 *__restrict__ t, const double2 *__restrict__ x,
                                              const double2 *__restrict__ b, double2 *__restrict__ r,
                                              double2 *__restrict__ p, float2 *__restrict__ rs,
                                              float2 *__restrict__ ps, int nblocks, double *partials,
                                              const CGState *st, int gate)
{
    if (gate_closed(&st->flags, gate)) return;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    if (blk >= nblocks) return;
    const int k = blk * (NT / TILE) + (threadIdx.x >> 6);
    const int tile = k < g.ntiles ? tile_of(g, k) : 0;
    const int lane = threadIdx.x & 63;
    const int h = tile * TILE + lane;
    double s = 0.0;
    if (k < g.ntiles) {
        const int hc = h < g.Vh ? h : g.Vh - 1;
        double acc[6];
        dslash_site<PH>(g, fat, lng, t, 0, tile, lane, hc, acc);
        if (h < g.Vh) {
            const double m = st->m4;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const size_t i = (size_t)h * 3 + c;
                double2 xv = x[i], bv = b[i], v;
                v.x = bv.x - fma(m, xv.x, -acc[2 * c]);
                v.y = bv.y - fma(m, xv.y, -acc[2 * c + 1]);
                if (r) ntstore(v, r + i);
                if (p) ntstore(v, p + i);
                if (rs) ntstore(make_float2((float)v.x, (float)v.y), rs + i);
                if (ps) ntstore(make_float2((float)v.x, (float)v.y), ps + i);
                s = fma(v.x, v.x, s);
                s = fma(v.y, v.y, s);
            }
        }
    }
    block_partial<NT>(s, partials, blk);
}

constexpr int CG_NT = 256;
static inline int dslash_nb(const Geom &g) { return (g.ntiles + CG_NT / TILE - 1) / (CG_NT / TILE); }

// ------------------------------------------------------------------ host side
size_t cg_partials_count(const Geom &g)
{
    size_t a = (size_t)dslash_nb(g), b = (size_t)blas_blocks((long long)g.Vh * 3);
    return a > b ? a : b;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Gap between carved workspace buffers: consecutive vectors start at
// different offsets modulo the HBM channel interleave.
constexpr size_t SKEW = 4352;

size_t cg_workspace_bytes(const Geom &g, int mode)
{
    const size_t v64 = align256((size_t)g.Vh * 3 * 16), v32 = align256((size_t)g.Vh * 3 * 8);
    size_t bytes = align256(sizeof(CGState)) + 2 * align256(cg_partials_count(g) * sizeof(double)) + 3 * SKEW;
    if (mode == HISQ_CG_PLAIN_F64 || mode == HISQ_CG_PLAIN_F64C) bytes += 3 * (v64 + SKEW);  // r p t
    else bytes += 2 * (v64 + SKEW) + 4 * (v32 + SKEW);                      // r64 t64 | xs rs ps ts
    return bytes;
}

void *pinned_slot(int slot)
{
    static thread_local char *h = nullptr;
    if (slot < 0 || slot >= PIN_SLOTS) return nullptr;
    if (!h) {
        if (hipHostMalloc((void **)&h, PIN_SLOT_BYTES * PIN_SLOTS, hipHostMallocDefault) != hipSuccess) h = nullptr;
    }
    return h ? h + (size_t)slot * PIN_SLOT_BYTES : nullptr;
}
static_assert(sizeof(CGState) <= PIN_SLOT_BYTES, "CGState does not fit its pinned slot");

hipStream_t capture_stream()
{
    static thread_local hipStream_t s = nullptr;
    if (!s) {
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    }
    return s;
}

// Run `iter_fn` (which enqueues one iteration on a stream) until the state
// reports done or `max_iter` iterations were queued.  Every `K` iterations
// the state is copied to pinned memory and inspected; with use_graph the K
// iterations are captured once and replayed.
struct NoPause {
    hipError_t operator()(hipStream_t) const { return hipSuccess; }
};

// pause_fn (mixed solvers): enqueues the reliable update when a state check
// finds one pending; the iterations then resume.
struct NoCheck {
    void operator()(int) const {}
};

// on_check(n): called after every state read-back with the number of
// iterations that ran (were not gated off) since the previous one.
template <class IterFn, class PauseFn = NoPause, class CheckFn = NoCheck>
static int run_iterations(IterFn iter_fn, hipStream_t s, CGState *dstate, CGState *hstate, int K, int max_iter,
                          bool use_graph, int already, PauseFn pause_fn = PauseFn(), CheckFn on_check = CheckFn())
{
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    if (use_graph) {
        hipStream_t cs = capture_stream();
        if (!cs) return fail(HISQ_EHIP, "cannot create capture stream");
        HISQ_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < K; ++k) {
            hipError_t e = iter_fn(cs);
            if (e != hipSuccess) {
                hipGraph_t junk;
                hipStreamEndCapture(cs, &junk);
                if (junk) hipGraphDestroy(junk);
                return hip_fail(e, "CG iteration launch (capture)");
            }
        }
        HISQ_HIP(hipStreamEndCapture(cs, &graph));
        HISQ_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    }
    int queued = already;
    int rc = HISQ_OK;
    while (queued < max_iter) {
        const int k = (max_iter - queued) < K ? (max_iter - queued) : K;
        if (use_graph && k == K) {
            hipError_t e = hipGraphLaunch(exec, s);
            if (e != hipSuccess) { rc = hip_fail(e, "hipGraphLaunch"); break; }
        } else {
            for (int i = 0; i < k; ++i) {
                hipError_t e = iter_fn(s);
                if (e != hipSuccess) { rc = hip_fail(e, "CG iteration launch"); break; }
            }
            if (rc) break;
        }
        queued += k;
        const int before = hstate->iter;
        hipError_t e = hipMemcpyAsync(hstate, dstate, sizeof(CGState), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { rc = hip_fail(e, "CG state read-back"); break; }
        on_check(hstate->iter - before);
        if (hstate->flags.done) break;
        if (hstate->flags.reliable) {
            e = pause_fn(s);
            if (e != hipSuccess) { rc = hip_fail(e, "reliable update launch"); break; }
        }
    }
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    return rc;
}

static int read_state(CGState *h, const CGState *d, hipStream_t s)
{
    HISQ_HIP(hipMemcpyAsync(h, d, sizeof(CGState), hipMemcpyDeviceToHost, s));
    HISQ_HIP(hipStreamSynchronize(s));
    return HISQ_OK;
}

struct Carver {
    char *p;
    size_t left;
    void *take(size_t n)
    {
        n = align256(n) + SKEW;
        if (n > left) return nullptr;
        void *r = p;
        p += n;
        left -= n;
        return r;
    }
};

// Launch helpers shared by the solvers: every reduction is a producer
// kernel writing per-block partials followed by k_finalize.
struct Launch {
    const Geom &g;
    CGState *st;
    double *part;    // partials of the reduction in flight
    double *part_p;  // partials of |p|^2, kept from one iteration to the next
    long long n;     // complex entries per vector
    int nbl, nbd;
    dim3 gb, gd;
    Launch(const Geom &g_, CGState *st_, double *part_, double *part_p_)
        : g(g_), st(st_), part(part_), part_p(part_p_), n((long long)g_.Vh * 3), nbl(blas_blocks((long long)g_.Vh * 3)),
          nbd(dslash_nb(g_)), gb(nbl), gd(xcd_grid(dslash_nb(g_)))
    {
    }
    void fin(hipStream_t q, int nparts, int mode, int gate) const
    {
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_NT), 0, q, (const double *)part, nparts, st, mode, gate);
    }
    template <class T> void norm2(hipStream_t q, const T *x, int mode) const
    {
        hipLaunchKernelGGL((k_dot_state<T>), gb, dim3(BL_NT), 0, q, x, x, n, part);
        fin(q, nbl, mode, GATE_ALWAYS);
    }
    // r = b - (m4 x - D_eo t) [+ copies], |r|^2 -> mode; t must hold D_oe x
    template <class PH>
    void resid(hipStream_t q, const void *fat, const void *lng, const double2 *t, const void *x, const void *b,
               double2 *r, double2 *p, float2 *rs, float2 *ps, int mode, int gate) const
    {
        hipLaunchKernelGGL((k_resid<PH, CG_NT>), gd, dim3(CG_NT), 0, q, g, (const char *)fat, (const char *)lng, t,
                           (const double2 *)x, (const double2 *)b, r, p, rs, ps, nbd, part, (const CGState *)st, gate);
        fin(q, nbd, mode, gate);
    }
    // |p|^2 partials into part_p (before the first iteration and after restarts)
    template <class T> void pnorm(hipStream_t q, const T *p) const
    {
        hipLaunchKernelGGL((k_dot_state<T>), gb, dim3(BL_NT), 0, q, p, p, n, part_p);
    }
    // t = D_oe p ; alpha = rr / (m4 |p|^2 + |t|^2)
    // e0 / e1 (may be NULL): events recorded right before and after the main kernel
    template <class P>
    void dp(hipStream_t q, const void *fat, const void *lng, const void *p, void *t, hipEvent_t e0 = nullptr,
            hipEvent_t e1 = nullptr) const
    {
        using V = typename P::cvec;
        if (e0) hipEventRecord(e0, q);
        hipLaunchKernelGGL((k_cg_Dp<P, CG_NT, cg_waves<P>()>), gd, dim3(CG_NT), 0, q, g, (const char *)fat,
                           (const char *)lng, (const V *)p, (V *)t, nbd, part, (const CGState *)st);
        if (e1) hipEventRecord(e1, q);
        hipLaunchKernelGGL(k_finalize_pap, dim3(1), dim3(FIN_NT), 0, q, (const double *)part_p, nbl,
                           (const double *)part, nbd, st);
    }
    // x += alpha p ; r -= alpha (m4 p - D_eo t) ; |r|^2 -> mode
    template <class P>
    void ap_update(hipStream_t q, const void *fat, const void *lng, const void *t, const void *p, void *x, void *r,
                   int mode, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) const
    {
        using V = typename P::cvec;
        if (e0) hipEventRecord(e0, q);
        hipLaunchKernelGGL((k_cg_Ap_upd<P, CG_NT, cg_waves<P>()>), gd, dim3(CG_NT), 0, q, g, (const char *)fat,
                           (const char *)lng, (const V *)t, (const V *)p, (V *)x, (V *)r, nbd, part,
                           (const CGState *)st);
        if (e1) hipEventRecord(e1, q);
        fin(q, nbd, mode, GATE_PAUSE);
    }
    // p = r + beta p ; |p|^2 partials into part_p
    template <class T> void pupd(hipStream_t q, T *p, const T *r, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) const
    {
        if (e0) hipEventRecord(e0, q);
        hipLaunchKernelGGL((k_cg_p_norm<T>), gb, dim3(BL_NT), 0, q, p, r, n, part_p, (const CGState *)st);
        if (e1) hipEventRecord(e1, q);
    }
};

// The fused CG kernels follow the tile order of the Dslash shape tuned for
// (lattice, precision of their links).
static Geom cg_geom(const Geom &g, int prec)
{
    Geom c = g;
    apply_order(c, DSLASH_SHAPES[tuned_dslash_shape(g, prec)].order);
    return c;
}

static void finish_stats(hisq_cg_stats &stats, const CGState *hs, int status, int restarts, double bytes,
                         std::chrono::steady_clock::time_point t0)
{
    stats.iters = hs->iter;
    stats.restarts = restarts;
    stats.reliable_updates = hs->nupdates;
    stats.true_resid = hs->bb > 0 ? std::sqrt(hs->rr_true / hs->bb) : 0.0;
    stats.iter_resid = hs->bb > 0 ? std::sqrt(hs->rr / hs->bb) : 0.0;
    stats.bytes_moved = bytes;
    stats.status = status;
    stats.time_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Byte model of a CG iteration per even site: the two Dslash link streams and
// seven vector streams (p read and t written by the first Dslash; t, p read,
// x and r read and written by the update epilogue, where A p stays in
// registers; r, p read and p written by the direction update).  A true
// residual (x read, t written; t, x, b read, r written) moves the links
// twice and six vectors.
static double cg_iter_bytes(int prec) { return 2 * link_bytes_site(prec) + 7 * vec_bytes(prec); }
static double cg_resid_bytes(int prec) { return 2 * link_bytes_site(prec) + 6 * vec_bytes(prec); }

static int zero_source_exit(void *x, size_t v64, hipStream_t s, hisq_cg_stats &stats,
                            std::chrono::steady_clock::time_point t0)
{
    HISQ_HIP(hipMemsetAsync(x, 0, v64, s));
    HISQ_HIP(hipStreamSynchronize(s));
    stats.iters = 0;
    stats.true_resid = 0.0;
    stats.status = HISQ_OK;
    stats.time_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return HISQ_OK;
}

// Kernel timing of the plain solver (opts->use_graph == 2): the iterations
// launch directly, with HIP events right before and after each of the three
// main kernels, slot i % K of K slots per state check; after each check the
// slots of the iterations that ran are read and summed.
struct IterTimer {
    int K = 0;
    std::vector<hipEvent_t> ev;
    double sum[3] = { 0.0, 0.0, 0.0 };
    long long n = 0;
    int slot = 0;
    bool start(int k)
    {
        ev.assign(6 * (size_t)k, nullptr);
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) return false;
        K = k;
        return true;
    }
    hipEvent_t at(int i) const { return K ? ev[6 * (size_t)(slot % K) + i] : nullptr; }
    void next() { if (K) ++slot; }
    void collect(int ran)
    {
        for (int j = 0; j < std::min(ran, K); ++j)
            for (int c = 0; c < 3; ++c) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, ev[6 * (size_t)j + 2 * c], ev[6 * (size_t)j + 2 * c + 1]) == hipSuccess)
                    sum[c] += 1e3 * ms;
            }
        n += std::min(ran, K);
        slot = 0;
    }
    ~IterTimer()
    {
        for (auto &e : ev)
            if (e) hipEventDestroy(e);
    }
};

template <class PH>
int cg_plain(double mass, double tol, const void *fat, const void *lng, const void *b, void *x, const Geom &g,
             const hisq_cg_opts &o, void *ws, size_t ws_bytes, hisq_cg_stats &stats, hipStream_t s)
{
    Carver c{ (char *)ws, ws_bytes };
    const size_t v64 = (size_t)g.Vh * 3 * 16;
    CGState *st = (CGState *)c.take(sizeof(CGState));
    double *part = (double *)c.take(cg_partials_count(g) * sizeof(double));
    double *part_p = (double *)c.take(cg_partials_count(g) * sizeof(double));
    double2 *r = (double2 *)c.take(v64), *p = (double2 *)c.take(v64), *t = (double2 *)c.take(v64);
    if (!t) return fail(HISQ_EWORKSPACE, "cg_solve: workspace too small");
    CGState *hs = pinned_state();
    if (!hs) return fail(HISQ_EHIP, "cg_solve: pinned state allocation failed");
    const Geom gc = cg_geom(g, PH::prec);
    const Launch L(gc, st, part, part_p);

    auto t0 = std::chrono::steady_clock::now();
    HISQ_HIP(hipMemsetAsync(st, 0, sizeof(CGState), s));
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, st, tol * tol, 0.0, 4.0 * mass * mass);
    L.norm2(s, (const double2 *)b, FIN_BB);
    HISQ_HIP(launch_dslash<PH>(g, fat, lng, x, t, 1, s));  // r = p = b - A x0
    L.template resid<PH>(s, fat, lng, t, x, b, r, p, nullptr, nullptr, FIN_INIT_PLAIN, GATE_ALWAYS);
    L.pnorm<double2>(s, p);
    HISQ_HIP(hipGetLastError());
    int rc = read_state(hs, st, s);
    if (rc) return rc;
    if (hs->bb == 0.0) return zero_source_exit(x, v64, s, stats, t0);

    IterTimer tm;
    if (o.use_graph == 2 && !tm.start(o.check_every)) return fail(HISQ_EHIP, "cg_solve: event creation failed");
    auto iter = [&](hipStream_t q) -> hipError_t {
        L.dp<PH>(q, fat, lng, p, t, tm.at(0), tm.at(1));
        L.ap_update<PH>(q, fat, lng, t, p, x, r, FIN_UPD_PLAIN, tm.at(2), tm.at(3));
        L.pupd<double2>(q, p, r, tm.at(4), tm.at(5));
        tm.next();
        return hipGetLastError();
    };
    auto on_check = [&](int ran) { if (tm.K) tm.collect(ran); };

    int restarts = 0;
    int status = HISQ_OK;
    while (true) {
        if (!hs->flags.done) {
            rc = run_iterations(iter, s, st, hs, o.check_every, o.max_iter, o.use_graph != 0 && o.use_graph != 2, hs->iter, NoPause(),
                                on_check);
            if (rc) return rc;
        }
        if (hs->flags.done == CG_BREAKDOWN) { status = HISQ_EBREAKDOWN; break; }
        // true residual r = b - A x in FP64
        HISQ_HIP(launch_dslash<PH>(g, fat, lng, x, t, 1, s));
        L.template resid<PH>(s, fat, lng, t, x, b, r, nullptr, nullptr, nullptr, FIN_TRUE, GATE_ALWAYS);
        HISQ_HIP(hipGetLastError());
        rc = read_state(hs, st, s);
        if (rc) return rc;
        if (hs->rr_true <= hs->stop2) { status = HISQ_OK; break; }
        if (hs->iter >= o.max_iter || restarts >= 3) { status = HISQ_ENOCONV; break; }
        ++restarts;  // restart from x: r = p = b - A x (t still holds D_oe x)
        L.template resid<PH>(s, fat, lng, t, x, b, r, p, nullptr, nullptr, FIN_INIT_PLAIN, GATE_ALWAYS);
        L.pnorm<double2>(s, p);
        HISQ_HIP(hipGetLastError());
        rc = read_state(hs, st, s);
        if (rc) return rc;
    }
    const double bytes = ((double)hs->iter * cg_iter_bytes(PH::prec) + (2 + 2 * restarts) * cg_resid_bytes(PH::prec)) * g.Vh;
    finish_stats(stats, hs, status, restarts, bytes, t0);
    for (int c = 0; c < 3; ++c) stats.kernel_us[c] = tm.n ? tm.sum[c] / tm.n : 0.0;
    if (status == HISQ_EBREAKDOWN) return fail(status, "cg_solve: breakdown (<p,Ap> <= 0 or not finite)");
    if (status == HISQ_ENOCONV) return fail(status, "cg_solve: not converged within max_iter");
    return HISQ_OK;
}

int cg_plain_f64(double mass, double tol, const void *fat, const void *lng, const void *b, void *x, const Geom &g,
                 const hisq_cg_opts &o, void *ws, size_t ws_bytes, hisq_cg_stats &stats, hipStream_t s)
{
    return cg_plain<PF64>(mass, tol, fat, lng, b, x, g, o, ws, ws_bytes, stats, s);
}

// Default reliable-update trigger for inner links PS.  With 16-bit links the
// inner operator is ~1e-5 away from A and the iterated residual drifts from
// the true one within a cycle: frequent updates (every fall by 0.7) keep the
// iteration count at the FP32 level (at 32^4, m = 0.005: 7647 iterations
// against 12 230 at 0.1; at m = 0.002 the solve converges at all).  FP32 inner
// links are insensitive to it and keep the customary 0.1.
template <class PS> constexpr double default_delta()
{
    return (PS::prec == HISQ_F16S || PS::prec == HISQ_I16S || PS::prec == HISQ_I16SC) ? 0.7 : 0.1;
}

template <class PH, class PS>
int cg_mixed(double mass, double tol, const void *fat, const void *lng, const void *fat_lo, const void *lng_lo,
             const void *b, void *x, const Geom &g, const hisq_cg_opts &o, void *ws, size_t ws_bytes,
             hisq_cg_stats &stats, hipStream_t s)
{
    Carver c{ (char *)ws, ws_bytes };
    const size_t v64 = (size_t)g.Vh * 3 * 16, v32 = (size_t)g.Vh * 3 * 8;
    CGState *st = (CGState *)c.take(sizeof(CGState));
    double *part = (double *)c.take(cg_partials_count(g) * sizeof(double));
    double *part_p = (double *)c.take(cg_partials_count(g) * sizeof(double));
    double2 *r64 = (double2 *)c.take(v64), *t64 = (double2 *)c.take(v64);
    float2 *xs = (float2 *)c.take(v32), *rs = (float2 *)c.take(v32), *ps = (float2 *)c.take(v32),
           *ts = (float2 *)c.take(v32);
    if (!ts) return fail(HISQ_EWORKSPACE, "cg_solve: workspace too small");
    CGState *hs = pinned_state();
    if (!hs) return fail(HISQ_EHIP, "cg_solve: pinned state allocation failed");
    const Geom gc = cg_geom(g, PS::prec);
    const Launch L(gc, st, part, part_p);
    const double delta = o.delta > 0 ? o.delta : default_delta<PS>();

    auto t0 = std::chrono::steady_clock::now();
    HISQ_HIP(hipMemsetAsync(st, 0, sizeof(CGState), s));
    HISQ_HIP(hipMemsetAsync(xs, 0, v32, s));
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, st, tol * tol, delta * delta, 4.0 * mass * mass);
    L.norm2(s, (const double2 *)b, FIN_BB);
    HISQ_HIP(launch_dslash<PH>(g, fat, lng, x, t64, 1, s));
    L.template resid<PH>(s, fat, lng, t64, x, b, r64, nullptr, rs, ps, FIN_INIT_MIXED, GATE_ALWAYS);
    L.pnorm<float2>(s, ps);
    HISQ_HIP(hipGetLastError());
    int rc = read_state(hs, st, s);
    if (rc) return rc;
    if (hs->bb == 0.0) return zero_source_exit(x, v64, s, stats, t0);

    const dim3 gb(L.nbl), bb(BL_NT);
    // one inner iteration; a reliable update request pauses the rest of the graph
    auto iter = [&](hipStream_t q) -> hipError_t {
        L.dp<PS>(q, fat_lo, lng_lo, ps, ts);
        L.ap_update<PS>(q, fat_lo, lng_lo, ts, ps, xs, rs, FIN_UPD_MIXED);
        L.pupd<float2>(q, ps, rs);
        return hipGetLastError();
    };
    // the reliable update: x += xs, r = b - A x in FP64, rs = float(r), then the direction update
    auto reliable = [&](hipStream_t q) -> hipError_t {
        hipLaunchKernelGGL(k_accum, gb, bb, 0, q, (double2 *)x, xs, L.n, (const CGState *)st);
        hipError_t e = launch_dslash<PH>(g, fat, lng, x, t64, 1, q, &st->flags, GATE_RELIABLE);
        if (e != hipSuccess) return e;
        L.template resid<PH>(q, fat, lng, t64, x, b, r64, nullptr, rs, nullptr, FIN_RELIABLE, GATE_RELIABLE);
        L.pupd<float2>(q, ps, rs);
        return hipGetLastError();
    };

    rc = run_iterations(iter, s, st, hs, o.check_every, o.max_iter, o.use_graph != 0, 0, reliable);
    if (rc) return rc;
    if (hs->flags.done == CG_STALLED) {
        // The low-precision operator cannot drive the true residual down: fold
        // the inner solution into x and finish with plain CG on the outer links.
        hipLaunchKernelGGL(k_clear_done, dim3(1), dim3(1), 0, s, st);
        hipLaunchKernelGGL(k_force_reliable, dim3(1), dim3(1), 0, s, st);
        hipLaunchKernelGGL(k_accum, gb, bb, 0, s, (double2 *)x, xs, L.n, (const CGState *)st);
        HISQ_HIP(hipGetLastError());
        const int used = hs->iter, nupd = hs->nupdates;
        hisq_cg_opts o2 = o;
        o2.max_iter = o.max_iter - used;
        if (o2.max_iter <= 0) o2.max_iter = 1;
        hisq_cg_stats s2;
        std::memset(&s2, 0, sizeof(s2));
        rc = cg_plain<PH>(mass, tol, fat, lng, b, x, g, o2, ws, ws_bytes, s2, s);
        stats = s2;
        stats.iters = used + s2.iters;
        stats.reliable_updates = nupd;
        stats.fallback_used = 1;
        stats.fallback_iters = s2.iters;
        stats.bytes_moved += ((double)used * cg_iter_bytes(PS::prec) + (nupd + 1) * cg_resid_bytes(PH::prec)) * g.Vh;
        stats.time_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return rc;
    }
    int status = HISQ_OK;
    if (hs->flags.done == CG_BREAKDOWN) {
        status = HISQ_EBREAKDOWN;
    } else if (hs->flags.done != CG_CONVERGED) {
        // out of iterations: fold the inner solution in and measure the true residual
        hipLaunchKernelGGL(k_force_reliable, dim3(1), dim3(1), 0, s, st);
        hipLaunchKernelGGL(k_accum, gb, bb, 0, s, (double2 *)x, xs, L.n, (const CGState *)st);
        HISQ_HIP(launch_dslash<PH>(g, fat, lng, x, t64, 1, s));
        L.template resid<PH>(s, fat, lng, t64, x, b, r64, nullptr, rs, nullptr, FIN_RELIABLE, GATE_ALWAYS);
        HISQ_HIP(hipGetLastError());
        rc = read_state(hs, st, s);
        if (rc) return rc;
        status = hs->rr_true <= hs->stop2 ? HISQ_OK : HISQ_ENOCONV;
    }
    // inner iterations on PS, every reliable update (and the start) one FP64 true residual
    const double bytes =
        ((double)hs->iter * cg_iter_bytes(PS::prec) + (hs->nupdates + 1) * cg_resid_bytes(PH::prec)) * g.Vh;
    finish_stats(stats, hs, status, 0, bytes, t0);
    if (status == HISQ_EBREAKDOWN) return fail(status, "cg_solve: breakdown (<p,Ap> <= 0 or not finite)");
    if (status == HISQ_ENOCONV) return fail(status, "cg_solve: not converged within max_iter");
    return HISQ_OK;
}

int default_check_every(const Geom &g) { return g.Vh <= 65536 ? 50 : (g.Vh <= 1048576 ? 25 : 10); }

hisq_cg_opts resolve_opts(const hisq_cg_opts *opts, const Geom &g)
{
    hisq_cg_opts o;
    if (opts) o = *opts;
    else {
        o.mode = HISQ_CG_PLAIN_F64;
        o.max_iter = 0;
        o.check_every = 0;
        o.use_graph = 1;
        o.delta = 0.0;
        o.shift_tol = 0.0;
        o.shift_only = 0;
    }
    if (o.max_iter <= 0) o.max_iter = 100000;
    if (o.check_every <= 0) o.check_every = default_check_every(g);
    if (!(o.delta > 0)) o.delta = 0.0;  // each solver applies the default of its inner links
    if (!(o.shift_tol > 0)) o.shift_tol = 0.0;
    return o;
}

// ------------------------------------------------------------------ standalone dot
template <class T>
__global__ __launch_bounds__(BL_NT) void k_dot2(const T *__restrict__ x, const T *__restrict__ y, long long n,
                                                double *partials)
{
    double sr = 0.0, si = 0.0;
    for (long long i = (long long)blockIdx.x * BL_NT + threadIdx.x; i < n; i += (long long)gridDim.x * BL_NT) {
        double2 a = cv_d(x[i]), b = cv_d(y[i]);
        sr = fma(a.x, b.x, sr);
        sr = fma(a.y, b.y, sr);
        si = fma(a.x, b.y, si);
        si = fma(-a.y, b.x, si);
    }
    __shared__ double lds[2 * (BL_NT / 64)];
    block_sum2<BL_NT>(sr, si, lds);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = sr;
        partials[2 * blockIdx.x + 1] = si;
    }
}

__global__ __launch_bounds__(FIN_NT) void k_dot2_fin(const double *__restrict__ partials, int nb, double *out)
{
    __shared__ double lds[2 * (FIN_NT / 64)];
    double acc[2] = { 0.0, 0.0 };
    strided_sums<FIN_NT, 2, 4>(partials, nb, acc);
    double ar = acc[0], ai = acc[1];
    block_sum2<FIN_NT>(ar, ai, lds);
    if (threadIdx.x == 0) {
        out[0] = ar;
        out[1] = ai;
    }
}

}  // namespace hisq

using namespace hisq;


extern "C" size_t hisq_workspace_bytes(const char *solver, const int dims[4], int nrhs, int mode, int channels)
{
    Geom g;
    if (!solver || make_geom(dims, g)) return 0;
    if (!std::strcmp(solver, "cg")) {
        if (mode < HISQ_CG_PLAIN_F64 || mode > HISQ_CG_MIXED_I16SC) return 0;
        return cg_workspace_bytes(g, mode);
    }
    if (!std::strcmp(solver, "cg_multi")) return cg_multi_workspace_bytes(g, nrhs, mode);
    if (!std::strcmp(solver, "fat_paths")) return fat_paths_ws_bytes(dims);
    if (!std::strcmp(solver, "dot")) return DOT_WS_BYTES;
    if (!std::strcmp(solver, "fcg")) {
        if (channels != 4 && channels != 8 && channels != 16) return 0;
        return fcg_ws_bytes(g, channels);
    }
    return 0;
}

extern "C" int cg_solve(double mass, double tol, const void *fat, const void *lng, const void *fat_lo,
                        const void *lng_lo, const void *b, void *x, const int dims[4], const hisq_cg_opts *opts,
                        void *workspace, size_t ws_bytes, hisq_cg_stats *stats, void *stream)
{
    hisq_cg_stats local;
    std::memset(&local, 0, sizeof(local));
    hisq_cg_stats &st = stats ? *stats : local;
    std::memset(&st, 0, sizeof(st));
    Geom g;
    int rc = make_geom(dims, g);
    if (rc) return st.status = rc;
    hisq_cg_opts o = resolve_opts(opts, g);
    if (!fat || !lng || !b || !x) return st.status = fail(HISQ_EINVAL, "cg_solve: NULL pointer");
    if (!aligned16({fat, lng, fat_lo, lng_lo, b, x, workspace}))
        return st.status = fail(HISQ_EINVAL, "cg_solve: device pointers must be 16-byte aligned");
    if (b == x) return st.status = fail(HISQ_EALIAS, "cg_solve: b and x alias");
    if (!(tol > 0) || !(mass >= 0)) return st.status = fail(HISQ_EINVAL, "cg_solve: need tol > 0 and mass >= 0");
    if (o.mode != HISQ_CG_PLAIN_F64 && o.mode != HISQ_CG_PLAIN_F64C && (!fat_lo || !lng_lo))
        return st.status = fail(HISQ_EINVAL, "cg_solve: mixed mode needs fat_lo and lng_lo");
    if (o.mode < HISQ_CG_PLAIN_F64 || o.mode > HISQ_CG_MIXED_I16SC)
        return st.status = fail(HISQ_EINVAL, "cg_solve: unknown mode");
    if (!(o.delta < 1.0)) return st.status = fail(HISQ_EINVAL, "cg_solve: opts->delta must be below 1");
    if (!workspace || ws_bytes < cg_workspace_bytes(g, o.mode))
        return st.status = fail(HISQ_EWORKSPACE, "cg_solve: workspace NULL or smaller than hisq_workspace_bytes()");
    hipStream_t s = (hipStream_t)stream;
    {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return st.status = hip_fail(e, "cg_solve: pending work failed");
    }
    switch (o.mode) {
    case HISQ_CG_PLAIN_F64: rc = cg_plain<PF64>(mass, tol, fat, lng, b, x, g, o, workspace, ws_bytes, st, s); break;
    case HISQ_CG_PLAIN_F64C: rc = cg_plain<PF64C>(mass, tol, fat, lng, b, x, g, o, workspace, ws_bytes, st, s); break;
    case HISQ_CG_MIXED_F32:
        rc = cg_mixed<PF64, PF32>(mass, tol, fat, lng, fat_lo, lng_lo, b, x, g, o, workspace, ws_bytes, st, s);
        break;
    case HISQ_CG_MIXED_F16S:
        rc = cg_mixed<PF64, PF16S>(mass, tol, fat, lng, fat_lo, lng_lo, b, x, g, o, workspace, ws_bytes, st, s);
        break;
    case HISQ_CG_MIXED_I16S:
        rc = cg_mixed<PF64, PI16S>(mass, tol, fat, lng, fat_lo, lng_lo, b, x, g, o, workspace, ws_bytes, st, s);
        break;
    case HISQ_CG_MIXED_F32C:
        rc = cg_mixed<PF64C, PF32C>(mass, tol, fat, lng, fat_lo, lng_lo, b, x, g, o, workspace, ws_bytes, st, s);
        break;
    default:
        rc = cg_mixed<PF64C, PI16SC>(mass, tol, fat, lng, fat_lo, lng_lo, b, x, g, o, workspace, ws_bytes, st, s);
    }
    st.status = rc;
    return rc;
}

namespace hisq {
// Deterministic dot product on scratch `ws` (>= DOT_WS_BYTES of device memory).
int dot_on(const void *x, const void *y, long long n, int prec, double out_host[2], char *ws, hipStream_t s)
{
    if (n == 0) {
        out_host[0] = out_host[1] = 0.0;
        return HISQ_OK;
    }
    double *part = (double *)ws;
    double *out = (double *)(ws + DOT_PART_BYTES);
    const int nb = (int)std::min<long long>((n + 255) / 256, BLAS_MAX_BLOCKS);
    if ((size_t)nb * 2 * sizeof(double) > DOT_PART_BYTES) return fail(HISQ_EWORKSPACE, "dot: partials exceed the scratch");
    if (prec == HISQ_F64 || prec == HISQ_F64C)
        hipLaunchKernelGGL((k_dot2<double2>), dim3(nb), dim3(BL_NT), 0, s, (const double2 *)x, (const double2 *)y, n,
                           part);
    else
        hipLaunchKernelGGL((k_dot2<float2>), dim3(nb), dim3(BL_NT), 0, s, (const float2 *)x, (const float2 *)y, n,
                           part);
    hipLaunchKernelGGL(k_dot2_fin, dim3(1), dim3(FIN_NT), 0, s, (const double *)part, nb, out);
    HISQ_HIP(hipGetLastError());
    HISQ_HIP(hipMemcpyAsync(out_host, out, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HISQ_HIP(hipStreamSynchronize(s));
    return HISQ_OK;
}
}  // namespace hisq

extern "C" int hisq_dot(const void *x, const void *y, long long n, int prec, double out_host[2], void *workspace,
                        size_t ws_bytes, void *stream)
{
    if (!x || !y || !out_host || n < 0) return fail(HISQ_EINVAL, "hisq_dot: bad argument");
    if (!aligned16({x, y, workspace}))
        return fail(HISQ_EINVAL, "hisq_dot: device pointers must be 16-byte aligned");
    if (prec < HISQ_F64 || prec > HISQ_I16SC) return fail(HISQ_EINVAL, "hisq_dot: bad precision");
    if (!workspace || ws_bytes < DOT_WS_BYTES)
        return fail(HISQ_EWORKSPACE, "hisq_dot: workspace NULL or smaller than hisq_workspace_bytes(\"dot\")");
    return dot_on(x, y, n, prec, out_host, (char *)workspace, (hipStream_t)stream);
}
