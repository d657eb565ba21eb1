// HISQ Dslash kernels (Sec. 3 operator) and the dslash_apply / hisq_apply_A
// entry points.
//
// One thread per output site; a wavefront owns one 64-site tile, so every
// link load instruction of a wavefront reads one contiguous 1 KB (FP64),
// 1 KB/512 B (FP32) or 1 KB/512 B (FP16+scale) span and each link byte is
// read once.  Links are streamed with nontemporal loads so they do not evict
// the neighbour vectors, which are re-read by up to 16 sites and stay in L2
// (the grid is ordered so that each XCD works on one contiguous slab).
#include "dslash_core.hpp"

namespace hisq {

template <class P, int NT, int W, int UNR, int ORD>
__global__ __launch_bounds__(NT) HISQ_WAVES(W) void k_dslash(Geom g, const char *__restrict__ fat, const char *__restrict__ lng,
                                               const typename P::cvec *__restrict__ src,
                                               typename P::cvec *__restrict__ dst, int parity, int nblocks,
                                               const SolverFlags *flags, int gate)
{
    if (gate_closed(flags, gate)) return;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    if (blk >= nblocks) return;
    const int k = blk * (NT / TILE) + (threadIdx.x >> 6);
    if (k >= g.ntiles) return;
    const int tile = ORD ? tile_of(g, k) : k;
    const int lane = threadIdx.x & 63;
    const int h = tile * TILE + lane;
    const int hc = h < g.Vh ? h : g.Vh - 1;
    typename P::real acc[6];
    dslash_site<P, UNR>(g, fat, lng, src, parity, tile, lane, hc, acc);
    if (h < g.Vh) {
        typename P::cvec *o = dst + (size_t)h * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            typename P::cvec v;
            v.x = acc[2 * c];
            v.y = acc[2 * c + 1];
            ntstore(v, o + c);
        }
    }
}

// y = m4 * x - D src on parity 0 (second half of A = 4m^2 - D_eo D_oe)
template <class P, int NT>
__global__ __launch_bounds__(NT) HISQ_WAVES((P::prec == HISQ_F64 || P::prec == HISQ_F64C) ? 6 : 8) void k_dslash_axmy(Geom g, const char *__restrict__ fat,
                                                    const char *__restrict__ lng,
                                                    const typename P::cvec *__restrict__ src,
                                                    const typename P::cvec *__restrict__ x,
                                                    typename P::cvec *__restrict__ y, double m4, int nblocks)
{
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    if (blk >= nblocks) return;
    const int tile = blk * (NT / TILE) + (threadIdx.x >> 6);
    if (tile >= g.ntiles) return;
    const int lane = threadIdx.x & 63;
    const int h = tile * TILE + lane;
    const int hc = h < g.Vh ? h : g.Vh - 1;
    typename P::real acc[6];
    dslash_site<P>(g, fat, lng, src, 0, tile, lane, hc, acc);
    if (h < g.Vh) {
        const typename P::real m = (typename P::real)m4;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            typename P::cvec xv = x[(size_t)h * 3 + c], v;
            v.x = fma(m, xv.x, -acc[2 * c]);
            v.y = fma(m, xv.y, -acc[2 * c + 1]);
            y[(size_t)h * 3 + c] = v;
        }
    }
}

// Launch shapes of the single-RHS Dslash: threads per block, minimum
// wavefronts per SIMD (1 = no constraint), how many of the 16 terms are
// unrolled together and the tile order.  All shapes compute every site with
// the same arithmetic in the same order, so their outputs are bitwise
// identical; the autotuner picks one per (lattice, precision).
const DslashShape DSLASH_SHAPES[N_DSLASH_SHAPES] = {
    { 256, 8, 1, 0 }, { 128, 8, 1, 0 }, { 64, 8, 1, 0 }, { 256, 1, 16, 0 }, { 256, 4, 4, 0 },
    { 512, 8, 1, 0 }, { 256, 6, 1, 0 }, { 256, 8, 1, 1 }, { 256, 6, 1, 1 }, { 256, 6, 2, 0 }, { 256, 5, 2, 0 },
    { 256, 5, 2, 2 }, { 256, 5, 2, 3 },
};

static inline int blocks_for(const Geom &g, int nt) { return (g.ntiles + nt / TILE - 1) / (nt / TILE); }

template <class P, int NT, int W, int UNR, int ORD = 0>
static void launch_shape(const Geom &g0, const void *fat, const void *lng, const void *src, void *dst, int parity,
                         hipStream_t s, const SolverFlags *flags, int gate)
{
    Geom g = g0;
    if (ORD) apply_order(g, ORD);
    if (ORD && !g.oP) {  // the lattice has no such order: plain order
        launch_shape<P, NT, W, UNR, 0>(g0, fat, lng, src, dst, parity, s, flags, gate);
        return;
    }
    const int nb = blocks_for(g, NT);
    hipLaunchKernelGGL((k_dslash<P, NT, W, UNR, (ORD != 0)>), dim3(xcd_grid(nb)), dim3(NT), 0, s, g, (const char *)fat,
                       (const char *)lng, (const typename P::cvec *)src, (typename P::cvec *)dst, parity, nb, flags,
                       gate);
}

template <class P>
hipError_t launch_dslash_shape(int shape, const Geom &g, const void *fat, const void *lng, const void *src, void *dst,
                               int parity, hipStream_t s, const SolverFlags *flags, int gate)
{
    switch (shape) {
    case 1: launch_shape<P, 128, 8, 1>(g, fat, lng, src, dst, parity, s, flags, gate); break;
    case 2: launch_shape<P, 64, 8, 1>(g, fat, lng, src, dst, parity, s, flags, gate); break;
    case 3: launch_shape<P, 256, 1, 16>(g, fat, lng, src, dst, parity, s, flags, gate); break;
    case 4: launch_shape<P, 256, 4, 4>(g, fat, lng, src, dst, parity, s, flags, gate); break;
    case 5: launch_shape<P, 512, 8, 1>(g, fat, lng, src, dst, parity, s, flags, gate); break;
    case 6: launch_shape<P, 256, 6, 1>(g, fat, lng, src, dst, parity, s, flags, gate); break;
    case 7: launch_shape<P, 256, 8, 1, 1>(g, fat, lng, src, dst, parity, s, flags, gate); break;
    case 8: launch_shape<P, 256, 6, 1, 1>(g, fat, lng, src, dst, parity, s, flags, gate); break;
    case 9: launch_shape<P, 256, 6, 2>(g, fat, lng, src, dst, parity, s, flags, gate); break;
    case 10: launch_shape<P, 256, 5, 2>(g, fat, lng, src, dst, parity, s, flags, gate); break;
    case 11: launch_shape<P, 256, 5, 2, 2>(g, fat, lng, src, dst, parity, s, flags, gate); break;
    case 12: launch_shape<P, 256, 5, 2, 3>(g, fat, lng, src, dst, parity, s, flags, gate); break;
    default: launch_shape<P, 256, 8, 1>(g, fat, lng, src, dst, parity, s, flags, gate); break;
    }
    return hipGetLastError();
}

template <class P>
hipError_t launch_dslash(const Geom &g, const void *fat, const void *lng, const void *src, void *dst, int parity,
                         hipStream_t s, const SolverFlags *flags, int gate)
{
    return launch_dslash_shape<P>(tuned_dslash_shape(g, P::prec), g, fat, lng, src, dst, parity, s, flags, gate);
}

#define HISQ_INST(P)                                                                                             \
    template hipError_t launch_dslash<P>(const Geom &, const void *, const void *, const void *, void *, int,    \
                                         hipStream_t, const SolverFlags *, int);                                 \
    template hipError_t launch_dslash_shape<P>(int, const Geom &, const void *, const void *, const void *,      \
                                               void *, int, hipStream_t, const SolverFlags *, int);
HISQ_INST(PF64)
HISQ_INST(PF32)
HISQ_INST(PF16S)
HISQ_INST(PI16S)
HISQ_INST(PF64C)
HISQ_INST(PF32C)
HISQ_INST(PI16SC)
#undef HISQ_INST

constexpr int AXMY_NT = 256;

template <class P>
static hipError_t launch_apply_A(const Geom &g, double mass, const void *fat, const void *lng, const void *x, void *y,
                                 void *tmp, hipStream_t s)
{
    hipError_t e = launch_dslash<P>(g, fat, lng, x, tmp, 1, s);
    if (e != hipSuccess) return e;
    const int nb = blocks_for(g, AXMY_NT);
    hipLaunchKernelGGL((k_dslash_axmy<P, AXMY_NT>), dim3(xcd_grid(nb)), dim3(AXMY_NT), 0, s, g,
                       (const char *)fat, (const char *)lng, (const typename P::cvec *)tmp,
                       (const typename P::cvec *)x, (typename P::cvec *)y, 4.0 * mass * mass, nb);
    return hipGetLastError();
}

}  // namespace hisq

using namespace hisq;

extern "C" int dslash_apply(const void *fat, const void *lng, const void *src, void *dst, int parity,
                            const int dims[4], int prec, void *stream)
{
    Geom g;
    int rc = make_geom(dims, g);
    if (rc) return rc;
    if (!fat || !lng || !src || !dst) return fail(HISQ_EINVAL, "dslash_apply: NULL pointer");
    if (!aligned16({fat, lng, src, dst}))
        return fail(HISQ_EINVAL, "dslash_apply: device pointers must be 16-byte aligned");
    if (parity != 0 && parity != 1) return fail(HISQ_EINVAL, "dslash_apply: parity must be 0 or 1");
    if (src == dst) return fail(HISQ_EALIAS, "dslash_apply: src and dst alias");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    switch (prec) {
    case HISQ_F64: e = launch_dslash<PF64>(g, fat, lng, src, dst, parity, s); break;
    case HISQ_F32: e = launch_dslash<PF32>(g, fat, lng, src, dst, parity, s); break;
    case HISQ_F16S: e = launch_dslash<PF16S>(g, fat, lng, src, dst, parity, s); break;
    case HISQ_I16S: e = launch_dslash<PI16S>(g, fat, lng, src, dst, parity, s); break;
    case HISQ_F64C: e = launch_dslash<PF64C>(g, fat, lng, src, dst, parity, s); break;
    case HISQ_F32C: e = launch_dslash<PF32C>(g, fat, lng, src, dst, parity, s); break;
    case HISQ_I16SC: e = launch_dslash<PI16SC>(g, fat, lng, src, dst, parity, s); break;
    default: return fail(HISQ_EINVAL, "dslash_apply: unknown precision");
    }
    if (e != hipSuccess) return hip_fail(e, "dslash_apply launch");
    return HISQ_OK;
}

extern "C" int hisq_apply_A(double mass, const void *fat, const void *lng, const void *x, void *y, void *tmp,
                            const int dims[4], int prec, void *stream)
{
    Geom g;
    int rc = make_geom(dims, g);
    if (rc) return rc;
    if (!fat || !lng || !x || !y || !tmp) return fail(HISQ_EINVAL, "hisq_apply_A: NULL pointer");
    if (!aligned16({fat, lng, x, y, tmp}))
        return fail(HISQ_EINVAL, "hisq_apply_A: device pointers must be 16-byte aligned");
    if (x == y || x == tmp || y == tmp) return fail(HISQ_EALIAS, "hisq_apply_A: x, y, tmp must be distinct");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    switch (prec) {
    case HISQ_F64: e = launch_apply_A<PF64>(g, mass, fat, lng, x, y, tmp, s); break;
    case HISQ_F32: e = launch_apply_A<PF32>(g, mass, fat, lng, x, y, tmp, s); break;
    case HISQ_F16S: e = launch_apply_A<PF16S>(g, mass, fat, lng, x, y, tmp, s); break;
    case HISQ_I16S: e = launch_apply_A<PI16S>(g, mass, fat, lng, x, y, tmp, s); break;
    case HISQ_F64C: e = launch_apply_A<PF64C>(g, mass, fat, lng, x, y, tmp, s); break;
    case HISQ_F32C: e = launch_apply_A<PF32C>(g, mass, fat, lng, x, y, tmp, s); break;
    case HISQ_I16SC: e = launch_apply_A<PI16SC>(g, mass, fat, lng, x, y, tmp, s); break;
    default: return fail(HISQ_EINVAL, "hisq_apply_A: unknown precision");
    }
    if (e != hipSuccess) return hip_fail(e, "hisq_apply_A launch");
    return HISQ_OK;
}
