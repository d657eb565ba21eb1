// Per-site HISQ Dslash, shared by every kernel that applies the operator.
//
// Sec. 3 of the paper: at each site the operator reads 16 link matrices (a
// one-link and a three-link matrix for each of the 8 directions +-mu) and 16
// neighbour colour vectors, and sums 16 matrix-vector products.  The packed
// links already hold -U^dag for the backward directions, so every term is a
// plain product M_d(n) psi(n + k_d).
#pragma once

#include "hisq_common.hpp"

namespace hisq {

// Directions in the packed layout, per field: 0..3 = +x,+y,+z,+t ; 4..7 = -x,-y,-z,-t.
// Fat links hop 1 site, long links 3 sites.

template <class P>
__device__ __forceinline__ void cmac(typename P::real acc[6], const typename P::real m[18], typename P::cvec s0,
                                     typename P::cvec s1, typename P::cvec s2)
{
    const typename P::real sr[3] = { s0.x, s1.x, s2.x };
    const typename P::real si[3] = { s0.y, s1.y, s2.y };
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const typename P::real mr = m[2 * (3 * a + b)], mi = m[2 * (3 * a + b) + 1];
            acc[2 * a] = fma(mr, sr[b], acc[2 * a]);
            acc[2 * a] = fma(-mi, si[b], acc[2 * a]);
            acc[2 * a + 1] = fma(mr, si[b], acc[2 * a + 1]);
            acc[2 * a + 1] = fma(mi, sr[b], acc[2 * a + 1]);
        }
    }
}

// acc += M psi for a two-row matrix: rows 0 and 1 from m[0..11], row 2 =
// c conj(row0 x row1) taken one entry at a time straight into acc[4..5], so
// the third row is never held in registers.
template <class P>
__device__ __forceinline__ void cmac_two_row(typename P::real acc[6], const typename P::real m[12],
                                             typename P::real c, typename P::cvec s0, typename P::cvec s1,
                                             typename P::cvec s2)
{
    using R = typename P::real;
    const R sr[3] = { s0.x, s1.x, s2.x };
    const R si[3] = { s0.y, s1.y, s2.y };
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const R mr = m[2 * (3 * a + b)], mi = m[2 * (3 * a + b) + 1];
            acc[2 * a] = fma(mr, sr[b], acc[2 * a]);
            acc[2 * a] = fma(-mi, si[b], acc[2 * a]);
            acc[2 * a + 1] = fma(mr, si[b], acc[2 * a + 1]);
            acc[2 * a + 1] = fma(mi, sr[b], acc[2 * a + 1]);
        }
    }
    R tr = 0, ti = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        const R ar1 = m[2 * j1], ai1 = m[2 * j1 + 1], ar2 = m[2 * j2], ai2 = m[2 * j2 + 1];
        const R br1 = m[6 + 2 * j1], bi1 = m[6 + 2 * j1 + 1], br2 = m[6 + 2 * j2], bi2 = m[6 + 2 * j2 + 1];
        // x_j = a_{j+1} b_{j+2} - a_{j+2} b_{j+1}
        const R xr = (ar1 * br2 - ai1 * bi2) - (ar2 * br1 - ai2 * bi1);
        const R xi = (ar1 * bi2 + ai1 * br2) - (ar2 * bi1 + ai2 * br1);
        // conj(x_j) s_j
        tr = fma(xr, sr[j], tr);
        tr = fma(xi, si[j], tr);
        ti = fma(xr, si[j], ti);
        ti = fma(-xi, sr[j], ti);
    }
    acc[4] = fma(c, tr, acc[4]);
    acc[5] = fma(c, ti, acc[5]);
}

// acc = (D src)(h) for the site h of parity `parity` (h < Vh), whose links
// sit at lane `lane` of tile `tile`.  The 16 terms are taken UNR at a time:
// a fully unrolled body lets the compiler hoist every load and run out of
// registers, a partly unrolled one keeps UNR matrices in flight per thread
// and leaves the latency hiding to the other resident wavefronts.
template <class P, int UNR = 1>
__device__ __forceinline__ void dslash_site(const Geom &g, const char *__restrict__ fat,
                                            const char *__restrict__ lng,
                                            const typename P::cvec *__restrict__ src, int parity, int tile,
                                            int lane, int h, typename P::real acc[6])
{
    int x, y, z, t;
    site_coords(g, h, parity, x, y, z, t);
    const size_t tix = (size_t)parity * g.ntiles + tile;
    const char *fb = fat + tix * P::Fat::tile_bytes;
    const char *lb = lng + tix * P::Long::tile_bytes;
#pragma unroll
    for (int i = 0; i < 6; ++i) acc[i] = 0;
    // one-link terms, then three-link terms (separate loops keep one loader live)
#pragma unroll UNR
    for (int d = 0; d < 8; ++d) {
        const int nh = nbr_h(g, h, x, y, z, t, d & 3, (d >> 2) ? -1 : 1);
        typename P::real m[18];
        P::Fat::load_dir(fb, d, lane, m);
        const typename P::cvec *s = src + (size_t)nh * 3;
        cmac<P>(acc, m, s[0], s[1], s[2]);
    }
#pragma unroll UNR
    for (int d = 0; d < 8; ++d) {
        const int nh = nbr_h(g, h, x, y, z, t, d & 3, (d >> 2) ? -3 : 3);
        const typename P::cvec *s = src + (size_t)nh * 3;
        if constexpr (P::Long::two_row) {
            typename P::real m[12];
            const typename P::real c = P::Long::load_rows(lb, d, lane, m);
            cmac_two_row<P>(acc, m, c, s[0], s[1], s[2]);
        } else {
            typename P::real m[18];
            P::Long::load_dir(lb, d, lane, m);
            cmac<P>(acc, m, s[0], s[1], s[2]);
        }
    }
}

// Kernel gates read from a solver's device-resident state (NULL: always run).
struct SolverFlags {
    int done;      // nonzero: solve finished (converged or broke down)
    int reliable;  // nonzero: a reliable update is pending this iteration
};
enum { GATE_ALWAYS = 0, GATE_NOT_DONE = 1, GATE_RELIABLE = 2 };

__device__ __forceinline__ bool gate_closed(const SolverFlags *f, int gate)
{
    if (gate == GATE_ALWAYS || f == nullptr) return false;
    if (f->done) return true;
    return gate == GATE_RELIABLE && !f->reliable;
}

// Launch helpers (defined in dslash.hip).  launch_dslash uses the shape the
// autotuner chose for (dims, precision), launch_dslash_shape a given one.
struct DslashShape {
    int nt;      // threads per block
    int waves;   // minimum wavefronts per SIMD the compiler must allow
    int unroll;  // terms of the 16 unrolled together
    int order;   // tile order (apply_order): 0 plain, 1 default blocks, 2 and 3 8- and 4-plane t-blocks by all z
};
constexpr int N_DSLASH_SHAPES = 13;
extern const DslashShape DSLASH_SHAPES[N_DSLASH_SHAPES];
int tuned_dslash_shape(const Geom &g, int prec);            // tune.cpp
int tuned_choice(const char *kind, const Geom &g, int prec, int n, int fallback);
void set_tuned_choice(const char *kind, const Geom &g, int prec, int n, int v);
void set_tuned_dslash_shape(const Geom &g, int prec, int shape);

template <class P>
hipError_t launch_dslash(const Geom &g, const void *fat, const void *lng, const void *src, void *dst, int parity,
                         hipStream_t s, const SolverFlags *flags = nullptr, int gate = GATE_ALWAYS);
template <class P>
hipError_t launch_dslash_shape(int shape, const Geom &g, const void *fat, const void *lng, const void *src, void *dst,
                               int parity, hipStream_t s, const SolverFlags *flags = nullptr, int gate = GATE_ALWAYS);

}  // namespace hisq
