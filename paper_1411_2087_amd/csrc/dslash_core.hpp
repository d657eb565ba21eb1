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
        typename P::real m[18];
        P::Long::load_dir(lb, d, lane, m);
        const typename P::cvec *s = src + (size_t)nh * 3;
        cmac<P>(acc, m, s[0], s[1], s[2]);
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
};
constexpr int N_DSLASH_SHAPES = 7;
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
