// Batched solves of the even-odd system for several right-hand sides or
// several masses (Sec. 3: the multishift CG of gauge generation solves one
// source for 9 or 11 masses; its working set is (36 + 2 N_m) 48 V bytes).
//
// MULTI_RHS: nrhs systems A(m_i) x_i = b_i advance together.  Every Dslash is
// one launch over all right-hand sides: a thread loads each link matrix once
// and applies it to the G right-hand sides it owns, so the link stream (96% of
// the single-RHS bytes) is shared by the batch.  Inner iterations run on FP32
// vectors and links with FP64 dot accumulation; each right-hand side keeps
// its own alpha, beta, reliable-update trigger and convergence flag, and the
// FP64 reliable update / true-residual Dslash runs only for the right-hand
// sides that asked for it (a per-RHS mask).
//
// MULTI_SHIFT: one source b and masses m_i: shifted CG (Jegerlehner 1996,
// the residual polynomials of all shifted systems are collinear with the
// base system's) runs one Dslash pair per iteration for all shifts in FP32,
// then every x_i is refined to tol by the MULTI_RHS solver started from it.
//
// Internal vectors are site-major [Vh][N][3] so that the N right-hand sides
// of a neighbour are one contiguous read.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "cg_internal.hpp"

namespace hisq {

constexpr int MAXR = 16;

struct MultiState {
    SolverFlags flags;  // done: every RHS finished ; reliable: some RHS has an update pending
    int n;              // right-hand sides in use
    unsigned active;    // bit r: RHS r still iterating
    unsigned relmask;   // bit r: reliable update pending for RHS r
    int iter;           // batch iterations
    int iters[MAXR], nupd[MAXR], status[MAXR];
    double tol2, delta2;
    double m4[MAXR], bb[MAXR], stop2[MAXR], rr[MAXR], rr_true[MAXR], maxrr[MAXR], alpha[MAXR], beta[MAXR];
    // shifted CG
    double sigma0, rr0, bb0, stop0, alpha0, beta0, a_prev, b_prev;
    double dsig[MAXR], zeta[MAXR], zeta_prev[MAXR], zeta_next[MAXR], alpha_s[MAXR], beta_s[MAXR];
    double rr_s[MAXR];  // |zeta_i r|^2: shift i's recursive residual after its last iteration
    int ms_status;
};

enum { EPI_STORE = 0, EPI_RESID = 2, EPI_STORE_NORM = 3, EPI_UPD = 4 };
enum { MASK_ACTIVE = 0, MASK_RELIABLE = 1, MASK_ALL = 2 };

__device__ __forceinline__ unsigned pick_mask(const MultiState *st, int which)
{
    return which == MASK_ACTIVE ? st->active : (which == MASK_RELIABLE ? st->relmask : ((1u << st->n) - 1u));
}

// Right-hand sides whose neighbour vectors a thread loads together before
// multiplying any of them, where the vectors do not go through LDS: 2 in
// FP64 (12 double registers), up to 4 in FP32.
template <class P> constexpr int md_chunk() { return sizeof(typename P::real) == 4 ? 4 : 2; }

// Orders LDS writes by some lanes of a wavefront before reads by others
// (a wavefront's LDS instructions execute in order; this keeps the compiler
// from moving them across each other).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ multi-RHS Dslash
// N right-hand sides in [Vh][N][3]; each thread owns G of them for one site,
// N/G consecutive threads share a site (their link loads hit the same
// addresses and are served once).  Persistent: blocks stride over site units
// inside the slab of their XCD.
//
// FP32 neighbour vectors go through LDS.  A wavefront's S = 64 G / N sites
// need, per direction, S neighbour blocks of N x 24 contiguous bytes; loaded
// by the owning threads (each its G x 24 bytes) one instruction touches up to
// 3 cache lines per site and the vector L1 stalls the address unit.  Instead
// consecutive lanes load consecutive 16-byte chunks of the S blocks (each lane
// gets the neighbour index of the block it loads from the lane that computed
// it), the chunks go to LDS in that order, and each thread reads its G
// right-hand sides back.  With that and every neighbour load issued ahead of
// the mask tests, the N = 16 Dslash at 32^4 went from 745 to 431 us.
// PIPE (FP32 links, LDS staging): the link and neighbour loads of direction
// d + 1 leave before the products of direction d, so one direction's
// latency overlaps the previous direction's arithmetic instead of being
// hidden only by other wavefronts.  Full FP32 matrices only: a two-row or
// 16-bit link is rebuilt or converted as soon as it arrives, which would
// wait for the load at the point where it is issued.
//   EPI_STORE      : dst = D src
//   EPI_STORE_NORM : dst = D src, partial |dst|^2 per RHS
//   EPI_UPD        : (FP32) with x = p: a = m4_r p - D src in registers, dst (= xs) += alpha_r p,
//                    rs -= alpha_r a, partial |rs|^2 per RHS
//   EPI_RESID      : (FP64) dst = b - (m4_r x - D src), rs = float(dst), partial |dst|^2 per RHS
template <class P, int N, int G, int NT, int EPI, bool PIPE = false>
__global__ __launch_bounds__(NT) void k_mdslash(Geom g, const char *__restrict__ fat, const char *__restrict__ lng,
                                                const typename P::cvec *__restrict__ src,
                                                typename P::cvec *__restrict__ dst,
                                                const typename P::cvec *__restrict__ x,
                                                const typename P::cvec *__restrict__ b, float2 *__restrict__ rs,
                                                int parity, int nunits, double *partials, const MultiState *st,
                                                int which_mask, int gate)
{
    using R = typename P::real;
    using V = typename P::cvec;
    constexpr int TPS = N / G;        // threads per site
    constexpr int SPB = NT / TPS;     // sites per block per unit
    // LDS staging of the neighbour blocks (FP32, N >= 2 and even G: 16-byte chunks)
    constexpr bool MD_LDS = sizeof(R) == 4 && N >= 2 && G % 2 == 0;
    constexpr int MD_K4 = 3 * N / 2;                      // 16-byte chunks per site block
    constexpr int MD_C4 = (64 / TPS) * MD_K4;             // chunks per wavefront and direction
    constexpr int MD_RR = (MD_C4 + 63) / 64;              // load rounds
    constexpr bool MD_PIPE = PIPE && MD_LDS && std::is_same<P, PF32>::value;
    // PIPE with TPS >= 2: the S links of a wavefront's sites are loaded once, cooperatively, and staged in LDS
    // (pitch 20 floats per site: 16-byte aligned, the S sites' 4-bank groups distinct)
    constexpr int MD_S = 64 / TPS;
    constexpr bool MD_LSH = MD_PIPE && TPS >= 2;
    constexpr int MD_LR = (4 * MD_S + 63) / 64;  // rounds of the 4 S 16-byte link chunks
    __shared__ float4 stage_all[MD_LDS ? NT / 64 : 1][MD_LDS ? MD_C4 : 1];
    __shared__ __align__(16) float lstage_all[MD_LSH ? NT / 64 : 1][MD_LSH ? MD_S * 20 : 4];
    float4 *stage = stage_all[MD_LDS ? (threadIdx.x >> 6) : 0];
    float *lstage = lstage_all[MD_LSH ? (threadIdx.x >> 6) : 0];
    const int wl = threadIdx.x & 63;
    if (solver_gate_closed(&st->flags, gate)) return;
    const unsigned mask = pick_mask(st, which_mask);
    const int grp = threadIdx.x % TPS;
    const int r0 = grp * G;
    double part[G];
#pragma unroll
    for (int j = 0; j < G; ++j) part[j] = 0.0;
    double m4[G], al[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
        m4[j] = (EPI == EPI_RESID || EPI == EPI_UPD) ? st->m4[r0 + j] : 0.0;
        al[j] = (EPI == EPI_UPD) ? st->alpha[r0 + j] : 0.0;
    }

    // XCD-aware persistent order: XCD k walks the k-th slab of units
    const int xcd = blockIdx.x % NXCD, local = blockIdx.x / NXCD, per_xcd = gridDim.x / NXCD;
    const int units_per_xcd = (nunits + NXCD - 1) / NXCD;
    for (int u = local; u < units_per_xcd; u += per_xcd) {
        const int unit = xcd * units_per_xcd + u;
        if (unit >= nunits) break;
        // the unit's sites in processing order; with the blocked tile order
        // (g.oP != 0, tile_of) the t and z neighbours of the sites in flight
        // were gathered shortly before and are still in L2
        const int s_ord = unit * SPB + threadIdx.x / TPS;
        const int site = s_ord < g.Vh ? tile_of(g, s_ord / TILE) * TILE + s_ord % TILE : s_ord;
        const int h = site < g.Vh ? site : g.Vh - 1;
        const int tile = h / TILE, lane = h % TILE;
        int cx, cy, cz, ct;
        site_coords(g, h, parity, cx, cy, cz, ct);
        const size_t tix = (size_t)parity * g.ntiles + tile;
        const char *fat_t = fat + tix * P::Fat::tile_bytes;
        const char *lng_t = lng + tix * P::Long::tile_bytes;
        R acc[G][6];
#pragma unroll
        for (int j = 0; j < G; ++j)
#pragma unroll
            for (int i = 0; i < 6; ++i) acc[j][i] = 0;
        if constexpr (MD_PIPE) {
            // native vectors: copies of HIP's float4 struct go through memory
            typedef float f4v __attribute__((ext_vector_type(4)));
            typedef float f2v __attribute__((ext_vector_type(2)));
            R mn[18];             // the link of the next direction, in flight (TPS = 1)
            f4v lpre[MD_LR];      // its chunks (TPS >= 2): chunk j = row j / S (4 floats) of site j % S
            f2v ltail = { 0.f, 0.f };  // entries 16, 17 of site wl (wl < S)
            f4v pre[MD_RR];       // its neighbour chunks, in flight
            // the wavefront's sites are lanes L0 .. L0 + S - 1 of one tile (S divides 64); a wavefront past
            // the lattice reads the last tile (its results are not stored)
            const int s_w = unit * SPB + (threadIdx.x >> 6) * MD_S;
            const int blk64 = s_w / TILE, L0 = s_w % TILE;
            const int wtile = blk64 < g.ntiles ? tile_of(g, blk64) : g.ntiles - 1;
            const size_t wtix = (size_t)parity * g.ntiles + wtile;
            const char *wfat = fat + wtix * P::Fat::tile_bytes, *wlng = lng + wtix * P::Long::tile_bytes;
            // step d: publish direction d, issue the loads of d + 1, then the products of d
            // (step -1 only issues direction 0)
#pragma unroll 1
            for (int d = -1; d < 16; ++d) {
                R m[18];
                if (d >= 0) {
                    if constexpr (!MD_LSH) {
#pragma unroll
                        for (int i = 0; i < 18; ++i) m[i] = mn[i];
                    }
                    wave_sync();  // every lane has read the previous direction's blocks and link
#pragma unroll
                    for (int q = 0; q < MD_RR; ++q) {
                        const int j = q * 64 + wl;
                        if ((MD_C4 % 64 == 0) || j < MD_C4) reinterpret_cast<f4v *>(stage)[j] = pre[q];
                    }
                    if constexpr (MD_LSH) {
#pragma unroll
                        for (int q = 0; q < MD_LR; ++q) {
                            const int j = q * 64 + wl;
                            if (((4 * MD_S) % 64 == 0) || j < 4 * MD_S)
                                *reinterpret_cast<f4v *>(lstage + (j % MD_S) * 20 + 4 * (j / MD_S)) = lpre[q];
                        }
                        if (wl < MD_S) *reinterpret_cast<f2v *>(lstage + wl * 20 + 16) = ltail;
                    }
                    wave_sync();
                    if constexpr (MD_LSH) {
                        const float *ms = lstage + (wl / TPS) * 20;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const f4v v = *reinterpret_cast<const f4v *>(ms + 4 * r);
                            m[4 * r] = v.x; m[4 * r + 1] = v.y; m[4 * r + 2] = v.z; m[4 * r + 3] = v.w;
                        }
                        const f2v t2 = *reinterpret_cast<const f2v *>(ms + 16);
                        m[16] = t2.x;
                        m[17] = t2.y;
                    }
                }
                if (d + 1 < 16) {
                    const int dn = d + 1, mu = dn & 3;
                    const bool is_long = dn >= 8;
                    const int k = (is_long ? 3 : 1) * (((dn >> 2) & 1) ? -1 : 1);
                    const int nh = nbr_h(g, h, cx, cy, cz, ct, mu, k);
                    if constexpr (MD_LSH) {
                        const char *blk = (is_long ? wlng : wfat) + (size_t)(dn & 7) * P::Fat::block_bytes;
#pragma unroll
                        for (int q = 0; q < MD_LR; ++q) {
                            const int j = q * 64 + wl;
                            if (((4 * MD_S) % 64 == 0) || j < 4 * MD_S)
                                lpre[q] = __builtin_nontemporal_load(
                                    reinterpret_cast<const f4v *>(blk) + (j / MD_S) * TILE + L0 + j % MD_S);
                        }
                        if (wl < MD_S)
                            ltail = __builtin_nontemporal_load(reinterpret_cast<const f2v *>(blk + 4 * TILE * 16) + L0 + wl);
                    } else if (is_long) {
                        P::Long::load_dir(lng_t, dn & 7, lane, mn);
                    } else {
                        P::Fat::load_dir(fat_t, dn & 7, lane, mn);
                    }
#pragma unroll
                    for (int q = 0; q < MD_RR; ++q) {
                        const int j = q * 64 + wl;
                        const bool in = (MD_C4 % 64 == 0) || j < MD_C4;
                        const int sj = (in ? j : 0) / MD_K4, kj = (in ? j : 0) - sj * MD_K4;
                        const int ns = __shfl(nh, sj * TPS);
                        pre[q] = reinterpret_cast<const f4v *>(src)[(size_t)ns * MD_K4 + kj];
                    }
                }
                if (d < 0) continue;
                const float4 *o = stage + (wl / TPS) * MD_K4 + r0 * 3 / 2;
                float f[6 * G];
#pragma unroll
                for (int q = 0; q < 3 * G / 2; ++q) {
                    const float4 w = o[q];
                    f[4 * q] = w.x;
                    f[4 * q + 1] = w.y;
                    f[4 * q + 2] = w.z;
                    f[4 * q + 3] = w.w;
                }
#pragma unroll
                for (int j = 0; j < G; ++j)
                    cmac<P>(acc[j], m, make_float2(f[6 * j], f[6 * j + 1]), make_float2(f[6 * j + 2], f[6 * j + 3]),
                            make_float2(f[6 * j + 4], f[6 * j + 5]));
            }
        } else
#pragma unroll 1
        for (int d = 0; d < 16; ++d) {
            const int mu = d & 3;
            const bool is_long = d >= 8;
            const int k = (is_long ? 3 : 1) * (((d >> 2) & 1) ? -1 : 1);
            const int nh = nbr_h(g, h, cx, cy, cz, ct, mu, k);
            R m[18];  // a two-row long link is rebuilt in full: it serves G right-hand sides
            if (is_long) P::Long::load_dir(lng_t, d & 7, lane, m);
            else P::Fat::load_dir(fat_t, d & 7, lane, m);
            if constexpr (MD_LDS) {
                wave_sync();  // every lane has read the previous direction's blocks
#pragma unroll
                for (int q = 0; q < MD_RR; ++q) {
                    const int j = q * 64 + wl;
                    const bool in = (MD_C4 % 64 == 0) || j < MD_C4;
                    const int sj = (in ? j : 0) / MD_K4, kj = (in ? j : 0) - sj * MD_K4;
                    const int ns = __shfl(nh, sj * TPS);
                    const float4 w = reinterpret_cast<const float4 *>(src)[(size_t)ns * MD_K4 + kj];
                    if (in) stage[j] = w;
                }
                wave_sync();
                const float4 *o = stage + (wl / TPS) * MD_K4 + r0 * 3 / 2;
                float f[6 * G];
#pragma unroll
                for (int q = 0; q < 3 * G / 2; ++q) {
                    const float4 w = o[q];
                    f[4 * q] = w.x;
                    f[4 * q + 1] = w.y;
                    f[4 * q + 2] = w.z;
                    f[4 * q + 3] = w.w;
                }
                // products for every RHS, active or not (the mask guards the
                // stores only): a per-lane test here split the G products into
                // branches and doubled the N = 8 Dslash at G = 8 (413 -> 230 us)
#pragma unroll
                for (int j = 0; j < G; ++j)
                    cmac<P>(acc[j], m, make_float2(f[6 * j], f[6 * j + 1]), make_float2(f[6 * j + 2], f[6 * j + 3]),
                            make_float2(f[6 * j + 4], f[6 * j + 5]));
            } else {
                const V *s = src + ((size_t)nh * N + r0) * 3;
                // the chunk's vectors are loaded whether or not their RHS is active
                // (the loads then leave together; a load under the mask test would
                // wait for the previous RHS's products), the products only for active ones
                constexpr int CH = G < md_chunk<P>() ? G : md_chunk<P>();
#pragma unroll
                for (int j0 = 0; j0 < G; j0 += CH) {
                    V v[CH][3];
#pragma unroll
                    for (int j = 0; j < CH; ++j)
#pragma unroll
                        for (int c = 0; c < 3; ++c) v[j][c] = s[3 * (j0 + j) + c];
#pragma unroll
                    for (int j = 0; j < CH; ++j)
                        if (mask & (1u << (r0 + j0 + j))) cmac<P>(acc[j0 + j], m, v[j][0], v[j][1], v[j][2]);
                }
            }
        }
        if (site < g.Vh) {
#pragma unroll
            for (int j = 0; j < G; ++j) {
                if (!(mask & (1u << (r0 + j)))) continue;
                const size_t base = ((size_t)site * N + r0 + j) * 3;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    V v;
                    if (EPI == EPI_UPD) {
                        const V pv = x[base + c];
                        const R ax = fma((R)m4[j], pv.x, -acc[j][2 * c]), ay = fma((R)m4[j], pv.y, -acc[j][2 * c + 1]);
                        const R a = (R)al[j];
                        V xv = dst[base + c];
                        float2 rv = rs[base + c];
                        xv.x = fma(a, pv.x, xv.x);
                        xv.y = fma(a, pv.y, xv.y);
                        rv.x = fmaf(-(float)a, (float)ax, rv.x);
                        rv.y = fmaf(-(float)a, (float)ay, rv.y);
                        ntstore(rv, rs + base + c);
                        part[j] = fma((double)rv.x, (double)rv.x, part[j]);
                        part[j] = fma((double)rv.y, (double)rv.y, part[j]);
                        ntstore(xv, dst + base + c);
                        continue;
                    }
                    if (EPI == EPI_STORE || EPI == EPI_STORE_NORM) {
                        v.x = acc[j][2 * c];
                        v.y = acc[j][2 * c + 1];
                        if (EPI == EPI_STORE_NORM) {
                            part[j] = fma((double)v.x, (double)v.x, part[j]);
                            part[j] = fma((double)v.y, (double)v.y, part[j]);
                        }
                    } else {
                        V xv = x[base + c], bv = b[base + c];
                        v.x = bv.x - fma((R)m4[j], xv.x, -acc[j][2 * c]);
                        v.y = bv.y - fma((R)m4[j], xv.y, -acc[j][2 * c + 1]);
                        rs[base + c] = make_float2((float)v.x, (float)v.y);
                        part[j] = fma((double)v.x, (double)v.x, part[j]);
                        part[j] = fma((double)v.y, (double)v.y, part[j]);
                    }
                    if (N == 1) ntstore(v, dst + base + c);  // measured: streaming helps one RHS only
                    else dst[base + c] = v;
                }
            }
        }
    }
    if (EPI != EPI_STORE) {
        // fixed-order per-RHS block partials: [blk][N]
        __shared__ double red[NT * G];
#pragma unroll
        for (int j = 0; j < G; ++j) red[threadIdx.x * G + j] = part[j];
        __syncthreads();
        if (threadIdx.x < N) {
            const int r = threadIdx.x, gr = r / G, j = r % G;
            double s = 0.0;
            for (int t = 0; t < SPB; ++t) s += red[(t * TPS + gr) * G + j];
            partials[(size_t)blockIdx.x * N + r] = s;
        }
    }
}

// ------------------------------------------------------------------ batched BLAS
// One thread per (site, RHS) pair j = site * N + r: its 3 colours are 24 B
// (FP32) or 48 B (FP64) contiguous and a wavefront covers 64 consecutive
// pairs, so loads are contiguous; per-RHS scalars come from LDS.
constexpr int MB_NT = 256;
constexpr int FIN_NT_M = 256;
constexpr int MULTI_MAX_BLOCKS = 2048;

static inline int mblocks(long long pairs)
{
    long long nb = (pairs + MB_NT - 1) / MB_NT;
    return (int)std::min<long long>(std::max<long long>(nb, 1), MULTI_MAX_BLOCKS);
}

// per-RHS block partials of the values `v` each thread accumulated for RHS
// r = j % N (the same for every pair this thread visits, since the grid
// stride is a multiple of N)
template <int N>
__device__ __forceinline__ void mblock_partials(double v, double *partials)
{
    __shared__ double red[MB_NT];
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x < N) {
        double s = 0.0;
        for (int t = threadIdx.x; t < MB_NT; t += N) s += red[t];
        partials[(size_t)blockIdx.x * N + threadIdx.x] = s;
    }
}

// PS = RS + beta PS (active RHS) ; partial |PS|^2 per RHS (the first half of the next <p, A p>)
template <int N>
__global__ __launch_bounds__(MB_NT) void k_mp_norm(float2 *__restrict__ ps, const float2 *__restrict__ rs,
                                                   long long npairs, double *partials, const MultiState *st)
{
    if (paused(st->flags)) return;
    const int r = threadIdx.x % N;
    const bool on = (st->active >> r) & 1u;
    const float bt = (float)st->beta[r];
    double acc = 0.0;
    if (on) {
        for (long long j = (long long)blockIdx.x * MB_NT + threadIdx.x; j < npairs; j += (long long)gridDim.x * MB_NT) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const long long i = j * 3 + c;
                float2 pv = ps[i], rv = rs[i];
                pv.x = fmaf(bt, pv.x, rv.x);
                pv.y = fmaf(bt, pv.y, rv.y);
                ntstore(pv, ps + i);
                acc = fma((double)pv.x, (double)pv.x, fma((double)pv.y, (double)pv.y, acc));
            }
        }
    }
    mblock_partials<N>(acc, partials);
}

// partial |V_r|^2 per RHS of an FP32 batched vector
template <int N>
__global__ __launch_bounds__(MB_NT) void k_mnorm32(const float2 *__restrict__ v, long long npairs, double *partials)
{
    double acc = 0.0;
    for (long long j = (long long)blockIdx.x * MB_NT + threadIdx.x; j < npairs; j += (long long)gridDim.x * MB_NT)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float2 a = v[j * 3 + c];
            acc = fma((double)a.x, (double)a.x, fma((double)a.y, (double)a.y, acc));
        }
    mblock_partials<N>(acc, partials);
}

// Reliable update of the RHS in relmask at the end of the captured iterations.
// Their inner iteration ran on past the trigger, so p = r_in + beta p_old was
// built from the iterated residual; the update replaces r_in by r_true and p by
// r_true + beta p_old, i.e. p += r_true - r_in.  Before the FP64 residual:
// X64 += XS, XS = 0, PS -= RS (and flags.reliable opens the update's gates).
template <int N>
__global__ __launch_bounds__(MB_NT) void k_mrel_pre(double2 *__restrict__ x, float2 *__restrict__ xs,
                                                   float2 *__restrict__ ps, const float2 *__restrict__ rs,
                                                   long long npairs, const MultiState *st)
{
    if (st->flags.done) return;
    const int r = threadIdx.x % N;
    if (!((st->relmask >> r) & 1u)) return;
    for (long long j = (long long)blockIdx.x * MB_NT + threadIdx.x; j < npairs; j += (long long)gridDim.x * MB_NT) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const long long i = j * 3 + c;
            const float2 v = xs[i], rv = rs[i];
            double2 a = x[i];
            a.x += (double)v.x;
            a.y += (double)v.y;
            x[i] = a;
            xs[i] = make_float2(0.f, 0.f);
            float2 pv = ps[i];
            pv.x -= rv.x;
            pv.y -= rv.y;
            ps[i] = pv;
        }
    }
}

// After the FP64 residual (RS = float(r_true) for the RHS in relmask): PS += RS
// for those, and the |p|^2 partials of every active RHS for the next <p, A p>.
template <int N>
__global__ __launch_bounds__(MB_NT) void k_mrel_post(float2 *__restrict__ ps, const float2 *__restrict__ rs,
                                                    long long npairs, double *partials, const MultiState *st)
{
    if (st->flags.done) return;
    const int r = threadIdx.x % N;
    const bool on = (st->active >> r) & 1u, upd = (st->relmask >> r) & 1u;
    double acc = 0.0;
    if (on) {
        for (long long j = (long long)blockIdx.x * MB_NT + threadIdx.x; j < npairs; j += (long long)gridDim.x * MB_NT) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const long long i = j * 3 + c;
                float2 pv = ps[i];
                if (upd) {
                    const float2 rv = rs[i];
                    pv.x += rv.x;
                    pv.y += rv.y;
                    ps[i] = pv;
                }
                acc = fma((double)pv.x, (double)pv.x, fma((double)pv.y, (double)pv.y, acc));
            }
        }
    }
    mblock_partials<N>(acc, partials);
}

__global__ void k_mrel_open(MultiState *st)
{
    if (threadIdx.x || blockIdx.x) return;
    st->flags.reliable = st->relmask != 0;
}

// X64 += XS ; XS = 0 for the RHS in `which_mask`
template <int N>
__global__ __launch_bounds__(MB_NT) void k_maccum(double2 *__restrict__ x, float2 *__restrict__ xs, long long npairs,
                                                  const MultiState *st, int which_mask, int gate)
{
    if (gate_closed(&st->flags, gate)) return;
    const int r = threadIdx.x % N;
    if (!((pick_mask(st, which_mask) >> r) & 1u)) return;
    for (long long j = (long long)blockIdx.x * MB_NT + threadIdx.x; j < npairs; j += (long long)gridDim.x * MB_NT) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const long long i = j * 3 + c;
            float2 v = xs[i];
            double2 a = x[i];
            a.x += (double)v.x;
            a.y += (double)v.y;
            x[i] = a;
            xs[i] = make_float2(0.f, 0.f);
        }
    }
}

// partial |V_r|^2 per RHS of an FP64 batched vector
template <int N>
__global__ __launch_bounds__(MB_NT) void k_mnorm(const double2 *__restrict__ v, long long npairs, double *partials)
{
    double acc = 0.0;
    for (long long j = (long long)blockIdx.x * MB_NT + threadIdx.x; j < npairs; j += (long long)gridDim.x * MB_NT)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double2 a = v[j * 3 + c];
            acc = fma(a.x, a.x, fma(a.y, a.y, acc));
        }
    mblock_partials<N>(acc, partials);
}

// ------------------------------------------------------------------ shifted CG (FP32)
// base system (A0 + sigma0) on single vectors p, r, ap, t; shifted solutions
// and directions x_i, p_i batched [Vh][N][3].
template <class PS>
__global__ __launch_bounds__(256) HISQ_WAVES(8) void k_ms_ap(Geom g, const char *__restrict__ fat,
                                                          const char *__restrict__ lng,
                                                          const float2 *__restrict__ t, const float2 *__restrict__ p,
                                                          float2 *__restrict__ ap, int nblocks, double *partials,
                                                          const MultiState *st)
{
    if (st->flags.done) return;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    if (blk >= nblocks) return;
    const int tile = blk * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int h = tile * TILE + lane;
    double s = 0.0;
    if (tile < g.ntiles) {
        const int hc = h < g.Vh ? h : g.Vh - 1;
        float acc[6];
        dslash_site<PS>(g, fat, lng, t, 0, tile, lane, hc, acc);
        if (h < g.Vh) {
            const float m = (float)st->sigma0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float2 pv = p[(size_t)h * 3 + c], v;
                v.x = fmaf(m, pv.x, -acc[2 * c]);
                v.y = fmaf(m, pv.y, -acc[2 * c + 1]);
                ap[(size_t)h * 3 + c] = v;
                s = fma((double)pv.x, (double)v.x, fma((double)pv.y, (double)v.y, s));
            }
        }
    }
    block_partial<256>(s, partials, blk);
}

// r -= alpha ap ; partial |r|^2   (single vectors, n complex entries)
__global__ __launch_bounds__(MB_NT) void k_ms_r(float2 *__restrict__ r, const float2 *__restrict__ ap, long long n,
                                                double *partials, const MultiState *st)
{
    if (st->flags.done) return;
    const float a = (float)st->alpha0;
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * MB_NT + threadIdx.x; i < n; i += (long long)gridDim.x * MB_NT) {
        float2 rv = r[i], av = ap[i];
        rv.x = fmaf(-a, av.x, rv.x);
        rv.y = fmaf(-a, av.y, rv.y);
        r[i] = rv;
        acc = fma((double)rv.x, (double)rv.x, fma((double)rv.y, (double)rv.y, acc));
    }
    block_partial<MB_NT>(acc, partials, blockIdx.x);
}

// x_i += alpha_i p_i (active shifts)
template <int N>
__global__ __launch_bounds__(MB_NT) void k_ms_x(float2 *__restrict__ xs, const float2 *__restrict__ ps,
                                                long long npairs, const MultiState *st)
{
    if (st->flags.done) return;
    const int r = threadIdx.x % N;
    if (!((st->active >> r) & 1u)) return;
    const float a = (float)st->alpha_s[r];
    for (long long j = (long long)blockIdx.x * MB_NT + threadIdx.x; j < npairs; j += (long long)gridDim.x * MB_NT) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const long long i = j * 3 + c;
            float2 xv = xs[i], pv = ps[i];
            xv.x = fmaf(a, pv.x, xv.x);
            xv.y = fmaf(a, pv.y, xv.y);
            xs[i] = xv;
        }
    }
}

// p_i = zeta_i r + beta_i p_i (active shifts) ; p = r + beta p
template <int N>
__global__ __launch_bounds__(MB_NT) void k_ms_p(float2 *__restrict__ ps, float2 *__restrict__ p,
                                                const float2 *__restrict__ rv_, long long npairs, const MultiState *st)
{
    if (st->flags.done) return;
    const int r = threadIdx.x % N;
    const bool on = (st->active >> r) & 1u;
    const float z = (float)st->zeta[r], bt = (float)st->beta_s[r], b0 = (float)st->beta0;
    for (long long j = (long long)blockIdx.x * MB_NT + threadIdx.x; j < npairs; j += (long long)gridDim.x * MB_NT) {
        const long long site = j / N;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float2 rv = rv_[site * 3 + c];
            if (on) {
                const long long i = j * 3 + c;
                float2 pv = ps[i];
                pv.x = fmaf(bt, pv.x, z * rv.x);
                pv.y = fmaf(bt, pv.y, z * rv.y);
                ps[i] = pv;
            }
            if (r == 0) {
                float2 q = p[site * 3 + c];
                q.x = fmaf(b0, q.x, rv.x);
                q.y = fmaf(b0, q.y, rv.y);
                p[site * 3 + c] = q;
            }
        }
    }
}

enum { FS_BB = 0, FS_PAP = 1, FS_UPD = 2 };

__global__ __launch_bounds__(FIN_NT_M) void k_msfinalize(const double *__restrict__ partials, int nb, MultiState *st,
                                                         int mode)
{
    if (st->flags.done && mode != FS_BB) return;
    __shared__ double lds[FIN_NT_M / 64];
    double acc[1] = { 0.0 };
    strided_sums<FIN_NT_M, 1, 8>(partials, nb, acc);
    const double v = block_sum<FIN_NT_M>(acc[0], lds);
    if (threadIdx.x) return;
    const int n = st->n;
    switch (mode) {
    case FS_BB:
        st->bb0 = v;
        st->rr0 = v;
        st->stop0 = st->tol2 * v;
        for (int i = 0; i < n; ++i) st->rr_s[i] = v;
        break;
    case FS_PAP: {
        if (!(v > 0.0) || !isfinite(v)) {
            st->ms_status = HISQ_EBREAKDOWN;
            st->flags.done = 1;
            break;
        }
        const double al = st->rr0 / v;
        st->alpha0 = al;
        for (int i = 0; i < n; ++i) {
            if (!(st->active & (1u << i))) continue;
            const double z = st->zeta[i], zp = st->zeta_prev[i];
            const double den = zp * st->a_prev * (1.0 + al * st->dsig[i]) + al * st->b_prev * (zp - z);
            const double zn = z * zp * st->a_prev / den;
            st->zeta_next[i] = zn;
            st->alpha_s[i] = al * zn / z;
        }
        break;
    }
    case FS_UPD: {
        st->iter += 1;
        if (!isfinite(v)) {
            st->ms_status = HISQ_EBREAKDOWN;
            st->flags.done = 1;
            break;
        }
        const double be = v / st->rr0;
        st->beta0 = be;
        for (int i = 0; i < n; ++i) {
            if (!(st->active & (1u << i))) continue;
            st->iters[i] += 1;
            const double q = st->zeta_next[i] / st->zeta[i];
            st->beta_s[i] = be * q * q;
            st->zeta_prev[i] = st->zeta[i];
            st->zeta[i] = st->zeta_next[i];
            st->rr_s[i] = st->zeta[i] * st->zeta[i] * v;
            if (st->rr_s[i] <= st->stop0) st->active &= ~(1u << i);
        }
        st->a_prev = st->alpha0;
        st->b_prev = be;
        st->rr0 = v;
        if (!st->active) st->flags.done = 1;
        break;
    }
    }
}

__global__ void k_ms_init(MultiState *st, int n, double tol2, double sigma0, const double *dsig)
{
    if (threadIdx.x || blockIdx.x) return;
    st->flags.done = 0;
    st->flags.reliable = 0;
    st->n = n;
    st->active = (1u << n) - 1u;
    st->relmask = 0;
    st->iter = 0;
    st->tol2 = tol2;
    st->sigma0 = sigma0;
    st->a_prev = 1.0;
    st->b_prev = 0.0;
    st->ms_status = HISQ_OK;
    for (int i = 0; i < MAXR; ++i) {
        st->dsig[i] = i < n ? dsig[i] : 0.0;
        st->zeta[i] = st->zeta_prev[i] = st->zeta_next[i] = 1.0;
        st->alpha_s[i] = st->beta_s[i] = 0.0;
        st->rr_s[i] = 0.0;
        st->iters[i] = 0;
    }
}

// r = p = float(b), p_i = float(b) for all shifts, x_i = 0
template <int N>
__global__ __launch_bounds__(MB_NT) void k_ms_start(const double2 *__restrict__ b, float2 *__restrict__ r,
                                                    float2 *__restrict__ p, float2 *__restrict__ ps,
                                                    float2 *__restrict__ xs, long long npairs)
{
    for (long long j = (long long)blockIdx.x * MB_NT + threadIdx.x; j < npairs; j += (long long)gridDim.x * MB_NT) {
        const long long site = j / N;
        const int rr = (int)(j % N);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double2 bv = b[site * 3 + c];
            const float2 f = make_float2((float)bv.x, (float)bv.y);
            ps[j * 3 + c] = f;
            xs[j * 3 + c] = make_float2(0.f, 0.f);
            if (rr == 0) {
                r[site * 3 + c] = f;
                p[site * 3 + c] = f;
            }
        }
    }
}

// boundary [n][Vh][3] complex128 <-> internal [Vh][N][3]; slots r >= n are zero
template <int N>
__global__ __launch_bounds__(MB_NT) void k_to_batched(const double2 *__restrict__ in, double2 *__restrict__ out,
                                                      long long vh, int n, int same_source)
{
    const long long tot = vh * N * 3;
    for (long long i = (long long)blockIdx.x * MB_NT + threadIdx.x; i < tot; i += (long long)gridDim.x * MB_NT) {
        const int c = (int)(i % 3);
        const int r = (int)((i / 3) % N);
        const long long h = i / (3 * N);
        out[i] = r < n ? in[(same_source ? 0 : (long long)r * vh * 3) + h * 3 + c] : make_double2(0.0, 0.0);
    }
}

template <int N>
__global__ __launch_bounds__(MB_NT) void k_from_batched(const double2 *__restrict__ in, double2 *__restrict__ out,
                                                        long long vh, int n)
{
    const long long tot = (long long)n * vh * 3;
    for (long long i = (long long)blockIdx.x * MB_NT + threadIdx.x; i < tot; i += (long long)gridDim.x * MB_NT) {
        const int c = (int)(i % 3);
        const long long h = (i / 3) % vh;
        const int r = (int)(i / (3 * vh));
        out[i] = in[(h * N + r) * 3 + c];
    }
}

// float(x) of a batched FP64 vector
__global__ __launch_bounds__(MB_NT) void k_to_float(const double2 *__restrict__ in, float2 *__restrict__ out,
                                                    long long n)
{
    for (long long i = (long long)blockIdx.x * MB_NT + threadIdx.x; i < n; i += (long long)gridDim.x * MB_NT)
        out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

__global__ __launch_bounds__(MB_NT) void k_to_double(const float2 *__restrict__ in, double2 *__restrict__ out,
                                                     long long n)
{
    for (long long i = (long long)blockIdx.x * MB_NT + threadIdx.x; i < n; i += (long long)gridDim.x * MB_NT)
        out[i] = make_double2((double)in[i].x, (double)in[i].y);
}

// Column list of a batch compaction: new column c takes old column col[c]
// (c < n); columns n..N2-1 of the new batch are zero.
struct Cols {
    int col[MAXR];
    int n;
};

// dst [Vh][N2][3] <- the listed columns of src [Vh][N][3]
template <class T, int N, int N2>
__global__ __launch_bounds__(MB_NT) void k_mcompact(const T *__restrict__ src, T *__restrict__ dst, long long vh,
                                                    Cols cols)
{
    const long long tot = vh * N2 * 3;
    for (long long i = (long long)blockIdx.x * MB_NT + threadIdx.x; i < tot; i += (long long)gridDim.x * MB_NT) {
        const int k = (int)(i % 3);
        const int c = (int)((i / 3) % N2);
        const long long h = i / (3 * N2);
        T v;
        v.x = 0;
        v.y = 0;
        if (c < cols.n) v = src[(h * N + cols.col[c]) * 3 + k];
        dst[i] = v;
    }
}

// out [Vh][3] <- column `col` of x [Vh][N][3]
template <int N>
__global__ __launch_bounds__(MB_NT) void k_mcolumn(const double2 *__restrict__ x, double2 *__restrict__ out,
                                                   long long vh, int col)
{
    const long long tot = vh * 3;
    for (long long i = (long long)blockIdx.x * MB_NT + threadIdx.x; i < tot; i += (long long)gridDim.x * MB_NT)
        out[i] = x[((i / 3) * N + col) * 3 + (i % 3)];
}

// ------------------------------------------------------------------ finalisers
enum {
    FM_BB = 0,        // bb_r, stop2_r
    FM_INIT = 1,      // rr = rr_true = maxrr ; active = rr > stop2
    FM_PAP = 2,       // alpha_r or breakdown
    FM_UPD = 3,       // rr_new: reliable trigger or beta
    FM_RELIABLE = 4,  // true residual of the updated RHS
    FM_FINAL = 5,     // rr_true of every RHS (final check)
};

__device__ void mfinalize(MultiState *st, int mode, const double *v)
{
    const int n = st->n;
    switch (mode) {
    case FM_BB:
        for (int r = 0; r < n; ++r) { st->bb[r] = v[r]; st->stop2[r] = st->tol2 * v[r]; }
        break;
    case FM_INIT: {
        unsigned act = 0;
        for (int r = 0; r < n; ++r) {
            st->rr[r] = st->rr_true[r] = st->maxrr[r] = v[r];
            if (st->bb[r] > 0.0 && v[r] > st->stop2[r]) act |= 1u << r;
        }
        st->active = act;
        st->relmask = 0;
        st->flags.reliable = 0;
        st->flags.done = act == 0;
        break;
    }
    case FM_PAP:
        for (int r = 0; r < n; ++r) {
            if (!(st->active & (1u << r))) continue;
            if (!(v[r] > 0.0) || !isfinite(v[r])) {
                st->status[r] = HISQ_EBREAKDOWN;
                st->active &= ~(1u << r);
                st->alpha[r] = 0.0;
            } else {
                st->alpha[r] = st->rr[r] / v[r];
            }
        }
        if (!st->active) st->flags.done = 1;
        break;
    case FM_UPD:
        st->iter += 1;
        for (int r = 0; r < n; ++r) {
            if (!(st->active & (1u << r))) continue;
            st->iters[r] += 1;
            const double x = v[r];
            if (!isfinite(x)) {
                st->status[r] = HISQ_EBREAKDOWN;
                st->active &= ~(1u << r);
            } else {
                // a reliable update is due: flag it for the end of the captured
                // iterations and keep iterating (the batch is not paused)
                if (x <= st->stop2[r] || x < st->delta2 * st->maxrr[r]) st->relmask |= 1u << r;
                st->maxrr[r] = fmax(st->maxrr[r], x);
                st->beta[r] = x / st->rr[r];
                st->rr[r] = x;
            }
        }
        if (!st->active) st->flags.done = 1;
        break;
    case FM_RELIABLE:
        for (int r = 0; r < n; ++r) {
            if (!(st->relmask & (1u << r))) continue;
            const double x = v[r];
            st->rr_true[r] = x;
            st->nupd[r] += 1;
            st->beta[r] = x / st->rr[r];
            st->rr[r] = x;
            st->maxrr[r] = x;
            if (!isfinite(x)) {
                st->status[r] = HISQ_EBREAKDOWN;
                st->active &= ~(1u << r);
            } else if (x <= st->stop2[r]) {
                st->status[r] = HISQ_OK;
                st->active &= ~(1u << r);
            }
        }
        st->relmask = 0;
        st->flags.reliable = 0;
        if (!st->active) st->flags.done = 1;
        break;
    case FM_FINAL:
        for (int r = 0; r < n; ++r) st->rr_true[r] = v[r];
        break;
    }
}

// Column sums of red[FIN_NT_M][N] into tot[N]: wave w takes columns w, w + 4,
// ..., each lane adds 4 rows and a butterfly finishes (fixed order).
template <int N>
__device__ __forceinline__ void column_sums(const double *red, double *tot)
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int r = w; r < N; r += FIN_NT_M / 64) {
        double v = 0.0;
        for (int t = l; t < FIN_NT_M; t += 64) v += red[t * N + r];
        v = wave_sum(v);
        if (l == 0) tot[r] = v;
    }
}

// Rows of partials [nblocks][N] a finaliser thread loads before adding any:
// 16 loads in flight per thread whatever N is.
template <int N> constexpr int fin_rows() { return N >= 16 ? 1 : 16 / N; }

// One pass over the [nblocks][N] partials: thread i keeps the N sums of
// blocks i, i + 256, ... in registers, then the 256 x N sums are added
// column by column.
template <int N>
__global__ __launch_bounds__(FIN_NT_M) void k_mfinalize(const double *__restrict__ partials, int nblocks,
                                                        MultiState *st, int mode, int gate)
{
    if (solver_gate_closed(&st->flags, gate)) return;  // first: paused iterations stay cheap
    __shared__ double red[FIN_NT_M * N];
    __shared__ double tot[N];
    double acc[N];
#pragma unroll
    for (int r = 0; r < N; ++r) acc[r] = 0.0;
    strided_sums<FIN_NT_M, N, fin_rows<N>()>(partials, nblocks, acc);
#pragma unroll
    for (int r = 0; r < N; ++r) red[threadIdx.x * N + r] = acc[r];
    __syncthreads();
    column_sums<N>(red, tot);
    __syncthreads();
    if (threadIdx.x == 0) mfinalize(st, mode, tot);
}

// <p_r, A p_r> = m4_r |p_r|^2 + |D_oe p_r|^2 (D_eo = -D_oe^dag) from the partials of
// k_mp_norm / k_mnorm32 ([npp][N]) and of the EPI_STORE_NORM Dslash ([ntt][N]), then FM_PAP.
template <int N>
__global__ __launch_bounds__(FIN_NT_M) void k_mfinalize_pap(const double *__restrict__ part_t, int ntt,
                                                            const double *__restrict__ part_p, int npp, MultiState *st)
{
    if (paused(st->flags)) return;
    __shared__ double red[FIN_NT_M * N];
    __shared__ double tot[N];
    double acc[N];
#pragma unroll
    for (int r = 0; r < N; ++r) acc[r] = 0.0;
    strided_sums<FIN_NT_M, N, fin_rows<N>()>(part_t, ntt, acc);
    double accp[N];
#pragma unroll
    for (int r = 0; r < N; ++r) accp[r] = 0.0;
    strided_sums<FIN_NT_M, N, fin_rows<N>()>(part_p, npp, accp);
    __shared__ double tt[N];
#pragma unroll
    for (int r = 0; r < N; ++r) red[threadIdx.x * N + r] = acc[r];
    __syncthreads();
    column_sums<N>(red, tt);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < N; ++r) red[threadIdx.x * N + r] = accp[r];
    __syncthreads();
    column_sums<N>(red, tot);
    __syncthreads();
    if (threadIdx.x < N) tot[threadIdx.x] = fma(st->m4[threadIdx.x], tot[threadIdx.x], tt[threadIdx.x]);
    __syncthreads();
    if (threadIdx.x == 0) mfinalize(st, FM_PAP, tot);
}

__global__ void k_mstate_init(MultiState *st, int n, double tol2, double delta2, const double *m4)
{
    if (threadIdx.x || blockIdx.x) return;
    st->flags.done = 0;
    st->flags.reliable = 0;
    st->n = n;
    st->active = 0;
    st->relmask = 0;
    st->iter = 0;
    st->tol2 = tol2;
    st->delta2 = delta2;
    for (int r = 0; r < MAXR; ++r) {
        st->iters[r] = st->nupd[r] = 0;
        st->status[r] = HISQ_ENOCONV;
        st->m4[r] = r < n ? m4[r] : 0.0;
        st->alpha[r] = st->beta[r] = 0.0;
    }
}

// n right-hand sides, all active (standalone multi-RHS Dslash and its tuner)
__global__ void k_mstate_all(MultiState *st, int n)
{
    if (threadIdx.x || blockIdx.x) return;
    st->flags.done = 0;
    st->flags.reliable = 0;
    st->n = n;
    st->active = (1u << n) - 1u;
    st->relmask = 0;
}

// every still-active RHS gets a reliable update (used when max_iter is hit)
__global__ void k_mforce_reliable(MultiState *st)
{
    if (threadIdx.x || blockIdx.x) return;
    st->relmask = st->active;
    st->flags.reliable = st->relmask != 0;
    st->flags.done = 0;
}

// ------------------------------------------------------------------ host side
static int device_cus()
{
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }
constexpr size_t MSKEW = 4352;

// Launch shapes of the multi-RHS Dslash: RHS per thread G (as a divisor of N),
// threads per block, whether the next direction's loads are issued ahead
// (FP32 links; elsewhere the pipelined shapes run the plain loop), and the
// tile order (apply_order codes: 1 the default (z, t) blocks, 3 and 4 blocks
// of 4 and 2 t-planes by the whole z extent, 5 of 8 x 16), which decides how
// often the N x 24-byte neighbour blocks are fetched again (~9 times per
// launch at N = 16 in plain order).  Chosen per (lattice, N) by
// hisq_tune_multi.
struct MShape {
    int gdiv;  // G = N / gdiv
    int nt;
    int pipe;
    int order;
};
constexpr int N_MSHAPES = 16;
static const MShape MSHAPES[N_MSHAPES] = { { 1, 256, 0, 0 }, { 2, 256, 0, 0 }, { 4, 256, 0, 0 }, { 1, 128, 0, 0 },
                                           { 4, 256, 1, 0 }, { 2, 256, 1, 0 }, { 1, 256, 0, 1 }, { 2, 256, 0, 1 },
                                           { 4, 256, 0, 1 }, { 4, 256, 1, 1 }, { 2, 256, 1, 1 }, { 4, 256, 1, 3 },
                                           { 2, 256, 1, 3 }, { 4, 256, 1, 4 }, { 2, 256, 1, 4 }, { 4, 256, 1, 5 } };

template <class PS> static int mshape_for(const Geom &g, int N) { return tuned_choice("mdslash", g, PS::prec, N, 0); }

// Link storage of the batched solvers: the outer FP64 links (reliable
// updates, true residuals) and the inner FP32 links, both full or both with
// two-row long links.
struct MultiLinks32 {
    using PH = PF64;
    using PS = PF32;
};
struct MultiLinks32C {
    using PH = PF64C;
    using PS = PF32C;
};
// 16-bit fixed-point inner links (full, or with two-row long links)
struct MultiLinks16 {
    using PH = PF64;
    using PS = PI16S;
};
struct MultiLinks16C {
    using PH = PF64C;
    using PS = PI16SC;
};

// Default reliable-update trigger for inner links PS: frequent updates for the
// 16-bit forms, whose inner operator is ~1e-5 away from A (at 0.1 their batch
// stalled at m = 0.002 on 32^4); FP32 keeps the customary 0.1.
template <class PS> constexpr double multi_default_delta()
{
    return (PS::prec == HISQ_I16S || PS::prec == HISQ_I16SC) ? 0.7 : 0.1;
}

template <class P, int N, int G, int NT, int EPI, bool PIPE = false>
static hipError_t launch_md(const Geom &g, const void *fat, const void *lng, const void *src, void *dst,
                            const void *x, const void *b, float2 *rs, int parity, double *part, const MultiState *st,
                            int which, int gate, hipStream_t s, int *nblk_out)
{
    constexpr int SPB = NT / (N / G);
    const int nunits = (g.Vh + SPB - 1) / SPB;
    static int occ = -1;
    if (occ < 0) {
        int o = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, (const void *)k_mdslash<P, N, G, NT, EPI, PIPE>, NT, 0) !=
                hipSuccess || o <= 0)
            o = 1;
        occ = o;
    }
    int grid = std::min(nunits, device_cus() * occ);
    grid = std::min(std::max((grid + NXCD - 1) / NXCD * NXCD, NXCD), MULTI_MAX_BLOCKS);
    using V = typename P::cvec;
    hipLaunchKernelGGL((k_mdslash<P, N, G, NT, EPI, PIPE>), dim3(grid), dim3(NT), 0, s, g, (const char *)fat,
                       (const char *)lng, (const V *)src, (V *)dst, (const V *)x, (const V *)b, rs, parity, nunits,
                       part, st, which, gate);
    if (nblk_out) *nblk_out = grid;
    return hipGetLastError();
}

// dispatch over the tuned shape (FP32 inner kernels) or a fixed one (FP64)
template <class P, int N, int EPI>
static hipError_t launch_md_shape(int shape, const Geom &g0, const void *fat, const void *lng, const void *src,
                                  void *dst, const void *x, const void *b, float2 *rs, int parity, double *part,
                                  const MultiState *st, int which, int gate, hipStream_t s, int *nblk)
{
    constexpr int G1 = N, G2 = N >= 2 ? N / 2 : 1, G4 = N >= 4 ? N / 4 : 1;
    Geom g = g0;
    if (shape >= 0 && shape < N_MSHAPES) apply_order(g, MSHAPES[shape].order);  // unchanged where it cannot
    switch (shape) {
    case 1: return launch_md<P, N, G2, 256, EPI>(g, fat, lng, src, dst, x, b, rs, parity, part, st, which, gate, s, nblk);
    case 2: return launch_md<P, N, G4, 256, EPI>(g, fat, lng, src, dst, x, b, rs, parity, part, st, which, gate, s, nblk);
    case 3: return launch_md<P, N, G1, 128, EPI>(g, fat, lng, src, dst, x, b, rs, parity, part, st, which, gate, s, nblk);
    case 4: return launch_md<P, N, G4, 256, EPI, true>(g, fat, lng, src, dst, x, b, rs, parity, part, st, which, gate, s,
                                                      nblk);
    case 5: case 10: case 12: case 14:
        return launch_md<P, N, G2, 256, EPI, true>(g, fat, lng, src, dst, x, b, rs, parity, part, st, which, gate, s, nblk);
    case 6: return launch_md<P, N, G1, 256, EPI>(g, fat, lng, src, dst, x, b, rs, parity, part, st, which, gate, s, nblk);
    case 7: return launch_md<P, N, G2, 256, EPI>(g, fat, lng, src, dst, x, b, rs, parity, part, st, which, gate, s, nblk);
    case 8: return launch_md<P, N, G4, 256, EPI>(g, fat, lng, src, dst, x, b, rs, parity, part, st, which, gate, s, nblk);
    case 9: case 11: case 13: case 15:
        return launch_md<P, N, G4, 256, EPI, true>(g, fat, lng, src, dst, x, b, rs, parity, part, st, which, gate, s, nblk);
    default: return launch_md<P, N, G1, 256, EPI>(g, fat, lng, src, dst, x, b, rs, parity, part, st, which, gate, s, nblk);
    }
}

struct MultiBufs {
    MultiState *st;
    double *part;
    double *part_p;                     // partials of |p|^2, kept from one iteration to the next
    double2 *x64, *b64, *r64, *t64;     // [Vh][N][3] FP64
    float2 *xs, *rs, *ps, *ts;          // [Vh][N][3] FP32
    float2 *p1, *r1, *ap1, *t1;         // [Vh][3] FP32 (shifted CG base system)
    double *dm;                          // small device array: masses or shifts
};

// partials: per-RHS block sums of the batched kernels, or one per Dslash block of the shifted CG
static size_t multi_partials(const Geom &g, int N)
{
    return std::max((size_t)MULTI_MAX_BLOCKS * N, (size_t)((g.ntiles + 3) / 4)) + 64;
}

size_t cg_multi_ws_for(const Geom &g, int N)
{
    const size_t vp = (size_t)g.Vh * N * 3;
    size_t b = al256(sizeof(MultiState)) + 2 * al256(multi_partials(g, N) * sizeof(double)) +
               al256(64 * sizeof(double)) + 4 * MSKEW;
    b += 4 * (al256(vp * 16) + MSKEW) + 4 * (al256(vp * 8) + MSKEW) + 4 * (al256((size_t)g.Vh * 3 * 8) + MSKEW);
    return b + 4096;
}
static_assert(sizeof(MultiState) <= PIN_SLOT_BYTES, "MultiState does not fit its pinned slot");

static int pad_n(int n) { return n <= 1 ? 1 : n <= 2 ? 2 : n <= 4 ? 4 : n <= 8 ? 8 : 16; }

size_t cg_multi_workspace_bytes(const Geom &g, int nrhs, int mode)
{
    if (nrhs < 1 || nrhs > MAXR || (mode != HISQ_MULTI_RHS && mode != HISQ_MULTI_SHIFT)) return 0;
    return cg_multi_ws_for(g, pad_n(nrhs));
}

static bool carve(MultiBufs &B, void *ws, size_t bytes, const Geom &g, int N)
{
    char *p = (char *)ws;
    size_t left = bytes;
    auto take = [&](size_t n) -> void * {
        n = al256(n) + MSKEW;
        if (n > left) return nullptr;
        void *r = p;
        p += n;
        left -= n;
        return r;
    };
    const size_t vp = (size_t)g.Vh * N * 3, v1 = (size_t)g.Vh * 3;
    B.st = (MultiState *)take(sizeof(MultiState));
    B.part = (double *)take(multi_partials(g, N) * sizeof(double));
    B.part_p = (double *)take(multi_partials(g, N) * sizeof(double));
    B.dm = (double *)take(64 * sizeof(double));
    B.x64 = (double2 *)take(vp * 16);
    B.b64 = (double2 *)take(vp * 16);
    B.r64 = (double2 *)take(vp * 16);
    B.t64 = (double2 *)take(vp * 16);
    B.xs = (float2 *)take(vp * 8);
    B.rs = (float2 *)take(vp * 8);
    B.ps = (float2 *)take(vp * 8);
    B.ts = (float2 *)take(vp * 8);
    B.p1 = (float2 *)take(v1 * 8);
    B.r1 = (float2 *)take(v1 * 8);
    B.ap1 = (float2 *)take(v1 * 8);
    B.t1 = (float2 *)take(v1 * 8);
    return B.t1 != nullptr;
}

// run_multi returns MULTI_SHRINK (> 0) when at a state check no more than
// `shrink_at` right-hand sides are still iterating.
constexpr int MULTI_SHRINK = 1;

struct NoMultiPause {
    hipError_t operator()(hipStream_t) const { return hipSuccess; }
};

template <class F, class PauseFn = NoMultiPause>
static int run_multi(F iter_fn, hipStream_t s, MultiState *dst, MultiState *hst, int K, int max_iter, bool graph,
                     int shrink_at = -1, PauseFn pause_fn = PauseFn())
{
    hipGraphExec_t exec = nullptr;
    hipGraph_t gr = nullptr;
    if (graph) {
        hipStream_t cs = capture_stream();
        if (!cs) return fail(HISQ_EHIP, "cannot create capture stream");
        HISQ_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < K; ++k) {
            hipError_t e = iter_fn(cs);
            if (e != hipSuccess) {
                hipGraph_t junk = nullptr;
                hipStreamEndCapture(cs, &junk);
                if (junk) hipGraphDestroy(junk);
                return hip_fail(e, "batched CG iteration launch (capture)");
            }
        }
        HISQ_HIP(hipStreamEndCapture(cs, &gr));
        HISQ_HIP(hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0));
    }
    int queued = 0, rc = HISQ_OK;
    while (queued < max_iter) {
        const int k = std::min(K, max_iter - queued);
        if (graph && k == K) {
            hipError_t e = hipGraphLaunch(exec, s);
            if (e != hipSuccess) { rc = hip_fail(e, "hipGraphLaunch"); break; }
        } else {
            for (int i = 0; i < k && !rc; ++i) {
                hipError_t e = iter_fn(s);
                if (e != hipSuccess) rc = hip_fail(e, "batched CG iteration launch");
            }
            if (rc) break;
        }
        queued += k;
        hipError_t e = hipMemcpyAsync(hst, dst, sizeof(MultiState), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { rc = hip_fail(e, "batched CG state read-back"); break; }
        if (hst->flags.done) break;
        if (hst->flags.reliable || hst->relmask) {
            e = pause_fn(s);
            if (e != hipSuccess) { rc = hip_fail(e, "reliable update launch"); break; }
            e = hipMemcpyAsync(hst, dst, sizeof(MultiState), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) { rc = hip_fail(e, "batched CG state read-back"); break; }
            if (hst->flags.done) break;
        }
        if (shrink_at >= 0 && __builtin_popcount(hst->active) <= shrink_at) { rc = MULTI_SHRINK; break; }
    }
    if (exec) hipGraphExecDestroy(exec);
    if (gr) hipGraphDestroy(gr);
    return rc;
}

static int read_mstate(MultiState *h, const MultiState *d, hipStream_t s)
{
    HISQ_HIP(hipMemcpyAsync(h, d, sizeof(MultiState), hipMemcpyDeviceToHost, s));
    HISQ_HIP(hipStreamSynchronize(s));
    return HISQ_OK;
}

// Results of the right-hand sides as they leave the batch, by caller index.
struct MultiOut {
    double2 *x;        // caller's x [n][Vh][3]
    int orig[MAXR];    // batch column -> caller index
    int iters[MAXR], nupd[MAXR], status[MAXR];
    double rr_true[MAXR], bb[MAXR], rr[MAXR];
    double bytes;      // algorithmic bytes moved so far (the whole batched solve)
};

// Byte model of the batched iteration with N columns of inner links PS, per
// site: two Dslash link streams, then the vector streams of the three
// kernels (norm epilogue: p read, t written; update epilogue: t read, p
// read, x and r read and written; direction update: r read, p read and
// written), 11 FP32 vectors per column.
template <class PS> static double multi_iter_bytes(int N) { return 2 * link_bytes_site(PS::prec) + 11 * 24.0 * N; }
// One deferred reliable-update pass for k flagged columns: the two FP64
// Dslash link streams, then per column x64 read and written, x, p read and
// written, r read (k_mrel_pre), x64 read, t64 written, t64 read, x64 and b
// read, r64 and r written (the two Dslashes), p read and written, r read.
template <class PH> static double multi_rel_bytes(int k)
{
    return 2 * link_bytes_site(PH::prec) + k * (2 * 48.0 + 4 * 24.0 + 24 + 48 * 6 + 24 + 3 * 24);
}

// Batched reliable-update CG, set-up: R64 = B - A X64 for every RHS, RS =
// float(R64), PS = RS (B.b64 and B.x64 [Vh][N][3] FP64 on entry).
template <class M, int N>
static int multi_rhs_init(int n, const double *masses, double tol, const void *fat, const void *lng, const Geom &g,
                          const hisq_cg_opts &o, MultiBufs &B, MultiState *hs, hipStream_t s)
{
    const long long np = (long long)g.Vh * N;
    const int nbm = mblocks(np);
    const double delta = o.delta > 0 ? o.delta : multi_default_delta<typename M::PS>();
    double m4[MAXR];
    for (int r = 0; r < n; ++r) m4[r] = 4.0 * masses[r] * masses[r];
    HISQ_HIP(hipMemcpyAsync(B.dm, m4, n * sizeof(double), hipMemcpyHostToDevice, s));
    HISQ_HIP(hipMemsetAsync(B.xs, 0, (size_t)np * 3 * 8, s));
    hipLaunchKernelGGL(k_mstate_init, dim3(1), dim3(1), 0, s, B.st, n, tol * tol, delta * delta, (const double *)B.dm);
    hipLaunchKernelGGL((k_mnorm<N>), dim3(nbm), dim3(MB_NT), 0, s, (const double2 *)B.b64, np, B.part);
    hipLaunchKernelGGL((k_mfinalize<N>), dim3(1), dim3(FIN_NT_M), 0, s, (const double *)B.part, nbm, B.st, (int)FM_BB,
                       (int)GATE_ALWAYS);
    int nb = 0;
    HISQ_HIP((launch_md_shape<typename M::PH, N, EPI_STORE>(0, g, fat, lng, B.x64, B.t64, nullptr, nullptr, nullptr, 1, B.part,
                                                  B.st, MASK_ALL, GATE_ALWAYS, s, &nb)));
    HISQ_HIP((launch_md_shape<typename M::PH, N, EPI_RESID>(0, g, fat, lng, B.t64, B.r64, B.x64, B.b64, B.rs, 0, B.part, B.st,
                                                  MASK_ALL, GATE_ALWAYS, s, &nb)));
    hipLaunchKernelGGL((k_mfinalize<N>), dim3(1), dim3(FIN_NT_M), 0, s, (const double *)B.part, nb, B.st, (int)FM_INIT,
                       (int)GATE_ALWAYS);
    HISQ_HIP(hipMemcpyAsync(B.ps, B.rs, (size_t)np * 3 * 8, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL((k_mnorm32<N>), dim3(nbm), dim3(MB_NT), 0, s, (const float2 *)B.ps, np, B.part_p);
    HISQ_HIP(hipGetLastError());
    return read_mstate(hs, B.st, s);
}

template <class M, int N>
static int multi_rhs_run(const void *fat, const void *lng, const void *fat_lo, const void *lng_lo, const Geom &g,
                         const hisq_cg_opts &o, MultiBufs &B, MultiState *hs, hipStream_t s, int iter_offset,
                         MultiOut &out);

// Launch shape of the batched iteration's two Dslash launches on this
// lattice and inner link storage: the one chosen before, or chosen now by
// timing the pair (norm epilogue, update epilogue) for every shape.  The
// update epilogue holds more registers per RHS than the plain Dslash, so the
// plain-Dslash choice of hisq_tune_multi is not reused.  The timing runs on
// scratch: a state with every RHS active in p1 (the shifted CG's base-system
// vectors are free here), x and r of the update in t64, partials in part;
// p is only read and ts holds nothing live before the iteration starts.
template <class PS, int N>
static int md_shape_or_tune(const Geom &g, const void *fat_lo, const void *lng_lo, MultiBufs &B, hipStream_t s)
{
    int shape = tuned_choice("mdslash_cg", g, PS::prec, N, -1);
    if (shape >= 0) return shape;
    if ((size_t)g.Vh * 3 * 8 < sizeof(MultiState)) return 0;
    MultiState *tst = (MultiState *)B.p1;
    float2 *xs_t = (float2 *)B.t64, *rs_t = xs_t + (size_t)g.Vh * N * 3;
    if (hipMemsetAsync(tst, 0, sizeof(MultiState), s) != hipSuccess) return 0;
    hipLaunchKernelGGL(k_mstate_all, dim3(1), dim3(1), 0, s, tst, N);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return 0;
    if (hipEventCreate(&e1) != hipSuccess) { hipEventDestroy(e0); return 0; }
    double best_us = 1e300;
    int best_i = 0;
    bool ok = true;
    for (int i = 0; i < N_MSHAPES && ok; ++i) {
        if (N % MSHAPES[i].gdiv) continue;
        auto go = [&]() {
            return launch_md_shape<PS, N, EPI_STORE_NORM>(i, g, fat_lo, lng_lo, B.ps, B.ts, nullptr, nullptr,
                                                          nullptr, 1, B.part, tst, MASK_ACTIVE, GATE_ALWAYS, s,
                                                          nullptr) == hipSuccess &&
                   launch_md_shape<PS, N, EPI_UPD>(i, g, fat_lo, lng_lo, B.ts, xs_t, B.ps, nullptr, rs_t, 0, B.part,
                                                   tst, MASK_ACTIVE, GATE_ALWAYS, s, nullptr) == hipSuccess;
        };
        constexpr int reps = 5;
        for (int w = 0; w < 2; ++w) ok = ok && go();
        ok = ok && hipEventRecord(e0, s) == hipSuccess;
        for (int k = 0; k < reps; ++k) ok = ok && go();
        ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0;
        ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        if (ok && ms / reps < best_us) { best_us = ms / reps; best_i = i; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (!ok) return 0;
    set_tuned_choice("mdslash_cg", g, PS::prec, N, best_i);
    return best_i;
}

// column c of the batch leaves: its FP64 solution goes to the caller's x
template <int N>
static void retire(MultiBufs &B, const MultiState *hs, const Geom &g, int c, MultiOut &out, hipStream_t s)
{
    const int r = out.orig[c];
    hipLaunchKernelGGL((k_mcolumn<N>), dim3(mblocks((long long)g.Vh)), dim3(MB_NT), 0, s, (const double2 *)B.x64,
                       out.x + (size_t)r * g.Vh * 3, (long long)g.Vh, c);
    out.iters[r] = hs->iters[c];
    out.nupd[r] = hs->nupd[c];
    out.status[r] = hs->status[c];
    out.rr_true[r] = hs->rr_true[c];
    out.bb[r] = hs->bb[c];
    out.rr[r] = hs->rr[c];
}

// The batch shrinks to the next power of two that holds the right-hand
// sides still iterating: finished columns leave, the live ones are packed
// into [Vh][N2][3] in the same buffers (through the scratch vectors t64 and
// ts), their per-RHS state moves with them, and the iteration continues
// with the N2 kernels.  Nothing restarts: x, r, p and every scalar are kept.
template <class M, int N, int N2>
static int shrink_to(const void *fat, const void *lng, const void *fat_lo, const void *lng_lo, const Geom &g,
                     const hisq_cg_opts &o, MultiBufs &B, MultiState *hs, hipStream_t s, int iter_offset,
                     MultiOut &out, const Cols &live)
{
    const long long vh = g.Vh, np = vh * N, np2 = vh * N2;
    const int nbm = mblocks(np), nb2 = mblocks(np2);
    hipLaunchKernelGGL((k_mcompact<double2, N, N2>), dim3(nb2), dim3(MB_NT), 0, s, (const double2 *)B.x64, B.t64, vh,
                       live);
    HISQ_HIP(hipMemcpyAsync(B.x64, B.t64, (size_t)np2 * 48, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL((k_mcompact<double2, N, N2>), dim3(nb2), dim3(MB_NT), 0, s, (const double2 *)B.b64, B.t64, vh,
                       live);
    HISQ_HIP(hipMemcpyAsync(B.b64, B.t64, (size_t)np2 * 48, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL((k_mcompact<float2, N, N2>), dim3(nb2), dim3(MB_NT), 0, s, (const float2 *)B.rs, B.ts, vh, live);
    HISQ_HIP(hipMemcpyAsync(B.rs, B.ts, (size_t)np2 * 24, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL((k_mcompact<float2, N, N2>), dim3(nb2), dim3(MB_NT), 0, s, (const float2 *)B.ps, B.ts, vh, live);
    HISQ_HIP(hipMemcpyAsync(B.ps, B.ts, (size_t)np2 * 24, hipMemcpyDeviceToDevice, s));
    HISQ_HIP(hipMemsetAsync(B.xs, 0, (size_t)np * 24, s));
    hipLaunchKernelGGL((k_mnorm32<N2>), dim3(nb2), dim3(MB_NT), 0, s, (const float2 *)B.ps, np2, B.part_p);
    HISQ_HIP(hipGetLastError());
    (void)nbm;
    // the state, compacted on the host
    MultiState ns = *hs;
    int orig2[MAXR];
    for (int c = 0; c < MAXR; ++c) {
        const bool on = c < live.n;
        const int k = on ? live.col[c] : 0;
        orig2[c] = on ? out.orig[k] : -1;
        ns.iters[c] = on ? hs->iters[k] : 0;
        ns.nupd[c] = on ? hs->nupd[k] : 0;
        ns.status[c] = on ? hs->status[k] : HISQ_OK;
        ns.m4[c] = on ? hs->m4[k] : 0.0;
        ns.bb[c] = on ? hs->bb[k] : 0.0;
        ns.stop2[c] = on ? hs->stop2[k] : 0.0;
        ns.rr[c] = on ? hs->rr[k] : 0.0;
        ns.rr_true[c] = on ? hs->rr_true[k] : 0.0;
        ns.maxrr[c] = on ? hs->maxrr[k] : 0.0;
        ns.alpha[c] = on ? hs->alpha[k] : 0.0;
        ns.beta[c] = on ? hs->beta[k] : 0.0;
    }
    ns.n = live.n;
    ns.active = (1u << live.n) - 1u;
    ns.relmask = 0;
    ns.flags.done = 0;
    ns.flags.reliable = 0;
    *hs = ns;
    std::memcpy(out.orig, orig2, sizeof(orig2));
    HISQ_HIP(hipMemcpyAsync(B.st, hs, sizeof(MultiState), hipMemcpyHostToDevice, s));
    HISQ_HIP(hipStreamSynchronize(s));
    return multi_rhs_run<M, N2>(fat, lng, fat_lo, lng_lo, g, o, B, hs, s, iter_offset, out);
}

// Batched reliable-update CG iterations from the state multi_rhs_init (or a
// shrink) left; every right-hand side ends in the caller's x and in `out`.
template <class M, int N>
static int multi_rhs_run(const void *fat, const void *lng, const void *fat_lo, const void *lng_lo, const Geom &g,
                         const hisq_cg_opts &o, MultiBufs &B, MultiState *hs, hipStream_t s, int iter_offset,
                         MultiOut &out)
{
    const long long np = (long long)g.Vh * N;
    const int nbm = mblocks(np);
    using PS = typename M::PS;
    const int shape = md_shape_or_tune<PS, N>(g, fat_lo, lng_lo, B, s);
    auto iter = [&](hipStream_t q) -> hipError_t {
        // t = D_oe p and |t|^2 ; alpha = rr / (m4 |p|^2 + |t|^2)
        int nb1 = 0;
        hipError_t e = launch_md_shape<PS, N, EPI_STORE_NORM>(shape, g, fat_lo, lng_lo, B.ps, B.ts, nullptr,
                                                                nullptr, nullptr, 1, B.part, B.st, MASK_ACTIVE,
                                                                GATE_PAUSE, q, &nb1);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_mfinalize_pap<N>), dim3(1), dim3(FIN_NT_M), 0, q, (const double *)B.part, nb1,
                           (const double *)B.part_p, nbm, B.st);
        // x += alpha p ; r -= alpha (m4 p - D_eo t) ; |r|^2
        e = launch_md_shape<PS, N, EPI_UPD>(shape, g, fat_lo, lng_lo, B.ts, B.xs, B.ps, nullptr, B.rs, 0, B.part,
                                              B.st, MASK_ACTIVE, GATE_PAUSE, q, &nb1);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_mfinalize<N>), dim3(1), dim3(FIN_NT_M), 0, q, (const double *)B.part, nb1, B.st,
                           (int)FM_UPD, (int)GATE_PAUSE);
        // p = r + beta p ; |p|^2 (a pending reliable update pauses the batch here)
        hipLaunchKernelGGL((k_mp_norm<N>), dim3(nbm), dim3(MB_NT), 0, q, B.ps, (const float2 *)B.rs, np, B.part_p,
                           (const MultiState *)B.st);
        return hipGetLastError();
    };
    // reliable updates of the RHS that asked for one during the last captured
    // iterations (they kept iterating; see k_mrel_pre), all at once
    auto reliable = [&](hipStream_t q) -> hipError_t {
        out.bytes += multi_rel_bytes<typename M::PH>(__builtin_popcount(hs->relmask)) * g.Vh;
        hipLaunchKernelGGL(k_mrel_open, dim3(1), dim3(1), 0, q, B.st);
        hipLaunchKernelGGL((k_mrel_pre<N>), dim3(nbm), dim3(MB_NT), 0, q, B.x64, B.xs, B.ps, (const float2 *)B.rs, np,
                           (const MultiState *)B.st);
        hipError_t e;
        int nb2 = 0;
        e = launch_md_shape<typename M::PH, N, EPI_STORE>(0, g, fat, lng, B.x64, B.t64, nullptr, nullptr, nullptr, 1, B.part,
                                                B.st, MASK_RELIABLE, GATE_RELIABLE, q, &nb2);
        if (e != hipSuccess) return e;
        e = launch_md_shape<typename M::PH, N, EPI_RESID>(0, g, fat, lng, B.t64, B.r64, B.x64, B.b64, B.rs, 0, B.part, B.st,
                                                MASK_RELIABLE, GATE_RELIABLE, q, &nb2);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_mrel_post<N>), dim3(nbm), dim3(MB_NT), 0, q, B.ps, (const float2 *)B.rs, np, B.part_p,
                           (const MultiState *)B.st);
        hipLaunchKernelGGL((k_mfinalize<N>), dim3(1), dim3(FIN_NT_M), 0, q, (const double *)B.part, nb2, B.st,
                           (int)FM_RELIABLE, (int)GATE_RELIABLE);
        return hipGetLastError();
    };
    int rc = HISQ_OK;
    if (!hs->flags.done) {
        const int budget = std::max(1, o.max_iter - iter_offset - hs->iter);
        const int it0 = hs->iter;
        rc = run_multi(iter, s, B.st, hs, o.check_every, budget, o.use_graph != 0, N > 1 ? N / 2 : -1, reliable);
        if (rc < 0) return rc;
        out.bytes += (double)(hs->iter - it0) * multi_iter_bytes<PS>(N) * g.Vh;
    }
    if constexpr (N > 1) {
        if (rc == MULTI_SHRINK) {
            // fold every inner solution (x64 += xs, xs = 0), let the finished columns leave
            hipLaunchKernelGGL(k_mforce_reliable, dim3(1), dim3(1), 0, s, B.st);
            hipLaunchKernelGGL((k_maccum<N>), dim3(nbm), dim3(MB_NT), 0, s, B.x64, B.xs, np, (const MultiState *)B.st,
                               (int)MASK_ALL, (int)GATE_ALWAYS);
            Cols live;
            live.n = 0;
            for (int c = 0; c < hs->n; ++c) {
                if ((hs->active >> c) & 1u) live.col[live.n++] = c;
                else retire<N>(B, hs, g, c, out, s);
            }
            HISQ_HIP(hipGetLastError());
            const int n2 = pad_n(live.n);
            if (n2 == 1) return shrink_to<M, N, 1>(fat, lng, fat_lo, lng_lo, g, o, B, hs, s, iter_offset, out, live);
            if constexpr (N > 2) if (n2 == 2) return shrink_to<M, N, 2>(fat, lng, fat_lo, lng_lo, g, o, B, hs, s, iter_offset, out, live);
            if constexpr (N > 4) if (n2 == 4) return shrink_to<M, N, 4>(fat, lng, fat_lo, lng_lo, g, o, B, hs, s, iter_offset, out, live);
            if constexpr (N > 8) if (n2 == 8) return shrink_to<M, N, 8>(fat, lng, fat_lo, lng_lo, g, o, B, hs, s, iter_offset, out, live);
            return fail(HISQ_EINVAL, "cg_solve_multi: internal batch size error");
        }
    }
    // fold the inner solutions of RHS still running and measure every true residual
    hipLaunchKernelGGL(k_mforce_reliable, dim3(1), dim3(1), 0, s, B.st);
    hipLaunchKernelGGL((k_maccum<N>), dim3(nbm), dim3(MB_NT), 0, s, B.x64, B.xs, np, (const MultiState *)B.st,
                       (int)MASK_ALL, (int)GATE_ALWAYS);
    int nb = 0;
    HISQ_HIP((launch_md_shape<typename M::PH, N, EPI_STORE>(0, g, fat, lng, B.x64, B.t64, nullptr, nullptr, nullptr, 1, B.part,
                                                  B.st, MASK_ALL, GATE_ALWAYS, s, &nb)));
    HISQ_HIP((launch_md_shape<typename M::PH, N, EPI_RESID>(0, g, fat, lng, B.t64, B.r64, B.x64, B.b64, B.rs, 0, B.part, B.st,
                                                  MASK_ALL, GATE_ALWAYS, s, &nb)));
    hipLaunchKernelGGL((k_mfinalize<N>), dim3(1), dim3(FIN_NT_M), 0, s, (const double *)B.part, nb, B.st, (int)FM_FINAL,
                       (int)GATE_ALWAYS);
    HISQ_HIP(hipGetLastError());
    out.bytes += multi_rel_bytes<typename M::PH>(N) * g.Vh;
    rc = read_mstate(hs, B.st, s);
    if (rc) return rc;
    for (int c = 0; c < hs->n; ++c) retire<N>(B, hs, g, c, out, s);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

// Shifted CG for one source and n shifts in FP32 (stage 1 of MULTI_SHIFT);
// leaves the shifted solutions in B.xs.
template <class M, int N>
static int multi_shift_core(int n, const double *masses, double tol_ms, const void *fat_lo, const void *lng_lo,
                            const void *b, const Geom &g, const hisq_cg_opts &o, MultiBufs &B, MultiState *hs,
                            hipStream_t s)
{
    const long long np = (long long)g.Vh * N, n1 = (long long)g.Vh * 3;
    const int nbm = mblocks(np), nb1 = mblocks(n1);
    const int nbd = (g.ntiles + 3) / 4;
    double sig0 = 1e300;
    for (int i = 0; i < n; ++i) sig0 = std::min(sig0, 4.0 * masses[i] * masses[i]);
    double ds[MAXR];
    for (int i = 0; i < n; ++i) ds[i] = 4.0 * masses[i] * masses[i] - sig0;
    HISQ_HIP(hipMemcpyAsync(B.dm, ds, n * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ms_init, dim3(1), dim3(1), 0, s, B.st, n, tol_ms * tol_ms, sig0, (const double *)B.dm);
    hipLaunchKernelGGL((k_ms_start<N>), dim3(nbm), dim3(MB_NT), 0, s, (const double2 *)b, B.r1, B.p1, B.ps, B.xs, np);
    // |b|^2 from the FP64 source
    hipLaunchKernelGGL((k_mnorm<1>), dim3(nb1), dim3(MB_NT), 0, s, (const double2 *)b, (long long)g.Vh, B.part);
    hipLaunchKernelGGL(k_msfinalize, dim3(1), dim3(FIN_NT_M), 0, s, (const double *)B.part, nb1, B.st, (int)FS_BB);
    HISQ_HIP(hipGetLastError());
    int rc0 = read_mstate(hs, B.st, s);
    if (rc0) return rc0;
    if (hs->bb0 == 0.0) return HISQ_OK;  // zero source: every x_i = 0 (already in B.xs)
    auto iter = [&](hipStream_t q) -> hipError_t {
        hipError_t e = launch_dslash<typename M::PS>(g, fat_lo, lng_lo, B.p1, B.t1, 1, q, &B.st->flags, GATE_NOT_DONE);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_ms_ap<typename M::PS>, dim3(xcd_grid(nbd)), dim3(256), 0, q, g, (const char *)fat_lo,
                           (const char *)lng_lo, (const float2 *)B.t1, (const float2 *)B.p1, B.ap1, nbd, B.part,
                           (const MultiState *)B.st);
        hipLaunchKernelGGL(k_msfinalize, dim3(1), dim3(FIN_NT_M), 0, q, (const double *)B.part, nbd, B.st,
                           (int)FS_PAP);
        hipLaunchKernelGGL((k_ms_x<N>), dim3(nbm), dim3(MB_NT), 0, q, B.xs, (const float2 *)B.ps, np,
                           (const MultiState *)B.st);
        hipLaunchKernelGGL(k_ms_r, dim3(nb1), dim3(MB_NT), 0, q, B.r1, (const float2 *)B.ap1, n1, B.part,
                           (const MultiState *)B.st);
        hipLaunchKernelGGL(k_msfinalize, dim3(1), dim3(FIN_NT_M), 0, q, (const double *)B.part, nb1, B.st,
                           (int)FS_UPD);
        hipLaunchKernelGGL((k_ms_p<N>), dim3(nbm), dim3(MB_NT), 0, q, B.ps, B.p1, (const float2 *)B.r1, np,
                           (const MultiState *)B.st);
        return hipGetLastError();
    };
    int rc = run_multi(iter, s, B.st, hs, o.check_every, o.max_iter, o.use_graph != 0);
    if (rc) return rc;
    return hs->ms_status;
}

template <class M, int N>
static int cg_multi_impl(int n, const double *masses, double tol, int mode, const void *fat, const void *lng,
                         const void *fat_lo, const void *lng_lo, const void *b, void *x, const Geom &g,
                         const hisq_cg_opts &o, void *ws, size_t ws_bytes, hisq_cg_stats *stats, hipStream_t s)
{
    MultiBufs B;
    if (!carve(B, ws, ws_bytes, g, N)) return fail(HISQ_EWORKSPACE, "cg_solve_multi: workspace too small");
    MultiState *hs = (MultiState *)pinned_slot(PIN_MULTI);
    if (!hs) return fail(HISQ_EHIP, "cg_solve_multi: pinned state allocation failed");
    const long long np = (long long)g.Vh * N;
    const int nbm = mblocks(np);
    auto t0 = std::chrono::steady_clock::now();
    HISQ_HIP(hipMemsetAsync(B.st, 0, sizeof(MultiState), s));
    int ms_iters[MAXR] = { 0 };
    double ms_resid[MAXR] = { 0.0 };
    bool ms_conv[MAXR] = { false };
    int offset = 0;
    MultiOut out;
    std::memset(&out, 0, sizeof(out));
    out.x = (double2 *)x;
    for (int c = 0; c < MAXR; ++c) out.orig[c] = c < n ? c : -1;
    const bool shift_only = mode == HISQ_MULTI_SHIFT && o.shift_only;
    if (mode == HISQ_MULTI_SHIFT) {
        // The shifted phase has no reliable updates: its iterated residuals
        // drift from the true ones, and the refinement restarts the Krylov
        // space.  By default it stops at 1e-3: that cut the lightest of 8
        // masses at 32^4 from 19 854 to 19 238 total iterations (FP32 inner
        // links) and from 23 529 to 20 288 (16-bit inner links) against 1e-5.
        const double tol_ms = o.shift_tol > 0 ? o.shift_tol : std::max(tol, 1e-3);
        int rc = multi_shift_core<M, N>(n, masses, tol_ms, fat_lo, lng_lo, b, g, o, B, hs, s);
        if (rc) return fail(rc, "cg_solve_multi: shifted CG broke down");
        for (int i = 0; i < n; ++i) {
            ms_iters[i] = hs->iters[i];
            ms_resid[i] = hs->bb0 > 0 ? std::sqrt(hs->rr_s[i] / hs->bb0) : 0.0;
            ms_conv[i] = hs->bb0 == 0.0 || !((hs->active >> i) & 1u);
        }
        offset = hs->iter;
        // per iteration: two Dslash link streams; base vectors p, t (first
        // Dslash), t, p, A p (second), r, r, A p (residual update), r, p, p
        // (direction): 11; per shift x, x, p (solution) and p, p (direction)
        out.bytes += (double)hs->iter * (2 * link_bytes_site(M::PS::prec) + 11 * 24.0 + 5 * 24.0 * N) * g.Vh;
        const long long nv = np * 3;
        hipLaunchKernelGGL(k_to_double, dim3(nbm), dim3(MB_NT), 0, s, (const float2 *)B.xs, B.x64, nv);
        hipLaunchKernelGGL((k_to_batched<N>), dim3(nbm), dim3(MB_NT), 0, s, (const double2 *)b, B.b64, (long long)g.Vh,
                           n, 1);
    } else {
        HISQ_HIP(hipMemsetAsync(B.x64, 0, (size_t)np * 3 * 16, s));
        hipLaunchKernelGGL((k_to_batched<N>), dim3(nbm), dim3(MB_NT), 0, s, (const double2 *)b, B.b64, (long long)g.Vh,
                           n, 0);
    }
    HISQ_HIP(hipGetLastError());
    // FP64 true residuals of the starting x (the shifted solutions, or 0)
    int rc = multi_rhs_init<M, N>(n, masses, tol, fat, lng, g, o, B, hs, s);
    if (rc) return rc;
    out.bytes += multi_rel_bytes<typename M::PH>(N) * g.Vh;
    if (shift_only) {
        for (int c = 0; c < n; ++c) retire<N>(B, hs, g, c, out, s);
        HISQ_HIP(hipGetLastError());
    } else {
        rc = multi_rhs_run<M, N>(fat, lng, fat_lo, lng_lo, g, o, B, hs, s, offset, out);
        if (rc) return rc;
    }
    HISQ_HIP(hipStreamSynchronize(s));
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int worst = HISQ_OK;
    for (int r = 0; r < n; ++r) {
        const double tr = out.bb[r] > 0 ? std::sqrt(out.rr_true[r] / out.bb[r]) : 0.0;
        int st;
        if (shift_only) st = ms_conv[r] ? HISQ_OK : HISQ_ENOCONV;
        else st = out.bb[r] == 0.0 ? HISQ_OK
                                   : (tr <= tol ? HISQ_OK : (out.status[r] == HISQ_EBREAKDOWN ? HISQ_EBREAKDOWN : HISQ_ENOCONV));
        if (st != HISQ_OK && worst == HISQ_OK) worst = st;
        if (stats) {
            stats[r].iters = shift_only ? ms_iters[r] : out.iters[r] + ms_iters[r];
            stats[r].reliable_updates = shift_only ? 0 : out.nupd[r];
            stats[r].restarts = 0;
            stats[r].status = st;
            stats[r].true_resid = tr;
            stats[r].time_s = dt;
            stats[r].iter_resid = shift_only ? ms_resid[r] : (out.bb[r] > 0 ? std::sqrt(out.rr[r] / out.bb[r]) : 0.0);
            stats[r].bytes_moved = out.bytes;
        }
    }
    if (worst == HISQ_EBREAKDOWN) return fail(worst, "cg_solve_multi: breakdown in some right-hand side");
    if (worst == HISQ_ENOCONV)
        return fail(worst, shift_only ? "cg_solve_multi: some shift did not reach shift_tol within max_iter"
                                      : "cg_solve_multi: some right-hand side not converged");
    return HISQ_OK;
}

// ------------------------------------------------------------------ autotuner of the multi-RHS Dslash
template <class PS, int N>
static int tune_multi_impl(const Geom &g, const void *fat, const void *lng, const void *src, void *dst, void *ws,
                           size_t ws_bytes, int reps, int *best, double *us, hipStream_t s)
{
    if (ws_bytes < 4096) return fail(HISQ_EWORKSPACE, "hisq_tune_multi: workspace too small");
    MultiState *st = (MultiState *)ws;
    hipLaunchKernelGGL(k_mstate_all, dim3(1), dim3(1), 0, s, st, N);  // every RHS active for the timing
    hipEvent_t e0, e1;
    HISQ_HIP(hipEventCreate(&e0));
    HISQ_HIP(hipEventCreate(&e1));
    double best_us = 1e300;
    int best_i = 0, rc = HISQ_OK;
    for (int i = 0; i < N_MSHAPES && !rc; ++i) {
        if (N / MSHAPES[i].gdiv < 1 || (N % MSHAPES[i].gdiv)) { if (us) us[i] = -1; continue; }
        auto go = [&]() {
            return launch_md_shape<PS, N, EPI_STORE>(i, g, fat, lng, src, dst, nullptr, nullptr, nullptr, 1, nullptr,
                                                    st, MASK_ACTIVE, GATE_ALWAYS, s, nullptr);
        };
        for (int w = 0; w < 2; ++w) if (go() != hipSuccess) rc = HISQ_EHIP;
        hipEventRecord(e0, s);
        for (int k = 0; k < reps; ++k) if (go() != hipSuccess) rc = HISQ_EHIP;
        hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) rc = HISQ_EHIP;
        float ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        const double t = 1e3 * ms / reps;
        if (us) us[i] = t;
        if (t < best_us) { best_us = t; best_i = i; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return fail(rc, "hisq_tune_multi: launch failed");
    set_tuned_choice("mdslash", g, PS::prec, N, best_i);
    if (best) *best = best_i;
    return HISQ_OK;
}

// one timed-or-plain launch of the multi-RHS FP32 Dslash (for benchmarks and tests)
template <int N>
static int mdslash_apply_impl(const Geom &g, const void *fat, const void *lng, const void *src, void *dst, int parity,
                              void *ws, hipStream_t s)
{
    MultiState *st = (MultiState *)ws;
    hipLaunchKernelGGL(k_mstate_all, dim3(1), dim3(1), 0, s, st, N);
    HISQ_HIP((launch_md_shape<PF32, N, EPI_STORE>(mshape_for<PF32>(g, N), g, fat, lng, src, dst, nullptr, nullptr, nullptr,
                                                  parity, nullptr, st, MASK_ACTIVE, GATE_ALWAYS, s, nullptr)));
    return HISQ_OK;
}

template <class M>
static int cg_multi_dispatch(int nrhs, const double *masses, double tol, int mode, const void *fat, const void *lng,
                             const void *fat_lo, const void *lng_lo, const void *b, void *x, const Geom &g,
                             const hisq_cg_opts &o, void *ws, size_t ws_bytes, hisq_cg_stats *stats, hipStream_t s)
{
    switch (pad_n(nrhs)) {
    case 1: return cg_multi_impl<M, 1>(nrhs, masses, tol, mode, fat, lng, fat_lo, lng_lo, b, x, g, o, ws, ws_bytes, stats, s);
    case 2: return cg_multi_impl<M, 2>(nrhs, masses, tol, mode, fat, lng, fat_lo, lng_lo, b, x, g, o, ws, ws_bytes, stats, s);
    case 4: return cg_multi_impl<M, 4>(nrhs, masses, tol, mode, fat, lng, fat_lo, lng_lo, b, x, g, o, ws, ws_bytes, stats, s);
    case 8: return cg_multi_impl<M, 8>(nrhs, masses, tol, mode, fat, lng, fat_lo, lng_lo, b, x, g, o, ws, ws_bytes, stats, s);
    default: return cg_multi_impl<M, 16>(nrhs, masses, tol, mode, fat, lng, fat_lo, lng_lo, b, x, g, o, ws, ws_bytes, stats, s);
    }
}

}  // namespace hisq

using namespace hisq;

extern "C" int cg_solve_multi(int nrhs, const double *masses, double tol, int mode, const void *fat, const void *lng,
                              const void *fat_lo, const void *lng_lo, const void *b, void *x, const int dims[4],
                              const hisq_cg_opts *opts, void *workspace, size_t ws_bytes, hisq_cg_stats *stats,
                              void *stream)
{
    if (stats && nrhs > 0) std::memset(stats, 0, sizeof(hisq_cg_stats) * std::min(nrhs, MAXR));
    Geom g;
    int rc = make_geom(dims, g);
    if (rc) return rc;
    if (nrhs < 1 || nrhs > MAXR) return fail(HISQ_EINVAL, "cg_solve_multi: nrhs must be 1..16");
    if (mode != HISQ_MULTI_RHS && mode != HISQ_MULTI_SHIFT) return fail(HISQ_EINVAL, "cg_solve_multi: unknown mode");
    if (!masses || !fat || !lng || !fat_lo || !lng_lo || !b || !x) return fail(HISQ_EINVAL, "cg_solve_multi: NULL pointer");
    if (!aligned16({fat, lng, fat_lo, lng_lo, b, x, workspace}))
        return fail(HISQ_EINVAL, "cg_solve_multi: device pointers must be 16-byte aligned");
    if (b == x) return fail(HISQ_EALIAS, "cg_solve_multi: b and x alias");
    if (!(tol > 0)) return fail(HISQ_EINVAL, "cg_solve_multi: need tol > 0");
    for (int r = 0; r < nrhs; ++r)
        if (!(masses[r] > 0)) return fail(HISQ_EINVAL, "cg_solve_multi: masses must be > 0");
    hisq_cg_opts o = resolve_opts(opts, g);
    if (!(o.delta < 1.0)) return fail(HISQ_EINVAL, "cg_solve_multi: opts->delta must be below 1");
    if (!(o.shift_tol < 1.0)) return fail(HISQ_EINVAL, "cg_solve_multi: opts->shift_tol must be below 1");
    if (!workspace || ws_bytes < cg_multi_workspace_bytes(g, nrhs, mode))
        return fail(HISQ_EWORKSPACE, "cg_solve_multi: workspace NULL or smaller than hisq_workspace_bytes()");
    if (o.mode != HISQ_CG_PLAIN_F64 && o.mode != HISQ_CG_MIXED_F32 && o.mode != HISQ_CG_MIXED_F32C &&
        o.mode != HISQ_CG_MIXED_I16S && o.mode != HISQ_CG_MIXED_I16SC)
        return fail(HISQ_EINVAL, "cg_solve_multi: opts->mode must be PLAIN_F64 / MIXED_F32 (F64 + F32 links), "
                                 "MIXED_F32C (F64C + F32C), MIXED_I16S (F64 + I16S) or MIXED_I16SC (F64C + I16SC)");
    hipStream_t s = (hipStream_t)stream;
    HISQ_HIP(hipStreamSynchronize(s));
    switch (o.mode) {
    case HISQ_CG_MIXED_F32C:
        return cg_multi_dispatch<MultiLinks32C>(nrhs, masses, tol, mode, fat, lng, fat_lo, lng_lo, b, x, g, o,
                                                workspace, ws_bytes, stats, s);
    case HISQ_CG_MIXED_I16S:
        return cg_multi_dispatch<MultiLinks16>(nrhs, masses, tol, mode, fat, lng, fat_lo, lng_lo, b, x, g, o,
                                               workspace, ws_bytes, stats, s);
    case HISQ_CG_MIXED_I16SC:
        return cg_multi_dispatch<MultiLinks16C>(nrhs, masses, tol, mode, fat, lng, fat_lo, lng_lo, b, x, g, o,
                                                workspace, ws_bytes, stats, s);
    default:
        return cg_multi_dispatch<MultiLinks32>(nrhs, masses, tol, mode, fat, lng, fat_lo, lng_lo, b, x, g, o,
                                               workspace, ws_bytes, stats, s);
    }
}

extern "C" int hisq_tune_multi(const void *fat, const void *lng, const void *src, void *dst, const int dims[4], int nrhs,
                               void *workspace, size_t ws_bytes, int reps, int *best_shape, double *us_per_shape,
                               void *stream)
{
    Geom g;
    int rc = make_geom(dims, g);
    if (rc) return rc;
    if (!fat || !lng || !src || !dst || !workspace) return fail(HISQ_EINVAL, "hisq_tune_multi: NULL pointer");
    if (!aligned16({fat, lng, src, dst, workspace}))
        return fail(HISQ_EINVAL, "hisq_tune_multi: device pointers must be 16-byte aligned");
    if (src == dst) return fail(HISQ_EALIAS, "hisq_tune_multi: src and dst alias");
    if (nrhs != pad_n(nrhs) || nrhs > MAXR) return fail(HISQ_EINVAL, "hisq_tune_multi: nrhs must be 1, 2, 4, 8 or 16");
    if (reps <= 0) reps = 10;
    hipStream_t s = (hipStream_t)stream;
    switch (nrhs) {
    case 1: return tune_multi_impl<PF32, 1>(g, fat, lng, src, dst, workspace, ws_bytes, reps, best_shape, us_per_shape, s);
    case 2: return tune_multi_impl<PF32, 2>(g, fat, lng, src, dst, workspace, ws_bytes, reps, best_shape, us_per_shape, s);
    case 4: return tune_multi_impl<PF32, 4>(g, fat, lng, src, dst, workspace, ws_bytes, reps, best_shape, us_per_shape, s);
    case 8: return tune_multi_impl<PF32, 8>(g, fat, lng, src, dst, workspace, ws_bytes, reps, best_shape, us_per_shape, s);
    default: return tune_multi_impl<PF32, 16>(g, fat, lng, src, dst, workspace, ws_bytes, reps, best_shape, us_per_shape, s);
    }
}

extern "C" int hisq_dslash_multi(const void *fat, const void *lng, const void *src, void *dst, int parity, int nrhs,
                                 const int dims[4], void *workspace, size_t ws_bytes, void *stream)
{
    Geom g;
    int rc = make_geom(dims, g);
    if (rc) return rc;
    if (!fat || !lng || !src || !dst || !workspace) return fail(HISQ_EINVAL, "hisq_dslash_multi: NULL pointer");
    if (!aligned16({fat, lng, src, dst, workspace}))
        return fail(HISQ_EINVAL, "hisq_dslash_multi: device pointers must be 16-byte aligned");
    if (src == dst) return fail(HISQ_EALIAS, "hisq_dslash_multi: src and dst alias");
    if (parity != 0 && parity != 1) return fail(HISQ_EINVAL, "hisq_dslash_multi: parity must be 0 or 1");
    if (nrhs != pad_n(nrhs) || nrhs > MAXR) return fail(HISQ_EINVAL, "hisq_dslash_multi: nrhs must be 1, 2, 4, 8 or 16");
    if (ws_bytes < 4096) return fail(HISQ_EWORKSPACE, "hisq_dslash_multi: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    switch (nrhs) {
    case 1: return mdslash_apply_impl<1>(g, fat, lng, src, dst, parity, workspace, s);
    case 2: return mdslash_apply_impl<2>(g, fat, lng, src, dst, parity, workspace, s);
    case 4: return mdslash_apply_impl<4>(g, fat, lng, src, dst, parity, workspace, s);
    case 8: return mdslash_apply_impl<8>(g, fat, lng, src, dst, parity, workspace, s);
    default: return mdslash_apply_impl<16>(g, fat, lng, src, dst, parity, workspace, s);
    }
}

extern "C" int hisq_multi_shape(const int dims[4], int nrhs, int shape)
{
    Geom g;
    int rc = make_geom(dims, g);
    if (rc) return rc;
    if (nrhs != pad_n(nrhs) || nrhs > MAXR) return fail(HISQ_EINVAL, "hisq_multi_shape: nrhs must be 1, 2, 4, 8 or 16");
    if (shape == -2) return N_MSHAPES;
    if (shape < -2 || shape >= N_MSHAPES) return fail(HISQ_EINVAL, "hisq_multi_shape: no such shape");
    if (shape >= 0) {
        if (nrhs % MSHAPES[shape].gdiv) return fail(HISQ_EINVAL, "hisq_multi_shape: shape does not divide nrhs");
        set_tuned_choice("mdslash", g, HISQ_F32, nrhs, shape);
    }
    return mshape_for<PF32>(g, nrhs);
}
