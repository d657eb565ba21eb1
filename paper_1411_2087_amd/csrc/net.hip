// Gauge-covariant linear network used as a preconditioner of the even-odd CG.
//
// A layer maps C_in colour-vector fields on the full lattice to C_out:
//     out^a(x) = sum_b sum_{k=0..8} W_k^{ab} (T_k in^b)(x)
// T_0 = 1, T_{+mu} phi(x) = F_mu(x) phi(x+mu), T_{-mu} phi(x) = F_mu(x-mu)^dag
// phi(x-mu), with F the folded one-link ("fat") field of the operator
// (Sec. 3) read from its packed FP32 form.  Four layers 1 -> C -> C -> C -> 1,
// no nonlinearity, so the network is linear and commutes with gauge
// transformations.  An even-site input is embedded on the full lattice (odd
// sites zero); the output's even part is the preconditioned vector.
//
// A layer kernel takes one 64-site tile (one wavefront of sites, the tile of
// the packed links) of one parity.  The 9 C_in transported fields are taken
// in slices of 16 (transport, channel) pairs: each thread computes one site's
// transport of four channels along one direction in FP32 (one link load for
// the four), the slice goes to LDS as BF16 in the real embedding, and the
// channel mixing accumulates
//     [Re out; Im out] (2 C_out x 192) += [[Wr, -Wi], [Wi, Wr]] (2 C_out x 32)
//                                         x [Re T; Im T] (32 x 192)
// on v_mfma_f32_16x16x32_bf16 with FP32 accumulation, so the LDS holds one
// slice (15 KB) and the transports are computed once per site and channel.
// The gradient with respect to the input is the same kernel with
// W'_{k'}^{ba} = conj(W_{k}^{ab}), k' the adjoint transport of k
// (T_{+mu}^dag = T_{-mu}); the weight gradient G_k^{ab} = sum_x <T_k in^b, g^a>
// = sum_x <in^b, T_{adj k} g^a> is taken in the same kernel from those
// transports of g (k_net_bwd), with the sites (and Re/Im) as the K dimension,
// and a fixed-order FP64 sum of the per-workgroup partials.  The C -> 1 layer
// mixes first and transports once (k_net_layer_mt, FP32).
//
// Feature layout: [batch][channel][parity][h][colour] complex64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "dslash_core.hpp"

namespace hisq {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int NET_NT = 256;     // four wavefronts; wave q transports the pairs 4q..4q+3 of a slice
constexpr int MPAD = 32;        // GEMM rows: Re and Im of up to 16 output channels
constexpr int SK = 32;          // K of one slice: 16 (transport, channel) pairs, Re parts then Im parts
constexpr int NCOL = 3 * TILE;  // GEMM columns of a 64-site tile: (site, colour)
constexpr int WG_MAX_BLOCKS = 1024;  // a multiple of NXCD

// The 9 transports of a layer with CIN input channels in slices of 16
// (transport, channel) pairs: KG transports per slice, pair pi -> transport
// kg = pi / CIN of the slice, channel pi % CIN.  Pairs past transport 8 are zero.
template <int CIN> struct Slices {
    static constexpr int KG = CIN >= 16 ? 1 : 16 / CIN;
    static constexpr int N = (9 + KG - 1) / KG;
};
__host__ __device__ constexpr int slices_of(int cin) { return cin >= 16 ? 9 : (9 + 16 / cin - 1) / (16 / cin); }
__host__ __device__ constexpr int kg_of(int cin) { return cin >= 16 ? 1 : 16 / cin; }
constexpr int ADJ[9] = { 0, 5, 6, 7, 8, 1, 2, 3, 4 };

__device__ __forceinline__ size_t feat_idx(int b, int C, int c, int p, int Vh, int h)
{
    return ((((size_t)b * C + c) * 2 + p) * Vh + h) * 3;
}

// The colour vector of site h (3 complex64, 24 bytes at 24 h of a 16-byte aligned field block) with one 16-byte
// and one 8-byte load: for even h the first two colours are 16-byte aligned, for odd h the last two.
__device__ __forceinline__ void load_cvec(const float2 *__restrict__ v, int h, float2 out[3])
{
    const bool odd = h & 1;
    const float4 q4 = *reinterpret_cast<const float4 *>(v + (odd ? 1 : 0));
    const float2 q2 = v[odd ? 0 : 2];
    out[0] = odd ? q2 : make_float2(q4.x, q4.y);
    out[1] = odd ? make_float2(q4.x, q4.y) : make_float2(q4.z, q4.w);
    out[2] = odd ? make_float2(q4.z, q4.w) : q2;
}

// One packed FP32 link (18 floats) with plain loads: the four pair groups of
// a slice read the same matrix, so it should stay in the caches.
__device__ __forceinline__ void load_link32(const char *__restrict__ blk, int lane, float m[18])
{
    const float4 *p4 = reinterpret_cast<const float4 *>(blk) + lane;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 v = p4[q * TILE];
        m[4 * q] = v.x; m[4 * q + 1] = v.y; m[4 * q + 2] = v.z; m[4 * q + 3] = v.w;
    }
    const float2 v = reinterpret_cast<const float2 *>(blk + 4 * TILE * 16)[lane];
    m[16] = v.x;
    m[17] = v.y;
}

// o = sg M phi for a row-major complex 3x3 M (18 floats) and sg = +-1, as
// explicit fmaf chains: every kernel that transports gets the same bits.
__device__ __forceinline__ void matvec32(const float m[18], float sg, float2 s0, float2 s1, float2 s2, float o[6])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float *r = m + 6 * a;
        float re = r[4] * s2.x;
        re = fmaf(-r[5], s2.y, re);
        re = fmaf(r[2], s1.x, re);
        re = fmaf(-r[3], s1.y, re);
        re = fmaf(r[0], s0.x, re);
        re = fmaf(-r[1], s0.y, re);
        float im = r[4] * s2.y;
        im = fmaf(r[5], s2.x, im);
        im = fmaf(r[2], s1.y, im);
        im = fmaf(r[3], s1.x, im);
        im = fmaf(r[0], s0.y, im);
        im = fmaf(r[1], s0.x, im);
        o[2 * a] = sg * re;
        o[2 * a + 1] = sg * im;
    }
}

// The site a thread transports at: its h (clamped to the last site for the
// ragged tail of the last tile) and coordinates, computed once per tile.
struct NetSite {
    int hc, x, y, z, t;
    bool valid;
};
__device__ __forceinline__ NetSite net_site(const Geom &g, int p, int tile, int lane)
{
    NetSite s;
    const int h = tile * TILE + lane;
    s.valid = h < g.Vh;
    s.hc = s.valid ? h : g.Vh - 1;
    site_coords(g, s.hc, p, s.x, s.y, s.z, s.t);
    return s;
}

// The CH channels of a unit's tile (64 sites of one parity and batch entry)
// as float4 pairs of consecutive colour entries, TileFeat::NV per thread, all
// loads issued before any value is used.  Every extent is even, so Vh and a
// tile's first site are multiples of 8: the tile's entries in the lattice end
// at an even index, a pair lies wholly inside or outside, and pairs outside
// read as zero.
template <int CH> struct TileFeat {
    static constexpr int NP = CH * NCOL / 2;  // pairs of the tile
    static constexpr int NV = (NP + NET_NT - 1) / NET_NT;
    float4 v[NV];
};
// (The thread index goes through an opaque copy: in a loop over units the
// compiler would otherwise keep every entry's offsets from the first unit on,
// in registers the loop needs.)
__device__ __forceinline__ int opaque_tid()
{
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}
template <int CH>
__device__ __forceinline__ void tile_feat_load(const Geom &g, const float2 *__restrict__ f, int b, int p, int tile,
                                               TileFeat<CH> &t)
{
    const int nvalid = min(NCOL, (g.Vh - tile * TILE) * 3), tid = opaque_tid();
#pragma unroll
    for (int it = 0; it < TileFeat<CH>::NV; ++it) {
        const int i = tid + it * NET_NT, c = i / (NCOL / 2), jc = 2 * (i % (NCOL / 2));
        t.v[it] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (i < TileFeat<CH>::NP && jc < nvalid)
            t.v[it] = *reinterpret_cast<const float4 *>(f + feat_idx(b, CH, c, p, g.Vh, tile * TILE) + jc);
    }
}
// Row c of `rows` gets (s0 e_r, s0 e_i) and row c + CH (s1 e_i, s2 e_r) of
// each entry e of channel c, as BF16 at K = 2 jc, 2 jc + 1 (pitch PK).
template <int CH, int PK>
__device__ __forceinline__ void tile_feat_put(const TileFeat<CH> &t, __bf16 *rows, float s1, float s2)
{
    const int tid = opaque_tid();
#pragma unroll
    for (int it = 0; it < TileFeat<CH>::NV; ++it) {
        const int i = tid + it * NET_NT, c = i / (NCOL / 2), jc = 2 * (i % (NCOL / 2));
        if (i >= TileFeat<CH>::NP) continue;
        const float4 e = t.v[it];
        *reinterpret_cast<bf16x4 *>(rows + c * PK + 2 * jc) = bf16x4{ (__bf16)e.x, (__bf16)e.y, (__bf16)e.z, (__bf16)e.w };
        *reinterpret_cast<bf16x4 *>(rows + (CH + c) * PK + 2 * jc) =
            bf16x4{ (__bf16)(s1 * e.y), (__bf16)(s2 * e.x), (__bf16)(s1 * e.w), (__bf16)(s2 * e.z) };
    }
}

// The loads of a thread's four pairs of one slice when they share one
// transport (C_in >= 4): the link and the four neighbour (or own) vectors,
// kept raw so that the MFMA of the previous slice can run while they arrive.
struct SliceRaw {
    float m[18];
    float2 v[4][3];
    float sg;  // sign of the packed link (backward slots hold -F^dag)
    int kind;  // 0: T_0 (v is the result), 1: transport, 2: padding (zero)
};

template <int CIN, bool SIGNED = false, bool WIDE = false>
__device__ __forceinline__ void slice_load(const Geom &g, const char *__restrict__ fat, const float2 *__restrict__ in,
                                           int p, int tile, int lane, const NetSite &st, int j, int q, SliceRaw &r)
{
    static_assert(CIN >= 4, "one transport per thread and slice");
    constexpr int KG = Slices<CIN>::KG;
    const size_t ch_stride = (size_t)2 * g.Vh * 3;
    const int k = j * KG + (4 * q) / CIN, c0 = (4 * q) % CIN;
    r.kind = k == 0 ? 0 : (k < 9 ? 1 : 2);
    r.sg = 1.0f;
    if (r.kind == 2) return;
    int hn = st.hc, pn = p;
    if (k > 0) {
        const int d = k - 1;
        hn = nbr_h(g, st.hc, st.x, st.y, st.z, st.t, d & 3, d >= 4 ? -1 : 1);
        pn = 1 - p;
        load_link32(fat + (((size_t)p * g.ntiles + tile) * 8 + d) * PF32::block_bytes, lane, r.m);
        r.sg = (SIGNED && d >= 4) ? -1.0f : 1.0f;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float2 *v = in + (c0 + i) * ch_stride + (size_t)pn * g.Vh * 3 + (size_t)hn * 3;
        if constexpr (WIDE) {
            load_cvec(v, hn, r.v[i]);
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) r.v[i][a] = v[a];
        }
    }
}

__device__ __forceinline__ void slice_finish(const SliceRaw &r, float tv[4][6])
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (r.kind == 1) {
            matvec32(r.m, r.sg, r.v[i][0], r.v[i][1], r.v[i][2], tv[i]);
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                tv[i][2 * a] = r.kind == 0 ? r.v[i][a].x : 0.f;
                tv[i][2 * a + 1] = r.kind == 0 ? r.v[i][a].y : 0.f;
            }
        }
    }
}

// The four (transport, channel) pairs 4q..4q+3 of slice j at the thread's
// site of parity p (lane `lane` of `tile`): tv[i] = (T_k phi^c)(x) for pair
// 4q + i, colours (re, im) x 3; zero for padding pairs.  T_0 = 1; T_{1+d}:
// packed direction d (0..3 = +x..+t holds F_mu(x), 4..7 = -x..-t holds
// -F_mu(x-mu)^dag) times the neighbour one hop along d.  With SIGNED the
// backward transports get the packed link's sign undone; without it they come
// out as -T_k, and the kernels carry the sign in the weights instead
// (k_net_prep negates them, k_net_wgrad_reduce their gradients): negation is
// exact in BF16, so the products are the same bits, and 24 multiplies per
// slice and wavefront are saved.  Lanes past Vh (clamped to the last site)
// get finite values that no stored output uses: the layer stores only sites
// below Vh, and the weight gradient multiplies them by zero upstream gradients.
// in: the channels of one batch entry, [c][parity][Vh][3].
template <int CIN, bool SIGNED = false, bool WIDE = false>
__device__ __forceinline__ void slice_transport(const Geom &g, const char *__restrict__ fat,
                                                const float2 *__restrict__ in, int p, int tile, int lane,
                                                const NetSite &st, int j, int q, float tv[4][6])
{
    const int hc = st.hc, x = st.x, y = st.y, z = st.z, t = st.t;
    const size_t ch_stride = (size_t)2 * g.Vh * 3;
    const char *tb = fat + ((size_t)p * g.ntiles + tile) * 8 * PF32::block_bytes;
    if constexpr (CIN >= 4) {
        SliceRaw r;
        slice_load<CIN, SIGNED, WIDE>(g, fat, in, p, tile, lane, st, j, q, r);
        slice_finish(r, tv);
        return;
    } else {
        // CIN == 1: one slice holds every transport; pair i of group q is transport 4q + i
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * q + i;
            if (k == 0) {
                float2 e[3];
                const float2 *v = in + (size_t)p * g.Vh * 3 + (size_t)hc * 3;
                if constexpr (WIDE) load_cvec(v, hc, e);
                else for (int a = 0; a < 3; ++a) e[a] = v[a];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    tv[i][2 * a] = e[a].x;
                    tv[i][2 * a + 1] = e[a].y;
                }
            } else if (k < 9) {
                const int d = k - 1;
                const int nh = nbr_h(g, hc, x, y, z, t, d & 3, d >= 4 ? -1 : 1);
                float m[18];
                load_link32(tb + (size_t)d * PF32::block_bytes, lane, m);
                float2 e[3];
                const float2 *v = in + (size_t)(1 - p) * g.Vh * 3 + (size_t)nh * 3;
                if constexpr (WIDE) load_cvec(v, nh, e);
                else for (int a = 0; a < 3; ++a) e[a] = v[a];
                matvec32(m, (SIGNED && d >= 4) ? -1.0f : 1.0f, e[0], e[1], e[2], tv[i]);
            } else {
#pragma unroll
                for (int e = 0; e < 6; ++e) tv[i][e] = 0.f;
            }
        }
    }
}

// ------------------------------------------------------------------ weights -> BF16 GEMM operand
// A[j][m][kk] (slices x 32 x 32) for out = sum_k W_k T_k in: row m < COUT'
// is Re out^m, row COUT' + a is Im out^a; column kk < 16 takes the real
// part of pair kk of slice j, kk >= 16 the imaginary part of pair kk - 16;
// the real embedding [[Wr, -Wi], [Wi, Wr]], negated for the backward
// transports k = 5..8 (the kernels take them without the packed sign).
// adjoint: the matrix of the
// input-gradient layer (C_in' = COUT, C_out' = CIN, W'_k^{ac} =
// conj(W_{adj k}^{ca}), T_{+mu}^dag = T_{-mu}).
template <int CIN, int COUT>
__global__ void k_net_prep(const float2 *__restrict__ W, __bf16 *__restrict__ A, int adjoint)
{
    const int ci = adjoint ? COUT : CIN, co = adjoint ? CIN : COUT;
    const int ns = slices_of(ci), kgs = kg_of(ci);
    for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < ns * MPAD * SK; i += blockDim.x * gridDim.x) {
        const int j = i / (MPAD * SK), m = (i / SK) % MPAD, kk = i % SK;
        const int pi = kk % 16;
        const bool im_col = kk >= 16, im_row = m >= co;
        const int k = j * kgs + pi / ci, c = pi % ci;
        float v = 0.f;
        if (m < 2 * co && k < 9) {
            const int a = im_row ? m - co : m;
            float2 w;
            if (!adjoint) {
                w = W[((size_t)k * COUT + a) * CIN + c];
            } else {
                const float2 u = W[((size_t)ADJ[k] * COUT + c) * CIN + a];
                w = make_float2(u.x, -u.y);
            }
            v = !im_row ? (!im_col ? w.x : -w.y) : (!im_col ? w.y : w.x);
            if (k >= 5) v = -v;  // the kernels transport backward without the packed sign
        }
        A[i] = (__bf16)v;
    }
}

// ------------------------------------------------------------------ layer (forward and input gradient)
// Work units u = (batch entry, tile, parity), u = (b ntiles + tile) 2 + p, in
// XCD order: each XCD takes a contiguous range of units (xcd_block), so the
// neighbour tiles a unit transports from are in flight on the same XCD and
// are served by its L2 instead of being fetched once per XCD.
__device__ __forceinline__ void net_unit(int u, int ntiles, int &b, int &tile, int &p)
{
    b = u / (2 * ntiles);
    tile = (u >> 1) % ntiles;
    p = u & 1;
}

// One unit per workgroup: a 64-site tile of one parity and batch entry.  Per slice:
// the tile's 16 x 192 transported values go to LDS as BF16 (B[column][K]),
// then the four waves run v_mfma_f32_16x16x32_bf16 on 16-column tiles
// 3q..3q+2 for every 16-row tile of the output (FP32 accumulation).
template <int CIN, int COUT>
__global__ __launch_bounds__(NET_NT) void k_net_layer(Geom g, const char *__restrict__ fat,
                                                      const float2 *__restrict__ in, float2 *__restrict__ out,
                                                      const __bf16 *__restrict__ A, int batch)
{
    using S = Slices<CIN>;
    constexpr int MT = (2 * COUT + 15) / 16;  // 16-row tiles of the output
    constexpr int PB = SK + 8;                // LDS pitch of a column (bf16)
    __shared__ __align__(16) __bf16 F[2][NCOL * PB];  // two slices: one mixed while the next is written
    const int u = xcd_block(blockIdx.x, gridDim.x);
    if (u >= batch * 2 * g.ntiles) return;  // the grid is rounded up to a multiple of the XCD count
    int b, tile, p;
    net_unit(u, g.ntiles, b, tile, p);
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const float2 *inb = in + (size_t)b * CIN * 2 * g.Vh * 3;
    const NetSite site = net_site(g, p, tile, lane);
    floatx4 acc[3][MT];
#pragma unroll
    for (int n = 0; n < 3; ++n)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[n][mt] = floatx4{ 0.f, 0.f, 0.f, 0.f };
    const int r16 = lane & 15, k8 = 8 * (lane >> 4);
    auto put = [&](__bf16 *Fs, const float tv[4][6]) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            __bf16 *col = Fs + (3 * lane + a) * PB;
            const bf16x4 re = { (__bf16)tv[0][2 * a], (__bf16)tv[1][2 * a], (__bf16)tv[2][2 * a], (__bf16)tv[3][2 * a] };
            const bf16x4 im = { (__bf16)tv[0][2 * a + 1], (__bf16)tv[1][2 * a + 1], (__bf16)tv[2][2 * a + 1],
                                (__bf16)tv[3][2 * a + 1] };
            *reinterpret_cast<bf16x4 *>(col + 4 * q) = re;
            *reinterpret_cast<bf16x4 *>(col + 16 + 4 * q) = im;
        }
    };
    auto mix = [&](const __bf16 *Fs, int j) {
        bf16x8 av[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
            av[mt] = *reinterpret_cast<const bf16x8 *>(A + ((size_t)j * MPAD + mt * 16 + r16) * SK + k8);
#pragma unroll
        for (int n = 0; n < 3; ++n) {
            const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(Fs + ((3 * q + n) * 16 + r16) * PB + k8);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                acc[n][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mt], bv, acc[n][mt], 0, 0, 0);
        }
    };
    {
        float tv[4][6];
        slice_transport<CIN, false, CIN == 1>(g, fat, inb, p, tile, lane, site, 0, q, tv);
        put(F[0], tv);
    }
    __syncthreads();
#pragma unroll 1
    for (int j = 0; j < S::N; ++j) {
        // slice j is in F[j & 1]; F[(j + 1) & 1] was last read before the previous barrier
        if constexpr (CIN >= 4) {
            SliceRaw r;
            const bool more = j + 1 < S::N;
            if (more) slice_load<CIN>(g, fat, inb, p, tile, lane, site, j + 1, q, r);  // in flight over the MFMA
            mix(F[j & 1], j);
            if (more) {
                float tv[4][6];
                slice_finish(r, tv);
                put(F[(j + 1) & 1], tv);
            }
        } else {
            mix(F[j & 1], j);
            if (j + 1 < S::N) {
                float tv[4][6];
                slice_transport<CIN, false, CIN == 1>(g, fat, inb, p, tile, lane, site, j + 1, q, tv);
                put(F[(j + 1) & 1], tv);
            }
        }
        __syncthreads();
    }
    // D[row][col]: lane holds column r16 of its tile and rows 4 (lane >> 4) + 0..3
    float *o = reinterpret_cast<float *>(out);
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        const int col = (3 * q + n) * 16 + r16, s = col / 3, a = col % 3, h = tile * TILE + s;
        if (h >= g.Vh) continue;
        if constexpr (COUT == 16) {
            // row tile 0 holds Re, row tile 1 Im of the same four channels
#pragma unroll
            for (int i = 0; i < 4; ++i)
                out[feat_idx(b, COUT, 4 * (lane >> 4) + i, p, g.Vh, h) + a] = make_float2(acc[n][0][i], acc[n][1][i]);
            continue;
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = mt * 16 + 4 * (lane >> 4) + i;
                if (m < 2 * COUT) {
                    const int ch = m < COUT ? m : m - COUT;
                    o[2 * (feat_idx(b, COUT, ch, p, g.Vh, h) + a) + (m < COUT ? 0 : 1)] = acc[n][mt][i];
                }
            }
    }
}

// ------------------------------------------------------------------ C -> 1 layer: mix, then transport
// With one output channel the two linear maps are cheaper the other way
// round: out(x) = sum_k T_k (sum_c W_k^c in^c)(x).  At the neighbour x + k_d
// the CIN channels are mixed into one colour vector, which the link then
// carries: 12 CIN + 36 FMAs per transport instead of 36 CIN and the mixing,
// in FP32 on the VALU (no MFMA, no rounding of the operands to BF16).  One
// workgroup per unit (64-site tile of one parity and batch entry, units in
// XCD order, so that a CU's few units in flight keep their neighbour tiles
// in its XCD's L2); wave q takes the directions 2q and 2q + 1 and the
// channels 4q .. 4q + 3 of T_0, one thread per site, and the four partial
// sums meet in LDS.  W: the layer's FP32 weights [9][1][CIN]; with adjoint,
// those of a 1 -> CIN layer [9][CIN][1] taken as conj(W_{adj k}^{c}) (the
// input gradient of that layer).
template <int CIN>
__global__ __launch_bounds__(NET_NT) void k_net_layer_mt(Geom g, const char *__restrict__ fat,
                                                         const float2 *__restrict__ in, float2 *__restrict__ out,
                                                         const float2 *__restrict__ W, int batch, int adjoint)
{
    static_assert(CIN % 4 == 0, "four waves share the channels of T_0");
    __shared__ float part[4][6][TILE];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int u = xcd_block(blockIdx.x, gridDim.x);
    if (u >= batch * 2 * g.ntiles) return;  // the grid is rounded up to a multiple of the XCD count
    int b, tile, p;
    net_unit(u, g.ntiles, b, tile, p);
    const NetSite st = net_site(g, p, tile, lane);
    const float2 *inb = in + (size_t)b * CIN * 2 * g.Vh * 3;
    const size_t ch_stride = (size_t)2 * g.Vh * 3;
    const char *tb = fat + ((size_t)p * g.ntiles + tile) * 8 * PF32::block_bytes;
    const float wsg = adjoint ? -1.f : 1.f;  // conjugate for the adjoint
    // v += sum over channels c0 .. c0 + NC - 1 of W_k^c in^c at (parity pn, site hn)
    auto mixin = [&](int k, int pn, int hn, int c0, auto nc, float v[6]) {
        const float2 *src = inb + (size_t)pn * g.Vh * 3 + (size_t)hn * 3;
        const float2 *wk = W + (size_t)(adjoint ? ADJ[k] : k) * CIN;
#pragma unroll
        for (int i = 0; i < decltype(nc)::value; ++i) {
            const int c = c0 + i;
            const float2 w = wk[c];
            const float wr = w.x, wi = wsg * w.y;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float2 e = src[c * ch_stride + a];
                v[2 * a] = fmaf(wr, e.x, v[2 * a]);
                v[2 * a] = fmaf(-wi, e.y, v[2 * a]);
                v[2 * a + 1] = fmaf(wr, e.y, v[2 * a + 1]);
                v[2 * a + 1] = fmaf(wi, e.x, v[2 * a + 1]);
            }
        }
    };
    float o[6] = { 0.f, 0.f, 0.f, 0.f, 0.f, 0.f };
    mixin(0, p, st.hc, q * (CIN / 4), std::integral_constant<int, CIN / 4>{}, o);
#pragma unroll 1
    for (int dd = 0; dd < 2; ++dd) {
        const int d = 2 * q + dd;
        const int hn = nbr_h(g, st.hc, st.x, st.y, st.z, st.t, d & 3, d >= 4 ? -1 : 1);
        float v[6] = { 0.f, 0.f, 0.f, 0.f, 0.f, 0.f }, m[18], t[6];
        mixin(d + 1, 1 - p, hn, 0, std::integral_constant<int, CIN>{}, v);
        load_link32(tb + (size_t)d * PF32::block_bytes, lane, m);
        // the backward slots hold -F^dag: undo the sign
        matvec32(m, d >= 4 ? -1.f : 1.f, make_float2(v[0], v[1]), make_float2(v[2], v[3]), make_float2(v[4], v[5]),
                 t);
#pragma unroll
        for (int i = 0; i < 6; ++i) o[i] += t[i];
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) part[q][i][lane] = o[i];
    __syncthreads();
    // thread (wave a, lane) stores colour a of site lane: the four partials in a fixed order
    const int a = q;
    if (a >= 3 || tile * TILE + lane >= g.Vh) return;
    const float re = ((part[0][2 * a][lane] + part[1][2 * a][lane]) + part[2][2 * a][lane]) + part[3][2 * a][lane];
    const float im =
        ((part[0][2 * a + 1][lane] + part[1][2 * a + 1][lane]) + part[2][2 * a + 1][lane]) + part[3][2 * a + 1][lane];
    out[feat_idx(b, 1, 0, p, g.Vh, tile * TILE + lane) + a] = make_float2(re, im);
}

// ------------------------------------------------------------------ transports (inspection of the operands)
// out[b][k][c][parity][Vh][3] = (T_k in^c) for k = 0..8, the FP32 values the
// layer kernels round to BF16 (same device function, same bits).
template <int CIN>
__global__ __launch_bounds__(NET_NT) void k_net_transport(Geom g, const char *__restrict__ fat,
                                                          const float2 *__restrict__ in, float2 *__restrict__ out)
{
    using S = Slices<CIN>;
    const int tile = blockIdx.x, p = blockIdx.y, b = blockIdx.z;
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int h = tile * TILE + lane;
    const float2 *inb = in + (size_t)b * CIN * 2 * g.Vh * 3;
    const NetSite site = net_site(g, p, tile, lane);
    for (int j = 0; j < S::N; ++j) {
        float tv[4][6];
        slice_transport<CIN, true>(g, fat, inb, p, tile, lane, site, j, q, tv);
        if (h >= g.Vh) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int pi = 4 * q + i, k = j * S::KG + pi / CIN, c = pi % CIN;
            if (k >= 9) continue;
            float2 *dst = out + feat_idx(b * 9 + k, CIN, c, p, g.Vh, h);
#pragma unroll
            for (int a = 0; a < 3; ++a) dst[a] = make_float2(tv[i][2 * a], tv[i][2 * a + 1]);
        }
    }
}

// ------------------------------------------------------------------ weight gradient
// G_k^{ac} = sum_x <T_k in^c, g^a>: per 64-site tile the real GEMM
//   [Re G; Im G] (2 COUT x 16 pairs) += [[gr, gi], [gi, -gr]] (2 COUT x 384) x [Re T; Im T] (384 x 16)
// with K = (column, re/im) interleaved.  g goes to LDS once per tile, each
// slice's transports once per slice (all four waves, into registers while the
// slice before is multiplied, then into the one LDS slice buffer); the MFMAs
// of slice j (every row tile, all 12 K steps) belong to wave j % 4, which
// keeps the accumulators of its slices only (at most 3).  37.5 KB of LDS and
// at most 128 VGPRs: 4 workgroups per CU.  Blocks stride over (batch, tile, parity) units;
// each block writes its partial [slice][row][pair] (FP32), summed in FP64 by
// k_net_wgrad_reduce.
template <int CIN, int COUT>
__global__ __launch_bounds__(NET_NT, 4) void k_net_wgrad(Geom g, const char *__restrict__ fat,
                                                      const float2 *__restrict__ in, const float2 *__restrict__ gout,
                                                      int batch, float *__restrict__ partials)
{
    using S = Slices<CIN>;
    constexpr int MT = (2 * COUT + 15) / 16;
    constexpr int KT = 2 * NCOL;  // K per tile
    constexpr int PK = KT + 8;    // LDS pitch (bf16)
    constexpr int PART = S::N * MT * 256;
    __shared__ __align__(16) __bf16 lds[(16 + MT * 16) * PK];
    __bf16 *Fb = lds;                          // B: [pair][K], one slice
    __bf16 *Ga = lds + 16 * PK;                // A: [row][K]
    static_assert(PART * 4 <= (16 + MT * 16) * PK * 2, "partial reduction does not fit the LDS operands");
    constexpr int NSL = (S::N + 3) / 4;  // slices a wave owns: j = q, q + 4, ...
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int r16 = lane & 15, k8 = 8 * (lane >> 4);
    floatx4 acc[NSL][MT];
#pragma unroll
    for (int jj = 0; jj < NSL; ++jj)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[jj][mt] = floatx4{ 0.f, 0.f, 0.f, 0.f };
    // rows 2 COUT .. 16 MT - 1 of the g operand stay zero
    for (int i = threadIdx.x; i < (MT * 16 - 2 * COUT) * PK; i += NET_NT) Ga[2 * COUT * PK + i] = (__bf16)0.f;
    // persistent: XCD k walks the k-th contiguous range of units (gridDim.x is a multiple of NXCD)
    const int units = batch * 2 * g.ntiles;
    const int xcd = blockIdx.x % NXCD, per_xcd = gridDim.x / NXCD, units_per_xcd = (units + NXCD - 1) / NXCD;
#pragma unroll 1
    for (int v = blockIdx.x / NXCD; v < units_per_xcd; v += per_xcd) {
        const int u = xcd * units_per_xcd + v;
        if (u >= units) break;
        int b, tile, p;
        net_unit(u, g.ntiles, b, tile, p);
        const float2 *inb = in + (size_t)b * CIN * 2 * g.Vh * 3;
        const NetSite site = net_site(g, p, tile, lane);
        // g's rows [g_r, g_i] and [g_i, -g_r]; (the previous unit's last slice ended with a barrier: its
        // operands have been read)
        {
            TileFeat<COUT> gt;
            tile_feat_load<COUT>(g, gout, b, p, tile, gt);
            tile_feat_put<COUT, PK>(gt, Ga, 1.f, -1.f);
        }
        auto put = [&](__bf16 *Fb, const float tv[4][6]) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                __bf16 *row = Fb + (4 * q + i) * PK + 6 * lane;
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    *reinterpret_cast<bf16x2 *>(row + 2 * a) = bf16x2{ (__bf16)tv[i][2 * a], (__bf16)tv[i][2 * a + 1] };
            }
        };
        {
            float tv[4][6];
            slice_transport<CIN, false, CIN == 1>(g, fat, inb, p, tile, lane, site, 0, q, tv);
            put(Fb, tv);
        }
        __syncthreads();  // g and slice 0 are in LDS
        // unrolled: acc[j] must stay in registers; slice j + 1's loads are in flight over slice j's MFMA
#pragma unroll
        for (int j = 0; j < S::N; ++j) {
            const bool more = j + 1 < S::N;
            float tv[4][6];
            // the next slice's transport goes to registers while the owner wave multiplies this one
            if (more) slice_transport<CIN, false, CIN == 1>(g, fat, inb, p, tile, lane, site, j + 1, q, tv);
            if (q == (j & 3)) {  // this slice's owner (wave-uniform)
#pragma unroll
                for (int ks = 0; ks < KT / SK; ++ks) {
                    const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(Fb + r16 * PK + SK * ks + k8);
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        const bf16x8 av = *reinterpret_cast<const bf16x8 *>(Ga + (mt * 16 + r16) * PK + SK * ks + k8);
                        acc[j >> 2][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[j >> 2][mt], 0, 0, 0);
                    }
                }
            }
            if (more) {
                __syncthreads();  // every wave is done with slice j
                put(Fb, tv);
            }
            __syncthreads();
        }
    }
    // every (slice, row tile) accumulator has one owner: gathered through LDS for a coalesced store
    float *red = reinterpret_cast<float *>(lds);
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < NSL; ++jj) {
        const int j = q + 4 * jj;
        if (j < S::N)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) red[((j * MT + mt) * 16 + 4 * (lane >> 4) + i) * 16 + r16] = acc[jj][mt][i];
    }
    __syncthreads();
    float *dst = partials + (size_t)blockIdx.x * PART;
    for (int i = threadIdx.x; i < PART; i += NET_NT) dst[i] = red[i];
}

// ------------------------------------------------------------------ fused backward of a layer
// For a layer with input x (CO channels) and upstream gradient g (CI
// channels): the input gradient dx = sum_k W'_k T_k g (the adjoint layer,
// as k_net_layer<CI, CO>) and the weight gradient re-associated onto the
// same transports of g,
//     G_k^{ac} = sum_x <T_k x^c, g^a> = sum_y <x^c, T_k^dag g^a> = sum_y <x^c, T_{adj k} g^a>,
// so each slice of transported g is computed once and serves both GEMMs.
// The mixing is the layer kernel's; for the weight gradient x's own-site
// values go to LDS once per unit as the A operand [[x_r, x_i], [-x_i, x_r]]
// (rows Re and Im of channel c, K = (column, re/im)), the slice once more as
// B [pair][K], and R_{(k',a)}^c = sum_y conj(x^c) T'_{k'} g^a accumulates on
// the owner wave j % 4 as in k_net_wgrad.  The packed backward slots give
// T'_{k'} = -T_{k'} for k' >= 5; the partial stores, at slot k = adj k' of
// the forward layer's layout, the sum k_net_wgrad would have formed there
// with unsigned transports: -R for k' >= 1 and R for k' = 0, so that
// k_net_wgrad_reduce<CO, CI> finishes it unchanged.  Persistent workgroups
// over the units in XCD order (as k_net_wgrad); the input gradient of each
// unit is stored when its slices are done.  One slice buffer of each layout,
// 53 KB of LDS for CO = 16: three workgroups per CU.
template <int CI, int CO>
__global__ __launch_bounds__(NET_NT, 3) void k_net_bwd(Geom g, const char *__restrict__ fat,
                                                    const float2 *__restrict__ gup, const float2 *__restrict__ x,
                                                    float2 *__restrict__ dx, const __bf16 *__restrict__ A, int batch,
                                                    float *__restrict__ partials)
{
    using S = Slices<CI>;                   // slices of the transported upstream gradient
    constexpr int MTX = (2 * CO + 15) / 16;  // 16-row tiles of dx and of the x operand
    constexpr int KT = 2 * NCOL, PK = KT + 8, PB = SK + 8;
    constexpr int KGF = Slices<CO>::KG;      // the forward layer's partial layout
    constexpr int MTF = (2 * CI + 15) / 16;
    constexpr int PART = Slices<CO>::N * MTF * 256;
    constexpr int NSL = (S::N + 3) / 4;
    __shared__ __align__(16) __bf16 lds[(MTX * 16 + 16) * PK + NCOL * PB];
    __bf16 *Xa = lds;                  // weight gradient A: [row][K]
    __bf16 *Fb = lds + MTX * 16 * PK;  // weight gradient B: [pair][K]
    __bf16 *F = Fb + 16 * PK;          // mixing B: [column][pairs re | pairs im]
    static_assert(PART * 4 <= (int)sizeof(lds), "partial reduction does not fit the LDS operands");
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int r16 = lane & 15, k8 = 8 * (lane >> 4);
    floatx4 accw[NSL][MTX];
#pragma unroll
    for (int jj = 0; jj < NSL; ++jj)
#pragma unroll
        for (int mt = 0; mt < MTX; ++mt) accw[jj][mt] = floatx4{ 0.f, 0.f, 0.f, 0.f };
    // rows 2 CO .. 16 MTX - 1 of the x operand stay zero
    for (int i = threadIdx.x; i < (MTX * 16 - 2 * CO) * PK; i += NET_NT) Xa[2 * CO * PK + i] = (__bf16)0.f;
    auto put = [&](const float tv[4][6]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            __bf16 *row = Fb + (4 * q + i) * PK + 6 * lane;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                *reinterpret_cast<bf16x2 *>(row + 2 * a) = bf16x2{ (__bf16)tv[i][2 * a], (__bf16)tv[i][2 * a + 1] };
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            __bf16 *col = F + (3 * lane + a) * PB;
            const bf16x4 re = { (__bf16)tv[0][2 * a], (__bf16)tv[1][2 * a], (__bf16)tv[2][2 * a], (__bf16)tv[3][2 * a] };
            const bf16x4 im = { (__bf16)tv[0][2 * a + 1], (__bf16)tv[1][2 * a + 1], (__bf16)tv[2][2 * a + 1],
                                (__bf16)tv[3][2 * a + 1] };
            *reinterpret_cast<bf16x4 *>(col + 4 * q) = re;
            *reinterpret_cast<bf16x4 *>(col + 16 + 4 * q) = im;
        }
    };
    const int units = batch * 2 * g.ntiles;
    const int xcd = blockIdx.x % NXCD, per_xcd = gridDim.x / NXCD, units_per_xcd = (units + NXCD - 1) / NXCD;
#pragma unroll 1
    for (int v = blockIdx.x / NXCD; v < units_per_xcd; v += per_xcd) {
        const int u = xcd * units_per_xcd + v;
        if (u >= units) break;
        int b, tile, p;
        net_unit(u, g.ntiles, b, tile, p);
        const float2 *gb = gup + (size_t)b * CI * 2 * g.Vh * 3;
        const NetSite site = net_site(g, p, tile, lane);
        // the weights operand does not depend on the unit: an opaque copy of its
        // pointer keeps the compiler from hoisting every slice's load out of the
        // unit loop (72 registers held for the whole kernel)
        const __bf16 *Au = A;
        asm volatile("" : "+s"(Au));
        // x's rows [x_r, x_i] and [-x_i, x_r]; (the previous unit's last slice ended with a barrier: its
        // operands have been read)
        {
            TileFeat<CO> xt;
            tile_feat_load<CO>(g, x, b, p, tile, xt);
            tile_feat_put<CO, PK>(xt, Xa, -1.f, 1.f);
        }
        floatx4 acc[3][MTX];
#pragma unroll
        for (int n = 0; n < 3; ++n)
#pragma unroll
            for (int mt = 0; mt < MTX; ++mt) acc[n][mt] = floatx4{ 0.f, 0.f, 0.f, 0.f };
        {
            float tv[4][6];
            slice_transport<CI, false, CI == 1>(g, fat, gb, p, tile, lane, site, 0, q, tv);
            put(tv);
        }
        __syncthreads();  // x and slice 0 are in LDS
        // unrolled: accw[j >> 2] must stay in registers; slice j + 1's loads are in flight over slice j's MFMA
#pragma unroll
        for (int j = 0; j < S::N; ++j) {
            const bool more = j + 1 < S::N;
            // the next slice's transport goes to registers while this one is multiplied
            float tv[4][6];
            if (more) slice_transport<CI, false, CI == 1>(g, fat, gb, p, tile, lane, site, j + 1, q, tv);
            {  // mixing: the layer kernel's column tiles 3q..3q+2
                bf16x8 av[MTX];
#pragma unroll
                for (int mt = 0; mt < MTX; ++mt)
                    av[mt] = *reinterpret_cast<const bf16x8 *>(Au + ((size_t)j * MPAD + mt * 16 + r16) * SK + k8);
#pragma unroll
                for (int n = 0; n < 3; ++n) {
                    const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(F + ((3 * q + n) * 16 + r16) * PB + k8);
#pragma unroll
                    for (int mt = 0; mt < MTX; ++mt)
                        acc[n][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[mt], bv, acc[n][mt], 0, 0, 0);
                }
            }
            if (q == (j & 3)) {  // this slice's weight-gradient owner (wave-uniform)
#pragma unroll
                for (int ks = 0; ks < KT / SK; ++ks) {
                    const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(Fb + r16 * PK + SK * ks + k8);
#pragma unroll
                    for (int mt = 0; mt < MTX; ++mt) {
                        const bf16x8 av = *reinterpret_cast<const bf16x8 *>(Xa + (mt * 16 + r16) * PK + SK * ks + k8);
                        accw[j >> 2][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, accw[j >> 2][mt], 0, 0, 0);
                    }
                }
            }
            __syncthreads();  // every wave is done with slice j
            if (more) {
                put(tv);
                __syncthreads();
            }
        }
        // the unit's input gradient (the layer kernel's store)
#pragma unroll
        for (int n = 0; n < 3; ++n) {
            const int col = (3 * q + n) * 16 + r16, s = col / 3, a = col % 3, h = tile * TILE + s;
            if (h >= g.Vh) continue;
            if constexpr (CO == 16) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    dx[feat_idx(b, CO, 4 * (lane >> 4) + i, p, g.Vh, h) + a] = make_float2(acc[n][0][i], acc[n][1][i]);
                continue;
            }
            float *o = reinterpret_cast<float *>(dx);
#pragma unroll
            for (int mt = 0; mt < MTX; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int m = mt * 16 + 4 * (lane >> 4) + i;
                    if (m < 2 * CO) {
                        const int ch = m < CO ? m : m - CO;
                        o[2 * (feat_idx(b, CO, ch, p, g.Vh, h) + a) + (m < CO ? 0 : 1)] = acc[n][mt][i];
                    }
                }
        }
    }
    // scatter every owned (slice, row tile) into the forward layer's partial layout, then a coalesced store
    float *red = reinterpret_cast<float *>(lds);
    __syncthreads();
    for (int i = threadIdx.x; i < PART; i += NET_NT) red[i] = 0.f;
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < NSL; ++jj) {
        const int j = q + 4 * jj;
        if (j >= S::N) continue;
        const int kp = j * S::KG + r16 / CI, a = r16 % CI;  // column: pair (k', a) of the slice
        if (kp >= 9) continue;
        const int kf = ADJ[kp], jf = kf / KGF;
#pragma unroll
        for (int mt = 0; mt < MTX; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = mt * 16 + 4 * (lane >> 4) + i;
                if (row >= 2 * CO) continue;
                const bool re = row < CO;
                const int c = re ? row : row - CO, mf = re ? a : CI + a;
                const float val = kp ? -accw[jj][mt][i] : accw[jj][mt][i];
                red[((jf * MTF + mf / 16) * 16 + mf % 16) * 16 + (kf % KGF) * CO + c] = val;
            }
    }
    __syncthreads();
    float *dst = partials + (size_t)blockIdx.x * PART;
    for (int i = threadIdx.x; i < PART; i += NET_NT) dst[i] = red[i];
}

// grad_w from the per-workgroup partials [nblocks][PART] (FP32): each entry
// summed over the workgroups in FP64 in a fixed order -- a workgroup takes 64
// consecutive entries (coalesced reads), its four waves the workgroups g,
// g + 4, ... (four running sums each), the four groups added in order -- then
// written to its place: entry ((j MT + mt) 16 + r) 16 + pi is row m = 16 mt + r
// (Re of channel m, or Im of m - COUT) and pair pi (transport j KG + pi / CIN,
// channel pi % CIN) of slice j.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_net_wgrad_reduce(const float *__restrict__ partials, int nblocks,
                                                          float *__restrict__ gw)
{
    using S = Slices<CIN>;
    constexpr int MT = (2 * COUT + 15) / 16;
    constexpr int PART = S::N * MT * 256;
    const int l = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + l;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (e < PART) {
        int bl = grp;
        for (; bl + 12 < nblocks; bl += 16) {
            s0 += partials[(size_t)bl * PART + e];
            s1 += partials[(size_t)(bl + 4) * PART + e];
            s2 += partials[(size_t)(bl + 8) * PART + e];
            s3 += partials[(size_t)(bl + 12) * PART + e];
        }
        for (; bl < nblocks; bl += 4) s0 += partials[(size_t)bl * PART + e];
    }
    __shared__ double red[4][64];
    red[grp][l] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (grp || e >= PART) return;
    const double tot = ((red[0][l] + red[1][l]) + red[2][l]) + red[3][l];
    const int pi = e % 16, m = (e / 16) % (MT * 16), j = e / (16 * MT * 16);
    const int k = j * S::KG + pi / CIN, c = pi % CIN;
    if (m >= 2 * COUT || k >= 9) return;
    const int a = m < COUT ? m : m - COUT;
    // backward transports were taken without the packed sign (the weights carry it)
    gw[2 * (((size_t)k * COUT + a) * CIN + c) + (m < COUT ? 0 : 1)] = (float)(k >= 5 ? -tot : tot);
}

// ------------------------------------------------------------------ embedding, loss, Adam
// full[b][0][p][h] = (p == 0 ? even[b][h] : 0)
__global__ void k_net_embed(const float2 *__restrict__ even, float2 *__restrict__ full, int batch, int vh)
{
    const long long n = (long long)batch * 2 * vh * 3;
    for (long long i = threadIdx.x + (long long)blockIdx.x * blockDim.x; i < n; i += (long long)blockDim.x * gridDim.x) {
        const long long per = 2LL * vh * 3;
        const int b = (int)(i / per);
        const long long r = i % per;
        full[i] = r < (long long)vh * 3 ? even[(long long)b * vh * 3 + r] : make_float2(0.f, 0.f);
    }
}

__global__ void k_net_extract(const float2 *__restrict__ full, float2 *__restrict__ even, int batch, int vh)
{
    const long long n = (long long)batch * vh * 3;
    for (long long i = threadIdx.x + (long long)blockIdx.x * blockDim.x; i < n; i += (long long)blockDim.x * gridDim.x) {
        const int b = (int)(i / ((long long)vh * 3));
        even[i] = full[(long long)b * 2 * vh * 3 + i % ((long long)vh * 3)];
    }
}

// per-sample partial sums |y - x|^2 and |x|^2: partials[(b * nb + blk) * 2 + {0,1}]
__global__ __launch_bounds__(256) void k_net_lossparts(const float2 *__restrict__ y, const float2 *__restrict__ x,
                                                       int vh, double *partials)
{
    const int b = blockIdx.y, nb = gridDim.x;
    const long long n = (long long)vh * 3, off = (long long)b * n;
    double d = 0.0, xx = 0.0;
    for (long long i = threadIdx.x + (long long)blockIdx.x * 256; i < n; i += 256LL * nb) {
        const float2 yv = y[off + i], xv = x[off + i];
        const double dr = (double)yv.x - xv.x, di = (double)yv.y - xv.y;
        d = fma(dr, dr, fma(di, di, d));
        xx = fma((double)xv.x, xv.x, fma((double)xv.y, xv.y, xx));
    }
    __shared__ double lds[8];
    double sd = block_sum<256>(d, lds);
    double sx = block_sum<256>(xx, lds);
    if (threadIdx.x == 0) {
        partials[((size_t)b * nb + blockIdx.x) * 2] = sd;
        partials[((size_t)b * nb + blockIdx.x) * 2 + 1] = sx;
    }
}

// loss = mean_b d_b / xx_b ; coef_b = 2 / (batch xx_b); out[0] = loss, out[1 + b] = coef_b
__global__ __launch_bounds__(256) void k_net_lossfin(const double *__restrict__ partials, int nb, int batch,
                                                     double *out)
{
    __shared__ double lds[8];
    double loss = 0.0;
    for (int b = 0; b < batch; ++b) {
        double d = 0.0, xx = 0.0;
        for (int i = threadIdx.x; i < nb; i += 256) {
            d += partials[((size_t)b * nb + i) * 2];
            xx += partials[((size_t)b * nb + i) * 2 + 1];
        }
        d = block_sum<256>(d, lds);
        xx = block_sum<256>(xx, lds);
        if (threadIdx.x == 0) {
            loss += xx > 0 ? d / xx : 0.0;
            out[1 + b] = xx > 0 ? 2.0 / (batch * xx) : 0.0;
        }
    }
    if (threadIdx.x == 0) out[0] = loss / batch;
}

// g_b = coef_b (y_b - x_b) (even sites)
__global__ void k_net_lossgrad(const float2 *__restrict__ y, const float2 *__restrict__ x, const double *coef,
                               float2 *__restrict__ g, int batch, int vh)
{
    const long long n = (long long)batch * vh * 3;
    for (long long i = threadIdx.x + (long long)blockIdx.x * blockDim.x; i < n; i += (long long)blockDim.x * gridDim.x) {
        const int b = (int)(i / ((long long)vh * 3));
        const float c = (float)coef[1 + b];
        g[i] = make_float2(c * (y[i].x - x[i].x), c * (y[i].y - x[i].y));
    }
}

// Adam (Kingma & Ba 2014) on the real and imaginary parts
__global__ void k_net_adam(float *__restrict__ w, const float *__restrict__ gr, float *__restrict__ m,
                           float *__restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1,
                           float c2)
{
    for (long long i = threadIdx.x + (long long)blockIdx.x * blockDim.x; i < n; i += (long long)blockDim.x * gridDim.x) {
        const float gi = gr[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// ------------------------------------------------------------------ host side
static bool net_channels_ok(int C) { return C == 4 || C == 8 || C == 16; }

size_t net_weight_count_c(int C) { return 9ull * (C * 1 + C * C + C * C + 1 * C); }

// offsets (in complex numbers) of each layer's weights inside the flat array
static size_t w_off(int C, int layer)
{
    const size_t s[4] = { 9ull * C * 1, 9ull * C * C, 9ull * C * C, 9ull * 1 * C };
    size_t o = 0;
    for (int i = 0; i < layer; ++i) o += s[i];
    return o;
}

static size_t feat_bytes(const Geom &g, int batch, int C) { return (size_t)batch * C * 2 * g.Vh * 3 * 8; }
static size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }
constexpr size_t ABF_SLOT = (size_t)9 * MPAD * SK * 2;  // one layer's BF16 operand: up to 9 slices

size_t net_act_bytes_g(const Geom &g, int C, int batch)
{
    return 4 * a256(ABF_SLOT) + a256(feat_bytes(g, batch, 1)) * 2 + 3 * a256(feat_bytes(g, batch, C));
}

struct NetActs {
    __bf16 *A[4];
    float2 *in[4];  // layer inputs
    float2 *out;    // last layer output
};

static NetActs net_acts(void *acts, const Geom &g, int C, int batch)
{
    NetActs r;
    char *p = (char *)acts;
    for (int i = 0; i < 4; ++i) { r.A[i] = (__bf16 *)p; p += a256(ABF_SLOT); }
    r.in[0] = (float2 *)p; p += a256(feat_bytes(g, batch, 1));
    for (int i = 1; i < 4; ++i) { r.in[i] = (float2 *)p; p += a256(feat_bytes(g, batch, C)); }
    r.out = (float2 *)p;
    return r;
}

template <int CIN, int COUT>
static void layer_launch(const Geom &g, const void *fat, const float2 *in, float2 *out, const __bf16 *A, int batch,
                         hipStream_t s)
{
    const int grid = xcd_grid(batch * 2 * g.ntiles);
    hipLaunchKernelGGL((k_net_layer<CIN, COUT>), dim3(grid), dim3(NET_NT), 0, s, g, (const char *)fat, in, out, A,
                       batch);
}

template <int CIN>
static void layer_mt_launch(const Geom &g, const void *fat, const float2 *in, float2 *out, const float2 *W, int batch,
                            int adjoint, hipStream_t s)
{
    const int grid = xcd_grid(batch * 2 * g.ntiles);
    hipLaunchKernelGGL((k_net_layer_mt<CIN>), dim3(grid), dim3(NET_NT), 0, s, g, (const char *)fat, in, out, W, batch,
                       adjoint);
}

template <int CIN, int COUT>
static void prep_launch(const float2 *W, __bf16 *A, int adjoint, hipStream_t s)
{
    hipLaunchKernelGGL((k_net_prep<CIN, COUT>), dim3(8), dim3(256), 0, s, W, A, adjoint);
}

// The BF16 weight operands of layers 1-3 (layer 4 reads its FP32 weights).
template <int C>
static void net_prep_t(const float2 *W, const NetActs &a, hipStream_t s)
{
    prep_launch<1, C>(W + w_off(C, 0), a.A[0], 0, s);
    prep_launch<C, C>(W + w_off(C, 1), a.A[1], 0, s);
    prep_launch<C, C>(W + w_off(C, 2), a.A[2], 0, s);
}

// The four layers, from the embedded input slot to the last layer's output slot.
template <int C>
static void net_layers_t(const Geom &g, const void *fat, const float2 *W, const NetActs &a, int batch, hipStream_t s)
{
    layer_launch<1, C>(g, fat, a.in[0], a.in[1], a.A[0], batch, s);
    layer_launch<C, C>(g, fat, a.in[1], a.in[2], a.A[1], batch, s);
    layer_launch<C, C>(g, fat, a.in[2], a.in[3], a.A[2], batch, s);
    layer_mt_launch<C>(g, fat, a.in[3], a.out, W + w_off(C, 3), batch, 0, s);
}

template <int C>
static int net_forward_t(const Geom &g, const void *fat, const float2 *W, const float2 *in_even, float2 *out_even,
                         void *acts, int batch, hipStream_t s)
{
    NetActs a = net_acts(acts, g, C, batch);
    net_prep_t<C>(W, a, s);
    const long long ne = (long long)batch * 2 * g.Vh * 3;
    const int nb = (int)std::min<long long>((ne + 255) / 256, 4096);
    hipLaunchKernelGGL(k_net_embed, dim3(nb), dim3(256), 0, s, in_even, a.in[0], batch, g.Vh);
    net_layers_t<C>(g, fat, W, a, batch, s);
    if (out_even) hipLaunchKernelGGL(k_net_extract, dim3(nb), dim3(256), 0, s, (const float2 *)a.out, out_even, batch, g.Vh);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

static_assert(WG_MAX_BLOCKS % NXCD == 0, "the weight-gradient grid is a whole number of XCD groups");
constexpr size_t WG_PART_FLOATS = (size_t)9 * 2 * 256;  // the largest per-block partial (9 slices, 32 rows)

// A persistent weight-gradient grid: the workgroups of `kern` that are
// resident at once (occupancy x CUs, found once per kernel), at most one per
// unit and WG_MAX_BLOCKS, rounded up to a whole number of XCD groups.
static int persistent_blocks(const void *kern, int &resident, const Geom &g, int batch)
{
    if (!resident) {
        int occ = 0, cus = 0, dev = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, NET_NT, 0) != hipSuccess || occ <= 0) occ = 1;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        resident = occ * cus;
    }
    const long long units = (long long)batch * 2 * g.ntiles;
    return xcd_grid((int)std::min<long long>(std::min<long long>(units, resident), WG_MAX_BLOCKS));
}
template <int CIN, int COUT>
static int wgrad_blocks(const Geom &g, int batch)
{
    static int resident = 0;
    return persistent_blocks((const void *)k_net_wgrad<CIN, COUT>, resident, g, batch);
}
template <int CI, int CO>
static int bwd_blocks(const Geom &g, int batch)
{
    static int resident = 0;
    return persistent_blocks((const void *)k_net_bwd<CI, CO>, resident, g, batch);
}

// Backward workspace: dl/d in4, dl/d in3, dl/d in2 (C channels each), dl/d out
// (the embedded gradient) and dl/d in1 (one channel each), every block at a
// multiple of 256 bytes; then the weight-gradient partials and the four BF16
// operands of the adjoint layers.
struct NetGrads {
    float2 *gin[4];  // gin[l] = dl/d (input of layer l + 1)
    float2 *gout;    // dl/d (output of layer 4), full lattice
    float *part;
    __bf16 *A[4];
};

static NetGrads net_grads(void *ws, const Geom &g, int C, int batch)
{
    NetGrads r;
    char *p = (char *)ws;
    for (int l = 3; l >= 1; --l) { r.gin[l] = (float2 *)p; p += a256(feat_bytes(g, batch, C)); }
    r.gout = (float2 *)p; p += a256(feat_bytes(g, batch, 1));
    r.gin[0] = (float2 *)p; p += a256(feat_bytes(g, batch, 1));
    r.part = (float *)p; p += a256((size_t)WG_MAX_BLOCKS * WG_PART_FLOATS * sizeof(float));
    for (int i = 0; i < 4; ++i) { r.A[i] = (__bf16 *)p; p += a256(ABF_SLOT); }
    return r;
}

size_t net_bwd_ws_bytes_g(const Geom &g, int C, int batch)
{
    return 3 * a256(feat_bytes(g, batch, C)) + 2 * a256(feat_bytes(g, batch, 1)) +
           a256((size_t)WG_MAX_BLOCKS * WG_PART_FLOATS * sizeof(float)) + 4 * a256(ABF_SLOT);
}

template <int CIN, int COUT>
static void wgrad_launch(const Geom &g, const void *fat, const float2 *in, const float2 *gout, int batch, float *part,
                         float2 *gw, hipStream_t s)
{
    const int nb = wgrad_blocks<CIN, COUT>(g, batch);
    hipLaunchKernelGGL((k_net_wgrad<CIN, COUT>), dim3(nb), dim3(NET_NT), 0, s, g, (const char *)fat, in, gout, batch,
                       part);
    constexpr int part_entries = Slices<CIN>::N * ((2 * COUT + 15) / 16) * 256;
    hipLaunchKernelGGL((k_net_wgrad_reduce<CIN, COUT>), dim3((part_entries + 63) / 64), dim3(256), 0, s,
                       (const float *)part, nb, (float *)gw);
}

// The backward of a layer with input x (CO channels) and upstream gradient
// gup (CI channels): dx through the adjoint layer and the layer's weight
// gradient from the same transports of gup (k_net_bwd), then the fixed-order
// reduction of the partials in the layout of the forward layer <CO, CI>.
template <int CI, int CO>
static void bwd_launch(const Geom &g, const void *fat, const float2 *gup, const float2 *x, float2 *dx,
                       const __bf16 *A, int batch, float *part, float2 *gw, hipStream_t s)
{
    const int nb = bwd_blocks<CI, CO>(g, batch);
    hipLaunchKernelGGL((k_net_bwd<CI, CO>), dim3(nb), dim3(NET_NT), 0, s, g, (const char *)fat, gup, x, dx, A, batch,
                       part);
    constexpr int part_entries = Slices<CO>::N * ((2 * CI + 15) / 16) * 256;
    hipLaunchKernelGGL((k_net_wgrad_reduce<CO, CI>), dim3((part_entries + 63) / 64), dim3(256), 0, s,
                       (const float *)part, nb, (float *)gw);
}

template <int C>
static int net_backward_t(const Geom &g, const void *fat, const float2 *W, const void *acts, const float2 *gout_even,
                          float2 *gw, float2 *gin_even, int batch, void *ws, hipStream_t s)
{
    NetActs a = net_acts(const_cast<void *>(acts), g, C, batch);
    NetGrads d = net_grads(ws, g, C, batch);
    const long long ne = (long long)batch * 2 * g.Vh * 3;
    const int nb = (int)std::min<long long>((ne + 255) / 256, 4096);
    // gradient of the last layer's output: even part given, odd part zero
    hipLaunchKernelGGL(k_net_embed, dim3(nb), dim3(256), 0, s, gout_even, d.gout, batch, g.Vh);
    prep_launch<C, 1>(W + w_off(C, 3), d.A[3], 1, s);
    prep_launch<C, C>(W + w_off(C, 2), d.A[2], 1, s);
    prep_launch<C, C>(W + w_off(C, 1), d.A[1], 1, s);
    // layers 4, 3, 2: dl/d in and dl/dW from one set of transports of the upstream gradient
    bwd_launch<1, C>(g, fat, d.gout, a.in[3], d.gin[3], d.A[3], batch, d.part, gw + w_off(C, 3), s);
    bwd_launch<C, C>(g, fat, d.gin[3], a.in[2], d.gin[2], d.A[2], batch, d.part, gw + w_off(C, 2), s);
    bwd_launch<C, C>(g, fat, d.gin[2], a.in[1], d.gin[1], d.A[1], batch, d.part, gw + w_off(C, 1), s);
    // layer 1 (one input channel): its weight gradient transports the input instead
    wgrad_launch<1, C>(g, fat, a.in[0], d.gin[1], batch, d.part, gw + w_off(C, 0), s);
    if (gin_even) {
        layer_mt_launch<C>(g, fat, d.gin[1], d.gin[0], W + w_off(C, 0), batch, 1, s);  // dl/d in1 (C -> 1)
        hipLaunchKernelGGL(k_net_extract, dim3(nb), dim3(256), 0, s, (const float2 *)d.gin[0], gin_even, batch, g.Vh);
    }
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

// For a caller that applies the network repeatedly with fixed weights (the
// flexible CG): the weight operands once (net_prep_dispatch), then per
// application the four layers alone (net_layers_dispatch), reading the
// embedded input slot of `acts` and leaving the last layer's full-lattice
// output in its output slot; net_acts_io gives both slots ([batch][1][parity]
// [Vh][3] complex64, even parity first).
int net_prep_dispatch(const Geom &g, const void *W, int C, void *acts, int batch, hipStream_t s)
{
    switch (C) {
    case 4: net_prep_t<4>((const float2 *)W, net_acts(acts, g, 4, batch), s); break;
    case 8: net_prep_t<8>((const float2 *)W, net_acts(acts, g, 8, batch), s); break;
    default: net_prep_t<16>((const float2 *)W, net_acts(acts, g, 16, batch), s); break;
    }
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

int net_layers_dispatch(const Geom &g, const void *fat, const void *W, int C, void *acts, int batch, hipStream_t s)
{
    switch (C) {
    case 4: net_layers_t<4>(g, fat, (const float2 *)W, net_acts(acts, g, 4, batch), batch, s); break;
    case 8: net_layers_t<8>(g, fat, (const float2 *)W, net_acts(acts, g, 8, batch), batch, s); break;
    default: net_layers_t<16>(g, fat, (const float2 *)W, net_acts(acts, g, 16, batch), batch, s); break;
    }
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

void net_acts_io(void *acts, const Geom &g, int C, int batch, void **in_full, void **out_full)
{
    const NetActs a = net_acts(acts, g, C, batch);
    *in_full = a.in[0];
    *out_full = a.out;
}

int net_forward_dispatch(const Geom &g, const void *fat, const void *W, int C, const void *in_even, void *out_even,
                         void *acts, int batch, hipStream_t s)
{
    switch (C) {
    case 4: return net_forward_t<4>(g, fat, (const float2 *)W, (const float2 *)in_even, (float2 *)out_even, acts, batch, s);
    case 8: return net_forward_t<8>(g, fat, (const float2 *)W, (const float2 *)in_even, (float2 *)out_even, acts, batch, s);
    default: return net_forward_t<16>(g, fat, (const float2 *)W, (const float2 *)in_even, (float2 *)out_even, acts, batch, s);
    }
}

}  // namespace hisq

using namespace hisq;

extern "C" size_t net_weight_count(int channels) { return net_channels_ok(channels) ? net_weight_count_c(channels) : 0; }

extern "C" size_t net_act_bytes(const int dims[4], int channels, int batch)
{
    Geom g;
    if (make_geom(dims, g) || !net_channels_ok(channels) || batch < 1) return 0;
    return net_act_bytes_g(g, channels, batch);
}

extern "C" size_t net_backward_ws_bytes(const int dims[4], int channels, int batch)
{
    Geom g;
    if (make_geom(dims, g) || !net_channels_ok(channels) || batch < 1) return 0;
    return net_bwd_ws_bytes_g(g, channels, batch);
}

extern "C" int net_forward(const void *fat, const void *weights, int channels, const void *in, void *out, void *acts,
                           size_t act_bytes, int batch, const int dims[4], void *stream)
{
    Geom g;
    int rc = make_geom(dims, g);
    if (rc) return rc;
    if (!net_channels_ok(channels)) return fail(HISQ_EINVAL, "net_forward: channels must be 4, 8 or 16");
    if (batch < 1) return fail(HISQ_EINVAL, "net_forward: batch must be >= 1");
    if (!fat || !weights || !in || !acts) return fail(HISQ_EINVAL, "net_forward: NULL pointer");
    if (act_bytes < net_act_bytes_g(g, channels, batch)) return fail(HISQ_EWORKSPACE, "net_forward: acts buffer too small");
    if (!aligned16({fat, weights, in, out, acts}))
        return fail(HISQ_EINVAL, "net_forward: device pointers must be 16-byte aligned");
    if (in == out) return fail(HISQ_EALIAS, "net_forward: in and out alias");
    return net_forward_dispatch(g, fat, weights, channels, in, out, acts, batch, (hipStream_t)stream);
}

extern "C" int net_backward(const void *fat, const void *weights, int channels, const void *acts, size_t act_bytes,
                            const void *grad_out, void *grad_w, void *grad_in, int batch, const int dims[4],
                            void *workspace, size_t ws_bytes, void *stream)
{
    Geom g;
    int rc = make_geom(dims, g);
    if (rc) return rc;
    if (!net_channels_ok(channels)) return fail(HISQ_EINVAL, "net_backward: channels must be 4, 8 or 16");
    if (batch < 1) return fail(HISQ_EINVAL, "net_backward: batch must be >= 1");
    if (!fat || !weights || !acts || !grad_out || !grad_w || !workspace) return fail(HISQ_EINVAL, "net_backward: NULL pointer");
    if (act_bytes < net_act_bytes_g(g, channels, batch)) return fail(HISQ_EWORKSPACE, "net_backward: acts buffer too small");
    if (ws_bytes < net_bwd_ws_bytes_g(g, channels, batch)) return fail(HISQ_EWORKSPACE, "net_backward: workspace too small");
    if (!aligned16({fat, weights, acts, grad_out, grad_w, grad_in, workspace}))
        return fail(HISQ_EINVAL, "net_backward: device pointers must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    switch (channels) {
    case 4: return net_backward_t<4>(g, fat, (const float2 *)weights, acts, (const float2 *)grad_out, (float2 *)grad_w, (float2 *)grad_in, batch, workspace, s);
    case 8: return net_backward_t<8>(g, fat, (const float2 *)weights, acts, (const float2 *)grad_out, (float2 *)grad_w, (float2 *)grad_in, batch, workspace, s);
    default: return net_backward_t<16>(g, fat, (const float2 *)weights, acts, (const float2 *)grad_out, (float2 *)grad_w, (float2 *)grad_in, batch, workspace, s);
    }
}

extern "C" int net_transport(const void *fat, const void *in, void *out, int channels, int batch, const int dims[4],
                             void *stream)
{
    Geom g;
    int rc = make_geom(dims, g);
    if (rc) return rc;
    if (channels != 1 && !net_channels_ok(channels)) return fail(HISQ_EINVAL, "net_transport: channels must be 1, 4, 8 or 16");
    if (batch < 1) return fail(HISQ_EINVAL, "net_transport: batch must be >= 1");
    if (!fat || !in || !out) return fail(HISQ_EINVAL, "net_transport: NULL pointer");
    if (!aligned16({fat, in, out}))
        return fail(HISQ_EINVAL, "net_transport: device pointers must be 16-byte aligned");
    if (in == out) return fail(HISQ_EALIAS, "net_transport: in and out alias");
    const dim3 grid(g.ntiles, 2, batch);
    hipStream_t s = (hipStream_t)stream;
    switch (channels) {
    case 1: hipLaunchKernelGGL((k_net_transport<1>), grid, dim3(NET_NT), 0, s, g, (const char *)fat, (const float2 *)in, (float2 *)out); break;
    case 4: hipLaunchKernelGGL((k_net_transport<4>), grid, dim3(NET_NT), 0, s, g, (const char *)fat, (const float2 *)in, (float2 *)out); break;
    case 8: hipLaunchKernelGGL((k_net_transport<8>), grid, dim3(NET_NT), 0, s, g, (const char *)fat, (const float2 *)in, (float2 *)out); break;
    default: hipLaunchKernelGGL((k_net_transport<16>), grid, dim3(NET_NT), 0, s, g, (const char *)fat, (const float2 *)in, (float2 *)out);
    }
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

extern "C" int net_loss(const void *y, const void *x, int batch, const int dims[4], double *loss_host, void *grad_y,
                        void *workspace, size_t ws_bytes, void *stream)
{
    Geom g;
    int rc = make_geom(dims, g);
    if (rc) return rc;
    if (!y || !x || batch < 1) return fail(HISQ_EINVAL, "net_loss: bad argument");
    if (!aligned16({y, x, grad_y, workspace}))
        return fail(HISQ_EINVAL, "net_loss: device pointers must be 16-byte aligned");
    const int nb = 64;
    const size_t need = a256((size_t)batch * nb * 2 * sizeof(double)) + a256((size_t)(batch + 1) * sizeof(double));
    if (!workspace || ws_bytes < need) return fail(HISQ_EWORKSPACE, "net_loss: workspace too small");
    double *part = (double *)workspace;
    double *out = (double *)((char *)workspace + a256((size_t)batch * nb * 2 * sizeof(double)));
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_net_lossparts, dim3(nb, batch), dim3(256), 0, s, (const float2 *)y, (const float2 *)x, g.Vh, part);
    hipLaunchKernelGGL(k_net_lossfin, dim3(1), dim3(256), 0, s, (const double *)part, nb, batch, out);
    if (grad_y) {
        const long long n = (long long)batch * g.Vh * 3;
        hipLaunchKernelGGL(k_net_lossgrad, dim3((unsigned)std::min<long long>((n + 255) / 256, 4096)), dim3(256), 0, s,
                           (const float2 *)y, (const float2 *)x, (const double *)out, (float2 *)grad_y, batch, g.Vh);
    }
    HISQ_HIP(hipGetLastError());
    if (loss_host) {
        HISQ_HIP(hipMemcpyAsync(loss_host, out, sizeof(double), hipMemcpyDeviceToHost, s));
        HISQ_HIP(hipStreamSynchronize(s));
    }
    return HISQ_OK;
}

extern "C" int net_adam_step(void *weights, const void *grad_w, void *m, void *v, long long n_complex, double lr,
                             int step, void *stream)
{
    if (!weights || !grad_w || !m || !v || n_complex <= 0 || step < 1 || !(lr > 0))
        return fail(HISQ_EINVAL, "net_adam_step: bad argument");
    if (!aligned16({weights, grad_w, m, v}))
        return fail(HISQ_EINVAL, "net_adam_step: device pointers must be 16-byte aligned");
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow(0.9, step)), c2 = (float)(1.0 - std::pow(0.999, step));
    const long long n = 2 * n_complex;
    hipLaunchKernelGGL(k_net_adam, dim3((unsigned)std::min<long long>((n + 255) / 256, 1024)), dim3(256), 0,
                       (hipStream_t)stream, (float *)weights, (const float *)grad_w, (float *)m, (float *)v, n,
                       (float)lr, b1, b2, 1e-8f, c1, c2);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}
