// Internal definitions shared by the HIP sources of libhisq.so (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstddef>
#include <cstdint>
#include <initializer_list>
#include <string>

#include "../../include/hisq.h"

namespace hisq {

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
// The kernels read fields, links and workspaces with 16-byte loads: every
// device pointer an entry point takes must be 16-byte aligned (device
// allocations are 256-byte aligned).  NULL counts as aligned.
inline bool aligned16(std::initializer_list<const void *> ps)
{
    for (const void *p : ps)
        if (reinterpret_cast<uintptr_t>(p) & 15) return false;
    return true;
}

#define HISQ_HIP(call)                                        \
    do {                                                      \
        hipError_t _e = (call);                               \
        if (_e != hipSuccess) return ::hisq::hip_fail(_e, #call); \
    } while (0)

// ------------------------------------------------------------------ geometry
// Sites of one parity are numbered h = lex >> 1; a tile is 64 consecutive h
// (one wavefront), the unit of the packed link layout.
constexpr int TILE = 64;

struct Geom {
    int L[4];    // Lx, Ly, Lz, Lt
    int Lxh;     // Lx / 2
    int Vh;      // sites per parity
    int ntiles;  // ceil(Vh / 64)
    int sy, sz, st;  // h-strides of y, z, t: Lxh, Lxh*Ly, Lxh*Ly*Lz
    // Tile processing order (oP == 0: tile k is processed k-th).  Blocked:
    // the oP tiles of one (z, t) plane, then otb planes along t, then ozb
    // along z, then the next t block, then the next z block, so that the
    // +-1 and +-3 neighbours in t and z of the tiles in flight were read a
    // few hundred tiles earlier and are still in L2.
    int oP, otb, ozb, ontb;
};

int make_geom(const int dims[4], Geom &g);  // HISQ_OK or HISQ_EDIMS/EINVAL
// Switch g to the blocked tile order; false (g unchanged) when a tile would
// straddle two (z, t) planes (Lx/2 * Ly not a multiple of 64).
bool blocked_order(Geom &g);
// Tile orders of the Dslash-type kernels: 0 plain; 1 blocked in the default
// (z, t) blocks (blocked_order); 2, 3, 4 blocks of 8, 4, 2 t-planes by the
// whole z extent; 5 blocks of 8 t- by 16 z-planes.  The XCDs take contiguous
// ranges of the order, so with 2-4 each XCD still holds whole t-slabs while t
// is the fast direction inside them.  g is left in plain order where the
// lattice does not allow the requested one.
void apply_order(Geom &g, int order);

// tile processed k-th
__device__ __forceinline__ int tile_of(const Geom &g, int k)
{
    if (g.oP == 0) return k;
    const int p = k % g.oP;
    int r = k / g.oP;
    const int ti = r % g.otb;
    r /= g.otb;
    const int zi = r % g.ozb;
    r /= g.ozb;
    const int tB = r % g.ontb, zB = r / g.ontb;
    return p + g.oP * (zB * g.ozb + zi + g.L[2] * (tB * g.otb + ti));
}

// Packed bytes per (tile, direction) block and per field.
size_t dir_block_bytes(int prec);
size_t packed_field_bytes(const Geom &g, int prec);

__device__ __forceinline__ void site_coords(const Geom &g, int h, int parity, int &x, int &y, int &z, int &t)
{
    int r = h / g.Lxh;
    int xh = h - r * g.Lxh;
    y = r % g.L[1];
    int r2 = r / g.L[1];
    z = r2 % g.L[2];
    t = r2 / g.L[2];
    x = 2 * xh + ((parity + y + z + t) & 1);
}

__device__ __forceinline__ int wrap(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

// h of the neighbour n + k * mu-hat (|k| <= 3 < L).  The neighbour has the
// opposite parity when k is odd.
__device__ __forceinline__ int nbr_h(const Geom &g, int h, int x, int y, int z, int t, int mu, int k)
{
    switch (mu) {
    case 0: {
        int xn = wrap(x + k, g.L[0]);
        return h - (x >> 1) + (xn >> 1);
    }
    case 1: return h + (wrap(y + k, g.L[1]) - y) * g.sy;
    case 2: return h + (wrap(z + k, g.L[2]) - z) * g.sz;
    default: return h + (wrap(t + k, g.L[3]) - t) * g.st;
    }
}

// XCD-aware workgroup order: the dispatcher hands consecutive workgroups to
// the 8 XCDs in turn, so logical block b' = (b % 8) * (G / 8) + b / 8 gives
// each XCD one contiguous slab of the lattice (its L2 then holds the slab's
// neighbour vectors).  G is the launched grid, a multiple of 8.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_block(int b, int G) { return (b % NXCD) * (G / NXCD) + b / NXCD; }
inline int xcd_grid(int nblocks) { return (nblocks + NXCD - 1) / NXCD * NXCD; }

// Occupancy target: at least W wavefronts per SIMD, i.e. at most 512/W VGPRs.
// The Dslash kernels are latency-bound streams; 8 waves/SIMD keeps a whole
// 32^4 half-lattice (8192 waves) resident in one round.
#define HISQ_WAVES(W) __attribute__((amdgpu_waves_per_eu(W)))

// ------------------------------------------------------------------ reductions
// Wave64 sum by butterfly (xor) shuffles: every lane gets the total.  The
// order is fixed, so results are reproducible.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide fixed-order sum; result valid in thread 0.  `lds` holds one
// double per wave.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) s += lds[i];
    }
    __syncthreads();
    return s;
}

template <int NT>
__device__ __forceinline__ void block_sum2(double &a, double &b, double *lds)
{
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { lds[2 * w] = a; lds[2 * w + 1] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) { sa += lds[2 * i]; sb += lds[2 * i + 1]; }
        a = sa;
        b = sb;
    }
    __syncthreads();
}

// First stage of a deterministic grid reduction: each block writes its
// fixed-order partial sum to partials[blk].  A one-block finalize kernel
// launched after it sums the partials in a fixed order.  (A last-block-done
// scheme would need a device-scope release fence per block, which on a
// multi-XCD part writes back the L2 each time; a separate kernel needs one
// kernel boundary.)
template <int NT>
__device__ __forceinline__ void block_partial(double v, double *partials, int blk)
{
    __shared__ double lds[NT / 64];
    double s = block_sum<NT>(v, lds);
    if (threadIdx.x == 0) partials[blk] = s;
}

// acc[r] += p[i * W + r] for r < W and i = threadIdx.x, threadIdx.x + NT, ...
// < n, in increasing i.  U rows are loaded before any is added, so a thread
// has U * W loads in flight per round trip (a plain strided loop waits for
// each load before the next: one memory latency per row).  The order of the
// additions is that of the plain loop, so the sums are the same to the bit.
template <int NT, int W, int U>
__device__ __forceinline__ void strided_sums(const double *__restrict__ p, int n, double acc[W])
{
    for (int i0 = threadIdx.x; i0 < n; i0 += U * NT) {
        double v[U][W];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * NT;
#pragma unroll
            for (int r = 0; r < W; ++r) v[u][r] = i < n ? p[(size_t)i * W + r] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (i0 + u * NT < n) {
#pragma unroll
                for (int r = 0; r < W; ++r) acc[r] += v[u][r];
            }
        }
    }
}


// ------------------------------------------------------------------ streaming loads / stores
// Nontemporal (streaming) accesses on native clang vectors; the HIP vector
// structs are reinterpreted as those.
typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf2 __attribute__((ext_vector_type(2)));
typedef float nf4 __attribute__((ext_vector_type(4)));
typedef unsigned nu2 __attribute__((ext_vector_type(2)));
typedef unsigned nu4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 ntload(const double2 *p)
{
    nd2 v = __builtin_nontemporal_load(reinterpret_cast<const nd2 *>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 ntload(const float2 *p)
{
    nf2 v = __builtin_nontemporal_load(reinterpret_cast<const nf2 *>(p));
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ float4 ntload(const float4 *p)
{
    nf4 v = __builtin_nontemporal_load(reinterpret_cast<const nf4 *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint2 ntload(const uint2 *p)
{
    nu2 v = __builtin_nontemporal_load(reinterpret_cast<const nu2 *>(p));
    return make_uint2(v.x, v.y);
}
__device__ __forceinline__ uint4 ntload(const uint4 *p)
{
    nu4 v = __builtin_nontemporal_load(reinterpret_cast<const nu4 *>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float ntload(const float *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void ntstore(double2 v, double2 *p)
{
    nd2 w = { v.x, v.y };
    __builtin_nontemporal_store(w, reinterpret_cast<nd2 *>(p));
}
__device__ __forceinline__ void ntstore(float2 v, float2 *p)
{
    nf2 w = { v.x, v.y };
    __builtin_nontemporal_store(w, reinterpret_cast<nf2 *>(p));
}

// ------------------------------------------------------------------ precision traits
// Packed link block of one (tile, direction): the 9 complex entries of the
// 64 sites' matrices in element planes, each plane contiguous over the 64
// lanes so that one wavefront load instruction reads one contiguous span.
//   F64 : 9 planes of double2                        (9216 B)
//   F32 : 4 planes of float4 (entries 2q, 2q+1) + 1 plane of float2 (entry 8)   (4608 B)
//   F16S: 2 planes of 4 x half2 (entries 0-3, 4-7) + 1 plane {half2 entry 8, float scale} (2560 B)
struct PF64 {
    static constexpr bool two_row = false;
    using real = double;
    using cvec = double2;
    static constexpr int prec = HISQ_F64;
    static constexpr size_t block_bytes = 9 * TILE * 16;
    using Fat = PF64;
    using Long = PF64;
    static constexpr size_t tile_bytes = 8 * block_bytes;  // the 8 directions of one 64-site tile
    __device__ __forceinline__ static void load_dir(const char *tile, int d, int lane, real m[18])
    {
        load(tile + (size_t)d * block_bytes, lane, m);
    }
    __device__ __forceinline__ static void load(const char *blk, int lane, double m[18])
    {
        const double2 *p = reinterpret_cast<const double2 *>(blk) + lane;
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            double2 v = ntload(p + e * TILE);
            m[2 * e] = v.x;
            m[2 * e + 1] = v.y;
        }
    }
};

struct PF32 {
    static constexpr bool two_row = false;
    using real = float;
    using cvec = float2;
    static constexpr int prec = HISQ_F32;
    static constexpr size_t block_bytes = TILE * 72;
    using Fat = PF32;
    using Long = PF32;
    static constexpr size_t tile_bytes = 8 * block_bytes;  // the 8 directions of one 64-site tile
    __device__ __forceinline__ static void load_dir(const char *tile, int d, int lane, real m[18])
    {
        load(tile + (size_t)d * block_bytes, lane, m);
    }
    __device__ __forceinline__ static void load(const char *blk, int lane, float m[18])
    {
        const float4 *p4 = reinterpret_cast<const float4 *>(blk) + lane;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float4 v = ntload(p4 + q * TILE);
            m[4 * q] = v.x; m[4 * q + 1] = v.y; m[4 * q + 2] = v.z; m[4 * q + 3] = v.w;
        }
        const float2 *p2 = reinterpret_cast<const float2 *>(blk + 4 * TILE * 16) + lane;
        float2 v = ntload(p2);
        m[16] = v.x;
        m[17] = v.y;
    }
};

struct PF16S {
    static constexpr bool two_row = false;
    using real = float;
    using cvec = float2;
    static constexpr int prec = HISQ_F16S;
    static constexpr size_t block_bytes = TILE * 40;
    using Fat = PF16S;
    using Long = PF16S;
    static constexpr size_t tile_bytes = 8 * block_bytes;  // the 8 directions of one 64-site tile
    __device__ __forceinline__ static void load_dir(const char *tile, int d, int lane, real m[18])
    {
        load(tile + (size_t)d * block_bytes, lane, m);
    }
    __device__ __forceinline__ static void load(const char *blk, int lane, float m[18])
    {
        const uint4 *p4 = reinterpret_cast<const uint4 *>(blk) + lane;
        uint4 a = ntload(p4);
        uint4 b = ntload(p4 + TILE);
        const uint2 *p2 = reinterpret_cast<const uint2 *>(blk + 2 * TILE * 16) + lane;
        uint2 c = ntload(p2);
        const float s = __uint_as_float(c.y);
        const unsigned w[9] = { a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x };
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            __half2 hv = *reinterpret_cast<const __half2 *>(&w[e]);
            float2 f = __half22float2(hv);
            m[2 * e] = f.x * s;
            m[2 * e + 1] = f.y * s;
        }
    }
};

// 16-bit fixed point with the same per-matrix FP32 scale: entry = q * scale / 32767,
// |q| <= 32767.  Same 40 B per matrix as PF16S, 16x finer steps for entries near
// the scale (bounded values do not need an exponent).
struct PI16S {
    static constexpr bool two_row = false;
    using real = float;
    using cvec = float2;
    static constexpr int prec = HISQ_I16S;
    static constexpr size_t block_bytes = TILE * 40;
    using Fat = PI16S;
    using Long = PI16S;
    static constexpr size_t tile_bytes = 8 * block_bytes;  // the 8 directions of one 64-site tile
    __device__ __forceinline__ static void load_dir(const char *tile, int d, int lane, real m[18])
    {
        load(tile + (size_t)d * block_bytes, lane, m);
    }
    __device__ __forceinline__ static void load(const char *blk, int lane, float m[18])
    {
        const uint4 *p4 = reinterpret_cast<const uint4 *>(blk) + lane;
        uint4 a = ntload(p4);
        uint4 b = ntload(p4 + TILE);
        const uint2 *p2 = reinterpret_cast<const uint2 *>(blk + 2 * TILE * 16) + lane;
        uint2 c = ntload(p2);
        const float s = __uint_as_float(c.y) * (1.0f / 32767.0f);
        const unsigned w[9] = { a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x };
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            m[2 * e] = (float)(short)(w[e] & 0xFFFFu) * s;
            m[2 * e + 1] = (float)(short)(w[e] >> 16) * s;
        }
    }
};

// Two-row form of a long (three-link) matrix that is +-SU(3) (Sec. 4: store two
// rows, rebuild the third; the staggered phase and boundary sign enter the
// rebuild): rows 0 and 1 are stored, row 2 = c conj(row0 x row1) with c = det
// = +-1 kept as one bit per lane in a 64-bit word per direction after the
// tile's 8 direction blocks.
__device__ __forceinline__ unsigned long long sign_word(const char *tile, size_t block_bytes, int d)
{
    return *reinterpret_cast<const unsigned long long *>(tile + 8 * block_bytes + 8 * (size_t)d);
}

template <class R>
__device__ __forceinline__ void third_row(R m[18], R c)
{
    // r0 = m[0..5], r1 = m[6..11] (re, im pairs); x = r0 x r1 ; row2 = c * conj(x)
    const R a0r = m[0], a0i = m[1], a1r = m[2], a1i = m[3], a2r = m[4], a2i = m[5];
    const R b0r = m[6], b0i = m[7], b1r = m[8], b1i = m[9], b2r = m[10], b2i = m[11];
    const R x0r = (a1r * b2r - a1i * b2i) - (a2r * b1r - a2i * b1i);
    const R x0i = (a1r * b2i + a1i * b2r) - (a2r * b1i + a2i * b1r);
    const R x1r = (a2r * b0r - a2i * b0i) - (a0r * b2r - a0i * b2i);
    const R x1i = (a2r * b0i + a2i * b0r) - (a0r * b2i + a0i * b2r);
    const R x2r = (a0r * b1r - a0i * b1i) - (a1r * b0r - a1i * b0i);
    const R x2i = (a0r * b1i + a0i * b1r) - (a1r * b0i + a1i * b0r);
    m[12] = c * x0r; m[13] = -c * x0i;
    m[14] = c * x1r; m[15] = -c * x1i;
    m[16] = c * x2r; m[17] = -c * x2i;
}

struct PF64R {
    using real = double;
    using cvec = double2;
    static constexpr size_t block_bytes = 6 * TILE * 16;
    static constexpr bool two_row = true;
    static constexpr size_t tile_bytes = 8 * block_bytes + 64;
    // rows 0 and 1 into m[0..11]; returns the sign c of the third row
    __device__ __forceinline__ static double load_rows(const char *tile, int d, int lane, double m[12])
    {
        const double2 *p = reinterpret_cast<const double2 *>(tile + (size_t)d * block_bytes) + lane;
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            double2 v = ntload(p + e * TILE);
            m[2 * e] = v.x;
            m[2 * e + 1] = v.y;
        }
        return ((sign_word(tile, block_bytes, d) >> lane) & 1ull) ? -1.0 : 1.0;
    }
    __device__ __forceinline__ static void load_dir(const char *tile, int d, int lane, double m[18])
    {
        const double c = load_rows(tile, d, lane, m);
        third_row<double>(m, c);
    }
};

struct PF32R {
    using real = float;
    using cvec = float2;
    static constexpr size_t block_bytes = 3 * TILE * 16;
    static constexpr bool two_row = true;
    static constexpr size_t tile_bytes = 8 * block_bytes + 64;
    __device__ __forceinline__ static float load_rows(const char *tile, int d, int lane, float m[12])
    {
        const float4 *p = reinterpret_cast<const float4 *>(tile + (size_t)d * block_bytes) + lane;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            float4 v = ntload(p + q * TILE);
            m[4 * q] = v.x; m[4 * q + 1] = v.y; m[4 * q + 2] = v.z; m[4 * q + 3] = v.w;
        }
        return ((sign_word(tile, block_bytes, d) >> lane) & 1ull) ? -1.0f : 1.0f;
    }
    __device__ __forceinline__ static void load_dir(const char *tile, int d, int lane, float m[18])
    {
        const float c = load_rows(tile, d, lane, m);
        third_row<float>(m, c);
    }
};

// 16-bit fixed-point two-row form: rows 0 and 1 as 6 words of two int16
// (re, im) scaled by a per-matrix FP32 scale (the largest |re|, |im| of the
// two rows), in a plane of uint4 (words 0-3), one of uint2 (words 4-5) and
// one of the scale: 28 bytes per matrix, and the sign word as above.
struct PI16R {
    using real = float;
    using cvec = float2;
    static constexpr size_t block_bytes = TILE * 28;
    static constexpr bool two_row = true;
    static constexpr size_t tile_bytes = 8 * block_bytes + 64;
    __device__ __forceinline__ static float load_rows(const char *tile, int d, int lane, float m[12])
    {
        const char *blk = tile + (size_t)d * block_bytes;
        const uint4 a = ntload(reinterpret_cast<const uint4 *>(blk) + lane);
        const uint2 b = ntload(reinterpret_cast<const uint2 *>(blk + TILE * 16) + lane);
        const float s = ntload(reinterpret_cast<const float *>(blk + TILE * 24) + lane) * (1.0f / 32767.0f);
        const unsigned w[6] = { a.x, a.y, a.z, a.w, b.x, b.y };
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            m[2 * e] = (float)(short)(w[e] & 0xFFFFu) * s;
            m[2 * e + 1] = (float)(short)(w[e] >> 16) * s;
        }
        return ((sign_word(tile, block_bytes, d) >> lane) & 1ull) ? -1.0f : 1.0f;
    }
    __device__ __forceinline__ static void load_dir(const char *tile, int d, int lane, float m[18])
    {
        const float c = load_rows(tile, d, lane, m);
        third_row<float>(m, c);
    }
};

// FP64 / FP32 / 16-bit fixed point with two-row long links (the fat field
// stays full: smeared links are not SU(3)).
struct PF64C {
    using real = double;
    using cvec = double2;
    static constexpr int prec = HISQ_F64C;
    using Fat = PF64;
    using Long = PF64R;
};
struct PF32C {
    using real = float;
    using cvec = float2;
    static constexpr int prec = HISQ_F32C;
    using Fat = PF32;
    using Long = PF32R;
};
struct PI16SC {
    using real = float;
    using cvec = float2;
    static constexpr int prec = HISQ_I16SC;
    using Fat = PI16S;
    using Long = PI16R;
};

}  // namespace hisq
