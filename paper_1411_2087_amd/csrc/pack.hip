// Link packing: canonical [mu][lex][3][3] complex128 -> the tiled packed
// form read by the Dslash kernels.
//
// For every output site n of each parity the packed field holds the 8
// matrices that multiply n's neighbours: U_mu(n) for +mu and
// -U_mu(n - k mu)^dag for -mu (k = 1 fat, 3 long).  Storing the backward
// links at the output site doubles the storage but makes every link read of
// the Dslash contiguous and single-use, the locality argument of Sec. 4
// ("both forward and backward links are stored at each site").
#include "hisq_common.hpp"

namespace hisq {

template <int PREC>
__device__ __forceinline__ void store_block(char *blk, int lane, const double m[18]);

template <>
__device__ __forceinline__ void store_block<HISQ_F64>(char *blk, int lane, const double m[18])
{
    double2 *p = reinterpret_cast<double2 *>(blk) + lane;
#pragma unroll
    for (int e = 0; e < 9; ++e) p[e * TILE] = make_double2(m[2 * e], m[2 * e + 1]);
}

template <>
__device__ __forceinline__ void store_block<HISQ_F32>(char *blk, int lane, const double m[18])
{
    float4 *p4 = reinterpret_cast<float4 *>(blk) + lane;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        p4[q * TILE] = make_float4((float)m[4 * q], (float)m[4 * q + 1], (float)m[4 * q + 2], (float)m[4 * q + 3]);
    float2 *p2 = reinterpret_cast<float2 *>(blk + 4 * TILE * 16) + lane;
    *p2 = make_float2((float)m[16], (float)m[17]);
}

template <>
__device__ __forceinline__ void store_block<HISQ_F16S>(char *blk, int lane, const double m[18])
{
    double mx = 0.0;
#pragma unroll
    for (int i = 0; i < 18; ++i) mx = fmax(mx, fabs(m[i]));
    const float scale = (float)mx;
    const double inv = scale > 0.0f ? 1.0 / (double)scale : 0.0;
    unsigned w[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        __half2 hv = __floats2half2_rn((float)(m[2 * e] * inv), (float)(m[2 * e + 1] * inv));
        w[e] = *reinterpret_cast<unsigned *>(&hv);
    }
    uint4 *p4 = reinterpret_cast<uint4 *>(blk) + lane;
    p4[0] = make_uint4(w[0], w[1], w[2], w[3]);
    p4[TILE] = make_uint4(w[4], w[5], w[6], w[7]);
    uint2 *p2 = reinterpret_cast<uint2 *>(blk + 2 * TILE * 16) + lane;
    *p2 = make_uint2(w[8], __float_as_uint(scale));
}

template <>
__device__ __forceinline__ void store_block<HISQ_I16S>(char *blk, int lane, const double m[18])
{
    double mx = 0.0;
#pragma unroll
    for (int i = 0; i < 18; ++i) mx = fmax(mx, fabs(m[i]));
    const float scale = (float)mx;
    const double inv = scale > 0.0f ? 32767.0 / (double)scale : 0.0;
    unsigned w[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        int qr = (int)rint(m[2 * e] * inv), qi = (int)rint(m[2 * e + 1] * inv);
        qr = qr > 32767 ? 32767 : (qr < -32767 ? -32767 : qr);
        qi = qi > 32767 ? 32767 : (qi < -32767 ? -32767 : qi);
        w[e] = ((unsigned)qr & 0xFFFFu) | (((unsigned)qi & 0xFFFFu) << 16);
    }
    uint4 *p4 = reinterpret_cast<uint4 *>(blk) + lane;
    p4[0] = make_uint4(w[0], w[1], w[2], w[3]);
    p4[TILE] = make_uint4(w[4], w[5], w[6], w[7]);
    uint2 *p2 = reinterpret_cast<uint2 *>(blk + 2 * TILE * 16) + lane;
    *p2 = make_uint2(w[8], __float_as_uint(scale));
}

template <int PREC>
__global__ __launch_bounds__(256) void k_pack(const double2 *__restrict__ canon, char *__restrict__ out, Geom g,
                                              int hop, size_t block_bytes)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = 2LL * g.ntiles * 8 * TILE;
    if (i >= total) return;
    const int lane = (int)(i % TILE);
    const long long rest = i / TILE;
    const int d = (int)(rest % 8);
    const long long pt = rest / 8;  // parity * ntiles + tile
    const int tile = (int)(pt % g.ntiles);
    const int parity = (int)(pt / g.ntiles);
    const int h = tile * TILE + lane;
    double m[18];
#pragma unroll
    for (int e = 0; e < 18; ++e) m[e] = 0.0;
    if (h < g.Vh) {
        int c[4];
        site_coords(g, h, parity, c[0], c[1], c[2], c[3]);
        const int mu = d & 3;
        const bool bwd = d >= 4;
        if (bwd) c[mu] = wrap(c[mu] - hop, g.L[mu]);
        const long long V = 2LL * g.Vh;
        const long long lex = c[0] + (long long)g.L[0] * (c[1] + (long long)g.L[1] * (c[2] + (long long)g.L[2] * c[3]));
        const double2 *u = canon + (mu * V + lex) * 9;
        if (!bwd) {
#pragma unroll
            for (int e = 0; e < 9; ++e) { double2 v = u[e]; m[2 * e] = v.x; m[2 * e + 1] = v.y; }
        } else {
            // -U^dag: entry (a, b) = -conj(U_ba)
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    double2 v = u[3 * b + a];
                    m[2 * (3 * a + b)] = -v.x;
                    m[2 * (3 * a + b) + 1] = v.y;
                }
        }
    }
    char *blk = out + ((size_t)pt * 8 + d) * block_bytes;
    store_block<PREC>(blk, lane, m);
}

// Two-row long links: rows 0 and 1 of every matrix, plus the sign word of
// each (tile, direction) built with a wavefront ballot.  `status` is set when
// a matrix is not +-SU(3) to 1e-6 (padding lanes are exempt).
template <int PREC, class R>
__global__ __launch_bounds__(256) void k_pack_rows(const double2 *__restrict__ canon, char *__restrict__ out, Geom g,
                                                   int hop, int *status)
{
    constexpr size_t BB = R::block_bytes, TB = R::tile_bytes;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = 2LL * g.ntiles * 8 * TILE;  // a multiple of 64: whole wavefronts only
    if (i >= total) return;
    const int lane = (int)(i % TILE);
    const long long rest = i / TILE;
    const int d = (int)(rest % 8);
    const long long pt = rest / 8;
    const int tile = (int)(pt % g.ntiles), parity = (int)(pt / g.ntiles);
    const int h = tile * TILE + lane;
    double m[18];
#pragma unroll
    for (int e = 0; e < 18; ++e) m[e] = 0.0;
    bool neg = false;
    if (h < g.Vh) {
        int c[4];
        site_coords(g, h, parity, c[0], c[1], c[2], c[3]);
        const int mu = d & 3;
        const bool bwd = d >= 4;
        if (bwd) c[mu] = wrap(c[mu] - hop, g.L[mu]);
        const long long V = 2LL * g.Vh;
        const long long lex = c[0] + (long long)g.L[0] * (c[1] + (long long)g.L[1] * (c[2] + (long long)g.L[2] * c[3]));
        const double2 *u = canon + (mu * V + lex) * 9;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const double2 v = bwd ? u[3 * b + a] : u[3 * a + b];
                m[2 * (3 * a + b)] = bwd ? -v.x : v.x;
                m[2 * (3 * a + b) + 1] = v.y;
            }
        // det by cofactors of row 0; c = sign(Re det)
        const double c0r = m[8] * m[16] - m[9] * m[17] - (m[10] * m[14] - m[11] * m[15]);
        const double c0i = m[8] * m[17] + m[9] * m[16] - (m[10] * m[15] + m[11] * m[14]);
        const double c1r = m[10] * m[12] - m[11] * m[13] - (m[6] * m[16] - m[7] * m[17]);
        const double c1i = m[10] * m[13] + m[11] * m[12] - (m[6] * m[17] + m[7] * m[16]);
        const double c2r = m[6] * m[14] - m[7] * m[15] - (m[8] * m[12] - m[9] * m[13]);
        const double c2i = m[6] * m[15] + m[7] * m[14] - (m[8] * m[13] + m[9] * m[12]);
        const double dr = m[0] * c0r - m[1] * c0i + m[2] * c1r - m[3] * c1i + m[4] * c2r - m[5] * c2i;
        const double di = m[0] * c0i + m[1] * c0r + m[2] * c1i + m[3] * c1r + m[4] * c2i + m[5] * c2r;
        neg = dr < 0.0;
        const double cs = neg ? -1.0 : 1.0;
        // unitarity of the stored rows and agreement of row 2 with its rebuild
        double dev = fabs(dr - cs) + fabs(di);
        double rb[18];
#pragma unroll
        for (int e = 0; e < 18; ++e) rb[e] = m[e];
        third_row<double>(rb, cs);
#pragma unroll
        for (int e = 12; e < 18; ++e) dev = fmax(dev, fabs(rb[e] - m[e]));
        if (!(dev <= 1e-6)) atomicOr(status, 1);
    }
    const unsigned long long word = __ballot(neg);
    char *tile_base = out + (size_t)pt * TB;
    if (lane == 0) *reinterpret_cast<unsigned long long *>(tile_base + 8 * BB + 8 * (size_t)d) = word;
    if constexpr (PREC == HISQ_F64C) {
        double2 *q = reinterpret_cast<double2 *>(tile_base + (size_t)d * BB) + lane;
#pragma unroll
        for (int e = 0; e < 6; ++e) q[e * TILE] = make_double2(m[2 * e], m[2 * e + 1]);
    } else if constexpr (PREC == HISQ_I16SC) {
        // rows 0 and 1 in 16-bit fixed point against their largest |re|, |im|
        double mx = 0.0;
#pragma unroll
        for (int i = 0; i < 12; ++i) mx = fmax(mx, fabs(m[i]));
        const float scale = (float)mx;
        const double inv = scale > 0.0f ? 32767.0 / (double)scale : 0.0;
        unsigned w[6];
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            int qr = (int)rint(m[2 * e] * inv), qi = (int)rint(m[2 * e + 1] * inv);
            qr = qr > 32767 ? 32767 : (qr < -32767 ? -32767 : qr);
            qi = qi > 32767 ? 32767 : (qi < -32767 ? -32767 : qi);
            w[e] = ((unsigned)qr & 0xFFFFu) | (((unsigned)qi & 0xFFFFu) << 16);
        }
        char *blk = tile_base + (size_t)d * BB;
        reinterpret_cast<uint4 *>(blk)[lane] = make_uint4(w[0], w[1], w[2], w[3]);
        reinterpret_cast<uint2 *>(blk + TILE * 16)[lane] = make_uint2(w[4], w[5]);
        reinterpret_cast<float *>(blk + TILE * 24)[lane] = scale;
    } else {
        float4 *q = reinterpret_cast<float4 *>(tile_base + (size_t)d * BB) + lane;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            q[k * TILE] = make_float4((float)m[4 * k], (float)m[4 * k + 1], (float)m[4 * k + 2], (float)m[4 * k + 3]);
    }
}

size_t dir_block_bytes(int prec)
{
    switch (prec) {
    case HISQ_F64: return PF64::block_bytes;
    case HISQ_F32: return PF32::block_bytes;
    case HISQ_F16S: return PF16S::block_bytes;
    case HISQ_I16S: return PI16S::block_bytes;
    case HISQ_F64C: return PF64::block_bytes;  // the fat field
    case HISQ_F32C: return PF32::block_bytes;
    case HISQ_I16SC: return PI16S::block_bytes;
    default: return 0;
    }
}

// fat: full blocks; long of the compressed precisions: two-row tiles plus a
// 256-byte status word after the last tile
static size_t long_field_bytes(const Geom &g, int prec)
{
    if (prec == HISQ_F64C) return 2ull * g.ntiles * PF64R::tile_bytes + 256;
    if (prec == HISQ_F32C) return 2ull * g.ntiles * PF32R::tile_bytes + 256;
    if (prec == HISQ_I16SC) return 2ull * g.ntiles * PI16R::tile_bytes + 256;
    return 2ull * g.ntiles * 8 * dir_block_bytes(prec);
}

size_t packed_field_bytes(const Geom &g, int prec)
{
    const size_t f = 2ull * g.ntiles * 8 * dir_block_bytes(prec), l = long_field_bytes(g, prec);
    return dir_block_bytes(prec) ? (f > l ? f : l) : 0;
}

}  // namespace hisq

using namespace hisq;

extern "C" size_t hisq_packed_link_bytes(const int dims[4], int prec)
{
    Geom g;
    if (make_geom(dims, g)) return 0;
    return packed_field_bytes(g, prec);
}

extern "C" int hisq_pack_links(const void *fat_canon, const void *long_canon, const int dims[4], int prec,
                               void *fat_out, void *long_out, void *stream)
{
    Geom g;
    int rc = make_geom(dims, g);
    if (rc) return rc;
    if (!fat_canon || !long_canon || !fat_out || !long_out) return fail(HISQ_EINVAL, "hisq_pack_links: NULL pointer");
    if (!aligned16({fat_canon, long_canon, fat_out, long_out}))
        return fail(HISQ_EINVAL, "hisq_pack_links: device pointers must be 16-byte aligned");
    if (fat_out == long_out) return fail(HISQ_EALIAS, "hisq_pack_links: fat_out and long_out alias");
    const size_t bb = dir_block_bytes(prec);
    if (!bb) return fail(HISQ_EINVAL, "hisq_pack_links: unknown precision");
    hipStream_t s = (hipStream_t)stream;
    const long long total = 2LL * g.ntiles * 8 * TILE;
    const dim3 grid((unsigned)((total + 255) / 256)), block(256);
    if (prec == HISQ_F64C || prec == HISQ_F32C || prec == HISQ_I16SC) {
        const int fp = prec == HISQ_F64C ? HISQ_F64 : (prec == HISQ_F32C ? HISQ_F32 : HISQ_I16S);
        const size_t fbb = dir_block_bytes(fp);
        if (fp == HISQ_F64)
            hipLaunchKernelGGL(k_pack<HISQ_F64>, grid, block, 0, s, (const double2 *)fat_canon, (char *)fat_out, g, 1, fbb);
        else if (fp == HISQ_F32)
            hipLaunchKernelGGL(k_pack<HISQ_F32>, grid, block, 0, s, (const double2 *)fat_canon, (char *)fat_out, g, 1, fbb);
        else
            hipLaunchKernelGGL(k_pack<HISQ_I16S>, grid, block, 0, s, (const double2 *)fat_canon, (char *)fat_out, g, 1, fbb);
        int *status = reinterpret_cast<int *>((char *)long_out + long_field_bytes(g, prec) - 256);
        HISQ_HIP(hipMemsetAsync(status, 0, sizeof(int), s));
        if (prec == HISQ_F64C)
            hipLaunchKernelGGL((k_pack_rows<HISQ_F64C, PF64R>), grid, block, 0, s, (const double2 *)long_canon,
                               (char *)long_out, g, 3, status);
        else if (prec == HISQ_F32C)
            hipLaunchKernelGGL((k_pack_rows<HISQ_F32C, PF32R>), grid, block, 0, s, (const double2 *)long_canon,
                               (char *)long_out, g, 3, status);
        else
            hipLaunchKernelGGL((k_pack_rows<HISQ_I16SC, PI16R>), grid, block, 0, s, (const double2 *)long_canon,
                               (char *)long_out, g, 3, status);
        HISQ_HIP(hipGetLastError());
        int h_status = 0;
        HISQ_HIP(hipMemcpyAsync(&h_status, status, sizeof(int), hipMemcpyDeviceToHost, s));
        HISQ_HIP(hipStreamSynchronize(s));
        if (h_status) return fail(HISQ_EINVAL, "hisq_pack_links: a long link is not +-SU(3) to 1e-6; use an uncompressed precision");
        return HISQ_OK;
    }
    for (int f = 0; f < 2; ++f) {
        const double2 *in = (const double2 *)(f ? long_canon : fat_canon);
        char *out = (char *)(f ? long_out : fat_out);
        const int hop = f ? 3 : 1;
        switch (prec) {
        case HISQ_F64: hipLaunchKernelGGL(k_pack<HISQ_F64>, grid, block, 0, s, in, out, g, hop, bb); break;
        case HISQ_F32: hipLaunchKernelGGL(k_pack<HISQ_F32>, grid, block, 0, s, in, out, g, hop, bb); break;
        case HISQ_F16S: hipLaunchKernelGGL(k_pack<HISQ_F16S>, grid, block, 0, s, in, out, g, hop, bb); break;
        default: hipLaunchKernelGGL(k_pack<HISQ_I16S>, grid, block, 0, s, in, out, g, hop, bb); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "hisq_pack_links launch");
    }
    return HISQ_OK;
}
