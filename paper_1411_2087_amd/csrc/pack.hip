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

size_t dir_block_bytes(int prec)
{
    switch (prec) {
    case HISQ_F64: return PF64::block_bytes;
    case HISQ_F32: return PF32::block_bytes;
    case HISQ_F16S: return PF16S::block_bytes;
    case HISQ_I16S: return PI16S::block_bytes;
    default: return 0;
    }
}

size_t packed_field_bytes(const Geom &g, int prec) { return 2ull * g.ntiles * 8 * dir_block_bytes(prec); }

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
    if (fat_out == long_out) return fail(HISQ_EALIAS, "hisq_pack_links: fat_out and long_out alias");
    const size_t bb = dir_block_bytes(prec);
    if (!bb) return fail(HISQ_EINVAL, "hisq_pack_links: unknown precision");
    hipStream_t s = (hipStream_t)stream;
    const long long total = 2LL * g.ntiles * 8 * TILE;
    const dim3 grid((unsigned)((total + 255) / 256)), block(256);
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
