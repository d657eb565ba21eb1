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
// Each layer is one kernel per 32-site tile of one parity: the 9*C_in
// transported fields of the tile are computed in FP32 and written to LDS as
// BF16 (the real embedding [Re; Im]), then the channel mixing is a real GEMM
//     [Re out; Im out] (2 C_out x 96) = [[Wr, -Wi], [Wi, Wr]] (2 C_out x 18 C_in)
//                                       x [Re F; Im F] (18 C_in x 96)
// on v_mfma_f32_32x32x16_bf16 with FP32 accumulation.  The gradient with
// respect to the input is the same kernel with W'_{k'}^{ba} = conj(W_{k}^{ab}),
// k' the adjoint transport of k (T_{+mu}^dag = T_{-mu}); the weight gradient
// G_k^{ab} = sum_x <T_k in^b, g^a> is a split-K MFMA over sites followed by a
// fixed-order sum of the per-workgroup partials.
//
// Feature layout: [batch][channel][parity][h][colour] complex64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "dslash_core.hpp"

namespace hisq {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int NET_SW = 32;              // sites per workgroup tile (forward)
constexpr int NET_COLS = 3 * NET_SW;    // GEMM columns per tile
constexpr int NET_NT = 128;             // two wavefronts
constexpr int WG_SW = 16;               // sites per unit (weight gradient)
constexpr int WG_COLS = 3 * WG_SW;
constexpr int MPAD = 32;                // GEMM rows (2 C_out <= 32)
constexpr int WG_MAX_BLOCKS = 1024;

__host__ __device__ constexpr int kpad_of(int cin) { return (18 * cin + 15) / 16 * 16; }
__host__ __device__ constexpr int npad_of(int cin) { return (9 * cin + 31) / 32 * 32; }
constexpr int ADJ[9] = { 0, 5, 6, 7, 8, 1, 2, 3, 4 };

__device__ __forceinline__ __bf16 to_bf16(float f) { return (__bf16)f; }  // round to nearest even

__device__ __forceinline__ size_t feat_idx(int b, int C, int c, int p, int Vh, int h)
{
    return ((((size_t)b * C + c) * 2 + p) * Vh + h) * 3;
}

// (T_k phi^c)(x)_a for all channels c of `in`, for the site h of parity p:
// calls emit(k, c, re, im).  Rows of the packed fat links: +mu holds
// U_mu(x), -mu holds -U_mu(x-mu)^dag.
template <int CIN, class Emit>
__device__ __forceinline__ void transport_site(const Geom &g, const char *__restrict__ fat,
                                               const float2 *__restrict__ in, int b, int p, int h, int a, Emit emit)
{
    int x, y, z, t;
    site_coords(g, h, p, x, y, z, t);
    // k = 0
#pragma unroll 4
    for (int c = 0; c < CIN; ++c) {
        float2 v = in[feat_idx(b, CIN, c, p, g.Vh, h) + a];
        emit(0, c, v.x, v.y);
    }
    const int tile = h / TILE, lane = h % TILE;
    const size_t tile_off = ((size_t)p * g.ntiles + tile) * 8 * PF32::block_bytes;
#pragma unroll 1
    for (int d = 0; d < 8; ++d) {
        const int mu = d & 3;
        const bool bwd = d >= 4;
        const int nh = nbr_h(g, h, x, y, z, t, mu, bwd ? -1 : 1);
        float m[18];
        PF32::load(fat + tile_off + (size_t)d * PF32::block_bytes, lane, m);
        const float sg = bwd ? -1.0f : 1.0f;  // packed backward link is -U^dag
        const float m0r = sg * m[6 * a], m0i = sg * m[6 * a + 1], m1r = sg * m[6 * a + 2], m1i = sg * m[6 * a + 3],
                    m2r = sg * m[6 * a + 4], m2i = sg * m[6 * a + 5];
#pragma unroll 4
        for (int c = 0; c < CIN; ++c) {
            const float2 *s = in + feat_idx(b, CIN, c, 1 - p, g.Vh, nh);
            const float2 s0 = s[0], s1 = s[1], s2 = s[2];
            float re = m0r * s0.x - m0i * s0.y;
            float im = m0r * s0.y + m0i * s0.x;
            re = fmaf(m1r, s1.x, re); re = fmaf(-m1i, s1.y, re);
            im = fmaf(m1r, s1.y, im); im = fmaf(m1i, s1.x, im);
            re = fmaf(m2r, s2.x, re); re = fmaf(-m2i, s2.y, re);
            im = fmaf(m2r, s2.y, im); im = fmaf(m2i, s2.x, im);
            emit(1 + d, c, re, im);
        }
    }
}

// ------------------------------------------------------------------ weights -> BF16 GEMM operand
// A[m][kk] (MPAD x kpad) for out = sum_k W_k T_k in.  transposed_adjoint:
// the matrix of the input-gradient layer (C_in' = COUT, C_out' = CIN).
template <int CIN, int COUT>
__global__ void k_net_prep(const float2 *__restrict__ W, __bf16 *__restrict__ A, int adjoint)
{
    // the GEMM layer has (ci, co) = (CIN, COUT), or (COUT, CIN) for the adjoint
    const int ci = adjoint ? COUT : CIN, co = adjoint ? CIN : COUT;
    const int kp = kpad_of(ci);
    for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < MPAD * kp; i += blockDim.x * gridDim.x) {
        const int m = i / kp, kk = i % kp;
        float v = 0.f;
        if (m < 2 * co && kk < 18 * ci) {
            const bool im_row = m >= co, im_col = kk >= 9 * ci;
            const int a = im_row ? m - co : m;   // output channel of the GEMM layer
            const int q = im_col ? kk - 9 * ci : kk;
            const int k = q / ci, c = q % ci;   // transport, input channel of the GEMM layer
            float2 w;
            if (!adjoint) {
                w = W[((size_t)k * COUT + a) * CIN + c];
            } else {  // W'_{k}^{a c} = conj(W_{adj k}^{c a})
                float2 u = W[((size_t)ADJ[k] * COUT + c) * CIN + a];
                w = make_float2(u.x, -u.y);
            }
            // [[Wr, -Wi], [Wi, Wr]]
            v = !im_row ? (!im_col ? w.x : -w.y) : (!im_col ? w.y : w.x);
        }
        A[i] = to_bf16(v);
    }
}

// ------------------------------------------------------------------ layer (forward and input gradient)
template <int CIN, int COUT>
__global__ __launch_bounds__(NET_NT) void k_net_layer(Geom g, const char *__restrict__ fat,
                                                      const float2 *__restrict__ in, float2 *__restrict__ out,
                                                      const __bf16 *__restrict__ A)
{
    constexpr int KP = kpad_of(CIN);
    constexpr int PITCH = KP + 8;  // bf16 per LDS row (padding spreads the banks)
    __shared__ __align__(16) __bf16 F[NET_COLS * PITCH];
    const int p = blockIdx.y, b = blockIdx.z;
    const int h0 = blockIdx.x * NET_SW;
    // phase 1: transported fields of the tile -> F[col][kk] (BF16), col = site*3 + colour
    if (threadIdx.x < NET_COLS) {
        const int col = threadIdx.x, s = col / 3, a = col % 3, h = h0 + s;
        __bf16 *row = F + col * PITCH;
        if (h < g.Vh) {
            transport_site<CIN>(g, fat, in, b, p, h, a, [&](int k, int c, float re, float im) {
                row[k * CIN + c] = to_bf16(re);
                row[9 * CIN + k * CIN + c] = to_bf16(im);
            });
        } else {
            for (int q = 0; q < 18 * CIN; ++q) row[q] = to_bf16(0.f);
        }
        for (int q = 18 * CIN; q < KP; ++q) row[q] = to_bf16(0.f);
    }
    __syncthreads();
    // phase 2: MFMA, wave w takes column tiles w, w + 2
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int j = w; j < NET_COLS / 32; j += 2) {
        floatx16 acc = {};
#pragma unroll
        for (int kb = 0; kb < KP / 16; ++kb) {
            const bf16x8 av = *reinterpret_cast<const bf16x8 *>(A + (l % 32) * KP + kb * 16 + 8 * (l / 32));
            const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(F + (j * 32 + l % 32) * PITCH + kb * 16 + 8 * (l / 32));
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
        }
        const int col = j * 32 + l % 32, s = col / 3, a = col % 3, h = h0 + s;
        if (h < g.Vh) {
            float *o = reinterpret_cast<float *>(out);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = 8 * (r / 4) + 4 * (l / 32) + (r % 4);
                if (m < 2 * COUT) {
                    const int ch = m < COUT ? m : m - COUT;
                    o[2 * (feat_idx(b, COUT, ch, p, g.Vh, h) + a) + (m < COUT ? 0 : 1)] = acc[r];
                }
            }
        }
    }
}

// ------------------------------------------------------------------ weight gradient (split-K over sites)
// partials[block][MPAD][NP] (float): rows m < COUT -> Re G, COUT <= m < 2COUT -> Im G; column q = k*CIN + c.
template <int CIN, int COUT>
__global__ __launch_bounds__(NET_NT) void k_net_wgrad(Geom g, const char *__restrict__ fat,
                                                      const float2 *__restrict__ in, const float2 *__restrict__ gout,
                                                      int batch, float *__restrict__ partials)
{
    constexpr int NP = npad_of(CIN);
    constexpr int FP = 2 * WG_COLS + 8;      // F2 row pitch (bf16)
    constexpr int GP = 2 * WG_COLS + 8;      // G row pitch
    constexpr int NTILES = NP / 32;
    __shared__ __align__(16) __bf16 F2[NP * FP];
    __shared__ __align__(16) __bf16 G2[MPAD * GP];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    floatx16 acc[(NTILES + 1) / 2];
#pragma unroll
    for (int i = 0; i < (NTILES + 1) / 2; ++i) acc[i] = floatx16{};
    const int tiles_per_par = (g.Vh + WG_SW - 1) / WG_SW;
    const int nunits = batch * 2 * tiles_per_par;
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
        const int b = u / (2 * tiles_per_par), rem = u % (2 * tiles_per_par);
        const int p = rem / tiles_per_par, h0 = (rem % tiles_per_par) * WG_SW;
        __syncthreads();  // previous unit's LDS reads are done
        // zero the padding rows of F2 and all of G2's unused rows
        for (int i = threadIdx.x; i < (NP - 9 * CIN) * FP; i += NET_NT) F2[9 * CIN * FP + i] = to_bf16(0.f);
        if (threadIdx.x < WG_COLS) {
            const int col = threadIdx.x, s = col / 3, a = col % 3, h = h0 + s;
            if (h < g.Vh) {
                transport_site<CIN>(g, fat, in, b, p, h, a, [&](int k, int c, float re, float im) {
                    F2[(k * CIN + c) * FP + col] = to_bf16(re);
                    F2[(k * CIN + c) * FP + WG_COLS + col] = to_bf16(im);
                });
            } else {
                for (int q = 0; q < 9 * CIN; ++q) {
                    F2[q * FP + col] = to_bf16(0.f);
                    F2[q * FP + WG_COLS + col] = to_bf16(0.f);
                }
            }
            // G2 rows: [gr, gi] (Re G) and [gi, -gr] (Im G)
            for (int m = 0; m < MPAD; ++m) {
                float v1 = 0.f, v2 = 0.f;
                if (m < 2 * COUT && h < g.Vh) {
                    const int ch = m < COUT ? m : m - COUT;
                    const float2 gv = gout[feat_idx(b, COUT, ch, p, g.Vh, h) + a];
                    if (m < COUT) { v1 = gv.x; v2 = gv.y; } else { v1 = gv.y; v2 = -gv.x; }
                }
                G2[m * GP + col] = to_bf16(v1);
                G2[m * GP + WG_COLS + col] = to_bf16(v2);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < (NTILES + 1) / 2; ++i) {
            const int j = w + 2 * i;
            if (j >= NTILES) break;
#pragma unroll
            for (int kb = 0; kb < 2 * WG_COLS / 16; ++kb) {
                const bf16x8 av = *reinterpret_cast<const bf16x8 *>(G2 + (l % 32) * GP + kb * 16 + 8 * (l / 32));
                const bf16x8 bv =
                    *reinterpret_cast<const bf16x8 *>(F2 + (j * 32 + l % 32) * FP + kb * 16 + 8 * (l / 32));
                acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[i], 0, 0, 0);
            }
        }
    }
    float *dst = partials + (size_t)blockIdx.x * MPAD * NP;
#pragma unroll
    for (int i = 0; i < (NTILES + 1) / 2; ++i) {
        const int j = w + 2 * i;
        if (j >= NTILES) break;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int m = 8 * (r / 4) + 4 * (l / 32) + (r % 4);
            dst[m * NP + j * 32 + l % 32] = acc[i][r];
        }
    }
}

// grad_w[k][a][c] = sum over blocks, fixed order
template <int CIN, int COUT>
__global__ void k_net_wgrad_reduce(const float *__restrict__ partials, int nblocks, float2 *__restrict__ gw)
{
    constexpr int NP = npad_of(CIN);
    const int n = 9 * COUT * CIN;
    for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < n; i += blockDim.x * gridDim.x) {
        const int k = i / (COUT * CIN), a = (i / CIN) % COUT, c = i % CIN;
        const int q = k * CIN + c;
        double re = 0.0, im = 0.0;
        for (int bl = 0; bl < nblocks; ++bl) {
            re += partials[((size_t)bl * MPAD + a) * NP + q];
            im += partials[((size_t)bl * MPAD + COUT + a) * NP + q];
        }
        gw[i] = make_float2((float)re, (float)im);
    }
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
constexpr size_t ABF_SLOT = (size_t)MPAD * 288 * 2;  // one layer's BF16 operand (C <= 16)

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
    const dim3 grid((g.Vh + NET_SW - 1) / NET_SW, 2, batch);
    hipLaunchKernelGGL((k_net_layer<CIN, COUT>), grid, dim3(NET_NT), 0, s, g, (const char *)fat, in, out, A);
}

template <int CIN, int COUT>
static void prep_launch(const float2 *W, __bf16 *A, int adjoint, hipStream_t s)
{
    hipLaunchKernelGGL((k_net_prep<CIN, COUT>), dim3(8), dim3(256), 0, s, W, A, adjoint);
}

template <int C>
static int net_forward_t(const Geom &g, const void *fat, const float2 *W, const float2 *in_even, float2 *out_even,
                         void *acts, int batch, hipStream_t s)
{
    NetActs a = net_acts(acts, g, C, batch);
    prep_launch<1, C>(W + w_off(C, 0), a.A[0], 0, s);
    prep_launch<C, C>(W + w_off(C, 1), a.A[1], 0, s);
    prep_launch<C, C>(W + w_off(C, 2), a.A[2], 0, s);
    prep_launch<C, 1>(W + w_off(C, 3), a.A[3], 0, s);
    const long long ne = (long long)batch * 2 * g.Vh * 3;
    const int nb = (int)std::min<long long>((ne + 255) / 256, 4096);
    hipLaunchKernelGGL(k_net_embed, dim3(nb), dim3(256), 0, s, in_even, a.in[0], batch, g.Vh);
    layer_launch<1, C>(g, fat, a.in[0], a.in[1], a.A[0], batch, s);
    layer_launch<C, C>(g, fat, a.in[1], a.in[2], a.A[1], batch, s);
    layer_launch<C, C>(g, fat, a.in[2], a.in[3], a.A[2], batch, s);
    layer_launch<C, 1>(g, fat, a.in[3], a.out, a.A[3], batch, s);
    if (out_even) hipLaunchKernelGGL(k_net_extract, dim3(nb), dim3(256), 0, s, (const float2 *)a.out, out_even, batch, g.Vh);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

static int wgrad_blocks() { return 512; }

size_t net_bwd_ws_bytes_g(const Geom &g, int C, int batch)
{
    return 2 * a256(feat_bytes(g, batch, C)) + a256(feat_bytes(g, batch, 1)) +
           a256((size_t)wgrad_blocks() * MPAD * 160 * sizeof(float)) + 4 * a256(ABF_SLOT);
}

template <int CIN, int COUT>
static void wgrad_launch(const Geom &g, const void *fat, const float2 *in, const float2 *gout, int batch, float *part,
                         float2 *gw, hipStream_t s)
{
    const int nb = wgrad_blocks();
    hipLaunchKernelGGL((k_net_wgrad<CIN, COUT>), dim3(nb), dim3(NET_NT), 0, s, g, (const char *)fat, in, gout, batch,
                       part);
    hipLaunchKernelGGL((k_net_wgrad_reduce<CIN, COUT>), dim3(16), dim3(256), 0, s, (const float *)part, nb, gw);
}

template <int C>
static int net_backward_t(const Geom &g, const void *fat, const float2 *W, const void *acts, const float2 *gout_even,
                          float2 *gw, float2 *gin_even, int batch, void *ws, hipStream_t s)
{
    NetActs a = net_acts(const_cast<void *>(acts), g, C, batch);
    char *p = (char *)ws;
    float2 *g1 = (float2 *)p; p += a256(feat_bytes(g, batch, C));
    float2 *g2 = (float2 *)p; p += a256(feat_bytes(g, batch, C));
    float2 *gl = (float2 *)p; p += a256(feat_bytes(g, batch, 1));
    float *part = (float *)p; p += a256((size_t)wgrad_blocks() * MPAD * 160 * sizeof(float));
    __bf16 *Ab[4];
    for (int i = 0; i < 4; ++i) { Ab[i] = (__bf16 *)p; p += a256(ABF_SLOT); }
    const long long ne = (long long)batch * 2 * g.Vh * 3;
    const int nb = (int)std::min<long long>((ne + 255) / 256, 4096);
    // gradient of the last layer's output: even part given, odd part zero
    hipLaunchKernelGGL(k_net_embed, dim3(nb), dim3(256), 0, s, gout_even, gl, batch, g.Vh);
    prep_launch<C, 1>(W + w_off(C, 3), Ab[3], 1, s);
    prep_launch<C, C>(W + w_off(C, 2), Ab[2], 1, s);
    prep_launch<C, C>(W + w_off(C, 1), Ab[1], 1, s);
    prep_launch<1, C>(W + w_off(C, 0), Ab[0], 1, s);
    // layer 4: C -> 1
    wgrad_launch<C, 1>(g, fat, a.in[3], gl, batch, part, gw + w_off(C, 3), s);
    layer_launch<1, C>(g, fat, gl, g1, Ab[3], batch, s);       // dl/d in4 (adjoint layer: 1 -> C)
    wgrad_launch<C, C>(g, fat, a.in[2], g1, batch, part, gw + w_off(C, 2), s);
    layer_launch<C, C>(g, fat, g1, g2, Ab[2], batch, s);       // dl/d in3
    wgrad_launch<C, C>(g, fat, a.in[1], g2, batch, part, gw + w_off(C, 1), s);
    layer_launch<C, C>(g, fat, g2, g1, Ab[1], batch, s);       // dl/d in2
    wgrad_launch<1, C>(g, fat, a.in[0], g1, batch, part, gw + w_off(C, 0), s);
    if (gin_even) {
        layer_launch<C, 1>(g, fat, g1, gl, Ab[0], batch, s);   // dl/d in1 (C -> 1)
        hipLaunchKernelGGL(k_net_extract, dim3(nb), dim3(256), 0, s, (const float2 *)gl, gin_even, batch, g.Vh);
    }
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
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
    hipStream_t s = (hipStream_t)stream;
    switch (channels) {
    case 4: return net_backward_t<4>(g, fat, (const float2 *)weights, acts, (const float2 *)grad_out, (float2 *)grad_w, (float2 *)grad_in, batch, workspace, s);
    case 8: return net_backward_t<8>(g, fat, (const float2 *)weights, acts, (const float2 *)grad_out, (float2 *)grad_w, (float2 *)grad_in, batch, workspace, s);
    default: return net_backward_t<16>(g, fat, (const float2 *)weights, acts, (const float2 *)grad_out, (float2 *)grad_w, (float2 *)grad_in, batch, workspace, s);
    }
}

extern "C" int net_loss(const void *y, const void *x, int batch, const int dims[4], double *loss_host, void *grad_y,
                        void *workspace, size_t ws_bytes, void *stream)
{
    Geom g;
    int rc = make_geom(dims, g);
    if (rc) return rc;
    if (!y || !x || batch < 1) return fail(HISQ_EINVAL, "net_loss: bad argument");
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
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow(0.9, step)), c2 = (float)(1.0 - std::pow(0.999, step));
    const long long n = 2 * n_complex;
    hipLaunchKernelGGL(k_net_adam, dim3((unsigned)std::min<long long>((n + 255) / 256, 1024)), dim3(256), 0,
                       (hipStream_t)stream, (float *)weights, (const float *)grad_w, (float *)m, (float *)v, n,
                       (float)lr, b1, b2, 1e-8f, c1, c2);
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}
