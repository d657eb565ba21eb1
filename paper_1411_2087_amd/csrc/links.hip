// Link construction on the GPU: the three-link (Naik) products of Sec. 4 of
// the paper, path-summed (smeared) one-link matrices and the folding of the
// staggered phases.
//
// Fields are canonical complex128 [mu][t][z][y][x][3][3]: matrix (mu, n) is
// 9 double2 at offset 9 (mu V + lex(n)).  One thread builds one output
// matrix; the 3x3 complex products run in FP64 registers.  All indexing is
// periodic: the boundary sign enters only through hisq_fold_links.
#include <cmath>

#include "hisq_common.hpp"

namespace hisq {

struct M3 {
    double2 e[9];
};

__device__ __forceinline__ M3 ld_m3(const double2 *__restrict__ p)
{
    M3 m;
#pragma unroll
    for (int i = 0; i < 9; ++i) m.e[i] = p[i];
    return m;
}

__device__ __forceinline__ void st_m3(double2 *__restrict__ p, const M3 &m)
{
#pragma unroll
    for (int i = 0; i < 9; ++i) ntstore(m.e[i], p + i);
}

// c = a b, with a and/or b taken as their adjoint
template <bool DA, bool DB>
__device__ __forceinline__ M3 mm(const M3 &a, const M3 &b)
{
    M3 c;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double re = 0, im = 0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double2 x = DA ? a.e[3 * k + i] : a.e[3 * i + k];
                const double2 y = DB ? b.e[3 * j + k] : b.e[3 * k + j];
                const double xi = DA ? -x.y : x.y;
                const double yi = DB ? -y.y : y.y;
                re = fma(x.x, y.x, re);
                re = fma(-xi, yi, re);
                im = fma(x.x, yi, im);
                im = fma(xi, y.x, im);
            }
            c.e[3 * i + j] = make_double2(re, im);
        }
    }
    return c;
}

__device__ __forceinline__ void axpy_m3(double a, const M3 &x, M3 &y)
{
#pragma unroll
    for (int i = 0; i < 9; ++i) y.e[i] = make_double2(fma(a, x.e[i].x, y.e[i].x), fma(a, x.e[i].y, y.e[i].y));
}

struct Lex {
    int L[4];
    long long s[4];  // lex strides 1, Lx, Lx Ly, Lx Ly Lz
    long long V;
};

__device__ __forceinline__ void lex_coords(const Lex &g, long long n, int c[4])
{
    c[0] = (int)(n % g.L[0]);
    n /= g.L[0];
    c[1] = (int)(n % g.L[1]);
    n /= g.L[1];
    c[2] = (int)(n % g.L[2]);
    c[3] = (int)(n / g.L[2]);
}

// lex index of the site n whose coordinates are c, moved by k along mu (|k| < L_mu)
__device__ __forceinline__ long long lex_hop(const Lex &g, long long n, const int c[4], int mu, int k)
{
    int v = c[mu] + k;
    v += (v < 0) ? g.L[mu] : 0;
    v -= (v >= g.L[mu]) ? g.L[mu] : 0;
    return n + (long long)(v - c[mu]) * g.s[mu];
}

__device__ __forceinline__ long long lex_hop2(const Lex &g, long long n, const int c[4], int mu, int k, int nu, int j)
{
    int cc[4] = { c[0], c[1], c[2], c[3] };
    const long long m = lex_hop(g, n, c, mu, k);
    int v = cc[mu] + k;
    cc[mu] = v < 0 ? v + g.L[mu] : (v >= g.L[mu] ? v - g.L[mu] : v);
    return lex_hop(g, m, cc, nu, j);
}

// ------------------------------------------------------------------ LDS staging
// A canonical matrix is 144 contiguous bytes, so a lane that loads its own
// matrix touches a new cache line with every 16-byte load.  The block instead
// reads the NT matrices its threads need cooperatively, consecutive lanes on
// consecutive 16-byte words (contiguous wherever the sites' matrices are),
// through LDS laid out [thread][element]; each thread then takes its 9
// words.  Reads of 16 bytes at a 144-byte lane stride touch 16 different
// bank groups per quarter-wave, so the LDS side runs conflict-free.
template <int NT>
struct Stage {
    double2 m[NT * 9];
    long long idx[NT];
};

// every thread of the block calls this (idx < 0: nothing to load for this thread)
template <int NT>
__device__ __forceinline__ M3 gather(Stage<NT> &st, const double2 *__restrict__ base, long long idx)
{
    __syncthreads();  // the previous use of st is finished
    st.idx[threadIdx.x] = idx;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int q = threadIdx.x + NT * i;
        const int j = q / 9;
        const long long s = st.idx[j];
        if (s >= 0) st.m[q] = base[9 * s + (q - 9 * j)];
    }
    __syncthreads();
    M3 m;
#pragma unroll
    for (int e = 0; e < 9; ++e) m.e[e] = st.m[9 * threadIdx.x + e];
    return m;
}

// store the block's NT matrices to the contiguous out[n0 .. n0 + count)
template <int NT>
__device__ __forceinline__ void scatter(Stage<NT> &st, double2 *__restrict__ out, long long n0, int count, const M3 &m)
{
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 9; ++e) st.m[9 * threadIdx.x + e] = m.e[e];
    __syncthreads();
    double2 *o = out + 9 * n0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int q = threadIdx.x + NT * i;
        if (q < 9 * count) ntstore(st.m[q], o + q);
    }
}

// ------------------------------------------------------------------ three-link products
template <int NT>
__global__ void __launch_bounds__(NT) k_three_link(Lex g, const double2 *__restrict__ thin, double2 *__restrict__ out)
{
    __shared__ Stage<NT> st;
    const long long n0 = (long long)blockIdx.x * NT;
    const long long n = n0 + threadIdx.x;
    const int mu = blockIdx.y;
    const bool live = n < g.V;
    int c[4] = { 0, 0, 0, 0 };
    if (live) lex_coords(g, n, c);
    const double2 *U = thin + 9 * (size_t)mu * g.V;
    const M3 a = gather<NT>(st, U, live ? n : -1);
    const M3 b = gather<NT>(st, U, live ? lex_hop(g, n, c, mu, 1) : -1);
    const M3 ab = mm<false, false>(a, b);
    const M3 d = gather<NT>(st, U, live ? lex_hop(g, n, c, mu, 2) : -1);
    const int count = (int)(g.V - n0 < NT ? g.V - n0 : NT);
    scatter<NT>(st, out + 9 * (size_t)mu * g.V, n0, count, mm<false, false>(ab, d));
}

// ------------------------------------------------------------------ staples
// For the mu-link field Vf and direction nu, at every site n:
//   S(n) = [sign + ] U_nu(n) Vf(n+nu) U_nu(n+mu)^dag
//        + [sign - ] U_nu(n-nu)^dag Vf(n-nu) U_nu(n-nu+mu)
// then  S_out(n) = S(n)                      (if S_out)
//       F(n)     = c_init Uinit(n) + c S(n)   (if Uinit)   or   F(n) += c S(n)   (if F)
enum { ST_PLUS = 1, ST_MINUS = 2 };

template <int NT>
__global__ void __launch_bounds__(NT) k_staple(Lex g, const double2 *__restrict__ thin,
                                               const double2 *__restrict__ Vf, int mu, int nu, int signs,
                                               double2 *__restrict__ S_out, double2 *__restrict__ F, double c,
                                               const double2 *__restrict__ Uinit, double c_init)
{
    __shared__ Stage<NT> st;
    const long long n0 = (long long)blockIdx.x * NT;
    const long long n = n0 + threadIdx.x;
    const bool live = n < g.V;
    const int count = (int)(g.V - n0 < NT ? g.V - n0 : NT);
    int cd[4] = { 0, 0, 0, 0 };
    if (live) lex_coords(g, n, cd);
    const double2 *Un = thin + 9 * (size_t)nu * g.V;
    M3 S;
#pragma unroll
    for (int i = 0; i < 9; ++i) S.e[i] = make_double2(0.0, 0.0);
    if (signs & ST_PLUS) {
        const M3 a = gather<NT>(st, Un, live ? n : -1);
        const M3 v = gather<NT>(st, Vf, live ? lex_hop(g, n, cd, nu, 1) : -1);
        const M3 av = mm<false, false>(a, v);
        const M3 b = gather<NT>(st, Un, live ? lex_hop(g, n, cd, mu, 1) : -1);
        axpy_m3(1.0, mm<false, true>(av, b), S);
    }
    if (signs & ST_MINUS) {
        const long long m = live ? lex_hop(g, n, cd, nu, -1) : -1;
        const M3 a = gather<NT>(st, Un, m);
        const M3 v = gather<NT>(st, Vf, m);
        const M3 av = mm<true, false>(a, v);
        const M3 b = gather<NT>(st, Un, live ? lex_hop2(g, n, cd, nu, -1, mu, 1) : -1);
        axpy_m3(1.0, mm<false, false>(av, b), S);
    }
    if (S_out) scatter<NT>(st, S_out, n0, count, S);
    if (F) {
        M3 f;
        if (Uinit) {
            const M3 u = gather<NT>(st, Uinit, live ? n : -1);
#pragma unroll
            for (int i = 0; i < 9; ++i) f.e[i] = make_double2(c_init * u.e[i].x, c_init * u.e[i].y);
        } else {
            f = gather<NT>(st, F, live ? n : -1);
        }
        axpy_m3(c, S, f);
        scatter<NT>(st, F, n0, count, f);
    }
}

// out = c U (the one-link term alone, when no staple is summed)
template <int NT>
__global__ void __launch_bounds__(NT) k_scale_links(long long n9, const double2 *__restrict__ in,
                                                    double2 *__restrict__ out, double c)
{
    const long long i = (long long)blockIdx.x * NT + threadIdx.x;
    if (i >= n9) return;
    const double2 v = in[i];
    out[i] = make_double2(c * v.x, c * v.y);
}

// ------------------------------------------------------------------ phases
// links_mu(n) *= eta_mu(n) b_mu(n): eta_x = 1, eta_y = (-1)^x, eta_z = (-1)^(x+y),
// eta_t = (-1)^(x+y+z); b = -1 on t-links with t + hop >= Lt when antiperiodic.
template <int NT>
__global__ void __launch_bounds__(NT) k_fold(Lex g, double2 *__restrict__ links, int hop, int anti)
{
    const long long n = (long long)blockIdx.x * NT + threadIdx.x;
    const int mu = blockIdx.y;
    if (n >= g.V) return;
    int c[4];
    lex_coords(g, n, c);
    int e = 0;
    for (int k = 0; k < mu; ++k) e += c[k];
    bool neg = (e & 1) != 0;
    if (mu == 3 && anti && c[3] + hop >= g.L[3]) neg = !neg;
    if (!neg) return;
    double2 *p = links + 9 * ((size_t)mu * g.V + n);
#pragma unroll
    for (int i = 0; i < 9; ++i) p[i] = make_double2(-p[i].x, -p[i].y);
}

static int make_lex(const int dims[4], Lex &l)
{
    Geom g;
    int rc = make_geom(dims, g);
    if (rc) return rc;
    for (int i = 0; i < 4; ++i) l.L[i] = dims[i];
    l.s[0] = 1;
    for (int i = 1; i < 4; ++i) l.s[i] = l.s[i - 1] * dims[i - 1];
    l.V = l.s[3] * dims[3];
    return HISQ_OK;
}

static bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

constexpr int LNT = 256;

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? HISQ_OK : hip_fail(e, what);
}

size_t fat_paths_ws_bytes(const int dims[4])
{
    Lex l;
    if (make_lex(dims, l)) return 0;
    return 3 * align_up((size_t)l.V * 144, 256);
}

}  // namespace hisq

using namespace hisq;

extern "C" int hisq_three_link(const void *thin, void *out, const int dims[4], void *stream)
{
    Lex l;
    int rc = make_lex(dims, l);
    if (rc) return rc;
    if (!thin || !out) return fail(HISQ_EINVAL, "hisq_three_link: NULL pointer");
    if (!aligned16({thin, out}))
        return fail(HISQ_EINVAL, "hisq_three_link: device pointers must be 16-byte aligned");
    const size_t bytes = (size_t)l.V * 4 * 144;
    if (overlaps(thin, bytes, out, bytes)) return fail(HISQ_EALIAS, "hisq_three_link: out overlaps thin");
    dim3 grid((unsigned)((l.V + LNT - 1) / LNT), 4);
    hipLaunchKernelGGL(k_three_link<LNT>, grid, dim3(LNT), 0, (hipStream_t)stream, l, (const double2 *)thin,
                       (double2 *)out);
    return check_launch("hisq_three_link");
}

extern "C" int hisq_fat_paths(const void *thin, const double coeff[5], void *out, const int dims[4], void *workspace,
                              size_t ws_bytes, void *stream)
{
    Lex l;
    int rc = make_lex(dims, l);
    if (rc) return rc;
    if (!thin || !out || !coeff) return fail(HISQ_EINVAL, "hisq_fat_paths: NULL pointer");
    if (!aligned16({thin, out, workspace}))
        return fail(HISQ_EINVAL, "hisq_fat_paths: device pointers must be 16-byte aligned");
    for (int i = 0; i < 5; ++i)
        if (!std::isfinite(coeff[i])) return fail(HISQ_EINVAL, "hisq_fat_paths: coefficient not finite");
    const size_t bytes = (size_t)l.V * 4 * 144;
    if (overlaps(thin, bytes, out, bytes)) return fail(HISQ_EALIAS, "hisq_fat_paths: out overlaps thin");
    const size_t need = fat_paths_ws_bytes(dims);
    if (!workspace || ws_bytes < need)
        return fail(HISQ_EWORKSPACE, "hisq_fat_paths: workspace NULL or smaller than hisq_workspace_bytes()");
    if (overlaps(workspace, need, thin, bytes) || overlaps(workspace, need, out, bytes))
        return fail(HISQ_EALIAS, "hisq_fat_paths: workspace overlaps a link field");
    hipStream_t s = (hipStream_t)stream;
    const size_t fb = align_up((size_t)l.V * 144, 256);
    double2 *T3 = (double2 *)workspace;
    double2 *T5 = (double2 *)((char *)workspace + fb);
    double2 *TL = (double2 *)((char *)workspace + 2 * fb);
    const double c1 = coeff[0], c3 = coeff[1], c5 = coeff[2], c7 = coeff[3], cl = coeff[4];
    const dim3 grid((unsigned)((l.V + LNT - 1) / LNT)), blk(LNT);
    const double2 *U = (const double2 *)thin;
    const bool need3 = c3 != 0 || c5 != 0 || c7 != 0;
    for (int mu = 0; mu < 4; ++mu) {
        const double2 *Umu = U + 9 * (size_t)mu * l.V;
        double2 *F = (double2 *)out + 9 * (size_t)mu * l.V;
        bool init = true;  // the first launch that touches F writes c1 U_mu + c S
        if (!need3 && cl == 0) {
            hipLaunchKernelGGL(k_scale_links<LNT>, dim3((unsigned)((9 * l.V + LNT - 1) / LNT)), blk, 0, s, 9 * l.V,
                               Umu, F, c1);
            continue;
        }
        for (int nu = 0; nu < 4; ++nu) {
            if (nu == mu) continue;
            if (need3) {
                hipLaunchKernelGGL(k_staple<LNT>, grid, blk, 0, s, l, U, Umu, mu, nu, ST_PLUS | ST_MINUS,
                                   (c5 != 0 || c7 != 0) ? T3 : (double2 *)nullptr, F, c3, init ? Umu : nullptr, c1);
                init = false;
            }
            if (cl != 0) {
                for (int sg = ST_PLUS; sg <= ST_MINUS; sg <<= 1) {
                    hipLaunchKernelGGL(k_staple<LNT>, grid, blk, 0, s, l, U, Umu, mu, nu, sg, TL,
                                       (double2 *)nullptr, 0.0, (const double2 *)nullptr, 0.0);
                    hipLaunchKernelGGL(k_staple<LNT>, grid, blk, 0, s, l, U, (const double2 *)TL, mu, nu, sg,
                                       (double2 *)nullptr, F, cl, init ? Umu : nullptr, c1);
                    init = false;
                }
            }
            if (c5 == 0 && c7 == 0) continue;
            for (int rho = 0; rho < 4; ++rho) {
                if (rho == mu || rho == nu) continue;
                hipLaunchKernelGGL(k_staple<LNT>, grid, blk, 0, s, l, U, (const double2 *)T3, mu, rho,
                                   ST_PLUS | ST_MINUS, c7 != 0 ? T5 : (double2 *)nullptr, F, c5, nullptr, 0.0);
                if (c7 == 0) continue;
                const int sig = 6 - mu - nu - rho;
                hipLaunchKernelGGL(k_staple<LNT>, grid, blk, 0, s, l, U, (const double2 *)T5, mu, sig,
                                   ST_PLUS | ST_MINUS, (double2 *)nullptr, F, c7, nullptr, 0.0);
            }
        }
    }
    return check_launch("hisq_fat_paths");
}

extern "C" int hisq_fold_links(void *links, const int dims[4], int hop, int antiperiodic_t, void *stream)
{
    Lex l;
    int rc = make_lex(dims, l);
    if (rc) return rc;
    if (!links) return fail(HISQ_EINVAL, "hisq_fold_links: NULL pointer");
    if (!aligned16({links}))
        return fail(HISQ_EINVAL, "hisq_fold_links: device pointers must be 16-byte aligned");
    if (hop != 1 && hop != 3) return fail(HISQ_EINVAL, "hisq_fold_links: hop must be 1 or 3");
    dim3 grid((unsigned)((l.V + LNT - 1) / LNT), 4);
    hipLaunchKernelGGL(k_fold<LNT>, grid, dim3(LNT), 0, (hipStream_t)stream, l, (double2 *)links, hop,
                       antiperiodic_t ? 1 : 0);
    return check_launch("hisq_fold_links");
}
