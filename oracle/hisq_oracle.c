/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 implementation of the improved-staggered (HISQ) Dslash
 * and the even-odd conjugate-gradient solve it drives, written from the
 * paper's description of the operator (Sec. 3: at each site, for each of the
 * eight positive and negative directions, a one-link and a three-link matrix
 * multiply a neighbouring colour vector: 16 matrix-vector products and 15
 * vector sums, 1146 flops) and of even-odd preconditioning (Sec. 4).  Only the
 * test-suite, the package smoke check and the benchmark's CPU-baseline leg
 * may load this library; the GPU library shares no code with it.
 *
 * Conventions (readings of what the paper leaves unstated):
 *   sites      n = (x,y,z,t), lex = x + Lx*(y + Ly*(z + Lz*t)), parity (x+y+z+t) mod 2
 *   vectors    [h][color] complex over the Vh = V/2 sites of one parity, h = lex >> 1
 *   links      [mu][lex][row][col] complex, staggered phases and boundary signs
 *              already folded in (the paper absorbs the phases into the gauge field)
 *   Dslash     (D psi)(n) = sum_mu  F_mu(n) psi(n+mu) - F_mu(n-mu)^dag psi(n-mu)
 *                                 + L_mu(n) psi(n+3mu) - L_mu(n-3mu)^dag psi(n-3mu)
 *              neighbours taken periodically; no factor 1/2
 *   even-odd   A = 4 m^2 - D_eo D_oe on the even sites (M = 2m + D, A = M^dag M
 *              restricted to even sites), Hermitian positive definite
 *   CG         textbook Hestenes-Stiefel from x0, stop when |r| <= tol |b|, then
 *              recompute r = b - A x and restart from x (at most 3 restarts)
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static int64_t vol(const int L[4]) { return (int64_t)L[0] * L[1] * L[2] * L[3]; }

static void coords(int64_t lex, const int L[4], int c[4])
{
    for (int mu = 0; mu < 4; ++mu) { c[mu] = (int)(lex % L[mu]); lex /= L[mu]; }
}

static int64_t lex_of(const int c[4], const int L[4])
{
    return c[0] + (int64_t)L[0] * (c[1] + (int64_t)L[1] * (c[2] + (int64_t)L[2] * c[3]));
}

/* lexicographic index of the site with checkerboard index h and parity p:
 * lex is 2h or 2h+1, the two neighbours along x in one row (Lx is even) */
static int64_t site_of_h(int64_t h, int p, const int L[4])
{
    int c[4];
    coords(2 * h, L, c);
    return (((c[0] + c[1] + c[2] + c[3]) & 1) == p) ? 2 * h : 2 * h + 1;
}

/* lex of n + k * mu-hat, periodic */
static int64_t shifted(const int c[4], int mu, int k, const int L[4])
{
    int d[4] = { c[0], c[1], c[2], c[3] };
    d[mu] = ((d[mu] + k) % L[mu] + L[mu]) % L[mu];
    return lex_of(d, L);
}

static const cplx *link(const cplx *U, int mu, int64_t lex, int64_t V) { return U + ((int64_t)mu * V + lex) * 9; }

/* acc += sign * M psi  (M row-major 3x3) */
static void madd(cplx acc[3], double sign, const cplx *M, const cplx *psi)
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) acc[a] += sign * M[3 * a + b] * psi[b];
}

/* acc += sign * M^dag psi */
static void madd_dag(cplx acc[3], double sign, const cplx *M, const cplx *psi)
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) acc[a] += sign * conj(M[3 * b + a]) * psi[b];
}

/* dst (parity p) = D src (parity 1-p).  Sec. 3: 16 links, 16 neighbours. */
void or_dslash(const int L[4], const double *fat_, const double *lng_, const double *src_, double *dst_, int p)
{
    const cplx *fat = (const cplx *)fat_, *lng = (const cplx *)lng_, *src = (const cplx *)src_;
    cplx *dst = (cplx *)dst_;
    const int64_t V = vol(L), Vh = V / 2;
#pragma omp parallel for schedule(static)
    for (int64_t h = 0; h < Vh; ++h) {
        int64_t n = site_of_h(h, p, L);
        int c[4];
        coords(n, L, c);
        cplx acc[3] = { 0, 0, 0 };
        for (int mu = 0; mu < 4; ++mu) {
            int64_t f1 = shifted(c, mu, +1, L), b1 = shifted(c, mu, -1, L);
            int64_t f3 = shifted(c, mu, +3, L), b3 = shifted(c, mu, -3, L);
            madd(acc, +1.0, link(fat, mu, n, V), src + (f1 >> 1) * 3);
            madd_dag(acc, -1.0, link(fat, mu, b1, V), src + (b1 >> 1) * 3);
            madd(acc, +1.0, link(lng, mu, n, V), src + (f3 >> 1) * 3);
            madd_dag(acc, -1.0, link(lng, mu, b3, V), src + (b3 >> 1) * 3);
        }
        for (int a = 0; a < 3; ++a) dst[h * 3 + a] = acc[a];
    }
}

/* Componentwise scale of the Dslash: scale[h][a] = sum over the 16 terms and
 * the colour b of |M_ab| |psi_b| (|(M^dag)_ab| = |M_ba| for the backward
 * terms), the natural bound for the rounding error of output component (h, a). */
void or_dslash_absscale(const int L[4], const double *fat_, const double *lng_, const double *src_,
                              double *scale, int p)
{
    const cplx *fat = (const cplx *)fat_, *lng = (const cplx *)lng_, *src = (const cplx *)src_;
    const int64_t V = vol(L), Vh = V / 2;
#pragma omp parallel for schedule(static)
    for (int64_t h = 0; h < Vh; ++h) {
        int64_t n = site_of_h(h, p, L);
        int c[4];
        coords(n, L, c);
        double acc[3] = { 0, 0, 0 };
        for (int mu = 0; mu < 4; ++mu) {
            int64_t f1 = shifted(c, mu, +1, L), b1 = shifted(c, mu, -1, L);
            int64_t f3 = shifted(c, mu, +3, L), b3 = shifted(c, mu, -3, L);
            const cplx *Mf1 = link(fat, mu, n, V), *Mb1 = link(fat, mu, b1, V);
            const cplx *Mf3 = link(lng, mu, n, V), *Mb3 = link(lng, mu, b3, V);
            const cplx *pf1 = src + (f1 >> 1) * 3, *pb1 = src + (b1 >> 1) * 3;
            const cplx *pf3 = src + (f3 >> 1) * 3, *pb3 = src + (b3 >> 1) * 3;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    acc[a] += cabs(Mf1[3 * a + b]) * cabs(pf1[b]) + cabs(Mb1[3 * b + a]) * cabs(pb1[b]) +
                              cabs(Mf3[3 * a + b]) * cabs(pf3[b]) + cabs(Mb3[3 * b + a]) * cabs(pb3[b]);
        }
        for (int a = 0; a < 3; ++a) scale[h * 3 + a] = acc[a];
    }
}

/* y = A x = 4 m^2 x - D_eo D_oe x on even sites; tmp holds Vh odd vectors. */
void or_apply_A(const int L[4], double mass, const double *fat, const double *lng, const double *x_, double *y_,
                double *tmp)
{
    const int64_t n3 = vol(L) / 2 * 3;
    or_dslash(L, fat, lng, x_, tmp, 1);
    or_dslash(L, fat, lng, tmp, y_, 0);
    const cplx *x = (const cplx *)x_;
    cplx *y = (cplx *)y_;
    const double m2 = 4.0 * mass * mass;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n3; ++i) y[i] = m2 * x[i] - y[i];
}

double or_norm2(int64_t n3, const double *x_)
{
    const cplx *x = (const cplx *)x_;
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t i = 0; i < n3; ++i) s += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
    return s;
}

/* <x, y> = sum conj(x) y; result in out[0] (re), out[1] (im) */
void or_dot(int64_t n3, const double *x_, const double *y_, double out[2])
{
    const cplx *x = (const cplx *)x_, *y = (const cplx *)y_;
    double sr = 0.0, si = 0.0;
#pragma omp parallel for reduction(+ : sr, si) schedule(static)
    for (int64_t i = 0; i < n3; ++i) {
        cplx v = conj(x[i]) * y[i];
        sr += creal(v);
        si += cimag(v);
    }
    out[0] = sr;
    out[1] = si;
}

/* |b - A x| / |b| */
double or_true_residual(const int L[4], double mass, const double *fat, const double *lng, const double *b_,
                        const double *x_)
{
    const int64_t n3 = vol(L) / 2 * 3;
    double *ax = (double *)malloc(sizeof(cplx) * n3);
    double *tmp = (double *)malloc(sizeof(cplx) * n3);
    or_apply_A(L, mass, fat, lng, x_, ax, tmp);
    const cplx *b = (const cplx *)b_;
    cplx *r = (cplx *)ax;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n3; ++i) r[i] = b[i] - r[i];
    double rr = or_norm2(n3, ax), bb = or_norm2(n3, b_);
    free(ax);
    free(tmp);
    return bb > 0 ? sqrt(rr / bb) : sqrt(rr);
}

/* Conjugate gradient on A x = b (even sites).  x holds x0 on entry and the
 * solution on exit.  history (may be NULL) receives |r_k|/|b| of the
 * recursively updated residual for k = 0 .. max_iter.  Returns 0 when the
 * recomputed residual meets tol, 1 otherwise; *iters counts all iterations,
 * *true_rel the final |b - A x|/|b|. */
int or_cg(const int L[4], double mass, double tol, int max_iter, const double *fat, const double *lng,
          const double *b_, double *x_, int *iters, double *true_rel, double *history)
{
    const int64_t n3 = vol(L) / 2 * 3;
    cplx *r = (cplx *)malloc(sizeof(cplx) * n3);
    cplx *p = (cplx *)malloc(sizeof(cplx) * n3);
    cplx *ap = (cplx *)malloc(sizeof(cplx) * n3);
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * n3);
    const cplx *b = (const cplx *)b_;
    cplx *x = (cplx *)x_;
    const double bb = or_norm2(n3, b_);
    int k = 0, status = 1;
    if (bb == 0.0) {
        memset(x, 0, sizeof(cplx) * n3);
        if (iters) *iters = 0;
        if (true_rel) *true_rel = 0.0;
        free(r); free(p); free(ap); free(tmp);
        return 0;
    }
    for (int restart = 0; restart <= 3 && k < max_iter; ++restart) {
        /* r = b - A x, p = r */
        or_apply_A(L, mass, fat, lng, (const double *)x, (double *)ap, (double *)tmp);
        for (int64_t i = 0; i < n3; ++i) { r[i] = b[i] - ap[i]; p[i] = r[i]; }
        double rr = or_norm2(n3, (const double *)r);
        if (history && restart == 0) history[0] = sqrt(rr / bb);
        if (rr <= tol * tol * bb) { status = 0; break; }
        while (k < max_iter) {
            or_apply_A(L, mass, fat, lng, (const double *)p, (double *)ap, (double *)tmp);
            double pap[2];
            or_dot(n3, (const double *)p, (const double *)ap, pap);
            double alpha = rr / pap[0];
            for (int64_t i = 0; i < n3; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * ap[i]; }
            double rr_new = or_norm2(n3, (const double *)r);
            ++k;
            if (history) history[k] = sqrt(rr_new / bb);
            if (rr_new <= tol * tol * bb) break;
            double beta = rr_new / rr;
            for (int64_t i = 0; i < n3; ++i) p[i] = r[i] + beta * p[i];
            rr = rr_new;
        }
        double tr = or_true_residual(L, mass, fat, lng, b_, (const double *)x);
        if (true_rel) *true_rel = tr;
        if (tr <= tol) { status = 0; break; }
    }
    if (iters) *iters = k;
    free(r); free(p); free(ap); free(tmp);
    return status;
}

/* number of OpenMP threads the oracle's parallel loops use */
#ifdef _OPENMP
#include <omp.h>
#endif
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the parallel loops from now on (timing runs) */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
