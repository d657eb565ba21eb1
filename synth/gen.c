/*
 * Seeded synthetic inputs for the staggered (HISQ) Dslash and its CG solve.
 *
 * This module only draws random numbers and lays them out: gauge links,
 * sources and gauge transformations.  It holds none of the operator's
 * arithmetic and is shared, as input, by the CPU oracle and the GPU library.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC11), written here from its published
 * definition.  Every value is a pure function of (seed, counter), so a field
 * is reproducible element by element regardless of thread count.
 *
 * Layouts (complex numbers are interleaved re, im doubles):
 *   links   [mu=x,y,z,t][lex][row][col],  lex = x + Lx*(y + Ly*(z + Lz*t))
 *   vectors [h][color] over the sites of one parity, h = lex >> 1
 *
 * Workload of the paper's benchmark problem (Sec. 3): HISQ links, i.e. a
 * smeared one-link ("fat") field and a three-link ("long") field; here the
 * fat link is 0.6 * Haar SU(3) + 0.1 * complex Gaussian noise and the long
 * link is Haar SU(3), with the staggered phases (Sec. 4) and the
 * time-direction boundary sign folded in by syn_fold().
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

/* stream identifiers (third counter word, high byte = kind) */
enum { KIND_FAT = 1, KIND_LONG = 2, KIND_SRC = 3, KIND_HAAR = 4, KIND_GAUSS = 5 };

void syn_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* One complex Gaussian z = (g1 + i g2)/sqrt(2), E|z|^2 = 1, from one Philox
 * block: two 53-bit uniforms, then Box-Muller. */
static void cgauss(uint64_t seed, uint64_t index, uint32_t stream, uint32_t block, double z[2])
{
    uint32_t ctr[4] = { (uint32_t)index, (uint32_t)(index >> 32), stream, block };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t r[4];
    syn_philox4x32_10(ctr, key, r);
    const double inv53 = 1.0 / 9007199254740992.0; /* 2^-53 */
    double u1 = ((double)(r[0] >> 5) * 67108864.0 + (double)(r[1] >> 6)) * inv53;
    double u2 = ((double)(r[2] >> 5) * 67108864.0 + (double)(r[3] >> 6)) * inv53;
    u1 = 1.0 - u1; /* (0, 1] so that log is finite */
    double rad = sqrt(-2.0 * log(u1));
    double th = 6.283185307179586476925286766559 * u2;
    const double s = 0.70710678118654752440084436210485;
    z[0] = s * rad * cos(th);
    z[1] = s * rad * sin(th);
}

/* 3x3 complex matrix m[row][col][re/im] filled with complex Gaussians from
 * blocks first_block .. first_block+8. */
static void gauss_matrix(uint64_t seed, uint64_t index, uint32_t stream, uint32_t first_block, double m[18])
{
    for (int e = 0; e < 9; ++e) cgauss(seed, index, stream, first_block + (uint32_t)e, &m[2 * e]);
}

/* Haar-distributed SU(3) from a Gaussian matrix (Mezzadri, "How to generate
 * random matrices from the classical compact groups", 2007): orthonormalise
 * the columns (Gram-Schmidt, which is the QR factorisation with a positive
 * real diagonal in R), then remove the determinant's phase with one cube
 * root.  Left-multiplying the Gaussian matrix by a fixed SU(3) element leaves
 * its law and the determinant unchanged, so the result is left-invariant,
 * i.e. Haar on SU(3). */
static void haar_from_gauss(double m[18])
{
    for (int c = 0; c < 3; ++c) {
        /* two projection passes ("twice is enough", Giraud et al. 2005) keep
         * the columns orthonormal to rounding even for ill-conditioned draws */
        for (int pass = 0; pass < 2; ++pass)
        for (int k = 0; k < c; ++k) {
            /* proj = <q_k, v_c> = sum_r conj(q_rk) v_rc */
            double pr = 0.0, pi = 0.0;
            for (int r = 0; r < 3; ++r) {
                double qr = m[2 * (3 * r + k)], qi = m[2 * (3 * r + k) + 1];
                double vr = m[2 * (3 * r + c)], vi = m[2 * (3 * r + c) + 1];
                pr += qr * vr + qi * vi;
                pi += qr * vi - qi * vr;
            }
            for (int r = 0; r < 3; ++r) {
                double qr = m[2 * (3 * r + k)], qi = m[2 * (3 * r + k) + 1];
                m[2 * (3 * r + c)] -= pr * qr - pi * qi;
                m[2 * (3 * r + c) + 1] -= pr * qi + pi * qr;
            }
        }
        double nrm = 0.0;
        for (int r = 0; r < 3; ++r) nrm += m[2 * (3 * r + c)] * m[2 * (3 * r + c)] + m[2 * (3 * r + c) + 1] * m[2 * (3 * r + c) + 1];
        nrm = 1.0 / sqrt(nrm);
        for (int r = 0; r < 3; ++r) { m[2 * (3 * r + c)] *= nrm; m[2 * (3 * r + c) + 1] *= nrm; }
    }
    /* det by cofactor expansion along row 0 */
#define RE(r, c) m[2 * (3 * (r) + (c))]
#define IM(r, c) m[2 * (3 * (r) + (c)) + 1]
    double c0r = RE(1,1)*RE(2,2) - IM(1,1)*IM(2,2) - (RE(1,2)*RE(2,1) - IM(1,2)*IM(2,1));
    double c0i = RE(1,1)*IM(2,2) + IM(1,1)*RE(2,2) - (RE(1,2)*IM(2,1) + IM(1,2)*RE(2,1));
    double c1r = RE(1,2)*RE(2,0) - IM(1,2)*IM(2,0) - (RE(1,0)*RE(2,2) - IM(1,0)*IM(2,2));
    double c1i = RE(1,2)*IM(2,0) + IM(1,2)*RE(2,0) - (RE(1,0)*IM(2,2) + IM(1,0)*RE(2,2));
    double c2r = RE(1,0)*RE(2,1) - IM(1,0)*IM(2,1) - (RE(1,1)*RE(2,0) - IM(1,1)*IM(2,0));
    double c2i = RE(1,0)*IM(2,1) + IM(1,0)*RE(2,1) - (RE(1,1)*IM(2,0) + IM(1,1)*RE(2,0));
    double dr = RE(0,0)*c0r - IM(0,0)*c0i + RE(0,1)*c1r - IM(0,1)*c1i + RE(0,2)*c2r - IM(0,2)*c2i;
    double di = RE(0,0)*c0i + IM(0,0)*c0r + RE(0,1)*c1i + IM(0,1)*c1r + RE(0,2)*c2i + IM(0,2)*c2r;
#undef RE
#undef IM
    double ph = -atan2(di, dr) / 3.0;
    double fr = cos(ph), fi = sin(ph);
    for (int e = 0; e < 9; ++e) {
        double a = m[2 * e], b = m[2 * e + 1];
        m[2 * e] = a * fr - b * fi;
        m[2 * e + 1] = a * fi + b * fr;
    }
}

static int64_t volume(const int d[4]) { return (int64_t)d[0] * d[1] * d[2] * d[3]; }

/* Unfolded random links: fat = 0.6*U + 0.1*Z, long = U' (U, U' Haar SU(3),
 * Z complex Gaussian).  Either output may be NULL. */
void syn_links(const int dims[4], uint64_t seed, double *fat, double *lng)
{
    const int64_t V = volume(dims);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        for (int mu = 0; mu < 4; ++mu) {
            double u[18], z[18];
            if (fat) {
                gauss_matrix(seed, (uint64_t)s, (KIND_FAT << 24) | (uint32_t)mu, 0, u);
                haar_from_gauss(u);
                gauss_matrix(seed, (uint64_t)s, (KIND_FAT << 24) | (uint32_t)mu, 9, z);
                double *o = fat + ((int64_t)mu * V + s) * 18;
                for (int e = 0; e < 18; ++e) o[e] = 0.6 * u[e] + 0.1 * z[e];
            }
            if (lng) {
                gauss_matrix(seed, (uint64_t)s, (KIND_LONG << 24) | (uint32_t)mu, 0, u);
                haar_from_gauss(u);
                double *o = lng + ((int64_t)mu * V + s) * 18;
                memcpy(o, u, sizeof(u));
            }
        }
    }
}

/* Free-field links c1 * 1 (fat) and c3 * 1 (long), unfolded. */
void syn_unit_links(const int dims[4], double c1, double c3, double *fat, double *lng)
{
    const int64_t V = volume(dims);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < 4 * V; ++s) {
        double *f = fat + s * 18, *l = lng + s * 18;
        memset(f, 0, 18 * sizeof(double));
        memset(l, 0, 18 * sizeof(double));
        for (int a = 0; a < 3; ++a) { f[2 * (4 * a)] = c1; l[2 * (4 * a)] = c3; }
    }
}

/* Fold the staggered phases and the time boundary sign into the links, in
 * place.  Phases (the MILC convention; the paper absorbs them into the gauge
 * field, Sec. 4): eta_x = 1, eta_y = (-1)^x, eta_z = (-1)^(x+y),
 * eta_t = (-1)^(x+y+z).  With antiperiodic_t, a t-link that crosses the
 * t = Lt-1 -> 0 boundary changes sign: the fat link at t = Lt-1 and the long
 * (three-hop) links at t >= Lt-3. */
void syn_fold(const int dims[4], int antiperiodic_t, double *fat, double *lng)
{
    const int64_t V = volume(dims);
    const int Lx = dims[0], Ly = dims[1], Lz = dims[2], Lt = dims[3];
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        int x = (int)(s % Lx);
        int y = (int)((s / Lx) % Ly);
        int z = (int)((s / ((int64_t)Lx * Ly)) % Lz);
        int t = (int)(s / ((int64_t)Lx * Ly * Lz));
        for (int mu = 0; mu < 4; ++mu) {
            int eta_exp = (mu == 0) ? 0 : (mu == 1) ? x : (mu == 2) ? x + y : x + y + z;
            double sf = (eta_exp & 1) ? -1.0 : 1.0;
            double sl = sf;
            if (mu == 3 && antiperiodic_t) {
                if (t + 1 >= Lt) sf = -sf;
                if (t + 3 >= Lt) sl = -sl;
            }
            double *f = fat + ((int64_t)mu * V + s) * 18;
            double *l = lng + ((int64_t)mu * V + s) * 18;
            for (int e = 0; e < 18; ++e) { f[e] *= sf; l[e] *= sl; }
        }
    }
}

/* Complex Gaussian colour vectors on the Vh = V/2 sites of one parity,
 * [h][color]; `rhs` selects an independent stream. */
void syn_source(const int dims[4], uint64_t seed, int rhs, double *out)
{
    const int64_t Vh = volume(dims) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t h = 0; h < Vh; ++h)
        for (int c = 0; c < 3; ++c)
            cgauss(seed, (uint64_t)h, (KIND_SRC << 24) | (uint32_t)rhs, (uint32_t)c, out + (h * 3 + c) * 2);
}

/* n independent Haar SU(3) matrices [n][3][3] (gauge transformations). */
void syn_haar(uint64_t seed, int64_t n, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double m[18];
        gauss_matrix(seed, (uint64_t)i, KIND_HAAR << 24, 0, m);
        haar_from_gauss(m);
        memcpy(out + i * 18, m, sizeof(m));
    }
}

/* n complex Gaussians (E|z|^2 = 1) on stream `stream` (initial weights,
 * training sources). */
void syn_gauss(uint64_t seed, uint32_t stream, int64_t n, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        cgauss(seed, (uint64_t)i, (KIND_GAUSS << 24) | (stream & 0xFFFFFFu), 0, out + 2 * i);
}
