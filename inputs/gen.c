/*
 * Seeded synthetic inputs: SU(3) gauge fields and random sources.
 *
 * This file is shared by the FP64 oracle tests and by the GPU path's tests and
 * benchmark.  It contains none of the method's arithmetic (no Dirac operator,
 * no solver, no contraction): only a counter-based random generator and the
 * standard quenched gauge-field update used to produce the link fields.
 *
 *  - Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11 "Parallel random numbers:
 *    as easy as 1, 2, 3"), written from its published definition.
 *  - Links U = exp(i eps H), H = sum_a h_a lambda_a / 2, h_a ~ N(0,1).
 *  - Wilson plaquette action at coupling beta, updated by Cabibbo-Marinari
 *    pseudo-heatbath over the three SU(2) subgroups with the Kennedy-Pendleton
 *    SU(2) sampler, plus SU(2) over-relaxation.  The paper generates its
 *    ensembles with HMC; any correct algorithm samples the same distribution.
 *
 * Layouts: sites lexicographic with time slowest, idx = ((t*L1+x1)*L2+x2)*L3+x3;
 * links [site][mu][3][3] row-major complex128, U_mu(x) joins x and x+mu.
 * Every random draw is keyed by (seed, stream) with a counter built from the
 * link coordinates and the sweep number, so the result does not depend on the
 * number of threads.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------ Philox */
static inline void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

void gen_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(0xD2511F53u, c0, &hi0, &lo0);
        mulhilo32(0xCD9E8D57u, c2, &hi1, &lo1);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A stream of uniforms in (0,1] drawn from one Philox counter family. */
typedef struct {
    uint32_t key[2];
    uint32_t ctr[4];
    uint32_t buf[4];
    int used;
} rng_t;

static void rng_init(rng_t *r, uint64_t seed, uint32_t stream, uint32_t a, uint32_t b, uint32_t c)
{
    r->key[0] = (uint32_t)seed;
    r->key[1] = (uint32_t)(seed >> 32) ^ (stream * 0x85EBCA6Bu);
    r->ctr[0] = a; r->ctr[1] = b; r->ctr[2] = c; r->ctr[3] = 0;
    r->used = 4;
}

static double rng_uniform(rng_t *r) /* (0,1] */
{
    if (r->used == 4) {
        gen_philox4x32_10(r->ctr, r->key, r->buf);
        r->ctr[3]++;
        r->used = 0;
    }
    uint32_t u = r->buf[r->used++];
    return ((double)u + 1.0) * (1.0 / 4294967296.0);
}

static double rng_normal(rng_t *r)
{
    double u1 = rng_uniform(r), u2 = rng_uniform(r);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

/* ----------------------------------------------------------- SU(3) helpers */
static inline void m3_mul(const cplx *a, const cplx *b, cplx *c)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            c[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}
static inline void m3_mul_an(const cplx *a, const cplx *b, cplx *c) /* a^dag b */
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            c[3 * i + j] = conj(a[i]) * b[j] + conj(a[3 + i]) * b[3 + j] + conj(a[6 + i]) * b[6 + j];
}
static inline void m3_mul_na(const cplx *a, const cplx *b, cplx *c) /* a b^dag */
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            c[3 * i + j] = a[3 * i] * conj(b[3 * j]) + a[3 * i + 1] * conj(b[3 * j + 1]) +
                           a[3 * i + 2] * conj(b[3 * j + 2]);
}

/* Project a 3x3 matrix onto SU(3): Gram-Schmidt on rows 0,1, row 2 = conj(r0 x r1). */
static void su3_reunit(cplx *u)
{
    double n = 0;
    for (int j = 0; j < 3; ++j) n += creal(u[j] * conj(u[j]));
    n = 1.0 / sqrt(n);
    for (int j = 0; j < 3; ++j) u[j] *= n;
    cplx d = 0;
    for (int j = 0; j < 3; ++j) d += conj(u[j]) * u[3 + j];
    for (int j = 0; j < 3; ++j) u[3 + j] -= d * u[j];
    n = 0;
    for (int j = 0; j < 3; ++j) n += creal(u[3 + j] * conj(u[3 + j]));
    n = 1.0 / sqrt(n);
    for (int j = 0; j < 3; ++j) u[3 + j] *= n;
    u[6] = conj(u[1] * u[5] - u[2] * u[4]);
    u[7] = conj(u[2] * u[3] - u[0] * u[5]);
    u[8] = conj(u[0] * u[4] - u[1] * u[3]);
}

/* exp(i eps H) for H Hermitian, by scaling-and-squaring of a Taylor series. */
static void su3_exp_iH(const cplx *H, double eps, cplx *out)
{
    cplx X[9];
    double nrm = 0;
    for (int k = 0; k < 9; ++k) {
        X[k] = I * eps * H[k];
        nrm += creal(X[k] * conj(X[k]));
    }
    nrm = sqrt(nrm);
    int s = 0;
    while (nrm > 0.05) { nrm *= 0.5; ++s; }
    double sc = ldexp(1.0, -s);
    for (int k = 0; k < 9; ++k) X[k] *= sc;
    cplx R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, T[9], P[9];
    memcpy(T, R, sizeof T);
    for (int n = 1; n <= 14; ++n) {
        m3_mul(T, X, P);
        for (int k = 0; k < 9; ++k) T[k] = P[k] / (double)n;
        for (int k = 0; k < 9; ++k) R[k] += T[k];
    }
    for (int i = 0; i < s; ++i) {
        m3_mul(R, R, P);
        memcpy(R, P, sizeof P);
    }
    su3_reunit(R);
    memcpy(out, R, sizeof R);
}

/* ---------------------------------------------------------------- geometry */
typedef struct { int L[4]; long V; } geom_t;

static inline long site_index(const geom_t *g, const int x[4])
{
    return ((long)(x[0] * g->L[1] + x[1]) * g->L[2] + x[2]) * g->L[3] + x[3];
}
static inline void site_coords(const geom_t *g, long idx, int x[4])
{
    x[3] = (int)(idx % g->L[3]); idx /= g->L[3];
    x[2] = (int)(idx % g->L[2]); idx /= g->L[2];
    x[1] = (int)(idx % g->L[1]); idx /= g->L[1];
    x[0] = (int)idx;
}
static inline long shift(const geom_t *g, const int x[4], int mu, int d)
{
    int y[4] = {x[0], x[1], x[2], x[3]};
    y[mu] = (y[mu] + d + g->L[mu]) % g->L[mu];
    return site_index(g, y);
}

#define LINK(U, s, mu) ((U) + ((s) * 4 + (mu)) * 9)

/* ------------------------------------------------------- public generators */

/* U_mu(x) = exp(i eps H), H = sum_a h_a lambda_a/2 with h_a ~ N(0,1). */
void gen_random_links(const int L[4], uint64_t seed, double eps, double *Uout)
{
    geom_t g = {{L[0], L[1], L[2], L[3]}, (long)L[0] * L[1] * L[2] * L[3]};
    cplx *U = (cplx *)Uout;
    const double s3 = 1.0 / sqrt(3.0);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; ++s) {
        for (int mu = 0; mu < 4; ++mu) {
            rng_t r;
            rng_init(&r, seed, 1u, (uint32_t)s, (uint32_t)mu, 0u);
            double h[8];
            for (int a = 0; a < 8; ++a) h[a] = rng_normal(&r);
            /* sum_a h_a lambda_a / 2 written out with the Gell-Mann matrices */
            cplx H[9];
            H[0] = 0.5 * (h[2] + s3 * h[7]);
            H[4] = 0.5 * (-h[2] + s3 * h[7]);
            H[8] = 0.5 * (-2.0 * s3 * h[7]);
            H[1] = 0.5 * (h[0] - I * h[1]);
            H[3] = conj(H[1]);
            H[2] = 0.5 * (h[3] - I * h[4]);
            H[6] = conj(H[2]);
            H[5] = 0.5 * (h[5] - I * h[6]);
            H[7] = conj(H[5]);
            su3_exp_iH(H, eps, LINK(U, s, mu));
        }
    }
}

/* Sum of staples A with S_local = -(beta/3) Re tr(U_mu(x) A). */
static void staple(const geom_t *g, const cplx *U, long s, int mu, cplx *A)
{
    int x[4];
    site_coords(g, s, x);
    memset(A, 0, 9 * sizeof(cplx));
    long xpm = shift(g, x, mu, 1);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        cplx t1[9], t2[9];
        /* upper: U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag */
        long xpn = shift(g, x, nu, 1);
        m3_mul_na(LINK(U, xpm, nu), LINK(U, xpn, mu), t1);
        m3_mul_na(t1, LINK(U, s, nu), t2);
        for (int k = 0; k < 9; ++k) A[k] += t2[k];
        /* lower: U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu) */
        int xm[4] = {x[0], x[1], x[2], x[3]};
        xm[nu] = (xm[nu] - 1 + g->L[nu]) % g->L[nu];
        long xmn = site_index(g, xm);
        long xpmmn = shift(g, xm, mu, 1);
        cplx t3[9];
        m3_mul(LINK(U, xmn, mu), LINK(U, xpmmn, nu), t1); /* U_mu(x-nu) U_nu(x+mu-nu) */
        /* (U_mu(x-nu) U_nu(x+mu-nu))^dag U_nu(x-nu) */
        m3_mul_an(t1, LINK(U, xmn, nu), t3);
        for (int k = 0; k < 9; ++k) A[k] += t3[k];
    }
}

/* SU(2) element as quaternion (a0, a1, a2, a3): a0 + i a.sigma. */
static void su2_from_block(const cplx *W, int i, int j, double a[4])
{
    cplx w00 = W[3 * i + i], w01 = W[3 * i + j], w10 = W[3 * j + i], w11 = W[3 * j + j];
    a[0] = 0.5 * creal(w00 + w11);
    a[3] = 0.5 * cimag(w00 - w11);
    a[2] = 0.5 * creal(w01 - w10);
    a[1] = 0.5 * cimag(w01 + w10);
}
/* Left-multiply rows i,j of U by the 2x2 matrix of quaternion r. */
static void su2_apply_left(const double r[4], int i, int j, cplx *U)
{
    cplx m00 = r[0] + I * r[3], m01 = r[2] + I * r[1];
    cplx m10 = -r[2] + I * r[1], m11 = r[0] - I * r[3];
    for (int c = 0; c < 3; ++c) {
        cplx ui = U[3 * i + c], uj = U[3 * j + c];
        U[3 * i + c] = m00 * ui + m01 * uj;
        U[3 * j + c] = m10 * ui + m11 * uj;
    }
}
static inline void quat_mul(const double a[4], const double b[4], double c[4])
{
    /* (a0 + i a.s)(b0 + i b.s) = a0b0 - a.b + i(a0 b + b0 a - a x b) */
    c[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    c[1] = a[0] * b[1] + b[0] * a[1] - (a[2] * b[3] - a[3] * b[2]);
    c[2] = a[0] * b[2] + b[0] * a[2] - (a[3] * b[1] - a[1] * b[3]);
    c[3] = a[0] * b[3] + b[0] * a[3] - (a[1] * b[2] - a[2] * b[1]);
}

/* One link: Cabibbo-Marinari heatbath then n_or over-relaxation passes. */
static void update_link(cplx *Ul, const cplx *A, double beta, int n_hb, int n_or, rng_t *r)
{
    static const int sub[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int pass = 0; pass < n_hb + n_or; ++pass) {
        for (int k = 0; k < 3; ++k) {
            cplx W[9];
            m3_mul(Ul, A, W);
            double a[4];
            su2_from_block(W, sub[k][0], sub[k][1], a);
            double kk = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3]);
            if (kk < 1e-14) continue;
            double v[4] = {a[0] / kk, a[1] / kk, a[2] / kk, a[3] / kk};
            double vd[4] = {v[0], -v[1], -v[2], -v[3]};
            double R[4];
            if (pass < n_hb) {
                /* weight exp((beta/3) Re tr_2(R W)) = exp(alpha x0), alpha = 2 beta k / 3 */
                double alpha = 2.0 * beta * kk / 3.0, x0;
                for (int tries = 0;; ++tries) {
                    double r1 = rng_uniform(r), r2 = rng_uniform(r), r3 = rng_uniform(r), r4 = rng_uniform(r);
                    double c = cos(2.0 * M_PI * r2);
                    double lam2 = -(log(r1) + c * c * log(r3)) / (2.0 * alpha);
                    if (r4 * r4 <= 1.0 - lam2) { x0 = 1.0 - 2.0 * lam2; break; }
                    if (tries > 10000) { x0 = 1.0; break; }
                }
                double rad = sqrt(fmax(0.0, 1.0 - x0 * x0));
                double ct = 2.0 * rng_uniform(r) - 1.0, ph = 2.0 * M_PI * rng_uniform(r);
                double st = sqrt(fmax(0.0, 1.0 - ct * ct));
                double X[4] = {x0, rad * st * cos(ph), rad * st * sin(ph), rad * ct};
                quat_mul(X, vd, R); /* R = X V^dag */
            } else {
                quat_mul(vd, vd, R); /* R = (V^dag)^2 keeps Re tr(R W) fixed */
            }
            su2_apply_left(R, sub[k][0], sub[k][1], Ul);
        }
    }
    su3_reunit(Ul);
}

/* Sweeps over the links of the time range [t0,t1).  If freeze_first_slice,
 * the spatial links on slice t0 are not touched (the level-1 boundary). */
static void sweep_range(const geom_t *g, cplx *U, double beta, uint64_t seed, uint32_t stream,
                        int sweep_id, int n_hb, int n_or, int t0, int t1, int freeze_first_slice)
{
    long V3 = (long)g->L[1] * g->L[2] * g->L[3];
    for (int mu = 0; mu < 4; ++mu) {
        for (int par = 0; par < 2; ++par) {
#pragma omp parallel for schedule(static)
            for (long s = (long)t0 * V3; s < (long)t1 * V3; ++s) {
                int x[4];
                site_coords(g, s, x);
                if (((x[0] + x[1] + x[2] + x[3]) & 1) != par) continue;
                if (freeze_first_slice && mu != 0 && x[0] == t0) continue;
                cplx A[9];
                staple(g, U, s, mu, A);
                rng_t r;
                rng_init(&r, seed, stream, (uint32_t)s, (uint32_t)(mu | (sweep_id << 2)), 0x5EEDu);
                update_link(LINK(U, s, mu), A, beta, n_hb, n_or, &r);
            }
        }
    }
}

/* Hot start (random SU(3) links) then nsweeps of (1 heatbath + n_or OR). */
void gen_heatbath(const int L[4], double beta, uint64_t seed, int nsweeps, int n_or, int hot_start,
                  double *Uinout)
{
    geom_t g = {{L[0], L[1], L[2], L[3]}, (long)L[0] * L[1] * L[2] * L[3]};
    cplx *U = (cplx *)Uinout;
    if (hot_start) gen_random_links(L, seed ^ 0xA5A5A5A5ull, 10.0, Uinout);
    for (int sw = 0; sw < nsweeps; ++sw)
        sweep_range(&g, U, beta, seed, 2u, sw, 1, n_or, 0, L[0], 0);
}

/* Level-1 update of the slab [t0,t1): nsweeps sweeps restricted to the slab
 * with the spatial links of slice t0 frozen.  The update of one slab then
 * depends only on its own links and on frozen links. */
void gen_level1_update(const int L[4], double beta, uint64_t seed, uint32_t update_id, int t0, int t1,
                       int nsweeps, int n_or, double *Uinout)
{
    geom_t g = {{L[0], L[1], L[2], L[3]}, (long)L[0] * L[1] * L[2] * L[3]};
    for (int sw = 0; sw < nsweeps; ++sw)
        sweep_range(&g, (cplx *)Uinout, beta, seed, 3u + update_id, sw, 1, n_or, t0, t1, 1);
}

/* Replicate a field of dims Ls periodically into dims L (L multiple of Ls). */
void gen_tile(const int Ls[4], const double *Usmall, const int L[4], double *Uout)
{
    geom_t gs = {{Ls[0], Ls[1], Ls[2], Ls[3]}, (long)Ls[0] * Ls[1] * Ls[2] * Ls[3]};
    geom_t g = {{L[0], L[1], L[2], L[3]}, (long)L[0] * L[1] * L[2] * L[3]};
    const cplx *us = (const cplx *)Usmall;
    cplx *u = (cplx *)Uout;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; ++s) {
        int x[4];
        site_coords(&g, s, x);
        int y[4] = {x[0] % Ls[0], x[1] % Ls[1], x[2] % Ls[2], x[3] % Ls[3]};
        memcpy(LINK(u, s, 0), LINK(us, site_index(&gs, y), 0), 36 * sizeof(cplx));
    }
}

/* Average plaquette (1/3) Re tr U_munu over all sites and planes. */
double gen_plaquette(const int L[4], const double *Uin)
{
    geom_t g = {{L[0], L[1], L[2], L[3]}, (long)L[0] * L[1] * L[2] * L[3]};
    const cplx *U = (const cplx *)Uin;
    double sum = 0;
#pragma omp parallel for reduction(+ : sum) schedule(static)
    for (long s = 0; s < g.V; ++s) {
        int x[4];
        site_coords(&g, s, x);
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                cplx a[9], b[9], c[9];
                m3_mul(LINK(U, s, mu), LINK(U, shift(&g, x, mu, 1), nu), a);
                m3_mul_na(a, LINK(U, shift(&g, x, nu, 1), mu), b);
                m3_mul_na(b, LINK(U, s, nu), c);
                sum += creal(c[0] + c[4] + c[8]) / 3.0;
            }
    }
    return sum / (6.0 * g.V);
}

/* n complex Gaussian numbers with E|z|^2 = 1, keyed by (seed, stream). */
void gen_gaussian(uint64_t seed, uint32_t stream, long n, double *out)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        rng_t r;
        rng_init(&r, seed, stream, (uint32_t)i, (uint32_t)(i >> 32), 0x6A55u);
        out[2 * i] = rng_normal(&r) * M_SQRT1_2;
        out[2 * i + 1] = rng_normal(&r) * M_SQRT1_2;
    }
}

/* n uniforms in (0,1], keyed by (seed, stream). */
void gen_uniform(uint64_t seed, uint32_t stream, long n, double *out)
{
    for (long i = 0; i < n; ++i) {
        rng_t r;
        rng_init(&r, seed, stream, (uint32_t)i, (uint32_t)(i >> 32), 0x0u);
        out[i] = rng_uniform(&r);
    }
}
