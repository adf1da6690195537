/*
 * FP64 CPU oracle for the domain-decomposed Wilson(-clover) propagator.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no source with the GPU path: its own gamma
 * matrices, indexing, stencil and solver.
 *
 * What it computes (plain definitions, no blocking, no even-odd split):
 *
 *  - Wilson-Dirac operator (Appendix A, eq. wdo):  D = D_w + m0 with
 *      D_w = 1/2 { gamma_mu (nabla*_mu + nabla_mu) - nabla*_mu nabla_mu },
 *    which written out per site is
 *      D psi(x) = (m0 + 4) psi(x)
 *                 - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                               + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ].
 *    m0 = 1/(2 kappa) - 4 so that 2 kappa D = 1 - kappa D_hop (Section 6).
 *  - O(a) improvement (mentioned in the footnotes of Sections 4 and 6, not
 *    defined by the paper, so parity unpinned against the paper: the tests
 *    pin it to the definition below): the Sheikholeslami-Wohlert term
 *      c_sw (i/4) sum_{mu,nu} sigma_{mu nu} Fhat_{mu nu}(x),
 *    sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu], Fhat = (Q_{mu nu} - Q_{nu mu})/8,
 *    Q_{mu nu}(x) the sum of the four plaquettes of the (mu,nu) plane at x.
 *  - Dirichlet restriction to a hyper-cubic domain Gamma (Section 2, eq.
 *    blkdec): D_Gamma = P_Gamma D P_Gamma, i.e. every hop that leaves Gamma is
 *    dropped while the site-diagonal part (mass and clover, built from the
 *    full gauge field) is kept.  S^(i) = D_Gamma_i^{-1} (eq. diric).
 *  - Fermion boundary conditions: periodic in space; in time (argument tbc)
 *    0 periodic, 1 antiperiodic (a hop across the time boundary picks up -1)
 *    or 2 open (hops across the time boundary are dropped, the site-diagonal
 *    part is kept: the fermion field vanishes beyond the first and last time
 *    slices, the set-up the paper assumes in Sections 2 and 5.2).
 *  - BiCGstab (van der Vorst 1992) on the unpreconditioned D_Gamma, with the
 *    true residual recomputed and the iteration restarted from it until
 *    ||b - D_Gamma x|| <= tol ||b|| per right-hand side.
 *
 * Layouts: site = ((t*L1+x1)*L2+x2)*L3+x3; spinor [rhs][site][spin][colour];
 * links [site][mu][3][3]; clover term [site][12][12] with index spin*3+colour.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Chiral (Weyl) basis: gamma_0 = [[0,-1],[-1,0]], gamma_k = [[0,-i s_k],[i s_k,0]]. */
static const cplx G[4][4][4] = {
    {{0, 0, -1, 0}, {0, 0, 0, -1}, {-1, 0, 0, 0}, {0, -1, 0, 0}},
    {{0, 0, 0, -I}, {0, 0, -I, 0}, {0, I, 0, 0}, {I, 0, 0, 0}},
    {{0, 0, 0, -1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}},
    {{0, 0, -I, 0}, {0, 0, 0, I}, {I, 0, 0, 0}, {0, -I, 0, 0}},
};

void oracle_gamma(int mu, double *out) /* 4x4 complex, row-major */
{
    memcpy(out, G[mu], sizeof(G[mu]));
}

typedef struct {
    int L[4];
    long V;
} lat_t;

static void lat_init(lat_t *g, const int L[4])
{
    for (int m = 0; m < 4; ++m) g->L[m] = L[m];
    g->V = (long)L[0] * L[1] * L[2] * L[3];
}
static inline void coords(const lat_t *g, long s, int x[4])
{
    x[3] = (int)(s % g->L[3]); s /= g->L[3];
    x[2] = (int)(s % g->L[2]); s /= g->L[2];
    x[1] = (int)(s % g->L[1]); s /= g->L[1];
    x[0] = (int)s;
}
static inline long index_of(const lat_t *g, const int x[4])
{
    return ((long)(x[0] * g->L[1] + x[1]) * g->L[2] + x[2]) * g->L[3] + x[3];
}
static inline int inside(const int x[4], const int lo[4], const int hi[4])
{
    for (int m = 0; m < 4; ++m)
        if (x[m] < lo[m] || x[m] >= hi[m]) return 0;
    return 1;
}

static inline const cplx *link(const cplx *U, long s, int mu) { return U + (s * 4 + mu) * 9; }

static void mm(const cplx *a, const cplx *b, cplx *c)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx t = 0;
            for (int k = 0; k < 3; ++k) t += a[3 * i + k] * b[3 * k + j];
            c[3 * i + j] = t;
        }
}
static void dag(const cplx *a, cplx *c)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) c[3 * i + j] = conj(a[3 * j + i]);
}
static void mm4(const cplx *a, const cplx *b, const cplx *c, const cplx *d, cplx *out)
{
    cplx t1[9], t2[9];
    mm(a, b, t1);
    mm(t1, c, t2);
    mm(t2, d, out);
}

/* Q_{mu nu}(x): the four plaquettes of the (mu,nu) plane that start and end at x. */
static void clover_leaves(const lat_t *g, const cplx *U, long s, int mu, int nu, cplx *Q)
{
    int x[4];
    coords(g, s, x);
    /* neighbour index x + a*mu + b*nu (periodic gauge field) */
    long n[3][3];
    for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b) {
            int t[4] = {x[0], x[1], x[2], x[3]};
            t[mu] = (t[mu] + a + g->L[mu]) % g->L[mu];
            t[nu] = (t[nu] + b + g->L[nu]) % g->L[nu];
            n[a + 1][b + 1] = index_of(g, t);
        }
#define AT(a, b) n[(a) + 1][(b) + 1]
    cplx d1[9], d2[9], P[9];
    memset(Q, 0, 9 * sizeof(cplx));
    /* leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag */
    dag(link(U, AT(0, 1), mu), d1);
    dag(link(U, s, nu), d2);
    mm4(link(U, s, mu), link(U, AT(1, 0), nu), d1, d2, P);
    for (int k = 0; k < 9; ++k) Q[k] += P[k];
    /* leaf 2: U_nu(x) U_mu(x-mu+nu)^dag U_nu(x-mu)^dag U_mu(x-mu) */
    dag(link(U, AT(-1, 1), mu), d1);
    dag(link(U, AT(-1, 0), nu), d2);
    mm4(link(U, s, nu), d1, d2, link(U, AT(-1, 0), mu), P);
    for (int k = 0; k < 9; ++k) Q[k] += P[k];
    /* leaf 3: U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu) */
    dag(link(U, AT(-1, 0), mu), d1);
    dag(link(U, AT(-1, -1), nu), d2);
    mm4(d1, d2, link(U, AT(-1, -1), mu), link(U, AT(0, -1), nu), P);
    for (int k = 0; k < 9; ++k) Q[k] += P[k];
    /* leaf 4: U_nu(x-nu)^dag U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^dag */
    dag(link(U, AT(0, -1), nu), d1);
    dag(link(U, s, mu), d2);
    mm4(d1, link(U, AT(0, -1), mu), link(U, AT(1, -1), nu), d2, P);
    for (int k = 0; k < 9; ++k) Q[k] += P[k];
#undef AT
}

/* Field strength Fhat_{mu nu}(x) = (Q_{mu nu} - Q_{nu mu}) / 8 with Q_{nu mu} = Q_{mu nu}^dag. */
void oracle_field_strength(const int L[4], const double *Ud, int mu, int nu, double *Fout)
{
    lat_t g;
    lat_init(&g, L);
    const cplx *U = (const cplx *)Ud;
    cplx *F = (cplx *)Fout;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; ++s) {
        cplx Q[9];
        clover_leaves(&g, U, s, mu, nu, Q);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) F[s * 9 + 3 * i + j] = (Q[3 * i + j] - conj(Q[3 * j + i])) / 8.0;
    }
}

/* sigma_{mu nu} = (i/2)(gamma_mu gamma_nu - gamma_nu gamma_mu) */
static void sigma_table(cplx sig[4][4][4][4])
{
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu)
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    cplx t = 0;
                    for (int c = 0; c < 4; ++c) t += G[mu][a][c] * G[nu][c][b] - G[nu][a][c] * G[mu][c][b];
                    sig[mu][nu][a][b] = 0.5 * I * t;
                }
}

/* 12x12 clover term of site s: c_sw (i/4) sum_{mu,nu} sigma_{mu nu} (x) Fhat_{mu nu}. */
static void clover_site(const lat_t *g, const cplx *U, double csw, cplx sig[4][4][4][4], long s, cplx *Cs)
{
    memset(Cs, 0, 144 * sizeof(cplx));
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu) {
            if (mu == nu) continue;
            cplx Q[9], F[9];
            clover_leaves(g, U, s, mu, nu, Q);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) F[3 * i + j] = (Q[3 * i + j] - conj(Q[3 * j + i])) / 8.0;
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    cplx w = csw * 0.25 * I * sig[mu][nu][a][b];
                    if (w == 0) continue;
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) Cs[(a * 3 + i) * 12 + b * 3 + j] += w * F[3 * i + j];
                }
        }
}

/* The clover term of every site, [V][12][12]. */
void oracle_clover_term(const int L[4], const double *Ud, double csw, double *Cout)
{
    lat_t g;
    lat_init(&g, L);
    const cplx *U = (const cplx *)Ud;
    cplx *C = (cplx *)Cout;
    cplx sig[4][4][4][4];
    sigma_table(sig);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < g.V; ++s) clover_site(&g, U, csw, sig, s, C + s * 144);
}

/* The hopping term H psi(x) = sum_mu [(1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^dag psi(x-mu)],
 * restricted to the domain [lo,hi) (hops leaving it are dropped), with sign -1
 * on hops across the time boundary when antiperiodic (tbc 1) and no such hops
 * when open (tbc 2). Output zero outside the domain. */
static void hop_site(const lat_t *g, const cplx *U, int tbc, const int lo[4], const int hi[4],
                     const cplx *in, long s, cplx *out /* [12] */)
{
    int x[4];
    coords(g, s, x);
    memset(out, 0, 12 * sizeof(cplx));
    for (int mu = 0; mu < 4; ++mu) {
        for (int dir = 0; dir < 2; ++dir) {
            int y[4] = {x[0], x[1], x[2], x[3]};
            int d = dir == 0 ? 1 : -1;
            y[mu] = x[mu] + d;
            double sign = 1.0;
            if (y[mu] < 0 || y[mu] >= g->L[mu]) {
                y[mu] = (y[mu] + g->L[mu]) % g->L[mu];
                if (mu == 0 && tbc == 2) continue; /* open: no hop across the time boundary */
                if (mu == 0 && tbc == 1) sign = -1.0;
            }
            if (!inside(y, lo, hi)) continue;
            long sy = index_of(g, y);
            const cplx *psi = in + sy * 12;
            cplx Upsi[12]; /* colour rotation of each spin component */
            if (dir == 0) {
                const cplx *u = link(U, s, mu);
                for (int a = 0; a < 4; ++a)
                    for (int i = 0; i < 3; ++i)
                        Upsi[a * 3 + i] = u[3 * i] * psi[a * 3] + u[3 * i + 1] * psi[a * 3 + 1] +
                                          u[3 * i + 2] * psi[a * 3 + 2];
            } else {
                const cplx *u = link(U, sy, mu);
                for (int a = 0; a < 4; ++a)
                    for (int i = 0; i < 3; ++i)
                        Upsi[a * 3 + i] = conj(u[i]) * psi[a * 3] + conj(u[3 + i]) * psi[a * 3 + 1] +
                                          conj(u[6 + i]) * psi[a * 3 + 2];
            }
            /* spin projector (1 - d*gamma_mu) */
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 3; ++i) {
                    cplx t = Upsi[a * 3 + i];
                    for (int b = 0; b < 4; ++b) t -= d * G[mu][a][b] * Upsi[b * 3 + i];
                    out[a * 3 + i] += sign * t;
                }
        }
    }
}

/* out = D_Gamma in for nrhs vectors of length V*12 (clover may be NULL). */
void oracle_apply_D(const int L[4], const double *Ud, const double *Cd, double kappa, int tbc,
                    const int lo[4], const int hi[4], int nrhs, const double *ind, double *outd)
{
    lat_t g;
    lat_init(&g, L);
    const cplx *U = (const cplx *)Ud, *C = (const cplx *)Cd, *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    double diag = 1.0 / (2.0 * kappa); /* m0 + 4 */
    for (int r = 0; r < nrhs; ++r) {
        const cplx *ir = in + (long)r * g.V * 12;
        cplx *orr = out + (long)r * g.V * 12;
#pragma omp parallel for schedule(static)
        for (long s = 0; s < g.V; ++s) {
            int x[4];
            coords(&g, s, x);
            cplx *o = orr + s * 12;
            if (!inside(x, lo, hi)) {
                memset(o, 0, 12 * sizeof(cplx));
                continue;
            }
            cplx h[12];
            hop_site(&g, U, tbc, lo, hi, ir, s, h);
            const cplx *p = ir + s * 12;
            for (int k = 0; k < 12; ++k) {
                cplx t = diag * p[k] - 0.5 * h[k];
                if (C)
                    for (int j = 0; j < 12; ++j) t += C[s * 144 + k * 12 + j] * p[j];
                o[k] = t;
            }
        }
    }
}

/* (D_Gamma in)(x) at the listed sites only, for checks of large fields one
 * site at a time: out[r][k][12] = (D_Gamma in_r)(sites[k]).  The clover term
 * (csw != 0) of each listed site is built there, as oracle_clover_term builds
 * it; the rest is oracle_apply_D's arithmetic for that site. */
void oracle_apply_D_sites(const int L[4], const double *Ud, double csw, double kappa, int tbc,
                          const int lo[4], const int hi[4], int nrhs, long nsites, const long *sites,
                          const double *ind, double *outd)
{
    lat_t g;
    lat_init(&g, L);
    const cplx *U = (const cplx *)Ud, *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    double diag = 1.0 / (2.0 * kappa);
    cplx sig[4][4][4][4];
    sigma_table(sig);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nsites; ++k) {
        long s = sites[k];
        int x[4];
        coords(&g, s, x);
        cplx Cs[144];
        if (csw != 0) clover_site(&g, U, csw, sig, s, Cs);
        for (int r = 0; r < nrhs; ++r) {
            const cplx *ir = in + (long)r * g.V * 12;
            cplx *o = out + ((long)r * nsites + k) * 12;
            if (!inside(x, lo, hi)) {
                memset(o, 0, 12 * sizeof(cplx));
                continue;
            }
            cplx h[12];
            hop_site(&g, U, tbc, lo, hi, ir, s, h);
            const cplx *p = ir + s * 12;
            for (int a = 0; a < 12; ++a) {
                cplx t = diag * p[a] - 0.5 * h[a];
                if (csw != 0)
                    for (int j = 0; j < 12; ++j) t += Cs[a * 12 + j] * p[j];
                o[a] = t;
            }
        }
    }
}

/* out = D_hop in (domain-restricted hopping term, no diagonal). */
void oracle_apply_hop(const int L[4], const double *Ud, int tbc, const int lo[4], const int hi[4],
                      int nrhs, const double *ind, double *outd)
{
    lat_t g;
    lat_init(&g, L);
    const cplx *U = (const cplx *)Ud, *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    for (int r = 0; r < nrhs; ++r) {
        const cplx *ir = in + (long)r * g.V * 12;
        cplx *orr = out + (long)r * g.V * 12;
#pragma omp parallel for schedule(static)
        for (long s = 0; s < g.V; ++s) {
            int x[4];
            coords(&g, s, x);
            if (!inside(x, lo, hi)) {
                memset(orr + s * 12, 0, 12 * sizeof(cplx));
                continue;
            }
            hop_site(&g, U, tbc, lo, hi, ir, s, orr + s * 12);
        }
    }
}

/* ------------------------------------------------------------- BiCGstab */
static cplx dotc(long n, const cplx *a, const cplx *b) /* sum conj(a) b */
{
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (long i = 0; i < n; ++i) {
        cplx t = conj(a[i]) * b[i];
        re += creal(t);
        im += cimag(t);
    }
    return re + I * im;
}
static double norm2(long n, const cplx *a) { return creal(dotc(n, a, a)); }

/* Solve D_Gamma x = b for each rhs (x zero outside Gamma).  info[r] receives
 * the iteration count and res[r] the final true relative residual.
 * Returns 0 if every rhs reached tol. */
int oracle_solve(const int L[4], const double *Ud, const double *Cd, double kappa, int tbc,
                 const int lo[4], const int hi[4], int nrhs, const double *bd, double *xd, double tol,
                 int maxiter, int *iters, double *res)
{
    lat_t g;
    lat_init(&g, L);
    long n = g.V * 12;
    int status = 0;
    cplx *r = malloc(n * sizeof(cplx)), *rh = malloc(n * sizeof(cplx)), *p = malloc(n * sizeof(cplx));
    cplx *v = malloc(n * sizeof(cplx)), *s = malloc(n * sizeof(cplx)), *t = malloc(n * sizeof(cplx));
    cplx *bm = malloc(n * sizeof(cplx));
    for (int k = 0; k < nrhs; ++k) {
        const cplx *b = (const cplx *)bd + (long)k * n;
        cplx *x = (cplx *)xd + (long)k * n;
        /* restrict the source to the domain: D_Gamma acts on fields on Gamma */
#pragma omp parallel for schedule(static)
        for (long q = 0; q < g.V; ++q) {
            int xc[4];
            coords(&g, q, xc);
            int in = inside(xc, lo, hi);
            for (int c = 0; c < 12; ++c) {
                bm[q * 12 + c] = in ? b[q * 12 + c] : 0;
                x[q * 12 + c] = 0;
            }
        }
        double bn = sqrt(norm2(n, bm));
        int it = 0;
        double rel = 0;
        if (bn == 0) {
            iters[k] = 0;
            res[k] = 0;
            continue;
        }
        for (int cycle = 0; cycle < 50; ++cycle) {
            /* true residual */
            oracle_apply_D(L, Ud, Cd, kappa, tbc, lo, hi, 1, (const double *)x, (double *)r);
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) r[i] = bm[i] - r[i];
            rel = sqrt(norm2(n, r)) / bn;
            if (rel <= tol || it >= maxiter) break;
            memcpy(rh, r, n * sizeof(cplx));
            memset(p, 0, n * sizeof(cplx));
            memset(v, 0, n * sizeof(cplx));
            cplx rho = 1, alpha = 1, omega = 1;
            while (it < maxiter) {
                cplx rho_new = dotc(n, rh, r);
                if (cabs(rho_new) == 0) break;
                cplx beta = (rho_new / rho) * (alpha / omega);
                rho = rho_new;
#pragma omp parallel for schedule(static)
                for (long i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
                oracle_apply_D(L, Ud, Cd, kappa, tbc, lo, hi, 1, (const double *)p, (double *)v);
                cplx rv = dotc(n, rh, v);
                if (cabs(rv) == 0) break;
                alpha = rho / rv;
#pragma omp parallel for schedule(static)
                for (long i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
                oracle_apply_D(L, Ud, Cd, kappa, tbc, lo, hi, 1, (const double *)s, (double *)t);
                double tt = norm2(n, t);
                omega = tt > 0 ? dotc(n, t, s) / tt : 0;
#pragma omp parallel for schedule(static)
                for (long i = 0; i < n; ++i) {
                    x[i] += alpha * p[i] + omega * s[i];
                    r[i] = s[i] - omega * t[i];
                }
                ++it;
                /* leave the recursion early and restart from the true residual */
                if (sqrt(norm2(n, r)) <= 0.1 * tol * bn || omega == 0) break;
            }
        }
        iters[k] = it;
        res[k] = rel;
        if (!(rel <= tol)) status = 1;
    }
    free(r); free(rh); free(p); free(v); free(s); free(t); free(bm);
    return status;
}

/* ---------------------------------------------------- level-1 gauge updates
 * Quenched updates of the links of a time slab [t0,t1) with the spatial links
 * of slice t0 kept fixed (the level-1 updates of the two-level integration,
 * Section 3.1): Wilson plaquette action S = beta sum_P (1 - Re tr U_P / 3);
 * each link is updated by Cabibbo-Marinari heatbath over the SU(2) subgroups
 * (0,1), (0,2), (1,2) with the Kennedy-Pendleton sampler, then n_or SU(2)
 * over-relaxation passes, then projected back onto SU(3).  Links of one
 * direction and one site parity do not enter each other's staples, so a
 * sweep is: for mu, for parity, every such link (in any order).
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key
 * (seed low word, seed high word ^ stream * 0x85EBCA6B), counter (site,
 * mu | sweep << 2, 0x5EED, n) with n counting the blocks of four 32-bit words
 * of that link; a uniform in (0,1] is (w + 1) / 2^32. */
#include <stdint.h>

static const double kPi = 3.14159265358979323846;

void oracle_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]}, k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * x[0], p1 = (uint64_t)0xCD9E8D57u * x[2];
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x[1] ^ k0, y1 = (uint32_t)p1;
        const uint32_t y2 = (uint32_t)(p0 >> 32) ^ x[3] ^ k1, y3 = (uint32_t)p0;
        x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    memcpy(out, x, sizeof x);
}

typedef struct { uint32_t key[2], ctr[4], w[4]; int left; } draws_t;

static void draws_init(draws_t *d, uint64_t seed, uint32_t stream, uint32_t c0, uint32_t c1)
{
    d->key[0] = (uint32_t)seed;
    d->key[1] = (uint32_t)(seed >> 32) ^ (stream * 0x85EBCA6Bu);
    d->ctr[0] = c0; d->ctr[1] = c1; d->ctr[2] = 0x5EEDu; d->ctr[3] = 0;
    d->left = 0;
}
static double draw(draws_t *d) /* uniform in (0,1] */
{
    if (d->left == 0) {
        oracle_philox(d->ctr, d->key, d->w);
        d->ctr[3] += 1;
        d->left = 4;
    }
    const uint32_t w = d->w[4 - d->left];
    d->left -= 1;
    return ((double)w + 1.0) / 4294967296.0;
}

static void mat3(const cplx *a, int da, const cplx *b, int db, cplx *c) /* c = a b with optional adjoints */
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k)
                s += (da ? conj(a[3 * k + i]) : a[3 * i + k]) * (db ? conj(b[3 * j + k]) : b[3 * k + j]);
            c[3 * i + j] = s;
        }
}

/* A = sum_{nu != mu} of the upper and lower staples of U_mu(x), so that the
 * part of the action that depends on U_mu(x) is -(beta/3) Re tr(U_mu(x) A). */
static void staple_sum(const lat_t *g, const cplx *U, long s, int mu, cplx *A)
{
    int x[4];
    coords(g, s, x);
    memset(A, 0, 9 * sizeof(cplx));
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        int y[4];
        cplx t[9], w[9];
        /* U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag */
        memcpy(y, x, sizeof y); y[mu] = (y[mu] + 1) % g->L[mu];
        const cplx *a = link(U, index_of(g, y), nu);
        memcpy(y, x, sizeof y); y[nu] = (y[nu] + 1) % g->L[nu];
        mat3(a, 0, link(U, index_of(g, y), mu), 1, t);
        mat3(t, 0, link(U, s, nu), 1, w);
        for (int k = 0; k < 9; ++k) A[k] += w[k];
        /* U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu) */
        memcpy(y, x, sizeof y); y[nu] = (y[nu] - 1 + g->L[nu]) % g->L[nu];
        const long xmn = index_of(g, y);
        y[mu] = (y[mu] + 1) % g->L[mu];
        mat3(link(U, index_of(g, y), nu), 1, link(U, xmn, mu), 1, t);
        mat3(t, 0, link(U, xmn, nu), 0, w);
        for (int k = 0; k < 9; ++k) A[k] += w[k];
    }
}

/* quaternion q = (q0, q1, q2, q3) <-> q0 + i (q1 s1 + q2 s2 + q3 s3) */
static void quat_of_block(const cplx *W, int i, int j, double q[4])
{
    q[0] = 0.5 * (creal(W[3 * i + i]) + creal(W[3 * j + j]));
    q[1] = 0.5 * (cimag(W[3 * i + j]) + cimag(W[3 * j + i]));
    q[2] = 0.5 * (creal(W[3 * i + j]) - creal(W[3 * j + i]));
    q[3] = 0.5 * (cimag(W[3 * i + i]) - cimag(W[3 * j + j]));
}
static void quat_times(const double a[4], const double b[4], double c[4])
{
    c[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    c[1] = a[0] * b[1] + b[0] * a[1] - (a[2] * b[3] - a[3] * b[2]);
    c[2] = a[0] * b[2] + b[0] * a[2] - (a[3] * b[1] - a[1] * b[3]);
    c[3] = a[0] * b[3] + b[0] * a[3] - (a[1] * b[2] - a[2] * b[1]);
}
/* rows i, j of U <- the 2x2 matrix of quaternion r times those rows */
static void rows_times_quat(const double r[4], int i, int j, cplx *U)
{
    const cplx m00 = r[0] + I * r[3], m01 = r[2] + I * r[1], m10 = -r[2] + I * r[1], m11 = r[0] - I * r[3];
    for (int c = 0; c < 3; ++c) {
        const cplx ui = U[3 * i + c], uj = U[3 * j + c];
        U[3 * i + c] = m00 * ui + m01 * uj;
        U[3 * j + c] = m10 * ui + m11 * uj;
    }
}

/* Kennedy-Pendleton: x0 in [-1,1] with density ~ sqrt(1 - x0^2) exp(alpha x0). */
static double kp_x0(double alpha, draws_t *d)
{
    for (int tries = 0; tries <= 10000; ++tries) {
        const double r1 = draw(d), r2 = draw(d), r3 = draw(d), r4 = draw(d);
        const double c = cos(2.0 * kPi * r2);
        const double lam2 = -(log(r1) + c * c * log(r3)) / (2.0 * alpha);
        if (r4 * r4 <= 1.0 - lam2) return 1.0 - 2.0 * lam2;
    }
    return 1.0;
}

void oracle_kp_sample(double alpha, uint64_t seed, long n, double *out)
{
    for (long k = 0; k < n; ++k) {
        draws_t d;
        draws_init(&d, seed, 1u, (uint32_t)k, 0u);
        out[k] = kp_x0(alpha, &d);
    }
}

/* Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1). */
static void to_su3(cplx *u)
{
    double n = 0;
    for (int j = 0; j < 3; ++j) n += creal(u[j] * conj(u[j]));
    n = 1.0 / sqrt(n);
    for (int j = 0; j < 3; ++j) u[j] *= n;
    cplx p = 0;
    for (int j = 0; j < 3; ++j) p += conj(u[j]) * u[3 + j];
    for (int j = 0; j < 3; ++j) u[3 + j] -= p * u[j];
    n = 0;
    for (int j = 0; j < 3; ++j) n += creal(u[3 + j] * conj(u[3 + j]));
    n = 1.0 / sqrt(n);
    for (int j = 0; j < 3; ++j) u[3 + j] *= n;
    u[6] = conj(u[1] * u[5] - u[2] * u[4]);
    u[7] = conj(u[2] * u[3] - u[0] * u[5]);
    u[8] = conj(u[0] * u[4] - u[1] * u[3]);
}

static void update_one_link(cplx *Ul, const cplx *A, double beta, int n_or, draws_t *d)
{
    static const int sub[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int pass = 0; pass < 1 + n_or; ++pass)
        for (int k = 0; k < 3; ++k) {
            cplx W[9];
            mat3(Ul, 0, A, 0, W);
            double q[4];
            quat_of_block(W, sub[k][0], sub[k][1], q);
            const double norm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
            if (norm < 1e-14) continue;
            const double vdag[4] = {q[0] / norm, -q[1] / norm, -q[2] / norm, -q[3] / norm};
            double R[4];
            if (pass == 0) {
                /* SU(2) weight exp((beta/3) Re tr_2(R W)) = exp(alpha x0), alpha = 2 beta |q| / 3 */
                const double x0 = kp_x0(2.0 * beta * norm / 3.0, d);
                const double rad = sqrt(fmax(0.0, 1.0 - x0 * x0));
                const double ct = 2.0 * draw(d) - 1.0, ph = 2.0 * kPi * draw(d);
                const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
                const double X[4] = {x0, rad * st * cos(ph), rad * st * sin(ph), rad * ct};
                quat_times(X, vdag, R);
            } else {
                quat_times(vdag, vdag, R); /* over-relaxation: Re tr(R W) unchanged */
            }
            rows_times_quat(R, sub[k][0], sub[k][1], Ul);
        }
    to_su3(Ul);
}

void oracle_level1_update(const int L[4], double beta, uint64_t seed, uint32_t stream, int t0, int t1,
                          int nsweeps, int n_or, double *Ud)
{
    lat_t g;
    lat_init(&g, L);
    cplx *U = (cplx *)Ud;
    const long V3 = (long)L[1] * L[2] * L[3];
    for (int sweep = 0; sweep < nsweeps; ++sweep)
        for (int mu = 0; mu < 4; ++mu)
            for (int par = 0; par < 2; ++par) {
#pragma omp parallel for schedule(static)
                for (long s = (long)t0 * V3; s < (long)t1 * V3; ++s) {
                    int x[4];
                    coords(&g, s, x);
                    if (((x[0] + x[1] + x[2] + x[3]) & 1) != par) continue;
                    if (mu != 0 && x[0] == t0) continue; /* frozen spatial links of the first slice */
                    cplx A[9];
                    staple_sum(&g, U, s, mu, A);
                    draws_t d;
                    draws_init(&d, seed, stream, (uint32_t)s, (uint32_t)(mu | (sweep << 2)));
                    update_one_link((cplx *)link(U, s, mu), A, beta, n_or, &d);
                }
            }
}

/* Average plaquette (1/3) Re tr U_P over all sites and the six planes. */
double oracle_plaquette(const int L[4], const double *Ud)
{
    lat_t g;
    lat_init(&g, L);
    const cplx *U = (const cplx *)Ud;
    double sum = 0;
#pragma omp parallel for reduction(+ : sum) schedule(static)
    for (long s = 0; s < g.V; ++s) {
        int x[4];
        coords(&g, s, x);
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                int y[4];
                cplx t[9], w[9];
                memcpy(y, x, sizeof y); y[mu] = (y[mu] + 1) % g.L[mu];
                mat3(link(U, s, mu), 0, link(U, index_of(&g, y), nu), 0, t);
                memcpy(y, x, sizeof y); y[nu] = (y[nu] + 1) % g.L[nu];
                mat3(t, 0, link(U, index_of(&g, y), mu), 1, w);
                mat3(w, 0, link(U, s, nu), 1, t);
                sum += creal(t[0] + t[4] + t[8]) / 3.0;
            }
    }
    return sum / (6.0 * g.V);
}
