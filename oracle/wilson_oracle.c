/*
 * Wilson-fermion oracle: a plain, slow, FP64 CPU implementation of the
 * Wilson-Dirac operator M = 1 - kappa H and of the even-odd preconditioned
 * conjugate-gradient solve of M x = b.
 *
 * TEST INFRASTRUCTURE ONLY.  Built into oracle/liboracle.so with the
 * staggered oracle and loaded by the test-suite, the smoke check and the
 * CPU-baseline timing.  The HIP library never links, loads or calls it, and
 * it shares no code, header, table or constant with the HIP path.
 *
 * Source: P. Majumdar, arXiv:1311.2719.  The paper's second workload is an
 * N_f = 2 Wilson-fermion HMC program (Sec. 2 and Sec. 6, "Performance & Discussion"); it
 * does not write the operator out, so the textbook form is taken (each point
 * a documented reading):
 *   (H psi)(x) = sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
 *                        + (1 + gamma_mu) U_mu(x - mu)^dagger psi(x - mu) ],
 *   M = 1 - kappa H (Wilson parameter r = 1), the same sites, links and
 *   boundary conditions as the staggered oracle (periodic in x, y, z; a hop
 *   across the t boundary picks up -1 when the field is antiperiodic in t);
 *   gamma matrices of a chiral basis (gamma_5 = gamma_1 gamma_2 gamma_3
 *   gamma_4 = diag(1, 1, -1, -1)), written out as 4x4 matrices below and
 *   multiplied in full (no spin projection);
 *   even-odd preconditioning: with D_eo the hops from odd to even sites,
 *   Mhat = 1 - kappa^2 D_eo D_oe on the even sites, the CG of the paper's
 *   Sec. 4 applied to Mhat^dagger Mhat x_e = Mhat^dagger bhat with
 *   bhat = b_e + kappa D_eo b_o, then x_o = b_o + kappa D_oe x_e; it stops
 *   when <r,r> < tol^2 <Mhat^dagger bhat, Mhat^dagger bhat>.
 *
 * Data layout (re, im interleaved): U [site][mu][a][b] as in the staggered
 * oracle; spinors [site][spin 4][colour 3], full lattice.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define I_ _Complex_I

/* gamma_mu[mu][row][col], mu = 0..3 = x, y, z, t */
static const cplx kGamma[4][4][4] = {
    {{0, 0, 0, I_}, {0, 0, I_, 0}, {0, -I_, 0, 0}, {-I_, 0, 0, 0}},
    {{0, 0, 0, -1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}},
    {{0, 0, I_, 0}, {0, 0, 0, -I_}, {-I_, 0, 0, 0}, {0, I_, 0, 0}},
    {{0, 0, 1, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}, {0, 1, 0, 0}},
};

static int64_t w_volume(const int32_t L[4]) { return (int64_t)L[0] * L[1] * L[2] * L[3]; }

static void w_coords(int64_t s, const int32_t L[4], int32_t c[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = (int32_t)(s % L[mu]);
        s /= L[mu];
    }
}

static int64_t w_site(const int32_t c[4], const int32_t L[4])
{
    return c[0] + (int64_t)L[0] * (c[1] + (int64_t)L[1] * (c[2] + (int64_t)L[2] * c[3]));
}

static int w_parity(const int32_t c[4]) { return (c[0] + c[1] + c[2] + c[3]) & 1; }

static int w_bad_dims(const int32_t L[4])
{
    for (int mu = 0; mu < 4; ++mu)
        if (L[mu] < 2 || (L[mu] & 1))
            return 1;
    return 0;
}

/* entries of the spin-colour vector at site s: [spin][colour] */
static const cplx *spin_r(const double *v, int64_t s) { return (const cplx *)(v + s * 24); }
static cplx *spin_w(double *v, int64_t s) { return (cplx *)(v + s * 24); }

/* (H psi)(x) at one site, added into out_site with factor f */
static void hop_site(const int32_t L[4], int32_t tap, const double *U, const double *psi, int64_t s, cplx f,
                     cplx *out_site)
{
    int32_t c[4];
    w_coords(s, L, c);
    for (int mu = 0; mu < 4; ++mu) {
        for (int dir = 0; dir < 2; ++dir) { /* 0: forward, 1: backward */
            int32_t n[4] = {c[0], c[1], c[2], c[3]};
            double bsign = 1.0;
            const double *u;
            if (dir == 0) {
                n[mu] = c[mu] + 1 == L[mu] ? 0 : c[mu] + 1;
                if (tap && mu == 3 && c[3] == L[3] - 1)
                    bsign = -1.0;
                u = U + (s * 4 + mu) * 18;
            } else {
                n[mu] = c[mu] == 0 ? L[mu] - 1 : c[mu] - 1;
                if (tap && mu == 3 && c[3] == 0)
                    bsign = -1.0;
                u = U + (w_site(n, L) * 4 + mu) * 18;
            }
            const cplx *um = (const cplx *)u;
            const cplx *q = spin_r(psi, w_site(n, L));
            /* colour: w[sp][a] = sum_b V(a,b) q[sp][b], V = U or U^dagger */
            cplx w[4][3];
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    cplx acc = 0;
                    for (int b = 0; b < 3; ++b) {
                        const cplx v = dir == 0 ? um[a * 3 + b] : conj(um[b * 3 + a]);
                        acc += v * q[sp * 3 + b];
                    }
                    w[sp][a] = bsign * acc;
                }
            /* spin: (1 -+ gamma_mu) w */
            const double sg = dir == 0 ? -1.0 : 1.0;
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    cplx acc = w[sp][a];
                    for (int t = 0; t < 4; ++t)
                        acc += sg * kGamma[mu][sp][t] * w[t][a];
                    out_site[sp * 3 + a] += f * acc;
                }
        }
    }
}

/* out = H psi on the sites of out_parity (2 = all); other sites untouched. */
int orc_wilson_hop(const int32_t L[4], int32_t tap, const double *U, const double *psi, double *out,
                   int32_t out_parity)
{
    if (w_bad_dims(L) || out_parity < 0 || out_parity > 2)
        return -1;
    const int64_t V = w_volume(L);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        int32_t c[4];
        w_coords(s, L, c);
        if (out_parity != 2 && w_parity(c) != out_parity)
            continue;
        cplx *o = spin_w(out, s);
        for (int k = 0; k < 12; ++k)
            o[k] = 0;
        hop_site(L, tap, U, psi, s, 1.0, o);
    }
    return 0;
}

/* out = M psi = psi - kappa H psi on every site. */
int orc_wilson_apply(const int32_t L[4], int32_t tap, const double *U, double kappa, const double *psi, double *out)
{
    if (w_bad_dims(L))
        return -1;
    const int64_t V = w_volume(L);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        cplx *o = spin_w(out, s);
        const cplx *p = spin_r(psi, s);
        for (int k = 0; k < 12; ++k)
            o[k] = p[k];
        hop_site(L, tap, U, psi, s, -kappa, o);
    }
    return 0;
}

/* gamma_mu as 16 complex (row-major), for tests of the basis */
int orc_wilson_gamma(int32_t mu, double *out)
{
    if (mu < 0 || mu > 3)
        return -1;
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            out[2 * (r * 4 + c)] = creal(kGamma[mu][r][c]);
            out[2 * (r * 4 + c) + 1] = cimag(kGamma[mu][r][c]);
        }
    return 0;
}

/* ---- even-odd preconditioned CG ----------------------------------------- */

/* y = v restricted to parity par (other sites set to zero) */
static void w_restrict(const int32_t L[4], int32_t par, const double *v, double *y)
{
    const int64_t V = w_volume(L);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        int32_t c[4];
        w_coords(s, L, c);
        const int on = w_parity(c) == par;
        for (int k = 0; k < 24; ++k)
            y[s * 24 + k] = on ? v[s * 24 + k] : 0.0;
    }
}

/* Mhat v on the even sites: v - kappa^2 D_eo (D_oe v); tmp is scratch */
static void w_mhat(const int32_t L[4], int32_t tap, const double *U, double kappa, const double *v, double *out,
                   double *tmp)
{
    orc_wilson_hop(L, tap, U, v, tmp, 1);
    w_restrict(L, 1, tmp, tmp);
    orc_wilson_hop(L, tap, U, tmp, out, 0);
    const int64_t V = w_volume(L);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        int32_t c[4];
        w_coords(s, L, c);
        for (int k = 0; k < 24; ++k)
            out[s * 24 + k] = w_parity(c) == 0 ? v[s * 24 + k] - kappa * kappa * out[s * 24 + k] : 0.0;
    }
}

/* gamma_5 v: spins 2, 3 change sign */
static void w_gamma5(const int32_t L[4], const double *v, double *out)
{
    const int64_t V = w_volume(L);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s)
        for (int k = 0; k < 24; ++k)
            out[s * 24 + k] = k < 12 ? v[s * 24 + k] : -v[s * 24 + k];
}

/* Mhat^dagger v = gamma_5 Mhat gamma_5 v (gamma_5-hermiticity of H) */
static void w_mhat_dag(const int32_t L[4], int32_t tap, const double *U, double kappa, const double *v,
                       double *out, double *tmp, double *tmp2)
{
    w_gamma5(L, v, tmp2);
    w_mhat(L, tap, U, kappa, tmp2, out, tmp);
    w_gamma5(L, out, out);
}

static double w_norm2(const int32_t L[4], const double *v)
{
    const int64_t n = w_volume(L) * 24;
    double acc = 0.0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
    for (int64_t i = 0; i < n; ++i)
        acc += v[i] * v[i];
    return acc;
}

typedef struct {
    int32_t status; /* 0 converged, -6 iteration limit, -7 breakdown */
    int32_t iters;
    double rr;       /* final <r,r> of the normal equations */
    double bb;       /* <Mhat^dagger bhat, Mhat^dagger bhat> */
    double true_rel; /* ||b - M x|| / ||b||, full lattice */
} orc_wilson_result;

/* Solve M x = b (full lattice) by CG on the even-odd normal equations. */
int orc_wilson_cg(const int32_t L[4], int32_t tap, const double *U, double kappa, double tol, int32_t maxiter,
                  const double *b, double *x, orc_wilson_result *res)
{
    if (w_bad_dims(L) || !(tol > 0) || maxiter < 0)
        return -1;
    const int64_t n = w_volume(L) * 24;
    double *bh = calloc(n, sizeof(double)), *rhs = calloc(n, sizeof(double)), *r = calloc(n, sizeof(double));
    double *p = calloc(n, sizeof(double)), *ap = calloc(n, sizeof(double)), *atap = calloc(n, sizeof(double));
    double *xe = calloc(n, sizeof(double)), *t1 = calloc(n, sizeof(double)), *t2 = calloc(n, sizeof(double));
    double *t3 = calloc(n, sizeof(double));
    if (!bh || !rhs || !r || !p || !ap || !atap || !xe || !t1 || !t2 || !t3)
        return -2;
    /* bhat = b_e + kappa D_eo b_o */
    w_restrict(L, 1, b, t1);
    orc_wilson_hop(L, tap, U, t1, t2, 0);
    w_restrict(L, 0, t2, t2);
    w_restrict(L, 0, b, bh);
    for (int64_t i = 0; i < n; ++i)
        bh[i] += kappa * t2[i];
    /* rhs = Mhat^dagger bhat; x_e = 0, r = p = rhs */
    w_mhat_dag(L, tap, U, kappa, bh, rhs, t1, t3);
    memcpy(r, rhs, n * sizeof(double));
    memcpy(p, rhs, n * sizeof(double));
    const double bb = w_norm2(L, rhs);
    double rr = bb;
    int it = 0, status = 0;
    if (bb > 0) {
        while (rr >= tol * tol * bb) {
            if (it >= maxiter) {
                status = -6;
                break;
            }
            w_mhat(L, tap, U, kappa, p, ap, t1);           /* ap = Mhat p */
            const double pap = w_norm2(L, ap);              /* <p, Mhat^dag Mhat p> */
            if (!(pap > 0)) {
                status = -7;
                break;
            }
            const double alpha = rr / pap;
            w_mhat_dag(L, tap, U, kappa, ap, atap, t1, t3); /* atap = Mhat^dag Mhat p */
            for (int64_t i = 0; i < n; ++i) {
                xe[i] += alpha * p[i];
                r[i] -= alpha * atap[i];
            }
            const double rn = w_norm2(L, r);
            const double beta = rn / rr;
            rr = rn;
            for (int64_t i = 0; i < n; ++i)
                p[i] = r[i] + beta * p[i];
            ++it;
        }
    }
    /* x_o = b_o + kappa D_oe x_e */
    orc_wilson_hop(L, tap, U, xe, t1, 1);
    w_restrict(L, 1, t1, t1);
    w_restrict(L, 1, b, t2);
    for (int64_t i = 0; i < n; ++i)
        x[i] = xe[i] + t2[i] + kappa * t1[i];
    /* true residual of the full system */
    orc_wilson_apply(L, tap, U, kappa, x, t1);
    for (int64_t i = 0; i < n; ++i)
        t1[i] = b[i] - t1[i];
    const double b2 = w_norm2(L, b);
    res->status = status;
    res->iters = it;
    res->rr = rr;
    res->bb = bb;
    res->true_rel = b2 > 0 ? sqrt(w_norm2(L, t1) / b2) : 0.0;
    free(bh);
    free(rhs);
    free(r);
    free(p);
    free(ap);
    free(atap);
    free(xe);
    free(t1);
    free(t2);
    free(t3);
    return 0;
}
