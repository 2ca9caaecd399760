/*
 * Staggered-fermion oracle: a plain, slow, FP64 CPU implementation of the
 * staggered hopping operator D and of the conjugate-gradient solve of
 * (m^2 - D^2) x = b.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is built into oracle/liboracle.so and
 * loaded by the test-suite, the smoke check and the CPU-baseline timing.  The
 * HIP library never links, loads or calls it, and it shares no code, header,
 * table or constant with the HIP path.
 *
 * Source: P. Majumdar, "Lattice Simulations using OpenACC compilers",
 * LATTICE 2013 (arXiv:1311.2719).
 *   Sec. 3 ("Matrix-vector multiplication routine"): the fermion matrix acts
 *     site by site, combining forward and backward neighbours with the links
 *     u and the daggered links ud; the routine may act on a range of sites
 *     and accumulates into its output.
 *   Sec. 4 ("Single GPU conjugate gradient routine"): CG on the normal
 *     operator over one half (one parity) of the lattice, x = 0 at the start,
 *     denominator <ap,ap> + <p,p>, the second half reconstructed as y = K x.
 * The paper elides the operator's body.  The readings taken here (each is a
 * documented choice, not a quotation):
 *   - sites lexicographic, s = x + Lx*(y + Ly*(z + Lz*t)); mu = 0..3 = x,y,z,t;
 *   - eta_mu(x) = (-1)^(x_0 + ... + x_{mu-1});
 *   - periodic in x, y, z; a hop across the t boundary picks up -1 when the
 *     field is antiperiodic in t;
 *   - (D chi)(x) = 1/2 sum_mu eta_mu(x) [ U_mu(x) chi(x+mu)
 *                                        - U_mu(x-mu)^dagger chi(x-mu) ];
 *   - the mass is explicit: the solve is (m^2 - D^2) x = b, so the paper's
 *     <ap,ap> + <p,p> becomes <ap,ap> + m^2 <p,p> and atap = p + K^dagger ap
 *     becomes m^2 p - D ap (K = D/m in the paper's scaled form);
 *   - stop when <r,r> < tol^2 <b,b> on the parity system being solved.
 *
 * Data layout (all arrays interleave re, im as two doubles):
 *   U   [site][mu][a][b]  3x3 complex, row-major (a = row);
 *   vec [site][colour]    3 complex per site, full lattice.
 * A "parity system" vector is a full-lattice vector of which only the sites of
 * one parity are read or written.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

typedef struct {
    int32_t status;     /* 0 converged, 1 iteration limit reached */
    int32_t iters;      /* CG iterations (summed over restarts) */
    int32_t restarts;   /* restarts taken after a failed true-residual check */
    int32_t pad;
    double rr;          /* last iterated <r,r> */
    double bb;          /* <b,b> of the system */
    double true_rel;    /* ||b - A x|| / ||b|| in FP64 at exit */
} orc_cg_result;

/* ------------------------------------------------------------------ */
/* Lattice geometry                                                    */
/* ------------------------------------------------------------------ */

static int64_t volume(const int32_t L[4])
{
    return (int64_t)L[0] * L[1] * L[2] * L[3];
}

static void coords_of(int64_t s, const int32_t L[4], int32_t c[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        c[mu] = (int32_t)(s % L[mu]);
        s /= L[mu];
    }
}

static int64_t site_of(const int32_t c[4], const int32_t L[4])
{
    return c[0] + (int64_t)L[0] * (c[1] + (int64_t)L[1] * (c[2] + (int64_t)L[2] * c[3]));
}

static int parity_of(const int32_t c[4])
{
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* eta_mu(x) = (-1)^(sum of the coordinates before mu) */
static double eta(int mu, const int32_t c[4])
{
    int sum = 0;
    for (int nu = 0; nu < mu; ++nu)
        sum += c[nu];
    return (sum & 1) ? -1.0 : 1.0;
}

static const cplx *link(const double *U, int64_t s, int mu)
{
    return (const cplx *)(U + ((s * 4 + mu) * 9) * 2);
}

static const cplx *cvec(const double *v, int64_t s)
{
    return (const cplx *)(v + s * 6);
}

static cplx *cvec_w(double *v, int64_t s)
{
    return (cplx *)(v + s * 6);
}

/* ------------------------------------------------------------------ */
/* The operator                                                        */
/* ------------------------------------------------------------------ */

/* (D in)(x) at one site, written out from the definition. */
static void dslash_site(const int32_t L[4], int32_t tap, const double *U,
                        const double *in, int64_t s, cplx out[3])
{
    int32_t c[4];
    coords_of(s, L, c);
    cplx acc[3] = {0, 0, 0};
    for (int mu = 0; mu < 4; ++mu) {
        const double e = eta(mu, c);

        /* forward hop: + eta U_mu(x) chi(x + mu) */
        int32_t cf[4] = {c[0], c[1], c[2], c[3]};
        cf[mu] = (c[mu] + 1) % L[mu];
        double sf = (tap && mu == 3 && c[3] == L[3] - 1) ? -1.0 : 1.0;
        const cplx *Uf = link(U, s, mu);
        const cplx *chf = cvec(in, site_of(cf, L));
        for (int a = 0; a < 3; ++a) {
            cplx t = 0;
            for (int b = 0; b < 3; ++b)
                t += Uf[a * 3 + b] * chf[b];
            acc[a] += e * sf * t;
        }

        /* backward hop: - eta U_mu(x - mu)^dagger chi(x - mu) */
        int32_t cb[4] = {c[0], c[1], c[2], c[3]};
        cb[mu] = (c[mu] + L[mu] - 1) % L[mu];
        double sb = (tap && mu == 3 && c[3] == 0) ? -1.0 : 1.0;
        int64_t sbk = site_of(cb, L);
        const cplx *Ub = link(U, sbk, mu);
        const cplx *chb = cvec(in, sbk);
        for (int a = 0; a < 3; ++a) {
            cplx t = 0;
            for (int b = 0; b < 3; ++b)
                t += conj(Ub[b * 3 + a]) * chb[b];
            acc[a] -= e * sb * t;
        }
    }
    for (int a = 0; a < 3; ++a)
        out[a] = 0.5 * acc[a];
}

static int bad_dims(const int32_t L[4])
{
    for (int mu = 0; mu < 4; ++mu)
        if (L[mu] < 2 || (L[mu] & 1))
            return 1;
    return 0;
}

/*
 * out(x) = (D in)(x) for every site x of parity out_parity (0 even, 1 odd,
 * 2 = all sites).  Sites of the other parity are left untouched.
 * Returns 0, or -1 for bad arguments.
 */
int orc_dslash(const int32_t L[4], int32_t tap, const double *U,
               const double *in, double *out, int32_t out_parity)
{
    if (bad_dims(L) || out_parity < 0 || out_parity > 2)
        return -1;
    const int64_t V = volume(L);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        int32_t c[4];
        coords_of(s, L, c);
        if (out_parity != 2 && parity_of(c) != out_parity)
            continue;
        cplx r[3];
        dslash_site(L, tap, U, in, s, r);
        cplx *o = cvec_w(out, s);
        o[0] = r[0];
        o[1] = r[1];
        o[2] = r[2];
    }
    return 0;
}

/* (D in) at the listed sites only: out[i] holds the 3 colours of sites[i]. */
int orc_dslash_sites(const int32_t L[4], int32_t tap, const double *U,
                     const double *in, const int64_t *sites, int64_t n,
                     double *out)
{
    if (bad_dims(L))
        return -1;
    const int64_t V = volume(L);
    for (int64_t i = 0; i < n; ++i)
        if (sites[i] < 0 || sites[i] >= V)
            return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        cplx r[3];
        dslash_site(L, tap, U, in, sites[i], r);
        cplx *o = (cplx *)(out + i * 6);
        o[0] = r[0];
        o[1] = r[1];
        o[2] = r[2];
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Vector helpers restricted to a parity (2 = all sites)                */
/* ------------------------------------------------------------------ */

static int on_parity(int64_t s, const int32_t L[4], int32_t par)
{
    if (par == 2)
        return 1;
    int32_t c[4];
    coords_of(s, L, c);
    return parity_of(c) == par;
}

/* <u, v> = sum over sites of the parity and colours of conj(u) v */
static cplx dot(const int32_t L[4], int32_t par, const double *u, const double *v)
{
    const int64_t V = volume(L);
    double re = 0, im = 0;
#pragma omp parallel for schedule(static) reduction(+ : re, im)
    for (int64_t s = 0; s < V; ++s) {
        if (!on_parity(s, L, par))
            continue;
        const cplx *a = cvec(u, s), *b = cvec(v, s);
        for (int k = 0; k < 3; ++k) {
            cplx t = conj(a[k]) * b[k];
            re += creal(t);
            im += cimag(t);
        }
    }
    return re + I * im;
}

static double norm2(const int32_t L[4], int32_t par, const double *u)
{
    return creal(dot(L, par, u, u));
}

/* y = a*x + b*y on the parity */
static void axpby(const int32_t L[4], int32_t par, double a, const double *x,
                  double b, double *y)
{
    const int64_t V = volume(L);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        if (!on_parity(s, L, par))
            continue;
        for (int k = 0; k < 6; ++k)
            y[s * 6 + k] = a * x[s * 6 + k] + b * y[s * 6 + k];
    }
}

static void set_zero(const int32_t L[4], int32_t par, double *y)
{
    const int64_t V = volume(L);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s)
        if (on_parity(s, L, par))
            for (int k = 0; k < 6; ++k)
                y[s * 6 + k] = 0.0;
}

static void copy_par(const int32_t L[4], int32_t par, const double *x, double *y)
{
    const int64_t V = volume(L);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s)
        if (on_parity(s, L, par))
            for (int k = 0; k < 6; ++k)
                y[s * 6 + k] = x[s * 6 + k];
}

/* ------------------------------------------------------------------ */
/* The normal operator A = m^2 - D^2                                   */
/* ------------------------------------------------------------------ */

/*
 * out = (m^2 - D^2) in on the sites of parity par (2 = all).  D^2 maps a
 * parity onto itself, so only the sites of par in `in` are read.  tmp is a
 * full-lattice work vector.
 */
static void apply_normal(const int32_t L[4], int32_t tap, const double *U,
                         double m, int32_t par, const double *in, double *out,
                         double *tmp)
{
    const int64_t V = volume(L);
    const int32_t other = (par == 2) ? 2 : 1 - par;
    double *src = calloc(6 * V, sizeof(double));
    double *dd = calloc(6 * V, sizeof(double));
    copy_par(L, par, in, src);               /* in, restricted to par     */
    orc_dslash(L, tap, U, src, tmp, other);  /* tmp = D in                */
    orc_dslash(L, tap, U, tmp, dd, par);     /* dd  = D D in on par       */
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s)
        if (on_parity(s, L, par))
            for (int k = 0; k < 6; ++k)
                out[s * 6 + k] = m * m * in[s * 6 + k] - dd[s * 6 + k];
    free(src);
    free(dd);
}

int orc_apply_normal(const int32_t L[4], int32_t tap, const double *U,
                     double m, int32_t par, const double *in, double *out)
{
    if (bad_dims(L) || par < 0 || par > 2)
        return -1;
    double *tmp = malloc(sizeof(double) * 6 * volume(L));
    if (!tmp)
        return -2;
    apply_normal(L, tap, U, m, par, in, out, tmp);
    free(tmp);
    return 0;
}

/* ||b - A x|| / ||b|| on parity par, in FP64 */
double orc_true_residual(const int32_t L[4], int32_t tap, const double *U,
                         double m, int32_t par, const double *b, const double *x)
{
    const int64_t n = 6 * volume(L);
    double *ax = calloc(n, sizeof(double));
    double *tmp = malloc(sizeof(double) * n);
    apply_normal(L, tap, U, m, par, x, ax, tmp);
    axpby(L, par, 1.0, b, -1.0, ax); /* ax = b - A x */
    double rr = norm2(L, par, ax), bb = norm2(L, par, b);
    free(ax);
    free(tmp);
    return bb > 0 ? sqrt(rr / bb) : sqrt(rr);
}

/* ------------------------------------------------------------------ */
/* CG in the form of the paper's Sec. 4 loop, one parity system         */
/* ------------------------------------------------------------------ */

/*
 * One CG pass from x = 0 on the parity system par (0 or 1):
 *   r = b, p = r, rr = <r,r>; stop at once if rr < tol^2 <b,b>;
 *   repeat: ap = D p (other parity); alpha = rr / (<ap,ap> + m^2 <p,p>);
 *           x += alpha p; atap = m^2 p - D ap; r -= alpha atap;
 *           rn = <r,r>; stop if rn < stop2; beta = rn/rr; p = r + beta p.
 * The stop threshold is passed in (tol^2 <b,b> of the original source, so
 * that a restart on a residual keeps the original target).
 * Returns the number of iterations; *rr_out holds the last <r,r>.  If
 * alphas / betas are not NULL they receive alpha and beta of every
 * iteration (beta of the last one is the ratio rn/rr that would have been
 * used next).
 */
static int cg_pass(const int32_t L[4], int32_t tap, const double *U, double m,
                   int32_t par, double stop2, int32_t maxiter, const double *b,
                   double *x, double *r, double *p, double *ap, double *atap,
                   double *rr_out, double *alphas, double *betas)
{
    const int32_t other = 1 - par;
    set_zero(L, par, x);
    copy_par(L, par, b, r);
    copy_par(L, par, r, p);
    double rr = norm2(L, par, r);
    int it = 0;
    if (rr < stop2 || rr == 0.0) {
        *rr_out = rr;
        return 0;
    }
    for (it = 1; it <= maxiter; ++it) {
        set_zero(L, other, ap);
        orc_dslash(L, tap, U, p, ap, other);                 /* ap = D p      */
        double pap = norm2(L, other, ap) + m * m * norm2(L, par, p);
        double alpha = rr / pap;
        axpby(L, par, alpha, p, 1.0, x);                     /* x += alpha p  */
        orc_dslash(L, tap, U, ap, atap, par);                /* atap = D ap   */
        axpby(L, par, m * m, p, -1.0, atap);                 /* m^2 p - D ap  */
        axpby(L, par, -alpha, atap, 1.0, r);                 /* r -= alpha Ap */
        double rn = norm2(L, par, r);
        if (alphas)
            alphas[it - 1] = alpha;
        if (betas)
            betas[it - 1] = rn / rr;
        if (rn < stop2) {
            rr = rn;
            break;
        }
        double beta = rn / rr;
        rr = rn;
        axpby(L, par, 1.0, r, beta, p);                      /* p = r + beta p */
    }
    *rr_out = rr;
    return it > maxiter ? maxiter : it;
}

/*
 * Solve (m^2 - D^2) x = b on parity system par (0, 1), or on both (2) as two
 * independent systems.  After each CG pass the true residual is computed in
 * FP64; if it is above tol the pass is repeated on the true residual and the
 * correction added to x (x0 = 0 inside every pass, as in the paper).
 * If y is not NULL, y = D x on the opposite parity (all sites for par = 2):
 * the paper's second-half reconstruction.
 * Returns 0 if converged, 1 if maxiter was reached, negative on bad input.
 */
int orc_cg_solve(const int32_t L[4], int32_t tap, const double *U, double m,
                 double tol, int32_t maxiter, int32_t max_restarts, int32_t par,
                 const double *b, double *x, double *y, orc_cg_result *res)
{
    if (bad_dims(L) || par < 0 || par > 2 || !(m > 0) || !(tol > 0) || maxiter < 0)
        return -1;
    if (par == 2) {
        orc_cg_result r0, r1;
        int s0 = orc_cg_solve(L, tap, U, m, tol, maxiter, max_restarts, 0, b, x, NULL, &r0);
        int s1 = orc_cg_solve(L, tap, U, m, tol, maxiter, max_restarts, 1, b, x, NULL, &r1);
        if (s0 < 0 || s1 < 0)
            return -1;
        if (y)
            orc_dslash(L, tap, U, x, y, 2);
        if (res) {
            res->status = (s0 || s1) ? 1 : 0;
            res->iters = r0.iters > r1.iters ? r0.iters : r1.iters;
            res->restarts = r0.restarts > r1.restarts ? r0.restarts : r1.restarts;
            res->rr = r0.rr + r1.rr;
            res->bb = r0.bb + r1.bb;
            res->true_rel = orc_true_residual(L, tap, U, m, 2, b, x);
        }
        return (s0 || s1) ? 1 : 0;
    }
    const int64_t n = 6 * volume(L);
    double *r = calloc(n, sizeof(double)), *p = calloc(n, sizeof(double));
    double *ap = calloc(n, sizeof(double)), *atap = calloc(n, sizeof(double));
    double *dx = calloc(n, sizeof(double)), *src = calloc(n, sizeof(double));
    double *tmp = calloc(n, sizeof(double));
    const double bb = norm2(L, par, b);
    const double stop2 = tol * tol * bb;
    int total = 0, restarts = 0, status = 0;
    double rr = 0, rel = 0;

    set_zero(L, par, x);
    copy_par(L, par, b, src);
    for (;;) {
        int it = cg_pass(L, tap, U, m, par, stop2, maxiter - total, src, dx, r, p,
                         ap, atap, &rr, NULL, NULL);
        total += it;
        axpby(L, par, 1.0, dx, 1.0, x);                      /* x += correction */
        /* true residual in FP64: src = b - A x */
        apply_normal(L, tap, U, m, par, x, src, tmp);
        axpby(L, par, 1.0, b, -1.0, src);
        double tr = norm2(L, par, src);
        rel = bb > 0 ? sqrt(tr / bb) : sqrt(tr);
        if (tr <= stop2)
            break;
        if (total >= maxiter || restarts >= max_restarts) {
            status = 1;
            break;
        }
        ++restarts;
    }
    if (y) {
        int32_t other = 1 - par;
        orc_dslash(L, tap, U, x, y, other);
    }
    if (res) {
        res->status = status;
        res->iters = total;
        res->restarts = restarts;
        res->rr = rr;
        res->bb = bb;
        res->true_rel = rel;
    }
    free(r); free(p); free(ap); free(atap); free(dx); free(src); free(tmp);
    return status;
}

/*
 * One CG pass from x = 0 on parity system par, exactly the paper's loop and
 * stopping rule, with no true-residual restart.  Used to compare the GPU's
 * iterates step by step: maxiter bounds the iterations, so the k-th iterate
 * is available by passing maxiter = k and tol = 0.
 */
int orc_cg_pass(const int32_t L[4], int32_t tap, const double *U, double m,
                double tol, int32_t maxiter, int32_t par, const double *b,
                double *x, orc_cg_result *res)
{
    if (bad_dims(L) || par < 0 || par > 1 || !(m > 0) || tol < 0 || maxiter < 0)
        return -1;
    const int64_t n = 6 * volume(L);
    double *r = calloc(n, sizeof(double)), *p = calloc(n, sizeof(double));
    double *ap = calloc(n, sizeof(double)), *atap = calloc(n, sizeof(double));
    const double bb = norm2(L, par, b);
    double rr = 0;
    int it = cg_pass(L, tap, U, m, par, tol * tol * bb, maxiter, b, x, r, p, ap, atap, &rr, NULL, NULL);
    if (res) {
        res->status = rr < tol * tol * bb ? 0 : 1;
        res->iters = it;
        res->restarts = 0;
        res->rr = rr;
        res->bb = bb;
        res->true_rel = orc_true_residual(L, tap, U, m, par, b, x);
    }
    free(r); free(p); free(ap); free(atap);
    return 0;
}

/*
 * The same single pass, also returning alpha_k and beta_k of every iteration
 * k = 1..iters (arrays of maxiter doubles).  These are the coefficients of
 * the Lanczos process that CG carries out implicitly; the eigenvalues of the
 * tridiagonal matrix built from them (the Ritz values) approximate the
 * spectrum of the parity system's operator from the inside, extreme ones
 * first, which gives an estimate of its condition number.
 */
int orc_cg_coefficients(const int32_t L[4], int32_t tap, const double *U, double m,
                        double tol, int32_t maxiter, int32_t par, const double *b,
                        double *x, double *alphas, double *betas, orc_cg_result *res)
{
    if (bad_dims(L) || par < 0 || par > 1 || !(m > 0) || tol < 0 || maxiter < 0 || !alphas || !betas)
        return -1;
    const int64_t n = 6 * volume(L);
    double *r = calloc(n, sizeof(double)), *p = calloc(n, sizeof(double));
    double *ap = calloc(n, sizeof(double)), *atap = calloc(n, sizeof(double));
    const double bb = norm2(L, par, b);
    double rr = 0;
    int it = cg_pass(L, tap, U, m, par, tol * tol * bb, maxiter, b, x, r, p, ap, atap, &rr, alphas, betas);
    if (res) {
        res->status = rr < tol * tol * bb ? 0 : 1;
        res->iters = it;
        res->restarts = 0;
        res->rr = rr;
        res->bb = bb;
        res->true_rel = orc_true_residual(L, tap, U, m, par, b, x);
    }
    free(r); free(p); free(ap); free(atap);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Textbook CG on the whole lattice (no even/odd split)                */
/* ------------------------------------------------------------------ */

/*
 * Plain CG on A = m^2 - D^2 over all sites, starting from the x passed in.
 * Used for the tight reference solve (tol down to rounding, with restarts
 * from the true residual).  Returns iterations, or -1 on bad input.
 */
int orc_cg_full(const int32_t L[4], int32_t tap, const double *U, double m,
                double tol, int32_t maxiter, int32_t max_restarts,
                const double *b, double *x, orc_cg_result *res)
{
    if (bad_dims(L) || !(m > 0) || tol < 0 || maxiter < 0)
        return -1;
    const int64_t n = 6 * volume(L);
    double *r = calloc(n, sizeof(double)), *p = calloc(n, sizeof(double));
    double *ap = calloc(n, sizeof(double)), *tmp = calloc(n, sizeof(double));
    const double bb = norm2(L, 2, b);
    const double stop2 = tol * tol * bb;
    int total = 0, restarts = 0;
    double rr = 0, best = INFINITY;
    for (;;) {
        /* r = b - A x (true residual) */
        apply_normal(L, tap, U, m, 2, x, ap, tmp);
        memcpy(r, b, sizeof(double) * n);
        axpby(L, 2, -1.0, ap, 1.0, r);
        memcpy(p, r, sizeof(double) * n);
        rr = norm2(L, 2, r);
        if (rr <= stop2 || restarts > max_restarts || total >= maxiter || !(rr < best))
            break;
        best = rr;
        for (int it = 0; it < maxiter - total; ++it) {
            apply_normal(L, tap, U, m, 2, p, ap, tmp);
            double alpha = rr / creal(dot(L, 2, p, ap));
            axpby(L, 2, alpha, p, 1.0, x);
            axpby(L, 2, -alpha, ap, 1.0, r);
            double rn = norm2(L, 2, r);
            ++total;
            if (rn <= stop2) {
                rr = rn;
                break;
            }
            axpby(L, 2, 1.0, r, rn / rr, p);
            rr = rn;
        }
        ++restarts;
    }
    if (res) {
        res->status = rr <= stop2 ? 0 : 1;
        res->iters = total;
        res->restarts = restarts;
        res->rr = rr;
        res->bb = bb;
        res->true_rel = bb > 0 ? sqrt(rr / bb) : sqrt(rr);
    }
    free(r); free(p); free(ap); free(tmp);
    return total;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---- host bandwidth reference (no part of the method) ------------------ */

/* STREAM-style triad a = b + s c over n doubles, reps times, with the
 * OpenMP threads of the oracle; returns the wall seconds of the best rep.
 * The CPU's own bandwidth roofline for the oracle timings. */
static double wall_seconds(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

double orc_stream_triad(int64_t n, double *a, const double *b, const double *c, double s, int reps)
{
    double best = 1e30;
    for (int r = 0; r < reps; ++r) {
        const double t0 = wall_seconds();
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            a[i] = b[i] + s * c[i];
        const double t = wall_seconds() - t0;
        if (t < best)
            best = t;
    }
    return best;
}
