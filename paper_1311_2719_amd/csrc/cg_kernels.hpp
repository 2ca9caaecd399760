// Fused conjugate-gradient kernels for (m^2 - D^2) x = b on one parity,
// batched over systems that share a gauge field.
//
// The iteration is the loop of the paper's Sec. 4 with the mass explicit,
// rearranged into two kernels so that every vector is streamed once and every
// scalar stays on the device:
//   K1  p' = r + beta p (formed on the fly at every gathered neighbour, and
//       stored once at the partner site), ap = D p' on the other parity,
//       <ap,ap> and <p',p'>;          finalize: alpha = rr / (m^2 <p',p'> + <ap,ap>)
//   K2  Ap = m^2 p' - D ap; x += alpha p'; r -= alpha Ap; <r,r>   (Ap never stored)
//                                     finalize: stopping test, beta = rn / rr
// p and p' alternate between two buffers per system (pcur).
// FP64 residual recomputation (reliable updates in mixed precision, and the
// final true-residual check in every mode):
//   RU2 t = D x on the other parity in FP64 (x = x_hi + x_lo)
//   RU3 x_hi += x_lo, x_lo = 0, r = b - m^2 x_hi + D t in FP64, <r,r>
// Each main kernel writes per-block partial sums; a one-block-per-system
// finalize kernel (k_cg_fin) launched right after it reduces them in a fixed
// order and evaluates the scalar recurrences and the stopping test of its
// system, so the host never reads a scalar inside the loop and no cross-block
// synchronisation (fence or atomic) is needed inside a kernel.
//
// Systems: nsys = 2*S, system j has parity j / S (its x, r, p live on that
// parity; ap and t on the other).  A tile is R systems of one parity that are
// processed together so each link entry is loaded once for all of them; the
// tiles take their systems from a per-parity list (perm) that the host
// compacts between epochs, so the number of tiles that read links follows the
// number of systems still running.  A system's partial sums depend only on
// the sites of each block, not on its tile, so compaction does not change
// results.
#pragma once

#include "hop.hpp"

namespace stag {

enum Phase : int32_t { PH_IDLE = 0, PH_INIT = 1, PH_RUN = 2, PH_DONE = 3 };

struct SysState {
    double mass2;
    double tol2;
    double stop2;    // tol^2 <b,b>
    double bb;
    double rr;       // <r,r> of the current (iterated) residual
    double pp;       // <p,p> of the stored search direction
    double alpha;
    double beta;
    double maxr2;    // largest <r,r> since the last residual recomputation
    double delta2;   // reliable-update threshold squared (0: final check only)
    double true_rr;  // <r,r> of the last FP64 residual recomputation
    double pad0;
    int32_t phase;
    int32_t ru_pending;  // residual recomputation requested
    int32_t stopping;    // status to report if the recomputation does not converge
    int32_t status;      // final status (phase == PH_DONE)
    int32_t iters;
    int32_t maxiter;
    int32_t n_ru;
    int32_t restarts;
    int32_t max_restarts;
    int32_t mixed;
    int32_t pcur;        // which of the two p buffers holds the current direction
    int32_t pad1;
};

struct CgArgs {
    Geom g;
    const void *links[2];      // links of the working precision, per output parity
    const dbl2 *links64[2];    // FP64 links, per output parity
    const int32_t *nbr[2];     // neighbour tables per output parity, or null
    void *p[2];                // [nsys] stored search directions (working precision), two buffers
    void *ap;                  // [nsys] stored spinors (working precision)
    void *r;                   // [nsys][3][Vh] complex of the compute type
    flt2 *xlo;                 // [nsys][3][Vh] (mixed precision only)
    dbl2 *tmp;                 // [nsys][3][Vh] FP64 work vector (other parity)
    dbl2 *const *xhi;          // [nsys] parity half of the caller's x
    const dbl2 *const *b;      // [nsys] parity half of the caller's b
    SysState *st;              // [nsys]
    const int *perm;           // [2][S] systems of each parity in tile order, -1 = none
    double *partials;          // [nsys][2][pstride]
    int S;                     // systems per parity
    int pstride;
    int remap;
};

template <typename T> struct vec2_of;
template <> struct vec2_of<double> { using type = dbl2; };
template <> struct vec2_of<float> { using type = flt2; };

template <class P> __device__ __forceinline__ void *spin_at(void *base, int j, int Vh)
{
    return (char *)base + (size_t)j * Vh * P::spinor_bytes;
}

template <class P> __device__ __forceinline__ cplx<typename P::real> load_colour(const void *base, int Vh, int s, int c)
{
    if constexpr (P::id == 2) {
        cplx<typename P::real> v[3];
        P::load_spinor(base, Vh, s, v);
        return v[c];
    } else {
        using v2 = typename vec2_of<typename P::real>::type;
        v2 t = ((const v2 *)base)[(int64_t)c * Vh + s];
        return {t.x, t.y};
    }
}

// Parity of a tile and the offset of its first entry in the system list.
__device__ __forceinline__ void tile_of(const CgArgs &a, int tile, int R, int &par, int &k0)
{
    const int tpp = a.S / R;
    par = tile / tpp;
    k0 = par * a.S + (tile % tpp) * R;
}

__device__ __forceinline__ bool finite_pos(double v) { return v > 0.0 && v < INFINITY; }

__device__ __forceinline__ double *partial_slot(const CgArgs &a, int j, int which)
{
    return a.partials + ((size_t)j * 2 + which) * a.pstride;
}

// ---- K1: p' = r + beta p, ap = D p' ---------------------------------------------

template <class P, int LPS, int R>
__global__ void __launch_bounds__(256) k_cg_ap(CgArgs a)
{
    using real = typename P::real;
    using v2 = typename vec2_of<real>::type;
    __shared__ double lds[2 * R * 4];
    int par, k0;
    tile_of(a, blockIdx.y, R, par, k0);
    const int pout = 1 - par;
    int js[R];
    bool act[R];
    real beta[R];
    int pc[R];
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = a.perm[k0 + r];
        js[r] = j < 0 ? 0 : j;
        const SysState &st = a.st[js[r]];
        act[r] = j >= 0 && st.phase == PH_RUN && !st.ru_pending;
        beta[r] = (real)st.beta;
        pc[r] = st.pcur;
        any |= act[r];
    }
    if (!any)
        return;
    const int Vh = a.g.Vh;
    int s, sub;
    site_of_thread<LPS>(logical_block(blockIdx.x, gridDim.x, a.remap) * blockDim.x + threadIdx.x, s, sub);
    double nrm[2 * R];
#pragma unroll
    for (int r = 0; r < 2 * R; ++r)
        nrm[r] = 0.0;
    if (s < Vh) {
        cplx<real> acc[R][3];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                acc[r][c] = czero<real>();
        auto load = [&](int r, int n, cplx<real> *chi) {
            const int j = js[r];
            const v2 *rv = (const v2 *)a.r + (size_t)j * 3 * Vh;
            cplx<real> pv[3];
            P::load_spinor(spin_at<P>(a.p[pc[r]], j, Vh), Vh, n, pv);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const v2 t = rv[(int64_t)c * Vh + n];
                chi[c].re = fma(beta[r], pv[c].re, t.x);
                chi[c].im = fma(beta[r], pv[c].im, t.y);
            }
        };
        hop_accumulate<P, LPS, R>(a.g, (const typename P::link_t *)a.links[pout], a.nbr[pout], pout, s, sub, act,
                                  acc, load);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!act[r])
                continue;
            const int j = js[r];
            void *out = spin_at<P>(a.ap, j, Vh);
            const v2 *rv = (const v2 *)a.r + (size_t)j * 3 * Vh;
            const void *pold = spin_at<P>(a.p[pc[r]], j, Vh);
            void *pnew = spin_at<P>(a.p[pc[r] ^ 1], j, Vh);
            if constexpr (P::id == 2) {
                if (sub == 0) {
                    P::store_spinor(out, Vh, s, acc[r]);
                    // the new direction at the partner site (same index, parity par)
                    cplx<real> pv[3];
                    P::load_spinor(pold, Vh, s, pv);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const v2 t = rv[(int64_t)c * Vh + s];
                        pv[c].re = fma(beta[r], pv[c].re, t.x);
                        pv[c].im = fma(beta[r], pv[c].im, t.y);
                    }
                    P::store_spinor(pnew, Vh, s, pv);
                    P::load_spinor(pnew, Vh, s, pv);  // the norm of the value D will read
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        nrm[R + r] += (double)pv[c].re * pv[c].re + (double)pv[c].im * pv[c].im;
                }
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (!owns_colour<LPS>(sub, c))
                        continue;
                    const int64_t o = (int64_t)c * Vh + s;
                    ((v2 *)out)[o] = v2{acc[r][c].re, acc[r][c].im};
                    const v2 po = ((const v2 *)pold)[o];
                    const v2 t = rv[o];
                    const v2 pn = v2{fma(beta[r], po.x, t.x), fma(beta[r], po.y, t.y)};
                    ((v2 *)pnew)[o] = pn;
                    nrm[R + r] += (double)pn.x * pn.x + (double)pn.y * pn.y;
                }
            }
            if (sub == 0) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    nrm[r] += (double)acc[r][c].re * acc[r][c].re + (double)acc[r][c].im * acc[r][c].im;
            }
        }
    }
    double tot;
    block_sum_multi<2 * R>(nrm, lds, tot);
    if (threadIdx.x < 2 * R) {
        const int j = a.perm[k0 + (int)threadIdx.x % R];
        if (j >= 0)
            partial_slot(a, j, (int)threadIdx.x / R)[blockIdx.x] = tot;
    }
}

// ---- K2: Ap = m^2 p - D ap, x += alpha p, r -= alpha Ap ------------------------

template <class P, int LPS, int R>
__global__ void __launch_bounds__(256) k_cg_update(CgArgs a)
{
    using real = typename P::real;
    using v2 = typename vec2_of<real>::type;
    __shared__ double lds[R * 4];
    int par, k0;
    tile_of(a, blockIdx.y, R, par, k0);
    int js[R];
    bool act[R];
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = a.perm[k0 + r];
        js[r] = j < 0 ? 0 : j;
        const SysState &st = a.st[js[r]];
        act[r] = j >= 0 && st.phase == PH_RUN && !st.ru_pending;
        any |= act[r];
    }
    if (!any)
        return;
    const int Vh = a.g.Vh;
    int s, sub;
    site_of_thread<LPS>(logical_block(blockIdx.x, gridDim.x, a.remap) * blockDim.x + threadIdx.x, s, sub);
    double nrm[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        nrm[r] = 0.0;
    if (s < Vh) {
        cplx<real> acc[R][3];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                acc[r][c] = czero<real>();
        auto load = [&](int r, int n, cplx<real> *chi) { P::load_spinor(spin_at<P>(a.ap, js[r], Vh), Vh, n, chi); };
        hop_accumulate<P, LPS, R>(a.g, (const typename P::link_t *)a.links[par], a.nbr[par], par, s, sub, act, acc,
                                  load);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!act[r])
                continue;
            const int j = js[r];
            const SysState &st = a.st[j];
            const real m2 = (real)st.mass2, alpha = (real)st.alpha;
            const void *pb = spin_at<P>(a.p[st.pcur], j, Vh);
            v2 *rv = (v2 *)a.r + (size_t)j * 3 * Vh;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (!owns_colour<LPS>(sub, c))
                    continue;
                const cplx<real> pv = load_colour<P>(pb, Vh, s, c);
                const int64_t o = (int64_t)c * Vh + s;
                if constexpr (P::id == 0) {
                    dbl2 *x = a.xhi[j];
                    const dbl2 xv = x[o];
                    x[o] = dbl2{fma(alpha, pv.re, xv.x), fma(alpha, pv.im, xv.y)};
                } else {
                    flt2 *xl = a.xlo + (size_t)j * 3 * Vh;
                    const flt2 xv = xl[o];
                    xl[o] = flt2{fmaf(alpha, pv.re, xv.x), fmaf(alpha, pv.im, xv.y)};
                }
                const real apr = m2 * pv.re - acc[r][c].re;
                const real api = m2 * pv.im - acc[r][c].im;
                v2 rr = rv[o];
                rr.x = fma(-alpha, apr, rr.x);
                rr.y = fma(-alpha, api, rr.y);
                rv[o] = rr;
                nrm[r] += (double)rr.x * rr.x + (double)rr.y * rr.y;
            }
        }
    }
    double tot;
    block_sum_multi<R>(nrm, lds, tot);
    if (threadIdx.x < R) {
        const int j = a.perm[k0 + (int)threadIdx.x];
        if (j >= 0)
            partial_slot(a, j, 0)[blockIdx.x] = tot;
    }
}

// ---- init: x = 0, r = b, p = r, beta = 0 ------------------------------------------

template <class P>
__global__ void __launch_bounds__(256) k_cg_init(CgArgs a)
{
    using real = typename P::real;
    using v2 = typename vec2_of<real>::type;
    __shared__ double lds[4];
    const int j = blockIdx.y;
    if (a.st[j].phase != PH_INIT)
        return;
    const int Vh = a.g.Vh;
    const int s = logical_block(blockIdx.x, gridDim.x, a.remap) * blockDim.x + threadIdx.x;
    double nrm[1] = {0.0};
    if (s < Vh) {
        const dbl2 *b = a.b[j];
        dbl2 *x = a.xhi[j];
        v2 *rv = (v2 *)a.r + (size_t)j * 3 * Vh;
        cplx<real> pv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t o = (int64_t)c * Vh + s;
            const dbl2 bv = b[o];
            x[o] = dbl2{0.0, 0.0};
            if constexpr (P::id != 0)
                a.xlo[(size_t)j * 3 * Vh + o] = flt2{0.f, 0.f};
            rv[o] = v2{(real)bv.x, (real)bv.y};
            pv[c] = {(real)bv.x, (real)bv.y};
            nrm[0] += bv.x * bv.x + bv.y * bv.y;
        }
        P::store_spinor(spin_at<P>(a.p[0], j, Vh), Vh, s, pv);
    }
    double tot;
    block_sum_multi<1>(nrm, lds, tot);
    if (threadIdx.x == 0)
        partial_slot(a, j, 0)[blockIdx.x] = tot;
}

// ---- RU2: t = D (x_hi + x_lo) on the other parity, FP64 -----------------------------

template <int LPS, bool MIXED>
__global__ void __launch_bounds__(256) k_ru_dx(CgArgs a)
{
    const int j = blockIdx.y;
    {
        const SysState &st = a.st[j];
        if (!(st.phase == PH_RUN && st.ru_pending))
            return;
    }
    const int par = j / a.S, pout = 1 - par;
    const int Vh = a.g.Vh;
    int s, sub;
    site_of_thread<LPS>(logical_block(blockIdx.x, gridDim.x, a.remap) * blockDim.x + threadIdx.x, s, sub);
    if (s >= Vh)
        return;
    const dbl2 *xh = a.xhi[j];
    const flt2 *xl = a.xlo + (size_t)j * 3 * Vh;
    const bool act[1] = {true};
    cplx<double> acc[1][3] = {{czero<double>(), czero<double>(), czero<double>()}};
    auto load = [&](int, int n, cplx<double> *chi) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            dbl2 v = xh[(int64_t)c * Vh + n];
            if constexpr (MIXED) {
                const flt2 w = xl[(int64_t)c * Vh + n];
                v.x += (double)w.x;
                v.y += (double)w.y;
            }
            chi[c] = {v.x, v.y};
        }
    };
    hop_accumulate<PrecF64, LPS, 1>(a.g, a.links64[pout], a.nbr[pout], pout, s, sub, act, acc, load);
    dbl2 *t = a.tmp + (size_t)j * 3 * Vh;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        if (owns_colour<LPS>(sub, c))
            t[(int64_t)c * Vh + s] = dbl2{acc[0][c].re, acc[0][c].im};
}

// ---- RU3: x_hi += x_lo, r = b - m^2 x_hi + D t in FP64 ----------------------------------

template <class P, int LPS>
__global__ void __launch_bounds__(256) k_ru_residual(CgArgs a)
{
    using real = typename P::real;
    using v2 = typename vec2_of<real>::type;
    constexpr bool MIXED = P::id != 0;
    __shared__ double lds[4];
    const int j = blockIdx.y;
    {
        const SysState &st = a.st[j];
        if (!(st.phase == PH_RUN && st.ru_pending))
            return;
    }
    const int par = j / a.S;
    const int Vh = a.g.Vh;
    int s, sub;
    site_of_thread<LPS>(logical_block(blockIdx.x, gridDim.x, a.remap) * blockDim.x + threadIdx.x, s, sub);
    double nrm[1] = {0.0};
    if (s < Vh) {
        const dbl2 *t = a.tmp + (size_t)j * 3 * Vh;
        const bool act[1] = {true};
        cplx<double> acc[1][3] = {{czero<double>(), czero<double>(), czero<double>()}};
        auto load = [&](int, int n, cplx<double> *chi) { PrecF64::load_spinor(t, Vh, n, chi); };
        hop_accumulate<PrecF64, LPS, 1>(a.g, a.links64[par], a.nbr[par], par, s, sub, act, acc, load);
        const double m2 = a.st[j].mass2;
        dbl2 *x = a.xhi[j];
        const dbl2 *b = a.b[j];
        v2 *rv = (v2 *)a.r + (size_t)j * 3 * Vh;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (!owns_colour<LPS>(sub, c))
                continue;
            const int64_t o = (int64_t)c * Vh + s;
            dbl2 xv = x[o];
            if constexpr (MIXED) {
                const flt2 w = a.xlo[(size_t)j * 3 * Vh + o];
                xv.x += (double)w.x;
                xv.y += (double)w.y;
                x[o] = xv;
                a.xlo[(size_t)j * 3 * Vh + o] = flt2{0.f, 0.f};
            }
            const dbl2 bv = b[o];
            const double rre = bv.x - m2 * xv.x + acc[0][c].re;
            const double rim = bv.y - m2 * xv.y + acc[0][c].im;
            rv[o] = v2{(real)rre, (real)rim};
            nrm[0] += rre * rre + rim * rim;
        }
    }
    double tot;
    block_sum_multi<1>(nrm, lds, tot);
    if (threadIdx.x == 0)
        partial_slot(a, j, 0)[blockIdx.x] = tot;
}

// ---- finalize kernels: one block per system ---------------------------------------
//
// Launched right after the main kernel of the same role, with the main
// kernel's block count.  The main kernels do not modify the state, so the
// finalize kernel re-evaluates exactly the activity test the main kernel
// used.

enum FinRole { FIN_INIT = 0, FIN_AP = 1, FIN_UPDATE = 2, FIN_RU = 3 };

template <int ROLE>
__global__ void __launch_bounds__(256) k_cg_fin(CgArgs a, int nblk)
{
    __shared__ double lds[4];
    const int j = blockIdx.x;
    SysState &st = a.st[j];
    bool act;
    if (ROLE == FIN_INIT)
        act = st.phase == PH_INIT;
    else if (ROLE == FIN_RU)
        act = st.phase == PH_RUN && st.ru_pending;
    else
        act = st.phase == PH_RUN && !st.ru_pending;
    if (!act)
        return;
    const double v0 = reduce_partials(partial_slot(a, j, 0), nblk, lds);
    double v1 = 0.0;
    if (ROLE == FIN_AP)
        v1 = reduce_partials(partial_slot(a, j, 1), nblk, lds);
    if (threadIdx.x != 0)
        return;
    if (ROLE == FIN_INIT) {
        const double bb = v0;
        st.bb = bb;
        st.stop2 = st.tol2 * bb;
        st.rr = bb;
        st.pp = bb;
        st.maxr2 = bb;
        st.iters = 0;
        st.n_ru = 0;
        st.restarts = 0;
        st.ru_pending = 0;
        st.stopping = 0;
        st.beta = 0.0;
        st.alpha = 0.0;
        st.pcur = 0;
        st.true_rr = bb;
        if (!(bb < INFINITY)) {
            st.phase = PH_DONE;
            st.status = STAG_ENONFINITE;
        } else if (bb == 0.0) {
            st.phase = PH_DONE;
            st.status = STAG_OK;
            st.true_rr = 0.0;
        } else {
            st.phase = PH_RUN;
        }
    } else if (ROLE == FIN_AP) {
        const double apap = v0, pp = v1;
        st.pcur ^= 1;
        st.pp = pp;
        const double pap = st.mass2 * pp + apap;
        if (!finite_pos(pap)) {
            st.ru_pending = 1;
            st.stopping = STAG_EBREAKDOWN;
        } else {
            st.alpha = st.rr / pap;
        }
    } else if (ROLE == FIN_UPDATE) {
        const double rn = v0;
        st.iters += 1;
        if (!(rn < INFINITY)) {
            st.ru_pending = 1;
            st.stopping = STAG_EBREAKDOWN;
        } else {
            const bool conv = rn < st.stop2;
            st.maxr2 = rn > st.maxr2 ? rn : st.maxr2;
            bool recompute = conv || rn < st.delta2 * st.maxr2;
            if (!conv && st.iters >= st.maxiter) {
                st.stopping = STAG_ENOCONV;
                recompute = true;
            }
            if (recompute) {
                // beta is formed from the recomputed residual; rr keeps the
                // previous iteration's value as its denominator
                st.ru_pending = 1;
            } else {
                st.beta = rn / st.rr;
                st.rr = rn;
            }
        }
    } else {
        const double trr = v0;
        st.n_ru += 1;
        st.ru_pending = 0;
        st.true_rr = trr;
        if (trr <= st.stop2) {
            st.phase = PH_DONE;
            st.status = STAG_OK;
        } else if (st.stopping) {
            st.phase = PH_DONE;
            st.status = st.stopping;
        } else if (!st.mixed) {
            // FP64: the recursive residual claimed convergence but the true one
            // disagrees: restart CG from the current x (fresh search direction).
            st.restarts += 1;
            if (st.restarts > st.max_restarts) {
                st.phase = PH_DONE;
                st.status = STAG_ENOCONV;
            } else {
                st.beta = 0.0;
                st.rr = trr;
                st.maxr2 = trr;
            }
        } else {
            // reliable update: keep the search direction, continue from the true residual
            st.beta = trr / st.rr;
            st.rr = trr;
            st.maxr2 = trr;
        }
    }
}

// ---- tuning probe: out_r = D in_r for R systems, no reductions -------------------
// blockIdx.y = tile; tiles alternate output parity like the CG kernels' tiles.

template <class P, int LPS, int R>
__global__ void __launch_bounds__(256) k_hop_probe(Geom g, const void *links, const int32_t *nbr, const void *in,
                                                    void *out, int remap)
{
    using real = typename P::real;
    const int Vh = g.Vh;
    const int pout = blockIdx.y & 1;
    int s, sub;
    site_of_thread<LPS>(logical_block(blockIdx.x, gridDim.x, remap) * blockDim.x + threadIdx.x, s, sub);
    if (s >= Vh)
        return;
    const size_t vb = (size_t)Vh * P::spinor_bytes;
    const char *inb = (const char *)in + (size_t)blockIdx.y * R * vb;
    char *outb = (char *)out + (size_t)blockIdx.y * R * vb;
    bool act[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        act[r] = true;
    cplx<real> acc[R][3];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            acc[r][c] = czero<real>();
    auto load = [&](int r, int n, cplx<real> *chi) { P::load_spinor(inb + r * vb, Vh, n, chi); };
    const typename P::link_t *lk = (const typename P::link_t *)links + (size_t)pout * 72 * Vh;
    hop_accumulate<P, LPS, R>(g, lk, nbr ? nbr + (size_t)pout * 8 * Vh : nullptr, pout, s, sub, act, acc, load);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        void *o = outb + r * vb;
        if constexpr (P::id == 2) {
            if (sub == 0)
                P::store_spinor(o, Vh, s, acc[r]);
        } else {
            using v2 = typename vec2_of<real>::type;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if (owns_colour<LPS>(sub, c))
                    ((v2 *)o)[(int64_t)c * Vh + s] = v2{acc[r][c].re, acc[r][c].im};
        }
    }
}

}  // namespace stag
