// Wilson-fermion kernels: the hopping term H of M = 1 - kappa H and the fused
// even-odd CG on Mhat^dagger Mhat, Mhat = 1 - kappa^2 D_eo D_oe (FP64).
//
// The paper's second workload is an N_f = 2 Wilson-fermion program (Sec. 2, Sec. 6);
// it does not write the operator out, so the textbook form is used:
//   (H psi)(x) = sum_mu [(1 - gamma_mu) W_mu(x) psi(x + mu) + (1 + gamma_mu) B_mu(x) psi(x - mu)],
//   W_mu(x) = s U_mu(x), B_mu(x) = s U_mu(x - mu)^dagger (s: the t-boundary sign),
// gamma matrices of a chiral basis with gamma_5 = diag(1, 1, -1, -1).
//
// Spin projection: 1 -+ gamma_mu has rank 2 in this basis, so each hop
// projects the neighbour's 4-spinor onto two spin components h0, h1, applies
// the 3x3 link to those only, and rebuilds spins 2 and 3 as multiples of
// them (half the colour arithmetic of the full product).
//
// Layout: links as for the staggered operator ([entry][tile][dir][site], FP64,
// two or three stored rows); spinors of one parity as 12 planes of Vh complex
// (plane = 3 * spin + colour), a full field as [parity][12][Vh].  The template
// parameter LP reads the links: PrecF64 with plain loads, PrecF64NT with
// non-temporal ones (fields whose links do not fit the Infinity Cache, where
// each link, read once per launch, would otherwise evict gathered spinors).
#pragma once

#include "hop.hpp"

namespace stag {
namespace wil {

// ---- spin projection tables ---------------------------------------------------------
// Coefficients coded 0: 1, 1: -1, 2: i, 3: -i.
// Direction d = mu (forward, 1 - gamma_mu) or 4 + mu (backward, 1 + gamma_mu):
//   h0 = psi_0 + a0 psi_k0, h1 = psi_1 + a1 psi_k1;
//   result spins (h0, h1, b2 h_j2, b3 h_j3).
struct Proj {
    int k0, a0, k1, a1, j2, b2, j3, b3;
};
__device__ constexpr Proj kProj[8] = {
    {3, 3, 2, 3, 1, 2, 0, 2},  // mu = x, forward
    {3, 0, 2, 1, 1, 1, 0, 0},  // mu = y, forward
    {2, 3, 3, 2, 0, 2, 1, 3},  // mu = z, forward
    {2, 1, 3, 1, 0, 1, 1, 1},  // mu = t, forward
    {3, 2, 2, 2, 1, 3, 0, 3},  // mu = x, backward
    {3, 1, 2, 0, 1, 0, 0, 1},  // mu = y, backward
    {2, 2, 3, 3, 0, 3, 1, 2},  // mu = z, backward
    {2, 0, 3, 0, 0, 0, 1, 0},  // mu = t, backward
};

template <int C> __device__ __forceinline__ cplx<double> times(const cplx<double> &z)
{
    if constexpr (C == 0)
        return z;
    else if constexpr (C == 1)
        return {-z.re, -z.im};
    else if constexpr (C == 2)
        return {-z.im, z.re};
    else
        return {z.im, -z.re};
}

// z times the coefficient coded c, without branches (c may be a runtime value:
// the coefficient is formed by selects of constants, and the product by
// multiplications, so the gathers around it are not split into separate
// basic blocks that each wait for their loads)
__device__ __forceinline__ cplx<double> times(int c, const cplx<double> &z)
{
    const double cr = c == 0 ? 1.0 : (c == 1 ? -1.0 : 0.0);
    const double ci = c == 2 ? 1.0 : (c == 3 ? -1.0 : 0.0);
    return {z.re * cr - z.im * ci, z.re * ci + z.im * cr};
}

// The projector of direction d, 4 bits per field, so that a lane-dependent
// choice between directions is one select of a constant word.
__host__ __device__ constexpr uint32_t pack_proj(const Proj &q)
{
    return (uint32_t)q.k0 | (uint32_t)q.a0 << 4 | (uint32_t)q.k1 << 8 | (uint32_t)q.a1 << 12 | (uint32_t)q.j2 << 16 |
           (uint32_t)q.b2 << 20 | (uint32_t)q.j3 << 24 | (uint32_t)q.b3 << 28;
}

__device__ __forceinline__ Proj unpack_proj(uint32_t w)
{
    return {(int)(w & 15), (int)(w >> 4 & 15), (int)(w >> 8 & 15), (int)(w >> 12 & 15),
            (int)(w >> 16 & 15), (int)(w >> 20 & 15), (int)(w >> 24 & 15), (int)(w >> 28)};
}

// Projector of direction j * LPS + sub.  The table is never read from memory:
// with j known at compile time (unrolled loop) the word is chosen among the
// LPS candidates of the lanes; with a runtime j (rolled loop, LPS = 1, the
// same in every lane) among all eight.
template <int LPS> __device__ __forceinline__ Proj proj_of(int j, int sub)
{
    const int d = j * LPS + sub;
    uint32_t w = pack_proj(kProj[0]);
#pragma unroll
    for (int t = 1; t < 8; ++t)
        w = d == t ? pack_proj(kProj[t]) : w;
    return unpack_proj(w);
}

// True when the t-boundary sign folded into Wilson link d of the site with
// coordinates c is negative.
__device__ __forceinline__ bool wilson_link_negative(const Geom &g, const SiteCoord &c, int d)
{
    const int ct = c.t, Lt = g.L[3], tap = g.tap;  // values first: the choice below is a select
    return tap && (d & 3) == 3 && (d >= 4 ? ct == 0 : ct == Lt - 1);
}

// acc[spin][colour] = (H psi)(s) for output site s of parity p_out, computed
// by LPS lanes (sub = 0 .. LPS-1; lane sub takes directions sub, sub + LPS,
// ...) and summed over them, so every lane of the site ends with the total.
// load(n, sp, col) returns component (sp, col) of the input at site n of the
// other parity (with gamma_5 or any fused combination applied by the caller).
template <int ROWS, int LPS, class LP, class Load>
__device__ __forceinline__ void wilson_hop(const Geom &g, const dbl2 *__restrict__ links, int p_out, int s, int sub,
                                           cplx<double> (&acc)[4][3], Load load)
{
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            acc[sp][a] = czero<double>();
    const SiteCoord c = decode_site(g, p_out, s);
    auto one_direction = [&](int j) {
        const int d = sub + j * LPS;
        const Proj q = proj_of<LPS>(j, sub);
        const int n = neighbour(g, c, s, d);
        cplx<double> U[9];
        const dbl2 *lp = links + link_offset(g.Vh, d, 0, s);
#pragma unroll
        for (int k = 0; k < 3 * ROWS; ++k)
            U[k] = LP::load_link(lp + (int64_t)k * 8 * g.Vh);
        if constexpr (ROWS == 2)
            third_row(U, wilson_link_negative(g, c, d) ? -1.0 : 1.0);
        cplx<double> h[2][3];
#pragma unroll
        for (int col = 0; col < 3; ++col) {
            const cplx<double> p0 = load(n, 0, col), p1 = load(n, 1, col);
            const cplx<double> pk0 = load(n, q.k0, col), pk1 = load(n, q.k1, col);  // spins 2, 3
            const cplx<double> t0 = times(q.a0, pk0), t1 = times(q.a1, pk1);
            h[0][col] = {p0.re + t0.re, p0.im + t0.im};
            h[1][col] = {p1.re + t1.re, p1.im + t1.im};
        }
        cplx<double> u[2][3];
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                u[k][a] = czero<double>();
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    cmac(u[k][a], U[a * 3 + b], h[k][b]);
            }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            acc[0][a].re += u[0][a].re;
            acc[0][a].im += u[0][a].im;
            acc[1][a].re += u[1][a].re;
            acc[1][a].im += u[1][a].im;
            const cplx<double> r2 = times(q.b2, q.j2 ? u[1][a] : u[0][a]);
            const cplx<double> r3 = times(q.b3, q.j3 ? u[1][a] : u[0][a]);
            acc[2][a].re += r2.re;
            acc[2][a].im += r2.im;
            acc[3][a].re += r3.re;
            acc[3][a].im += r3.im;
        }
    };
    if constexpr (LPS == 1) {
        // two directions per iteration: enough loads in flight without spilling
#pragma unroll 2
        for (int j = 0; j < 8; ++j)
            one_direction(j);
    } else {
#pragma unroll
        for (int j = 0; j < 8 / LPS; ++j)
            one_direction(j);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                acc[sp][a].re = lane_sum<LPS>(acc[sp][a].re);
                acc[sp][a].im = lane_sum<LPS>(acc[sp][a].im);
            }
    }
}

// Component k = 3 * spin + colour of the site is handled by lane k mod LPS.
template <int LPS> __device__ __forceinline__ bool owns_component(int sub, int sp, int col)
{
    return ((sp * 3 + col) % LPS) == sub;
}

// Component (spin, colour) of a 12-plane parity vector at site n.
__device__ __forceinline__ cplx<double> comp(const dbl2 *v, int Vh, int n, int sp, int col)
{
    const dbl2 t = v[(int64_t)(sp * 3 + col) * Vh + n];
    return {t.x, t.y};
}

__device__ __forceinline__ void put(dbl2 *v, int Vh, int n, int sp, int col, const cplx<double> &z)
{
    v[(int64_t)(sp * 3 + col) * Vh + n] = dbl2{z.re, z.im};
}

// Site and lane-within-site of this thread (LPS lanes per site, sub-major
// within a wavefront), false for threads past the last site.  With remap, the
// blocks of each XCD cover one contiguous range of sites (logical_block).
template <int LPS> __device__ __forceinline__ bool wsite(int Vh, int remap, int &s, int &sub)
{
    site_of_thread<LPS>((int)(logical_block(blockIdx.x, gridDim.x, remap) * blockDim.x + threadIdx.x), s, sub);
    return s < Vh;
}

// ---- the standalone hop: out_p = H_p in (one parity, or both with blockIdx.y) -------

template <int ROWS, int LPS, class LP>
__global__ void __launch_bounds__(128)
k_wilson_dslash(Geom g, const dbl2 *__restrict__ links, const dbl2 *__restrict__ in, dbl2 *__restrict__ out,
                int par_fixed, int remap)
{
    const int p = par_fixed >= 0 ? par_fixed : (int)blockIdx.y;
    const int Vh = g.Vh;
    int s, sub;
    if (!wsite<LPS>(Vh, remap, s, sub))
        return;
    const dbl2 *src = in + (size_t)(1 - p) * 12 * Vh;
    cplx<double> acc[4][3];
    wilson_hop<ROWS, LPS, LP>(g, links + link_parity_entries(ROWS, Vh) * p, p, s, sub, acc,
                          [&](int n, int sp, int col) { return comp(src, Vh, n, sp, col); });
    dbl2 *o = out + (size_t)p * 12 * Vh;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (owns_component<LPS>(sub, sp, a))
                put(o, Vh, s, sp, a, acc[sp][a]);
}

// ---- even-odd CG ------------------------------------------------------------------

enum WMode : int32_t { W_IDLE = 0, W_INIT = 1, W_CG = 2, W_DONE = 3 };

struct WState {
    double stop2;  // tol^2 <rhs, rhs>
    double tol2;
    double bb;
    double rr;     // <r,r>
    double beta;
    double pad[3];
    int32_t mode;
    int32_t status;
    int32_t iters;
    int32_t maxiter;
    int32_t pcur;  // buffer holding the current direction
    int32_t step;
    int32_t pad1[2];
};
static_assert(sizeof(WState) == 96, "state layout");

struct WArgs {
    Geom g;
    const dbl2 *links[2];  // per output parity
    double kappa;
    const dbl2 *b;         // caller's source [2][12][Vh]
    dbl2 *x;               // caller's solution [2][12][Vh]; even half iterated, odd half at the end
    dbl2 *bh;              // even: b_e + kappa D_eo b_o
    dbl2 *r;               // even
    dbl2 *p[2];            // even, two buffers
    dbl2 *ap;              // even: Mhat p'
    dbl2 *t;               // odd work vector
    WState *st[2];
    double *partials;      // [2 buffers][2 slots: 0 <ap,ap>, 1 <r,r>][pstride]
    int pstride;
    int remap;             // 1: XCD-contiguous site ranges (logical_block)
};

__device__ __forceinline__ double *wslot(const WArgs &a, int buf, int slot)
{
    return a.partials + ((size_t)buf * 2 + slot) * a.pstride;
}

// Totals of the first NS slots of partial buffer `buf` over nblk blocks,
// summed in a fixed order (strided per thread, then the wave and block trees).
template <int NS>
__device__ __forceinline__ void wtotals(const WArgs &a, int buf, int nblk, double *lds, double (&tot)[NS])
{
    double v[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k)
        v[k] = 0.0;
    for (int i0 = threadIdx.x; i0 < nblk; i0 += 4 * blockDim.x) {
        double q[4][NS];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * blockDim.x;
            const bool in = i < nblk;
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                const double v = wslot(a, buf, k)[in ? i : 0];  // in bounds; the guard selects
                q[u][k] = in ? v : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < NS; ++k)
                v[k] += q[u][k];
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const double t = wave_sum(v[k]);
        if (lane == 0)
            lds[k * nw + w] = t;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        double t = 0.0;
        for (int i = 0; i < nw; ++i)
            t += lds[k * nw + i];
        tot[k] = t;
    }
    __syncthreads();
}

// Block total of v into partial slot `slot` of buffer `buf` at this block.
__device__ __forceinline__ void wpartial(const WArgs &a, int buf, int slot, double v, double *lds)
{
    double arr[1] = {v};
    double out;
    block_sum_multi<1>(arr, lds, out);
    if (threadIdx.x == 0)
        wslot(a, buf, slot)[blockIdx.x] = out;
}

__device__ __forceinline__ bool wfinite_pos(double v) { return v > 0.0 && v < INFINITY; }

__device__ __forceinline__ int wuniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double wuniform(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// init 1 (even outputs): bh = b_e + kappa (H b)_e
template <int ROWS, int LPS, class LP> __global__ void __launch_bounds__(128) k_wil_bhat(WArgs a)
{
    const int Vh = a.g.Vh;
    int s, sub;
    if (!wsite<LPS>(Vh, a.remap, s, sub))
        return;
    const dbl2 *bo = a.b + (size_t)12 * Vh;
    cplx<double> acc[4][3];
    wilson_hop<ROWS, LPS, LP>(a.g, a.links[0], 0, s, sub, acc,
                          [&](int n, int sp, int col) { return comp(bo, Vh, n, sp, col); });
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (owns_component<LPS>(sub, sp, c)) {
                const cplx<double> be = comp(a.b, Vh, s, sp, c);
                put(a.bh, Vh, s, sp, c, {be.re + a.kappa * acc[sp][c].re, be.im + a.kappa * acc[sp][c].im});
            }
}

// odd outputs: t = H_oe (gamma_5 src).  With a state (K3 of a step) it runs
// only while the system iterates; without one (initialisation) always.
template <int ROWS, int LPS, class LP>
__global__ void __launch_bounds__(128) k_wil_odd_g5(WArgs a, const dbl2 *__restrict__ src, int ver, int check)
{
    if (check && a.st[ver ^ 1]->mode != W_CG)
        return;
    const int Vh = a.g.Vh;
    int s, sub;
    if (!wsite<LPS>(Vh, a.remap, s, sub))
        return;
    cplx<double> acc[4][3];
    wilson_hop<ROWS, LPS, LP>(a.g, a.links[1], 1, s, sub, acc, [&](int n, int sp, int col) {
        const cplx<double> z = comp(src, Vh, n, sp, col);
        return sp < 2 ? z : cplx<double>{-z.re, -z.im};
    });
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (owns_component<LPS>(sub, sp, c))
                put(a.t, Vh, s, sp, c, acc[sp][c]);
}

// init 3 (even outputs): r = bh - kappa^2 gamma_5 (H t)_e = Mhat^dagger bh;
// p[0] = r; x_e = 0; <r,r> into slot 1 of buffer 0
template <int ROWS, int LPS, class LP> __global__ void __launch_bounds__(128) k_wil_init(WArgs a)
{
    __shared__ double lds[4];
    const int Vh = a.g.Vh;
    int s, sub;
    double nrm = 0.0;
    if (wsite<LPS>(Vh, a.remap, s, sub)) {
        cplx<double> acc[4][3];
        wilson_hop<ROWS, LPS, LP>(a.g, a.links[0], 0, s, sub, acc,
                              [&](int n, int sp, int col) { return comp(a.t, Vh, n, sp, col); });
        const double k2 = a.kappa * a.kappa;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (!owns_component<LPS>(sub, sp, c))
                    continue;
                const double g5 = sp < 2 ? k2 : -k2;
                const cplx<double> bh = comp(a.bh, Vh, s, sp, c);
                const cplx<double> r = {bh.re - g5 * acc[sp][c].re, bh.im - g5 * acc[sp][c].im};
                put(a.r, Vh, s, sp, c, r);
                put(a.p[0], Vh, s, sp, c, r);
                put(a.x, Vh, s, sp, c, czero<double>());
                nrm += r.re * r.re + r.im * r.im;
            }
    }
    wpartial(a, 0, 1, nrm, lds);
}

// K1 (odd outputs): advance the state over the previous step, then
// t = H_oe p' with p' = r + beta p formed at every gathered neighbour; p' is
// also stored at the partner site (same index, even parity).
template <int ROWS, int LPS, class LP> __global__ void __launch_bounds__(128) k_wil_step1(WArgs a, int ver)
{
    __shared__ double lds[8];
    __shared__ __align__(16) WState sst;
    const int Vh = a.g.Vh, nblk = gridDim.x;
    if (threadIdx.x < sizeof(WState) / 16)
        ((uint4 *)&sst)[threadIdx.x] = ((const uint4 *)a.st[ver])[threadIdx.x];
    double tot[2];
    wtotals<2>(a, ver, nblk, lds, tot);  // its barriers also publish sst
    if (threadIdx.x == 0) {
        WState st = sst;
        st.step += 1;
        bool run = false;
        if (st.mode == W_INIT) {
            const double bb = tot[1];
            st.bb = bb;
            st.rr = bb;
            st.stop2 = st.tol2 * bb;
            st.beta = 0.0;
            st.iters = 0;
            if (!(bb < INFINITY)) {
                st.mode = W_DONE;
                st.status = STAG_ENONFINITE;
            } else if (bb == 0.0) {
                st.mode = W_DONE;
                st.status = STAG_OK;
            } else if (st.maxiter == 0) {
                st.mode = W_DONE;
                st.status = STAG_ENOCONV;
            } else {
                st.mode = W_CG;
                run = true;
            }
        } else if (st.mode == W_CG) {
            const double pap = tot[0], rn = tot[1];
            st.iters += 1;
            if (!wfinite_pos(pap) || !(rn < INFINITY)) {
                st.mode = W_DONE;
                st.status = STAG_EBREAKDOWN;
            } else if (rn < st.stop2) {
                st.rr = rn;
                st.mode = W_DONE;
                st.status = STAG_OK;
            } else if (st.iters >= st.maxiter) {
                st.rr = rn;
                st.mode = W_DONE;
                st.status = STAG_ENOCONV;
            } else {
                st.beta = rn / st.rr;
                st.rr = rn;
                run = true;
            }
        }
        if (run)
            st.pcur ^= 1;  // p' goes to the other buffer
        if (blockIdx.x == 0)
            *a.st[ver ^ 1] = st;
        sst = st;
    }
    __syncthreads();
    if (wuniform(sst.mode) != W_CG)
        return;
    const double beta = wuniform(sst.beta);
    const int pn = wuniform(sst.pcur);
    const dbl2 *pold = a.p[pn ^ 1];
    dbl2 *pnew = a.p[pn];
    int s, sub;
    if (!wsite<LPS>(Vh, a.remap, s, sub))
        return;
    cplx<double> acc[4][3];
    wilson_hop<ROWS, LPS, LP>(a.g, a.links[1], 1, s, sub, acc, [&](int n, int sp, int col) {
        const cplx<double> r = comp(a.r, Vh, n, sp, col), p = comp(pold, Vh, n, sp, col);
        return cplx<double>{fma(beta, p.re, r.re), fma(beta, p.im, r.im)};
    });
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (!owns_component<LPS>(sub, sp, c))
                continue;
            put(a.t, Vh, s, sp, c, acc[sp][c]);
            const cplx<double> r = comp(a.r, Vh, s, sp, c), p = comp(pold, Vh, s, sp, c);
            put(pnew, Vh, s, sp, c, {fma(beta, p.re, r.re), fma(beta, p.im, r.im)});
        }
}

// K2 (even outputs): ap = p' - kappa^2 (H t)_e = Mhat p'; <ap,ap> into slot 0
// of buffer ver^1
template <int ROWS, int LPS, class LP> __global__ void __launch_bounds__(128) k_wil_step2(WArgs a, int ver)
{
    __shared__ double lds[4];
    const WState *st = a.st[ver ^ 1];
    if (st->mode != W_CG)
        return;
    const dbl2 *pn = a.p[wuniform(st->pcur)];
    const int Vh = a.g.Vh;
    int s, sub;
    double nrm = 0.0;
    if (wsite<LPS>(Vh, a.remap, s, sub)) {
        cplx<double> acc[4][3];
        wilson_hop<ROWS, LPS, LP>(a.g, a.links[0], 0, s, sub, acc,
                              [&](int n, int sp, int col) { return comp(a.t, Vh, n, sp, col); });
        const double k2 = a.kappa * a.kappa;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (!owns_component<LPS>(sub, sp, c))
                    continue;
                const cplx<double> p = comp(pn, Vh, s, sp, c);
                const cplx<double> v = {p.re - k2 * acc[sp][c].re, p.im - k2 * acc[sp][c].im};
                put(a.ap, Vh, s, sp, c, v);
                nrm += v.re * v.re + v.im * v.im;
            }
    }
    wpartial(a, ver ^ 1, 0, nrm, lds);
}

// K4 (even outputs): alpha = rr / <ap,ap>; atap = ap - kappa^2 gamma_5 (H t)_e
// (= Mhat^dagger Mhat p'); x += alpha p'; r -= alpha atap; <r,r> into slot 1 of
// buffer ver^1
template <int ROWS, int LPS, class LP> __global__ void __launch_bounds__(128) k_wil_step4(WArgs a, int ver)
{
    __shared__ double lds[8];
    const WState *st = a.st[ver ^ 1];
    if (st->mode != W_CG)
        return;
    const int cur = ver ^ 1;
    const double rr = wuniform(st->rr);
    const dbl2 *pn = a.p[wuniform(st->pcur)];
    double tot[1];
    wtotals<1>(a, cur, gridDim.x, lds, tot);
    const double alpha = wfinite_pos(tot[0]) ? rr / tot[0] : 0.0;
    const int Vh = a.g.Vh;
    int s, sub;
    double nrm = 0.0;
    if (wsite<LPS>(Vh, a.remap, s, sub)) {
        cplx<double> acc[4][3];
        wilson_hop<ROWS, LPS, LP>(a.g, a.links[0], 0, s, sub, acc,
                              [&](int n, int sp, int col) { return comp(a.t, Vh, n, sp, col); });
        const double k2 = a.kappa * a.kappa;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (!owns_component<LPS>(sub, sp, c))
                    continue;
                const double g5 = sp < 2 ? k2 : -k2;
                const cplx<double> ap = comp(a.ap, Vh, s, sp, c);
                const cplx<double> atap = {ap.re - g5 * acc[sp][c].re, ap.im - g5 * acc[sp][c].im};
                const cplx<double> p = comp(pn, Vh, s, sp, c);
                const cplx<double> x = comp(a.x, Vh, s, sp, c);
                put(a.x, Vh, s, sp, c, {fma(alpha, p.re, x.re), fma(alpha, p.im, x.im)});
                cplx<double> r = comp(a.r, Vh, s, sp, c);
                r = {fma(-alpha, atap.re, r.re), fma(-alpha, atap.im, r.im)};
                put(a.r, Vh, s, sp, c, r);
                nrm += r.re * r.re + r.im * r.im;
            }
    }
    wpartial(a, cur, 1, nrm, lds);
}

// x_o = b_o + kappa (H x_e)_o
template <int ROWS, int LPS, class LP> __global__ void __launch_bounds__(128) k_wil_xodd(WArgs a)
{
    const int Vh = a.g.Vh;
    int s, sub;
    if (!wsite<LPS>(Vh, a.remap, s, sub))
        return;
    cplx<double> acc[4][3];
    wilson_hop<ROWS, LPS, LP>(a.g, a.links[1], 1, s, sub, acc,
                          [&](int n, int sp, int col) { return comp(a.x, Vh, n, sp, col); });
    const dbl2 *bo = a.b + (size_t)12 * Vh;
    dbl2 *xo = a.x + (size_t)12 * Vh;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (owns_component<LPS>(sub, sp, c)) {
                const cplx<double> b = comp(bo, Vh, s, sp, c);
                put(xo, Vh, s, sp, c, {b.re + a.kappa * acc[sp][c].re, b.im + a.kappa * acc[sp][c].im});
            }
}

// |b - M x|^2 on the sites of parity `par`, per block into slot `par` of
// buffer 0 (the solve is over when this runs)
template <int ROWS, int LPS, class LP> __global__ void __launch_bounds__(128) k_wil_resid(WArgs a, int par)
{
    __shared__ double lds[4];
    const int Vh = a.g.Vh;
    int s, sub;
    double nrm = 0.0;
    if (wsite<LPS>(Vh, a.remap, s, sub)) {
        const dbl2 *xin = a.x + (size_t)(1 - par) * 12 * Vh;
        cplx<double> acc[4][3];
        wilson_hop<ROWS, LPS, LP>(a.g, a.links[par], par, s, sub, acc,
                              [&](int n, int sp, int col) { return comp(xin, Vh, n, sp, col); });
        const dbl2 *bp = a.b + (size_t)par * 12 * Vh;
        const dbl2 *xp = a.x + (size_t)par * 12 * Vh;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (!owns_component<LPS>(sub, sp, c))
                    continue;
                const cplx<double> b = comp(bp, Vh, s, sp, c), x = comp(xp, Vh, s, sp, c);
                const double re = b.re - x.re + a.kappa * acc[sp][c].re;
                const double im = b.im - x.im + a.kappa * acc[sp][c].im;
                nrm += re * re + im * im;
            }
    }
    wpartial(a, 0, par, nrm, lds);
}

}  // namespace wil
}  // namespace stag
