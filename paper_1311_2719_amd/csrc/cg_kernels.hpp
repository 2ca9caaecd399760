// Fused conjugate-gradient kernels for (m^2 - D^2) x = b on one parity,
// batched over systems that share a gauge field.
//
// The iteration is the loop of the paper's Sec. 4 with the mass explicit,
// arranged as two kernels per step so that every vector is streamed once and
// every scalar stays on the device (large grids add a small reduction kernel
// after each, see below):
//   K1  prologue: reduce the previous step's partial sums and advance the
//       system's scalar state (beta, the stopping test, reliable-update
//       decisions); then, for a CG step, p' = r + beta p (formed on the fly at
//       every gathered neighbour and stored once at the partner site),
//       ap = D p' on the other parity, <ap,ap> and <p',p'>;
//   K2  prologue: alpha = rr / (m^2 <p',p'> + <ap,ap>) from K1's partials;
//       then Ap = m^2 p' - D ap; x += alpha p'; r -= alpha Ap; <r,r>
//       (Ap is never stored).
// A step of a system can instead be a residual recomputation in FP64
// (reliable update in mixed precision, the final true-residual check in every
// mode): K1 forms t = D (x_hi + x_lo) on the other parity, K2 forms
// x_hi += x_lo, x_lo = 0, r = b - m^2 x_hi + D t and <r,r>.
//
// Every block of a kernel derives the same scalars from the same partials
// (fixed summation order), so no block waits for another and no fence or
// atomic is used; the state advanced by K1 is written by one block into the
// other of two state buffers, which the following kernels read.  Partial sums
// alternate between two buffers the same way.  Each block of a prologue sums
// all per-block partials of the kernel before it, which costs blocks x
// partials reads; for large grids the host runs a small reduction kernel
// between the step kernels instead, which writes each slot's total to a
// separate array (CgArgs::psum, nread = 1), so that the step kernels can use
// as many blocks as the lattice needs.
//
// Systems: nsys = 2*S, system j has parity j / S (x, r, p on that parity; ap
// and t on the other).  A tile is R systems of one parity processed together
// so each link entry is loaded once for all of them; tiles take their systems
// from a per-parity list that the host compacts between epochs.  A system's
// partial sums depend only on the sites of each block, not on its tile, so
// compaction never changes results.
#pragma once

#include "hop.hpp"

namespace stag {

// What the step a state describes did (or, for INIT, what produced it).
enum Mode : int32_t { M_IDLE = 0, M_INIT = 1, M_CG = 2, M_RU = 3, M_DONE = 4 };

struct SysState {
    double mass2;
    double tol2;
    double stop2;    // tol^2 <b,b>
    double bb;
    double rr;       // <r,r> of the current (iterated) residual
    double pp;       // <p,p> of the last search direction
    double alpha;
    double beta;
    double maxr2;    // largest <r,r> since the last residual recomputation
    double delta2;   // reliable-update threshold squared (0: final check only)
    double true_rr;  // <r,r> of the last FP64 residual recomputation
    double pad0;
    int32_t mode;        // Mode
    int32_t stopping;    // status to report if the next recomputation does not converge
    int32_t status;      // final status (mode == M_DONE)
    int32_t iters;
    int32_t maxiter;
    int32_t n_ru;
    int32_t restarts;
    int32_t max_restarts;
    int32_t mixed;
    int32_t pcur;        // which of the two p buffers holds the current direction
    int32_t step;        // steps taken (the newer of the two state buffers has the larger value)
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
    SysState *st[2];           // [nsys] each: two state buffers
    const int *perm;           // [2][S] systems of each parity in tile order, -1 = none
    double *partials;          // [2 buffers][nsys][3 slots][pstride]
    int S;                     // systems per parity
    int pstride;
    int remap;
    // what a prologue sums: nread entries per slot at psum (stride psum_stride
    // between slots) -- the previous kernel's per-block partials (psum =
    // partials), or the totals a reduction kernel formed from them (nread = 1)
    const double *psum;
    int psum_stride;
    int nread;
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

// Partial sums: slot 0 <ap,ap>, slot 1 <p',p'>, slot 2 <r,r> (CG, residual
// recomputation or the source norm at initialisation).
__device__ __forceinline__ const double *psum_slot(const CgArgs &a, int buf, int j, int slot)
{
    const size_t nsys = 2 * (size_t)a.S;
    return a.psum + (((size_t)buf * nsys + j) * 3 + slot) * a.psum_stride;
}

__device__ __forceinline__ double *partial_slot(const CgArgs &a, int buf, int j, int slot)
{
    const size_t nsys = 2 * (size_t)a.S;
    return a.partials + (((size_t)buf * nsys + j) * 3 + slot) * a.pstride;
}

__device__ __forceinline__ bool finite_pos(double v) { return v > 0.0 && v < INFINITY; }

// ---- step prologue ------------------------------------------------------------------
// Every step kernel starts from the same few scalars per system: the state
// written by the previous kernel and the totals of its partial sums.  All of
// those loads are issued together, right after the tile's system list is read,
// so a prologue costs one memory round trip after that list: the states
// travel through LDS (16-byte vector loads, one thread per piece), the
// partial sums are loaded in unrolled groups before any of them is added.

// The tile's systems (-1 = empty place); false when the tile is empty.
template <int R> __device__ __forceinline__ bool tile_systems(const int *tile, int (&js)[R], bool (&valid)[R])
{
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = tile[r];
        valid[r] = j >= 0;
        js[r] = valid[r] ? j : 0;
        any |= valid[r];
    }
    return any;
}

constexpr int kStateVec = sizeof(SysState) / 16;
static_assert(sizeof(SysState) % 16 == 0, "state must be a whole number of 16-byte pieces");

// Per-thread strided sums of NS partial slots (slots 0 .. NS-1) of R systems:
// thread t adds entries t, t + blockDim, ... in increasing order, so the
// totals do not depend on the unroll depth.  The states of the R systems are
// loaded on the way and stored to `sst` once the sums' loads are in flight.
template <int R, int NS>
__device__ __forceinline__ void load_prologue(const CgArgs &a, int pbuf, const SysState *states, const int *tile,
                                              const int *js, const bool *valid, int nblk, SysState *sst,
                                              double (&v)[NS * R])
{
    constexpr int U = (NS * R >= 24) ? 1 : 24 / (NS * R);
    // states: kStateVec pieces per system, at most two pieces per thread (R * kStateVec <= 2 * 64)
    static_assert(R * kStateVec <= 128, "state staging assumes at most two pieces per thread");
    const int t0 = threadIdx.x, t1 = threadIdx.x + blockDim.x;
    const int n_pieces = R * kStateVec;
    uint4 q0{}, q1{};
    if (t0 < n_pieces) {
        const int j = tile[t0 / kStateVec];
        if (j >= 0)
            q0 = ((const uint4 *)(states + j))[t0 % kStateVec];
    }
    if (t1 < n_pieces) {
        const int j = tile[t1 / kStateVec];
        if (j >= 0)
            q1 = ((const uint4 *)(states + j))[t1 % kStateVec];
    }
    const double *base[NS * R];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < NS; ++k)
            base[r * NS + k] = psum_slot(a, pbuf, js[r], k);
#pragma unroll
    for (int k = 0; k < NS * R; ++k)
        v[k] = 0.0;
    for (int i0 = threadIdx.x; i0 < nblk; i0 += U * blockDim.x) {
        double buf[U][NS * R];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // every load is in bounds (index 0 past the end): the guard is a
            // select after the load, not a branch around it
            const int i = i0 + u * blockDim.x;
            const bool in = i < nblk;
#pragma unroll
            for (int k = 0; k < NS * R; ++k) {
                const double v = base[k][in ? i : 0];
                buf[u][k] = (in && valid[k / NS]) ? v : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < NS * R; ++k)
                v[k] += buf[u][k];
    }
    if (t0 < n_pieces)
        ((uint4 *)sst)[t0] = q0;
    if (t1 < n_pieces)
        ((uint4 *)sst)[t1] = q1;
}

// Values read from LDS that are the same in every lane, moved to scalar
// registers so that branches and addresses derived from them stay scalar.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uniform(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Wave sums of the per-thread sums into lds[k * nw + w]; after the barrier,
// thread r (< R) owns system r and reads its NS totals with wave_totals.
template <int N> __device__ __forceinline__ void wave_sums_to_lds(const double (&v)[N], double *lds)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double t = wave_sum(v[k]);
        if (lane == 0)
            lds[k * nw + w] = t;
    }
    __syncthreads();
}

__device__ __forceinline__ double wave_total(const double *lds, int k)
{
    const int nw = blockDim.x >> 6;
    double out = 0.0;
    for (int i = 0; i < nw; ++i)
        out += lds[k * nw + i];
    return out;
}

// Advance a system's state over the step whose partial sums are `t`.
__device__ __forceinline__ void advance(SysState &s, const double (&t)[3])
{
    s.step += 1;
    switch (s.mode) {
    case M_INIT: {
        const double bb = t[2];
        s.bb = bb;
        s.stop2 = s.tol2 * bb;
        s.rr = bb;
        s.pp = bb;
        s.maxr2 = bb;
        s.true_rr = bb;
        s.beta = 0.0;
        s.alpha = 0.0;
        s.pcur = 0;
        s.iters = 0;
        s.n_ru = 0;
        s.restarts = 0;
        s.stopping = 0;
        if (!(bb < INFINITY)) {
            s.mode = M_DONE;
            s.status = STAG_ENONFINITE;
        } else if (bb == 0.0) {
            s.mode = M_DONE;
            s.status = STAG_OK;
            s.true_rr = 0.0;
        } else {
            s.mode = M_CG;
        }
        break;
    }
    case M_CG: {
        s.pcur ^= 1;  // the previous K1 stored p' in the other buffer
        const double apap = t[0], pp = t[1];
        s.pp = pp;
        const double pap = s.mass2 * pp + apap;
        if (!finite_pos(pap)) {  // K2 skipped this system's update
            s.stopping = STAG_EBREAKDOWN;
            s.mode = M_RU;
            break;
        }
        s.alpha = s.rr / pap;
        const double rn = t[2];
        s.iters += 1;
        if (!(rn < INFINITY)) {
            s.stopping = STAG_EBREAKDOWN;
            s.mode = M_RU;
            break;
        }
        const bool conv = rn < s.stop2;
        s.maxr2 = rn > s.maxr2 ? rn : s.maxr2;
        bool recompute = conv || rn < s.delta2 * s.maxr2;
        if (!conv && s.iters >= s.maxiter) {
            s.stopping = STAG_ENOCONV;
            recompute = true;
        }
        if (recompute) {
            s.mode = M_RU;  // rr keeps the previous value as the denominator of beta
        } else {
            s.beta = rn / s.rr;
            s.rr = rn;
            s.mode = M_CG;
        }
        break;
    }
    case M_RU: {
        const double trr = t[2];
        s.n_ru += 1;
        s.true_rr = trr;
        if (trr <= s.stop2) {
            s.mode = M_DONE;
            s.status = STAG_OK;
        } else if (s.stopping) {
            s.mode = M_DONE;
            s.status = s.stopping;
        } else if (!s.mixed) {
            // FP64: the recursive residual claimed convergence but the true one
            // disagrees: restart CG from the current x (fresh search direction)
            s.restarts += 1;
            if (s.restarts > s.max_restarts) {
                s.mode = M_DONE;
                s.status = STAG_ENOCONV;
            } else {
                s.beta = 0.0;
                s.rr = trr;
                s.maxr2 = trr;
                s.mode = M_CG;
            }
        } else {
            // reliable update: keep the search direction, continue from the true residual
            s.beta = trr / s.rr;
            s.rr = trr;
            s.maxr2 = trr;
            s.mode = M_CG;
        }
        break;
    }
    default:
        break;
    }
}

// Directions per iteration of the rolled FP64 hop of a residual
// recomputation: two keeps the register budget of the single-site CG kernels
// while overlapping the loads of two directions.
constexpr int kRecomputeUnroll = 2;

// First site index handled by this thread in grid-stride round `it`.
__device__ __forceinline__ int64_t round_base(int it, int remap)
{
    return ((int64_t)it * gridDim.x + logical_block(blockIdx.x, gridDim.x, remap)) * blockDim.x + threadIdx.x;
}

// ---- own-site values of a step ------------------------------------------------------
// The values a step kernel reads at its own site (not gathered) are loaded
// in groups of G = 2 systems, all loads of a group before any use, so that a
// group costs one memory round trip instead of one per system (a store of
// one system cannot be passed by the next system's loads, which the compiler
// must assume may alias it).  With at most two systems per tile the single
// group is loaded before the hop, so its latency overlaps the gathers; larger
// tiles load each group after the hop, when the gathers' registers are free.
// Larger groups measured slower (the registers they hold lower occupancy).
template <class P, int R, int LPS> struct OwnSite {
    using real = typename P::real;
    using v2 = typename vec2_of<real>::type;
    using xv_t = typename std::conditional<P::id == 0, dbl2, flt2>::type;
    static constexpr bool kBeforeHop = R <= 2;
    static constexpr int G = R < 2 ? R : 2;  // systems per group
    v2 pr_[G][3], rr_[G][3];
    cplx<real> ps_[G][3];
    xv_t xx_[G][3];

    // K1: p (current buffer) and r of systems r0 .. r0 + G - 1 at the partner site
    template <class Args>
    __device__ __forceinline__ void load_k1(const Args &a, const int *js, const bool *cg, const int *pc, int s,
                                            int sub, int r0)
    {
        const int Vh = a.g.Vh;
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int r = r0 + q;
            if (r >= R || !cg[r])
                continue;
            const v2 *rv = (const v2 *)a.r + (size_t)js[r] * 3 * Vh;
            const void *pold = spin_at<P>(a.p[pc[r]], js[r], Vh);
            if constexpr (P::id == 2)
                P::load_spinor(pold, Vh, s, ps_[q]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (P::id != 2 && !owns_colour<LPS>(sub, c))
                    continue;
                rr_[q][c] = rv[(int64_t)c * Vh + s];
                if constexpr (P::id != 2)
                    pr_[q][c] = ((const v2 *)pold)[(int64_t)c * Vh + s];
            }
        }
    }
    // K2: p' (new buffer), x and r of systems r0 .. r0 + G - 1 at the own site.
    // x is read and written once per step, at its own site only: non-temporal
    // accesses keep it from evicting the gathered vectors (32^4 solves: FP16
    // +6%, FP32 +2%, FP64 unchanged; 16^4 within 1%).
    template <class Args>
    __device__ __forceinline__ void load_k2(const Args &a, const int *js, const bool *cg, const int *pn, int s,
                                            int sub, int r0)
    {
        const int Vh = a.g.Vh;
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int r = r0 + q;
            if (r >= R || !cg[r])
                continue;
            const int j = js[r];
            const void *pb = spin_at<P>(a.p[pn[r]], j, Vh);
            const v2 *rv = (const v2 *)a.r + (size_t)j * 3 * Vh;
            if constexpr (P::id == 2)
                P::load_spinor(pb, Vh, s, ps_[q]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (!owns_colour<LPS>(sub, c))
                    continue;
                const int64_t o = (int64_t)c * Vh + s;
                if constexpr (P::id != 2)
                    ps_[q][c] = load_colour<P>(pb, Vh, s, c);
                if constexpr (P::id == 0)
                    xx_[q][c] = __builtin_nontemporal_load(&a.xhi[j][o]);
                else
                    xx_[q][c] = __builtin_nontemporal_load(&a.xlo[(size_t)j * 3 * Vh + o]);
                rr_[q][c] = rv[o];
            }
        }
    }
};

// ---- residual recomputation (FP64), one system at one site --------------------------
// The reliable update of mixed precision and the final true-residual check.
// K1 side: t = D (x_hi + x_lo) on the other parity.
template <int LPS, int ROWS, int UNROLL = kRecomputeUnroll>
__device__ __forceinline__ void recompute_k1(const CgArgs &a, int j, int pout, int s, int sub)
{
    const int Vh = a.g.Vh;
    const dbl2 *xh = a.xhi[j];
    const flt2 *xl = a.xlo ? a.xlo + (size_t)j * 3 * Vh : nullptr;
    cplx<double> acc[1][3] = {{czero<double>(), czero<double>(), czero<double>()}};
    auto load = [&](int, int n, cplx<double> *chi) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            dbl2 v = xh[(int64_t)c * Vh + n];
            if (xl) {
                const flt2 w = xl[(int64_t)c * Vh + n];
                v.x += (double)w.x;
                v.y += (double)w.y;
            }
            chi[c] = {v.x, v.y};
        }
    };
    hop_accumulate<PrecF64, LPS, 1, decltype(load), true, ROWS, UNROLL>(a.g, a.links64[pout], a.nbr[pout],
                                                                                  pout, s, sub, acc, load);
    dbl2 *t = a.tmp + (size_t)j * 3 * Vh;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        if (owns_colour<LPS>(sub, c))
            t[(int64_t)c * Vh + s] = dbl2{acc[0][c].re, acc[0][c].im};
}

// K2 side: x_hi += x_lo, x_lo = 0, r = b - m^2 x_hi + D t; this lane's
// terms of <r,r> are added to nrm.
template <class P, int LPS, int ROWS, int UNROLL = kRecomputeUnroll>
__device__ __forceinline__ void recompute_k2(const CgArgs &a, int j, int par, int s, int sub, double m2d, double &nrm)
{
    using real = typename P::real;
    using v2 = typename vec2_of<real>::type;
    const int Vh = a.g.Vh;
    const dbl2 *t = a.tmp + (size_t)j * 3 * Vh;
    cplx<double> acc[1][3] = {{czero<double>(), czero<double>(), czero<double>()}};
    auto load = [&](int, int n, cplx<double> *chi) { PrecF64::load_spinor(t, Vh, n, chi); };
    hop_accumulate<PrecF64, LPS, 1, decltype(load), true, ROWS, UNROLL>(a.g, a.links64[par], a.nbr[par], par,
                                                                                  s, sub, acc, load);
    dbl2 *x = a.xhi[j];
    const dbl2 *b = a.b[j];
    v2 *rv = (v2 *)a.r + (size_t)j * 3 * Vh;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (!owns_colour<LPS>(sub, c))
            continue;
        const int64_t o = (int64_t)c * Vh + s;
        dbl2 xv = x[o];
        if constexpr (P::id != 0) {
            const flt2 w = a.xlo[(size_t)j * 3 * Vh + o];
            xv.x += (double)w.x;
            xv.y += (double)w.y;
            x[o] = xv;
            a.xlo[(size_t)j * 3 * Vh + o] = flt2{0.f, 0.f};
        }
        const dbl2 bv = b[o];
        const double rre = bv.x - m2d * xv.x + acc[0][c].re;
        const double rim = bv.y - m2d * xv.y + acc[0][c].im;
        rv[o] = v2{(real)rre, (real)rim};
        nrm += rre * rre + rim * rim;
    }
}

// ---- K1 -----------------------------------------------------------------------------

template <class P, int LPS, int R, int ROWS>
__global__ void __launch_bounds__(256) k_cg_step1(CgArgs a, int ver)
{
    using real = typename P::real;
    using v2 = typename vec2_of<real>::type;
    __shared__ double lds[3 * R * 4];
    const int tpp = a.S / R;
    const int par = blockIdx.y / tpp, k0 = par * a.S + (blockIdx.y % tpp) * R, pout = 1 - par;
    const int Vh = a.g.Vh;
    int js[R];
    bool valid[R];
    if (!tile_systems<R>(a.perm + k0, js, valid))
        return;
    // the previous step's totals and states; thread r (< R) advances system r
    __shared__ SysState sst[R];
    {
        double v[3 * R];
        load_prologue<R, 3>(a, ver, a.st[ver], a.perm + k0, js, valid, a.nread, sst, v);
        wave_sums_to_lds<3 * R>(v, lds);
        const int r = threadIdx.x;
        if (r < R) {
            const int j = a.perm[k0 + r];
            SysState st = sst[r];
            const bool live = j >= 0 && st.mode != M_IDLE && st.mode != M_DONE;
            if (live) {
                const double tot[3] = {wave_total(lds, 3 * r), wave_total(lds, 3 * r + 1), wave_total(lds, 3 * r + 2)};
                advance(st, tot);
            }
            // the state K2 of this step reads: advanced, or the same idle/done
            // state (never the stale one of two kernels ago)
            if (j >= 0 && blockIdx.x == 0)
                a.st[ver ^ 1][j] = st;
            if (!live)
                st.mode = M_IDLE;  // not running: nothing to do in this step
            sst[r] = st;
        }
        __syncthreads();
    }
    bool cg[R], ru[R];
    real beta[R];
    int pc[R];
    bool anycg = false, anyru = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int mode = valid[r] ? uniform(sst[r].mode) : (int)M_IDLE;
        cg[r] = mode == M_CG;
        ru[r] = mode == M_RU;
        beta[r] = (real)uniform(sst[r].beta);
        pc[r] = uniform(sst[r].pcur);
        anycg |= cg[r];
        anyru |= ru[r];
    }
    if (!anycg && !anyru)
        return;
    double nrm[2 * R];
#pragma unroll
    for (int r = 0; r < 2 * R; ++r)
        nrm[r] = 0.0;
    const int64_t nthreads = (int64_t)Vh * LPS;
    if (anycg) {
        for (int it = 0;; ++it) {
            const int64_t gt = round_base(it, a.remap);
            if (gt - threadIdx.x >= nthreads)
                break;
            int s, sub;
            site_of_thread<LPS>((int)gt, s, sub);
            if (s >= Vh)
                continue;
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
            // the partner site's p and r (same index, parity par)
            using Own = OwnSite<P, R, LPS>;
            Own own;
            if constexpr (Own::kBeforeHop)
                own.load_k1(a, js, cg, pc, s, sub, 0);
            hop_accumulate<P, LPS, R, decltype(load), false, ROWS>(a.g, (const typename P::link_t *)a.links[pout],
                                                                   a.nbr[pout], pout, s, sub, acc, load);
#pragma unroll
            for (int g = 0; g < R; g += Own::G) {
                if constexpr (!Own::kBeforeHop)
                    own.load_k1(a, js, cg, pc, s, sub, g);
#pragma unroll
                for (int q = 0; q < Own::G; ++q) {
                    const int r = g + q;
                    if (r >= R || !cg[r])
                        continue;
                    const int j = js[r];
                    void *out = spin_at<P>(a.ap, j, Vh);
                    void *pnew = spin_at<P>(a.p[pc[r] ^ 1], j, Vh);
                    if constexpr (P::id == 2) {
                        if (sub == 0) {
                            P::store_spinor(out, Vh, s, acc[r]);
                            // the new direction at the partner site (same index, parity par)
                            cplx<real> pv[3];
#pragma unroll
                            for (int c = 0; c < 3; ++c) {
                                const v2 t = own.rr_[q][c];
                                pv[c].re = fma(beta[r], own.ps_[q][c].re, t.x);
                                pv[c].im = fma(beta[r], own.ps_[q][c].im, t.y);
                            }
                            P::store_spinor_read_back(pnew, Vh, s, pv);  // pv: the value D will read
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
                            const v2 po = own.pr_[q][c], t = own.rr_[q][c];
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
        }
    }
    if (anyru) {
        for (int it = 0;; ++it) {
            const int64_t gt = round_base(it, a.remap);
            if (gt - threadIdx.x >= nthreads)
                break;
            int s, sub;
            site_of_thread<LPS>((int)gt, s, sub);
            if (s >= Vh)
                continue;
            // residual recomputation in FP64, one system at a time
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (ru[r])
                    recompute_k1<LPS, ROWS>(a, js[r], pout, s, sub);
        }
    }
    if (!anycg)
        return;
    double tot2;
    block_sum_multi<2 * R>(nrm, lds, tot2);
    if (threadIdx.x < 2 * R) {
        const int r = (int)threadIdx.x % R;
        const int j = a.perm[k0 + r];
        if (j >= 0)
            partial_slot(a, ver ^ 1, j, (int)threadIdx.x / R)[blockIdx.x] = tot2;
    }
}

// ---- K2 -----------------------------------------------------------------------------

template <class P, int LPS, int R, int ROWS>
__global__ void __launch_bounds__(256) k_cg_step2(CgArgs a, int ver)
{
    using real = typename P::real;
    using v2 = typename vec2_of<real>::type;
    __shared__ double lds[3 * R * 4];
    const int tpp = a.S / R;
    const int par = blockIdx.y / tpp, k0 = par * a.S + (blockIdx.y % tpp) * R;
    const int Vh = a.g.Vh;
    const int cur = ver ^ 1;  // the state K1 of this step wrote
    int js[R];
    bool valid[R];
    if (!tile_systems<R>(a.perm + k0, js, valid))
        return;
    // alpha from K1's partial sums (slots 0 and 1); thread r (< R) decides for system r
    __shared__ SysState sst[R];
    {
        double v[2 * R];
        load_prologue<R, 2>(a, cur, a.st[cur], a.perm + k0, js, valid, a.nread, sst, v);
        wave_sums_to_lds<2 * R>(v, lds);
        const int r = threadIdx.x;
        if (r < R) {
            const int j = a.perm[k0 + r];
            SysState st = sst[r];
            int mode = M_IDLE;
            double alpha = 0.0;
            if (j >= 0 && st.mode == M_CG) {
                const double pap = st.mass2 * wave_total(lds, 2 * r + 1) + wave_total(lds, 2 * r);
                if (finite_pos(pap)) {  // otherwise K1 of the next step reports the breakdown
                    mode = M_CG;
                    alpha = st.rr / pap;
                }
            } else if (j >= 0 && st.mode == M_RU) {
                mode = M_RU;
            }
            sst[r].mode = mode;
            sst[r].alpha = alpha;
        }
        __syncthreads();
    }
    bool cg[R], ru[R];
    real alpha[R], m2[R];
    int pnew[R];
    bool anycg = false, anyru = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int mode = valid[r] ? uniform(sst[r].mode) : (int)M_IDLE;
        cg[r] = mode == M_CG;
        ru[r] = mode == M_RU;
        alpha[r] = (real)uniform(sst[r].alpha);
        m2[r] = (real)uniform(sst[r].mass2);
        pnew[r] = uniform(sst[r].pcur) ^ 1;  // p' written by K1 of this step
        anycg |= cg[r];
        anyru |= ru[r];
    }
    if (!anycg && !anyru)
        return;
    double nrm[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        nrm[r] = 0.0;
    const int64_t nthreads = (int64_t)Vh * LPS;
    if (anycg) {
        for (int it = 0;; ++it) {
            const int64_t gt = round_base(it, a.remap);
            if (gt - threadIdx.x >= nthreads)
                break;
            int s, sub;
            site_of_thread<LPS>((int)gt, s, sub);
            if (s >= Vh)
                continue;
            cplx<real> acc[R][3];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    acc[r][c] = czero<real>();
            auto load = [&](int r, int n, cplx<real> *chi) {
                P::load_spinor(spin_at<P>(a.ap, js[r], Vh), Vh, n, chi);
            };
            // this site's p', x and r
            using Own = OwnSite<P, R, LPS>;
            Own own;
            if constexpr (Own::kBeforeHop)
                own.load_k2(a, js, cg, pnew, s, sub, 0);
            hop_accumulate<P, LPS, R, decltype(load), false, ROWS>(a.g, (const typename P::link_t *)a.links[par],
                                                                   a.nbr[par], par, s, sub, acc, load);
#pragma unroll
            for (int g = 0; g < R; g += Own::G) {
                if constexpr (!Own::kBeforeHop)
                    own.load_k2(a, js, cg, pnew, s, sub, g);
#pragma unroll
                for (int q = 0; q < Own::G; ++q) {
                    const int r = g + q;
                    if (r >= R || !cg[r])
                        continue;
                    const int j = js[r];
                    v2 *rv = (v2 *)a.r + (size_t)j * 3 * Vh;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        if (!owns_colour<LPS>(sub, c))
                            continue;
                        const cplx<real> pv = own.ps_[q][c];
                        const int64_t o = (int64_t)c * Vh + s;
                        if constexpr (P::id == 0) {
                            const dbl2 xv = own.xx_[q][c];
                            __builtin_nontemporal_store(dbl2{fma(alpha[r], pv.re, xv.x), fma(alpha[r], pv.im, xv.y)},
                                                        &a.xhi[j][o]);
                        } else {
                            const flt2 xv = own.xx_[q][c];
                            __builtin_nontemporal_store(flt2{fmaf(alpha[r], pv.re, xv.x), fmaf(alpha[r], pv.im, xv.y)},
                                                        &a.xlo[(size_t)j * 3 * Vh + o]);
                        }
                        const real apr = m2[r] * pv.re - acc[r][c].re;
                        const real api = m2[r] * pv.im - acc[r][c].im;
                        v2 rr = own.rr_[q][c];
                        rr.x = fma(-alpha[r], apr, rr.x);
                        rr.y = fma(-alpha[r], api, rr.y);
                        rv[o] = rr;
                        nrm[r] += (double)rr.x * rr.x + (double)rr.y * rr.y;
                    }
                }
            }
        }
    }
    if (anyru) {
        for (int it = 0;; ++it) {
            const int64_t gt = round_base(it, a.remap);
            if (gt - threadIdx.x >= nthreads)
                break;
            int s, sub;
            site_of_thread<LPS>((int)gt, s, sub);
            if (s >= Vh)
                continue;
            // residual recomputation in FP64, one system at a time
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (ru[r])
                    recompute_k2<P, LPS, ROWS>(a, js[r], par, s, sub, uniform(sst[r].mass2), nrm[r]);
        }
    }
    double tot2;
    block_sum_multi<R>(nrm, lds, tot2);
    if (threadIdx.x < R) {
        const int j = a.perm[k0 + (int)threadIdx.x];
        if (j >= 0)
            partial_slot(a, cur, j, 2)[blockIdx.x] = tot2;
    }
}

// ---- initialisation: x = 0, r = b, p = r; <b,b> into slot 2 of buffer 0 -------------
// Same grid shape as the step kernels (so the same number of partials), one
// grid row per system; systems in mode M_INIT only.

template <class P>
__global__ void __launch_bounds__(256) k_cg_init(CgArgs a, int lps)
{
    using real = typename P::real;
    using v2 = typename vec2_of<real>::type;
    __shared__ double lds[4];
    const int j = blockIdx.y;
    if (a.st[0][j].mode != M_INIT)
        return;
    const int Vh = a.g.Vh;
    double nrm[1] = {0.0};
    // one thread per site; the grid covers Vh * lps threads per round like the step kernels
    const int64_t nthreads = (int64_t)Vh * lps;
    for (int it = 0;; ++it) {
        const int64_t gt = round_base(it, a.remap);
        if (gt - threadIdx.x >= nthreads)
            break;
        if (gt % lps)
            continue;
        const int s = (int)(gt / lps);
        if (s >= Vh)
            continue;
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
        partial_slot(a, 0, j, 2)[blockIdx.x] = tot;
}

// ---- tuning probe: out_r = D in_r for R systems, no reductions -------------------
// blockIdx.y = tile; tiles alternate output parity like the CG kernels' tiles.

template <class P, int LPS, int R, int ROWS>
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
    cplx<real> acc[R][3];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            acc[r][c] = czero<real>();
    auto load = [&](int r, int n, cplx<real> *chi) { P::load_spinor(inb + r * vb, Vh, n, chi); };
    const typename P::link_t *lk = (const typename P::link_t *)links + link_parity_entries(ROWS, Vh) * pout;
    hop_accumulate<P, LPS, R, decltype(load), false, ROWS>(g, lk, nbr ? nbr + (size_t)pout * 8 * Vh : nullptr, pout, s,
                                                           sub, acc, load);
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
