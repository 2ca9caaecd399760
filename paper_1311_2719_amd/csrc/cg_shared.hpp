// CG step kernels for FP32 and FP16 working precision in which the systems
// of a tile share every link read through LDS.
//
// The register tiles of cg_kernels.hpp share a link load between the R
// systems one thread carries, so their per-thread state grows with R and the
// tuner settles on R = 2 or 3 at 24^4: every link is then read from HBM
// S / R times per kernel.  Here a block is W wavefronts, each running RR
// systems of the block's tile (R = W RR) on 64 consecutive output sites, one
// lane per site.  The block first reads the links of those 64 sites (8
// directions, stored rows), rebuilds row 2 where only two are stored,
// converts them to FP32 and keeps all nine entries in LDS; every wavefront
// then runs the hop of its RR systems with the links taken from there.  A
// link thus costs one HBM read per R systems (R up to 16: one tile per parity
// at 12 or 16 systems), the third row and the FP16 conversion are computed
// once per block instead of once per thread, and a wavefront holds the
// registers of RR systems only.
//
// The step arithmetic is that of k_cg_step1 / k_cg_step2 (the loop of the
// paper's Sec. 4 with the mass explicit): same products, same storage
// formats, same state machine (advance()); only the summation order of the
// partial sums differs (each system's sums stay in one wavefront: lane sums
// over the chunks a block visits, then the wavefront sum).
//
// LDS layout of one chunk: [entry 9][dir 8][site 64 + 8] of FP32 complex.  A
// wavefront reading one (entry, dir) for its 64 sites touches 512 contiguous
// bytes; the 8 padding entries per row put the eight directions of one
// staging store in different banks.
#pragma once

#include "cg_kernels.hpp"

namespace stag {

constexpr int kChunk = 64;              // output sites per block and round
constexpr int kLdsRow = kChunk + 8;     // padded row of one (entry, dir)
constexpr int kSharedMaxR = 16;         // systems per tile
// Directions of the hop whose gathers a wavefront keeps in flight together,
// and the wavefronts per SIMD the register allocation must allow.  A fully
// unrolled hop holds the gathers of all eight directions (about 130 VGPRs);
// occupancy, not unrolling, hides the gather latency here.  The residual
// recomputation (FP64, rare) runs its direction loop rolled so that it does
// not set the kernel's register budget.
constexpr int kSharedDirUnroll = 2;
constexpr int kSharedMinWaves = 1;

__device__ __forceinline__ int chunk_link_index(int k, int d, int i) { return (k * 8 + d) * kLdsRow + i; }

// Stage the links of output sites [s0, s0 + 64) (parity p_out) into lk.
// Consecutive threads take consecutive stored entries (site tile, direction,
// site), so every global load of a wavefront reads 512 contiguous bytes.  A
// block reads its links once: non-temporal loads leave the L2 to the
// gathered vectors (24^4, 12 systems per parity: 2% per step).
template <class P, int ROWS>
__device__ __forceinline__ void stage_chunk_links(const Geom &g, const typename P::link_t *__restrict__ links,
                                                  int p_out, int s0, flt2 *lk)
{
    const int Vh = g.Vh;
    const int n = (Vh - s0 >= kChunk ? kChunk : Vh - s0) * 8;  // Vh - s0 is a multiple of 8
    const typename P::link_t *base = links + (int64_t)(s0 >> 3) * 64;
    for (int it = threadIdx.x; it < n; it += blockDim.x) {
        const int d = (it >> 3) & 7;
        const int i = (it >> 6) * 8 + (it & 7);
        cplx<float> U[9];
#pragma unroll
        for (int k = 0; k < 3 * ROWS; ++k) {
            const auto v = __builtin_nontemporal_load(base + (int64_t)k * 8 * Vh + it);
            U[k] = {(float)v.x, (float)v.y};
        }
        if constexpr (ROWS == 2) {
            const SiteCoord c = decode_site(g, p_out, s0 + i);
            third_row(U, folded_negative(g, c, d) ? -2.f : 2.f);
        }
#pragma unroll
        for (int k = 0; k < 9; ++k)
            lk[chunk_link_index(k, d, i)] = flt2{U[k].re, U[k].im};
    }
}

// acc[q][a] += sum_d L_d(s)[a][b] chi_qd[b] for the RR systems of a
// wavefront, the links from the staged chunk (lane i = site s0 + i),
// load(q, n, chi) the input of system q at neighbour n.
template <bool TABLES, int RR, class Load>
__device__ __forceinline__ void hop_shared_impl(const Geom &g, const int32_t *__restrict__ nbr, int p_out, int s,
                                                int i, const flt2 *lk, cplx<float> (&acc)[RR][3], Load load)
{
    SiteCoord c;
    if constexpr (!TABLES)
        c = decode_site(g, p_out, s);
#pragma unroll kSharedDirUnroll
    for (int d = 0; d < 8; ++d) {
        int n;
        if constexpr (TABLES)
            n = nbr[(int64_t)d * g.Vh + s];
        else
            n = neighbour(g, c, s, d);
        cplx<float> chi[RR][3];
#pragma unroll
        for (int q = 0; q < RR; ++q)
            load(q, n, chi[q]);
        cplx<float> U[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const flt2 v = lk[chunk_link_index(k, d, i)];
            U[k] = {v.x, v.y};
        }
#pragma unroll
        for (int q = 0; q < RR; ++q)
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    cmac(acc[q][a], U[a * 3 + b], chi[q][b]);
    }
}

template <int RR, class Load>
__device__ __forceinline__ void hop_shared(const Geom &g, const int32_t *nbr, int p_out, int s, int i, const flt2 *lk,
                                           cplx<float> (&acc)[RR][3], Load load)
{
    if (nbr)
        hop_shared_impl<true, RR>(g, nbr, p_out, s, i, lk, acc, load);
    else
        hop_shared_impl<false, RR>(g, nbr, p_out, s, i, lk, acc, load);
}

// Totals of slots [0, NS) of system j's partial sums (the previous kernel's
// per-block sums, or the reduction kernel's totals), formed by one wavefront:
// lane l adds entries l, l + 64, ... in order, then the wavefront sum.
template <int NS> __device__ __forceinline__ void wave_prologue_sums(const CgArgs &a, int buf, int j, double (&t)[NS])
{
    const int lane = threadIdx.x & 63;
    double v[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k)
        v[k] = 0.0;
    for (int i = lane; i < a.nread; i += 64)
#pragma unroll
        for (int k = 0; k < NS; ++k)
            v[k] += psum_slot(a, buf, j, k)[i];
#pragma unroll
    for (int k = 0; k < NS; ++k)
        t[k] = wave_sum(v[k]);
}

// First site of the chunk a block takes in round `it`, or -1 past the end.
__device__ __forceinline__ int chunk_start(int it, int Vh, int remap)
{
    const int64_t ch = (int64_t)it * gridDim.x + logical_block(blockIdx.x, gridDim.x, remap);
    const int64_t s0 = ch * kChunk;
    return s0 < Vh ? (int)s0 : -1;
}

// ---- K1 -----------------------------------------------------------------------------
// A block of W wavefronts runs a tile of R = W RR systems; wavefront w takes
// places w RR .. w RR + RR - 1.  Like the register tiles, a wavefront gathers
// for each of its places, also places whose system is not in a CG step (their
// sums are discarded), so that the direction loop has no per-system branch.

template <class P, int W, int RR, int ROWS>
__global__ void __launch_bounds__(64 * W, kSharedMinWaves) k_cg_shared1(CgArgs a, int ver)
{
    constexpr int R = W * RR;
    static_assert(P::id != 0 && R <= kSharedMaxR, "shared-link tiles: FP32 / FP16 working precision");
    using real = typename P::real;
    using v2 = typename vec2_of<real>::type;
    __shared__ flt2 lk[9 * 8 * kLdsRow];
    __shared__ int modes[R];
    const int tpp = a.S / R;
    const int par = blockIdx.y / tpp, k0 = par * a.S + (blockIdx.y % tpp) * R, pout = 1 - par;
    const int Vh = a.g.Vh;
    // the wavefront index is the same in every lane: kept in a scalar register,
    // so that its systems, their states and pointers stay scalar too
    const int w = uniform((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    // prologue: this wavefront advances its own systems over the previous step
    int js[RR];
    bool cg[RR], ru[RR];
    real beta[RR];
    int pc[RR];
#pragma unroll
    for (int q = 0; q < RR; ++q) {
        const int j = a.perm[k0 + w * RR + q];
        int mode = M_IDLE, p = 0;
        double b = 0.0;
        if (j >= 0) {
            double t[3];
            wave_prologue_sums<3>(a, ver, j, t);
            SysState st = a.st[ver][j];
            const bool live = st.mode != M_IDLE && st.mode != M_DONE;
            if (live)
                advance(st, t);
            // the state K2 of this step reads: advanced, or the same idle/done state
            if (blockIdx.x == 0 && lane == 0)
                a.st[ver ^ 1][j] = st;
            mode = live ? uniform(st.mode) : (int)M_IDLE;
            b = uniform(st.beta);
            p = uniform(st.pcur);
        }
        js[q] = j;
        cg[q] = mode == M_CG;
        ru[q] = mode == M_RU;
        beta[q] = (real)b;
        pc[q] = p;
        if (lane == 0)
            modes[w * RR + q] = mode;
    }
    __syncthreads();
    bool anycg = false, anyru = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        anycg |= modes[r] == M_CG;
        anyru |= modes[r] == M_RU;
    }
    if (!anycg && !anyru)
        return;
    bool wcg = false;
#pragma unroll
    for (int q = 0; q < RR; ++q)
        wcg |= cg[q];
    // every place gathers in bounds: an empty place reads system 0's vectors
    const v2 *rv[RR];
    const void *pold[RR];
#pragma unroll
    for (int q = 0; q < RR; ++q) {
        const int jj = js[q] >= 0 ? js[q] : 0;
        rv[q] = (const v2 *)a.r + (size_t)jj * 3 * Vh;
        pold[q] = spin_at<P>(a.p[pc[q]], jj, Vh);
    }
    double nrm_ap[RR], nrm_p[RR];
#pragma unroll
    for (int q = 0; q < RR; ++q)
        nrm_ap[q] = nrm_p[q] = 0.0;
    for (int it = 0;; ++it) {
        const int s0 = chunk_start(it, Vh, a.remap);
        if (s0 < 0)
            break;
        if (anycg) {
            if (it > 0)
                __syncthreads();  // every wavefront is done with the previous chunk's links
            stage_chunk_links<P, ROWS>(a.g, (const typename P::link_t *)a.links[pout], pout, s0, lk);
            __syncthreads();
        }
        const int s = s0 + lane;
        if (s >= Vh)
            continue;
        if (wcg) {
            cplx<float> acc[RR][3];
#pragma unroll
            for (int q = 0; q < RR; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    acc[q][c] = czero<float>();
            // the partner site's p and r (same index, parity par): before the
            // gathers for a single system, after them for several
            cplx<real> po[RR][3];
            v2 ro[RR][3];
            auto own = [&]() {
#pragma unroll
                for (int q = 0; q < RR; ++q) {
                    P::load_spinor(pold[q], Vh, s, po[q]);
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        ro[q][c] = rv[q][(int64_t)c * Vh + s];
                }
            };
            if constexpr (RR == 1)
                own();
            auto load = [&](int q, int n, cplx<float> *chi) {
                cplx<real> pv[3];
                P::load_spinor(pold[q], Vh, n, pv);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const v2 t = rv[q][(int64_t)c * Vh + n];
                    chi[c].re = fma(beta[q], pv[c].re, t.x);
                    chi[c].im = fma(beta[q], pv[c].im, t.y);
                }
            };
            hop_shared<RR>(a.g, a.nbr[pout], pout, s, lane, lk, acc, load);
            if constexpr (RR > 1)
                own();
#pragma unroll
            for (int q = 0; q < RR; ++q) {
                if (!cg[q])
                    continue;
                const int j = js[q];
                cplx<real> pn[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    pn[c].re = fma(beta[q], po[q][c].re, ro[q][c].x);
                    pn[c].im = fma(beta[q], po[q][c].im, ro[q][c].y);
                }
                P::store_spinor(spin_at<P>(a.ap, j, Vh), Vh, s, acc[q]);
                void *pnew = spin_at<P>(a.p[pc[q] ^ 1], j, Vh);
                if constexpr (P::id == 2)
                    P::store_spinor_read_back(pnew, Vh, s, pn);  // pn: the value D will read
                else
                    P::store_spinor(pnew, Vh, s, pn);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    nrm_p[q] += (double)pn[c].re * pn[c].re + (double)pn[c].im * pn[c].im;
                    nrm_ap[q] += (double)acc[q][c].re * acc[q][c].re + (double)acc[q][c].im * acc[q][c].im;
                }
            }
        }
    }
    // residual recomputations (FP64, rare) after the CG work, by the whole
    // block: eight lanes per site, one direction each
    for (int r = 0; anyru && r < R; ++r) {
        if (modes[r] != M_RU)
            continue;
        const int j = a.perm[k0 + r];
        for (int it = 0;; ++it) {
            const int s0 = chunk_start(it, Vh, a.remap);
            if (s0 < 0)
                break;
            for (int t = threadIdx.x; t < kChunk * 8; t += blockDim.x) {  // whole wavefronts
                int sl, sub;
                site_of_thread<8>(t, sl, sub);
                if (s0 + sl < Vh)
                    recompute_k1<8, ROWS, 1>(a, j, pout, s0 + sl, sub);
            }
        }
    }
    if (!anycg)
        return;
#pragma unroll
    for (int q = 0; q < RR; ++q) {
        if (js[q] < 0)
            continue;
        const double tap = wave_sum(nrm_ap[q]), tpp2 = wave_sum(nrm_p[q]);
        if (lane == 0) {
            partial_slot(a, ver ^ 1, js[q], 0)[blockIdx.x] = tap;
            partial_slot(a, ver ^ 1, js[q], 1)[blockIdx.x] = tpp2;
        }
    }
}

// ---- K2 -----------------------------------------------------------------------------

template <class P, int W, int RR, int ROWS>
__global__ void __launch_bounds__(64 * W, kSharedMinWaves) k_cg_shared2(CgArgs a, int ver)
{
    constexpr int R = W * RR;
    static_assert(P::id != 0 && R <= kSharedMaxR, "shared-link tiles: FP32 / FP16 working precision");
    using real = typename P::real;
    using v2 = typename vec2_of<real>::type;
    __shared__ flt2 lk[9 * 8 * kLdsRow];
    __shared__ int modes[R];
    __shared__ double red[W];
    const int tpp = a.S / R;
    const int par = blockIdx.y / tpp, k0 = par * a.S + (blockIdx.y % tpp) * R;
    const int Vh = a.g.Vh;
    const int cur = ver ^ 1;  // the state K1 of this step wrote
    // the wavefront index is the same in every lane: kept in a scalar register,
    // so that its systems, their states and pointers stay scalar too
    const int w = uniform((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    // alpha from K1's partial sums (slots 0 and 1)
    int js[RR], pn_buf[RR];
    bool cg[RR], ru[RR];
    real al[RR], m2r[RR];
    double m2[RR];
#pragma unroll
    for (int q = 0; q < RR; ++q) {
        const int j = a.perm[k0 + w * RR + q];
        int mode = M_IDLE, pb = 0;
        double alpha = 0.0, mass2 = 0.0;
        if (j >= 0) {
            const SysState &st = a.st[cur][j];
            const int smode = st.mode;
            const double rr = st.rr;
            const int pcur = st.pcur;
            mass2 = st.mass2;
            double t[2];
            wave_prologue_sums<2>(a, cur, j, t);
            if (smode == M_CG) {
                const double pap = mass2 * t[1] + t[0];
                if (finite_pos(pap)) {  // otherwise K1 of the next step reports the breakdown
                    mode = M_CG;
                    alpha = rr / pap;
                }
            } else if (smode == M_RU) {
                mode = M_RU;
            }
            mode = uniform(mode);
            alpha = uniform(alpha);
            mass2 = uniform(mass2);
            pb = uniform(pcur) ^ 1;  // p' written by K1 of this step
        }
        js[q] = j;
        cg[q] = mode == M_CG;
        ru[q] = mode == M_RU;
        al[q] = (real)alpha;
        m2[q] = mass2;
        m2r[q] = (real)mass2;
        pn_buf[q] = pb;
        if (lane == 0)
            modes[w * RR + q] = mode;
    }
    __syncthreads();
    bool anycg = false, anyru = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        anycg |= modes[r] == M_CG;
        anyru |= modes[r] == M_RU;
    }
    if (!anycg && !anyru)
        return;
    bool wcg = false;
#pragma unroll
    for (int q = 0; q < RR; ++q)
        wcg |= cg[q];
    const void *apv[RR];
#pragma unroll
    for (int q = 0; q < RR; ++q)
        apv[q] = spin_at<P>(a.ap, js[q] >= 0 ? js[q] : 0, Vh);
    double nrm[RR];
#pragma unroll
    for (int q = 0; q < RR; ++q)
        nrm[q] = 0.0;
    for (int it = 0;; ++it) {
        const int s0 = chunk_start(it, Vh, a.remap);
        if (s0 < 0)
            break;
        if (anycg) {
            if (it > 0)
                __syncthreads();
            stage_chunk_links<P, ROWS>(a.g, (const typename P::link_t *)a.links[par], par, s0, lk);
            __syncthreads();
        }
        const int s = s0 + lane;
        if (s >= Vh)
            continue;
        if (wcg) {
            // this site's p', x and r: before the gathers for a single system,
            // after them for several
            cplx<real> pv[RR][3];
            flt2 xv[RR][3];
            v2 ro[RR][3];
            auto own = [&]() {
#pragma unroll
                for (int q = 0; q < RR; ++q) {
                    if (!cg[q])
                        continue;
                    const int j = js[q];
                    P::load_spinor(spin_at<P>(a.p[pn_buf[q]], j, Vh), Vh, s, pv[q]);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        xv[q][c] = a.xlo[(size_t)j * 3 * Vh + (int64_t)c * Vh + s];
                        ro[q][c] = ((const v2 *)a.r)[(size_t)j * 3 * Vh + (int64_t)c * Vh + s];
                    }
                }
            };
            if constexpr (RR == 1)
                own();
            cplx<float> acc[RR][3];
#pragma unroll
            for (int q = 0; q < RR; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    acc[q][c] = czero<float>();
            auto load = [&](int q, int n, cplx<float> *chi) { P::load_spinor(apv[q], Vh, n, chi); };
            hop_shared<RR>(a.g, a.nbr[par], par, s, lane, lk, acc, load);
            if constexpr (RR > 1)
                own();
#pragma unroll
            for (int q = 0; q < RR; ++q) {
                if (!cg[q])
                    continue;
                const int j = js[q];
                v2 *rv = (v2 *)a.r + (size_t)j * 3 * Vh;
                flt2 *xl = a.xlo + (size_t)j * 3 * Vh;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int64_t o = (int64_t)c * Vh + s;
                    xl[o] = flt2{fmaf(al[q], pv[q][c].re, xv[q][c].x), fmaf(al[q], pv[q][c].im, xv[q][c].y)};
                    const real apr = m2r[q] * pv[q][c].re - acc[q][c].re;
                    const real api = m2r[q] * pv[q][c].im - acc[q][c].im;
                    v2 rn = ro[q][c];
                    rn.x = fma(-al[q], apr, rn.x);
                    rn.y = fma(-al[q], api, rn.y);
                    rv[o] = rn;
                    nrm[q] += (double)rn.x * rn.x + (double)rn.y * rn.y;
                }
            }
        }
    }
    // residual recomputations (FP64, rare) after the CG work, by the whole
    // block (see K1); each one's partial sum is the block's total
    for (int r = 0; anyru && r < R; ++r) {
        if (modes[r] != M_RU)
            continue;
        const int j = a.perm[k0 + r];
        const double m2d = a.st[cur][j].mass2;
        double nr[1] = {0.0};
        for (int it = 0;; ++it) {
            const int s0 = chunk_start(it, Vh, a.remap);
            if (s0 < 0)
                break;
            for (int t = threadIdx.x; t < kChunk * 8; t += blockDim.x) {  // whole wavefronts
                int sl, sub;
                site_of_thread<8>(t, sl, sub);
                if (s0 + sl < Vh)
                    recompute_k2<P, 8, ROWS, 1>(a, j, par, s0 + sl, sub, m2d, nr[0]);
            }
        }
        double tot;
        block_sum_multi<1>(nr, red, tot);
        if (threadIdx.x == 0)
            partial_slot(a, cur, j, 2)[blockIdx.x] = tot;
    }
#pragma unroll
    for (int q = 0; q < RR; ++q) {
        if (js[q] < 0 || ru[q])
            continue;
        const double tot = wave_sum(nrm[q]);
        if (lane == 0)
            partial_slot(a, cur, js[q], 2)[blockIdx.x] = tot;
    }
}

}  // namespace stag
