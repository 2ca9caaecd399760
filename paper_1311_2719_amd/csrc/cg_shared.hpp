// CG step kernels for FP32 and FP16 working precision in which the systems
// of a tile share every link read through LDS.
//
// The register tiles of cg_kernels.hpp share a link load between the R
// systems one thread carries, so their per-thread state grows with R and the
// tuner settles on R = 2 or 3 at 24^4: every link is then read from HBM
// S / R times per kernel.  Here a block is R wavefronts; wavefront w runs
// system w of the block's tile on 64 consecutive output sites, one lane per
// site.  The block first reads the links of those 64 sites (8 directions,
// stored rows), rebuilds row 2 where only two are stored, converts them to
// FP32 and keeps all nine entries in LDS; every wavefront then runs a
// single-system hop that takes its links from there.  A link thus costs one
// HBM read per R systems (R up to 16, one tile per parity at 12 or 16
// systems), the third row and the FP16 conversion are computed once per
// block instead of once per thread, and a wavefront holds the registers of
// one system only.
//
// The step arithmetic is that of k_cg_step1 / k_cg_step2 (the loop of the
// paper's Sec. 4 with the mass explicit): same products, same storage
// formats, same state machine (advance()); only the summation order of the
// partial sums differs (one system per wavefront: lane sums over the chunks
// a block visits, then the wavefront sum).
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
constexpr int kSharedMaxR = 16;         // wavefronts (systems) per block
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
// site), so every global load of a wavefront reads 512 contiguous bytes.
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
        for (int k = 0; k < 3 * ROWS; ++k)
            U[k] = P::load_link(base + (int64_t)k * 8 * Vh + it);
        if constexpr (ROWS == 2) {
            const SiteCoord c = decode_site(g, p_out, s0 + i);
            third_row(U, folded_negative(g, c, d) ? -2.f : 2.f);
        }
#pragma unroll
        for (int k = 0; k < 9; ++k)
            lk[chunk_link_index(k, d, i)] = flt2{U[k].re, U[k].im};
    }
}

// acc[a] += sum_d L_d(s)[a][b] chi_d[b], the links from the staged chunk
// (lane i = site s0 + i), load(n, chi) the input at neighbour n.
template <bool TABLES, class Load>
__device__ __forceinline__ void hop_shared_impl(const Geom &g, const int32_t *__restrict__ nbr, int p_out, int s,
                                                int i, const flt2 *lk, cplx<float> (&acc)[3], Load load)
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
        cplx<float> chi[3];
        load(n, chi);
        cplx<float> U[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const flt2 v = lk[chunk_link_index(k, d, i)];
            U[k] = {v.x, v.y};
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                cmac(acc[a], U[a * 3 + b], chi[b]);
    }
}

template <class Load>
__device__ __forceinline__ void hop_shared(const Geom &g, const int32_t *nbr, int p_out, int s, int i, const flt2 *lk,
                                           cplx<float> (&acc)[3], Load load)
{
    if (nbr)
        hop_shared_impl<true>(g, nbr, p_out, s, i, lk, acc, load);
    else
        hop_shared_impl<false>(g, nbr, p_out, s, i, lk, acc, load);
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

template <class P, int R, int ROWS>
__global__ void __launch_bounds__(64 * R, kSharedMinWaves) k_cg_shared1(CgArgs a, int ver)
{
    static_assert(P::id != 0 && R <= kSharedMaxR, "shared-link tiles: FP32 / FP16 working precision");
    using real = typename P::real;
    using v2 = typename vec2_of<real>::type;
    __shared__ flt2 lk[9 * 8 * kLdsRow];
    __shared__ int modes[R];
    const int tpp = a.S / R;
    const int par = blockIdx.y / tpp, k0 = par * a.S + (blockIdx.y % tpp) * R, pout = 1 - par;
    const int Vh = a.g.Vh;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = a.perm[k0 + w];
    // prologue: this wavefront advances its own system over the previous step
    SysState st{};
    int mode = M_IDLE;
    if (j >= 0) {
        double t[3];
        wave_prologue_sums<3>(a, ver, j, t);
        st = a.st[ver][j];
        const bool live = st.mode != M_IDLE && st.mode != M_DONE;
        if (live)
            advance(st, t);
        // the state K2 of this step reads: advanced, or the same idle/done state
        if (blockIdx.x == 0 && lane == 0)
            a.st[ver ^ 1][j] = st;
        mode = live ? uniform(st.mode) : (int)M_IDLE;
    }
    if (lane == 0)
        modes[w] = mode;
    __syncthreads();
    bool anycg = false, anyru = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        anycg |= modes[r] == M_CG;
        anyru |= modes[r] == M_RU;
    }
    if (!anycg && !anyru)
        return;
    const bool cg = mode == M_CG, ru = mode == M_RU;
    const real beta = (real)uniform(st.beta);
    const int pc = uniform(st.pcur);
    const int jj = j >= 0 ? j : 0;
    const v2 *rv = (const v2 *)a.r + (size_t)jj * 3 * Vh;
    const void *pold = spin_at<P>(a.p[pc], jj, Vh);
    void *pnew = spin_at<P>(a.p[pc ^ 1], jj, Vh);
    void *apv = spin_at<P>(a.ap, jj, Vh);
    double nrm_ap = 0.0, nrm_p = 0.0;
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
        if (cg) {
            cplx<float> acc[3] = {czero<float>(), czero<float>(), czero<float>()};
            // the partner site's p and r (same index, parity par), loaded before the gathers
            cplx<real> po[3];
            v2 ro[3];
            P::load_spinor(pold, Vh, s, po);
#pragma unroll
            for (int c = 0; c < 3; ++c)
                ro[c] = rv[(int64_t)c * Vh + s];
            auto load = [&](int n, cplx<float> *chi) {
                cplx<real> pv[3];
                P::load_spinor(pold, Vh, n, pv);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const v2 t = rv[(int64_t)c * Vh + n];
                    chi[c].re = fma(beta, pv[c].re, t.x);
                    chi[c].im = fma(beta, pv[c].im, t.y);
                }
            };
            hop_shared(a.g, a.nbr[pout], pout, s, lane, lk, acc, load);
            cplx<real> pn[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                pn[c].re = fma(beta, po[c].re, ro[c].x);
                pn[c].im = fma(beta, po[c].im, ro[c].y);
            }
            P::store_spinor(apv, Vh, s, acc);
            if constexpr (P::id == 2)
                P::store_spinor_read_back(pnew, Vh, s, pn);  // pn: the value D will read
            else
                P::store_spinor(pnew, Vh, s, pn);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                nrm_p += (double)pn[c].re * pn[c].re + (double)pn[c].im * pn[c].im;
                nrm_ap += (double)acc[c].re * acc[c].re + (double)acc[c].im * acc[c].im;
            }
        } else if (ru) {
            recompute_k1<1, ROWS, 1>(a, j, pout, s, 0);
        }
    }
    if (!anycg || j < 0)
        return;
    const double tap = wave_sum(nrm_ap), tpp2 = wave_sum(nrm_p);
    if (lane == 0) {
        partial_slot(a, ver ^ 1, j, 0)[blockIdx.x] = tap;
        partial_slot(a, ver ^ 1, j, 1)[blockIdx.x] = tpp2;
    }
}

// ---- K2 -----------------------------------------------------------------------------

template <class P, int R, int ROWS>
__global__ void __launch_bounds__(64 * R, kSharedMinWaves) k_cg_shared2(CgArgs a, int ver)
{
    static_assert(P::id != 0 && R <= kSharedMaxR, "shared-link tiles: FP32 / FP16 working precision");
    using real = typename P::real;
    using v2 = typename vec2_of<real>::type;
    __shared__ flt2 lk[9 * 8 * kLdsRow];
    __shared__ int modes[R];
    const int tpp = a.S / R;
    const int par = blockIdx.y / tpp, k0 = par * a.S + (blockIdx.y % tpp) * R;
    const int Vh = a.g.Vh;
    const int cur = ver ^ 1;  // the state K1 of this step wrote
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = a.perm[k0 + w];
    // alpha from K1's partial sums (slots 0 and 1)
    int mode = M_IDLE;
    double alpha = 0.0, m2 = 0.0;
    int pn_buf = 0;
    if (j >= 0) {
        const SysState &st = a.st[cur][j];
        const int smode = st.mode;
        const double mass2 = st.mass2, rr = st.rr;
        const int pcur = st.pcur;
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
        m2 = uniform(mass2);
        pn_buf = uniform(pcur) ^ 1;  // p' written by K1 of this step
    }
    if (lane == 0)
        modes[w] = mode;
    __syncthreads();
    bool anycg = false, anyru = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        anycg |= modes[r] == M_CG;
        anyru |= modes[r] == M_RU;
    }
    if (!anycg && !anyru)
        return;
    const bool cg = mode == M_CG, ru = mode == M_RU;
    const real al = (real)alpha, m2r = (real)m2;
    const int jj = j >= 0 ? j : 0;
    const void *apv = spin_at<P>(a.ap, jj, Vh);
    const void *pb = spin_at<P>(a.p[pn_buf], jj, Vh);
    v2 *rv = (v2 *)a.r + (size_t)jj * 3 * Vh;
    flt2 *xl = a.xlo + (size_t)jj * 3 * Vh;
    double nrm = 0.0;
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
        if (cg) {
            // this site's p', x and r, loaded before the gathers
            cplx<real> pv[3];
            flt2 xv[3];
            v2 ro[3];
            P::load_spinor(pb, Vh, s, pv);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                xv[c] = xl[(int64_t)c * Vh + s];
                ro[c] = rv[(int64_t)c * Vh + s];
            }
            cplx<float> acc[3] = {czero<float>(), czero<float>(), czero<float>()};
            auto load = [&](int n, cplx<float> *chi) { P::load_spinor(apv, Vh, n, chi); };
            hop_shared(a.g, a.nbr[par], par, s, lane, lk, acc, load);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int64_t o = (int64_t)c * Vh + s;
                xl[o] = flt2{fmaf(al, pv[c].re, xv[c].x), fmaf(al, pv[c].im, xv[c].y)};
                const real apr = m2r * pv[c].re - acc[c].re;
                const real api = m2r * pv[c].im - acc[c].im;
                v2 rn = ro[c];
                rn.x = fma(-al, apr, rn.x);
                rn.y = fma(-al, api, rn.y);
                rv[o] = rn;
                nrm += (double)rn.x * rn.x + (double)rn.y * rn.y;
            }
        } else if (ru) {
            recompute_k2<P, 1, ROWS, 1>(a, j, par, s, 0, m2, nrm);
        }
    }
    if (j < 0)
        return;
    const double tot = wave_sum(nrm);
    if (lane == 0)
        partial_slot(a, cur, j, 2)[blockIdx.x] = tot;
}

}  // namespace stag
