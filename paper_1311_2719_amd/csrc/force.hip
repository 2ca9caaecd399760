// The molecular-dynamics force of the staggered pseudofermion action, from
// the fields the CG returns (the paper's HMD program around its CG, Sec. 2,
// Sec. 4 and Sec. 6; the action and force are not written out in the paper,
// the textbook reading is taken):
//
//   S_F = phi^dagger (m^2 - D_eo D_oe)^{-1} phi  (phi on the even sites),
//   W = x on the even sites, y = D_oe x on the odd sites,
//   F_mu(z) = TA[ eps(z) L_mu(z) W(z + mu) W(z)^dagger ],
//
// where L_mu(z) = eta_mu(z) b_mu(z) U_mu(z) / 2 is exactly the forward link
// the library stores at site z (staggered phase, the 1/2 and the t-boundary
// sign folded in), eps(z) = +1 on even and -1 on odd sites, and
// TA(Z) = (Z - Z^dagger)/2 - tr(Z - Z^dagger)/6.  dS_F/dw = 2 Re tr[i T F]
// for the variation U_mu(z) -> exp(i w T) U_mu(z).
//
// One thread per (site, direction): a block of 256 threads takes 64
// consecutive lexicographic sites and their four directions, so that the
// block's output is one contiguous 36 KB span of the complex128
// [V][4][3][3] result (lexicographic, the order of the gauge-field input).
// The threads compute their matrices into LDS; the block then writes the
// span with unit-stride stores (adding the old values when accumulating),
// instead of each thread storing its own 144 B with a stride of 576 B.
// Bytes per site: 4 forward links (FP64, stored rows), the site's and its
// four forward neighbours' W (48 B each, the neighbours' amortised to one),
// 4 x 144 B written (plus 4 x 144 B read when accumulating).
#include "runtime.hpp"

namespace stag {

namespace {

constexpr int kForceSites = 64;  // lexicographic sites per block

template <class P64, int ROWS>
__global__ void __launch_bounds__(256)
k_fermion_force(Geom g, const dbl2 *__restrict__ links, const dbl2 *__restrict__ w, dbl2 *__restrict__ force,
                double coeff, int accumulate)
{
    __shared__ dbl2 out[kForceSites * 4 * 9];
    const int Vh = g.Vh;
    const int64_t V = (int64_t)2 * Vh;
    const int64_t lex0 = (int64_t)blockIdx.x * kForceSites;
    const int nsite = (int)(V - lex0 < kForceSites ? V - lex0 : kForceSites);
    const int t = threadIdx.x, ls = t >> 2, mu = t & 3;
    if (ls < nsite) {
        // lexicographic site -> parity and checkerboard index (Lx is even)
        const int64_t lex = lex0 + ls;
        const int x = (int)(lex % g.L[0]);
        int64_t r = lex / g.L[0];
        const int y = (int)(r % g.L[1]);
        r /= g.L[1];
        const int z = (int)(r % g.L[2]);
        const int tt = (int)(r / g.L[2]);
        const int p = (x + y + z + tt) & 1;
        const int s = (int)(lex >> 1);
        const SiteCoord c = decode_site(g, p, s);
        cplx<double> wz[3];
        PrecF64::load_spinor(w + (size_t)p * 3 * Vh, Vh, s, wz);
        cplx<double> wf[3];
        PrecF64::load_spinor(w + (size_t)(1 - p) * 3 * Vh, Vh, neighbour(g, c, s, mu), wf);
        const dbl2 *lk = links + link_parity_entries(ROWS, Vh) * p;
        cplx<double> L[9];
#pragma unroll
        for (int k = 0; k < 3 * ROWS; ++k)
            L[k] = P64::load_link(lk + link_offset(Vh, mu, k, s));
        if constexpr (ROWS == 2)
            third_row(L, folded_negative(g, c, mu) ? -2.0 : 2.0);
        // B = L (W(z+mu) W(z)^dagger): B_ab = (L wf)_a conj(wz_b)
        cplx<double> lw[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lw[a] = czero<double>();
#pragma unroll
            for (int b = 0; b < 3; ++b)
                cmac(lw[a], L[a * 3 + b], wf[b]);
        }
        cplx<double> B[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                B[a * 3 + b] = {lw[a].re * wz[b].re + lw[a].im * wz[b].im, lw[a].im * wz[b].re - lw[a].re * wz[b].im};
        // traceless anti-Hermitian part, times the coefficient and eps(z)
        const double scale = p == 0 ? coeff : -coeff;
        const double tr_im = (B[0].im + B[4].im + B[8].im) / 3.0;
        dbl2 *o = out + (ls * 4 + mu) * 9;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const cplx<double> u = B[a * 3 + b], v = B[b * 3 + a];
                const double re = 0.5 * (u.re - v.re);
                const double im = 0.5 * (u.im + v.im) - (a == b ? tr_im : 0.0);
                o[a * 3 + b] = dbl2{scale * re, scale * im};
            }
        }
    }
    __syncthreads();
    // the block's span, unit stride
    dbl2 *dst = force + lex0 * 4 * 9;
    const int n = nsite * 4 * 9;
    for (int i = t; i < n; i += blockDim.x) {
        dbl2 v = out[i];
        if (accumulate)
            v += dst[i];
        dst[i] = v;
    }
}

}  // namespace

int fermion_force(GaugeField *f, const double *w, double *force, double coeff, int accumulate, hipStream_t s)
{
    const Geom &g = f->g;
    const int64_t V = (int64_t)2 * g.Vh;
    const dim3 grid((unsigned)((V + kForceSites - 1) / kForceSites));
    const dim3 block(kForceSites * 4);
#define STAG_FORCE_CASE(P64, ROWS)                                                                                   \
    hipLaunchKernelGGL((k_fermion_force<P64, ROWS>), grid, block, 0, s, g, (const dbl2 *)f->links[0],              \
                       (const dbl2 *)w, (dbl2 *)force, coeff, accumulate)
    if (f->nt_links) {
        if (f->rows == 2)
            STAG_FORCE_CASE(PrecF64NT, 2);
        else
            STAG_FORCE_CASE(PrecF64NT, 3);
    } else {
        if (f->rows == 2)
            STAG_FORCE_CASE(PrecF64, 2);
        else
            STAG_FORCE_CASE(PrecF64, 3);
    }
#undef STAG_FORCE_CASE
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(STAG_EHIP, "fermion force launch failed: %s", hipGetErrorString(e));
    return STAG_OK;
}

}  // namespace stag
