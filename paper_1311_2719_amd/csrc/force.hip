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
// One thread per site and parity computes the four forces of the links that
// leave the site; the output is complex128 [V][4][3][3] in the lexicographic
// order of the gauge-field input.  Bytes per site: 4 forward links (FP64,
// stored rows), the site's and its four forward neighbours' W (48 B each,
// the neighbours' amortised to one), 4 x 144 B written (plus 4 x 144 B read
// when accumulating).
#include "runtime.hpp"

namespace stag {

namespace {

template <int ROWS>
__global__ void __launch_bounds__(256)
k_fermion_force(Geom g, const dbl2 *__restrict__ links, const dbl2 *__restrict__ w, dbl2 *__restrict__ force,
                double coeff, int accumulate)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)2 * g.Vh)
        return;
    const int p = (int)(gid / g.Vh);
    const int s = (int)(gid % g.Vh);
    const int Vh = g.Vh;
    const SiteCoord c = decode_site(g, p, s);
    const int64_t lex = c.x + (int64_t)g.L[0] * (c.y + (int64_t)g.L[1] * (c.z + (int64_t)g.L[2] * c.t));
    // W at the site (parity p) and the sign eps(z), folded into the coefficient
    cplx<double> wz[3];
    PrecF64::load_spinor(w + (size_t)p * 3 * Vh, Vh, s, wz);
    const double scale = p == 0 ? coeff : -coeff;
    const dbl2 *lk = links + link_parity_entries(ROWS, Vh) * p;
    const dbl2 *wn = w + (size_t)(1 - p) * 3 * Vh;
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
        cplx<double> L[9];
#pragma unroll
        for (int k = 0; k < 3 * ROWS; ++k)
            L[k] = PrecF64::load_link(lk + link_offset(Vh, mu, k, s));
        if constexpr (ROWS == 2)
            third_row(L, folded_negative(g, c, mu) ? -2.0 : 2.0);
        cplx<double> wf[3];
        PrecF64::load_spinor(wn, Vh, neighbour(g, c, s, mu), wf);
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
        const double tr_im = (B[0].im + B[4].im + B[8].im) / 3.0;
        dbl2 *out = force + (lex * 4 + mu) * 9;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const cplx<double> x = B[a * 3 + b], y = B[b * 3 + a];
                double re = 0.5 * (x.re - y.re);
                double im = 0.5 * (x.im + y.im) - (a == b ? tr_im : 0.0);
                dbl2 v = dbl2{scale * re, scale * im};
                if (accumulate)
                    v += out[a * 3 + b];
                out[a * 3 + b] = v;
            }
        }
    }
}

}  // namespace

int fermion_force(GaugeField *f, const double *w, double *force, double coeff, int accumulate, hipStream_t s)
{
    const Geom &g = f->g;
    const int64_t n = (int64_t)2 * g.Vh;
    const int threads = 256;
    const dim3 grid((unsigned)((n + threads - 1) / threads));
    if (f->rows == 2)
        hipLaunchKernelGGL((k_fermion_force<2>), grid, dim3(threads), 0, s, g, (const dbl2 *)f->links[0],
                           (const dbl2 *)w, (dbl2 *)force, coeff, accumulate);
    else
        hipLaunchKernelGGL((k_fermion_force<3>), grid, dim3(threads), 0, s, g, (const dbl2 *)f->links[0],
                           (const dbl2 *)w, (dbl2 *)force, coeff, accumulate);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(STAG_EHIP, "fermion force launch failed: %s", hipGetErrorString(e));
    return STAG_OK;
}

}  // namespace stag
