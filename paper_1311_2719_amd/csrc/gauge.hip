// Gauge-field preparation (the role of the paper's `linkc_acc`, Sec. 4) and
// fermion layout conversion.
//
// From lexicographic links U_mu(x) (complex128 [V][4][3][3]) build, for each
// output parity p and checkerboard site s, the 8 links used by that site:
//   dir mu     : W_mu(x) =  1/2 eta_mu(x) s_fwd(x, mu) U_mu(x)
//   dir 4 + mu : B_mu(x) = -1/2 eta_mu(x) s_bwd(x, mu) U_mu(x - mu)^dagger
// (eta_mu(x - mu) = eta_mu(x) because eta_mu does not depend on x_mu), where
// s_fwd = -1 on a forward hop from t = Lt-1 and s_bwd = -1 on a backward hop
// from t = 0 when the field is antiperiodic in t.  The paper gathers ud = U^dagger
// through the backward neighbour table; storing B at the site that uses it
// makes all 8 link reads of a site unit-stride across lanes.
#include "runtime.hpp"

namespace stag {

namespace {

__global__ void __launch_bounds__(256)
k_prepare_links(Geom g, int tap, const double *__restrict__ U, dbl2 *__restrict__ l64,
                flt2 *__restrict__ l32, hlf2 *__restrict__ l16, int32_t *__restrict__ nbr,
                int *__restrict__ bad)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)2 * 8 * g.Vh;
    if (gid >= n)
        return;
    const int s = (int)(gid % g.Vh);
    const int d = (int)((gid / g.Vh) % 8);
    const int p = (int)(gid / ((int64_t)8 * g.Vh));
    const SiteCoord c = decode_site(g, p, s);
    const int co[4] = {c.x, c.y, c.z, c.t};
    const int mu = d & 3;
    int esum = 0;
    for (int nu = 0; nu < mu; ++nu)
        esum += co[nu];
    double fac = (esum & 1) ? -0.5 : 0.5;
    int src[4] = {c.x, c.y, c.z, c.t};
    const bool back = d >= 4;
    if (back) {
        src[mu] = co[mu] == 0 ? g.L[mu] - 1 : co[mu] - 1;
        fac = -fac;
        if (tap && mu == 3 && co[3] == 0)
            fac = -fac;
    } else if (tap && mu == 3 && co[3] == g.L[3] - 1) {
        fac = -fac;
    }
    const int64_t lex = src[0] + (int64_t)g.L[0] * (src[1] + (int64_t)g.L[1] * (src[2] + (int64_t)g.L[2] * src[3]));
    const double *u = U + (lex * 4 + mu) * 18;
    int nonfinite = 0;
    const int64_t pbase = (int64_t)p * 72 * g.Vh;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            // forward: entry (a,b) of U; backward: entry (a,b) of U^dagger = conj(U(b,a))
            const int k = back ? (b * 3 + a) : (a * 3 + b);
            double re = u[2 * k], im = u[2 * k + 1];
            if (back)
                im = -im;
            re *= fac;
            im *= fac;
            nonfinite |= !(isfinite(re) && isfinite(im));
            const int64_t o = pbase + link_offset(g.Vh, d, a * 3 + b, s);
            l64[o] = dbl2{re, im};
            if (l32)
                l32[o] = flt2{(float)re, (float)im};
            if (l16)
                l16[o] = hlf2{(_Float16)re, (_Float16)im};
        }
    }
    if (nonfinite)
        atomicOr(bad, 1);
    nbr[((int64_t)p * 8 + d) * g.Vh + s] = neighbour(g, c, s, d);
}

// lexicographic [V][3] <-> even-odd [2][3][Vh]
__global__ void __launch_bounds__(256)
k_pack(Geom g, dbl2 *__restrict__ lex, dbl2 *__restrict__ eo, int to_eo)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)2 * g.Vh)
        return;
    const int p = (int)(gid / g.Vh);
    const int s = (int)(gid % g.Vh);
    const SiteCoord c = decode_site(g, p, s);
    const int64_t l = c.x + (int64_t)g.L[0] * (c.y + (int64_t)g.L[1] * (c.z + (int64_t)g.L[2] * c.t));
#pragma unroll
    for (int col = 0; col < 3; ++col) {
        const int64_t e = ((int64_t)p * 3 + col) * g.Vh + s;
        if (to_eo)
            eo[e] = lex[l * 3 + col];
        else
            lex[l * 3 + col] = eo[e];
    }
}

}  // namespace

int gauge_prepare(Ctx *ctx, GaugeField *f, const double *links_dev, hipStream_t s)
{
    const Geom &g = f->g;
    const int64_t n = (int64_t)2 * 8 * g.Vh;
    int *bad = (int *)ctx->arena.alloc(256);
    if (!bad)
        return set_error(STAG_ENOMEM, "arena exhausted (gauge prep flag)");
    int rc = STAG_OK;
    hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), s);
    if (e == hipSuccess) {
        const int threads = 256;
        const int64_t blocks = (n + threads - 1) / threads;
        hipLaunchKernelGGL(k_prepare_links, dim3((unsigned)blocks), dim3(threads), 0, s, g, f->tap,
                           links_dev, (dbl2 *)f->links[0], (flt2 *)f->links[1], (hlf2 *)f->links[2],
                           f->nbr, bad);
        e = hipGetLastError();
    }
    int hbad = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        rc = set_error(STAG_EHIP, "gauge preparation failed: %s", hipGetErrorString(e));
    else if (hbad)
        rc = set_error(STAG_ENONFINITE, "gauge field holds NaN or Inf");
    ctx->arena.release(bad);
    return rc;
}

int launch_pack(const Geom &g, const double *lex, double *eo, int to_eo, hipStream_t s)
{
    const int threads = 256;
    const int64_t n = (int64_t)2 * g.Vh;
    const int64_t blocks = (n + threads - 1) / threads;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)blocks), dim3(threads), 0, s, g,
                       (dbl2 *)const_cast<double *>(lex), (dbl2 *)eo, to_eo);
    STAG_HIP_CHECK(hipGetLastError());
    return STAG_OK;
}

}  // namespace stag
