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
// makes all 8 link reads of a site unit-stride across lanes.  When every one
// of these matrices is 1/2 (with a sign) times a special unitary matrix, only
// their first two rows are stored and the kernels rebuild the third
// (two-row form, 2/3 of the link bytes).
#include <cstdlib>

#include "runtime.hpp"

namespace stag {

namespace {

// The link of direction d used by checkerboard site s of output parity p, with
// the folded factor (see above): w[k] = entry k (row-major) of W_mu(x) or
// B_mu(x).  Returns false if an entry is not finite.
__device__ bool folded_link(const Geom &g, const double *__restrict__ U, int p, int d, int s, dbl2 (&w)[9])
{
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
        if (g.tap && mu == 3 && co[3] == 0)
            fac = -fac;
    } else if (g.tap && mu == 3 && co[3] == g.L[3] - 1) {
        fac = -fac;
    }
    const int64_t lex = src[0] + (int64_t)g.L[0] * (src[1] + (int64_t)g.L[1] * (src[2] + (int64_t)g.L[2] * src[3]));
    const double *u = U + (lex * 4 + mu) * 18;
    bool finite = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            // forward: entry (a,b) of U; backward: entry (a,b) of U^dagger = conj(U(b,a))
            const int k = back ? (b * 3 + a) : (a * 3 + b);
            double re = u[2 * k], im = u[2 * k + 1];
            if (back)
                im = -im;
            w[a * 3 + b] = dbl2{re * fac, im * fac};
            finite = finite && isfinite(re) && isfinite(im);
        }
    }
    return finite;
}

// flags |= 1 if any entry is not finite; |= 2 if some stored matrix is not
// (1/2 sign) x a special unitary matrix to within `tol` in the sense the
// two-row form relies on: row 2 = conj(row 0 x row 1) / c.
__global__ void __launch_bounds__(256)
k_check_links(Geom g, const double *__restrict__ U, double tol, int *__restrict__ flags)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)2 * 8 * g.Vh)
        return;
    const int s = (int)(gid % g.Vh);
    const int d = (int)((gid / g.Vh) % 8);
    const int p = (int)(gid / ((int64_t)8 * g.Vh));
    dbl2 w[9];
    int f = 0;
    if (!folded_link(g, U, p, d, s, w)) {
        f = 1;
    } else {
        cplx<double> W[9];
        for (int k = 0; k < 9; ++k)
            W[k] = {w[k].x, w[k].y};
        const cplx<double> given[3] = {W[6], W[7], W[8]};
        third_row(W, folded_negative(g, decode_site(g, p, s), d) ? -2.0 : 2.0);
        double dev = 0.0;
        for (int k = 0; k < 3; ++k)
            dev = fmax(dev, fmax(fabs(W[6 + k].re - given[k].re), fabs(W[6 + k].im - given[k].im)));
        if (!(dev <= tol))
            f = 2;
    }
    if (f)
        atomicOr(flags, f);
}

// Write the 3 * ROWS stored entries of every link in FP64, FP32 and FP16, and
// the neighbour tables.
template <int ROWS>
__global__ void __launch_bounds__(256)
k_prepare_links(Geom g, const double *__restrict__ U, dbl2 *__restrict__ l64, flt2 *__restrict__ l32,
                hlf2 *__restrict__ l16, int32_t *__restrict__ nbr)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)2 * 8 * g.Vh)
        return;
    const int s = (int)(gid % g.Vh);
    const int d = (int)((gid / g.Vh) % 8);
    const int p = (int)(gid / ((int64_t)8 * g.Vh));
    dbl2 w[9];
    (void)folded_link(g, U, p, d, s, w);
    const int64_t pbase = link_parity_entries(ROWS, g.Vh) * p;
#pragma unroll
    for (int k = 0; k < 3 * ROWS; ++k) {
        const int64_t o = pbase + link_offset(g.Vh, d, k, s);
        l64[o] = w[k];
        l32[o] = flt2{(float)w[k].x, (float)w[k].y};
        l16[o] = hlf2{(_Float16)w[k].x, (_Float16)w[k].y};
    }
    nbr[((int64_t)p * 8 + d) * g.Vh + s] = neighbour(g, decode_site(g, p, s), s, d);
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

int nt_links_for(const GaugeField &f)
{
    if (const char *e = getenv("STAG_NT_LINKS"))
        if (e[0] == '0' || e[0] == '1')
            return e[0] == '1';
    const size_t fp64_link_bytes = (size_t)2 * link_parity_entries(f.rows, f.g.Vh) * link_entry_bytes_of(0);
    return fp64_link_bytes > ((size_t)256 << 20);
}

int gauge_check(Ctx *ctx, const Geom &g, const double *links_dev, hipStream_t s, bool &two_rows)
{
    const int64_t n = (int64_t)2 * 8 * g.Vh;
    int *flags = (int *)ctx->arena.alloc(256);
    if (!flags)
        return set_error(STAG_ENOMEM, "arena exhausted (gauge check flags)");
    int hflags = 0;
    hipError_t e = hipMemsetAsync(flags, 0, sizeof(int), s);
    if (e == hipSuccess) {
        const int threads = 256;
        hipLaunchKernelGGL(k_check_links, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0, s, g,
                           links_dev, kTwoRowTolerance, flags);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    ctx->arena.release(flags);
    if (e != hipSuccess)
        return set_error(STAG_EHIP, "gauge check failed: %s", hipGetErrorString(e));
    if (hflags & 1)
        return set_error(STAG_ENONFINITE, "gauge field holds NaN or Inf");
    two_rows = (hflags & 2) == 0;
    return STAG_OK;
}

int gauge_prepare(GaugeField *f, const double *links_dev, hipStream_t s)
{
    const Geom &g = f->g;
    const int64_t n = (int64_t)2 * 8 * g.Vh;
    const int threads = 256;
    const dim3 grid((unsigned)((n + threads - 1) / threads));
    if (f->rows == 2)
        hipLaunchKernelGGL((k_prepare_links<2>), grid, dim3(threads), 0, s, g, links_dev, (dbl2 *)f->links[0],
                           (flt2 *)f->links[1], (hlf2 *)f->links[2], f->nbr);
    else
        hipLaunchKernelGGL((k_prepare_links<3>), grid, dim3(threads), 0, s, g, links_dev, (dbl2 *)f->links[0],
                           (flt2 *)f->links[1], (hlf2 *)f->links[2], f->nbr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return set_error(STAG_EHIP, "gauge preparation failed: %s", hipGetErrorString(e));
    return STAG_OK;
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
