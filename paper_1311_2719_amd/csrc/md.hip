// Molecular dynamics around the CG (the paper's HMD program, Sec. 2 and
// Sec. 6; the paper names the Wilson gauge action and molecular dynamics but
// writes neither out, so the textbook readings are taken):
//   S_G = beta sum_{x, mu<nu} (1 - Re tr P_munu(x) / 3), links periodic;
//   F_G = -(beta / 6) TA[U_mu(x) Sigma_mu(x)], Sigma the sum of the six staples;
//   momenta Q anti-Hermitian traceless, H = -sum tr Q^2 + S_G + S_F;
//   dU/dt = Q U, dQ/dt = F_G + F_F (forces in the convention of force.hip);
//   leapfrog: Q += eps/2 F; n x { U = exp(eps Q) U, projected onto SU(3);
//   Q += eps F } with the last momentum step eps/2;
//   pseudofermion phi = m chi - D chi on the even sites.
// Links and momenta are complex128 [V][4][3][3] in the lexicographic order of
// the gauge-field input.
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "hop.hpp"
#include "runtime.hpp"

namespace stag {

namespace {

typedef cplx<double> cd;

struct Mat {
    cd e[9];
};

__device__ __forceinline__ Mat load_mat(const dbl2 *p)
{
    Mat m;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const dbl2 v = p[k];
        m.e[k] = {v.x, v.y};
    }
    return m;
}

__device__ __forceinline__ void store_mat(dbl2 *p, const Mat &m)
{
#pragma unroll
    for (int k = 0; k < 9; ++k)
        p[k] = dbl2{m.e[k].re, m.e[k].im};
}

// C = A B, with A or B daggered on request
template <bool DA, bool DB> __device__ __forceinline__ Mat mul(const Mat &A, const Mat &B)
{
    Mat C;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cd acc = czero<double>();
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                cd a = DA ? cd{A.e[k * 3 + i].re, -A.e[k * 3 + i].im} : A.e[i * 3 + k];
                cd b = DB ? cd{B.e[j * 3 + k].re, -B.e[j * 3 + k].im} : B.e[k * 3 + j];
                cmac(acc, a, b);
            }
            C.e[i * 3 + j] = acc;
        }
    return C;
}

__device__ __forceinline__ void add_to(Mat &A, const Mat &B)
{
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        A.e[k].re += B.e[k].re;
        A.e[k].im += B.e[k].im;
    }
}

// Lexicographic sites s = x + Lx (y + Ly (z + Lz t)); every lattice the
// library holds has fewer than 2^31 sites, so coordinates and indices are
// 32-bit (64-bit division is many times the cost on the GPU).
struct Lex {
    int32_t L[4];
    __device__ __forceinline__ void coords(int s, int (&c)[4]) const
    {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            c[d] = s % L[d];
            s /= L[d];
        }
        c[3] = s;
    }
    __device__ __forceinline__ int stride(int d) const
    {
        int st = 1;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            st *= k < d ? L[k] : 1;
        return st;
    }
    // site s (coordinates c) moved by `step` (+-1) along d, periodically
    __device__ __forceinline__ int step(int s, const int (&c)[4], int d, int step) const
    {
        const int st = stride(d), n = L[d], v = c[d] + step;
        return s + step * st + (v < 0 ? n * st : (v >= n ? -n * st : 0));
    }
    __device__ __forceinline__ int shift(int s, int mu, int step) const
    {
        int c[4];
        coords(s, c);
        return this->step(s, c, mu, step);
    }
};

// force (+)= coeff * (-beta/6) TA[U_mu(x) Sigma_mu(x)]; one thread per link
__global__ void __launch_bounds__(256)
k_gauge_force(Lex g, int64_t V, const dbl2 *__restrict__ U, dbl2 *__restrict__ force, double scale, int accumulate)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= V * 4)
        return;
    const int x = (int)(gid >> 2);
    const int mu = (int)(gid & 3);
    int c[4];
    g.coords(x, c);
    const int xpm = g.step(x, c, mu, 1);
    auto link = [&](int s, int nu) { return load_mat(U + ((int64_t)s * 4 + nu) * 9); };
    Mat S;
#pragma unroll
    for (int k = 0; k < 9; ++k)
        S.e[k] = czero<double>();
#pragma unroll 1
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu)
            continue;
        // x + mu - nu: the nu coordinate of x + mu is that of x
        const int xpn = g.step(x, c, nu, 1), xmn = g.step(x, c, nu, -1), xpm_mn = g.step(xpm, c, nu, -1);
        // U_nu(x+mu) U_mu(x+nu)^dagger U_nu(x)^dagger
        add_to(S, mul<false, true>(mul<false, true>(link(xpm, nu), link(xpn, mu)), link(x, nu)));
        // U_nu(x+mu-nu)^dagger U_mu(x-nu)^dagger U_nu(x-nu)
        add_to(S, mul<false, false>(mul<true, true>(link(xpm_mn, nu), link(xmn, mu)), link(xmn, nu)));
    }
    const Mat Z = mul<false, false>(link(x, mu), S);
    const double tr_im = (Z.e[0].im + Z.e[4].im + Z.e[8].im) / 3.0;
    dbl2 *out = force + gid * 9;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const cd p = Z.e[a * 3 + b], q = Z.e[b * 3 + a];
            const double re = 0.5 * (p.re - q.re);
            const double im = 0.5 * (p.im + q.im) - (a == b ? tr_im : 0.0);
            dbl2 v = dbl2{scale * re, scale * im};
            if (accumulate)
                v += out[a * 3 + b];
            out[a * 3 + b] = v;
        }
}

// exp(A) for A = eps Q anti-Hermitian: Taylor series of A / 2^k (norm <= 1/4)
// to order 12 (remainder below 1e-16), then k squarings
__device__ Mat expm(const Mat &A)
{
    double nrm = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k)
        nrm = fmax(nrm, fabs(A.e[k].re) + fabs(A.e[k].im));
    nrm *= 3.0;  // bounds the induced norm
    int sq = 0;
    while (nrm > 0.25 && sq < 60) {
        nrm *= 0.5;
        ++sq;
    }
    const double f = ldexp(1.0, -sq);
    Mat B;
#pragma unroll
    for (int k = 0; k < 9; ++k)
        B.e[k] = {A.e[k].re * f, A.e[k].im * f};
    // Horner: E = 1 + B (1 + B/2 (1 + B/3 (... (1 + B/12))))
    Mat E;
#pragma unroll
    for (int k = 0; k < 9; ++k)
        E.e[k] = czero<double>();
    E.e[0].re = E.e[4].re = E.e[8].re = 1.0;
    for (int n = 12; n >= 1; --n) {
        Mat T = mul<false, false>(B, E);
        const double c = 1.0 / n;
#pragma unroll
        for (int k = 0; k < 9; ++k)
            E.e[k] = {T.e[k].re * c, T.e[k].im * c};
        E.e[0].re += 1.0;
        E.e[4].re += 1.0;
        E.e[8].re += 1.0;
    }
    for (int i = 0; i < sq; ++i)
        E = mul<false, false>(E, E);
    return E;
}

// Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1)
__device__ Mat reunitarize(const Mat &M)
{
    Mat R;
    double n0 = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b)
        n0 += M.e[b].re * M.e[b].re + M.e[b].im * M.e[b].im;
    n0 = 1.0 / sqrt(n0);
#pragma unroll
    for (int b = 0; b < 3; ++b)
        R.e[b] = {M.e[b].re * n0, M.e[b].im * n0};
    cd d = czero<double>();  // <r0, m1> = sum conj(r0) m1
#pragma unroll
    for (int b = 0; b < 3; ++b)
        cmac(d, cd{R.e[b].re, -R.e[b].im}, M.e[3 + b]);
    double n1 = 0.0;
    cd r1[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        r1[b] = {M.e[3 + b].re - (d.re * R.e[b].re - d.im * R.e[b].im),
                 M.e[3 + b].im - (d.re * R.e[b].im + d.im * R.e[b].re)};
        n1 += r1[b].re * r1[b].re + r1[b].im * r1[b].im;
    }
    n1 = 1.0 / sqrt(n1);
#pragma unroll
    for (int b = 0; b < 3; ++b)
        R.e[3 + b] = {r1[b].re * n1, r1[b].im * n1};
    auto cross = [&](int i, int j) {
        // (r0 x r1) component formed from entries i, j
        const cd a = R.e[i], bb = R.e[3 + j], c = R.e[j], e = R.e[3 + i];
        return cd{a.re * bb.re - a.im * bb.im - (c.re * e.re - c.im * e.im),
                  a.re * bb.im + a.im * bb.re - (c.re * e.im + c.im * e.re)};
    };
    const cd z0 = cross(1, 2), z1 = cross(2, 0), z2 = cross(0, 1);
    R.e[6] = {z0.re, -z0.im};
    R.e[7] = {z1.re, -z1.im};
    R.e[8] = {z2.re, -z2.im};
    return R;
}

// U = reunitarize(exp(eps Q) U), one thread per link
__global__ void __launch_bounds__(256) k_link_update(int64_t nlinks, dbl2 *__restrict__ U, const dbl2 *__restrict__ Q,
                                                     double eps)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= nlinks)
        return;
    Mat A = load_mat(Q + gid * 9);
#pragma unroll
    for (int k = 0; k < 9; ++k)
        A.e[k] = {A.e[k].re * eps, A.e[k].im * eps};
    store_mat(U + gid * 9, reunitarize(mul<false, false>(expm(A), load_mat(U + gid * 9))));
}

// phi_e = m chi_e - phi_e (phi_e holds (D chi)_e), phi_o = 0; even-odd layout
__global__ void __launch_bounds__(256) k_pseudofermion(int Vh, const dbl2 *__restrict__ chi, dbl2 *__restrict__ phi,
                                                       double m)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)6 * Vh)
        return;
    if (gid < (int64_t)3 * Vh) {
        const dbl2 c = chi[gid], d = phi[gid];
        phi[gid] = dbl2{m * c.x - d.x, m * c.y - d.y};
    } else {
        phi[gid] = dbl2{0.0, 0.0};
    }
}

// Per-block partial sums of the energy terms, summed in a fixed order by the
// second kernel.  which = 0: -sum tr(Q^2) over links; 1: sum over sites and
// planes of (1 - Re tr P / 3); 2: Re sum over the even half of conj(a) b.
__global__ void __launch_bounds__(256)
k_energy_partials(int which, Lex g, int64_t n, const dbl2 *__restrict__ A, const dbl2 *__restrict__ B,
                  double *__restrict__ partials)
{
    __shared__ double lds[4];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (which == 0) {
            // -tr(Q Q) = sum_ab |Q_ab|^2 for anti-Hermitian Q
            const dbl2 *q = A + i * 9;
#pragma unroll
            for (int k = 0; k < 9; ++k)
                v += q[k].x * q[k].x + q[k].y * q[k].y;
        } else if (which == 1) {
            const int x = (int)i;
            auto link = [&](int s, int nu) { return load_mat(A + ((int64_t)s * 4 + nu) * 9); };
            for (int mu = 0; mu < 4; ++mu)
                for (int nu = mu + 1; nu < 4; ++nu) {
                    const Mat P = mul<false, true>(
                        mul<false, true>(mul<false, false>(link(x, mu), link(g.shift(x, mu, 1), nu)),
                                         link(g.shift(x, nu, 1), mu)),
                        link(x, nu));
                    v += 1.0 - (P.e[0].re + P.e[4].re + P.e[8].re) / 3.0;
                }
        } else {
            v += A[i].x * B[i].x + A[i].y * B[i].y;
        }
    }
    double arr[1] = {v};
    double tot;
    block_sum_multi<1>(arr, lds, tot);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256) k_energy_total(const double *__restrict__ partials, int n,
                                                      double *__restrict__ out)
{
    __shared__ double lds[4];
    const double t = reduce_partials(partials, n, lds);
    if (threadIdx.x == 0)
        *out = t;
}

constexpr int kEnergyBlocks = 1024;

}  // namespace

int gauge_force(const int32_t dims[4], const double *U, double *force, double beta, double coeff, int accumulate,
                hipStream_t s)
{
    Lex g;
    memcpy(g.L, dims, sizeof(g.L));
    const int64_t V = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    const dim3 grid((unsigned)((V * 4 + 255) / 256));
    hipLaunchKernelGGL(k_gauge_force, grid, dim3(256), 0, s, g, V, (const dbl2 *)U, (dbl2 *)force,
                       -coeff * beta / 6.0, accumulate);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(STAG_EHIP, "gauge force launch failed: %s", hipGetErrorString(e));
    return STAG_OK;
}

int link_update(int64_t V, double *U, const double *Q, double eps, hipStream_t s)
{
    const int64_t n = V * 4;
    hipLaunchKernelGGL(k_link_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, (dbl2 *)U,
                       (const dbl2 *)Q, eps);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(STAG_EHIP, "link update launch failed: %s", hipGetErrorString(e));
    return STAG_OK;
}

int pseudofermion(Ctx *ctx, GaugeField *f, const double *chi, double *phi, double mass, hipStream_t s)
{
    int rc = dslash(ctx, f, 0, STAG_EVEN, 0, f->g.Vh, chi, phi, 0, s);
    if (rc != STAG_OK)
        return rc;
    const int64_t n = (int64_t)6 * f->g.Vh;
    hipLaunchKernelGGL(k_pseudofermion, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, f->g.Vh,
                       (const dbl2 *)chi, (dbl2 *)phi, mass);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(STAG_EHIP, "pseudofermion launch failed: %s", hipGetErrorString(e));
    return STAG_OK;
}

// One energy term into *host_out (synchronous).  scratch: kEnergyBlocks + 1
// doubles of device memory.
static int energy_term(int which, const int32_t dims[4], const double *A, const double *B, int64_t n,
                       double *scratch, double *host_out, hipStream_t s)
{
    Lex g;
    memcpy(g.L, dims, sizeof(g.L));
    const int blocks = (int)std::min<int64_t>(kEnergyBlocks, std::max<int64_t>(1, (n + 255) / 256));
    hipLaunchKernelGGL(k_energy_partials, dim3(blocks), dim3(256), 0, s, which, g, n, (const dbl2 *)A,
                       (const dbl2 *)B, scratch);
    hipLaunchKernelGGL(k_energy_total, dim3(1), dim3(256), 0, s, scratch, blocks, scratch + kEnergyBlocks);
    STAG_HIP_CHECK(hipGetLastError());
    STAG_HIP_CHECK(hipMemcpyAsync(host_out, scratch + kEnergyBlocks, sizeof(double), hipMemcpyDeviceToHost, s));
    STAG_HIP_CHECK(hipStreamSynchronize(s));
    return STAG_OK;
}

int md_energies(const int32_t dims[4], const double *U, const double *Q, const double *phi, const double *x,
                double beta, double *scratch, double energies[3], hipStream_t s)
{
    const int64_t V = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    int rc = energy_term(0, dims, Q, nullptr, V * 4, scratch, &energies[0], s);
    if (rc == STAG_OK)
        rc = energy_term(1, dims, U, nullptr, V, scratch, &energies[1], s);
    energies[1] *= beta;
    energies[2] = 0.0;
    if (rc == STAG_OK && phi && x)  // the even half: 3 Vh complex entries
        rc = energy_term(2, dims, phi, x, 3 * V / 2, scratch, &energies[2], s);
    return rc;
}

int md_trajectory(Ctx *ctx, const int32_t dims[4], double *U, double *Q, const double *phi, const stag_md_params &p,
                  hipStream_t s, stag_md_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    stag_md_info inf;
    memset(&inf, 0, sizeof(inf));
    const Geom g0 = make_geom(dims);
    const int64_t V = 2 * (int64_t)g0.Vh;
    // a private field on the working links, rebuilt after every link update
    auto f = std::make_shared<GaugeField>();
    memcpy(f->dims, dims, sizeof(f->dims));
    f->tap = p.t_antiperiodic ? 1 : 0;
    f->g = g0;
    f->g.tap = f->tap;
    bool two_rows = false;
    int rc = gauge_check(ctx, f->g, U, s, two_rows);
    if (rc != STAG_OK)
        return rc;
    if (!two_rows)
        return set_error(STAG_EINVAL, "stag_md_trajectory: the links are not special unitary");
    const char *rows_env = getenv("STAG_LINK_ROWS");
    f->rows = rows_env && atoi(rows_env) == 3 ? 3 : 2;
    f->nt_links = nt_links_for(*f);
    const size_t vbytes = (size_t)2 * 3 * g0.Vh * 16;
    struct Owned {
        Ctx *c;
        std::vector<void *> p;
        ~Owned()
        {
            for (void *q : p)
                c->arena.release(q);
        }
        void *take(size_t n)
        {
            void *q = c->arena.alloc(n);
            if (q)
                p.push_back(q);
            return q;
        }
    } mem{ctx, {}};
    for (int k = 0; k < 3; ++k)
        f->links[k] = mem.take((size_t)2 * link_parity_entries(f->rows, g0.Vh) * link_entry_bytes_of(k));
    f->nbr = (int32_t *)mem.take(2 * 8 * g0.Vh * sizeof(int32_t));
    double *x = (double *)mem.take(vbytes), *y = (double *)mem.take(vbytes);
    double *scratch = (double *)mem.take((kEnergyBlocks + 1) * sizeof(double));
    if (!f->links[0] || !f->links[1] || !f->links[2] || !f->nbr || !x || !y || !scratch)
        return set_error(STAG_ENOMEM, "stag_md_trajectory: arena exhausted");
    stag_cg_params cp;
    memset(&cp, 0, sizeof(cp));
    cp.mass = p.mass;
    cp.tol = p.tol;
    cp.maxiter = p.maxiter;
    cp.precision = p.precision;
    cp.parity = STAG_EVEN;
    cp.max_restarts = 10;
    // W = x on the even sites and y = D_oe x on the odd sites, for the links in U
    auto solve = [&]() -> int {
        int r = gauge_check(ctx, f->g, U, s, two_rows);
        if (r != STAG_OK)
            return r;
        if (!two_rows)
            return set_error(STAG_EINVAL, "stag_md_trajectory: links left SU(3) beyond the two-row tolerance");
        r = gauge_prepare(f.get(), U, s);
        if (r != STAG_OK)
            return r;
        const double *bs[1] = {phi};
        double *xs[1] = {x}, *ys[1] = {y};
        stag_cg_info ci;
        r = cg_solve_batch(ctx, f, 1, &cp, bs, xs, ys, s, &ci);
        inf.cg_iters += ci.iters;
        inf.solves += 1;
        if (r != STAG_OK)
            return r;
        // x's odd half <- y's odd half
        STAG_HIP_CHECK(hipMemcpyAsync(x + 6 * g0.Vh, y + 6 * g0.Vh, vbytes / 2, hipMemcpyDeviceToDevice, s));
        return STAG_OK;
    };
    auto kick = [&](double w) -> int {  // Q += w (F_G + F_F)
        int r = gauge_force(dims, U, Q, p.beta, w, 1, s);
        if (r == STAG_OK)
            r = fermion_force(f.get(), x, Q, w, 1, s);
        return r;
    };
    struct DropBatches {  // the solve's cached workspace belongs to this private field
        Ctx *c;
        ~DropBatches() { drop_cached_batches(c, 0); }
    } drop{ctx};
    double e[3];
    if ((rc = solve()) != STAG_OK || (rc = md_energies(dims, U, Q, phi, x, p.beta, scratch, e, s)) != STAG_OK)
        return rc;
    inf.kinetic[0] = e[0];
    inf.gauge_action[0] = e[1];
    inf.fermion_action[0] = e[2];
    if ((rc = kick(0.5 * p.eps)) != STAG_OK)
        return rc;
    for (int k = 0; k < p.nsteps; ++k) {
        if ((rc = link_update(V, U, Q, p.eps, s)) != STAG_OK || (rc = solve()) != STAG_OK)
            return rc;
        if ((rc = kick(k < p.nsteps - 1 ? p.eps : 0.5 * p.eps)) != STAG_OK)
            return rc;
    }
    if ((rc = md_energies(dims, U, Q, phi, x, p.beta, scratch, e, s)) != STAG_OK)
        return rc;
    inf.kinetic[1] = e[0];
    inf.gauge_action[1] = e[1];
    inf.fermion_action[1] = e[2];
    inf.delta_h = (e[0] + e[1] + e[2]) - (inf.kinetic[0] + inf.gauge_action[0] + inf.fermion_action[0]);
    STAG_HIP_CHECK(hipStreamSynchronize(s));
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info)
        *info = inf;
    return STAG_OK;
}

}  // namespace stag
