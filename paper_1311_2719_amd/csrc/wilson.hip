// Wilson fermions (the paper's second workload, named in Sec. 2 and Sec. 6): gauge preparation,
// spin-colour vector layout, the standalone hop and the even-odd CG driver.
// The operator and the kernels are described in wilson_kernels.hpp.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "runtime.hpp"
#include "wilson_kernels.hpp"

namespace stag {

namespace {

// The link of direction d at checkerboard site s of output parity p for the
// Wilson operator: W_mu(x) = s_fwd U_mu(x) (d < 4), B_mu(x) = s_bwd
// U_mu(x - mu)^dagger (d >= 4), s_* the t-boundary signs.  False if an entry is
// not finite.
__device__ bool wilson_link(const Geom &g, const double *__restrict__ U, int p, int d, int s, dbl2 (&w)[9])
{
    const SiteCoord c = decode_site(g, p, s);
    const int mu = d & 3;
    int src[4] = {c.x, c.y, c.z, c.t};
    const bool back = d >= 4;
    double fac = wil::wilson_link_negative(g, c, d) ? -1.0 : 1.0;
    if (back)
        src[mu] = src[mu] == 0 ? g.L[mu] - 1 : src[mu] - 1;
    const int64_t lex = src[0] + (int64_t)g.L[0] * (src[1] + (int64_t)g.L[1] * (src[2] + (int64_t)g.L[2] * src[3]));
    const double *u = U + (lex * 4 + mu) * 18;
    bool finite = true;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int k = back ? (b * 3 + a) : (a * 3 + b);
            const double re = u[2 * k], im = back ? -u[2 * k + 1] : u[2 * k + 1];
            w[a * 3 + b] = dbl2{re * fac, im * fac};
            finite = finite && isfinite(re) && isfinite(im);
        }
    return finite;
}

// flags |= 1: an entry is not finite; |= 2: some link is not special unitary
// in the sense the two-row form relies on (row 2 = conj(row 0 x row 1) / c)
__global__ void __launch_bounds__(256) k_wcheck_links(Geom g, const double *__restrict__ U, double tol, int *flags)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)2 * 8 * g.Vh)
        return;
    const int s = (int)(gid % g.Vh), d = (int)((gid / g.Vh) % 8), p = (int)(gid / ((int64_t)8 * g.Vh));
    dbl2 w[9];
    int f = 0;
    if (!wilson_link(g, U, p, d, s, w)) {
        f = 1;
    } else {
        cplx<double> W[9];
        for (int k = 0; k < 9; ++k)
            W[k] = {w[k].x, w[k].y};
        const cplx<double> given[3] = {W[6], W[7], W[8]};
        third_row(W, wil::wilson_link_negative(g, decode_site(g, p, s), d) ? -1.0 : 1.0);
        double dev = 0.0;
        for (int k = 0; k < 3; ++k)
            dev = fmax(dev, fmax(fabs(W[6 + k].re - given[k].re), fabs(W[6 + k].im - given[k].im)));
        if (!(dev <= tol))
            f = 2;
    }
    if (f)
        atomicOr(flags, f);
}

template <int ROWS>
__global__ void __launch_bounds__(256) k_wprepare_links(Geom g, const double *__restrict__ U, dbl2 *__restrict__ l64)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)2 * 8 * g.Vh)
        return;
    const int s = (int)(gid % g.Vh), d = (int)((gid / g.Vh) % 8), p = (int)(gid / ((int64_t)8 * g.Vh));
    dbl2 w[9];
    (void)wilson_link(g, U, p, d, s, w);
    const int64_t base = link_parity_entries(ROWS, g.Vh) * p;
#pragma unroll
    for (int k = 0; k < 3 * ROWS; ++k)
        l64[base + link_offset(g.Vh, d, k, s)] = w[k];
}

// lexicographic [V][4][3] <-> even-odd [2][12][Vh]
__global__ void __launch_bounds__(256) k_pack_spinor(Geom g, dbl2 *__restrict__ lex, dbl2 *__restrict__ eo, int to_eo)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)2 * g.Vh)
        return;
    const int p = (int)(gid / g.Vh), s = (int)(gid % g.Vh);
    const SiteCoord c = decode_site(g, p, s);
    const int64_t l = c.x + (int64_t)g.L[0] * (c.y + (int64_t)g.L[1] * (c.z + (int64_t)g.L[2] * c.t));
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const int64_t e = ((int64_t)p * 12 + k) * g.Vh + s;
        if (to_eo)
            eo[e] = lex[l * 12 + k];
        else
            lex[l * 12 + k] = eo[e];
    }
}

// per-block partial sums of |v|^2 over n complex entries
__global__ void __launch_bounds__(256) k_norm2_partials(const dbl2 *__restrict__ v, int64_t n, double *out)
{
    __shared__ double lds[4];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const dbl2 t = v[i];
        acc += t.x * t.x + t.y * t.y;
    }
    double arr[1] = {acc};
    double tot;
    block_sum_multi<1>(arr, lds, tot);
    if (threadIdx.x == 0)
        out[blockIdx.x] = tot;
}

constexpr int kWBlock = 128;

}  // namespace

int wilson_prepare(Ctx *ctx, GaugeField *f, const double *links_dev, hipStream_t s)
{
    const Geom &g = f->g;
    const int64_t n = (int64_t)2 * 8 * g.Vh;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    int *flags = (int *)ctx->arena.alloc(256);
    if (!flags)
        return set_error(STAG_ENOMEM, "arena exhausted (gauge check flags)");
    int hflags = 0;
    hipError_t e = hipMemsetAsync(flags, 0, sizeof(int), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_wcheck_links, grid, block, 0, s, g, links_dev, kTwoRowTolerance, flags);
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
    const char *rows_env = getenv("STAG_LINK_ROWS");
    f->rows = (hflags & 2) == 0 && !(rows_env && atoi(rows_env) == 3) ? 2 : 3;
    const size_t lb = (size_t)2 * link_parity_entries(f->rows, g.Vh) * 16;
    f->links[0] = ctx->arena.alloc(lb);
    if (!f->links[0])
        return set_error(STAG_ENOMEM, "arena exhausted (%zu bytes of Wilson links)", lb);
    f->bytes = lb;
    f->nt_links = nt_links_for(*f);
    if (f->rows == 2)
        hipLaunchKernelGGL((k_wprepare_links<2>), grid, block, 0, s, g, links_dev, (dbl2 *)f->links[0]);
    else
        hipLaunchKernelGGL((k_wprepare_links<3>), grid, block, 0, s, g, links_dev, (dbl2 *)f->links[0]);
    e = hipGetLastError();
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        ctx->arena.release(f->links[0]);
        f->links[0] = nullptr;
        return set_error(STAG_EHIP, "Wilson gauge preparation failed: %s", hipGetErrorString(e));
    }
    return STAG_OK;
}

int launch_pack_spinor(const Geom &g, const double *lex, double *eo, int to_eo, hipStream_t s)
{
    const int64_t n = (int64_t)2 * g.Vh;
    hipLaunchKernelGGL(k_pack_spinor, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g,
                       (dbl2 *)const_cast<double *>(lex), (dbl2 *)eo, to_eo);
    STAG_HIP_CHECK(hipGetLastError());
    return STAG_OK;
}

namespace {

// The launches of the hop and of one solve, for one link format and one
// number of lanes per site.
template <int ROWS, int LPS, class LP> struct WLaunch {
    static dim3 grid(int Vh, int ny = 1) { return dim3((unsigned)(((int64_t)Vh * LPS + kWBlock - 1) / kWBlock), ny); }
    static void hop(const GaugeField *f, int pf, const double *in, double *out, int remap, hipStream_t s)
    {
        hipLaunchKernelGGL((wil::k_wilson_dslash<ROWS, LPS, LP>), grid(f->g.Vh, pf < 0 ? 2 : 1), dim3(kWBlock), 0, s, f->g,
                           (const dbl2 *)f->links[0], (const dbl2 *)in, (dbl2 *)out, pf, remap);
    }
    static void init(const wil::WArgs &a, hipStream_t s)
    {
        const dim3 g = grid(a.g.Vh);
        hipLaunchKernelGGL((wil::k_wil_bhat<ROWS, LPS, LP>), g, dim3(kWBlock), 0, s, a);
        hipLaunchKernelGGL((wil::k_wil_odd_g5<ROWS, LPS, LP>), g, dim3(kWBlock), 0, s, a, (const dbl2 *)a.bh, 0, 0);
        hipLaunchKernelGGL((wil::k_wil_init<ROWS, LPS, LP>), g, dim3(kWBlock), 0, s, a);
    }
    static void step(const wil::WArgs &a, hipStream_t s, int ver)
    {
        const dim3 g = grid(a.g.Vh);
        hipLaunchKernelGGL((wil::k_wil_step1<ROWS, LPS, LP>), g, dim3(kWBlock), 0, s, a, ver);
        hipLaunchKernelGGL((wil::k_wil_step2<ROWS, LPS, LP>), g, dim3(kWBlock), 0, s, a, ver);
        hipLaunchKernelGGL((wil::k_wil_odd_g5<ROWS, LPS, LP>), g, dim3(kWBlock), 0, s, a, (const dbl2 *)a.ap, ver, 1);
        hipLaunchKernelGGL((wil::k_wil_step4<ROWS, LPS, LP>), g, dim3(kWBlock), 0, s, a, ver);
    }
    static void finish(const wil::WArgs &a, hipStream_t s)
    {
        const dim3 g = grid(a.g.Vh);
        hipLaunchKernelGGL((wil::k_wil_xodd<ROWS, LPS, LP>), g, dim3(kWBlock), 0, s, a);
        hipLaunchKernelGGL((wil::k_wil_resid<ROWS, LPS, LP>), g, dim3(kWBlock), 0, s, a, 0);
        hipLaunchKernelGGL((wil::k_wil_resid<ROWS, LPS, LP>), g, dim3(kWBlock), 0, s, a, 1);
    }
};

struct WTable {
    void (*hop)(const GaugeField *, int, const double *, double *, int, hipStream_t);
    void (*init)(const wil::WArgs &, hipStream_t);
    void (*step)(const wil::WArgs &, hipStream_t, int);
    void (*finish)(const wil::WArgs &, hipStream_t);
};

template <int ROWS, int LPS, class LP> constexpr WTable wtable()
{
    using W = WLaunch<ROWS, LPS, LP>;
    return {W::hop, W::init, W::step, W::finish};
}

constexpr int kWLps[4] = {1, 2, 4, 8};

template <class LP> const WTable &wilson_table_of(int rows, int lps)
{
    static const WTable t[2][4] = {{wtable<2, 1, LP>(), wtable<2, 2, LP>(), wtable<2, 4, LP>(), wtable<2, 8, LP>()},
                                   {wtable<3, 1, LP>(), wtable<3, 2, LP>(), wtable<3, 4, LP>(), wtable<3, 8, LP>()}};
    return t[rows == 2 ? 0 : 1][lps == 1 ? 0 : lps == 2 ? 1 : lps == 4 ? 2 : 3];
}

// The launches for a field: its link format, the lanes per site and its
// choice of link loads (nt_links)
const WTable &wilson_table(const GaugeField *f, int lps)
{
    return f->nt_links ? wilson_table_of<PrecF64NT>(f->rows, lps) : wilson_table_of<PrecF64>(f->rows, lps);
}

// Lanes per site and block order (XCD-contiguous or not) for the Wilson
// kernels of a field: STAG_WILSON_LPS fixes the lanes, else the fastest hop
// on two full-field vectors of scratch (`in`, `out`, each [2][12][Vh]), timed
// once per field (by its first solve or first standalone hop); 4 lanes and
// the XCD order when no scratch is given.
KernelCfg wilson_cfg(Ctx *ctx, GaugeField *f, const double *in, double *out, hipStream_t s)
{
    const uint64_t key = (uint64_t)3 << 40;
    int lps_env = 0;
    if (const char *e = getenv("STAG_WILSON_LPS")) {
        const int v = atoi(e);
        if (v == 1 || v == 2 || v == 4 || v == 8)
            lps_env = v;
    }
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = f->tuned.find(key);
        if (it != f->tuned.end() && (!lps_env || it->second.lps == lps_env))
            return it->second;
    }
    KernelCfg best;
    best.lps = lps_env ? lps_env : 4;
    best.remap = 1;
    if (!in || !out)
        return best;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0)
            (void)hipEventDestroy(e0);
        return best;
    }
    // timed on one parity (half the sites), the work of each CG kernel: a
    // count that fills the GPU for the whole lattice can leave it half idle
    // there
    float best_ms = 1e30f;
    const int reps = 5;
    for (int L : kWLps) {
        if (lps_env && L != lps_env)
            continue;
        for (int remap = 1; remap >= 0; --remap) {
            const WTable &t = wilson_table(f, L);
            t.hop(f, 0, in, out, remap, s);
            (void)hipEventRecord(e0, s);
            for (int i = 0; i < reps; ++i)
                t.hop(f, 0, in, out, remap, s);
            (void)hipEventRecord(e1, s);
            float ms = 0.f;
            if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
                ms < best_ms * 0.97f) {
                best_ms = ms;
                best.lps = L;
                best.remap = remap;
            }
            if (getenv("STAG_TUNE_VERBOSE"))
                fprintf(stderr, "[stag tune wilson] V=%d lps=%d remap=%d: %.2f us per parity\n", 2 * f->g.Vh, L,
                        remap, ms * 1e3 / reps);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(ctx->mu);
    f->tuned[key] = best;
    return best;
}

}  // namespace

int wilson_dslash(Ctx *ctx, GaugeField *f, int out_parity, const double *in, double *out, hipStream_t s)
{
    bool tuned;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        tuned = f->tuned.count((uint64_t)3 << 40) != 0;
    }
    KernelCfg c = wilson_cfg(ctx, f, nullptr, nullptr, s);
    if (!tuned) {
        // the first hop of a field times the shapes on two scratch vectors
        // from the arena (as the first solve does on its workspace); without
        // the room, the defaults
        const size_t full = (size_t)2 * 12 * f->g.Vh * sizeof(dbl2);
        char *scratch = (char *)ctx->arena.alloc(2 * full);
        if (scratch) {
            if (hipMemsetAsync(scratch, 0, full, s) == hipSuccess)
                c = wilson_cfg(ctx, f, (const double *)scratch, (double *)(scratch + full), s);
            (void)hipStreamSynchronize(s);
            ctx->arena.release(scratch);
        }
    }
    wilson_table(f, c.lps).hop(f, out_parity == STAG_ALL ? -1 : out_parity, in, out, c.remap, s);
    STAG_HIP_CHECK(hipGetLastError());
    return STAG_OK;
}

int wilson_cg_solve(Ctx *ctx, GaugeField *f, double kappa, double tol, int maxiter, const double *b, double *x,
                    hipStream_t s, stag_cg_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    const Geom &g = f->g;
    const int Vh = g.Vh;
    // partial sums sized for the most lanes per site (the most blocks)
    const int nblk_max = (int)(((int64_t)Vh * 8 + kWBlock - 1) / kWBlock);
    const int pstride = (nblk_max + 63) & ~63;
    const size_t vec = (size_t)12 * Vh * sizeof(dbl2);
    const size_t bytes = 6 * vec + 256 + (size_t)4 * pstride * sizeof(double);
    char *mem = (char *)ctx->arena.alloc(bytes);
    if (!mem)
        return set_error(STAG_ENOMEM, "arena exhausted: Wilson CG workspace needs %zu bytes", bytes);
    struct Release {
        Arena &arena;
        void *p;
        hipStream_t s;
        ~Release()
        {
            (void)hipStreamSynchronize(s);
            arena.release(p);
        }
    } release{ctx->arena, mem, s};
    wil::WArgs a;
    memset(&a, 0, sizeof(a));
    a.g = g;
    a.links[0] = (const dbl2 *)f->links[0];
    a.links[1] = (const dbl2 *)f->links[0] + link_parity_entries(f->rows, Vh);
    a.kappa = kappa;
    a.b = (const dbl2 *)b;
    a.x = (dbl2 *)x;
    a.bh = (dbl2 *)mem;
    a.r = (dbl2 *)(mem + vec);
    a.p[0] = (dbl2 *)(mem + 2 * vec);
    a.p[1] = (dbl2 *)(mem + 3 * vec);
    a.ap = (dbl2 *)(mem + 4 * vec);
    a.t = (dbl2 *)(mem + 5 * vec);
    a.st[0] = (wil::WState *)(mem + 6 * vec);
    a.st[1] = a.st[0] + 1;
    a.partials = (double *)(mem + 6 * vec + 256);
    a.pstride = pstride;

    wil::WState *host = nullptr;
    STAG_HIP_CHECK(hipHostMalloc((void **)&host, 4 * sizeof(wil::WState), hipHostMallocDefault));
    std::vector<double> hpart(2 * (size_t)nblk_max);
    hipEvent_t ev = nullptr;
    struct HostRelease {
        wil::WState *h;
        hipEvent_t *e;
        ~HostRelease()
        {
            if (*e)
                (void)hipEventDestroy(*e);
            (void)hipHostFree(h);
        }
    } host_release{host, &ev};
    STAG_HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    memset(host, 0, 4 * sizeof(wil::WState));
    host[0].mode = wil::W_INIT;
    host[0].tol2 = tol * tol;
    host[0].maxiter = maxiter;
    host[1] = host[0];
    STAG_HIP_CHECK(hipMemcpyAsync(a.st[0], host, 2 * sizeof(wil::WState), hipMemcpyHostToDevice, s));

    // lanes per site: tuned on this workspace (bh|r and p[0]|p[1] are two
    // adjacent full-field vectors) before the solve uses it
    const KernelCfg cfg = wilson_cfg(ctx, f, (const double *)a.bh, (double *)a.p[0], s);
    const int lps = cfg.lps;
    a.remap = cfg.remap;
    const WTable &tab = wilson_table(f, lps);
    const int nblk = (int)(((int64_t)Vh * lps + kWBlock - 1) / kWBlock);
    tab.init(a, s);
    STAG_HIP_CHECK(hipGetLastError());
    // epochs of E iterations; the state after epoch n is read while epoch n+1 runs
    const int E = 16;
    int64_t it = 0;
    auto epoch = [&]() {
        for (int k = 0; k < E; ++k, ++it)
            tab.step(a, s, (int)(it & 1));
    };
    auto snapshot = [&]() -> hipError_t {
        hipError_t e = hipMemcpyAsync(host + 2, a.st[0], 2 * sizeof(wil::WState), hipMemcpyDeviceToHost, s);
        return e == hipSuccess ? hipEventRecord(ev, s) : e;
    };
    epoch();
    STAG_HIP_CHECK(snapshot());
    const int64_t budget = (int64_t)maxiter + 2 * E + 1;
    wil::WState last{};
    bool done = false;
    while (!done) {
        if (it < budget)
            epoch();
        STAG_HIP_CHECK(hipGetLastError());
        STAG_HIP_CHECK(hipEventSynchronize(ev));
        last = host[3].step > host[2].step ? host[3] : host[2];
        done = last.mode == wil::W_DONE || it >= budget;
        if (!done)
            STAG_HIP_CHECK(snapshot());
    }
    STAG_HIP_CHECK(hipMemcpyAsync(host + 2, a.st[0], 2 * sizeof(wil::WState), hipMemcpyDeviceToHost, s));
    tab.finish(a, s);
    STAG_HIP_CHECK(hipGetLastError());
    // |b - M x|^2 (slots 0 and 1 of buffer 0), then |b|^2 into buffer 1
    STAG_HIP_CHECK(hipMemcpyAsync(hpart.data(), a.partials, nblk * sizeof(double), hipMemcpyDeviceToHost, s));
    STAG_HIP_CHECK(hipMemcpyAsync(hpart.data() + nblk, a.partials + pstride, nblk * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
    STAG_HIP_CHECK(hipStreamSynchronize(s));
    double res2 = 0.0;
    for (int i = 0; i < 2 * nblk; ++i)
        res2 += hpart[i];
    const int nb2 = 256;
    double *bpart = a.partials + (size_t)2 * pstride;
    hipLaunchKernelGGL(k_norm2_partials, dim3(nb2 < 2 * pstride ? nb2 : 2 * pstride), dim3(256), 0, s,
                       (const dbl2 *)b, (int64_t)24 * Vh, bpart);
    STAG_HIP_CHECK(hipGetLastError());
    const int nb2u = nb2 < 2 * pstride ? nb2 : 2 * pstride;
    std::vector<double> hb(nb2u);
    STAG_HIP_CHECK(hipMemcpyAsync(hb.data(), bpart, nb2u * sizeof(double), hipMemcpyDeviceToHost, s));
    STAG_HIP_CHECK(hipStreamSynchronize(s));
    double bb = 0.0;
    for (double v : hb)
        bb += v;
    last = host[3].step > host[2].step ? host[3] : host[2];
    stag_cg_info inf;
    memset(&inf, 0, sizeof(inf));
    inf.status = last.mode == wil::W_DONE ? last.status : STAG_ENOCONV;
    inf.iters = last.iters;
    inf.iters_parity[0] = last.iters;  // the CG runs on the even sites
    inf.iters_parity[1] = -1;
    inf.true_rel_resid = bb > 0 ? std::sqrt(res2 / bb) : 0.0;
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info)
        *info = inf;
    if (inf.status != STAG_OK)
        return set_error(inf.status, "Wilson CG did not converge (status %d)", inf.status);
    return STAG_OK;
}

}  // namespace stag
