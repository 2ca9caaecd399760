// The standalone D_slash (the paper's matrix-vector routine of Sec. 3,
// `matrix-vector(offset, local_length, v, w)`, restricted to one parity or
// applied to the whole lattice) in FP64, FP32 or FP16, conversion of fermion
// fields between those storage precisions, and the kernel-configuration tuner.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "cg_launch.hpp"
#include "runtime.hpp"

namespace stag {

const CgLaunchTable &cg_table_f64();
const CgLaunchTable &cg_table_f32();
const CgLaunchTable &cg_table_f16();
const CgLaunchTable &cg_table_f64_r2();
const CgLaunchTable &cg_table_f32_r2();
const CgLaunchTable &cg_table_f16_r2();
const CgLaunchTable &cg_table_f64nt();
const CgLaunchTable &cg_table_f64nt_r2();

const CgLaunchTable &cg_table(int prec, int rows, int nt_links)
{
    if (prec == 0 && nt_links)
        return rows == 2 ? cg_table_f64nt_r2() : cg_table_f64nt();
    if (rows == 2)
        return prec == 0 ? cg_table_f64_r2() : prec == 1 ? cg_table_f32_r2() : cg_table_f16_r2();
    return prec == 0 ? cg_table_f64() : prec == 1 ? cg_table_f32() : cg_table_f16();
}

namespace {

// out(x) (+)= (D in)(x) for checkerboard sites [offset, offset + count) of the
// output parity (blockIdx.y selects the parity when par_fixed < 0), with
// links, vectors and arithmetic of precision P: FP64 / FP32 vectors are
// [parity][colour][Vh] complex, FP16 vectors [parity][Vh] records of three
// scaled half2 colours and their FP32 scale.
template <class P, int LPS, int ROWS>
__global__ void __launch_bounds__(256)
k_dslash(Geom g, const typename P::link_t *__restrict__ links, const int32_t *__restrict__ nbr,
         const void *__restrict__ in, void *__restrict__ out, int par_fixed, int offset, int count, int accumulate,
         int remap)
{
    using real = typename P::real;
    const int p = par_fixed >= 0 ? par_fixed : (int)blockIdx.y;
    const int Vh = g.Vh;
    int site, sub;
    site_of_thread<LPS>(logical_block(blockIdx.x, gridDim.x, remap) * blockDim.x + threadIdx.x, site, sub);
    if (site >= count)
        return;
    const int s = offset + site;
    const size_t half = (size_t)Vh * P::spinor_bytes;  // bytes of one parity half
    const char *src = (const char *)in + (size_t)(1 - p) * half;
    cplx<real> acc[1][3] = {{czero<real>(), czero<real>(), czero<real>()}};
    auto load = [&](int, int n, cplx<real> *chi) { P::load_spinor(src, Vh, n, chi); };
    hop_accumulate<P, LPS, 1, decltype(load), false, ROWS>(g, links + link_parity_entries(ROWS, Vh) * p,
                                                           nbr ? nbr + (size_t)p * 8 * Vh : nullptr, p, s, sub, acc,
                                                           load);
    char *o = (char *)out + (size_t)p * half;
    if constexpr (P::id == 2) {
        // one lane writes the whole record (every lane holds the lane sum)
        if (sub != 0)
            return;
        if (accumulate) {
            cplx<real> old[3];
            P::load_spinor(o, Vh, s, old);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                acc[0][c].re += old[c].re;
                acc[0][c].im += old[c].im;
            }
        }
        P::store_spinor(o, Vh, s, acc[0]);
    } else {
        using v2 = typename vec2_of<real>::type;
        v2 *ov = (v2 *)o;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (!owns_colour<LPS>(sub, c))
                continue;
            v2 v = v2{acc[0][c].re, acc[0][c].im};
            if (accumulate)
                v += ov[(int64_t)c * Vh + s];
            ov[(int64_t)c * Vh + s] = v;
        }
    }
}

// Convert a full-lattice field (both parities, 2 Vh sites) between vector
// storage precisions: FP64 / FP32 [parity][colour][Vh] complex, FP16
// [parity][Vh] records.  One thread per site.
template <class PI, class PO>
__global__ void __launch_bounds__(256) k_convert(int Vh, const void *__restrict__ in, void *__restrict__ out)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)2 * Vh)
        return;
    const int p = (int)(gid / Vh), s = (int)(gid % Vh);
    const char *ib = (const char *)in + (size_t)p * Vh * PI::spinor_bytes;
    char *ob = (char *)out + (size_t)p * Vh * PO::spinor_bytes;
    cplx<typename PI::real> v[3];
    PI::load_spinor(ib, Vh, s, v);
    cplx<typename PO::real> w[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        w[c] = {(typename PO::real)v[c].re, (typename PO::real)v[c].im};
    PO::store_spinor(ob, Vh, s, w);
}

template <class P>
hipError_t launch_dslash_p(const KernelCfg &cfg, const GaugeField *f, int par_fixed, int nparity, int offset,
                           int count, const void *in, void *out, int accumulate, hipStream_t s)
{
    const int64_t threads = (int64_t)count * cfg.lps;  // site = wave * (64/lps) + lane % (64/lps)
    dim3 grid((unsigned)((threads + cfg.block - 1) / cfg.block), (unsigned)nparity);
    dim3 block(cfg.block);
    const auto *lk = (const typename P::link_t *)f->links[P::id];
    const int32_t *nb = cfg.tables ? f->nbr : nullptr;
#define STAG_DSLASH_CASE(L, ROWS)                                                                                    \
    hipLaunchKernelGGL((k_dslash<P, L, ROWS>), grid, block, 0, s, f->g, lk, nb, in, out, par_fixed, offset, count,  \
                       accumulate, cfg.remap)
    const int key = cfg.lps * 4 + f->rows;
    switch (key) {
    case 1 * 4 + 3: STAG_DSLASH_CASE(1, 3); break;
    case 2 * 4 + 3: STAG_DSLASH_CASE(2, 3); break;
    case 4 * 4 + 3: STAG_DSLASH_CASE(4, 3); break;
    case 8 * 4 + 3: STAG_DSLASH_CASE(8, 3); break;
    case 1 * 4 + 2: STAG_DSLASH_CASE(1, 2); break;
    case 2 * 4 + 2: STAG_DSLASH_CASE(2, 2); break;
    case 4 * 4 + 2: STAG_DSLASH_CASE(4, 2); break;
    case 8 * 4 + 2: STAG_DSLASH_CASE(8, 2); break;
    default: return hipErrorInvalidValue;
    }
#undef STAG_DSLASH_CASE
    return hipGetLastError();
}

}  // namespace

int dslash(Ctx *ctx, GaugeField *f, int prec, int out_parity, int64_t offset, int64_t count, const void *in,
           void *out, int accumulate, hipStream_t s)
{
    return dslash_with(tune_config(ctx, f, prec, 1, s), f, prec, out_parity, offset, count, in, out, accumulate, s);
}

int dslash_with(const KernelCfg &cfg, GaugeField *f, int prec, int out_parity, int64_t offset, int64_t count,
                const void *in, void *out, int accumulate, hipStream_t s)
{
    const int Vh = f->g.Vh;
    const int par_fixed = out_parity == STAG_ALL ? -1 : out_parity;
    const int nparity = out_parity == STAG_ALL ? 2 : 1;
    const int off = out_parity == STAG_ALL ? 0 : (int)offset;
    const int cnt = out_parity == STAG_ALL ? Vh : (int)count;
    hipError_t e;
    switch (prec) {
    case 0:
        e = f->nt_links ? launch_dslash_p<PrecF64NT>(cfg, f, par_fixed, nparity, off, cnt, in, out, accumulate, s)
                        : launch_dslash_p<PrecF64>(cfg, f, par_fixed, nparity, off, cnt, in, out, accumulate, s);
        break;
    case 1: e = launch_dslash_p<PrecF32>(cfg, f, par_fixed, nparity, off, cnt, in, out, accumulate, s); break;
    case 2: e = launch_dslash_p<PrecF16>(cfg, f, par_fixed, nparity, off, cnt, in, out, accumulate, s); break;
    default: return set_error(STAG_EINVAL, "dslash: unknown precision %d", prec);
    }
    if (e != hipSuccess)
        return set_error(STAG_EHIP, "dslash launch failed: %s", hipGetErrorString(e));
    return STAG_OK;
}

int dslash_f64(Ctx *ctx, GaugeField *f, int out_parity, int64_t offset, int64_t count, const double *in,
               double *out, int accumulate, hipStream_t s)
{
    return dslash(ctx, f, 0, out_parity, offset, count, in, out, accumulate, s);
}

int convert_fermion(const Geom &g, int prec_in, const void *in, int prec_out, void *out, hipStream_t s)
{
    const int64_t n = (int64_t)2 * g.Vh;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
#define STAG_CONVERT_CASE(PI, PO) hipLaunchKernelGGL((k_convert<PI, PO>), grid, block, 0, s, g.Vh, in, out)
    switch (prec_in * 3 + prec_out) {
    case 0: STAG_CONVERT_CASE(PrecF64, PrecF64); break;
    case 1: STAG_CONVERT_CASE(PrecF64, PrecF32); break;
    case 2: STAG_CONVERT_CASE(PrecF64, PrecF16); break;
    case 3: STAG_CONVERT_CASE(PrecF32, PrecF64); break;
    case 4: STAG_CONVERT_CASE(PrecF32, PrecF32); break;
    case 5: STAG_CONVERT_CASE(PrecF32, PrecF16); break;
    case 6: STAG_CONVERT_CASE(PrecF16, PrecF64); break;
    case 7: STAG_CONVERT_CASE(PrecF16, PrecF32); break;
    case 8: STAG_CONVERT_CASE(PrecF16, PrecF16); break;
    default: return set_error(STAG_EINVAL, "convert: unknown precision");
    }
#undef STAG_CONVERT_CASE
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(STAG_EHIP, "convert launch failed: %s", hipGetErrorString(e));
    return STAG_OK;
}

// ---- tuner ----------------------------------------------------------------------

static bool env_cfg(KernelCfg &c)
{
    const char *e = getenv("STAG_KERNEL_CFG");  // "lps,block,rtile,tables,remap"
    if (!e || !*e)
        return false;
    int v[5];
    if (sscanf(e, "%d,%d,%d,%d,%d", &v[0], &v[1], &v[2], &v[3], &v[4]) != 5)
        return false;
    c.lps = v[0];
    c.block = v[1];
    c.rtile = v[2];
    c.tables = v[3];
    c.remap = v[4];
    return true;
}

static bool valid_lps(int l) { return l == 1 || l == 2 || l == 4 || l == 8; }

static int default_rtile(const CgLaunchTable &t, int nrhs)
{
    int best = 1;
    for (int i = 0; i < t.n_rtiles; ++i)
        if (nrhs % t.rtiles[i] == 0)
            best = std::max(best, t.rtiles[i]);
    return best;
}

static KernelCfg default_config(const GaugeField *f, int prec, int nrhs)
{
    KernelCfg best;
    best.lps = prec == 0 ? 2 : 1;
    best.block = 256;
    best.rtile = default_rtile(cg_table(prec, f->rows, f->nt_links), nrhs);
    best.tables = 0;
    best.remap = 1;
    return best;
}

KernelCfg cached_config(Ctx *ctx, GaugeField *f, int prec, int nrhs)
{
    const uint64_t key = ((uint64_t)prec << 32) | (uint32_t)nrhs;
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = f->tuned.find(key);
    return it != f->tuned.end() ? it->second : default_config(f, prec, nrhs);
}

KernelCfg tune_config(Ctx *ctx, GaugeField *f, int prec, int nrhs, hipStream_t s)
{
    const uint64_t key = ((uint64_t)prec << 32) | (uint32_t)nrhs;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = f->tuned.find(key);
        if (it != f->tuned.end())
            return it->second;
    }
    const CgLaunchTable &tab = cg_table(prec, f->rows, f->nt_links);
    KernelCfg best = default_config(f, prec, nrhs);
    KernelCfg forced;
    const char *tune_env = getenv("STAG_TUNE");
    const bool tune = !(tune_env && tune_env[0] == '0');
    if (env_cfg(forced)) {
        if (valid_lps(forced.lps) && forced.block >= 64 && forced.block <= 256 && forced.block % 64 == 0 &&
            nrhs % forced.rtile == 0)
            best = forced;
    } else if (tune) {
        // time out_r = D in_r on scratch vectors for every candidate; keep the
        // fastest per right-hand side
        std::vector<int> tiles;
        for (int i = 0; i < tab.n_rtiles; ++i)
            if (nrhs % tab.rtiles[i] == 0)
                tiles.push_back(tab.rtiles[i]);
        const bool verbose = getenv("STAG_TUNE_VERBOSE") != nullptr;
        // scratch vectors for every system of the solve shape (2 parities x nrhs)
        const size_t vbytes = (size_t)f->g.Vh * spinor_bytes_of(prec) * 2 * nrhs;
        void *in = ctx->arena.alloc(vbytes), *out = ctx->arena.alloc(vbytes);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        bool ok = in && out && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
                  hipMemsetAsync(in, 0, vbytes, s) == hipSuccess;
        double best_t = 1e30;
        const int lps_c[4] = {1, 2, 4, 8}, blk_c[3] = {64, 128, 256};
        for (int R : tiles) {
            for (int L : lps_c) {
                for (int B : blk_c) {
                    for (int T = 0; T < 2 && ok; ++T) {
                        for (int X = 0; X < 2 && ok; ++X) {
                            const int64_t threads = (int64_t)f->g.Vh * L;
                            dim3 grid((unsigned)((threads + B - 1) / B), (unsigned)(2 * nrhs / R)), block(B);
                            const void *links = f->links_for(prec, 0);
                            const int32_t *nb = T ? f->nbr_for(0) : nullptr;
                            auto run = [&]() { return tab.probe(L, R, grid, block, s, f->g, links, nb, in, out, X); };
                            if (run() != hipSuccess) {
                                ok = false;
                                break;
                            }
                            const int reps = 4;
                            (void)hipEventRecord(e0, s);
                            for (int i = 0; i < reps; ++i)
                                (void)run();
                            (void)hipEventRecord(e1, s);
                            if (hipEventSynchronize(e1) != hipSuccess) {
                                ok = false;
                                break;
                            }
                            float ms = 0.f;
                            (void)hipEventElapsedTime(&ms, e0, e1);
                            const double per_rhs = ms / reps / nrhs;
                            if (verbose)
                                fprintf(stderr, "[stag tune] V=%d prec=%d nrhs=%d lps=%d block=%d rtile=%d tables=%d "
                                                "remap=%d: %.2f us per rhs\n",
                                        2 * f->g.Vh, prec, nrhs, L, B, R, T, X, per_rhs * 1e3);
                            if (per_rhs < best_t * 0.995) {
                                best_t = per_rhs;
                                best.lps = L;
                                best.block = B;
                                best.rtile = R;
                                best.tables = T;
                                best.remap = X;
                            }
                        }
                    }
                }
            }
        }
        if (e0)
            (void)hipEventDestroy(e0);
        if (e1)
            (void)hipEventDestroy(e1);
        ctx->arena.release(in);
        ctx->arena.release(out);
        (void)hipGetLastError();
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    f->tuned[key] = best;
    return best;
}

}  // namespace stag
