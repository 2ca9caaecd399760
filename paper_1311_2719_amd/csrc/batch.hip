// Batch workspace and the per-iteration launch sequence; the blocking
// (batched) CG solve built on it.
#include <algorithm>
#include <chrono>
#include <map>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>

#include "batch.hpp"

namespace stag {

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static int blocks_for(int Vh, int lps, int block) { return (int)(((int64_t)Vh * lps + block - 1) / block); }

Batch::Batch(Ctx *ctx, std::shared_ptr<GaugeField> f, int prec, int slots, hipStream_t s)
    : ctx_(ctx), f_(std::move(f)), prec_(prec), S_(slots), s_(s)
{
}

Batch::~Batch()
{
    if (s_ || mem_)
        (void)hipStreamSynchronize(s_);  // no kernel may still use the workspace
    for (auto &kv : graphs_)
        (void)hipGraphExecDestroy(kv.second);
    if (cap_stream_)
        (void)hipStreamDestroy(cap_stream_);
    if (snap_ev_)
        (void)hipEventDestroy(snap_ev_);
    for (auto &e : tune_ev_)
        if (e)
            (void)hipEventDestroy(e);
    if (stage_ev_)
        (void)hipEventDestroy(stage_ev_);
    if (stage_ && !external_)
        (void)hipHostFree(stage_);
    if (mem_ && !external_)
        ctx_->arena.release(mem_);
}

size_t Batch::workspace_bytes(const Geom &g, int prec, int slots, int pstride)
{
    const size_t nsys = 2 * (size_t)slots, Vh = g.Vh;
    size_t b = 0;
    b += align256(nsys * Vh * spinor_bytes_of(prec)) * 3;       // p (two buffers), ap
    b += align256(nsys * 3 * Vh * (prec == 0 ? 16 : 8));         // r
    b += prec == 0 ? 0 : align256(nsys * 3 * Vh * 8);            // x_lo
    b += align256(nsys * 3 * Vh * 16);                           // tmp
    b += align256(nsys * sizeof(void *)) * 2;                    // pointer tables
    b += align256(nsys * sizeof(SysState)) * 2;                  // two state buffers
    b += align256(nsys * sizeof(int));                           // tile order
    b += align256(2 * nsys * 3 * (size_t)pstride * sizeof(double));  // partials
    b += align256(2 * nsys * 3 * sizeof(double));                    // their totals
    return b;
}

// Blocks that cover the sites of one parity once with shape c: a register
// tile takes block / lps sites, a shared-link block one chunk of 64.
static int blocks_needed(const Geom &g, const KernelCfg &c)
{
    return c.shared ? (g.Vh + kChunk - 1) / kChunk : blocks_for(g.Vh, c.lps, c.block);
}

// Largest grid row of a register-tile shape with a reduction kernel; the
// shared-link shapes may use the whole partial-sum slot.
constexpr int kTileGridCap = 2048;

// Blocks per tile row of shape c: enough to cover the sites once (the
// kernels stride over the sites when capped).  Without a reduction kernel the
// count is capped so that the partial sums every block reads back in the next
// kernel's prologue stay few; with one, by kTileGridCap (register tiles) or
// the partial buffer (shared-link tiles).  The tuned shape's count becomes the
// batch's fixed count (nblk_).
int Batch::grid_x(const KernelCfg &c) const
{
    const int need = blocks_needed(f_->g, c);
    if (uses_reduction(c))
        return std::min(need, c.shared ? pstride_ : std::min(pstride_, kTileGridCap));
    return std::min(need, std::max(128, 2048 / c.rtile));
}

// Whether shape c runs a reduction kernel between its step kernels: as the
// tuner chose (it times both), else once every prologue would sum about a
// thousand partials per slot set (the reduction costs one small launch after
// each step kernel).
bool cg_uses_reduction(const Geom &g, const KernelCfg &c)
{
    if (const char *e = getenv("STAG_CG_REDUCE"))  // "1": always, "0": never (tests, experiments)
        if (e[0] == '0' || e[0] == '1')
            return e[0] == '1';
    if (c.reduce >= 0)
        return c.reduce != 0;
    const int need = blocks_needed(g, c);
    const int fused = std::min(need, std::max(128, 2048 / c.rtile));
    return (int64_t)fused * c.rtile >= 1024;
}

bool Batch::uses_reduction(const KernelCfg &c) const { return cg_uses_reduction(f_->g, c); }

bool cg_tuned_shape(Ctx *ctx, const GaugeField *f, int prec, int slots, KernelCfg &out, bool &reduce)
{
    const uint64_t key = ((uint64_t)1 << 40) | ((uint64_t)prec << 32) | (uint32_t)slots;
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = f->tuned.find(key);
    if (it == f->tuned.end())
        return false;
    out = it->second;
    reduce = cg_uses_reduction(f->g, out);
    return true;
}

namespace {
// Total of the per-block partials [0, nblk) of slot slot0 + blockIdx.y of
// partial buffer buf, system blockIdx.x, in a fixed order, into that slot's
// entry of `totals` ([2 buffers][nsys][3 slots]).  Partials are only read, so
// running it again over unchanged partials gives the same totals.
__global__ void __launch_bounds__(256) k_cg_reduce(const double *partials, double *totals, int nsys, int pstride,
                                                   int buf, int slot0, int nblk)
{
    __shared__ double lds[4];
    const size_t k = ((size_t)buf * nsys + blockIdx.x) * 3 + slot0 + blockIdx.y;
    const double t = reduce_partials(partials + k * pstride, nblk, lds);
    if (threadIdx.x == 0)
        totals[k] = t;
}
}  // namespace

hipError_t Batch::launch_reduce(hipStream_t st, int buf, int slot0, int nslots, int nblk) const
{
    hipLaunchKernelGGL(k_cg_reduce, dim3((unsigned)nsys(), (unsigned)nslots), dim3(256), 0, st, partials_, totals_,
                       nsys(), pstride_, buf, slot0, nblk);
    return hipGetLastError();
}

size_t Batch::host_bytes_for(int slots)
{
    const size_t nsys = 2 * (size_t)slots;
    return 3 * nsys * sizeof(SysState) + 2 * nsys * sizeof(void *) + nsys * sizeof(int);
}

// Partial sums per slot: the widest grid row any shape may use (register
// tiles: kTileGridCap; shared-link tiles: up to 4096 chunks of 64 sites).
static int pstride_for(const Geom &g)
{
    const int p = std::min(4096, std::max(std::min(kTileGridCap, blocks_for(g.Vh, 8, 64)), (g.Vh + kChunk - 1) / kChunk));
    return (p + 63) & ~63;
}

size_t Batch::needed_bytes() const { return workspace_bytes(f_->g, prec_, S_, pstride_for(f_->g)); }

void Batch::carve(void *base)
{
    const Geom &g = f_->g;
    const size_t nsys = 2 * (size_t)S_, Vh = g.Vh;
    char *c = (char *)base;
    auto take = [&](size_t n) {
        char *r = c;
        c += align256(n);
        return (void *)r;
    };
    p_[0] = take(nsys * Vh * spinor_bytes_of(prec_));
    p_[1] = take(nsys * Vh * spinor_bytes_of(prec_));
    ap_ = take(nsys * Vh * spinor_bytes_of(prec_));
    r_ = take(nsys * 3 * Vh * (prec_ == 0 ? 16 : 8));
    xlo_ = prec_ == 0 ? nullptr : (flt2 *)take(nsys * 3 * Vh * 8);
    tmp_ = (dbl2 *)take(nsys * 3 * Vh * 16);
    xhi_d_ = (dbl2 **)take(nsys * sizeof(void *));
    b_d_ = (const dbl2 **)take(nsys * sizeof(void *));
    // the two state buffers are adjacent, so one copy takes a snapshot of both
    st_d_[0] = (SysState *)take(2 * nsys * sizeof(SysState));
    st_d_[1] = st_d_[0] + nsys;
    perm_d_ = (int *)take(nsys * sizeof(int));
    partials_ = (double *)take(2 * nsys * 3 * (size_t)pstride_ * sizeof(double));
    totals_ = (double *)take(2 * nsys * 3 * sizeof(double));
}

int Batch::mark_stage()
{
    if (!external_)
        STAG_HIP_CHECK(hipEventRecord(stage_ev_, s_));
    stage_busy_ = true;
    return STAG_OK;
}

void Batch::wait_stage()
{
    if (!stage_busy_)
        return;
    if (external_)
        (void)hipStreamSynchronize(s_);
    else
        (void)hipEventSynchronize(stage_ev_);
    stage_busy_ = false;
}

int Batch::create()
{
    const Geom &g = f_->g;
    pstride_ = pstride_for(g);
    bytes_ = workspace_bytes(g, prec_, S_, pstride_);
    mem_ = ctx_->arena.alloc(bytes_);
    if (!mem_)
        return set_error(STAG_ENOMEM, "arena exhausted: CG workspace needs %zu bytes (largest free block %zu)", bytes_,
                         ctx_->arena.largest_free());
    carve(mem_);
    STAG_HIP_CHECK(hipHostMalloc((void **)&stage_, host_bytes_for(S_), hipHostMallocDefault));
    if (const char *e = getenv("STAG_GRAPHS"))
        use_graphs_ = e[0] != '0';
    if (use_graphs_)
        STAG_HIP_CHECK(hipStreamCreateWithFlags(&cap_stream_, hipStreamNonBlocking));
    STAG_HIP_CHECK(hipEventCreateWithFlags(&snap_ev_, hipEventDisableTiming));
    STAG_HIP_CHECK(hipEventCreateWithFlags(&stage_ev_, hipEventDisableTiming));
    return finish_create();
}

int Batch::create_external(void *dev, size_t dev_bytes, void *host, size_t host_bytes)
{
    external_ = true;
    use_graphs_ = false;
    pstride_ = pstride_for(f_->g);
    bytes_ = workspace_bytes(f_->g, prec_, S_, pstride_);
    if (!dev || dev_bytes < bytes_ || !host || host_bytes < host_bytes_for(S_))
        return set_error(STAG_EINVAL, "CG workspace of %zu bytes does not fit the fixed %zu-byte buffer", bytes_,
                         dev_bytes);
    mem_ = dev;
    carve(mem_);
    stage_ = (SysState *)host;
    return finish_create();
}

int Batch::finish_create()
{
    const size_t nsys = 2 * (size_t)S_;
    snap_ = stage_ + nsys;
    xhi_h_ = (dbl2 **)(snap_ + 2 * nsys);
    b_h_ = (const dbl2 **)(xhi_h_ + nsys);
    perm_h_ = (int *)(b_h_ + nsys);
    memset(stage_, 0, host_bytes_for(S_));
    for (size_t j = 0; j < nsys; ++j)
        perm_h_[j] = (int)j;
    perm_last_.assign(perm_h_, perm_h_ + nsys);
    // kernel shape for this (field, precision, slots): tuned on this workspace
    const uint64_t key = ((uint64_t)1 << 40) | ((uint64_t)prec_ << 32) | (uint32_t)S_;
    bool have = false;
    {
        std::lock_guard<std::mutex> lk(ctx_->mu);
        auto it = f_->tuned.find(key);
        if (it != f_->tuned.end()) {
            cfg_ = it->second;
            have = true;
        }
    }
    auto small_key = [&](int R) {
        return ((uint64_t)2 << 40) | ((uint64_t)prec_ << 32) | ((uint64_t)S_ << 8) | (uint64_t)R;
    };
    if (have) {
        std::lock_guard<std::mutex> lk(ctx_->mu);
        for (int R = 1; R < cfg_.rtile; ++R) {
            auto it = f_->tuned.find(small_key(R));
            if (it != f_->tuned.end())
                small_.push_back(it->second);
        }
    } else if (external_) {
        cfg_ = default_cg_cfg();  // no timing runs without events; not cached
    } else {
        cfg_ = tune_cg();  // also fills small_
        std::lock_guard<std::mutex> lk(ctx_->mu);
        f_->tuned[key] = cfg_;
        for (const KernelCfg &c : small_)
            f_->tuned[small_key(c.rtile)] = c;
    }
    nblk_ = grid_x(cfg_);
    reduce_ = uses_reduction(cfg_);
    live_ = S_;
    // every block of a step kernel writes its partial sum at [blockIdx.x] of a
    // slot of pstride_ entries, and the prologues / the reduction kernel read
    // nblk_ of them: the grid must never be wider than a slot
    if (nblk_ < 1 || nblk_ > pstride_)
        return set_error(STAG_EINVAL, "CG grid of %d blocks exceeds the partial-sum slot (%d)", nblk_, pstride_);
    // every system starts idle, all systems listed
    STAG_HIP_CHECK(hipMemcpyAsync(st_d_[0], stage_, nsys * sizeof(SysState), hipMemcpyHostToDevice, s_));
    STAG_HIP_CHECK(hipMemcpyAsync(st_d_[1], stage_, nsys * sizeof(SysState), hipMemcpyHostToDevice, s_));
    STAG_HIP_CHECK(hipMemcpyAsync(xhi_d_, xhi_h_, nsys * sizeof(void *), hipMemcpyHostToDevice, s_));
    STAG_HIP_CHECK(hipMemcpyAsync(b_d_, b_h_, nsys * sizeof(void *), hipMemcpyHostToDevice, s_));
    STAG_HIP_CHECK(hipMemcpyAsync(perm_d_, perm_h_, nsys * sizeof(int), hipMemcpyHostToDevice, s_));
    int rc = mark_stage();
    if (rc != STAG_OK)
        return rc;
    // record the epochs the solve driver chooses from (powers of two), for
    // every tile shape, now, outside any solve
    for (int E = 2; use_graphs_ && E <= kEpochMax; E *= 2) {
        rc = record_epoch(E, cfg_);
        for (size_t i = 0; i < small_.size() && rc == STAG_OK; ++i)
            rc = record_epoch(E, small_[i]);
        if (rc != STAG_OK)
            return rc;
    }
    return STAG_OK;
}

int Batch::set_running(const std::vector<char> &running)
{
    const int n = nsys();
    std::vector<int> order(n, -1);
    live_ = 0;
    for (int par = 0; par < 2; ++par) {
        int k = par * S_;
        for (int i = 0; i < S_; ++i)
            if (running[par * S_ + i])
                order[k++] = par * S_ + i;
        live_ = std::max(live_, k - par * S_);
    }
    if (order == perm_last_)
        return STAG_OK;
    wait_stage();
    memcpy(perm_h_, order.data(), n * sizeof(int));
    perm_last_ = order;
    STAG_HIP_CHECK(hipMemcpyAsync(perm_d_, perm_h_, n * sizeof(int), hipMemcpyHostToDevice, s_));
    return mark_stage();
}

// Time K1 + K2 of one step with every system in a CG step on filled vectors.
double Batch::time_cg_config(const KernelCfg &c, int nblk, bool reduce)
{
    if (nblk < 1 || nblk > pstride_)  // partial sums are indexed by block: never past a slot
        return 1e30;
    const CgLaunchTable &t = cg_table(prec_, f_->rows, f_->nt_links);
    CgArgs a = args();
    for (int par = 0; par < 2; ++par)
        a.nbr[par] = c.tables ? f_->nbr_for(par) : nullptr;
    a.remap = c.remap;
    a.psum = reduce ? totals_ : partials_;
    a.psum_stride = reduce ? 1 : pstride_;
    a.nread = reduce ? 1 : nblk;
    if (c.shared && !t.shared1)
        return 1e30;
    dim3 grid((unsigned)nblk, (unsigned)(nsys() / c.rtile)), blk(c.block);
    auto step = [&]() {
        hipError_t e = c.shared ? t.shared1(c.rtile, c.block / 64, grid, s_, a, 0)
                                 : t.step1(c.lps, c.rtile, grid, blk, s_, a, 0);
        if (e == hipSuccess && reduce)
            e = launch_reduce(s_, 1, 0, 2, nblk);
        if (e == hipSuccess)
            e = c.shared ? t.shared2(c.rtile, c.block / 64, grid, s_, a, 0)
                         : t.step2(c.lps, c.rtile, grid, blk, s_, a, 0);
        if (e == hipSuccess && reduce)
            e = launch_reduce(s_, 1, 2, 1, nblk);
        return e;
    };
    if (step() != hipSuccess)
        return 1e30;
    // the faster of two runs of 5 steps: single short runs vary by more than
    // the differences between the leading shapes
    const int reps = 5;
    double best = 1e30;
    for (int run = 0; run < 2; ++run) {
        (void)hipEventRecord(tune_ev_[0], s_);
        for (int i = 0; i < reps; ++i)
            (void)step();
        (void)hipEventRecord(tune_ev_[1], s_);
        if (hipEventSynchronize(tune_ev_[1]) != hipSuccess)
            return 1e30;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, tune_ev_[0], tune_ev_[1]);
        best = std::min(best, (double)ms / reps);
    }
    return best;
}

KernelCfg Batch::default_cg_cfg() const
{
    KernelCfg best;
    best.lps = 1;
    best.block = 256;
    best.rtile = 1;
    best.tables = 0;
    best.remap = 1;
    const CgLaunchTable &t = cg_table(prec_, f_->rows, f_->nt_links);
    for (int i = 0; i < t.n_rtiles; ++i)
        if (S_ % t.rtiles[i] == 0)
            best.rtile = std::max(best.rtile, t.rtiles[i]);
    return best;
}

// The shared-link shape of compiled shape code `code` (W wavefronts of RR
// systems, shared_code(W, RR)); reduce: as KernelCfg::reduce.
static KernelCfg shared_shape(int code, int reduce)
{
    const int W = code % 100, RR = code / 100;
    KernelCfg c;
    c.lps = 1;
    c.block = 64 * W;
    c.rtile = W * RR;
    c.tables = 0;
    c.remap = 1;
    c.reduce = reduce;
    c.shared = 1;
    return c;
}

KernelCfg Batch::tune_cg()
{
    KernelCfg best = default_cg_cfg();
    const CgLaunchTable &t = cg_table(prec_, f_->rows, f_->nt_links);
    const char *env = getenv("STAG_KERNEL_CFG");
    if (env && *env) {
        KernelCfg c;
        const int n = sscanf(env, "%d,%d,%d,%d,%d,%d", &c.lps, &c.block, &c.rtile, &c.tables, &c.remap, &c.shared);
        if (n < 5 || c.rtile <= 0 || S_ % c.rtile)
            return best;
        if (n == 6 && c.shared) {
            bool have = false;
            const int W = c.block / 64;
            for (int i = 0; i < t.n_stiles; ++i)
                have |= c.block % 64 == 0 && W > 0 && c.rtile % W == 0 && t.stiles[i] == shared_code(W, c.rtile / W);
            if (have && c.lps == 1)
                return c;
            return best;
        }
        c.shared = 0;
        if ((c.lps == 1 || c.lps == 2 || c.lps == 4 || c.lps == 8) && c.block >= 64 && c.block <= 256 &&
            c.block % 64 == 0)
            return c;
        return best;
    }
    const char *tenv = getenv("STAG_TUNE");
    if (tenv && tenv[0] == '0')
        return best;
    // Every system in a CG step; vectors and the partial sums the first
    // prologue reads filled with a small positive pattern (bytes 0x3f), so the
    // state stays in CG steps and every kernel does its full work.  x points at
    // the FP64 work vector.
    const size_t nsys = 2 * (size_t)S_, Vh = f_->g.Vh;
    std::vector<SysState> st(nsys);
    memset(st.data(), 0, nsys * sizeof(SysState));
    for (auto &x : st) {
        x.mode = M_CG;
        x.mass2 = 1e-4;
        x.rr = 1.0;
        x.maxiter = 1 << 30;
        x.mixed = prec_ != STAG_FP64;
    }
    std::vector<dbl2 *> xs(nsys);
    for (size_t j = 0; j < nsys; ++j)
        xs[j] = tmp_ + j * 3 * Vh;
    const bool verbose = getenv("STAG_TUNE_VERBOSE") != nullptr;
    const size_t vec_bytes = (char *)tmp_ - (char *)p_[0] + nsys * 3 * Vh * 16;
    if (hipMemcpyAsync(st_d_[0], st.data(), nsys * sizeof(SysState), hipMemcpyHostToDevice, s_) != hipSuccess ||
        hipMemcpyAsync(xhi_d_, xs.data(), nsys * sizeof(void *), hipMemcpyHostToDevice, s_) != hipSuccess ||
        hipMemcpyAsync(perm_d_, perm_h_, nsys * sizeof(int), hipMemcpyHostToDevice, s_) != hipSuccess ||
        hipMemsetAsync(p_[0], 0x3f, vec_bytes, s_) != hipSuccess ||
        hipMemsetAsync(partials_, 0x3f, 2 * nsys * 3 * (size_t)pstride_ * sizeof(double), s_) != hipSuccess ||
        hipMemsetAsync(totals_, 0x3f, 2 * nsys * 3 * sizeof(double), s_) != hipSuccess ||
        hipEventCreate(&tune_ev_[0]) != hipSuccess || hipEventCreate(&tune_ev_[1]) != hipSuccess) {
        (void)hipStreamSynchronize(s_);
        return best;
    }
    double best_t = 1e30;
    const int lps_c[4] = {1, 2, 4, 8}, blk_c[3] = {64, 128, 256};
    for (int i = 0; i < t.n_rtiles; ++i) {
        const int R = t.rtiles[i];
        if (S_ % R)
            continue;
        for (int L : lps_c)
            for (int B : blk_c)
                for (int D = 0; D < 2; ++D) {
                    KernelCfg c;
                    c.lps = L;
                    c.block = B;
                    c.rtile = R;
                    c.tables = 0;
                    c.remap = 1;
                    c.reduce = D;
                    if (D == 1 && uses_reduction(c) == uses_reduction(KernelCfg{L, B, R, 0, 1, 0}))
                        continue;  // the mode is forced from the environment
                    const double ms = time_cg_config(c, grid_x(c), uses_reduction(c));
                    if (verbose)
                        fprintf(stderr, "[stag tune cg] V=%d prec=%d slots=%d lps=%d block=%d rtile=%d reduce=%d: "
                                        "%.2f us\n", 2 * f_->g.Vh, prec_, S_, L, B, R, D, ms * 1e3);
                    if (ms < best_t * 0.99) {
                        best_t = ms;
                        best = c;
                    }
                }
    }
    // shared-link tiles: one shape per tile size (one lane per site, a wavefront per system)
    for (int i = 0; i < t.n_stiles; ++i) {
        const int code = t.stiles[i];
        if (S_ % shared_shape(code, 0).rtile)
            continue;
        for (int D = 0; D < 2; ++D) {
            const KernelCfg c = shared_shape(code, D);
            if (D == 1 && uses_reduction(c) == uses_reduction(shared_shape(code, 0)))
                continue;  // the mode is forced from the environment
            const double ms = time_cg_config(c, grid_x(c), uses_reduction(c));
            if (verbose)
                fprintf(stderr, "[stag tune cg] V=%d prec=%d slots=%d shared rtile=%d waves=%d reduce=%d: %.2f us\n",
                        2 * f_->g.Vh, prec_, S_, c.rtile, c.block / 64, D, ms * 1e3);
            if (ms < best_t * 0.99) {
                best_t = ms;
                best = c;
            }
        }
    }
    for (int T = 0; T < 2; ++T)
        for (int X = 0; X < 2; ++X) {
            KernelCfg c = best;
            c.tables = T;
            c.remap = X;
            const double ms = time_cg_config(c, grid_x(c), uses_reduction(c));
            if (verbose)
                fprintf(stderr, "[stag tune cg] V=%d prec=%d slots=%d lps=%d block=%d rtile=%d tables=%d remap=%d: "
                                "%.2f us\n", 2 * f_->g.Vh, prec_, S_, c.lps, c.block, c.rtile, T, X, ms * 1e3);
            if (ms < best_t * 0.99) {
                best_t = ms;
                best = c;
            }
        }
    // Smaller tiles, for when fewer systems run than the tuned tile takes: a
    // tile's empty places still gather (they read the first system's values),
    // so a lone system in a large tile pays for the whole tile.  Each is tuned
    // at the tuned shape's block count, which every kernel of the batch keeps.
    const int nblk = grid_x(best);
    const bool reduce = uses_reduction(best);
    small_.clear();
    for (int R = 1; R < best.rtile; ++R) {
        if (S_ % R)
            continue;
        bool reg = false, shr = false;
        for (int i = 0; i < t.n_rtiles; ++i)
            reg |= t.rtiles[i] == R;
        for (int i = 0; i < t.n_stiles; ++i)
            shr |= shared_shape(t.stiles[i], 0).rtile == R;
        if (!reg && !shr)
            continue;
        KernelCfg sb;
        double sb_t = 1e30;
        for (int L : lps_c)
            for (int B : blk_c) {
                if (!reg)
                    break;
                KernelCfg c = best;
                c.shared = 0;
                c.lps = L;
                c.block = B;
                c.rtile = R;
                const double ms = time_cg_config(c, nblk, reduce);
                if (verbose)
                    fprintf(stderr, "[stag tune cg] small tile: V=%d prec=%d slots=%d lps=%d block=%d rtile=%d "
                                    "blocks=%d: %.2f us\n", 2 * f_->g.Vh, prec_, S_, L, B, R, nblk, ms * 1e3);
                if (ms < sb_t * 0.99) {
                    sb_t = ms;
                    sb = c;
                }
            }
        for (int i = 0; shr && i < t.n_stiles; ++i) {
            KernelCfg c = shared_shape(t.stiles[i], best.reduce);
            if (c.rtile != R)
                continue;
            c.tables = best.tables;
            c.remap = best.remap;
            const double ms = time_cg_config(c, nblk, reduce);
            if (verbose)
                fprintf(stderr, "[stag tune cg] small tile: V=%d prec=%d slots=%d shared rtile=%d waves=%d blocks=%d: "
                                "%.2f us\n", 2 * f_->g.Vh, prec_, S_, R, c.block / 64, nblk, ms * 1e3);
            if (ms < sb_t * 0.99) {
                sb_t = ms;
                sb = c;
            }
        }
        if (sb_t < 1e29)
            small_.push_back(sb);
    }
    (void)hipStreamSynchronize(s_);
    (void)hipGetLastError();
    return best;
}

void Batch::stage_system(int j, const stag_cg_params &p, const double *b_half, double *x_half)
{
    wait_stage();
    SysState &st = stage_[j];
    memset(&st, 0, sizeof(st));
    if (!b_half || !x_half) {
        st.mode = M_IDLE;
        xhi_h_[j] = nullptr;
        b_h_[j] = nullptr;
        return;
    }
    st.mode = M_INIT;
    st.mass2 = p.mass * p.mass;
    st.tol2 = p.tol * p.tol;
    st.maxiter = p.maxiter;
    st.max_restarts = p.max_restarts;
    st.mixed = prec_ != STAG_FP64;
    // default threshold per precision: FP32 keeps the residual to ~1e-7
    // relative, so it can run two decades between updates; FP16 (~1e-3)
    // needs one, or its iterate drifts and CG takes many more steps
    const double delta = p.delta > 0 ? p.delta : (prec_ == STAG_FP32_RU ? 0.01 : 0.1);
    st.delta2 = st.mixed ? delta * delta : 0.0;
    xhi_h_[j] = (dbl2 *)x_half;
    b_h_[j] = (const dbl2 *)b_half;
}

int Batch::upload_and_init(const std::vector<int> &systems)
{
    // every system at once (a blocking solve): whole arrays, four copies;
    // otherwise (admission next to running systems) only the staged ones
    std::vector<char> seen(nsys(), 0);
    int distinct = 0;
    for (int j : systems)
        if (j >= 0 && j < nsys() && !seen[j]) {
            seen[j] = 1;
            ++distinct;
        }
    if (distinct == nsys()) {
        const size_t ns = (size_t)nsys();
        STAG_HIP_CHECK(hipMemcpyAsync(st_d_[0], stage_, ns * sizeof(SysState), hipMemcpyHostToDevice, s_));
        STAG_HIP_CHECK(hipMemcpyAsync(st_d_[1], stage_, ns * sizeof(SysState), hipMemcpyHostToDevice, s_));
        STAG_HIP_CHECK(hipMemcpyAsync(xhi_d_, xhi_h_, ns * sizeof(void *), hipMemcpyHostToDevice, s_));
        STAG_HIP_CHECK(hipMemcpyAsync(b_d_, b_h_, ns * sizeof(void *), hipMemcpyHostToDevice, s_));
    } else {
        for (int j : systems) {
            // the staged state goes into both buffers: the first step reads buffer 0
            STAG_HIP_CHECK(hipMemcpyAsync(st_d_[0] + j, stage_ + j, sizeof(SysState), hipMemcpyHostToDevice, s_));
            STAG_HIP_CHECK(hipMemcpyAsync(st_d_[1] + j, stage_ + j, sizeof(SysState), hipMemcpyHostToDevice, s_));
            STAG_HIP_CHECK(hipMemcpyAsync(xhi_d_ + j, xhi_h_ + j, sizeof(void *), hipMemcpyHostToDevice, s_));
            STAG_HIP_CHECK(hipMemcpyAsync(b_d_ + j, b_h_ + j, sizeof(void *), hipMemcpyHostToDevice, s_));
        }
    }
    int rc = mark_stage();
    if (rc != STAG_OK)
        return rc;
    const CgArgs a = args();
    const CgLaunchTable &t = cg_table(prec_, f_->rows, f_->nt_links);
    dim3 grid((unsigned)nblk_, (unsigned)nsys());
    // one thread per site (the init kernel takes any block of up to 256 threads)
    hipError_t e = cfg_.shared ? t.init(grid, dim3(256), s_, a, 1) : t.init(grid, dim3(cfg_.block), s_, a, cfg_.lps);
    if (e == hipSuccess && reduce_)
        e = launch_reduce(s_, 0, 2, 1, nblk_);
    if (e != hipSuccess)
        return set_error(STAG_EHIP, "init launch failed: %s", hipGetErrorString(e));
    return STAG_OK;
}

CgArgs Batch::args() const
{
    CgArgs a;
    memset(&a, 0, sizeof(a));
    a.g = f_->g;
    for (int par = 0; par < 2; ++par) {
        a.links[par] = f_->links_for(prec_, par);
        a.links64[par] = (const dbl2 *)f_->links_for(0, par);
        a.nbr[par] = cfg_.tables ? f_->nbr_for(par) : nullptr;
    }
    a.p[0] = p_[0];
    a.p[1] = p_[1];
    a.ap = ap_;
    a.r = r_;
    a.xlo = xlo_;
    a.tmp = tmp_;
    a.xhi = xhi_d_;
    a.b = b_d_;
    a.st[0] = st_d_[0];
    a.st[1] = st_d_[1];
    a.perm = perm_d_;
    a.partials = partials_;
    a.S = S_;
    a.pstride = pstride_;
    a.remap = cfg_.remap;
    a.psum = reduce_ ? totals_ : partials_;
    a.psum_stride = reduce_ ? 1 : pstride_;
    a.nread = reduce_ ? 1 : nblk_;
    return a;
}

int Batch::launch_step(int ver, hipStream_t st, const KernelCfg &c)
{
    const CgLaunchTable &t = cg_table(prec_, f_->rows, f_->nt_links);
    const CgArgs a = args();
    const int R = c.rtile;
    dim3 grid((unsigned)nblk_, (unsigned)(nsys() / R)), blk(c.block);
    if (c.shared && !t.shared1)
        return set_error(STAG_EINVAL, "no shared-link CG tiles for precision %d", prec_);
    hipError_t e = c.shared ? t.shared1(R, c.block / 64, grid, st, a, ver) : t.step1(c.lps, R, grid, blk, st, a, ver);
    if (e == hipSuccess && reduce_)  // K1's partials: slots 0, 1 of buffer ver ^ 1
        e = launch_reduce(st, ver ^ 1, 0, 2, nblk_);
    if (e == hipSuccess)
        e = c.shared ? t.shared2(R, c.block / 64, grid, st, a, ver) : t.step2(c.lps, R, grid, blk, st, a, ver);
    if (e == hipSuccess && reduce_)  // K2's partials: slot 2 of buffer ver ^ 1
        e = launch_reduce(st, ver ^ 1, 2, 1, nblk_);
    if (e != hipSuccess)
        return set_error(STAG_EHIP, "CG kernel launch failed: %s", hipGetErrorString(e));
    return STAG_OK;
}

// Key of the recorded epoch of `steps` steps with shape c (one shape per tile size).
static int graph_key(const KernelCfg &c, int steps)
{
    return ((c.shared ? c.block / 64 : 0) * 64 + c.rtile) * 1024 + steps;
}

int Batch::record_epoch(int steps, const KernelCfg &c)
{
    const int key = graph_key(c, steps);
    if (graphs_.count(key))
        return STAG_OK;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    STAG_HIP_CHECK(hipStreamBeginCapture(cap_stream_, hipStreamCaptureModeThreadLocal));
    int rc = STAG_OK;
    for (int k = 0; k < steps && rc == STAG_OK; ++k)
        rc = launch_step(k & 1, cap_stream_, c);
    hipError_t e = hipStreamEndCapture(cap_stream_, &graph);
    if (rc != STAG_OK) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess)
        return set_error(STAG_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess)
        return set_error(STAG_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
    graphs_.emplace(key, exec);
    return STAG_OK;
}

const KernelCfg &Batch::epoch_cfg() const
{
    for (const KernelCfg &c : small_)
        if (c.rtile >= live_)
            return c;
    return cfg_;
}

int Batch::enqueue_epoch(int steps)
{
    steps += steps & 1;
    const KernelCfg &c = epoch_cfg();
    if (!use_graphs_) {
        for (int k = 0; k < steps; ++k) {
            int rc = launch_step(k & 1, s_, c);
            if (rc != STAG_OK)
                return rc;
        }
        return STAG_OK;
    }
    // The kernel arguments of an epoch depend only on this workspace, so an
    // epoch of a given length is recorded once and replayed: the launches of
    // all its kernels cost one graph launch on the host.
    int rc = record_epoch(steps, c);
    if (rc != STAG_OK)
        return rc;
    auto it = graphs_.find(graph_key(c, steps));
    STAG_HIP_CHECK(hipGraphLaunch(it->second, s_));
    return STAG_OK;
}

int Batch::enqueue_snapshot()
{
    // both state buffers in one copy (they are adjacent, as are their host
    // mirrors): each copy costs a few microseconds of stream time
    STAG_HIP_CHECK(hipMemcpyAsync(snap_, st_d_[0], 2 * nsys() * sizeof(SysState), hipMemcpyDeviceToHost, s_));
    if (!external_)
        STAG_HIP_CHECK(hipEventRecord(snap_ev_, s_));
    return STAG_OK;
}

int Batch::wait_snapshot()
{
    if (external_)
        STAG_HIP_CHECK(hipStreamSynchronize(s_));
    else
        STAG_HIP_CHECK(hipEventSynchronize(snap_ev_));
    return STAG_OK;
}

bool Batch::snapshot_ready() { return (external_ ? hipStreamQuery(s_) : hipEventQuery(snap_ev_)) == hipSuccess; }

// ---- the blocking solve ------------------------------------------------------------

static int validate_params(const stag_cg_params &p, int prec0)
{
    if (!(p.mass > 0) || !std::isfinite(p.mass))
        return set_error(STAG_EINVAL, "mass must be > 0 (got %g)", p.mass);
    if (!(p.tol > 0) || !std::isfinite(p.tol))
        return set_error(STAG_EINVAL, "tol must be > 0 (got %g)", p.tol);
    if (p.maxiter < 0)
        return set_error(STAG_EINVAL, "maxiter must be >= 0");
    if (p.max_restarts < 0)
        return set_error(STAG_EINVAL, "max_restarts must be >= 0");
    if (p.parity < STAG_EVEN || p.parity > STAG_ALL)
        return set_error(STAG_EINVAL, "parity must be STAG_EVEN, STAG_ODD or STAG_ALL");
    if (p.precision < STAG_FP64 || p.precision > STAG_FP16_RU)
        return set_error(STAG_EINVAL, "unknown precision %d", p.precision);
    if (p.precision == STAG_FP16_RU && p.delta > 0 && p.delta < STAG_FP16_DELTA_MIN)
        return set_error(STAG_EINVAL, "FP16 reliable-update threshold %g is below its floor %g", p.delta,
                         (double)STAG_FP16_DELTA_MIN);
    if (p.precision != prec0)
        return set_error(STAG_EINVAL, "all systems of a batch must use the same precision");
    return STAG_OK;
}

int validate_cg_params(const stag_cg_params &p) { return validate_params(p, p.precision); }

static int worse(int a, int b)
{
    if (a == STAG_OK)
        return b;
    return a;
}

void fill_info(const Batch &B, int slot, stag_cg_info *info)
{
    const int S = B.slots();
    int status = STAG_OK, iters = 0, nru = 0, rst = 0;
    double trr = 0, bb = 0;
    bool any = false;
    info->iters_parity[0] = info->iters_parity[1] = -1;
    for (int par = 0; par < 2; ++par) {
        const SysState &st = B.state(par * S + slot);
        if (st.mode == M_IDLE)
            continue;
        any = true;
        status = worse(status, st.mode == M_DONE ? st.status : STAG_ENOCONV);
        iters = std::max(iters, st.iters);
        info->iters_parity[par] = st.iters;
        nru += st.n_ru;
        rst = std::max(rst, st.restarts);
        trr += st.true_rr;
        bb += st.bb;
    }
    info->status = any ? status : STAG_OK;
    info->iters = iters;
    info->reliable_updates = nru;
    info->restarts = rst;
    info->true_rel_resid = bb > 0 ? std::sqrt(trr / bb) : std::sqrt(trr);
}

int acquire_batch(Ctx *ctx, const std::shared_ptr<GaugeField> &f, int prec, int slots, hipStream_t s,
                  std::shared_ptr<Batch> &out)
{
    {
        std::lock_guard<std::mutex> lk(ctx->cache_mu);
        for (auto it = ctx->batch_cache.begin(); it != ctx->batch_cache.end(); ++it) {
            Batch &b = **it;
            if (b.field() == f.get() && b.prec() == prec && b.slots() == slots && b.stream() == s) {
                out = *it;
                ctx->batch_cache.erase(it);
                return STAG_OK;
            }
        }
    }
    for (int attempt = 0; attempt < 2; ++attempt) {
        auto b = std::make_shared<Batch>(ctx, f, prec, slots, s);
        int rc = b->create();
        if (rc == STAG_OK) {
            out = b;
            return STAG_OK;
        }
        b.reset();
        if (rc != STAG_ENOMEM || attempt == 1)
            return rc;
        drop_cached_batches(ctx, -1);
    }
    return STAG_ENOMEM;
}

void release_batch(Ctx *ctx, std::shared_ptr<Batch> b)
{
    if (!b)
        return;
    std::lock_guard<std::mutex> lk(ctx->cache_mu);
    ctx->batch_cache.push_back(std::move(b));
    if (ctx->batch_cache.size() > 8)
        ctx->batch_cache.erase(ctx->batch_cache.begin());
}

void drop_cached_batches(Ctx *ctx, int32_t gauge_id)
{
    std::vector<std::shared_ptr<Batch>> dead;
    {
        std::lock_guard<std::mutex> lk(ctx->cache_mu);
        for (auto it = ctx->batch_cache.begin(); it != ctx->batch_cache.end();) {
            if (gauge_id < 0 || (*it)->field()->id == gauge_id) {
                dead.push_back(*it);
                it = ctx->batch_cache.erase(it);
            } else {
                ++it;
            }
        }
    }
    for (auto &b : dead)
        (void)hipStreamSynchronize(b->stream());
    dead.clear();
}

// Iterations left for the slowest running system.  A system's rate of
// convergence (decrease of log <r,r> per iteration) is the larger of its mean
// rate since the start of the solve and its rate over the iterations since
// the previous look, if there were at least 8 (the CG residual is not
// monotonic, so a shorter span says little); with neither known the result
// is kUnknownRemaining.
struct ConvergenceTrack {
    int iters = 0;
    double rr = 0.0;
};
constexpr int kUnknownRemaining = 1 << 20;

static int estimate_remaining(const Batch &B, std::vector<ConvergenceTrack> &track)
{
    double worst = 0;
    bool known = true;
    for (int j = 0; j < B.nsys(); ++j) {
        const SysState &st = B.state(j);
        ConvergenceTrack &t = track[j];
        const bool running = st.mode == M_CG || st.mode == M_RU;
        if (running) {
            double rate = 0.0;
            if (st.iters > 0 && st.bb > st.rr && st.rr > 0)
                rate = std::log(st.bb / st.rr) / st.iters;
            const int di = st.iters - t.iters;
            if (di >= 8 && t.rr > st.rr && st.rr > 0)
                rate = std::max(rate, std::log(t.rr / st.rr) / di);
            if (rate > 0 && st.stop2 > 0) {
                // CG iterations to the stopping test, plus the residual
                // recomputations on the way (one per factor 1/delta^2 of <r,r>)
                const double decades = std::log(std::max(st.rr / st.stop2, 1.0));
                double steps = decades / rate;
                if (st.delta2 > 0 && st.delta2 < 1)
                    steps += decades / -std::log(st.delta2);
                worst = std::max(worst, steps);
            } else {
                known = false;
            }
        }
        if (!running || st.iters - t.iters >= 8) {
            t.iters = st.iters;
            t.rr = st.rr;
        }
    }
    return known ? (int)std::ceil(worst) : kUnknownRemaining;
}

// The blocking solve of nrhs systems on workspace B (its slots = nrhs).
// fixed_mem: B lives in caller-provided memory, and nothing here may allocate
// (the kernel shape of y = D x is the cached or default one, never tuned).
static int run_solve(Ctx *ctx, Batch &B, const std::shared_ptr<GaugeField> &f, int nrhs,
                     const stag_cg_params *params, const double *const *b, double *const *x, double *const *y,
                     hipStream_t s, stag_cg_info *infos, bool fixed_mem)
{
    const auto t0 = std::chrono::steady_clock::now();
    int rc = STAG_OK;
    struct SyncOnExit {  // on an error return, drain the stream before the workspace goes
        hipStream_t s;
        ~SyncOnExit() { (void)hipStreamSynchronize(s); }
    } drain{s};
    const size_t half = (size_t)3 * f->g.Vh * 2;  // doubles per parity half
    std::vector<int> systems;
    std::vector<char> running(B.nsys(), 0);
    int max_iter = 0;
    for (int i = 0; i < nrhs; ++i) {
        max_iter = std::max(max_iter, params[i].maxiter);
        for (int par = 0; par < 2; ++par) {
            const int j = par * nrhs + i;
            const bool on = params[i].parity == STAG_ALL || params[i].parity == par;
            B.stage_system(j, params[i], on ? b[i] + par * half : nullptr, on ? x[i] + par * half : nullptr);
            systems.push_back(j);
            running[j] = on;
        }
    }
    // a workspace taken from the cache keeps the tile order of its last solve
    if ((rc = B.upload_and_init(systems)) != STAG_OK || (rc = B.set_running(running)) != STAG_OK)
        return rc;
    int E = 8, Emax = kEpochMax;
    const bool fixed_epoch = getenv("STAG_EPOCH") != nullptr;
    const bool epoch_log = getenv("STAG_EPOCH_VERBOSE") != nullptr;
    if (fixed_epoch)
        E = Emax = std::max(1, atoi(getenv("STAG_EPOCH")));
    std::vector<ConvergenceTrack> track(B.nsys());
    // pipelined: epoch n+1 is queued before the state after epoch n is read
    if ((rc = B.enqueue_epoch(E)) != STAG_OK || (rc = B.enqueue_snapshot()) != STAG_OK)
        return rc;
    int64_t budget = (int64_t)(max_iter + 1) * (int64_t)(2 + params[0].max_restarts) + 4096;
    bool done = false;
    while (!done && budget > 0) {
        if ((rc = B.enqueue_epoch(E)) != STAG_OK)
            return rc;
        const int inflight = E;
        budget -= E;
        if ((rc = B.wait_snapshot()) != STAG_OK)
            return rc;
        done = true;
        for (int j = 0; j < B.nsys(); ++j) {
            const int md = B.state(j).mode;
            if (md == M_INIT || md == M_CG || md == M_RU)
                done = false;
        }
        if (!done) {
            running.assign(B.nsys(), 0);
            for (int j = 0; j < B.nsys(); ++j)
                running[j] = B.state(j).mode == M_INIT || B.state(j).mode == M_CG || B.state(j).mode == M_RU;
            if ((rc = B.set_running(running)) != STAG_OK)
                return rc;
            // steps still needed after the state just read (CG steps to the
            // stopping test plus the final FP64 check), less the epoch in
            // flight; the next epoch covers about half of them (an epoch too
            // short costs a look at the state, which overlaps the epoch in
            // flight unless the epochs are very short; one too long costs
            // idle steps of a few microseconds each).  The shortest epoch is
            // 2 steps; 16 while the rate of convergence is not known yet.
            const int rem = estimate_remaining(B, track);
            const int ahead = rem == kUnknownRemaining ? 32 : rem + 1 - inflight;
            E = 2;
            if (ahead <= 16) {
                // the end is near: one epoch for all of it (a few idle steps
                // cost less than another look at the state)
                while (E < ahead)
                    E *= 2;
            } else {
                while (E * 2 <= std::min(Emax, ahead / 2))
                    E *= 2;
            }
            if (fixed_epoch)
                E = Emax;
            if (epoch_log)
                fprintf(stderr, "[stag epoch] in flight %d, remaining %d, next %d\n", inflight, rem, E);
            if ((rc = B.enqueue_snapshot()) != STAG_OK)
                return rc;
        }
    }
    if ((rc = B.enqueue_snapshot()) != STAG_OK || (rc = B.wait_snapshot()) != STAG_OK)
        return rc;
    // y = D x on the opposite parity of every solved system (Sec. 4, second half)
    int first_err = STAG_OK;
    for (int i = 0; i < nrhs; ++i) {
        if (y && y[i]) {
            const int par = params[i].parity;
            const int out_par = par == STAG_ALL ? STAG_ALL : 1 - par;
            rc = fixed_mem ? dslash_with(cached_config(ctx, f.get(), 0, 1), f.get(), 0, out_par, 0, f->g.Vh, x[i],
                                         y[i], 0, s)
                           : dslash_f64(ctx, f.get(), out_par, 0, f->g.Vh, x[i], y[i], 0, s);
            if (rc != STAG_OK)
                return rc;
        }
    }
    STAG_HIP_CHECK(hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < nrhs; ++i) {
        stag_cg_info inf;
        memset(&inf, 0, sizeof(inf));
        fill_info(B, i, &inf);
        inf.seconds = secs;
        if (!done && inf.status == STAG_OK)
            inf.status = STAG_ENOCONV;
        if (infos)
            infos[i] = inf;
        first_err = worse(first_err, inf.status);
    }
    if (first_err != STAG_OK)
        return set_error(first_err, "CG did not converge (status %d)", first_err);
    return STAG_OK;
}

static int validate_systems(int nrhs, const stag_cg_params *params, const double *const *b, double *const *x)
{
    const int prec = params[0].precision;
    for (int i = 0; i < nrhs; ++i) {
        int rc = validate_params(params[i], prec);
        if (rc != STAG_OK)
            return rc;
        if (!b[i] || !x[i])
            return set_error(STAG_EINVAL, "b and x must be device pointers");
    }
    return STAG_OK;
}

int cg_solve_batch(Ctx *ctx, const std::shared_ptr<GaugeField> &f, int nrhs, const stag_cg_params *params,
                   const double *const *b, double *const *x, double *const *y, hipStream_t s, stag_cg_info *infos)
{
    int rc = validate_systems(nrhs, params, b, x);
    if (rc != STAG_OK)
        return rc;
    std::shared_ptr<Batch> Bp;
    rc = acquire_batch(ctx, f, params[0].precision, nrhs, s, Bp);
    if (rc != STAG_OK)
        return rc;
    rc = run_solve(ctx, *Bp, f, nrhs, params, b, x, y, s, infos, false);
    // a workspace whose solve failed part-way is not reused
    if (rc == STAG_OK || rc == STAG_ENOCONV || rc == STAG_EBREAKDOWN || rc == STAG_ENONFINITE)
        release_batch(ctx, std::move(Bp));
    return rc;
}

int cg_solve_fixed(Ctx *ctx, const std::shared_ptr<GaugeField> &f, const stag_cg_params *params, const double *b,
                   double *x, double *y, hipStream_t s, stag_cg_info *info, void *dev, size_t dev_bytes, void *host,
                   size_t host_bytes)
{
    int rc = validate_systems(1, params, &b, &x);
    if (rc != STAG_OK)
        return rc;
    Batch B(ctx, f, params->precision, 1, s);
    if (B.needed_bytes() > dev_bytes)
        return set_error(STAG_EINVAL, "the solve needs a %zu-byte workspace; the fixed workspace holds %zu bytes",
                         B.needed_bytes(), dev_bytes);
    rc = B.create_external(dev, dev_bytes, host, host_bytes);
    if (rc != STAG_OK)
        return rc;
    double *ys[1] = {y};
    return run_solve(ctx, B, f, 1, params, &b, &x, ys, s, info, true);
}

}  // namespace stag
