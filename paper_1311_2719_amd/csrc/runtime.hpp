// Host-side runtime of libstagcg: context, HBM arena, gauge-field registry,
// error reporting, kernel-configuration tuner.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdarg>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "stagcg.h"
#include "stag_types.hpp"

namespace stag {

// ---- errors ------------------------------------------------------------------

int set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define STAG_HIP_CHECK(expr)                                                          \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return ::stag::set_error(STAG_EHIP, "%s failed: %s (%s:%d)", #expr,       \
                                     hipGetErrorString(e_), __FILE__, __LINE__);      \
    } while (0)

// ---- arena -------------------------------------------------------------------

// First-fit sub-allocator over a caller-owned device buffer.  Blocks are
// 256-byte aligned.  Thread-safe.
class Arena {
public:
    void init(void *base, size_t bytes);
    void *alloc(size_t bytes);
    void release(void *p);
    size_t used() const { return used_.load(); }
    size_t total() const { return size_; }
    size_t largest_free() const;

private:
    char *base_ = nullptr;
    size_t size_ = 0;
    mutable std::mutex mu_;
    std::map<size_t, size_t> free_;  // offset -> size
    std::map<size_t, size_t> live_;  // offset -> size
    std::atomic<size_t> used_{0};
};

// ---- kernel configuration ----------------------------------------------------

struct KernelCfg {
    int lps = 1;        // lanes per output site (1, 2, 4, 8)
    int block = 256;    // threads per block
    int rtile = 1;      // right-hand sides per link read
    int tables = 0;     // 1: read iup/idn tables, 0: compute neighbours
    int remap = 1;      // XCD-aware block order
    int reduce = -1;    // CG: 1 reduction kernel between step kernels, 0 prologues sum the
                        // partials, -1 chosen by grid size
    int shared = 0;     // CG, FP32 / FP16: 1 shared-link tiles (block = 64 rtile, one lane per site)
};

// ---- gauge field -------------------------------------------------------------

enum FieldKind : int32_t { FIELD_STAGGERED = 0, FIELD_WILSON = 1 };

struct GaugeField {
    int32_t id = 0;
    int32_t kind = FIELD_STAGGERED;  // which operator the links were prepared for
    int32_t dims[4] = {0, 0, 0, 0};
    int32_t tap = 1;
    Geom g{};
    int32_t rows = 3;                                // link rows stored (2: third row rebuilt)
    int32_t nt_links = 0;                            // 1: FP64 kernels read links non-temporally
    void *links[3] = {nullptr, nullptr, nullptr};  // per precision id: [2 parities][3 * rows][Vh / 8][8][8]
    int32_t *nbr = nullptr;                          // [2][8][Vh]
    std::atomic<int> users{0};                       // serving requests queued / running
    std::map<uint64_t, KernelCfg> tuned;             // key: (prec, nrhs)
    size_t bytes = 0;

    const void *links_for(int prec, int out_parity) const
    {
        const size_t per_parity = (size_t)link_parity_entries(rows, g.Vh) * link_entry_bytes_of(prec);
        return (const char *)links[prec] + (size_t)out_parity * per_parity;
    }
    const int32_t *nbr_for(int out_parity) const { return nbr + (size_t)out_parity * 8 * g.Vh; }
};

class Server;
class Batch;

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    Arena arena;
    int num_cus = 256;
    std::mutex mu;                                       // registry
    std::map<int32_t, std::shared_ptr<GaugeField>> fields;
    int32_t next_id = 1;
    std::unique_ptr<Server> server;
    // idle CG workspaces kept for reuse by later solves of the same shape
    std::mutex cache_mu;
    std::vector<std::shared_ptr<Batch>> batch_cache;
    // serving configuration
    int slots_per_field = 16;
    int epoch_iters = 16;
    int queue_capacity = 4096;

    std::shared_ptr<GaugeField> field(int32_t id);
};

// Current device guard: makes ctx->device current for the scope.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess)
            prev = -1;
        if (prev != dev)
            (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0)
            (void)hipSetDevice(prev);
    }
};

// ---- functions implemented in the .hip files -------------------------------

// Largest deviation (absolute, on entries of magnitude <= 1/2) between the
// given third row of a folded link and the row rebuilt from the other two for
// which a field is stored in two-row form; it bounds the change of D to about
// twice this, relative.
constexpr double kTwoRowTolerance = 1e-14;
// Check the lexicographic links on the device: ENONFINITE for NaN/Inf;
// two_rows = whether every folded link admits the two-row form.
int gauge_check(Ctx *ctx, const Geom &g, const double *links_dev, hipStream_t s, bool &two_rows);
// Whether the FP64 kernels of field f read its links non-temporally: when its
// FP64 links do not fit the Infinity Cache (STAG_NT_LINKS=0/1 forces it).
int nt_links_for(const GaugeField &f);
// Fill f->links (f->rows rows, every precision) and f->nbr from the links.
int gauge_prepare(GaugeField *f, const double *links_dev, hipStream_t s);

// Wilson fermions: check the links, choose the stored rows, allocate and fill
// f->links[0] (FP64; t-boundary sign folded, backward links daggered).
int wilson_prepare(Ctx *ctx, GaugeField *f, const double *links_dev, hipStream_t s);
// lexicographic [V][4][3] <-> even-odd [2][12][Vh] complex128
int launch_pack_spinor(const Geom &g, const double *lex, double *eo, int to_eo, hipStream_t s);
// out_p = (H in)_p on one parity or both (STAG_ALL)
int wilson_dslash(Ctx *ctx, GaugeField *f, int out_parity, const double *in, double *out, hipStream_t s);
// M x = b by CG on the even-odd normal equations
int wilson_cg_solve(Ctx *ctx, GaugeField *f, double kappa, double tol, int maxiter, const double *b, double *x,
                    hipStream_t s, stag_cg_info *info);
int launch_pack(const Geom &g, const double *lex, double *eo, int to_eo, hipStream_t s);
// out (+)= D in over a site range of one parity or the whole lattice, links,
// vectors and arithmetic in precision prec (0 FP64, 1 FP32, 2 FP16)
int dslash(Ctx *ctx, GaugeField *f, int prec, int out_parity, int64_t offset, int64_t count, const void *in,
           void *out, int accumulate, hipStream_t s);
int dslash_f64(Ctx *ctx, GaugeField *f, int out_parity, int64_t offset, int64_t count,
               const double *in, double *out, int accumulate, hipStream_t s);
// the same with a given kernel shape (no tuning, nothing allocated)
int dslash_with(const KernelCfg &cfg, GaugeField *f, int prec, int out_parity, int64_t offset, int64_t count,
                const void *in, void *out, int accumulate, hipStream_t s);
// force = (accumulate ? force : 0) + coeff F, F the pseudofermion force from
// w (the CG solution on the even sites, D_oe of it on the odd sites);
// force complex128 [V][4][3][3] lexicographic
int fermion_force(GaugeField *f, const double *w, double *force, double coeff, int accumulate, hipStream_t s);
// molecular dynamics (md.hip): links and momenta complex128 [V][4][3][3]
int gauge_force(const int32_t dims[4], const double *U, double *force, double beta, double coeff, int accumulate,
                hipStream_t s);
int link_update(int64_t V, double *U, const double *Q, double eps, hipStream_t s);
int pseudofermion(Ctx *ctx, GaugeField *f, const double *chi, double *phi, double mass, hipStream_t s);
int md_energies(const int32_t dims[4], const double *U, const double *Q, const double *phi, const double *x,
                double beta, double *scratch, double energies[3], hipStream_t s);
int md_trajectory(Ctx *ctx, const int32_t dims[4], double *U, double *Q, const double *phi, const stag_md_params &p,
                  hipStream_t s, stag_md_info *info);
// full-lattice fermion field from one storage precision to another
int convert_fermion(const Geom &g, int prec_in, const void *in, int prec_out, void *out, hipStream_t s);
KernelCfg tune_config(Ctx *ctx, GaugeField *f, int prec, int nrhs, hipStream_t s);
// the tuned shape if (prec, nrhs) has been tuned on f, else the default; never tunes
KernelCfg cached_config(Ctx *ctx, GaugeField *f, int prec, int nrhs);
// CG step shape tuned for (field, precision, slots), if a solve with that many
// slots has run; reduce: whether a reduction kernel runs between the steps.
bool cg_tuned_shape(Ctx *ctx, const GaugeField *f, int prec, int slots, KernelCfg &out, bool &reduce);
bool cg_uses_reduction(const Geom &g, const KernelCfg &c);

// Take a workspace for (field, precision, slots, stream) from the cache or
// create one; give it back with release_batch.  ENOMEM after evicting the cache.
int acquire_batch(Ctx *ctx, const std::shared_ptr<GaugeField> &f, int prec, int slots, hipStream_t s,
                  std::shared_ptr<Batch> &out);
void release_batch(Ctx *ctx, std::shared_ptr<Batch> b);
void drop_cached_batches(Ctx *ctx, int32_t gauge_id);  // all if gauge_id < 0

int cg_solve_batch(Ctx *ctx, const std::shared_ptr<GaugeField> &f, int nrhs,
                   const stag_cg_params *params, const double *const *b, double *const *x,
                   double *const *y, hipStream_t s, stag_cg_info *infos);
// One solve (stag_cg_solve on device pointers) whose workspace is the given
// device memory (dev_bytes) and host memory (host_bytes); allocates nothing.
int cg_solve_fixed(Ctx *ctx, const std::shared_ptr<GaugeField> &f, const stag_cg_params *params, const double *b,
                   double *x, double *y, hipStream_t s, stag_cg_info *info, void *dev, size_t dev_bytes, void *host,
                   size_t host_bytes);
// The library's fixed device workspace on `device`: set up once per device at
// stag_create (noalloc_setup), then looked up (noalloc_scratch; null if the
// set-up failed).  The host mirror is a fixed host buffer.
int noalloc_setup(int device);
void *noalloc_scratch(int device, size_t *bytes);
void *noalloc_host(int device, size_t *bytes);
std::mutex &noalloc_lock(int device);

}  // namespace stag
