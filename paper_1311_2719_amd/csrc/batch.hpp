// A batch of CG systems that share one gauge field: workspace, state and the
// launch sequence of one CG iteration.  Used by stag_cg_solve (one right-hand
// side, two parity systems), stag_cg_solve_batch and the serving scheduler.
#pragma once

#include <vector>

#include "cg_launch.hpp"
#include "runtime.hpp"

namespace stag {

// Longest epoch (CG steps between two looks at the state) of a solve.
constexpr int kEpochMax = 64;

class Batch {
public:
    Batch(Ctx *ctx, std::shared_ptr<GaugeField> f, int prec, int slots, hipStream_t s);
    ~Batch();
    Batch(const Batch &) = delete;
    Batch &operator=(const Batch &) = delete;

    // Allocate workspace from the arena and pinned host mirrors.  ENOMEM if
    // the arena cannot hold it.
    int create();
    // Use caller-provided memory instead: `dev` (device, dev_bytes >=
    // workspace_bytes) and `host` (ordinary host memory, host_bytes >=
    // host_bytes_for(slots)).  Nothing is allocated: no arena, pinned memory,
    // events, streams or graphs (the stream is synchronised where events
    // would be waited on); the shape is the field's tuned one if a solve of
    // this shape has run, else the default.  EINVAL if either buffer is too small.
    int create_external(void *dev, size_t dev_bytes, void *host, size_t host_bytes);
    static size_t host_bytes_for(int slots);
    // workspace bytes of this batch's field, precision and slots
    size_t needed_bytes() const;
    static size_t workspace_bytes(const Geom &g, int prec, int slots, int pstride);

    int slots() const { return S_; }
    int nsys() const { return 2 * S_; }
    int prec() const { return prec_; }
    const KernelCfg &cfg() const { return cfg_; }
    hipStream_t stream() const { return s_; }
    GaugeField *field() const { return f_.get(); }

    // Stage system j (= parity * slots + slot) for initialisation with source
    // b and solution x (parity halves, device), or mark it idle (b == x == null).
    void stage_system(int j, const stag_cg_params &p, const double *b_half, double *x_half);
    // Copy staged systems [j0, j0 + n) to the device and run the init kernel.
    int upload_and_init(const std::vector<int> &systems);
    // Enqueue `steps` CG steps (rounded up to an even number, so that every
    // epoch starts from state buffer 0), with the tile shape for the number of
    // running systems given to the last set_running.
    int enqueue_epoch(int steps);
    // Record (once) the graph of an epoch of `steps` steps with shape c.
    int record_epoch(int steps, const KernelCfg &c);
    // Enqueue a copy of the device state into the host snapshot and record an
    // event; wait_snapshot blocks until it has arrived.
    int enqueue_snapshot();
    int wait_snapshot();
    bool snapshot_ready();
    // Latest state of system j in the last snapshot (the newer of its two buffers).
    const SysState &state(int j) const
    {
        const SysState &a = snap_[j], &b = snap_[nsys() + j];
        return b.step > a.step ? b : a;
    }
    // Order in which the tiles take the systems: the systems flagged in
    // `running` first (per parity), the rest left out.  Stream-ordered: applies
    // to the kernels enqueued after this call.
    int set_running(const std::vector<char> &running);
    // Tile shape of the next epoch: the tuned shape, or while fewer systems
    // run per parity than it takes, the smallest tuned tile that holds them.
    const KernelCfg &epoch_cfg() const;

private:
    int launch_step(int ver, hipStream_t st, const KernelCfg &c);
    int finish_create();              // common tail of create / create_external
    void carve(void *base);           // device views into the workspace at base
    int mark_stage();                 // the staged host data are being copied
    void wait_stage();                // ... and may be overwritten after this
    int grid_x(const KernelCfg &c) const;
    bool uses_reduction(const KernelCfg &c) const;
    hipError_t launch_reduce(hipStream_t st, int buf, int slot0, int nslots, int nblk) const;
    // Tune the tile shape on this workspace; also fills small_.
    KernelCfg tune_cg();
    KernelCfg default_cg_cfg() const;
    double time_cg_config(const KernelCfg &c, int nblk, bool reduce);
    CgArgs args() const;

    Ctx *ctx_;
    std::shared_ptr<GaugeField> f_;
    int prec_, S_;
    hipStream_t s_;
    KernelCfg cfg_;
    // tuned shapes of tiles smaller than cfg_.rtile, ascending
    std::vector<KernelCfg> small_;
    // blocks per tile row of every kernel of this batch: a prologue reduces
    // one partial sum per block of the kernel before it, so the count never
    // changes between shapes
    int nblk_ = 0;
    // a reduction kernel sums each step kernel's partials before the next
    // kernel reads them (large grids); otherwise every prologue sums them
    bool reduce_ = false;
    int live_ = 0;  // running systems per parity (the larger count), from set_running
    int pstride_ = 0;
    void *mem_ = nullptr;
    size_t bytes_ = 0;
    // device views into mem_
    void *p_[2] = {nullptr, nullptr}, *ap_ = nullptr, *r_ = nullptr;
    flt2 *xlo_ = nullptr;
    dbl2 *tmp_ = nullptr;
    dbl2 **xhi_d_ = nullptr;
    const dbl2 **b_d_ = nullptr;
    SysState *st_d_[2] = {nullptr, nullptr};
    int *perm_d_ = nullptr;
    double *partials_ = nullptr;
    double *totals_ = nullptr;  // [2][nsys][3] totals of the partials (reduction kernel)
    // pinned host memory
    SysState *stage_ = nullptr;   // [nsys] staged initial states
    SysState *snap_ = nullptr;    // [2][nsys] last snapshot of both state buffers
    dbl2 **xhi_h_ = nullptr;
    const dbl2 **b_h_ = nullptr;
    int *perm_h_ = nullptr;
    std::vector<int> perm_last_;
    hipEvent_t snap_ev_ = nullptr, stage_ev_ = nullptr;
    hipEvent_t tune_ev_[2] = {nullptr, nullptr};
    bool stage_busy_ = false;
    bool external_ = false;  // memory from create_external: nothing owned, no events
    // epochs recorded once as HIP graphs (kernel nodes only) and replayed
    bool use_graphs_ = true;
    hipStream_t cap_stream_ = nullptr;
    std::map<int, hipGraphExec_t> graphs_;  // key: rtile * 1024 + steps
};

}  // namespace stag
