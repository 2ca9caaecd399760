// Serving: a scheduler thread that keeps gauge fields resident, admits CG
// requests into batch slots by memory, and runs each batch in epochs of CG
// iterations on its own stream, retiring converged requests and admitting new
// ones between epochs (continuous batching).
#pragma once

#include <deque>
#include <thread>
#include <unordered_map>

#include "batch.hpp"

namespace stag {

struct Request {
    uint64_t ticket = 0;
    std::shared_ptr<GaugeField> field;
    stag_cg_params params{};
    const double *b = nullptr;
    double *x = nullptr;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int state = 0;  // 0 queued, 1 running, 2 done
    stag_cg_info info{};
    // recorded on the context's stream at submit; the lane waits on it before
    // the request's first kernel, so the caller's earlier work on b and x is done
    hipEvent_t ready = nullptr;
};

struct Lane {
    std::shared_ptr<GaugeField> field;
    int prec = 0;
    hipStream_t stream = nullptr;
    std::unique_ptr<Batch> batch;
    std::vector<std::shared_ptr<Request>> slot;  // request per slot (null = free)
    std::deque<std::shared_ptr<Request>> queue;  // admitted to this lane, waiting for a slot
    bool snapshot_pending = false;
    bool epoch_queued = false;
    int active = 0;
    ~Lane();
};

class Server {
public:
    explicit Server(Ctx *ctx);
    ~Server();
    int submit(const std::shared_ptr<GaugeField> &f, const stag_cg_params &p, const double *b, double *x,
               uint64_t *ticket);
    int poll(uint64_t ticket, stag_cg_info *info, bool wait);
    int release(uint64_t ticket);
    void drop_field(int32_t gauge_id);

private:
    void run();
    bool step_lane(Lane &l);
    int ensure_batch(Lane &l);
    void retire(Lane &l, int slot, int status_override);
    static double now();
    hipEvent_t take_event();            // from the pool (or a new one); caller holds mu_
    void give_event(hipEvent_t e);      // back to the pool; caller holds mu_

    Ctx *ctx_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> tickets_;
    std::deque<std::shared_ptr<Request>> incoming_;
    std::vector<std::unique_ptr<Lane>> lanes_;  // touched by the scheduler thread only
    std::vector<int32_t> dropped_;
    std::vector<hipEvent_t> events_;  // idle events for Request::ready
    uint64_t next_ticket_ = 1;
    int outstanding_ = 0;
    bool stop_ = false;
    std::thread thread_;
};

}  // namespace stag
