// The serving scheduler (continuous batching of CG requests).
#include <algorithm>
#include <chrono>
#include <cstring>

#include "serve.hpp"

namespace stag {

void fill_info(const Batch &B, int slot, stag_cg_info *info);

Lane::~Lane()
{
    batch.reset();
    if (stream)
        (void)hipStreamDestroy(stream);
}

double Server::now()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

Server::Server(Ctx *ctx) : ctx_(ctx) { thread_ = std::thread([this] { run(); }); }

Server::~Server()
{
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_work_.notify_all();
    if (thread_.joinable())
        thread_.join();
    std::lock_guard<std::mutex> lk(mu_);
    for (auto &kv : tickets_) {
        Request &r = *kv.second;
        if (r.state != 2) {
            r.state = 2;
            r.info.status = STAG_ECANCELED;
            r.field->users.fetch_sub(1);
        }
        if (r.ready) {
            (void)hipEventDestroy(r.ready);
            r.ready = nullptr;
        }
    }
    for (hipEvent_t e : events_)
        (void)hipEventDestroy(e);
    events_.clear();
    cv_done_.notify_all();
}

hipEvent_t Server::take_event()
{
    if (!events_.empty()) {
        hipEvent_t e = events_.back();
        events_.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
        return nullptr;
    return e;
}

void Server::give_event(hipEvent_t e)
{
    if (e)
        events_.push_back(e);
}

int Server::submit(const std::shared_ptr<GaugeField> &f, const stag_cg_params &p, const double *b, double *x,
                   uint64_t *ticket)
{
    auto r = std::make_shared<Request>();
    r->field = f;
    r->params = p;
    r->b = b;
    r->x = x;
    r->t_submit = now();
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (stop_)
            return set_error(STAG_ECANCELED, "server is shutting down");
        if (outstanding_ >= ctx_->queue_capacity)
            return set_error(STAG_EAGAIN, "request queue full (%d outstanding)", outstanding_);
        r->ready = take_event();
        if (!r->ready || hipEventRecord(r->ready, ctx_->stream) != hipSuccess) {
            give_event(r->ready);
            return set_error(STAG_EHIP, "stag_submit: could not record the ordering event");
        }
        r->ticket = next_ticket_++;
        ++outstanding_;
        f->users.fetch_add(1);
        tickets_[r->ticket] = r;
        incoming_.push_back(r);
        *ticket = r->ticket;
    }
    cv_work_.notify_one();
    return STAG_OK;
}

int Server::poll(uint64_t ticket, stag_cg_info *info, bool wait)
{
    std::unique_lock<std::mutex> lk(mu_);
    auto it = tickets_.find(ticket);
    if (it == tickets_.end())
        return set_error(STAG_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    std::shared_ptr<Request> r = it->second;
    if (wait)
        cv_done_.wait(lk, [&] { return r->state == 2; });
    if (r->state != 2)
        return STAG_PENDING;
    if (info)
        *info = r->info;
    return r->info.status;
}

int Server::release(uint64_t ticket)
{
    std::lock_guard<std::mutex> lk(mu_);
    auto it = tickets_.find(ticket);
    if (it == tickets_.end())
        return set_error(STAG_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second->state != 2)
        return set_error(STAG_EBUSY, "ticket %llu is still pending", (unsigned long long)ticket);
    tickets_.erase(it);
    return STAG_OK;
}

void Server::drop_field(int32_t gauge_id)
{
    {
        std::lock_guard<std::mutex> lk(mu_);
        dropped_.push_back(gauge_id);
    }
    cv_work_.notify_one();
    // wait until the scheduler has released the field's lanes
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            bool pending = false;
            for (int32_t d : dropped_)
                pending |= d == gauge_id;
            if (!pending || stop_)
                return;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
}

// Workspace for the lane's batch; halves the slot count until it fits.
int Server::ensure_batch(Lane &l)
{
    if (l.batch)
        return STAG_OK;
    int S = ctx_->slots_per_field;
    for (;;) {
        std::unique_ptr<Batch> b(new Batch(ctx_, l.field, l.prec, S, l.stream));
        int rc = b->create();
        if (rc == STAG_OK) {
            l.batch = std::move(b);
            l.slot.assign(S, nullptr);
            l.active = 0;
            l.snapshot_pending = false;
            l.epoch_queued = false;
            return STAG_OK;
        }
        if (rc != STAG_ENOMEM || S == 1)
            return rc;
        S = S / 2;
    }
}

void Server::retire(Lane &l, int slot, int status_override)
{
    std::shared_ptr<Request> r = l.slot[slot];
    l.slot[slot] = nullptr;
    --l.active;
    stag_cg_info info;
    memset(&info, 0, sizeof(info));
    if (status_override == STAG_OK) {
        fill_info(*l.batch, slot, &info);
    } else {
        info.status = status_override;
    }
    {
        std::lock_guard<std::mutex> lk(mu_);
        r->t_done = now();
        info.seconds = r->t_done - r->t_submit;
        info.queue_seconds = r->t_admit > 0 ? r->t_admit - r->t_submit : 0.0;
        r->info = info;
        r->state = 2;
        --outstanding_;
        r->field->users.fetch_sub(1);
    }
    cv_done_.notify_all();
}

// One scheduling step of a lane; returns true if it made progress.
bool Server::step_lane(Lane &l)
{
    bool progress = false;
    Batch *B = l.batch.get();
    // keep one epoch queued beyond the outstanding snapshot
    if (B && l.active > 0 && !l.epoch_queued) {
        if (B->enqueue_epoch(ctx_->epoch_iters) == STAG_OK)
            l.epoch_queued = true;
        progress = true;
    }
    if (B && l.snapshot_pending && B->snapshot_ready()) {
        l.snapshot_pending = false;
        progress = true;
        for (int s = 0; s < B->slots(); ++s) {
            if (!l.slot[s])
                continue;
            bool done = true;
            for (int par = 0; par < 2; ++par) {
                const int md = B->state(par * B->slots() + s).mode;
                done &= md == M_DONE || md == M_IDLE;
            }
            if (done)
                retire(l, s, STAG_OK);
        }
    }
    if (!l.snapshot_pending) {
        // admit queued requests into free slots
        if (!l.queue.empty() && ensure_batch(l) == STAG_OK) {
            B = l.batch.get();
            std::vector<int> systems;
            const size_t half = (size_t)3 * l.field->g.Vh * 2;
            for (int s = 0; s < B->slots() && !l.queue.empty(); ++s) {
                if (l.slot[s])
                    continue;
                std::shared_ptr<Request> r = l.queue.front();
                l.queue.pop_front();
                l.slot[s] = r;
                ++l.active;
                // the caller's work on b and x, enqueued before submit, comes first
                hipEvent_t ready = nullptr;
                {
                    std::lock_guard<std::mutex> lk(mu_);
                    r->t_admit = now();
                    r->state = 1;
                    ready = r->ready;
                    r->ready = nullptr;
                }
                if (ready) {
                    (void)hipStreamWaitEvent(l.stream, ready, 0);
                    std::lock_guard<std::mutex> lk(mu_);
                    give_event(ready);
                }
                for (int par = 0; par < 2; ++par) {
                    const bool on = r->params.parity == STAG_ALL || r->params.parity == par;
                    B->stage_system(par * B->slots() + s, r->params, on ? r->b + par * half : nullptr,
                                    on ? r->x + par * half : nullptr);
                    systems.push_back(par * B->slots() + s);
                }
            }
            if (!systems.empty()) {
                if (B->upload_and_init(systems) != STAG_OK) {
                    for (size_t k = 0; k < systems.size(); k += 2) {
                        const int s = systems[k];  // parity-0 system index == slot
                        if (l.slot[s])
                            retire(l, s, STAG_EHIP);
                    }
                }
                l.epoch_queued = false;
                progress = true;
            }
        }
        if (B && l.active > 0) {
            // tiles take only the systems of occupied slots
            std::vector<char> running(B->nsys(), 0);
            for (int s = 0; s < B->slots(); ++s) {
                if (!l.slot[s])
                    continue;
                for (int par = 0; par < 2; ++par) {
                    const int par_req = l.slot[s]->params.parity;
                    running[par * B->slots() + s] = par_req == STAG_ALL || par_req == par;
                }
            }
            (void)B->set_running(running);
            if (B->enqueue_snapshot() == STAG_OK) {
                l.snapshot_pending = true;
                l.epoch_queued = false;
                progress = true;
            }
        }
    }
    return progress;
}

void Server::run()
{
    (void)hipSetDevice(ctx_->device);
    for (;;) {
        std::vector<std::shared_ptr<Request>> fresh;
        std::vector<int32_t> drops;
        {
            std::unique_lock<std::mutex> lk(mu_);
            bool busy = false;
            for (auto &l : lanes_)
                busy |= l->active > 0 || !l->queue.empty();
            if (!busy && incoming_.empty() && dropped_.empty() && !stop_)
                cv_work_.wait_for(lk, std::chrono::milliseconds(50));
            if (stop_)
                break;
            fresh.assign(incoming_.begin(), incoming_.end());
            incoming_.clear();
            drops = dropped_;
        }
        for (auto &r : fresh) {
            Lane *lane = nullptr;
            for (auto &l : lanes_)
                if (l->field->id == r->field->id && l->prec == r->params.precision)
                    lane = l.get();
            if (!lane) {
                std::unique_ptr<Lane> nl(new Lane());
                nl->field = r->field;
                nl->prec = r->params.precision;
                if (hipStreamCreateWithFlags(&nl->stream, hipStreamNonBlocking) != hipSuccess) {
                    std::lock_guard<std::mutex> lk(mu_);
                    give_event(r->ready);
                    r->ready = nullptr;
                    r->state = 2;
                    r->info.status = STAG_EHIP;
                    --outstanding_;
                    r->field->users.fetch_sub(1);
                    cv_done_.notify_all();
                    continue;
                }
                lane = nl.get();
                lanes_.push_back(std::move(nl));
            }
            lane->queue.push_back(r);
        }
        bool progress = false;
        for (auto &l : lanes_)
            progress |= step_lane(*l);
        // requests that can never be admitted: no memory even with every other lane idle
        for (auto &l : lanes_) {
            if (!l->batch && !l->queue.empty()) {
                bool others_busy = false;
                for (auto &o : lanes_)
                    others_busy |= o.get() != l.get() && o->batch != nullptr;
                if (!others_busy) {
                    while (!l->queue.empty()) {
                        std::shared_ptr<Request> r = l->queue.front();
                        l->queue.pop_front();
                        std::lock_guard<std::mutex> lk(mu_);
                        give_event(r->ready);
                        r->ready = nullptr;
                        r->state = 2;
                        r->info.status = STAG_ENOMEM;
                        --outstanding_;
                        r->field->users.fetch_sub(1);
                        cv_done_.notify_all();
                    }
                }
            }
        }
        // release the workspace of idle lanes so other fields can be admitted
        for (auto it = lanes_.begin(); it != lanes_.end();) {
            Lane &l = **it;
            bool dropped = false;
            for (int32_t d : drops)
                dropped |= d == l.field->id;
            if (l.active == 0 && l.queue.empty() && !l.snapshot_pending) {
                bool waiting_elsewhere = false;
                for (auto &o : lanes_)
                    waiting_elsewhere |= !o->batch && !o->queue.empty();
                if (dropped || waiting_elsewhere) {
                    (void)hipStreamSynchronize(l.stream);
                    it = lanes_.erase(it);
                    continue;
                }
            }
            ++it;
        }
        if (!drops.empty()) {
            std::lock_guard<std::mutex> lk(mu_);
            for (int32_t d : drops) {
                bool still = false;
                for (auto &l : lanes_)
                    still |= l->field->id == d;
                if (!still)
                    dropped_.erase(std::remove(dropped_.begin(), dropped_.end(), d), dropped_.end());
            }
        }
        if (!progress)
            std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    // shutdown: finish outstanding device work of every lane
    for (auto &l : lanes_)
        (void)hipStreamSynchronize(l->stream);
    lanes_.clear();
}

}  // namespace stag
