// Context-independent runtime pieces: error strings and the arena allocator.
#include "runtime.hpp"

#include <cstdio>

namespace stag {

static thread_local std::string g_last_error;

int set_error(int code, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void clear_error() { g_last_error.clear(); }

const char *last_error_cstr() { return g_last_error.c_str(); }

// ---- arena -------------------------------------------------------------------

static constexpr size_t kAlign = 256;

void Arena::init(void *base, size_t bytes)
{
    std::lock_guard<std::mutex> lk(mu_);
    uintptr_t b = (uintptr_t)base;
    uintptr_t a = (b + kAlign - 1) & ~(uintptr_t)(kAlign - 1);
    base_ = (char *)a;
    size_ = bytes > (a - b) ? ((bytes - (a - b)) & ~(kAlign - 1)) : 0;
    free_.clear();
    live_.clear();
    if (size_)
        free_[0] = size_;
    used_ = 0;
}

void *Arena::alloc(size_t bytes)
{
    if (bytes == 0)
        bytes = kAlign;
    bytes = (bytes + kAlign - 1) & ~(kAlign - 1);
    std::lock_guard<std::mutex> lk(mu_);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second >= bytes) {
            size_t off = it->first, sz = it->second;
            free_.erase(it);
            if (sz > bytes)
                free_[off + bytes] = sz - bytes;
            live_[off] = bytes;
            used_ += bytes;
            return base_ + off;
        }
    }
    return nullptr;
}

void Arena::release(void *p)
{
    if (!p)
        return;
    std::lock_guard<std::mutex> lk(mu_);
    size_t off = (size_t)((char *)p - base_);
    auto it = live_.find(off);
    if (it == live_.end())
        return;
    size_t sz = it->second;
    live_.erase(it);
    used_ -= sz;
    // insert and coalesce with neighbours
    auto ins = free_.emplace(off, sz).first;
    auto next = std::next(ins);
    if (next != free_.end() && ins->first + ins->second == next->first) {
        ins->second += next->second;
        free_.erase(next);
    }
    if (ins != free_.begin()) {
        auto prev = std::prev(ins);
        if (prev->first + prev->second == ins->first) {
            prev->second += ins->second;
            free_.erase(ins);
        }
    }
}

size_t Arena::largest_free() const
{
    std::lock_guard<std::mutex> lk(mu_);
    size_t best = 0;
    for (auto &kv : free_)
        best = kv.second > best ? kv.second : best;
    return best;
}

std::shared_ptr<GaugeField> Ctx::field(int32_t id)
{
    std::lock_guard<std::mutex> lk(mu);
    auto it = fields.find(id);
    return it == fields.end() ? nullptr : it->second;
}

}  // namespace stag
