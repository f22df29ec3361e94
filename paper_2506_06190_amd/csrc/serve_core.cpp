// Request queue, admission and continuous batching of the served form (see
// serve_core.h for the model).
#include "serve_core.h"

#include <algorithm>
#include <chrono>
#include <cstdint>

namespace nat {
namespace serve {

namespace {
size_t round_up(size_t b) { return (b + Arena::kAlign - 1) / Arena::kAlign * Arena::kAlign; }
}  // namespace

Arena::Arena(size_t capacity) : cap_(capacity / kAlign * kAlign)
{
    if (cap_)
        free_[0] = cap_;
}

size_t Arena::alloc(size_t bytes)
{
    const size_t want = round_up(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second < want)
            continue;
        const size_t off = it->first, sz = it->second;
        free_.erase(it);
        if (sz > want)
            free_[off + want] = sz - want;
        used_[off] = want;
        in_use_ += want;
        return off;
    }
    return SIZE_MAX;
}

void Arena::release(size_t offset)
{
    auto u = used_.find(offset);
    if (u == used_.end())
        return;
    size_t off = u->first, sz = u->second;
    used_.erase(u);
    in_use_ -= sz;
    // merge with the free neighbours
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + sz == next->first) {
        sz += next->second;
        next = free_.erase(next);
    }
    if (next != free_.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == off) {
            prev->second += sz;
            return;
        }
    }
    free_[off] = sz;
}

size_t Arena::largest_free() const
{
    size_t m = 0;
    for (const auto& f : free_)
        m = std::max(m, f.second);
    return m;
}

ServeCore::ServeCore(ServeBackend* backend, int32_t n_slots, int32_t max_batch, size_t budget)
    : be_(backend), max_batch_(std::max<int32_t>(1, max_batch)), arena_(budget)
{
    st_.budget = arena_.capacity();
    for (int32_t s = 0; s < n_slots; ++s)
        workers_.emplace_back(&ServeCore::worker, this, s);
}

ServeCore::~ServeCore()
{
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
        for (Request* r : queue_) {
            r->state = RS_CANCELLED;
            r->status = ST_CANCELLED;
            ++st_.cancelled;
        }
        queue_.clear();
    }
    cv_work_.notify_all();
    for (auto& t : workers_)
        t.join();
    cv_done_.notify_all();
}

int32_t ServeCore::submit(std::unique_ptr<Request> req, uint64_t* ticket)
{
    std::lock_guard<std::mutex> lk(mu_);
    if (round_up(req->solo_bytes) > arena_.capacity())
        return ST_BUDGET;
    if (stop_)
        return ST_INVALID;
    req->ticket = next_ticket_++;
    req->t_arrive = be_->now_ms();
    req->state = RS_QUEUED;
    req->status = ST_PENDING;
    Request* r = req.get();
    *ticket = r->ticket;
    reqs_[r->ticket] = std::move(req);
    queue_.push_back(r);
    ++st_.submitted;
    cv_work_.notify_one();
    return ST_OK;
}

int32_t ServeCore::cancel(uint64_t ticket)
{
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end() || it->second->state != RS_QUEUED)
        return ST_INVALID;
    Request* r = it->second.get();
    queue_.erase(std::find(queue_.begin(), queue_.end(), r));
    r->state = RS_CANCELLED;
    r->status = ST_CANCELLED;
    r->t_done = be_->now_ms();
    ++st_.cancelled;
    cv_done_.notify_all();
    cv_work_.notify_all();  // the head may have changed
    return ST_OK;
}

int32_t ServeCore::wait(uint64_t ticket, double timeout_ms, Request* out)
{
    std::unique_lock<std::mutex> lk(mu_);
    auto finished = [&] {
        auto it = reqs_.find(ticket);
        return it == reqs_.end() || it->second->state == RS_DONE ||
               it->second->state == RS_CANCELLED;
    };
    if (timeout_ms < 0.0) {
        cv_done_.wait(lk, finished);
    } else {
        const auto until = std::chrono::steady_clock::now() +
                           std::chrono::microseconds(static_cast<int64_t>(timeout_ms * 1e3));
        if (!cv_done_.wait_until(lk, until, finished))
            return ST_PENDING;
    }
    auto it = reqs_.find(ticket);
    if (it == reqs_.end())
        return ST_INVALID;
    Request* r = it->second.get();
    const int32_t status = r->status;
    if (out)
        *out = *r;
    reqs_.erase(it);
    return status;
}

ServeStats ServeCore::stats()
{
    std::lock_guard<std::mutex> lk(mu_);
    return st_;
}

// With the lock held: the batch the queue's head starts, within max_batch
// requests and the largest free block.  False if the head does not fit now.
bool ServeCore::form_batch(std::vector<Request*>& batch, size_t& bytes)
{
    batch.clear();
    Request* head = queue_.front();
    const size_t room = arena_.largest_free();
    batch.push_back(head);
    bytes = be_->batch_bytes(batch.data(), 1);
    if (bytes == 0 || round_up(bytes) > room)
        return false;
    if (head->exclusive)
        return true;
    for (size_t i = 1; i < queue_.size() && (int32_t)batch.size() < max_batch_; ++i) {
        Request* r = queue_[i];
        if (r->exclusive || r->group != head->group)
            continue;
        batch.push_back(r);
        const size_t b = be_->batch_bytes(batch.data(), (int32_t)batch.size());
        if (b == 0 || round_up(b) > room) {
            batch.pop_back();
            break;  // keep arrival order: nothing behind a request that does not fit joins
        }
        bytes = b;
    }
    return true;
}

void ServeCore::worker(int32_t slot)
{
    be_->slot_begin(slot);
    std::vector<Request*> batch;
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
        if (stop_)
            break;
        if (queue_.empty()) {
            cv_work_.wait(lk);
            continue;
        }
        size_t bytes = 0;
        if (!form_batch(batch, bytes)) {
            if (bytes != 0 && running_ > 0) {
                // the head waits for memory that running batches hold
                cv_work_.wait(lk);
                continue;
            }
            // the head cannot run at all: fail it rather than block the queue
            Request* h = queue_.front();
            queue_.pop_front();
            h->state = RS_DONE;
            h->status = bytes == 0 ? ST_INVALID : ST_BUDGET;
            h->t_start = h->t_done = be_->now_ms();
            ++st_.completed;
            cv_done_.notify_all();
            continue;
        }
        const size_t off = arena_.alloc(bytes);
        if (off == SIZE_MAX) {
            cv_work_.wait(lk);
            continue;
        }
        const uint64_t bid = next_batch_++;
        const double t0 = be_->now_ms();
        for (Request* r : batch) {
            queue_.erase(std::find(queue_.begin(), queue_.end(), r));
            r->state = RS_RUNNING;
            r->t_start = t0;
            r->batch_size = (int32_t)batch.size();
            r->slot = slot;
            r->batch_id = bid;
        }
        ++running_;
        ++st_.batches;
        st_.max_batch_seen = std::max<int64_t>(st_.max_batch_seen, (int64_t)batch.size());
        st_.max_concurrent = std::max(st_.max_concurrent, running_);
        st_.peak_bytes = std::max(st_.peak_bytes, arena_.in_use());
        if (!queue_.empty())
            cv_work_.notify_one();  // another free worker may start the next batch
        lk.unlock();
        be_->run(slot, batch.data(), (int32_t)batch.size(), off, bytes);
        lk.lock();
        arena_.release(off);
        --running_;
        const double t1 = be_->now_ms();
        for (Request* r : batch) {
            r->state = RS_DONE;
            r->t_done = t1;
            ++st_.completed;
        }
        cv_done_.notify_all();
        cv_work_.notify_all();
    }
    lk.unlock();
    be_->slot_end(slot);
}

}  // namespace serve
}  // namespace nat
