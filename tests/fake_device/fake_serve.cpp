// Host-only fake device for the served form's scheduling core: a batch
// "runs" by sleeping for its longest member's simulated duration, its
// workspace is a fixed overhead plus the members' bytes, and every arena
// block handed out is checked against the budget and against the blocks of
// the batches running at the same time.  Built with g++ by the tests.
#include <algorithm>
#include <chrono>
#include <cstdint>
#include <memory>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "serve_core.h"

using nat::serve::Request;

namespace {

struct FakeReq {
    size_t bytes;
    double run_ms;
    int32_t status;
};

class FakeBackend final : public nat::serve::ServeBackend {
public:
    FakeBackend(size_t budget, size_t overhead) : budget_(budget), overhead_(overhead) {}

    double now_ms() override
    {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0_)
            .count();
    }

    size_t batch_bytes(Request* const* r, int32_t n) override
    {
        size_t b = overhead_;
        for (int32_t i = 0; i < n; ++i)
            b += static_cast<FakeReq*>(r[i]->payload.get())->bytes;
        return b;
    }

    void run(int32_t, Request* const* r, int32_t n, size_t offset, size_t bytes) override
    {
        double ms = 0.0;
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (offset + bytes > budget_)
                ++violations_;
            for (const auto& blk : live_)
                if (offset < blk.first + blk.second && blk.first < offset + bytes)
                    ++violations_;
            live_.emplace_back(offset, bytes);
            for (int32_t i = 0; i < n; ++i)
                log_.push_back({(int64_t)r[i]->batch_id, (int64_t)r[i]->ticket});
        }
        for (int32_t i = 0; i < n; ++i) {
            const FakeReq* f = static_cast<FakeReq*>(r[i]->payload.get());
            ms = std::max(ms, f->run_ms);
            r[i]->status = f->status;
        }
        std::this_thread::sleep_for(std::chrono::microseconds((int64_t)(ms * 1e3)));
        std::lock_guard<std::mutex> lk(mu_);
        live_.erase(std::find(live_.begin(), live_.end(), std::make_pair(offset, bytes)));
    }

    std::mutex mu_;
    int64_t violations_ = 0;
    std::vector<std::pair<size_t, size_t>> live_;
    std::vector<std::pair<int64_t, int64_t>> log_;  // (batch id, ticket) in start order

private:
    size_t budget_, overhead_;
    std::chrono::steady_clock::time_point t0_ = std::chrono::steady_clock::now();
};

struct FakeServer {
    std::unique_ptr<FakeBackend> be;
    std::unique_ptr<nat::serve::ServeCore> core;
};

}  // namespace

extern "C" {

void* fs_create(int32_t n_slots, int32_t max_batch, uint64_t budget, uint64_t overhead)
{
    auto* s = new FakeServer();
    s->be.reset(new FakeBackend(budget, overhead));
    s->core.reset(new nat::serve::ServeCore(s->be.get(), n_slots, max_batch, budget));
    return s;
}

int32_t fs_submit(void* h, uint64_t bytes, double run_ms, int32_t exclusive, int32_t group,
                  int32_t status, uint64_t* ticket)
{
    auto* s = static_cast<FakeServer*>(h);
    std::unique_ptr<Request> r(new Request());
    r->payload = std::make_shared<FakeReq>(FakeReq{bytes, run_ms, status});
    r->exclusive = exclusive;
    r->group = group;
    Request* one = r.get();
    r->solo_bytes = s->be->batch_bytes(&one, 1);
    return s->core->submit(std::move(r), ticket);
}

// out: latency, queue, run (ms), batch size, slot, batch id
int32_t fs_wait(void* h, uint64_t ticket, double timeout_ms, double* out)
{
    auto* s = static_cast<FakeServer*>(h);
    Request r;
    const int32_t st = s->core->wait(ticket, timeout_ms, &r);
    if (out && st != nat::serve::ST_PENDING) {
        out[0] = r.t_done - r.t_arrive;
        out[1] = r.slot >= 0 ? r.t_start - r.t_arrive : out[0];
        out[2] = r.slot >= 0 ? r.t_done - r.t_start : 0.0;
        out[3] = r.batch_size;
        out[4] = r.slot;
        out[5] = (double)r.batch_id;
    }
    return st;
}

int32_t fs_cancel(void* h, uint64_t ticket) { return static_cast<FakeServer*>(h)->core->cancel(ticket); }

// out: submitted, completed, cancelled, batches, max batch, max concurrent,
// peak bytes, arena violations
void fs_stats(void* h, int64_t* out)
{
    auto* s = static_cast<FakeServer*>(h);
    const nat::serve::ServeStats st = s->core->stats();
    out[0] = st.submitted;
    out[1] = st.completed;
    out[2] = st.cancelled;
    out[3] = st.batches;
    out[4] = st.max_batch_seen;
    out[5] = st.max_concurrent;
    out[6] = (int64_t)st.peak_bytes;
    std::lock_guard<std::mutex> lk(s->be->mu_);
    out[7] = s->be->violations_;
}

// (batch id, ticket) pairs in the order batches started; returns the count
int64_t fs_batch_log(void* h, int64_t* out, int64_t max_pairs)
{
    auto* s = static_cast<FakeServer*>(h);
    std::lock_guard<std::mutex> lk(s->be->mu_);
    const int64_t n = std::min<int64_t>(max_pairs, (int64_t)s->be->log_.size());
    for (int64_t i = 0; i < n; ++i) {
        out[2 * i] = s->be->log_[i].first;
        out[2 * i + 1] = s->be->log_[i].second;
    }
    return (int64_t)s->be->log_.size();
}

// stops the server: queued requests are cancelled, running batches finish
void fs_destroy(void* h)
{
    auto* s = static_cast<FakeServer*>(h);
    s->core.reset();
    delete s;
}

}  // extern "C"
