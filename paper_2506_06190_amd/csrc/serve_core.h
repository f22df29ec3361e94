// Request queue, HBM-budgeted admission and continuous batching of the
// served form.  Plain C++17 with no HIP in it: the device work sits behind
// ServeBackend, so the same core runs over the GPU backend of the library
// and over a host-only fake device in tests.
//
// Model.  A server owns one arena of `budget` bytes of device memory and
// n_slots worker threads (one device stream each).  A free worker takes the
// request at the head of the queue, adds later compatible requests in
// arrival order while the batch stays within max_batch requests and its
// workspace still fits a free block of the arena, carves that block, runs
// the batch, and frees the block.  Workers are independent, so batches
// started by different workers overlap on the device, and a request waits
// only until some worker is free and the arena has room: requests join the
// running mix as slots and memory free up.  The head of the queue is never
// overtaken by a request it is incompatible with in a way that could starve
// it: heads are taken strictly in arrival order.
#ifndef NAT_SERVE_CORE_H
#define NAT_SERVE_CORE_H

#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace nat {
namespace serve {

enum ReqState { RS_QUEUED = 0, RS_RUNNING = 1, RS_DONE = 2, RS_CANCELLED = 3 };

// Status values shared with the C interface (nat_status).
enum : int32_t {
    ST_OK = 0, ST_INVALID = 1, ST_BUDGET = 2, ST_NOCONV = 3, ST_PENDING = 6, ST_CANCELLED = 7
};

struct Request {
    uint64_t ticket = 0;
    int32_t exclusive = 0;   // runs in a batch of its own
    int32_t group = 0;       // only requests of equal group share a batch
    size_t solo_bytes = 0;   // workspace of the request alone
    double t_arrive = 0.0;   // ms, backend clock
    double t_start = 0.0;
    double t_done = 0.0;
    int32_t state = RS_QUEUED;
    int32_t status = ST_PENDING;
    int32_t batch_size = 0;
    int32_t slot = -1;
    uint64_t batch_id = 0;
    std::shared_ptr<void> payload;  // the backend's copy of the request
};

// What the core needs from the device side.  batch_bytes and now_ms are
// called with the core's lock held and must not block.
class ServeBackend {
public:
    virtual ~ServeBackend() = default;
    virtual double now_ms() = 0;
    // workspace of the batch, or 0 if these requests cannot share a batch
    virtual size_t batch_bytes(Request* const* reqs, int32_t n) = 0;
    // run a batch in arena bytes [offset, offset + bytes); sets each
    // request's status.  Called from worker `slot` without the lock.
    virtual void run(int32_t slot, Request* const* reqs, int32_t n, size_t offset,
                     size_t bytes) = 0;
    virtual void slot_begin(int32_t /*slot*/) {}
    virtual void slot_end(int32_t /*slot*/) {}
};

// First-fit allocator over [0, capacity) with 256-byte granules.
class Arena {
public:
    static constexpr size_t kAlign = 256;
    explicit Arena(size_t capacity);
    // offset of a block of `bytes`, or SIZE_MAX when no free block is large enough
    size_t alloc(size_t bytes);
    void release(size_t offset);
    size_t largest_free() const;
    size_t in_use() const { return in_use_; }
    size_t capacity() const { return cap_; }

private:
    size_t cap_;
    size_t in_use_ = 0;
    std::map<size_t, size_t> free_;  // offset -> size
    std::map<size_t, size_t> used_;  // offset -> size
};

struct ServeStats {
    int64_t submitted = 0;
    int64_t completed = 0;
    int64_t cancelled = 0;
    int64_t batches = 0;
    int64_t max_batch_seen = 0;
    int32_t max_concurrent = 0;  // batches running at once, peak
    size_t peak_bytes = 0;       // arena bytes in use, peak
    size_t budget = 0;
};

class ServeCore {
public:
    ServeCore(ServeBackend* backend, int32_t n_slots, int32_t max_batch, size_t budget);
    ~ServeCore();  // cancels what is queued, finishes what runs, joins the workers
    ServeCore(const ServeCore&) = delete;
    ServeCore& operator=(const ServeCore&) = delete;

    // Queue a request (its solo_bytes, exclusive, group and payload set).
    // ST_BUDGET if it can never fit the arena; otherwise ST_OK and a ticket.
    int32_t submit(std::unique_ptr<Request> req, uint64_t* ticket);
    // Wait up to timeout_ms (< 0: forever) for the request to finish.  On
    // completion or cancellation copies it to *out, forgets the ticket and
    // returns its status; ST_PENDING if the wait timed out; ST_INVALID for an
    // unknown ticket.
    int32_t wait(uint64_t ticket, double timeout_ms, Request* out);
    // Cancel a request that has not started: ST_OK, else ST_INVALID.
    int32_t cancel(uint64_t ticket);
    ServeStats stats();

private:
    void worker(int32_t slot);
    bool form_batch(std::vector<Request*>& batch, size_t& bytes);

    ServeBackend* be_;
    int32_t max_batch_;
    Arena arena_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::deque<Request*> queue_;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs_;
    std::vector<std::thread> workers_;
    uint64_t next_ticket_ = 1;
    uint64_t next_batch_ = 1;
    int32_t running_ = 0;
    bool stop_ = false;
    ServeStats st_;
};

}  // namespace serve
}  // namespace nat

#endif
