// Serving scheduler core: request queue, admission by HBM footprint, batch
// slots, ticks and completion. Host-only C++ (no HIP), templated on an
// executor so that it can be driven by the GPU executor in the library and by
// a fake executor in the CPU tests.
//
// Executor interface (all calls come from the scheduler's own threads):
//   int64_t footprint(const dgo_request &r) const
//   dgo_status prepare(Req &r)                 // after admission, on a prep thread
//   dgo_status tick(std::vector<Req *> &active, int32_t chunk)
//       runs up to `chunk` iterations of every active request (a request's
//       first tick also assembles and initialises it) and returns when that
//       work is complete; sets r.done_iters
//   dgo_status finish(Req &r)                  // copy the result to the host
//   void release(Req &r)                       // drop per-request device state
// finish and release run on a completion thread, concurrently with the next
// tick (which no longer includes the request), so result copies overlap the
// device's work; the request keeps its slot and memory until it is retired
// after them.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/dgo_serve.h"

namespace dgo {
namespace srv {

inline double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator of byte ranges in [0, cap), 256-byte granules.
class Arena {
  public:
    explicit Arena(int64_t cap) : cap_(cap) {
        if (cap > 0) free_[0] = cap;
    }
    static int64_t round(int64_t b) { return (b + 255) & ~int64_t(255); }
    bool alloc(int64_t bytes, int64_t *off) {
        bytes = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const int64_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest > 0) free_[start] = rest;
                in_use_ += bytes;
                peak_ = std::max(peak_, in_use_);
                return true;
            }
        }
        return false;
    }
    void release(int64_t off, int64_t bytes) {
        bytes = round(bytes);
        in_use_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    int64_t cap() const { return cap_; }
    int64_t in_use() const { return in_use_; }
    int64_t peak() const { return peak_; }
    size_t pieces() const { return free_.size(); }

  private:
    int64_t cap_, in_use_ = 0, peak_ = 0;
    std::map<int64_t, int64_t> free_;
};

enum ReqState { Q_QUEUED, Q_PREPARING, Q_READY, Q_ACTIVE, Q_DONE };

struct Req {
    uint64_t ticket = 0;
    dgo_request in{};
    int64_t footprint = 0, arena_off = -1;
    int status = DGO_OK;
    int state = Q_QUEUED;
    int slot = -1;
    double t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;
    int32_t iters = 0, target = 0, done_iters = 0;
    bool initialised = false;
    void *exec = nullptr;  // executor's per-request state
};

template <class Exec>
class Scheduler {
  public:
    Scheduler(Exec &ex, const dgo_server_opts &o) : ex_(ex), o_(o), arena_(o.hbm_budget_bytes) {
        free_slots_.resize(o_.max_slots);
        for (int i = 0; i < o_.max_slots; ++i) free_slots_[i] = o_.max_slots - 1 - i;
        run_ = std::thread([this] { schedule_loop(); });
        done_ = std::thread([this] { complete_loop(); });
        for (int i = 0; i < std::max(1, o_.prep_threads); ++i)
            prep_.emplace_back([this] { prep_loop(); });
    }
    ~Scheduler() { shutdown(); }

    dgo_status submit(const dgo_request &r, uint64_t *ticket) {
        const int64_t fp = ex_.footprint(r);
        std::unique_lock<std::mutex> lk(mu_);
        if (stopping_) return DGO_ERR_SHUTDOWN;
        st_.submitted++;
        if (fp <= 0 || Arena::round(fp) > arena_.cap()) {
            st_.rejected++;
            return DGO_ERR_BUDGET;
        }
        auto q = std::make_unique<Req>();
        q->ticket = ++next_ticket_;
        q->in = r;
        q->footprint = fp;
        q->t_submit = now_s();
        q->target = o_.cg_iters;
        *ticket = q->ticket;
        queue_.push_back(q.get());
        reqs_[q->ticket] = std::move(q);
        cv_.notify_all();
        return DGO_OK;
    }

    dgo_status wait(uint64_t ticket, double timeout_s, dgo_req_stats *out) {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = reqs_.find(ticket);
        if (it == reqs_.end()) return DGO_ERR_INVALID_ARG;
        Req *q = it->second.get();
        // system_clock deadline: a timed wait through pthread_cond_timedwait
        const auto dl = std::chrono::system_clock::now() +
                        std::chrono::duration_cast<std::chrono::system_clock::duration>(
                            std::chrono::duration<double>(timeout_s));
        if (!done_cv_.wait_until(lk, dl, [&] { return q->state == Q_DONE; }))
            return DGO_ERR_TIMEOUT;
        if (out) {
            out->status = q->status;
            out->slot = q->slot;
            out->t_submit = q->t_submit;
            out->t_admit = q->t_admit;
            out->t_start = q->t_start;
            out->t_done = q->t_done;
            out->iters = q->iters;
            out->pad = 0;
            out->footprint = q->footprint;
        }
        const dgo_status s = (dgo_status)q->status;
        reqs_.erase(it);
        return s;
    }

    void stats(dgo_server_counters *o) {
        std::lock_guard<std::mutex> lk(mu_);
        *o = st_;
        o->queue_depth = (int64_t)queue_.size();
        o->active = (int64_t)n_admitted_;
        o->hbm_in_use = arena_.in_use();
        o->hbm_peak = arena_.peak();
        o->busy_s = busy_s_;
        o->now_s = now_s();
    }

    // Finish everything queued or running, then stop the threads.
    void shutdown() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (stopping_ && !run_.joinable()) return;
            stopping_ = true;
            cv_.notify_all();
        }
        for (auto &t : prep_)
            if (t.joinable()) t.join();
        if (run_.joinable()) run_.join();
        if (done_.joinable()) done_.join();
    }

    Arena &arena() { return arena_; }

  private:
    bool admissible_locked() {
        if (queue_.empty() || free_slots_.empty()) return false;
        int64_t off;
        Req *q = queue_.front();
        if (!arena_.alloc(q->footprint, &off)) return false;
        q->arena_off = off;
        return true;
    }

    // Preparation threads: admit the queue's head (FIFO) when a slot is free
    // and its footprint fits, then upload it and build its topology.
    void prep_loop() {
        for (;;) {
            Req *q = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return admissible_locked() || (stopping_ && queue_.empty()); });
                if (queue_.empty()) return;  // stopping and drained
                q = queue_.front();
                queue_.pop_front();
                q->slot = free_slots_.back();
                free_slots_.pop_back();
                q->state = Q_PREPARING;
                q->t_admit = now_s();
                n_admitted_++;
                st_.admitted++;
            }
            const dgo_status s = ex_.prepare(*q);
            if (s != DGO_OK) ex_.release(*q);
            std::lock_guard<std::mutex> lk(mu_);
            if (s != DGO_OK) {
                q->status = s;
                retire_locked(q, false);
            } else {
                q->state = Q_READY;
                ready_.push_back(q);
            }
            cv_.notify_all();
        }
    }

    // The executor's release(q) must have been called (outside the lock).
    void retire_locked(Req *q, bool ok) {
        if (q->arena_off >= 0) arena_.release(q->arena_off, q->footprint);
        q->arena_off = -1;
        free_slots_.push_back(q->slot);
        n_admitted_--;
        q->t_done = now_s();
        q->state = Q_DONE;
        if (ok)
            st_.completed++;
        else
            st_.failed++;
        done_cv_.notify_all();
        cv_.notify_all();
    }

    void schedule_loop() {
        std::vector<Req *> active;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] {
                    return !ready_.empty() || !active.empty() ||
                           (stopping_ && queue_.empty() && n_admitted_ == 0);
                });
                if (ready_.empty() && active.empty()) {
                    sched_done_ = true;
                    cv_.notify_all();
                    return;
                }
                const double t = now_s();
                while (!ready_.empty()) {
                    Req *q = ready_.front();
                    ready_.pop_front();
                    q->state = Q_ACTIVE;
                    q->t_start = t;
                    active.push_back(q);
                }
            }
            const double t0 = now_s();
            const int32_t chunk = o_.cg_chunk > 0 ? o_.cg_chunk : o_.cg_iters;
            const dgo_status s = ex_.tick(active, chunk);
            std::vector<Req *> keep, out;
            for (Req *q : active) {
                q->initialised = true;
                q->iters = q->done_iters;
                if (s != DGO_OK) {
                    q->status = s;
                    out.push_back(q);
                } else if (q->done_iters >= q->target) {
                    q->status = DGO_OK;
                    out.push_back(q);
                } else {
                    keep.push_back(q);
                }
            }
            const double t1 = now_s();
            std::lock_guard<std::mutex> lk(mu_);
            busy_s_ += t1 - t0;
            st_.ticks++;
            st_.max_batch = std::max<int64_t>(st_.max_batch, (int64_t)active.size());
            for (Req *q : out) completing_.push_back(q);
            if (!out.empty()) cv_.notify_all();
            active.swap(keep);
        }
    }

    // Completion thread: copy results out and release the requests that the
    // scheduler finished (or that a failed tick ended), then retire them.
    void complete_loop() {
        for (;;) {
            Req *q = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return !completing_.empty() || sched_done_; });
                if (completing_.empty()) return;  // the scheduler has stopped
                q = completing_.front();
                completing_.pop_front();
            }
            const bool ran = q->status == DGO_OK;
            const dgo_status f = ran ? ex_.finish(*q) : (dgo_status)q->status;
            ex_.release(*q);
            std::lock_guard<std::mutex> lk(mu_);
            q->status = f;
            retire_locked(q, f == DGO_OK);
        }
    }

    Exec &ex_;
    dgo_server_opts o_;
    Arena arena_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    std::deque<Req *> queue_, ready_, completing_;
    std::vector<int> free_slots_;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs_;
    uint64_t next_ticket_ = 0;
    int n_admitted_ = 0;
    bool stopping_ = false, sched_done_ = false;
    double busy_s_ = 0;
    dgo_server_counters st_{};
    std::thread run_, done_;
    std::vector<std::thread> prep_;
};

}  // namespace srv
}  // namespace dgo
