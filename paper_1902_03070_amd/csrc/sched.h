// Host-only request scheduler of the serving loop: admission by device-memory
// footprint, first-in-first-out order, a cap on running requests, cancellation
// and deadlines.  It holds no device state and makes no HIP call, so the same
// code runs in the server and, without a GPU, in the tests (which drive it
// with a simulated executor).  Not thread-safe: the server calls it under its
// lock.
#pragma once

#include <stdint.h>

#include <deque>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/tsvdmi.h"

namespace tsvd {

class Scheduler {
public:
    enum State { kUnknown = 0, kPending = 1, kActive = 2, kDone = 3 };

    void configure(int64_t budget_bytes, int max_active) {
        budget_ = budget_bytes;
        max_active_ = max_active;
    }

    // A new request of `footprint` bytes, submitted at time t, that must end by
    // `deadline` (0: none).  Returns its id (> 0), or TSVD_EBUSY when it can
    // never fit the budget.
    int64_t submit(int64_t footprint, double t, double deadline) {
        if (footprint > budget_) return TSVD_EBUSY;
        Entry e;
        e.id = next_id_++;
        e.footprint = footprint;
        e.t_submit = t;
        e.deadline = deadline;
        e.state = kPending;
        map_[e.id] = e;
        queue_.push_back(e.id);
        return e.id;
    }

    // Admits queued requests in arrival order while the head fits the memory
    // left and fewer than max_active run.  The head is never overtaken, so a
    // large request is not starved by later small ones.  Returns the ids.
    std::vector<int64_t> admit(double t) {
        std::vector<int64_t> out;
        while (!queue_.empty() && active_ < max_active_) {
            Entry& e = map_.at(queue_.front());
            if (held_ + e.footprint > budget_) break;
            queue_.pop_front();
            e.state = kActive;
            e.t_admit = t;
            held_ += e.footprint;
            peak_ = held_ > peak_ ? held_ : peak_;
            ++active_;
            ++admitted_;
            out.push_back(e.id);
        }
        return out;
    }

    // Queued requests past their deadline end with TSVD_ETIMEOUT.
    void expire(double t) {
        for (auto it = queue_.begin(); it != queue_.end();) {
            Entry& e = map_.at(*it);
            if (e.deadline > 0.0 && t > e.deadline) {
                e.state = kDone;
                e.status = TSVD_ETIMEOUT;
                ++completed_;
                it = queue_.erase(it);
            } else {
                ++it;
            }
        }
    }

    // Running requests that must stop before the next step: cancelled ones
    // (TSVD_ECANCELED) and those past their deadline (TSVD_ETIMEOUT).  Each is
    // returned once; the server then ends it with finish().
    std::vector<std::pair<int64_t, int>> take_stopped(double t) {
        std::vector<std::pair<int64_t, int>> out;
        for (auto& kv : map_) {
            Entry& e = kv.second;
            if (e.state != kActive || e.stop_sent) continue;
            int code = 0;
            if (e.cancel) code = TSVD_ECANCELED;
            else if (e.deadline > 0.0 && t > e.deadline) code = TSVD_ETIMEOUT;
            if (!code) continue;
            e.stop_sent = true;
            out.emplace_back(e.id, code);
        }
        return out;
    }

    // Cancels a request: a queued one ends at once, a running one at the next
    // step boundary.  Returns 0, 1 if it had already ended, TSVD_EINVAL if unknown.
    int cancel(int64_t id, double t) {
        (void)t;
        auto it = map_.find(id);
        if (it == map_.end()) return TSVD_EINVAL;
        Entry& e = it->second;
        if (e.state == kDone) return 1;
        if (e.state == kPending) {
            for (auto q = queue_.begin(); q != queue_.end(); ++q)
                if (*q == id) {
                    queue_.erase(q);
                    break;
                }
            e.state = kDone;
            e.status = TSVD_ECANCELED;
            ++completed_;
            return 0;
        }
        e.cancel = true;
        return 0;
    }

    // A running request ended with `status`; its memory is released.
    void finish(int64_t id, int status) {
        auto it = map_.find(id);
        if (it == map_.end() || it->second.state != kActive) return;
        Entry& e = it->second;
        e.state = kDone;
        e.status = status;
        held_ -= e.footprint;
        --active_;
        ++completed_;
    }

    State state(int64_t id) const {
        auto it = map_.find(id);
        return it == map_.end() ? kUnknown : it->second.state;
    }
    int status(int64_t id) const {
        auto it = map_.find(id);
        return it == map_.end() ? TSVD_EINVAL : it->second.status;
    }
    // Drops a finished request's record (after its result was collected).
    void forget(int64_t id) {
        auto it = map_.find(id);
        if (it != map_.end() && it->second.state == kDone) map_.erase(it);
    }

    int64_t held() const { return held_; }
    int64_t peak() const { return peak_; }
    int64_t admitted() const { return admitted_; }
    int64_t completed() const { return completed_; }
    int active() const { return active_; }
    int64_t queued() const { return (int64_t)queue_.size(); }

private:
    struct Entry {
        int64_t id = 0, footprint = 0;
        double t_submit = 0.0, t_admit = -1.0, deadline = 0.0;
        State state = kUnknown;
        int status = TSVD_OK;
        bool cancel = false, stop_sent = false;
    };
    int64_t budget_ = 0;
    int max_active_ = 1;
    int64_t next_id_ = 1, held_ = 0, peak_ = 0, admitted_ = 0, completed_ = 0;
    int active_ = 0;
    std::deque<int64_t> queue_;
    std::unordered_map<int64_t, Entry> map_;
};

}  // namespace tsvd
