// Admission control of the spectrum server: plain C++ (no HIP), so the policy
// can be exercised on the host alone.
//
// Every request carries the device bytes it may hold at its peak.  A request
// starts when a worker is free and its bytes fit in what the budget has left.
// The oldest waiting request goes first; when it does not fit, later requests
// that do fit may start ahead of it ("backfill"), but only max_bypass times,
// after which nothing new starts until the oldest one fits, so a large request
// cannot starve behind a stream of small ones.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>

namespace ftk {

class Admission {
  public:
    Admission(size_t budget, int max_running, int max_bypass)
        : budget_(budget), max_running_(max_running), max_bypass_(max_bypass)
    {
    }

    // false if the request could never fit
    bool submit(uint64_t ticket, size_t bytes)
    {
        if (bytes > budget_) return false;
        queue_.push_back({ticket, bytes, 0});
        return true;
    }

    // next request to start, if any may start now; reserves its bytes
    bool pick(uint64_t *ticket, size_t *bytes)
    {
        if (running_ >= max_running_ || queue_.empty()) return false;
        const size_t left = budget_ - in_use_;
        auto take = [&](std::deque<Item>::iterator it) {
            *ticket = it->ticket;
            *bytes = it->bytes;
            in_use_ += it->bytes;
            if (in_use_ > peak_) peak_ = in_use_;
            ++running_;
            queue_.erase(it);
            return true;
        };
        if (queue_.front().bytes <= left) return take(queue_.begin());
        if (queue_.front().bypassed >= max_bypass_) return false;
        for (auto it = queue_.begin() + 1; it != queue_.end(); ++it)
            if (it->bytes <= left) {
                ++queue_.front().bypassed;
                return take(it);
            }
        return false;
    }

    void release(size_t bytes)
    {
        in_use_ -= bytes;
        --running_;
    }

    // drops a waiting request (false if it is not waiting)
    bool cancel(uint64_t ticket)
    {
        for (auto it = queue_.begin(); it != queue_.end(); ++it)
            if (it->ticket == ticket) {
                queue_.erase(it);
                return true;
            }
        return false;
    }

    size_t budget() const { return budget_; }
    size_t in_use() const { return in_use_; }
    size_t peak() const { return peak_; }
    int running() const { return running_; }
    size_t waiting() const { return queue_.size(); }

  private:
    struct Item {
        uint64_t ticket;
        size_t bytes;
        int bypassed;
    };
    size_t budget_;
    int max_running_, max_bypass_;
    size_t in_use_ = 0, peak_ = 0;
    int running_ = 0;
    std::deque<Item> queue_;
};

}  // namespace ftk
