// Host-side admission of spinning block groups (host C++ only, no HIP).
//
// A multi-block Gram-Schmidt launch exchanges partial sums between the blocks of its
// group and waits for them on the device, so the whole group must be resident at once.
// Launches from different streams (concurrent solves, an engine beside single solves)
// could together need more resident blocks than the device holds and then wait on each
// other. Each such launch therefore holds a share of the device, in units of 1/kUnits of
// what the device holds of its kernel, from before it is enqueued until it is known to
// have finished; a request waits on the host until its share fits. Requests are served
// in arrival order (a large one is not overtaken by later small ones), and a request for
// more than the whole device is taken as the whole device (it then runs alone).
#pragma once

#include <condition_variable>
#include <mutex>

namespace abg {

class GroupBudget {
public:
    static constexpr long long kUnits = 1000000;

    // Units of a group of g blocks of a kernel the device holds `cap` blocks of at once
    // (0 for a single block: it exchanges nothing between blocks).
    static long long units_for(long long g, long long cap)
    {
        if (g <= 1 || cap <= 0) return 0;
        if (g >= cap) return kUnits;
        return (g * kUnits + cap - 1) / cap;
    }

    // Blocks until `units` fit beside what is held, after every earlier request.
    void acquire(long long units)
    {
        if (units <= 0) return;
        if (units > kUnits) units = kUnits;
        std::unique_lock<std::mutex> lk(mu_);
        const unsigned long long ticket = next_++;
        cv_.wait(lk, [&] { return serving_ == ticket && used_ + units <= kUnits; });
        used_ += units;
        ++serving_;
        cv_.notify_all();
    }

    // Returns what acquire(units) took. Safe to call from any thread (also from a HIP
    // stream callback: it touches only this object).
    void release(long long units)
    {
        if (units <= 0) return;
        if (units > kUnits) units = kUnits;
        {
            std::lock_guard<std::mutex> lk(mu_);
            used_ -= units;
        }
        cv_.notify_all();
    }

    long long in_use() const
    {
        std::lock_guard<std::mutex> lk(mu_);
        return used_;
    }

private:
    mutable std::mutex mu_;
    std::condition_variable cv_;
    long long used_ = 0;
    unsigned long long next_ = 0, serving_ = 0;
};

}  // namespace abg
