// Host unit checks of GroupBudget (paper_2110_01481_amd/csrc/group_budget.h), the
// admission of spinning Gram-Schmidt block groups. Built and run by
// tests/test_group_budget_host.py with g++; prints "ok" and exits 0 when every check
// holds, else names the failed check and exits 1.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <thread>
#include <vector>

#include "group_budget.h"

using abg::GroupBudget;

static int failures = 0;
#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            std::printf("FAILED: %s (line %d)\n", #c, __LINE__);   \
            ++failures;                                             \
        }                                                           \
    } while (0)

static void sleep_ms(int ms) { std::this_thread::sleep_for(std::chrono::milliseconds(ms)); }

int main()
{
    const long long U = GroupBudget::kUnits;
    // units of a group against the device's capacity for its kernel
    CHECK(GroupBudget::units_for(1, 1024) == 0);        // one block: no exchange
    CHECK(GroupBudget::units_for(0, 1024) == 0);
    CHECK(GroupBudget::units_for(256, 1024) == U / 4);
    CHECK(GroupBudget::units_for(1024, 1024) == U);
    CHECK(GroupBudget::units_for(5000, 1024) == U);     // more than the device: all of it
    CHECK(GroupBudget::units_for(3, 1000) == 3000);
    CHECK(GroupBudget::units_for(1, 3) == 0);
    CHECK(GroupBudget::units_for(2, 3) == (2 * U + 2) / 3);   // rounded up
    CHECK(GroupBudget::units_for(7, 0) == 0);           // unknown capacity: no hold

    // plain accounting
    {
        GroupBudget b;
        b.acquire(U / 2);
        b.acquire(U / 4);
        CHECK(b.in_use() == 3 * U / 4);
        b.release(U / 4);
        CHECK(b.in_use() == U / 2);
        b.acquire(0);
        b.acquire(-5);
        CHECK(b.in_use() == U / 2);
        b.release(U / 2);
        CHECK(b.in_use() == 0);
        b.acquire(3 * U);                               // clamped to the whole device
        CHECK(b.in_use() == U);
        b.release(3 * U);
        CHECK(b.in_use() == 0);
    }

    // a request that does not fit waits until enough is returned
    {
        GroupBudget b;
        b.acquire(3 * U / 4);
        std::atomic<int> got{0};
        std::thread t([&] {
            b.acquire(U / 2);
            got = 1;
        });
        sleep_ms(100);
        CHECK(got.load() == 0);
        b.release(3 * U / 4);
        t.join();
        CHECK(got.load() == 1);
        CHECK(b.in_use() == U / 2);
        b.release(U / 2);
    }

    // arrival order: a large request is not overtaken by later small ones that would fit
    {
        GroupBudget b;
        b.acquire(U / 2);
        std::atomic<int> order{0}, big_at{-1}, small_at{-1};
        std::thread big([&] {
            b.acquire(U);
            big_at = order++;
            b.release(U);
        });
        sleep_ms(100);                                  // the large request is queued first
        std::thread small([&] {
            b.acquire(U / 4);                           // fits now, but arrived later
            small_at = order++;
            b.release(U / 4);
        });
        sleep_ms(100);
        CHECK(big_at.load() == -1 && small_at.load() == -1);
        b.release(U / 2);
        big.join();
        small.join();
        CHECK(big_at.load() == 0 && small_at.load() == 1);
        CHECK(b.in_use() == 0);
    }

    // many threads: the units held never exceed the device, every request is served
    {
        GroupBudget b;
        std::atomic<long long> held{0}, peak{0};
        std::atomic<int> served{0};
        std::vector<std::thread> ts;
        for (int i = 0; i < 16; ++i)
            ts.emplace_back([&, i] {
                const long long u = (i % 4 + 1) * U / 5;    // 0.2 .. 0.8 of the device
                for (int r = 0; r < 50; ++r) {
                    b.acquire(u);
                    const long long h = held += u;
                    long long p = peak.load();
                    while (h > p && !peak.compare_exchange_weak(p, h)) {}
                    std::this_thread::yield();
                    held -= u;
                    b.release(u);
                    ++served;
                }
            });
        for (auto &t : ts) t.join();
        CHECK(peak.load() <= U);
        CHECK(served.load() == 16 * 50);
        CHECK(b.in_use() == 0);
    }

    // release from another thread (as a stream callback does)
    {
        GroupBudget b;
        b.acquire(U);
        std::thread r([&] { b.release(U); });
        r.join();
        CHECK(b.in_use() == 0);
    }

    if (failures) return 1;
    std::printf("ok\n");
    return 0;
}
