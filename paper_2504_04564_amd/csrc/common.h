// Internal helpers shared by the host-side translation units of libvdbc.
#pragma once
#include <atomic>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <thread>
#include <vector>

#include "../../include/vdbc.h"

namespace vdbc {

// Records the detail text of the failing call (thread-local) and returns s.
vdbc_status fail(vdbc_status s, const char* fmt, ...);
void clear_error();

// Runs fn(task) for task in [0, n) on `threads` workers (dynamic scheduling).
template <class F>
void parallel_for(uint64_t n, unsigned threads, F&& fn)
{
    if (threads <= 1 || n <= 1) {
        for (uint64_t i = 0; i < n; ++i) fn(i, 0u);
        return;
    }
    if (threads > n) threads = (unsigned)n;
    std::atomic<uint64_t> next{0};
    std::vector<std::thread> pool;
    pool.reserve(threads);
    for (unsigned t = 0; t < threads; ++t)
        pool.emplace_back([&, t] {
            for (;;) {
                uint64_t i = next.fetch_add(1, std::memory_order_relaxed);
                if (i >= n) break;
                fn(i, t);
            }
        });
    for (auto& th : pool) th.join();
}

inline unsigned worker_count(uint32_t requested)
{
    unsigned hw = std::thread::hardware_concurrency();
    if (hw == 0) hw = 1;
    if (requested == 0) return hw;
    return requested;
}

}  // namespace vdbc
