// Host-only checks of pdhg::JobQueue (built with g++ by tests/test_job_queue.py).
#include <atomic>
#include <chrono>
#include <cstdio>
#include <thread>

#include "job_queue.h"

using clk = std::chrono::steady_clock;

static double since(clk::time_point t0) {
    return std::chrono::duration<double>(clk::now() - t0).count();
}

int main() {
    // 1. a cap of one thread: push never blocks, jobs run one at a time, all run
    {
        std::atomic<int> active{0}, peak{0}, done{0};
        std::atomic<int> cancel{0};
        pdhg::JobQueue q(1, [&] { return cancel.load() != 0; });
        const auto t0 = clk::now();
        for (int i = 0; i < 5; ++i)
            q.push([&] {
                const int a = ++active;
                int p = peak.load();
                while (a > p && !peak.compare_exchange_weak(p, a)) {}
                std::this_thread::sleep_for(std::chrono::milliseconds(40));
                --active;
                ++done;
            });
        const double t_push = since(t0);
        q.close_and_join();
        std::printf("cap1 push_s %.4f total_s %.3f peak %d done %d started %d\n",
                    t_push, since(t0), peak.load(), done.load(), q.started());
    }
    // 2. a winner cancels: queued jobs are dropped, running ones see the flag
    {
        std::atomic<int> cancel{0}, ran{0};
        pdhg::JobQueue q(2, [&] { return cancel.load() != 0; });
        const auto t0 = clk::now();
        for (int i = 0; i < 6; ++i)
            q.push([&, i] {
                ++ran;
                if (i == 1) {
                    std::this_thread::sleep_for(std::chrono::milliseconds(30));
                    cancel.store(1);
                    q.notify();
                    return;
                }
                while (!cancel.load()) std::this_thread::sleep_for(std::chrono::milliseconds(2));
            });
        q.close_and_join();
        std::printf("cancel total_s %.3f ran %d started %d\n", since(t0), ran.load(),
                    q.started());
    }
    // 3. no cap: jobs overlap
    {
        std::atomic<int> active{0}, peak{0};
        std::atomic<int> cancel{0};
        pdhg::JobQueue q(0, [&] { return cancel.load() != 0; });
        for (int i = 0; i < 8; ++i)
            q.push([&] {
                const int a = ++active;
                int p = peak.load();
                while (a > p && !peak.compare_exchange_weak(p, a)) {}
                std::this_thread::sleep_for(std::chrono::milliseconds(60));
                --active;
            });
        q.close_and_join();
        std::printf("nocap peak %d started %d\n", peak.load(), q.started());
    }
    // 4. an external job holds the only slot: queued jobs start after it ends
    {
        std::atomic<int> cancel{0}, done{0};
        pdhg::JobQueue q(1, [&] { return cancel.load() != 0; });
        q.add_external();
        for (int i = 0; i < 3; ++i) q.push([&] { ++done; });
        std::this_thread::sleep_for(std::chrono::milliseconds(50));
        const int before = done.load();
        q.end_external();
        q.close_and_join();
        std::printf("external before %d done %d\n", before, done.load());
    }
    return 0;
}
