// cpu_steps.cpp -- the PDHG step pair on the host's cores.
//
// The solver in the paper has a multi-threaded CPU PDHG next to the GPU one
// (Section 4.1), and its discussion (Section 5) notes that the CPU iteration
// is bound by memory bandwidth, which a small fraction of the cores already
// saturates.  This file is that platform's hot path, for measuring
// iterations per second against the thread count:
// plain steps
//   x <- max(0, x - tau (c - A^T y)),  y <- y + sigma (b - A (2 x_new - x))
// over the explicit CSR of A^T (primal half) and of A (dual half), each half
// split into contiguous row ranges of equal nonzero counts, one per thread,
// with a barrier between halves.  Restarts and evaluations are not part of
// it; the GPU path is the solver.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"

namespace {

// Reusable barrier for a fixed number of threads.
class Barrier {
  public:
    explicit Barrier(int n) : n_(n) {}
    void wait() {
        std::unique_lock<std::mutex> lk(mu_);
        const long gen = gen_;
        if (++count_ == n_) {
            count_ = 0;
            ++gen_;
            cv_.notify_all();
        } else {
            cv_.wait(lk, [&] { return gen_ != gen; });
        }
    }

  private:
    std::mutex mu_;
    std::condition_variable cv_;
    int n_, count_ = 0;
    long gen_ = 0;
};

// Row ranges of equal nonzero count (plus one per row, so empty rows count).
std::vector<int64_t> split_rows(int64_t rows, const int64_t *rp, int parts) {
    std::vector<int64_t> cut((size_t)parts + 1, rows);
    cut[0] = 0;
    const double total = (double)rp[rows] + (double)rows;
    int64_t r = 0;
    for (int p = 1; p < parts; ++p) {
        const double goal = total * p / parts;
        while (r < rows && (double)rp[r] + (double)r < goal) ++r;
        cut[p] = r;
    }
    return cut;
}

}  // namespace

extern "C" int pdhg_cpu_steps(int64_t m, int64_t n, const int64_t *a_rp,
                              const int32_t *a_ci, const double *a_v,
                              const int64_t *at_rp, const int32_t *at_ci,
                              const double *at_v, const double *b,
                              const double *c, double tau, double sigma,
                              int K, int threads, double *x, double *y,
                              double *seconds) {
    if (m < 1 || n < 1 || K < 0 || threads < 1 || threads > 1024 || !a_rp ||
        !at_rp || !b || !c || !x || !y)
        return PDHG_E_ARG;
    if ((a_rp[m] > 0 && (!a_ci || !a_v)) || (at_rp[n] > 0 && (!at_ci || !at_v)) ||
        a_rp[m] != at_rp[n])
        return PDHG_E_ARG;
    try {
        std::vector<double> xe((size_t)n);
        const std::vector<int64_t> pc = split_rows(n, at_rp, threads);
        const std::vector<int64_t> dc = split_rows(m, a_rp, threads);
        Barrier bar(threads);
        auto work = [&](int t) {
            for (int k = 0; k < K; ++k) {
                // primal half over rows j of A^T: gathers y
                for (int64_t j = pc[t]; j < pc[t + 1]; ++j) {
                    double g = 0.0;
                    for (int64_t p = at_rp[j]; p < at_rp[j + 1]; ++p)
                        g += at_v[p] * y[at_ci[p]];
                    const double v = x[j] - tau * (c[j] - g);
                    const double xn = v < 0.0 ? 0.0 : v;
                    xe[j] = 2.0 * xn - x[j];
                    x[j] = xn;
                }
                bar.wait();
                // dual half over rows i of A: gathers 2 x_new - x_old
                for (int64_t i = dc[t]; i < dc[t + 1]; ++i) {
                    double q = 0.0;
                    for (int64_t p = a_rp[i]; p < a_rp[i + 1]; ++p)
                        q += a_v[p] * xe[a_ci[p]];
                    y[i] = y[i] + sigma * (b[i] - q);
                }
                bar.wait();
            }
        };
        const auto t0 = std::chrono::steady_clock::now();
        std::vector<std::thread> pool;
        for (int t = 1; t < threads; ++t) pool.emplace_back(work, t);
        work(0);
        for (auto &th : pool) th.join();
        if (seconds)
            *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    } catch (...) {
        return PDHG_E_OOM;
    }
    return PDHG_OK;
}
