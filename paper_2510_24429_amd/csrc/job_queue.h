// job_queue.h -- starts queued host jobs on threads, at most max_threads at
// a time, without ever blocking the thread that queues them.
//
// Algorithm 1 (Section 3.1) hands each snapshot to a CPU crossover thread
// while PDHG keeps iterating.  With a cap on the number of crossover threads,
// a snapshot that finds every thread busy must wait for one without holding
// up the PDHG loop: push() only queues the job, and a dispatcher thread
// starts it once a thread has returned.  When the caller's cancel predicate
// turns true, jobs not yet started are dropped.  Host code only.
#pragma once

#include <condition_variable>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace pdhg {

class JobQueue {
  public:
    // max_threads = 0: no limit.  cancelled() is polled under the queue's
    // lock; call notify() after making it true.
    JobQueue(int max_threads, std::function<bool()> cancelled)
        : max_(max_threads), cancelled_(std::move(cancelled)),
          dispatcher_([this] { dispatch(); }) {}
    ~JobQueue() { close_and_join(); }
    JobQueue(const JobQueue &) = delete;
    JobQueue &operator=(const JobQueue &) = delete;

    // Queue a job; returns at once.
    void push(std::function<void()> job) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            pending_.push_back(std::move(job));
        }
        cv_.notify_all();
    }

    // Wake the dispatcher (after the cancel predicate changed).
    void notify() { cv_.notify_all(); }

    // Jobs running now or started and not yet returned, beyond the caller.
    void add_external() {
        std::lock_guard<std::mutex> lk(mu_);
        ++running_;
    }
    void end_external() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            --running_;
        }
        cv_.notify_all();
    }

    // No more jobs: start the queued ones as threads free up (or drop them
    // once cancelled), then join every job thread.  Idempotent.
    void close_and_join() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            closing_ = true;
        }
        cv_.notify_all();
        if (dispatcher_.joinable()) dispatcher_.join();
    }

    int started() const { return started_; }

  private:
    bool slot_free() const { return max_ == 0 || running_ < max_; }

    void dispatch() {
        std::vector<std::thread> threads;
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            // wake for: a queued job with a free thread, a queued job to drop
            // after a cancel, or the end with nothing left queued
            cv_.wait(lk, [this] {
                return (closing_ && pending_.empty()) ||
                       (!pending_.empty() && (cancelled_() || slot_free()));
            });
            if (cancelled_()) pending_.clear();
            if (pending_.empty()) {
                if (closing_) break;
                continue;
            }
            std::function<void()> job = std::move(pending_.front());
            pending_.pop_front();
            ++running_;
            ++started_;
            threads.emplace_back([this, job] {
                job();
                {
                    std::lock_guard<std::mutex> g(mu_);
                    --running_;
                }
                cv_.notify_all();
            });
        }
        lk.unlock();
        for (auto &t : threads) t.join();
    }

    int max_;
    std::function<bool()> cancelled_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<std::function<void()>> pending_;
    int running_ = 0;
    int started_ = 0;
    bool closing_ = false;
    std::thread dispatcher_;   // last member: starts after the others exist
};

}  // namespace pdhg
