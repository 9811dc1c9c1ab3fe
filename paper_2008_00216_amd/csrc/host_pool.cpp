// Host worker pool for per-state loops of the planner (the matrices of many
// parameter sets, their plan pools).  Workers are started once and reused;
// one loop runs on the pool at a time, and a caller that finds it busy runs
// its loop inline.
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include <unistd.h>

#include "host.h"

namespace svmi {

namespace {

class WorkerPool {
public:
    WorkerPool() : pid_(getpid()) {
        const unsigned hw = std::thread::hardware_concurrency();
        const unsigned k = std::min(7u, hw > 1 ? hw - 1 : 0u);
        for (unsigned i = 0; i < k; ++i) th_->emplace_back([this] { work(); });
    }
    ~WorkerPool() {
        if (getpid() != pid_) return;   // forked child: the threads are not here (the list leaks)
        {
            std::lock_guard<std::mutex> l(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (std::thread& t : *th_) t.join();
        delete th_;
    }
    // fn(i) for every i in [0, n); returns when every call has returned and
    // every worker has left this loop
    void run(int n, const std::function<void(int)>& fn) {
        // a forked child has the pool's state but not its threads
        std::unique_lock<std::mutex> busy(run_mu_, std::try_to_lock);
        if (!busy.owns_lock() || th_->empty() || n < 2 || getpid() != pid_) {
            for (int i = 0; i < n; ++i) fn(i);
            return;
        }
        {
            std::lock_guard<std::mutex> l(mu_);
            fn_ = &fn;
            n_ = n;
            next_ = 0;
            finished_ = 0;
            ++gen_;
        }
        cv_.notify_all();
        for (int i = next_++; i < n; i = next_++) fn(i);
        std::unique_lock<std::mutex> l(mu_);
        done_.wait(l, [&] { return finished_ == (int)th_->size(); });
        fn_ = nullptr;
    }

private:
    void work() {
        uint64_t seen = 0;
        for (;;) {
            std::unique_lock<std::mutex> l(mu_);
            cv_.wait(l, [&] { return stop_ || gen_ != seen; });
            if (stop_) return;
            seen = gen_;
            const std::function<void(int)>* f = fn_;
            const int n = n_;
            l.unlock();
            for (int i = next_++; i < n; i = next_++) (*f)(i);
            l.lock();
            if (++finished_ == (int)th_->size()) done_.notify_all();
        }
    }
    const pid_t pid_;
    std::vector<std::thread>* th_ = new std::vector<std::thread>;
    std::mutex run_mu_, mu_;
    std::condition_variable cv_, done_;
    const std::function<void(int)>* fn_ = nullptr;
    int n_ = 0;
    std::atomic<int> next_{0};
    int finished_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};

WorkerPool& pool() {
    static WorkerPool p;
    return p;
}

}  // namespace

void host_parallel_for(int n, const std::function<void(int)>& fn) { pool().run(n, fn); }

}  // namespace svmi
