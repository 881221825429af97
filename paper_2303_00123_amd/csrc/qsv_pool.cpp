// Host worker pool of a context.  The batch planner lowers, fuses, plans and
// writes the records of every circuit of a batch in parallel on each call;
// starting and joining a thread per worker on every call cost more host time
// than the work of a small batch, so the threads are started once, on first
// use, and wait on a condition variable between calls.
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <mutex>
#include <thread>
#include <vector>

#include "qsv_internal.h"

namespace qsv {

class WorkerPool {
public:
    explicit WorkerPool(int workers) {
        th_.reserve(size_t(workers > 0 ? workers : 0));
        for (int t = 0; t < workers; ++t) {
            try {
                th_.emplace_back([this] { loop(); });
            } catch (...) {
                break;   // fewer workers than asked for
            }
        }
    }

    ~WorkerPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        wake_.notify_all();
        for (std::thread& t : th_) t.join();
    }

    size_t size() const { return th_.size(); }

    bool run(int n, void (*f)(void*, int), void* arg) {
        std::unique_lock<std::mutex> lk(mu_);
        f_ = f;
        arg_ = arg;
        n_ = n;
        next_.store(0);
        ok_.store(true);
        busy_ = int(th_.size());
        ++gen_;
        lk.unlock();
        wake_.notify_all();
        work();
        lk.lock();
        done_.wait(lk, [this] { return busy_ == 0; });
        return ok_.load();
    }

private:
    void work() {
        for (int i = next_.fetch_add(1); i < n_; i = next_.fetch_add(1)) {
            try {
                f_(arg_, i);
            } catch (...) {
                ok_.store(false);
            }
        }
    }

    void loop() {
        uint64_t seen = 0;
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            wake_.wait(lk, [&] { return stop_ || gen_ != seen; });
            if (stop_) return;
            seen = gen_;
            lk.unlock();
            work();
            lk.lock();
            if (--busy_ == 0) done_.notify_one();
        }
    }

    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable wake_, done_;
    bool stop_ = false;
    uint64_t gen_ = 0;   // one increment per run; a worker runs each generation once
    int busy_ = 0;       // workers still in the current generation
    // the current job (set under mu_ before gen_ changes)
    void (*f_)(void*, int) = nullptr;
    void* arg_ = nullptr;
    int n_ = 0;
    std::atomic<int> next_{0};
    std::atomic<bool> ok_{true};
};

WorkerPool* pool_create(int workers) {
    try {
        WorkerPool* p = new WorkerPool(workers);
        if (p->size() == 0) {
            delete p;
            return nullptr;
        }
        return p;
    } catch (...) {
        return nullptr;
    }
}

void pool_destroy(WorkerPool* p) { delete p; }

bool pool_run(WorkerPool* p, int n, void (*f)(void*, int), void* arg) { return p->run(n, f, arg); }

}  // namespace qsv
