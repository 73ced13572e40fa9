// Scheduling core of the serving loop, free of HIP so that it also builds
// with a plain host compiler (the thread-sanitizer and address-sanitizer
// stress tests compile it with g++).
//
// Requests arrive as Jobs carrying a snapshot of their render parameters.
// One scheduler thread runs a loop:
//   1. completion: a busy slot whose last batch has finished releases its
//      jobs (done or failed), their output bytes and their volume references;
//   2. admission: every free slot takes queued jobs in arrival order while
//      their output bytes fit in the budget left for in-flight work, up to a
//      batch limit, and starts them as one batch through the Backend.
// Jobs that arrive while others run are admitted as soon as a slot and
// memory free up; batches on different slots run concurrently.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/vr.h"
#include "params.h"

namespace vr {

inline uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Job {
    uint64_t ticket = 0;
    ReqParams params{};
    std::atomic<int>* refs = nullptr;  // in-flight count of the job's volume
    uint64_t out_bytes = 0;
    vr_ticket_info info{};
};

class Backend {
  public:
    virtual ~Backend() = default;
    virtual int slots() const = 0;
    // Start one batch on `slot`.  Returns VR_OK or the failure of the launch.
    // Called without the scheduler's lock held.
    virtual vr_status launch(int slot, const std::vector<Job*>& jobs) = 0;
    // True once the slot's last batch has finished; *err is its status and
    // *device_ns the time it took on the device.
    virtual bool finished(int slot, vr_status* err, uint64_t* device_ns) = 0;
    // Samples composited for job q of the slot's finished batch.
    virtual uint64_t samples(int slot, int q) const = 0;
};

// CPU stand-in: a batch "runs" for rays x ns_per_ray nanoseconds and
// reports one sample per ray; a batch that holds a request of width
// fail_width fails; launch() itself takes launch_ns (a slow enqueue).
class FakeBackend : public Backend {
  public:
    FakeBackend(int n, double ns_per_ray, int fail_width, uint64_t launch_ns = 0)
        : ns_per_ray_(ns_per_ray), fail_width_(fail_width), launch_ns_(launch_ns),
          start_(n, 0), end_(n, 0), fail_(n, false), rays_(n) {}
    int slots() const override { return (int)end_.size(); }
    vr_status launch(int slot, const std::vector<Job*>& jobs) override {
        double rays = 0.0;
        bool f = false;
        rays_[slot].clear();
        for (Job* j : jobs) {
            rays += (double)j->info.rays;
            rays_[slot].push_back(j->info.rays);
            f = f || j->params.width == fail_width_;
        }
        if (launch_ns_) std::this_thread::sleep_for(std::chrono::nanoseconds(launch_ns_));
        start_[slot] = now_ns();
        end_[slot] = start_[slot] + (uint64_t)(rays * ns_per_ray_);
        fail_[slot] = f;
        return VR_OK;
    }
    bool finished(int slot, vr_status* err, uint64_t* device_ns) override {
        if (now_ns() < end_[slot]) return false;
        *err = fail_[slot] ? VR_ERR_DEVICE : VR_OK;
        *device_ns = end_[slot] - start_[slot];
        return true;
    }
    uint64_t samples(int slot, int q) const override { return rays_[slot][q]; }

  private:
    double ns_per_ray_;
    int fail_width_;
    uint64_t launch_ns_;
    std::vector<uint64_t> start_, end_;
    std::vector<bool> fail_;
    std::vector<std::vector<uint64_t>> rays_;
};

class Scheduler {
  public:
    static constexpr int kMaxPending = 4096;

    // budget(): bytes available to in-flight outputs right now.  on_start
    // runs on the scheduler thread before its loop (e.g. to select a device).
    Scheduler(Backend* backend, int max_batch, std::function<uint64_t()> budget,
              std::function<void()> on_start = nullptr)
        : backend_(backend), max_batch_(max_batch), budget_(std::move(budget)),
          busy_(backend->slots()), running_(backend->slots()) {
        thread_ = std::thread([this, on_start] {
            if (on_start) on_start();
            loop();
        });
    }
    ~Scheduler() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        thread_.join();
        delete backend_;
    }

    // Queue a job; VR_ERR_BUSY when kMaxPending jobs are queued already.
    vr_status submit(std::unique_ptr<Job> job, uint64_t* ticket) {
        std::lock_guard<std::mutex> lk(mu_);
        if ((int)pending_.size() >= kMaxPending) return VR_ERR_BUSY;
        job->ticket = next_ticket_++;
        job->info.state = 0;
        job->info.t_arrive_ns = now_ns();
        if (job->refs) job->refs->fetch_add(1);
        *ticket = job->ticket;
        pending_.push_back(job.get());
        jobs_[job->ticket] = std::move(job);
        cv_.notify_all();
        return VR_OK;
    }

    // VR_ERR_NOT_FOUND for an unknown ticket.
    vr_status poll(uint64_t ticket, vr_ticket_info* info) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = jobs_.find(ticket);
        if (it == jobs_.end()) return VR_ERR_NOT_FOUND;
        *info = it->second->info;
        return VR_OK;
    }

    // VR_ERR_NOT_FOUND unknown, VR_ERR_BUSY still pending or running.
    vr_status release(uint64_t ticket) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = jobs_.find(ticket);
        if (it == jobs_.end()) return VR_ERR_NOT_FOUND;
        if (it->second->info.state < 2) return VR_ERR_BUSY;
        jobs_.erase(it);
        return VR_OK;
    }

    bool idle() {
        std::lock_guard<std::mutex> lk(mu_);
        return pending_.empty() && inflight_jobs_ == 0;
    }

  private:
    void finish(Job* j, int state, vr_status err, uint64_t t) {
        j->info.state = state;
        j->info.err = err;
        j->info.t_done_ns = t;
        if (j->refs) j->refs->fetch_sub(1);
    }

    // One pass of completion and admission; true if anything changed.  `lk`
    // holds mu_ on entry and on return; it is released around each launch,
    // so that submit and poll never wait for the backend.  Only this thread
    // touches busy_ and running_, and jobs in running_ are past pending
    // (state 1), which release() does not erase.
    bool step(std::unique_lock<std::mutex>& lk) {
        bool changed = false;
        const uint64_t t = now_ns();
        for (int s = 0; s < (int)busy_.size(); ++s) {
            if (!busy_[s]) continue;
            vr_status err = VR_OK;
            uint64_t device_ns = 0;
            if (!backend_->finished(s, &err, &device_ns)) continue;
            for (size_t q = 0; q < running_[s].size(); ++q) {
                Job* j = running_[s][q];
                // device start on the host clock: the completion stamp minus
                // the batch's span on the device
                j->info.t_start_ns = t - std::min(device_ns, t - j->info.t_admit_ns);
                if (err == VR_OK) j->info.samples = backend_->samples(s, (int)q);
                finish(j, err == VR_OK ? 2 : 3, err, t);
                inflight_bytes_ -= j->out_bytes;
                --inflight_jobs_;
            }
            running_[s].clear();
            busy_[s] = false;
            changed = true;
        }
        for (int s = 0; s < (int)busy_.size() && !pending_.empty(); ++s) {
            if (busy_[s]) continue;
            const uint64_t budget = budget_();
            std::vector<Job*>& batch = running_[s];
            // A job that can never fit fails at once instead of blocking the queue.
            while (!pending_.empty() && pending_.front()->out_bytes > budget) {
                Job* j = pending_.front();
                pending_.pop_front();
                finish(j, 3, VR_ERR_OUT_OF_MEMORY, now_ns());
                changed = true;
            }
            while (!pending_.empty() && (int)batch.size() < max_batch_ &&
                   inflight_bytes_ + pending_.front()->out_bytes <= budget) {
                Job* j = pending_.front();
                pending_.pop_front();
                inflight_bytes_ += j->out_bytes;
                ++inflight_jobs_;
                batch.push_back(j);
            }
            if (batch.empty()) break;  // memory is the limit: wait for completions
            const uint64_t ts = now_ns();
            for (Job* j : batch) {
                j->info.state = 1;
                j->info.t_admit_ns = ts;
            }
            lk.unlock();
            const vr_status st = backend_->launch(s, batch);
            lk.lock();
            if (st != VR_OK) {
                for (Job* j : batch) {
                    finish(j, 3, st, now_ns());
                    inflight_bytes_ -= j->out_bytes;
                    --inflight_jobs_;
                }
                batch.clear();
            } else {
                busy_[s] = true;
            }
            changed = true;
        }
        return changed;
    }

    void loop() {
        std::unique_lock<std::mutex> lk(mu_);
        uint64_t last_activity = now_ns();
        while (!stop_) {
            const bool changed = step(lk);
            bool any_busy = false;
            for (bool b : busy_) any_busy = any_busy || b;
            if (changed || any_busy) last_activity = now_ns();
            if (changed) continue;
            if (any_busy || now_ns() - last_activity < kSpinNs) {
                // Poll completions and arrivals at a fine grain without
                // holding the lock (a timed sleep, or a wake-up through the
                // condition variable, costs tens of microseconds).
                lk.unlock();
                std::this_thread::yield();
                lk.lock();
            } else {
                cv_.wait_for(lk, std::chrono::milliseconds(5));
            }
        }
    }

    // The loop keeps polling this long after its last activity before it
    // sleeps on the condition variable.
    static constexpr uint64_t kSpinNs = 2000000;

    Backend* backend_;
    int max_batch_;
    std::function<uint64_t()> budget_;
    std::mutex mu_;
    std::condition_variable cv_;
    bool stop_ = false;
    std::deque<Job*> pending_;
    std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs_;
    std::vector<bool> busy_;
    std::vector<std::vector<Job*>> running_;
    uint64_t inflight_bytes_ = 0;
    int inflight_jobs_ = 0;
    uint64_t next_ticket_ = 1;
    std::thread thread_;
};

}  // namespace vr
