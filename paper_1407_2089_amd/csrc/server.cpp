// Serving loop behind vr_submit / vr_poll / vr_release.
//
// Requests are queued with a snapshot of their parameters (transfer
// functions included).  One scheduler thread runs a loop:
//   1. completion: a busy slot whose last launch has finished releases its
//      tickets (done or failed), their output bytes and their volumes;
//   2. admission: every free slot takes queued requests in arrival order
//      while their output bytes fit in the memory budget left over by the
//      resident volumes and the requests already in flight, up to a batch
//      limit, and launches them as one batched launch on its own stream.
// Requests that arrive while others run are admitted as soon as a slot and
// memory free up; batches on different slots overlap on the device.  The
// loop only talks to the GPU through a Backend, so the scheduling logic is
// exercised on the CPU with a timed fake backend.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/vr_test.h"
#include "lib.h"

namespace vr {

static uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Job {
    uint64_t ticket = 0;
    ReqParams params{};
    vr_volume* vol = nullptr;
    uint64_t out_bytes = 0;
    vr_ticket_info info{};
};

class Backend {
  public:
    virtual ~Backend() = default;
    virtual int slots() const = 0;
    // Start one batch on `slot`.  Returns VR_OK or the failure of the launch.
    virtual vr_status launch(int slot, const std::vector<Job*>& jobs) = 0;
    // True once the slot's last batch has finished; *err is its status.
    virtual bool finished(int slot, vr_status* err) = 0;
};

// GPU backend: one stream, one batched-launch workspace and one completion
// event per slot.
class HipBackend : public Backend {
  public:
    HipBackend(vr_ctx* ctx, int n, vr_status* st) : ctx_(ctx) {
        *st = VR_OK;
        for (int s = 0; s < n; ++s) {
            hipStream_t stream = nullptr;
            hipEvent_t ev = nullptr;
            hipError_t e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) {
                *st = hip_fail(e, "serving stream");
                if (stream) (void)hipStreamDestroy(stream);
                return;
            }
            BatchSlot* b = batch_slot_create(ctx, stream, st);
            if (!b) {
                (void)hipEventDestroy(ev);
                (void)hipStreamDestroy(stream);
                return;
            }
            streams_.push_back(stream);
            events_.push_back(ev);
            slots_.push_back(b);
        }
    }
    ~HipBackend() override {
        for (size_t s = 0; s < slots_.size(); ++s) {
            batch_slot_destroy(slots_[s]);
            (void)hipEventDestroy(events_[s]);
            (void)hipStreamDestroy(streams_[s]);
        }
    }
    int slots() const override { return (int)slots_.size(); }
    vr_status launch(int slot, const std::vector<Job*>& jobs) override {
        params_.resize(jobs.size());
        for (size_t q = 0; q < jobs.size(); ++q) params_[q] = jobs[q]->params;
        // The loop never stops to tune: a shape class tuned by vr_render_batch
        // (or loaded from the cache file) is used, else the default tile.
        vr_status st = batch_enqueue(ctx_, slots_[slot], params_.data(), (int)jobs.size(),
                                     /*allow_tuning=*/false);
        if (st != VR_OK) return st;
        hipError_t e = hipEventRecord(events_[slot], streams_[slot]);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        return VR_OK;
    }
    bool finished(int slot, vr_status* err) override {
        hipError_t e = hipEventQuery(events_[slot]);
        if (e == hipErrorNotReady) return false;
        *err = e == hipSuccess ? VR_OK : VR_ERR_DEVICE;
        return true;
    }

  private:
    vr_ctx* ctx_;
    std::vector<hipStream_t> streams_;
    std::vector<hipEvent_t> events_;
    std::vector<BatchSlot*> slots_;
    std::vector<ReqParams> params_;
};

// CPU stand-in: a batch "runs" for rays x ns_per_ray nanoseconds; a batch
// that holds a request of width fail_width fails.
class FakeBackend : public Backend {
  public:
    FakeBackend(int n, double ns_per_ray, int fail_width)
        : ns_per_ray_(ns_per_ray), fail_width_(fail_width), end_(n, 0), fail_(n, false) {}
    int slots() const override { return (int)end_.size(); }
    vr_status launch(int slot, const std::vector<Job*>& jobs) override {
        double rays = 0.0;
        bool f = false;
        for (Job* j : jobs) {
            rays += (double)j->info.rays;
            f = f || j->params.width == fail_width_;
        }
        end_[slot] = now_ns() + (uint64_t)(rays * ns_per_ray_);
        fail_[slot] = f;
        return VR_OK;
    }
    bool finished(int slot, vr_status* err) override {
        if (now_ns() < end_[slot]) return false;
        *err = fail_[slot] ? VR_ERR_DEVICE : VR_OK;
        return true;
    }

  private:
    double ns_per_ray_;
    int fail_width_;
    std::vector<uint64_t> end_;
    std::vector<bool> fail_;
};

constexpr int kMaxPending = 4096;
constexpr int kDefaultSlots = 3;
constexpr int kMaxBatch = 32;

class Server {
  public:
    Server(vr_ctx* ctx, Backend* backend, int max_batch)
        : ctx_(ctx), backend_(backend), max_batch_(max_batch),
          busy_(backend->slots()), running_(backend->slots()) {
        thread_ = std::thread([this] { loop(); });
    }
    ~Server() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        thread_.join();
        delete backend_;
    }

    vr_status submit(const vr_render_req& r, uint64_t* ticket) {
        auto job = std::make_unique<Job>();
        {
            std::lock_guard<std::mutex> lk(r.vol->tf_mu);
            make_params(r, r.vol->tf, &job->params);
        }
        job->vol = r.vol;
        const uint64_t eyes = r.stereo ? 2 : 1;
        const uint64_t px = (uint64_t)r.width * (uint64_t)r.height * eyes;
        job->out_bytes = px * (16u + (r.out_samples ? 4u : 0u));
        job->info.rays = px;
        std::lock_guard<std::mutex> lk(mu_);
        if ((int)pending_.size() >= kMaxPending)
            return fail(VR_ERR_BUSY, "%d requests are already queued", kMaxPending);
        job->ticket = next_ticket_++;
        job->info.state = 0;
        job->info.t_arrive_ns = now_ns();
        r.vol->in_flight.fetch_add(1);
        *ticket = job->ticket;
        pending_.push_back(job.get());
        jobs_[job->ticket] = std::move(job);
        cv_.notify_all();
        return VR_OK;
    }

    vr_status poll(uint64_t ticket, vr_ticket_info* info) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = jobs_.find(ticket);
        if (it == jobs_.end()) return fail(VR_ERR_NOT_FOUND, "unknown ticket %llu",
                                           (unsigned long long)ticket);
        *info = it->second->info;
        return VR_OK;
    }

    vr_status release(uint64_t ticket) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = jobs_.find(ticket);
        if (it == jobs_.end()) return fail(VR_ERR_NOT_FOUND, "unknown ticket %llu",
                                           (unsigned long long)ticket);
        if (it->second->info.state < 2)
            return fail(VR_ERR_BUSY, "ticket %llu is still %s", (unsigned long long)ticket,
                        it->second->info.state == 0 ? "pending" : "running");
        jobs_.erase(it);
        return VR_OK;
    }

    bool idle() {
        std::lock_guard<std::mutex> lk(mu_);
        return pending_.empty() && inflight_jobs_ == 0;
    }

  private:
    // Budget for in-flight outputs: whatever the resident volumes leave.
    uint64_t serve_budget() const {
        const uint64_t used = ctx_->used.load();
        return ctx_->budget > used ? ctx_->budget - used : 0;
    }

    void finish(Job* j, int state, vr_status err, uint64_t t) {
        j->info.state = state;
        j->info.err = err;
        j->info.t_done_ns = t;
        j->vol->in_flight.fetch_sub(1);
    }

    // Returns true if anything changed.
    bool step() {
        bool changed = false;
        const uint64_t t = now_ns();
        for (int s = 0; s < (int)busy_.size(); ++s) {
            if (!busy_[s]) continue;
            vr_status err = VR_OK;
            if (!backend_->finished(s, &err)) continue;
            for (Job* j : running_[s]) {
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
            const uint64_t budget = serve_budget();
            std::vector<Job*>& batch = running_[s];
            // Requests that can never fit fail at once instead of blocking the queue.
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
                j->info.t_start_ns = ts;
            }
            vr_status st = backend_->launch(s, batch);
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
        if (ctx_->device >= 0) (void)hipSetDevice(ctx_->device);
        std::unique_lock<std::mutex> lk(mu_);
        while (!stop_) {
            const bool changed = step();
            bool any_busy = false;
            for (bool b : busy_) any_busy = any_busy || b;
            if (changed) continue;
            if (any_busy) {
                // Poll device completions at a fine grain without holding the
                // lock (a timed sleep would round up to tens of microseconds).
                lk.unlock();
                std::this_thread::yield();
                lk.lock();
            } else {
                cv_.wait_for(lk, std::chrono::milliseconds(5));
            }
        }
    }

    vr_ctx* ctx_;
    Backend* backend_;
    int max_batch_;
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

// Caller holds ctx->server_mu.
static vr_status ensure_server(vr_ctx* ctx) {
    if (ctx->server) return VR_OK;
    if (ctx->device < 0)
        return fail(VR_ERR_UNSUPPORTED, "validation-only context has no serving backend");
    vr_status st;
    (void)hipSetDevice(ctx->device);
    HipBackend* b = new HipBackend(ctx, kDefaultSlots, &st);
    if (st != VR_OK) {
        delete b;
        return st;
    }
    ctx->server = new Server(ctx, b, kMaxBatch);
    return VR_OK;
}

vr_status server_submit(vr_ctx* ctx, const vr_render_req* req, uint64_t* ticket) {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    vr_status st = ensure_server(ctx);
    if (st != VR_OK) return st;
    return ctx->server->submit(*req, ticket);
}

vr_status server_poll(vr_ctx* ctx, uint64_t ticket, vr_ticket_info* info) {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    if (!ctx->server) return fail(VR_ERR_NOT_FOUND, "unknown ticket");
    return ctx->server->poll(ticket, info);
}

vr_status server_release(vr_ctx* ctx, uint64_t ticket) {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    if (!ctx->server) return fail(VR_ERR_NOT_FOUND, "unknown ticket");
    return ctx->server->release(ticket);
}

vr_status server_stop(vr_ctx* ctx) {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    if (!ctx->server) return VR_OK;
    if (!ctx->server->idle()) return fail(VR_ERR_BUSY, "served tickets are pending or running");
    delete ctx->server;
    ctx->server = nullptr;
    return VR_OK;
}

}  // namespace vr

using namespace vr;

extern "C" {

vr_status vr_submit(vr_ctx* ctx, const vr_render_req* req, uint64_t* ticket) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    if (!ticket) return fail(VR_ERR_INVALID_ARG, "ticket is NULL");
    vr_status st = check_request(ctx, req);
    if (st != VR_OK) return st;
    st = server_submit(ctx, req, ticket);
    if (st != VR_OK) return st;
    return ok();
}

vr_status vr_poll(vr_ctx* ctx, uint64_t ticket, vr_ticket_info* info) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    if (!info) return fail(VR_ERR_INVALID_ARG, "info is NULL");
    vr_status st = server_poll(ctx, ticket, info);
    if (st != VR_OK) return st;
    return ok();
}

vr_status vr_release(vr_ctx* ctx, uint64_t ticket) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    vr_status st = server_release(ctx, ticket);
    if (st != VR_OK) return st;
    return ok();
}

vr_status vr_test_fake_backend(vr_ctx* ctx, int32_t slots, double ns_per_ray,
                               int32_t fail_width, int32_t max_batch) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    if (slots < 1 || slots > 64 || !(ns_per_ray >= 0.0) || max_batch < 1)
        return fail(VR_ERR_INVALID_ARG, "bad fake backend parameters");
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    if (ctx->server) {
        if (!ctx->server->idle()) return fail(VR_ERR_BUSY, "serving loop is busy");
        delete ctx->server;
    }
    ctx->server = new Server(ctx, new FakeBackend(slots, ns_per_ray, fail_width), max_batch);
    return ok();
}

}  // extern "C"
