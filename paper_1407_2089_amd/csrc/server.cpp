// Serving loop behind vr_submit / vr_poll / vr_release: the scheduling core
// (sched.h) driven by a GPU backend whose slots each own a stream, a
// batched-launch workspace and a completion event.  Requests are queued with
// a snapshot of their parameters, transfer functions included.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/vr_test.h"
#include "lib.h"
#include "sched.h"

namespace vr {

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
        hipError_t e;
        if (jobs.size() == 1) {
            // A lone request takes the plain launch: its parameters travel as
            // kernel arguments, with no table upload and no graph.
            e = launch_render(jobs[0]->params, ctx_->plain_tile, ctx_->clear_skip,
                              streams_[slot]);
            if (e != hipSuccess) return hip_fail(e, "render launch");
        } else {
            params_.resize(jobs.size());
            for (size_t q = 0; q < jobs.size(); ++q) params_[q] = jobs[q]->params;
            // The loop never stops to tune: a shape class tuned by
            // vr_render_batch (or loaded from the cache file) is used, else the
            // default tile.
            vr_status st = batch_enqueue(ctx_, slots_[slot], params_.data(), (int)jobs.size(),
                                         /*allow_tuning=*/false);
            if (st != VR_OK) return st;
        }
        e = hipEventRecord(events_[slot], streams_[slot]);
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

constexpr int kDefaultSlots = 3;
constexpr int kMaxBatch = 32;

// Bytes left for in-flight outputs: the budget minus the resident volumes.
static std::function<uint64_t()> serve_budget(vr_ctx* ctx) {
    return [ctx] {
        const uint64_t used = ctx->used.load();
        return ctx->budget > used ? ctx->budget - used : 0;
    };
}

// Snapshot of a request for the scheduler (caller validated it).
static std::unique_ptr<Job> make_job(const vr_render_req& r) {
    auto job = std::make_unique<Job>();
    {
        std::lock_guard<std::mutex> lk(r.vol->tf_mu);
        make_params(r, r.vol->tf, &job->params);
    }
    job->refs = &r.vol->in_flight;
    const uint64_t eyes = r.stereo ? 2 : 1;
    const uint64_t px = (uint64_t)r.width * (uint64_t)r.height * eyes;
    job->out_bytes = px * (16u + (r.out_samples ? 4u : 0u));
    job->info.rays = px;
    return job;
}

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
    const int device = ctx->device;
    ctx->server = new Scheduler(b, kMaxBatch, serve_budget(ctx),
                                [device] { (void)hipSetDevice(device); });
    return VR_OK;
}

vr_status server_submit(vr_ctx* ctx, const vr_render_req* req, uint64_t* ticket) {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    vr_status st = ensure_server(ctx);
    if (st != VR_OK) return st;
    st = ctx->server->submit(make_job(*req), ticket);
    if (st == VR_ERR_BUSY)
        return fail(st, "%d requests are already queued", Scheduler::kMaxPending);
    return st;
}

vr_status server_poll(vr_ctx* ctx, uint64_t ticket, vr_ticket_info* info) {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    if (!ctx->server) return fail(VR_ERR_NOT_FOUND, "unknown ticket");
    vr_status st = ctx->server->poll(ticket, info);
    if (st != VR_OK) return fail(st, "unknown ticket %llu", (unsigned long long)ticket);
    return st;
}

vr_status server_release(vr_ctx* ctx, uint64_t ticket) {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    if (!ctx->server) return fail(VR_ERR_NOT_FOUND, "unknown ticket");
    vr_status st = ctx->server->release(ticket);
    if (st == VR_ERR_NOT_FOUND)
        return fail(st, "unknown ticket %llu", (unsigned long long)ticket);
    if (st == VR_ERR_BUSY)
        return fail(st, "ticket %llu is still pending or running", (unsigned long long)ticket);
    return st;
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
    ctx->server = new Scheduler(new FakeBackend(slots, ns_per_ray, fail_width), max_batch,
                                serve_budget(ctx));
    return ok();
}

}  // extern "C"
