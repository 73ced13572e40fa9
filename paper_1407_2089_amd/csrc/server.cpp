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

// GPU backend: per slot one stream, one batched-launch workspace, a pair of
// timing events around the batch's kernels, a completion event after the
// read-back of its sample counters, and the counters themselves (one per
// request of the batch, device and pinned host copies).
class HipBackend : public Backend {
  public:
    HipBackend(vr_ctx* ctx, int n, int max_batch, vr_status* st)
        : ctx_(ctx), max_batch_(max_batch) {
        *st = VR_OK;
        for (int s = 0; s < n; ++s) {
            Slot sl;
            hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreate(&sl.t0);
            if (e == hipSuccess) e = hipEventCreate(&sl.t1);
            if (e == hipSuccess) e = hipMalloc(&sl.d_count, count_bytes(max_batch));
            if (e == hipSuccess)
                e = hipHostMalloc(&sl.h_count, count_bytes(max_batch), hipHostMallocDefault);
            if (e != hipSuccess) {
                *st = hip_fail(e, "serving slot");
                destroy(sl);
                return;
            }
            sl.batch = batch_slot_create(ctx, sl.stream, st);
            if (!sl.batch) {
                destroy(sl);
                return;
            }
            slots_.push_back(sl);
        }
    }
    ~HipBackend() override {
        for (Slot& sl : slots_) destroy(sl);
    }
    int slots() const override { return (int)slots_.size(); }
    vr_status launch(int slot, const std::vector<Job*>& jobs) override {
        Slot& sl = slots_[slot];
        const int n = (int)jobs.size();
        if (n > max_batch_) return fail(VR_ERR_INVALID_ARG, "batch of %d requests", n);
        sl.n = n;
        // counters cleared by a kernel-free memset on the stream: the batch's
        // graph is launched after it and does not contain it
        hipError_t e = hipMemsetAsync(sl.d_count, 0, count_bytes(n), sl.stream);
        if (e == hipSuccess) e = hipEventRecord(sl.t0, sl.stream);
        if (e != hipSuccess) return hip_fail(e, "serving launch");
        params_.resize(jobs.size());
        for (int q = 0; q < n; ++q) {
            params_[q] = jobs[q]->params;
            params_[q].nsamples = sl.d_count + (size_t)q * kCountSlots * kCountStride;
        }
        if (n == 1) {
            // A lone request takes the plain launch: its parameters travel as
            // kernel arguments, with no table upload and no graph.
            e = launch_render(params_[0], ctx_->plain_tile, ctx_->clear_skip, sl.stream);
            if (e != hipSuccess) return hip_fail(e, "render launch");
        } else {
            // The loop never stops to tune: a shape class tuned by
            // vr_tune_batch (or loaded from the cache file) is used, else the
            // default tile.
            vr_status st = batch_enqueue(ctx_, sl.batch, params_.data(), n);
            if (st != VR_OK) return st;
        }
        if ((e = hipEventRecord(sl.t1, sl.stream)) != hipSuccess ||
            (e = hipMemcpyAsync(sl.h_count, sl.d_count, count_bytes(n), hipMemcpyDeviceToHost,
                                sl.stream)) != hipSuccess ||
            (e = hipEventRecord(sl.done, sl.stream)) != hipSuccess)
            return hip_fail(e, "serving launch");
        return VR_OK;
    }
    bool finished(int slot, vr_status* err, uint64_t* device_ns) override {
        Slot& sl = slots_[slot];
        hipError_t e = hipEventQuery(sl.done);
        if (e == hipErrorNotReady) return false;
        *err = e == hipSuccess ? VR_OK : VR_ERR_DEVICE;
        float ms = 0.0f;
        *device_ns = 0;
        if (e == hipSuccess && hipEventElapsedTime(&ms, sl.t0, sl.t1) == hipSuccess && ms > 0.0f)
            *device_ns = (uint64_t)((double)ms * 1e6);
        return true;
    }
    uint64_t samples(int slot, int q) const override {
        const Slot& sl = slots_[slot];
        if (q >= sl.n) return 0;
        uint64_t s = 0;
        const unsigned long long* c = sl.h_count + (size_t)q * kCountSlots * kCountStride;
        for (int i = 0; i < kCountSlots; ++i) s += c[(size_t)i * kCountStride];
        return s;
    }

  private:
    // Counter slots of n requests (kCountSlots per request, one per line).
    static size_t count_bytes(int n) {
        return sizeof(unsigned long long) * (size_t)n * kCountSlots * kCountStride;
    }
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr, t0 = nullptr, t1 = nullptr;
        unsigned long long* d_count = nullptr;
        unsigned long long* h_count = nullptr;  // pinned
        BatchSlot* batch = nullptr;
        int n = 0;
    };
    static void destroy(Slot& sl) {
        if (sl.batch) batch_slot_destroy(sl.batch);  // synchronises the stream
        if (sl.d_count) (void)hipFree(sl.d_count);
        if (sl.h_count) (void)hipHostFree(sl.h_count);
        for (hipEvent_t ev : {sl.done, sl.t0, sl.t1})
            if (ev) (void)hipEventDestroy(ev);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        sl = Slot{};
    }

    vr_ctx* ctx_;
    int max_batch_;
    std::vector<Slot> slots_;
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
    HipBackend* b = new HipBackend(ctx, kDefaultSlots, kMaxBatch, &st);
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
                               int32_t fail_width, int32_t max_batch, double launch_ms) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    if (slots < 1 || slots > 64 || !(ns_per_ray >= 0.0) || max_batch < 1 ||
        !(launch_ms >= 0.0) || !(launch_ms <= 10000.0))
        return fail(VR_ERR_INVALID_ARG, "bad fake backend parameters");
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    if (ctx->server) {
        if (!ctx->server->idle()) return fail(VR_ERR_BUSY, "serving loop is busy");
        delete ctx->server;
    }
    ctx->server = new Scheduler(
        new FakeBackend(slots, ns_per_ray, fail_width, (uint64_t)(launch_ms * 1e6)), max_batch,
        serve_budget(ctx));
    return ok();
}

}  // extern "C"
