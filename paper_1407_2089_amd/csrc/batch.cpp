// Batched rendering: many requests (of different sizes, volumes, channel
// counts and precisions) in one launch.  Each (request, eye, wave tile) is
// one work item; the items of one data variant go to one kernel whose fixed
// grid of single-wave blocks takes them cyclically, most expensive request
// first, so one large view does not become the tail.  The launch (one kernel
// per variant present) is captured per stream, variant set and grid size
// into a HIP graph whose arguments point at fixed device tables; each batch
// only rewrites the tables.  Lit requests are launched one by one with the
// plain (lit) kernels on the same stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

#include "lib.h"

namespace vr {

double request_cost(const ReqParams& P) {
    // Rays times an upper estimate of samples per ray (box diagonal / step).
    double diag2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double len = (P.g.n[a] + 1.0) / (double)P.inv_sp[a];
        diag2 += len * len;
    }
    const double samples = std::sqrt(diag2) / (double)P.step;
    return (double)P.eyes * P.width * P.height * samples * (1.0 + 0.25 * P.channels);
}

static void free_tables(BatchSlot* s) {
    if (s->d_reqs) (void)hipFree(s->d_reqs);
    if (s->d_prefix) (void)hipFree(s->d_prefix);
    if (s->h_reqs) (void)hipHostFree(s->h_reqs);
    if (s->h_prefix) (void)hipHostFree(s->h_prefix);
    s->d_reqs = nullptr;
    s->d_prefix = nullptr;
    s->h_reqs = nullptr;
    s->h_prefix = nullptr;
    s->capacity = 0;
}

static void drop_graphs(BatchSlot* s) {
    for (auto& kv : s->graphs) {
        if (kv.second.second) (void)hipGraphExecDestroy(kv.second.second);
        if (kv.second.first) (void)hipGraphDestroy(kv.second.first);
    }
    s->graphs.clear();
}

void batch_slot_destroy(BatchSlot* s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    drop_graphs(s);
    free_tables(s);
    if (s->d_work) (void)hipFree(s->d_work);
    if (s->h_work) (void)hipHostFree(s->h_work);
    if (s->staged) (void)hipEventDestroy(s->staged);
    if (s->capture) (void)hipStreamDestroy(s->capture);
    delete s;
}

static vr_status grow(BatchSlot* s, int cap) {
    // Earlier launches on this stream may still read the old tables.
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    drop_graphs(s);  // the captured launches hold the old table addresses
    free_tables(s);
    if ((e = hipMalloc(&s->d_reqs, sizeof(ReqParams) * (size_t)cap)) != hipSuccess ||
        (e = hipMalloc(&s->d_prefix, sizeof(int32_t) * (size_t)cap)) != hipSuccess ||
        (e = hipHostMalloc(&s->h_reqs, sizeof(ReqParams) * (size_t)cap, hipHostMallocDefault)) !=
            hipSuccess ||
        (e = hipHostMalloc(&s->h_prefix, sizeof(int32_t) * (size_t)cap, hipHostMallocDefault)) !=
            hipSuccess) {
        free_tables(s);
        return fail(VR_ERR_OUT_OF_MEMORY, "batch tables for %d requests: %s", cap,
                    hipGetErrorString(e));
    }
    s->capacity = cap;
    return VR_OK;
}

BatchSlot* batch_slot_create(vr_ctx* ctx, hipStream_t stream, vr_status* st) {
    BatchSlot* s = new BatchSlot();
    s->stream = stream;
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&s->capture, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&s->staged, hipEventDisableTiming)) != hipSuccess ||
        (e = hipMalloc(&s->d_work, sizeof(BatchWork))) != hipSuccess ||
        (e = hipHostMalloc(&s->h_work, sizeof(BatchWork), hipHostMallocDefault)) != hipSuccess) {
        *st = hip_fail(e, "batch workspace");
        batch_slot_destroy(s);
        return nullptr;
    }
    *st = grow(s, 64);
    if (*st != VR_OK) {
        batch_slot_destroy(s);
        return nullptr;
    }
    return s;
}

BatchSlot* batch_slot_for(vr_ctx* ctx, hipStream_t stream, vr_status* st) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->batch_slots.find(stream);
    if (it != ctx->batch_slots.end()) {
        *st = VR_OK;
        return it->second;
    }
    BatchSlot* s = batch_slot_create(ctx, stream, st);
    if (s) ctx->batch_slots[stream] = s;
    return s;
}

static vr_status graph_for(BatchSlot* s, uint64_t mask, int blocks, hipGraphExec_t* out) {
    // variants present (48 bits) and the grid size (a power of two <= 2^17)
    const uint64_t key = mask << 16 | (uint64_t)(31 - __builtin_clz((unsigned)blocks));
    auto it = s->graphs.find(key);
    if (it != s->graphs.end()) {
        *out = it->second.second;
        return VR_OK;
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamBeginCapture(s->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = launch_batch(s->d_work, s->d_reqs, s->d_prefix, mask, blocks, s->capture);
    e = hipStreamEndCapture(s->capture, &graph);
    if (le != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(le, "batch launch capture");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    s->graphs[key] = {graph, exec};
    *out = exec;
    return VR_OK;
}

// Largest grid of a batch kernel, in single-wave blocks.
constexpr int kBatchBlocksMax = 1 << 17;

// ----------------------------------------------------------------- tuning
// Candidate wave tiles (pixels per wave, width x height).  Per-ray
// arithmetic does not depend on the tiling, so every candidate gives the
// same image bit for bit; only the speed differs.
static const TileShape kCandidates[] = {{8, 8}, {16, 4}, {4, 16}, {32, 2}, {64, 1}};

// Shape class: the set of data variants in the batch and the order of
// magnitude of its ray count.
static uint64_t shape_class(const ReqParams* params, int n) {
    uint64_t variants = 0;  // below 2^48: batched variants only
    double rays = 0.0;
    for (int q = 0; q < n; ++q) {
        variants |= 1ull << params[q].variant;
        rays += (double)params[q].eyes * params[q].width * params[q].height;
    }
    const int mag = rays > 1.0 ? (int)std::floor(std::log2(rays)) : 0;
    return ((uint64_t)variants << 8) | (uint64_t)mag;
}

static void load_tuning_cache(vr_ctx* ctx) {
    const char* path = std::getenv("VR_AUTOTUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    unsigned long long key;
    int a, b;
    while (std::fscanf(f, "%llx %d %d", &key, &a, &b) == 3)
        if (a > 0 && b > 0 && a * b == kWave) ctx->tuned[key] = TileShape{a, b};
    std::fclose(f);
}

static void save_tuning(uint64_t key, const TileShape& t) {
    const char* path = std::getenv("VR_AUTOTUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%llx %d %d\n", (unsigned long long)key, t.wave_w, t.wave_h);
    std::fclose(f);
}

static vr_status enqueue_with(vr_ctx* ctx, BatchSlot* s, const ReqParams* params, int n,
                              const TileShape& ts);

// Times every candidate on this batch (synchronously, on the slot's stream)
// and keeps the fastest for the batch's shape class.
static vr_status tune(vr_ctx* ctx, BatchSlot* s, const ReqParams* params, int n, uint64_t key,
                      TileShape* best) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return fail(VR_ERR_DEVICE, "autotune event");
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return fail(VR_ERR_DEVICE, "autotune event");
    }
    float best_ms = 1e30f;
    vr_status st = VR_OK;
    for (const TileShape& c : kCandidates) {
        float ms_total = 0.0f;
        for (int rep = 0; rep < 2 && st == VR_OK; ++rep) {  // first run warms caches
            (void)hipEventRecord(a, s->stream);
            st = enqueue_with(ctx, s, params, n, c);
            (void)hipEventRecord(b, s->stream);
            if (st == VR_OK && hipEventSynchronize(b) != hipSuccess)
                st = fail(VR_ERR_DEVICE, "autotune sync");
            float ms = 0.0f;
            if (st == VR_OK && rep == 1) {
                (void)hipEventElapsedTime(&ms, a, b);
                ms_total = ms;
            }
        }
        if (st != VR_OK) break;
        if (ms_total < best_ms) {
            best_ms = ms_total;
            *best = c;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st == VR_OK) {
        ctx->tuned[key] = *best;
        save_tuning(key, *best);
    }
    return st;
}

vr_status batch_enqueue(vr_ctx* ctx, BatchSlot* s, const ReqParams* params, int n,
                        bool allow_tuning) {
    if (n <= 0) return VR_OK;
    // Lit requests and large volumes take plain launches on the slot's stream
    // (the batch kernels are unlit and 32-bit addressed); the rest form the
    // batch.
    const auto plain = [](const ReqParams& P) {
        return P.light.on != 0 || variant_large(P.variant);
    };
    std::vector<ReqParams> unlit;
    bool any_plain = false;
    for (int q = 0; q < n && !any_plain; ++q) any_plain = plain(params[q]);
    if (any_plain) {
        for (int q = 0; q < n; ++q) {
            if (!plain(params[q])) {
                unlit.push_back(params[q]);
                continue;
            }
            const hipError_t e = launch_render(params[q], ctx->plain_tile, ctx->clear_skip,
                                               s->stream);
            if (e != hipSuccess) return hip_fail(e, "render launch");
        }
        params = unlit.data();
        n = (int)unlit.size();
        if (n == 0) return VR_OK;
    }
    TileShape ts = ctx->batch_tile;
    if (!ctx->forced_tile && ctx->autotune) {
        const uint64_t key = shape_class(params, n);
        std::unique_lock<std::mutex> lk(ctx->mu);
        if (!ctx->tuning_cache_loaded) {
            load_tuning_cache(ctx);
            ctx->tuning_cache_loaded = true;
        }
        auto it = ctx->tuned.find(key);
        if (it != ctx->tuned.end()) {
            ts = it->second;
        } else if (allow_tuning) {
            vr_status st = tune(ctx, s, params, n, key, &ts);
            if (st != VR_OK) return st;
        }
    }
    return enqueue_with(ctx, s, params, n, ts);
}

static vr_status enqueue_with(vr_ctx* ctx, BatchSlot* s, const ReqParams* params, int n,
                              const TileShape& ts) {
    hipError_t e;
    // Group by data variant (one persistent kernel each), most expensive
    // request first within a group.
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::vector<double> cost(n);
    for (int q = 0; q < n; ++q) cost[q] = request_cost(params[q]);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (params[a].variant != params[b].variant) return params[a].variant < params[b].variant;
        return cost[a] > cost[b];
    });

    if (n > s->capacity) {
        int cap = s->capacity;
        while (cap < n) cap *= 2;
        vr_status st = grow(s, cap);
        if (st != VR_OK) return st;
    }
    // The pinned staging buffers are reused: wait until the previous batch's
    // copies out of them have run.
    if (s->staged_pending) {
        if ((e = hipEventSynchronize(s->staged)) != hipSuccess) return hip_fail(e, "staging wait");
        s->staged_pending = false;
    }
    BatchWork* w = s->h_work;
    std::memset(w->group, 0, sizeof w->group);
    uint64_t mask = 0;
    int64_t items = 0;
    for (int q = 0; q < n; ++q) {
        const ReqParams& P = params[order[q]];
        BatchGroup& g = w->group[P.variant];
        if (g.n_req == 0) {
            g.first = q;
            items = 0;
        }
        s->h_reqs[q] = P;
        s->h_prefix[q] = (int32_t)items;
        items += tiles_per_eye(P.width, P.height, ts) * P.eyes;
        if (items > (1 << 30)) return fail(VR_ERR_INVALID_ARG, "batch has too many tiles");
        g.n_req += 1;
        g.n_items = (int32_t)items;
        if (items > 0) mask |= 1ull << P.variant;
    }
    if (mask == 0) return VR_OK;
    w->tile = ts;
    // Grid of every variant's kernel: the largest group's item count rounded
    // up to a power of two (a few captured graphs cover all batch sizes),
    // capped so that a block takes a handful of items of a large batch.
    int64_t most = 0;
    for (int v = 0; v < kBatchVariants; ++v) most = std::max<int64_t>(most, w->group[v].n_items);
    int blocks = kWave;
    while (blocks < most && blocks < kBatchBlocksMax) blocks *= 2;
    if ((e = hipMemcpyAsync(s->d_reqs, s->h_reqs, sizeof(ReqParams) * (size_t)n,
                            hipMemcpyHostToDevice, s->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(s->d_prefix, s->h_prefix, sizeof(int32_t) * (size_t)n,
                            hipMemcpyHostToDevice, s->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(s->d_work, s->h_work, sizeof(BatchWork), hipMemcpyHostToDevice,
                            s->stream)) != hipSuccess)
        return hip_fail(e, "batch table upload");
    if ((e = hipEventRecord(s->staged, s->stream)) != hipSuccess) return hip_fail(e, "event");
    s->staged_pending = true;

    if (ctx->use_graphs) {
        hipGraphExec_t exec = nullptr;
        vr_status st = graph_for(s, mask, blocks, &exec);
        if (st != VR_OK) return st;
        if ((e = hipGraphLaunch(exec, s->stream)) != hipSuccess)
            return hip_fail(e, "hipGraphLaunch");
    } else {
        if ((e = launch_batch(s->d_work, s->d_reqs, s->d_prefix, mask, blocks, s->stream)) !=
            hipSuccess)
            return hip_fail(e, "batch launch");
    }
    return VR_OK;
}

}  // namespace vr

using namespace vr;

extern "C" vr_status vr_test_batch_tile(vr_ctx* ctx, int32_t wave_w, int32_t wave_h) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    if (wave_w == 0 && wave_h == 0) {
        ctx->forced_tile = false;
        return ok();
    }
    if (wave_w <= 0 || wave_h <= 0 || wave_w * wave_h != kWave)
        return fail(VR_ERR_INVALID_ARG, "a wave tile is 64 pixels");
    ctx->batch_tile = TileShape{wave_w, wave_h};
    ctx->forced_tile = true;
    return ok();
}

extern "C" vr_status vr_test_plain_tile(vr_ctx* ctx, int32_t wave_w, int32_t wave_h) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    if (wave_w == 0 && wave_h == 0) {
        ctx->plain_tile = default_tile();
        return ok();
    }
    if (wave_w <= 0 || wave_h <= 0 || wave_w * wave_h != kWave)
        return fail(VR_ERR_INVALID_ARG, "a wave tile is 64 pixels");
    ctx->plain_tile = TileShape{wave_w, wave_h};
    return ok();
}

extern "C" vr_status vr_test_clear_skip(vr_ctx* ctx, int32_t on) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    ctx->clear_skip = on != 0;
    return ok();
}

extern "C" vr_status vr_test_large_addressing(vr_ctx* ctx, int32_t on) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    ctx->force_large = on != 0;
    return ok();
}

extern "C" vr_status vr_render_batch(vr_ctx* ctx, const vr_render_req* reqs, int32_t n,
                                     void* hip_stream) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    if (n < 0) return fail(VR_ERR_INVALID_ARG, "n < 0");
    if (n > 0 && !reqs) return fail(VR_ERR_INVALID_ARG, "requests are NULL");
    for (int q = 0; q < n; ++q) {
        vr_status st = check_request(ctx, &reqs[q]);
        if (st != VR_OK) {
            std::string m = vr_last_error();
            return fail(st, "request %d: %s", q, m.c_str());
        }
    }
    if (ctx->device < 0) return fail(VR_ERR_UNSUPPORTED, "validation-only context");
    if (n == 0) return ok();
    std::vector<ReqParams> P((size_t)n);
    for (int q = 0; q < n; ++q) {
        std::lock_guard<std::mutex> lk(reqs[q].vol->tf_mu);
        make_params(reqs[q], reqs[q].vol->tf, &P[q]);
    }
    DeviceGuard dg(ctx->device);
    vr_status st;
    BatchSlot* s = batch_slot_for(ctx, (hipStream_t)hip_stream, &st);
    if (!s) return st;
    st = batch_enqueue(ctx, s, P.data(), n);
    if (st != VR_OK) return st;
    return ok();
}
