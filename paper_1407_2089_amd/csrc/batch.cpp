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
#include <cstddef>
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
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
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

// The batch's kernels, one per variant present with its own grid, as
// parallel branches of one graph (built node by node), instantiated once per
// set of variants present; a batch whose grids differ from the last launch
// of that graph updates the nodes in place (no new instantiation: serving
// forms batches of ever-changing sizes).
static vr_status graph_for(BatchSlot* s, uint64_t mask, const int32_t* blocks,
                           hipGraphExec_t* out) {
    hipError_t e;
    auto it = s->graphs.find(mask);
    if (it != s->graphs.end()) {
        BatchSlot::Graph& g = it->second;
        for (int v = 0; v < kBatchVariants; ++v) {
            if (!(mask & (1ull << v)) || g.blocks[v] == blocks[v]) continue;
            e = set_batch_node_grid(g.exec, g.node[v], v, blocks[v], s->d_work, s->d_reqs,
                                    s->d_prefix);
            if (e != hipSuccess) return hip_fail(e, "batch graph update");
            g.blocks[v] = blocks[v];
        }
        *out = g.exec;
        return VR_OK;
    }
    BatchSlot::Graph g;
    if ((e = hipGraphCreate(&g.graph, 0)) != hipSuccess) return hip_fail(e, "hipGraphCreate");
    e = add_batch_nodes(g.graph, s->d_work, s->d_reqs, s->d_prefix, mask, blocks, g.node);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g.graph);
        return hip_fail(e, "batch graph nodes");
    }
    e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g.graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    for (int v = 0; v < kBatchVariants; ++v) g.blocks[v] = blocks[v];
    s->graphs[mask] = g;
    *out = g.exec;
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

// Lit requests and large volumes take plain launches on the slot's stream
// (the batch kernels are unlit and 32-bit addressed); the rest form the
// batch, returned in `rest`.
static vr_status launch_plain_part(vr_ctx* ctx, BatchSlot* s, const ReqParams* params, int n,
                                   std::vector<ReqParams>* rest) {
    rest->clear();
    for (int q = 0; q < n; ++q) {
        const ReqParams& P = params[q];
        if (P.light.on == 0 && !variant_large(P.variant)) {
            rest->push_back(P);
            continue;
        }
        const hipError_t e = launch_render(P, ctx->plain_tile, ctx->clear_skip, s->stream);
        if (e != hipSuccess) return hip_fail(e, "render launch");
    }
    return VR_OK;
}

static void ensure_tuning_cache(vr_ctx* ctx) {
    // caller holds ctx->mu
    if (!ctx->tuning_cache_loaded) {
        load_tuning_cache(ctx);
        ctx->tuning_cache_loaded = true;
    }
}

vr_status batch_tune(vr_ctx* ctx, BatchSlot* s, const ReqParams* params_in, int n,
                     TileShape* best) {
    std::vector<ReqParams> rest;
    vr_status st = launch_plain_part(ctx, s, params_in, n, &rest);
    if (st != VR_OK) return st;
    *best = ctx->batch_tile;
    if (rest.empty()) return VR_OK;
    const ReqParams* params = rest.data();
    n = (int)rest.size();
    const uint64_t key = shape_class(params, n);
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return fail(VR_ERR_DEVICE, "autotune event");
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return fail(VR_ERR_DEVICE, "autotune event");
    }
    // No lock is held while the candidates run: the tuned map is read and
    // written under ctx->mu only.
    float best_ms = 1e30f;
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
    if (st != VR_OK) return st;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ensure_tuning_cache(ctx);
        ctx->tuned[key] = *best;
    }
    save_tuning(key, *best);
    return VR_OK;
}

vr_status batch_enqueue(vr_ctx* ctx, BatchSlot* s, const ReqParams* params, int n) {
    if (n <= 0) return VR_OK;
    std::vector<ReqParams> rest;
    bool any_plain = false;
    for (int q = 0; q < n && !any_plain; ++q)
        any_plain = params[q].light.on != 0 || variant_large(params[q].variant);
    if (any_plain) {
        vr_status st = launch_plain_part(ctx, s, params, n, &rest);
        if (st != VR_OK) return st;
        params = rest.data();
        n = (int)rest.size();
        if (n == 0) return VR_OK;
    }
    TileShape ts = ctx->batch_tile;
    if (!ctx->forced_tile && ctx->autotune) {
        const uint64_t key = shape_class(params, n);
        std::lock_guard<std::mutex> lk(ctx->mu);
        ensure_tuning_cache(ctx);
        auto it = ctx->tuned.find(key);
        if (it != ctx->tuned.end()) ts = it->second;
    }
    return enqueue_with(ctx, s, params, n, ts);
}

// Lays out the device tables of a batch in host memory (no allocation:
// `order` and `cost` hold n entries of the caller's): requests grouped by data variant
// (one kernel each), most expensive first within a group (a stable insertion
// sort; batches are small), each request's first work item within its group,
// and each variant's grid: its item count rounded up to a power of two (a
// few instantiated graphs cover all batch sizes), at least one wave's worth
// and at most kBatchBlocksMax, so that a block takes a handful of items of a
// large group.  Returns VR_OK with *mask = 0 when no request has pixels.
static vr_status build_tables(const ReqParams* params, int n, const TileShape& ts, int* order,
                              double* cost, ReqParams* h_reqs, int32_t* h_prefix, BatchWork* w,
                              uint64_t* mask, int32_t* blocks) {
    for (int q = 0; q < n; ++q) cost[q] = request_cost(params[q]);
    for (int q = 0; q < n; ++q) {
        int i = q;
        while (i > 0) {
            const int o = order[i - 1];
            const bool after = params[o].variant > params[q].variant ||
                               (params[o].variant == params[q].variant && cost[o] < cost[q]);
            if (!after) break;
            order[i] = order[i - 1];
            --i;
        }
        order[i] = q;
    }
    std::memset(w->group, 0, sizeof w->group);
    *mask = 0;
    int64_t items = 0;
    for (int q = 0; q < n; ++q) {
        const ReqParams& P = params[order[q]];
        BatchGroup& g = w->group[P.variant];
        if (g.n_req == 0) {
            g.first = q;
            items = 0;
        }
        h_reqs[q] = P;
        h_prefix[q] = (int32_t)items;
        items += tiles_per_eye(P.width, P.height, ts) * P.eyes;
        if (items > (1 << 30)) return fail(VR_ERR_INVALID_ARG, "batch has too many tiles");
        g.n_req += 1;
        g.n_items = (int32_t)items;
        if (items > 0) *mask |= 1ull << P.variant;
    }
    w->tile = ts;
    for (int v = 0; v < kBatchVariants; ++v) {
        int32_t b = kWave;
        while (b < w->group[v].n_items && b < kBatchBlocksMax) b *= 2;
        blocks[v] = (*mask & (1ull << v)) ? b : 0;
    }
    return VR_OK;
}

static vr_status enqueue_with(vr_ctx* ctx, BatchSlot* s, const ReqParams* params, int n,
                              const TileShape& ts) {
    hipError_t e;
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
    std::vector<int> order((size_t)n);
    std::vector<double> cost((size_t)n);
    uint64_t mask = 0;
    int32_t blocks[kBatchVariants];
    vr_status st = build_tables(params, n, ts, order.data(), cost.data(), s->h_reqs, s->h_prefix,
                                s->h_work, &mask, blocks);
    if (st != VR_OK || mask == 0) return st;
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
        st = graph_for(s, mask, blocks, &exec);
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

// ------------------------------------------------- allocation-free batches
// vr_render_batch_noalloc keeps its tables in `scratch`, a static device
// array of this file (one copy per GPU, held until the process ends): the
// batch description, up to kNoAllocRequests request descriptors and their
// first work items.  Host code never passes `scratch` itself (its name is a
// host-side stand-in); it uses the address hipGetSymbolAddress gives on each
// device, kept in the context by vr_init.  Tables reach the array by an
// asynchronous copy from pinned staging (two halves that alternate; a half
// is rewritten once the copy out of it has run), then the variant kernels
// are launched directly.  Every call on a GPU shares that GPU's array: calls
// that overlap on the device (different streams, or contexts) race; calls on
// one stream are ordered.
constexpr int kNoAllocRequests = 256;
struct NoAllocTables {
    BatchWork work;
    ReqParams reqs[kNoAllocRequests];
    int32_t prefix[kNoAllocRequests];
};
constexpr size_t kNoAllocScratchBytes = (sizeof(NoAllocTables) + 255) & ~(size_t)255;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

vr_status noalloc_init(vr_ctx* ctx) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    ctx->noalloc_dev = (uint8_t*)ptr;
    ctx->noalloc_params = new ReqParams[kNoAllocRequests];
    for (int h = 0; h < 2; ++h) {
        if ((e = hipHostMalloc(&ctx->noalloc_host[h], sizeof(NoAllocTables),
                               hipHostMallocDefault)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&ctx->noalloc_ev[h], hipEventDisableTiming)) !=
                hipSuccess) {
            noalloc_release(ctx);
            return hip_fail(e, "allocation-free batch staging");
        }
    }
    return VR_OK;
}

void noalloc_release(vr_ctx* ctx) {
    for (int h = 0; h < 2; ++h) {
        if (ctx->noalloc_ev[h]) {
            (void)hipEventSynchronize(ctx->noalloc_ev[h]);
            (void)hipEventDestroy(ctx->noalloc_ev[h]);
        }
        if (ctx->noalloc_host[h]) (void)hipHostFree(ctx->noalloc_host[h]);
        ctx->noalloc_ev[h] = nullptr;
        ctx->noalloc_host[h] = nullptr;
    }
    ctx->noalloc_dev = nullptr;
    delete[] ctx->noalloc_params;
    ctx->noalloc_params = nullptr;
}

}  // namespace vr

using namespace vr;

extern "C" vr_status vr_render_batch_noalloc(vr_ctx* ctx, const vr_render_req* reqs, int32_t n,
                                             void* hip_stream) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    if (n < 0) return fail(VR_ERR_INVALID_ARG, "n < 0");
    if (n > kNoAllocRequests)
        return fail(VR_ERR_INVALID_ARG, "%d requests: the allocation-free batch takes at most %d",
                    n, kNoAllocRequests);
    if (n > 0 && !reqs) return fail(VR_ERR_INVALID_ARG, "requests are NULL");
    for (int q = 0; q < n; ++q) {
        vr_status st = check_request(ctx, &reqs[q]);
        if (st != VR_OK) return st;
    }
    if (ctx->device < 0) return fail(VR_ERR_UNSUPPORTED, "validation-only context");
    if (n == 0) return ok();
    if (!ctx->noalloc_dev) return fail(VR_ERR_DEVICE, "allocation-free batches are not set up");
    DeviceGuard dg(ctx->device);
    const hipStream_t stream = (hipStream_t)hip_stream;
    std::lock_guard<std::mutex> lk(ctx->noalloc_mu);
    const int h = ctx->noalloc_next;
    hipError_t e;
    if (ctx->noalloc_used[h] && (e = hipEventSynchronize(ctx->noalloc_ev[h])) != hipSuccess)
        return hip_fail(e, "staging wait");
    NoAllocTables* T = (NoAllocTables*)ctx->noalloc_host[h];
    // Parameters in the staging's request array first; lit requests and large
    // volumes take plain launches (their parameters travel as kernel
    // arguments), the rest are compacted to the front.
    int m = 0;
    for (int q = 0; q < n; ++q) {
        ReqParams P;
        {
            std::lock_guard<std::mutex> tl(reqs[q].vol->tf_mu);
            make_params(reqs[q], reqs[q].vol->tf, &P);
        }
        if (P.light.on != 0 || variant_large(P.variant)) {
            if ((e = launch_render(P, ctx->plain_tile, ctx->clear_skip, stream)) != hipSuccess)
                return hip_fail(e, "render launch");
            continue;
        }
        T->reqs[m++] = P;
    }
    if (m == 0) return ok();
    TileShape ts = ctx->batch_tile;
    if (!ctx->forced_tile && ctx->autotune) {
        std::lock_guard<std::mutex> tl(ctx->mu);
        auto it = ctx->tuned.find(shape_class(T->reqs, m));
        if (it != ctx->tuned.end()) ts = it->second;
    }
    // build_tables reads the parameters from a second array: the sorted copy
    // goes to the staging's tables.
    ReqParams* unsorted = ctx->noalloc_params;
    int order[kNoAllocRequests];
    double cost[kNoAllocRequests];
    for (int q = 0; q < m; ++q) unsorted[q] = T->reqs[q];
    uint64_t mask = 0;
    int32_t blocks[kBatchVariants];
    vr_status st = build_tables(unsorted, m, ts, order, cost, T->reqs, T->prefix, &T->work, &mask,
                                blocks);
    if (st != VR_OK) return st;
    if (mask == 0) return ok();
    NoAllocTables* D = (NoAllocTables*)ctx->noalloc_dev;
    const size_t bytes = offsetof(NoAllocTables, reqs) + sizeof(ReqParams) * (size_t)m;
    if ((e = hipMemcpyAsync(D, T, bytes, hipMemcpyHostToDevice, stream)) != hipSuccess ||
        (e = hipMemcpyAsync(D->prefix, T->prefix, sizeof(int32_t) * (size_t)m,
                            hipMemcpyHostToDevice, stream)) != hipSuccess ||
        (e = hipEventRecord(ctx->noalloc_ev[h], stream)) != hipSuccess)
        return hip_fail(e, "table upload");
    ctx->noalloc_used[h] = true;
    ctx->noalloc_next = 1 - h;
    if ((e = launch_batch(&D->work, D->reqs, D->prefix, mask, blocks, stream)) != hipSuccess)
        return hip_fail(e, "batch launch");
    return ok();
}

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
    if (on < 0 || on > 2) return fail(VR_ERR_INVALID_ARG, "on must be 0, 1 or 2");
    ctx->clear_skip = on != 0;
    ctx->cell_skip = on == 1;
    return ok();
}

extern "C" vr_status vr_test_large_addressing(vr_ctx* ctx, int32_t on) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    ctx->force_large = on != 0;
    return ok();
}

extern "C" vr_status vr_test_cell_shift(vr_ctx* ctx, int32_t shift) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    if (shift < 2 || shift > 5) return fail(VR_ERR_INVALID_ARG, "cell shift %d outside 2..5", shift);
    ctx->cell_shift = shift;
    return ok();
}

extern "C" vr_status vr_test_volume_large(const vr_volume* vol, int32_t* large) {
    if (!vol || !large) return fail(VR_ERR_INVALID_ARG, "volume or out is NULL");
    *large = vol->large ? 1 : 0;
    return ok();
}

// Validation and parameter snapshot shared by vr_render_batch and
// vr_tune_batch.
static vr_status batch_params(vr_ctx* ctx, const vr_render_req* reqs, int32_t n,
                              std::vector<ReqParams>* P) {
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
    P->resize((size_t)n);
    for (int q = 0; q < n; ++q) {
        std::lock_guard<std::mutex> lk(reqs[q].vol->tf_mu);
        make_params(reqs[q], reqs[q].vol->tf, &(*P)[q]);
    }
    return VR_OK;
}

extern "C" vr_status vr_render_batch(vr_ctx* ctx, const vr_render_req* reqs, int32_t n,
                                     void* hip_stream) {
    std::vector<ReqParams> P;
    vr_status st = batch_params(ctx, reqs, n, &P);
    if (st != VR_OK) return st;
    if (n == 0) return ok();
    DeviceGuard dg(ctx->device);
    BatchSlot* s = batch_slot_for(ctx, (hipStream_t)hip_stream, &st);
    if (!s) return st;
    st = batch_enqueue(ctx, s, P.data(), n);
    if (st != VR_OK) return st;
    return ok();
}

extern "C" vr_status vr_tune_batch(vr_ctx* ctx, const vr_render_req* reqs, int32_t n,
                                   void* hip_stream, int32_t* wave_w, int32_t* wave_h) {
    std::vector<ReqParams> P;
    vr_status st = batch_params(ctx, reqs, n, &P);
    if (st != VR_OK) return st;
    TileShape best = ctx->batch_tile;
    if (n > 0) {
        DeviceGuard dg(ctx->device);
        BatchSlot* s = batch_slot_for(ctx, (hipStream_t)hip_stream, &st);
        if (!s) return st;
        st = batch_tune(ctx, s, P.data(), n, &best);
        if (st != VR_OK) return st;
    }
    if (wave_w) *wave_w = best.wave_w;
    if (wave_h) *wave_h = best.wave_h;
    return ok();
}
