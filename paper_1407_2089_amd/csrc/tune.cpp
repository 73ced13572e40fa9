// Layout tuning: the voxel layout (brick edges and row pairs) chosen per
// dataset by measurement.  Every layout stores the same voxels and gives the
// same image bits; they differ in how many cache lines a wave's taps touch,
// which depends on the voxel word, the volume's shape and the views.  Each
// candidate is built from one frame in scratch storage and timed on the
// caller's views; the fastest (or, among those within 2 % of it, the one with
// the smallest storage) is written back into the description.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "lib.h"

namespace vr {

struct LayoutCandidate {
    int32_t brick[3];
    int32_t pairs;
};

// Candidates measured to lead for some word size in the layout sweep of a
// 512 x 512 x 64 frame (1-, 2-, 4-byte words, views through the top and the
// side faces), plus the defaults: the library default first, so that a tie
// keeps it.
static std::vector<LayoutCandidate> layout_candidates(const vr_volume_desc& d) {
    std::vector<LayoutCandidate> out = {
        {{0, 0, 0}, 0},  {{8, 8, 8}, 0},  {{8, 16, 8}, 0},   {{16, 16, 8}, 0},
        {{16, 8, 8}, 0}, {{8, 8, 4}, 0},  {{4, 16, 8}, 0},   {{16, 16, 16}, 0},
        {{0, 0, 0}, 1},  {{4, 16, 8}, 1}, {{8, 16, 8}, 1},   {{8, 32, 8}, 1},
        {{4, 32, 8}, 1}, {{16, 16, 16}, 1}};
    const int w = word_bytes(d.channels, d.dtype == VR_U16);
    out.erase(std::remove_if(out.begin(), out.end(),
                             [&](const LayoutCandidate& c) {
                                 return c.pairs && w > max_pair_word(true);
                             }),
              out.end());
    return out;
}

// Median of the event-timed renders of one request.
static vr_status time_view(vr_ctx* ctx, const vr_render_req& r, int reps, hipStream_t s,
                           hipEvent_t* ev, float* ms) {
    for (int i = 0; i < 2; ++i) {
        vr_status st = vr_render(ctx, &r, s);
        if (st != VR_OK) return st;
    }
    std::vector<float> t(reps);
    for (int i = 0; i < reps; ++i) {
        hipError_t e = hipEventRecord(ev[0], s);
        if (e != hipSuccess) return hip_fail(e, "event record");
        vr_status st = vr_render(ctx, &r, s);
        if (st != VR_OK) return st;
        e = hipEventRecord(ev[1], s);
        if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&t[i], ev[0], ev[1]);
        if (e != hipSuccess) return hip_fail(e, "render timing");
    }
    std::nth_element(t.begin(), t.begin() + reps / 2, t.end());
    *ms = t[reps / 2];
    return ok();
}

}  // namespace vr

using namespace vr;

extern "C" {

vr_status vr_tune_layout(vr_ctx* ctx, vr_volume_desc* desc, const vr_transfer* tfs,
                         const void* dev_frame, const vr_render_req* views, int32_t n_views,
                         int32_t reps, uint64_t max_bytes, void* hip_stream, float* best_ms) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    vr_status st = check_desc(desc);
    if (st != VR_OK) return st;
    if (!tfs) return fail(VR_ERR_INVALID_ARG, "transfer functions are NULL");
    if (!dev_frame) return fail(VR_ERR_INVALID_ARG, "frame is NULL");
    if (n_views < 1 || !views) return fail(VR_ERR_INVALID_ARG, "no views to time");
    if (reps < 1 || reps > 1000) return fail(VR_ERR_INVALID_ARG, "reps = %d outside 1..1000", reps);
    if (ctx->device < 0) return fail(VR_ERR_UNSUPPORTED, "validation-only context");
    DeviceGuard dg(ctx->device);
    const hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t ev[2] = {nullptr, nullptr};
    for (int i = 0; i < 2; ++i) {
        hipError_t e = hipEventCreate(&ev[i]);
        if (e != hipSuccess) {
            if (ev[0]) (void)hipEventDestroy(ev[0]);
            return hip_fail(e, "event create");
        }
    }
    const std::vector<LayoutCandidate> cands = layout_candidates(*desc);
    std::vector<float> times(cands.size(), -1.0f);      // -1: not a candidate here
    std::vector<uint64_t> sizes(cands.size(), 0);
    st = VR_OK;
    for (size_t ci = 0; ci < cands.size() && st == VR_OK; ++ci) {
        vr_volume_desc d = *desc;
        std::memcpy(d.brick, cands[ci].brick, sizeof d.brick);
        d.row_pairs = cands[ci].pairs;
        uint64_t total = 0, frame_bytes = 0;
        if (check_desc(&d) != VR_OK || vr_volume_storage_bytes(&d, &total) != VR_OK) continue;
        if (max_bytes != 0 && total > max_bytes) continue;
        sizes[ci] = total;
        d.frames = 1;
        if (vr_volume_storage_bytes(&d, &frame_bytes) != VR_OK) continue;
        void* mem = nullptr;
        if (hipMalloc(&mem, frame_bytes) != hipSuccess) {
            (void)hipGetLastError();
            continue;  // too large for the device now: not a candidate
        }
        vr_volume* vol = nullptr;
        if (vr_create_volume(ctx, &d, mem, frame_bytes, &vol) != VR_OK) {
            (void)hipFree(mem);
            continue;  // not admissible (row pairs of 8-byte words, budget)
        }
        for (int c = 0; c < d.channels && st == VR_OK; ++c) st = vr_set_transfer(vol, c, &tfs[c]);
        if (st == VR_OK) st = vr_upload_frame(vol, 0, dev_frame, s);
        float sum = 0.0f;
        for (int q = 0; q < n_views && st == VR_OK; ++q) {
            vr_render_req r = views[q];
            r.vol = vol;
            r.frame = 0;
            float ms = 0.0f;
            st = time_view(ctx, r, reps, s, ev, &ms);
            sum += ms;
        }
        hipError_t e = hipStreamSynchronize(s);
        if (st == VR_OK && e != hipSuccess) st = hip_fail(e, "tuning render");
        (void)vr_destroy_volume(vol);
        (void)hipFree(mem);
        if (st == VR_OK) times[ci] = sum;
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (st != VR_OK) return st;
    // The fastest, unless another candidate within 2 % of it (timing noise
    // between layouts this close) stores the volume in fewer bytes: then the
    // smallest of those.  Earlier candidates win ties.
    int fastest = -1;
    for (size_t ci = 0; ci < cands.size(); ++ci)
        if (times[ci] >= 0.0f && (fastest < 0 || times[ci] < times[fastest])) fastest = (int)ci;
    if (fastest < 0)
        return fail(VR_ERR_OUT_OF_MEMORY, "no candidate layout fits the limits or the device");
    int best = fastest;
    for (size_t ci = 0; ci < cands.size(); ++ci)
        if (times[ci] >= 0.0f && times[ci] <= 1.02f * times[fastest] && sizes[ci] < sizes[best])
            best = (int)ci;
    const float best_t = times[best];
    std::memcpy(desc->brick, cands[best].brick, sizeof desc->brick);
    desc->row_pairs = cands[best].pairs;
    if (best_ms) *best_ms = best_t;
    return ok();
}

}  // extern "C"
