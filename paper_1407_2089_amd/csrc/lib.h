// Internal host-side state of libvr (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/vr.h"
#include "kernels.h"
#include "params.h"

namespace vr {

// Makes the context's device current for the calling thread for the length
// of one entry point, and restores the caller's device afterwards.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int device) {
        if (device < 0 || hipGetDevice(&prev) != hipSuccess) {
            prev = -1;
            return;
        }
        if (prev == device || hipSetDevice(device) != hipSuccess) prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
    DeviceGuard(const DeviceGuard&) = delete;
    DeviceGuard& operator=(const DeviceGuard&) = delete;
};

class Scheduler;

// Workspace of batched launches on one stream: device tables that a captured
// graph reads, their pinned host staging copies, and the instantiated graph.
struct BatchSlot {
    hipStream_t stream = nullptr;   // the caller's stream this slot serves
    hipStream_t capture = nullptr;  // private stream used only for capture
    int capacity = 0;               // requests the tables can hold
    ReqParams* d_reqs = nullptr;
    int32_t* d_prefix = nullptr;
    BatchWork* d_work = nullptr;
    ReqParams* h_reqs = nullptr;    // pinned
    int32_t* h_prefix = nullptr;    // pinned
    BatchWork* h_work = nullptr;    // pinned
    hipEvent_t staged = nullptr;    // staging copies of the last batch done
    bool staged_pending = false;
    // Captured launches, one per (set of variants present, grid size) of a
    // batch (they hold the table addresses: dropped when the tables grow).
    // One instantiated graph per set of variants present (the key), with
    // each variant's node and the grid it was last launched with (updated in
    // place when a batch needs another).
    struct Graph {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipGraphNode_t node[kBatchVariants] = {};
        int32_t blocks[kBatchVariants] = {};
    };
    std::map<uint64_t, Graph> graphs;
};

// Sets the calling thread's error message and returns `st`.
vr_status fail(vr_status st, const char* fmt, ...);
vr_status ok();
vr_status hip_fail(hipError_t e, const char* what);

}  // namespace vr

struct vr_volume {
    vr_ctx* ctx = nullptr;
    vr_volume_desc desc{};
    vr::BrickGeom geom{};
    uint8_t* storage = nullptr;
    uint64_t bytes = 0;
    std::mutex tf_mu;
    vr_transfer tf[vr::kMaxChannels]{};
    bool large = false;             // large-volume addressing (64-bit, FP64 positions)
    std::atomic<int> in_flight{0};  // served tickets that read this volume
    // vr_stream_frame / vr_stream_ready: the render stream's work before an
    // upload, and per slot the end of its last upload (events are re-recorded;
    // a wait takes the record that precedes it).
    std::mutex stream_mu;
    hipStream_t relayout_stream = nullptr;  // created by the first upload
    hipEvent_t ev_before = nullptr;
    hipEvent_t ev_copied[2] = {nullptr, nullptr};  // per staging half: copy landed
    hipEvent_t ev_free[2] = {nullptr, nullptr};    // per staging half: relayout read it
    bool half_used[2] = {false, false};
    int next_half = 0;
    std::vector<hipEvent_t> ev_loaded;   // per slot, created by its first upload
};

struct vr_ctx {
    int device = -1;           // -1: validation-only context
    uint64_t budget = 0;
    std::atomic<uint64_t> used{0};
    std::atomic<int> volumes{0};
    std::mutex mu;
    // Batched-launch workspaces keyed by stream (batch.cpp).
    std::map<hipStream_t, vr::BatchSlot*> batch_slots;
    bool use_graphs = true;
    // Autotuner: chosen tile shape per shape class (batch.cpp).
    bool autotune = true;
    bool forced_tile = false;          // a test fixed the tile shape
    bool tuning_cache_loaded = false;
    vr::TileShape batch_tile{8, 8};
    vr::TileShape plain_tile{8, 8};  // wave tile of vr_render launches
    bool clear_skip = true;  // vr_render leaves out transparent samples' arithmetic
    bool cell_skip = true;   // rays jump over macro cells shown transparent
    bool force_large = false;  // new volumes take large-volume addressing (test hook)
    int cell_shift = vr::kCellShift;  // macro-cell edge of new volumes (test hook)
    std::map<uint64_t, vr::TileShape> tuned;
    vr::Scheduler* server = nullptr;  // created by the first vr_submit (server.cpp)
    std::mutex server_mu;
    // vr_render_batch_noalloc (batch.cpp): the device address of the
    // library's static scratch array on this context's device, and pinned
    // staging of its tables, all set up by vr_init.
    uint8_t* noalloc_dev = nullptr;
    void* noalloc_host[2] = {nullptr, nullptr};
    hipEvent_t noalloc_ev[2] = {nullptr, nullptr};
    bool noalloc_used[2] = {false, false};
    int noalloc_next = 0;
    vr::ReqParams* noalloc_params = nullptr;  // host array of kNoAllocRequests
    std::mutex noalloc_mu;
};

namespace vr {

// Validation helpers (api.cpp).
vr_status check_desc(const vr_volume_desc* d);
vr_status check_request(const vr_ctx* ctx, const vr_render_req* r);
BrickGeom make_geom(const vr_volume_desc& d);
// Macro cells of 2^shift sample corners per axis: cell counts, frame size.
void set_cell_shift(BrickGeom* g, int shift);
// True when the volume needs large-volume addressing: an axis above
// kFloatAxis voxels, or a frame of 2^31 stored words, 2^24 bricks or 4 GiB
// and more.
bool needs_large(const vr_volume_desc& d, const BrickGeom& g);
// Clamp bounds of the FP64 sample positions (large variants).
void set_clamp_d64(const BrickGeom& g, ReqParams* P);
// Fills the device parameters of a request from the volume's current transfer
// functions (or from `tf` when given).
void make_params(const vr_render_req& r, const vr_transfer* tf, ReqParams* P);
TileShape default_tile();

// Batched path (batch.cpp).
// Sets up vr_render_batch_noalloc on the context's device (the device is
// current): the scratch array's address and the pinned staging.
vr_status noalloc_init(vr_ctx* ctx);
void noalloc_release(vr_ctx* ctx);
// Enqueues a batch with the tile tuned for its shape class (or the default);
// never tunes and never waits for the device beyond its staging buffers.
vr_status batch_enqueue(vr_ctx* ctx, BatchSlot* slot, const ReqParams* params, int n);
// Times every candidate tile on this batch (synchronously) and records the
// fastest for its shape class.
vr_status batch_tune(vr_ctx* ctx, BatchSlot* slot, const ReqParams* params, int n,
                     TileShape* best);
BatchSlot* batch_slot_for(vr_ctx* ctx, hipStream_t stream, vr_status* st);
BatchSlot* batch_slot_create(vr_ctx* ctx, hipStream_t stream, vr_status* st);
void batch_slot_destroy(BatchSlot* slot);
// Estimated relative cost of a request (for ordering work).
double request_cost(const ReqParams& P);

// Serving (server.cpp).
vr_status server_submit(vr_ctx* ctx, const vr_render_req* req, uint64_t* ticket);
vr_status server_poll(vr_ctx* ctx, uint64_t ticket, vr_ticket_info* info);
vr_status server_release(vr_ctx* ctx, uint64_t ticket);
vr_status server_stop(vr_ctx* ctx);

}  // namespace vr
