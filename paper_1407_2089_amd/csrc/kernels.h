// Launchers of the HIP kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "params.h"

namespace vr {

// Requests of one data variant within a batch: reqs[first .. first + n_req)
// (most expensive first), their work items numbered from 0.
struct BatchGroup {
    int32_t first;
    int32_t n_req;
    int32_t n_items;
    int32_t pad_;
};

// Device-resident description of one batched launch.  With it the kernels
// take the request descriptors (grouped by variant) and each request's first
// work item within its group.  The host rewrites all three before each
// launch; their addresses stay fixed until the tables grow, so a captured
// graph can be replayed.  One kernel per data variant present works through
// that variant's group: a fixed grid of single-wave blocks, block b taking
// items b, b + grid, b + 2 grid, ... (after the XCD remap), so the hardware
// dispatcher balances the load as blocks finish, with no shared counter.
struct BatchWork {
    TileShape tile;
    BatchGroup group[kBatchVariants];
};

hipError_t launch_relayout(const BrickGeom& g, int channels, bool u16, int bits,
                           const void* src, uint8_t* dst, hipStream_t s);
// clear_skip = false selects the kernels that composite transparent samples
// in full (same output bits).
hipError_t launch_render(const ReqParams& P, const TileShape& ts, bool clear_skip,
                         hipStream_t s);
// Launch the batch kernels of the variants set in `mask`, blocks[v]
// single-wave blocks for variant v, one after the other on `s`.
hipError_t launch_batch(const BatchWork* dev_work, const ReqParams* dev_reqs,
                        const int32_t* dev_prefix, uint64_t mask, const int32_t* blocks,
                        hipStream_t s);
// The same kernels as independent nodes of `graph` (parallel branches: the
// variants' kernels may overlap on the device); nodes[v] receives variant
// v's node.
hipError_t add_batch_nodes(hipGraph_t graph, const BatchWork* dev_work,
                           const ReqParams* dev_reqs, const int32_t* dev_prefix, uint64_t mask,
                           const int32_t* blocks, hipGraphNode_t* nodes);
// Sets the grid of variant v's node in an instantiated batch graph.
hipError_t set_batch_node_grid(hipGraphExec_t exec, hipGraphNode_t node, int v, int blocks,
                               const BatchWork* dev_work, const ReqParams* dev_reqs,
                               const int32_t* dev_prefix);
hipError_t launch_debug_sample(const ReqParams& P, const float* pts, int n, float* out,
                               hipStream_t s);

}  // namespace vr
