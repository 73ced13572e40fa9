// Launchers of the HIP kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "params.h"

namespace vr {

// Device-resident description of one batched launch.  The host rewrites the
// pointed-to arrays before each launch; the pointers themselves stay fixed so
// a captured graph can be replayed.
struct BatchWork {
    const ReqParams* reqs;  // [n_req], most expensive request first
    const int32_t* prefix;  // [n_req] first work item of each request
    int32_t* counter;       // next unclaimed work item
    int32_t n_req;
    int32_t n_items;
    TileShape tile;
};

hipError_t launch_relayout(const BrickGeom& g, int channels, bool u16, int bits,
                           const void* src, uint8_t* dst, hipStream_t s);
hipError_t launch_render(const ReqParams& P, const TileShape& ts, hipStream_t s);
hipError_t launch_batch(const BatchWork* dev_work, int* dev_counter, int grid, hipStream_t s);
hipError_t launch_debug_sample(const ReqParams& P, const float* pts, int n, float* out,
                               hipStream_t s);
int batch_grid_blocks(int device);

}  // namespace vr
