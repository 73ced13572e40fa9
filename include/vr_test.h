/*
 * vr_test.h — test hooks of libvr (not for production callers).
 */
#ifndef VR_TEST_H
#define VR_TEST_H

#include "vr.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Replace the context's serving backend with a CPU stand-in, so the serving
 * loop (queueing, memory-based admission, slots, batching, completion,
 * failures) can be tested without a GPU, also on a validation-only context.
 * A batch occupies its slot for (sum of its requests' rays) x ns_per_ray
 * nanoseconds; a batch holding a request of width fail_width completes as
 * failed (VR_ERR_DEVICE on each of its tickets).  Up to max_batch requests
 * per batch.  Each launch itself takes launch_ms milliseconds (0 .. 10000) of
 * the serving thread, as a slow enqueue would.  A finished ticket reports one
 * composited sample per ray.  VR_ERR_BUSY if the current serving loop has
 * tickets pending or running. */
vr_status vr_test_fake_backend(vr_ctx* ctx, int32_t slots, double ns_per_ray,
                               int32_t fail_width, int32_t max_batch, double launch_ms);

/* Fix the wave tile of batched launches (wave_w x wave_h pixels per wave,
 * wave_w * wave_h = 64), bypassing the autotuner; 0, 0 hands the choice back
 * to the autotuner. */
vr_status vr_test_batch_tile(vr_ctx* ctx, int32_t wave_w, int32_t wave_h);

/* The same for plain vr_render launches (default 8 x 8 pixels per wave, one
 * wave per block); 0, 0 restores the default. */
vr_status vr_test_plain_tile(vr_ctx* ctx, int32_t wave_w, int32_t wave_h);

/* on = 0 makes vr_render composite transparent samples in full instead of
 * leaving out their arithmetic (a sample whose taps are all below every
 * channel's transfer-function floor has opacity exactly 0) and makes every
 * render (plain, batched, served) walk every sample instead of jumping over
 * macro cells whose maxima are below those floors; on = 2 keeps the
 * per-sample test but walks every sample.  The output bits and sample counts
 * are the same either way.  on = 1 (the default) restores both skips. */
vr_status vr_test_clear_skip(vr_ctx* ctx, int32_t on);

/* on = 1 makes volumes created afterwards on this context use the
 * large-volume addressing (64-bit byte offsets, FP64 ray set-up and sample
 * positions) that volumes with an axis above 8192 voxels or a frame of 2^31
 * stored words or 4 GiB and more always use, so that path can be compared
 * with the oracle on small volumes (row pairs of 8-byte words included).
 * on = 0 (the default) restores the choice by size. */
vr_status vr_test_large_addressing(vr_ctx* ctx, int32_t on);

/* Macro cells of 2^shift sample corners per axis (2..5; 3, cells of 8, is the
 * default) for volumes created afterwards on this context, to measure other
 * cell sizes.  A volume whose cells are smaller than the default needs more
 * storage than vr_volume_storage_bytes reports (up to 8x the cell table per
 * halving); vr_create_volume returns VR_ERR_OUT_OF_MEMORY when the storage
 * is short.  Images are the same bit for bit at every size. */
vr_status vr_test_cell_shift(vr_ctx* ctx, int32_t shift);

/* *large = 1 when the volume renders through the large-volume addressing
 * (chosen at creation by size, or forced by vr_test_large_addressing), else
 * 0.  Pure host query. */
vr_status vr_test_volume_large(const vr_volume* vol, int32_t* large);

/* Transparent-sample threshold of one channel with floor lo and ceiling hi
 * on bits-bit data: the folded transfer-function constants the kernels use
 * (u = clamp(raw * scale + bias, 0, 1)) and the largest raw tap value tmax
 * for which every field value interpolated from taps <= tmax gives u = 0 in
 * the kernels' FP32 arithmetic (-1 if none).  Pure host computation. */
vr_status vr_test_transparent_max(float lo, float hi, int32_t bits, float* scale, float* bias,
                                  int32_t* tmax);

/* Position in a launch's tile order (super-tile by super-tile) that
 * hardware block b of a launch of nblocks single-wave blocks takes, for
 * b = 0 .. nblocks - 1, written to tiles[b] (host memory).  Pure host
 * computation: a permutation of 0 .. nblocks - 1. */
vr_status vr_test_block_map(int32_t nblocks, int32_t* tiles);

#ifdef __cplusplus
}
#endif

#endif /* VR_TEST_H */
