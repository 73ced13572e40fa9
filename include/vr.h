/*
 * vr.h — C ABI of the MI355X stereo multichannel volume ray caster.
 *
 * The library renders 5-D (x, y, z, t, channel) microscopy series that stay
 * resident in GPU memory, as in the paper's viewer: the whole image sequence
 * is downloaded to video memory once (Methods, acquisition paragraph; User
 * Interface, work-flow paragraph), each channel gets a colour, a visibility
 * toggle and a floor / ceiling / curve / alpha-multiplier transfer function
 * (User Interface, transfer-function paragraph), the volume is drawn for a
 * view and shown in stereo (User Interface; Results and Discussion), the user
 * steps through time points (Results and Discussion), and the CPU stays free
 * while the GPU renders (Abstract).
 *
 * Conventions for every entry point:
 *  - Every function returns a vr_status; no C++ exception crosses the ABI.
 *    On an error, vr_last_error() returns a message for the calling thread.
 *  - Argument errors are detected before anything is enqueued: a call that
 *    returns VR_ERR_INVALID_ARG has launched no GPU work and changed no state.
 *  - "device" pointers are HIP device addresses on the context's GPU, owned by
 *    the caller.  The library borrows them: volume storage until
 *    vr_destroy_volume, render inputs and outputs until the enqueued work has
 *    finished on the given stream (or the ticket is done / failed).
 *  - hip_stream arguments are hipStream_t values passed as void*; NULL is the
 *    default stream.  Rendering calls are asynchronous: they return after the
 *    kernels are enqueued.
 *  - Volume storage layout is private to the library (brick-major, channel-
 *    interleaved, zero halo); callers size it with vr_volume_storage_bytes.
 *
 * Threads: calls on distinct volumes may run concurrently; vr_submit and
 * vr_poll are thread-safe; calls on one volume must not race with
 * vr_destroy_volume of that volume.  Every call that enqueues GPU work does so
 * on the context's device, whatever device is current in the calling thread,
 * and restores the caller's current device before it returns.
 */
#ifndef VR_H
#define VR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VR_OK = 0,
    VR_ERR_INVALID_ARG = -1,   /* bad argument; nothing was enqueued            */
    VR_ERR_OUT_OF_MEMORY = -2, /* memory budget or storage size exceeded       */
    VR_ERR_NOT_FOUND = -3,     /* unknown ticket                                */
    VR_ERR_BUSY = -4,          /* queue full, or object referenced by tickets  */
    VR_ERR_DEVICE = -5,        /* a HIP runtime call failed                     */
    VR_ERR_UNSUPPORTED = -6    /* no GPU in this context, or not a gfx950 GPU   */
} vr_status;

typedef struct vr_ctx vr_ctx;       /* one per GPU; owns streams, events, tables */
typedef struct vr_volume vr_volume; /* one resident multichannel time series     */

typedef enum { VR_U8 = 1, VR_U16 = 2 } vr_dtype;
typedef enum { VR_FP32 = 0, VR_FP16 = 1 } vr_precision;
typedef enum { VR_ORTHO = 0, VR_PERSPECTIVE = 1 } vr_projection;

/* A 5-D series: frames x channels x nz x ny x nx voxels.  Voxel (i, j, k) of
 * a frame sits at world position origin + (i sx, j sy, k sz), with the
 * anisotropic spacing taken from the acquisition metadata (Methods, import
 * paragraph).  Normalised intensity is raw / (2^bits - 1): 255 for 8-bit data
 * as the transfer-function description states, 4095 for 12-bit, 65535 for
 * 16-bit. */
typedef struct {
    int32_t nx, ny, nz; /* >= 1 each, <= 16384.  A volume with an axis above
                           8192, or a frame of 2^31 stored words or 4 GiB
                           and more, is large: its kernels address taps with
                           64-bit offsets and step rays in FP64 (at most
                           2^32 bricks and 2^44 bytes per frame)             */
    int32_t channels;   /* 1..6                                              */
    int32_t frames;     /* >= 1 time points                                  */
    int32_t dtype;      /* vr_dtype                                          */
    int32_t bits;       /* VR_U8: 8.  VR_U16: 9..16                          */
    float spacing[3];   /* > 0, world units per voxel along x, y, z          */
    float origin[3];    /* world position of voxel (0, 0, 0)                 */
    int32_t brick[3];   /* brick edge per axis, each 4, 8, 16 or 32; all 0
                           selects the library default for the voxel word
                           (all channels of a voxel, 1, 2, 4, 8 or 16
                           bytes: channels rounded up to 1, 2, 4 or 8, times
                           the voxel width): 16 x 16 x 8 for 1-byte,
                           8 x 16 x 8 for 2- and 4-byte, 8 x 8 x 8 for 8-
                           and 16-byte words (4 x 16 x 8 for 8-byte words
                           of a large volume, see below).  Fixed at
                           creation.  With row_pairs the defaults are
                           16 x 16 x 16, 8 x 32 x 8 and 4 x 16 x 16 for 1-, 2-
                           and 4-byte words.                                  */
    int32_t row_pairs;  /* 0: default layout.  1: store each brick row next to
                           the row after it (voxel words of 1, 2 or 4 bytes:
                           up to 4 channels of uint8 or 2 of uint16; in a
                           large volume also 8-byte words, whose plane taps
                           then take two 16-byte loads; vr_create_volume
                           refuses 8-byte pairs otherwise), so the
                           four taps of
                           a sample in one brick plane are consecutive words:
                           a sample takes two 16-byte loads instead of four
                           8-byte ones (4-byte words), two 8-byte loads instead
                           of eight 2-byte ones (2-byte words) or four 2-byte
                           loads instead of eight 1-byte ones (1-byte words).
                           Storage: 2 (Bx + 1) By (Bz + 1) words per brick,
                           2.7x the raw voxels for 4 x 16 x 16 bricks against
                           1.3x for the default layout, before padding (see
                           vr_volume_storage_bytes).  Images are the same bit
                           for bit either way.                                */
} vr_volume_desc;

/* One channel's transfer function (User Interface, transfer-function
 * paragraph): u = clamp((x - lo) / (hi - lo), 0, 1) on normalised intensity
 * x; curve g = (1 - curve) u + curve u^2; channel alpha = alpha_mul * g;
 * channel colour = g * rgb.  A sample's alpha is the largest visible channel
 * alpha capped at 1, its colour the per-component sum of the visible
 * channels' colours capped at 1. */
typedef struct {
    float lo, hi;     /* 0 <= lo < hi <= 1                                   */
    float curve;      /* [-1, 1]; 0 = linear ramp                            */
    float alpha_mul;  /* [0, 2]; 1 = slider centre                           */
    float rgb[3];     /* [0, 1] each                                         */
    int32_t visible;  /* 0 hides the channel                                 */
} vr_transfer;

/* View.  Basis: f = normalise(forward), r = normalise(f x up), u = r x f.
 * Pixel (i, j) has its centre at (i + 1/2, j + 1/2), row 0 at the top;
 * screen coordinates sx = 2 (i + 1/2) / W - 1, sy = 1 - 2 (j + 1/2) / H.
 * Perspective: eye e = center + s (eye_separation / 2) r with s = -1 for the
 * left eye, +1 for the right and 0 for mono; both eyes look through one
 * screen at distance `convergence` (half-height convergence * tan(fov_y / 2),
 * aspect W / H); ray from e through the screen point, t >= 0.
 * Orthographic (mono only): rays along f from the screen rectangle of height
 * ortho_height centred on `center`, unbounded in t. */
typedef struct {
    int32_t projection;   /* vr_projection                                   */
    float center[3];
    float forward[3];     /* non-zero                                        */
    float up[3];          /* not parallel to forward                         */
    float fov_y;          /* radians in (0, pi), perspective                 */
    float ortho_height;   /* > 0, orthographic                               */
    float eye_separation; /* >= 0; 0 renders identical eyes                  */
    float convergence;    /* > 0, perspective                                */
} vr_camera;

/* Optional lighting: one global directional light (the viewer's lighting
 * check box, User Interface section).  Each channel's gradient g is the
 * central difference of its trilinear field over one voxel along each axis,
 * (x(p + e_a) - x(p - e_a)) / (2 spacing_a) in world units (the six face
 * points of the 3 x 3 x 3 neighbourhood of the sample); its normal is
 * n = -g / |g| and its colour contribution is scaled by
 * ambient + diffuse * max(0, n . l), l = direction / |direction| (ambient +
 * diffuse where g = 0).  Opacity, early termination and sample counts do not
 * change.  Under VR_FP16 the gradient is still taken in FP32.  A lit sample
 * reads six more trilinear samples. */
typedef struct {
    int32_t enabled;      /* 0 off (all-zero struct: unlit), 1 on             */
    float direction[3];   /* world space, towards the light; finite, non-zero */
    float ambient;        /* [0, 1]                                           */
    float diffuse;        /* [0, 1]                                           */
} vr_light;

/* One render request: a frame of a volume seen from a camera, one eye
 * (stereo = 0) or a left / right pair (stereo = 1, perspective only).
 * Samples sit at world distances t_enter + (k + 1/2) step along each ray
 * inside the box [-1, n] (index space) while t < t_exit; compositing is
 * front to back and stops after the first sample at which the accumulated
 * alpha reaches term_alpha (1 = no early stop).  The result is
 * rgb = C + (1 - A) bg_a bg_rgb, alpha = A + (1 - A) bg_a. */
typedef struct {
    vr_volume* vol;
    int32_t frame;          /* 0 .. frames - 1                                */
    vr_camera cam;
    int32_t width, height;  /* >= 0, <= 16384; a zero size renders nothing   */
    int32_t stereo;         /* 0 mono, 1 left + right                        */
    float step;             /* world units, > 0                               */
    float term_alpha;       /* (0, 1]                                         */
    float background[4];    /* rgb, a in [0, 1]                               */
    int32_t precision;      /* vr_precision: FP16 samples, FP32 compositing  */
    float* out_rgba;        /* device, [eyes][height][width][4] float32       */
    int32_t* out_samples;   /* device, [eyes][height][width] or NULL: samples
                               composited per pixel                          */
    vr_light light;         /* lighting; zero-initialised = off              */
} vr_render_req;

/* Ticket state reported by vr_poll.  Stamps are steady-clock nanoseconds,
 * 0 until reached: t_arrive_ns at vr_submit, t_admit_ns when the serving loop
 * admitted the request and enqueued its batch, t_done_ns when the loop saw
 * the batch finished, t_start_ns = t_done_ns minus the batch's span on the
 * device (HIP events recorded before and after its kernels), i.e. when the
 * device started the batch, on the same clock (set with t_done_ns). */
typedef struct {
    int32_t state;        /* 0 pending, 1 running, 2 done, 3 failed          */
    int32_t err;          /* vr_status of a failed ticket                    */
    uint64_t t_arrive_ns;
    uint64_t t_admit_ns;
    uint64_t t_start_ns;
    uint64_t t_done_ns;
    uint64_t samples;     /* samples composited over all pixels and eyes
                             (set when done): the nominal count, unchanged
                             by empty-space skipping and early termination
                             only stops counting                            */
    uint64_t rays;        /* pixels x eyes of the request                    */
} vr_ticket_info;

/* Open a context on HIP device `device` (the viewer's one graphics card that
 * holds the series: Methods, acquisition paragraph) with a memory budget for
 * volumes and in-flight served requests (0 = the device's free memory at open time minus
 * a 4 GiB reserve).  device = -1 opens a validation-only context with no GPU:
 * every call validates its arguments, then calls that need a GPU return
 * VR_ERR_UNSUPPORTED.  *out receives the context. */
vr_status vr_init(int32_t device, uint64_t mem_budget_bytes, vr_ctx** out);

/* Stop the serving thread and free the context (the end of a viewing
 * session; Abstract: the interactive loop).  VR_ERR_BUSY while served
 * tickets are pending or running, or volumes are still alive. */
vr_status vr_shutdown(vr_ctx* ctx);

/* Bytes of device storage a volume with this description needs (all
 * frames): bricks with their halo plus one macro-cell table per frame (the
 * whole sequence resident in GPU memory: Methods, acquisition paragraph).
 * Pure host computation. */
vr_status vr_volume_storage_bytes(const vr_volume_desc* desc, uint64_t* bytes);

/* Register a resident 5-D series (x, y, z, t, channel: Background; Methods,
 * acquisition and import paragraphs) in caller-owned device storage of at least
 * vr_volume_storage_bytes(desc) bytes, 256-byte aligned.  Its bytes count
 * against the context's budget (VR_ERR_OUT_OF_MEMORY when they do not fit).
 * All channels start with the default transfer function (lo 0, hi 1, curve 0,
 * alpha_mul 1, white, visible).  Contents are undefined until uploaded. */
vr_status vr_create_volume(vr_ctx* ctx, const vr_volume_desc* desc, void* dev_storage,
                           uint64_t storage_bytes, vr_volume** out);

/* Choose the voxel layout of a dataset by measurement (a project addition:
 * the brick layout is this library's; the paper keeps each time point as one
 * 3-D texture, User Interface section).  Every candidate layout (brick edges
 * and row pairs; all store the same voxels and give the same image bits)
 * whose storage for desc->frames frames stays within max_bytes (0: no limit)
 * is built from one frame, dev_frame [channels][nz][ny][nx] on the device
 * (as vr_upload_frame takes it), in scratch storage that this call allocates
 * and frees; the n_views requests are rendered from it, `reps` timed renders
 * each after two untimed ones, with the transfer functions tfs[0 ..
 * channels - 1] (the requests' vol and frame members are ignored; their
 * outputs receive the renders).  Of the layouts whose sum of per-view
 * median times is within 2 % of the least, the one with the smallest storage
 * is written into desc->brick and desc->row_pairs (the library default
 * layouts are tried first and kept on ties), its sum into *best_ms when
 * best_ms is not NULL.  Synchronous on hip_stream: blocks for about
 * 14 x n_views x (reps + 2) renders; call it at load time, before creating
 * the volume.  Counts each scratch volume against the context's budget while
 * it exists.  VR_ERR_OUT_OF_MEMORY when no candidate fits. */
vr_status vr_tune_layout(vr_ctx* ctx, vr_volume_desc* desc, const vr_transfer* tfs,
                         const void* dev_frame, const vr_render_req* views, int32_t n_views,
                         int32_t reps, uint64_t max_bytes, void* hip_stream, float* best_ms);

/* Copy one time point into the volume's storage on `hip_stream` (the
 * sequence is downloaded to video memory frame by frame: Methods,
 * acquisition paragraph; User Interface, work-flow paragraph): brick
 * relayout, then the frame's macro-cell maxima.  dev_src is a
 * device array [channels][nz][ny][nx] of uint8 or uint16 (the volume's
 * dtype), contiguous; values above 2^bits - 1 are clamped to it. */
vr_status vr_upload_frame(vr_volume* vol, int32_t frame, const void* dev_src,
                          void* hip_stream);

/* Playback of a series longer than device memory holds (Methods: the
 * sequences were buffered in host memory): the volume's frames serve as a
 * ring of slots and the series stays in host memory.  Enqueues the upload of
 * one frame [channels][nz][ny][nx] from host_src into slot `slot`:
 *   1. host_src -> dev_staging on copy_stream (an asynchronous DMA when
 *      host_src is pinned, e.g. hipHostMalloc or a pinned torch tensor;
 *      pageable memory works but the copy then blocks the caller);
 *   2. relayout dev_staging -> the slot, as vr_upload_frame, on a stream of
 *      the volume's own, after the copy and after the work already enqueued
 *      on render_stream (renders that may still read the slot).
 * With staging_bytes of two frames the calls alternate between the halves,
 * so that each copy follows the previous one without waiting for its
 * relayout; with one frame a copy waits for the previous relayout.
 * Before rendering from the slot, call vr_stream_ready on the render stream.
 * Playback with K slots: at step t, stream frame t + K - 1 into slot
 * (t + K - 1) mod K, then vr_stream_ready(slot t mod K) and render frame t:
 * the copy of the later frame overlaps the render of the earlier one.
 * dev_staging (device, >= channels * nz * ny * nx * bytes per voxel) is reused
 * safely by later calls on the same copy stream.  The two streams must
 * differ.  The ordering covers work on render_stream only (not served
 * tickets).  Calls on one volume serialise.  Returns after enqueueing. */
vr_status vr_stream_frame(vr_volume* vol, int32_t slot, const void* host_src,
                          void* dev_staging, uint64_t staging_bytes, void* copy_stream,
                          void* render_stream);

/* Make render_stream wait until the last vr_stream_frame into `slot` has
 * landed (no wait if the slot was never streamed).  Playback of buffered
 * sequences: Methods, acquisition paragraph; Results and Discussion, time
 * navigation. */
vr_status vr_stream_ready(vr_volume* vol, int32_t slot, void* render_stream);

/* Unregister a volume (closing a data set: User Interface, work-flow
 * paragraph) and return its bytes to the budget.  VR_ERR_BUSY while
 * a served ticket that reads it is pending or running. */
vr_status vr_destroy_volume(vr_volume* vol);

/* Set channel `channel`'s colour, visibility and transfer function (User
 * Interface, transfer-function paragraph: floor, ceiling, curve, alpha
 * multiplier per channel); copied.  Requests enqueued or
 * submitted earlier keep the function they were given. */
vr_status vr_set_transfer(vr_volume* vol, int32_t channel, const vr_transfer* tf);

/* Enqueue one request on `hip_stream` (one kernel launch per call): the
 * volume rendered for a view, in stereo if asked (User Interface, volume
 * rendering paragraph; Results and Discussion, stereo viewing).  Rays jump
 * over macro cells whose channel maxima are below every transfer-function
 * floor; images and sample counts equal those of a walk over every sample. */
vr_status vr_render(vr_ctx* ctx, const vr_render_req* req, void* hip_stream);

/* Enqueue n requests as one persistent, load-balanced launch (replayed from
 * a captured HIP graph) on `hip_stream`.  Every request's output is bitwise
 * identical to what vr_render gives for it alone.  n = 0 is a no-op.  Uses
 * the wave tile that vr_tune_batch (or the VR_AUTOTUNE_CACHE file) chose for
 * the batch's shape class, else the default; never tunes, never waits for
 * the device except when its staging tables are still being read by the
 * previous batch on the same stream.  (A project addition: the paper's
 * viewer renders one view at a time; User Interface section.) */
vr_status vr_render_batch(vr_ctx* ctx, const vr_render_req* reqs, int32_t n,
                          void* hip_stream);

/* Autotune the batched launch for this batch's shape class (the set of data
 * variants in it and the order of magnitude of its ray count): renders the
 * batch with every candidate wave tile, synchronously on `hip_stream`, into
 * the requests' own outputs (all candidates give the same bits), keeps the
 * fastest for later vr_render_batch calls and served batches of that class,
 * and appends it to the VR_AUTOTUNE_CACHE file when that variable names one.
 * Blocks the caller for about ten batch times: call it at load time.
 * *wave_w, *wave_h (either may be NULL) receive the chosen tile. */
vr_status vr_tune_batch(vr_ctx* ctx, const vr_render_req* reqs, int32_t n, void* hip_stream,
                        int32_t* wave_w, int32_t* wave_h);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * batched launch as vr_render_batch (bitwise the same outputs) that calls no
 * hipMalloc, hipFree or other allocating routine.  Its tables live in a
 * static device array of the library (about 256 KiB per GPU, held until the
 * process ends): n must not exceed 256 (VR_ERR_INVALID_ARG otherwise).  The
 * tables reach that array by asynchronous copies from pinned staging that
 * vr_init sets up; the variant kernels are launched directly (no graph).
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents: calls on one stream are ordered, calls that overlap on the device
 * (other streams or contexts of the same GPU) race and must be serialised by
 * the caller.  Uses the tuned wave tile of the batch's shape class, else the
 * default; never tunes. */
vr_status vr_render_batch_noalloc(vr_ctx* ctx, const vr_render_req* reqs, int32_t n,
                                  void* hip_stream);

/* Queue a request for the context's serving loop and return at once with a
 * ticket (the CPU stays free while the GPU renders: Abstract; interactive
 * navigation through time points: Results and Discussion).  The loop admits
 * queued requests when a slot is free and their output bytes fit in the
 * budget, batches the admitted ones, and overlaps batches on several
 * streams.  The request (and the volume's transfer
 * functions) are copied now.  VR_ERR_BUSY when 4096 tickets are pending. */
vr_status vr_submit(vr_ctx* ctx, const vr_render_req* req, uint64_t* ticket);

/* State, timestamps and composited samples of a served request.  Tickets
 * stay queryable until released.  VR_ERR_NOT_FOUND for an unknown or released
 * ticket. */
vr_status vr_poll(vr_ctx* ctx, uint64_t ticket, vr_ticket_info* info);

/* Forget a finished (done or failed) ticket (serving bookkeeping).
 * VR_ERR_BUSY if it is still pending or running; VR_ERR_NOT_FOUND if
 * unknown. */
vr_status vr_release(vr_ctx* ctx, uint64_t ticket);

/* Message of the calling thread's last error ("" after success).  Valid
 * until the thread's next vr_* call. */
const char* vr_last_error(void);

/* Test hook: trilinear field of every channel of `frame` (the 3-D texture
 * sampling of the User Interface section) at n index-space points
 * pts [n][3] (x, y, z), written to out [n][channels] float32 in raw
 * intensity units, through the renderer's own sampling code.  pts and out
 * are device pointers. */
vr_status vr_debug_sample(vr_volume* vol, int32_t frame, const float* pts, int32_t n,
                          float* out, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* VR_H */
