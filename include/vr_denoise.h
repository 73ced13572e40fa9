/* Pre-render denoising of one channel of one frame (Methods, Background Noise
 * Removal): the stem-cell channel's background subtraction and median of
 * eq. (1), and the vasculature channel's sign-diffusion iteration of
 * eqs. (2)-(3).  Each channel of the paper's series is denoised on its own
 * before it is uploaded for rendering.
 *
 * Volumes are device arrays [nz][ny][nx] of uint8 (VR_U8) or uint16 (VR_U16),
 * contiguous, owned by the caller.  Every result is an integer computed in
 * exact integer arithmetic, so it is the same bit for bit on any device; the
 * noise estimate and the stopping test are IEEE double on the host.
 *
 * Errors: VR_ERR_INVALID_ARG for a bad description, kernel, pointer or a
 * workspace smaller than vr_denoise_workspace_bytes; VR_ERR_UNSUPPORTED on a
 * validation-only context (after validation); VR_ERR_DEVICE when HIP fails. */
#ifndef VR_DENOISE_H
#define VR_DENOISE_H

#include "vr.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One channel of one frame. */
typedef struct {
    int32_t nx, ny, nz;  /* >= 1 each; nx * ny * nz < 2^31                   */
    int32_t dtype;       /* VR_U8 or VR_U16                                  */
    int32_t bits;        /* VR_U8: 8.  VR_U16: 9..16.  Values lie in
                            [0, 2^bits - 1] (the iteration clamps to it)     */
} vr_grid;

/* Separable low-pass of eq. (1) (a Gaussian in the paper): per axis an odd
 * number of non-negative integer weights w[0 .. taps - 1] (taps <= 129, centre
 * tap r = (taps - 1) / 2) summing to exactly 2^shift, shift in [1, 16].  Each
 * pass computes out[i] = (sum_k w[k] v[clamp(i + k - r)] + 2^(shift - 1))
 * >> shift along its axis, edges clamped, rounded back to the voxel type;
 * passes run along x, then y, then z.  Host pointers, read during the call. */
typedef struct {
    const uint32_t* w[3];  /* x, y, z                                        */
    int32_t taps[3];
    int32_t shift;
} vr_lowpass;

/* Integer weights of the low-pass of eq. (1) as a quantised Gaussian of
 * width sigma voxels (the paper names a Gaussian filter without weights):
 * w[i] = round(2^shift g_i / sum_j g_j), g_i = exp(-k^2 / (2 sigma^2)) at
 * k = i - r for i = 0 .. 2r (ties to even), with the rounding remainder
 * added to the centre tap w[r] so that the weights sum to exactly 2^shift.
 * radius r: 0..64, or -1 for min(64, ceil(3 sigma)).  w (host, capacity
 * entries) receives the 2r + 1 weights and *taps their number.  Pure host
 * computation.  VR_ERR_INVALID_ARG for sigma <= 0 or not finite, shift
 * outside 1..16, capacity < 2r + 1, or when the rounded side weights alone
 * exceed 2^shift (a wide kernel at a small shift). */
vr_status vr_gaussian_weights(double sigma, int32_t shift, int32_t radius, uint32_t* w,
                              int32_t capacity, int32_t* taps);

/* Device workspace bytes that the two calls below need for `grid`: two
 * volumes of the voxel type (each rounded up to 256 bytes) plus
 * 1 MiB + 64 KiB + 256 bytes of tables. */
vr_status vr_denoise_workspace_bytes(const vr_grid* grid, uint64_t* bytes);

/* Stem-cell channel, eq. (1): B = the low-pass of src, then
 * dst = median3(max(src - B, 0)) with a 3 x 3 x 3 median (the 14th smallest
 * of 27, edges clamped).  `background` (device, may be NULL) receives B.
 * src, dst and background must not overlap each other or the workspace.
 * Enqueued on hip_stream; returns after the launches. */
vr_status vr_remove_background(vr_ctx* ctx, const vr_grid* grid, const vr_lowpass* lp,
                               const void* src, void* dst, void* background, void* workspace,
                               uint64_t workspace_bytes, void* hip_stream);

/* Result of vr_mrf_denoise. */
typedef struct {
    int32_t iterations;  /* images kept after the original (0: dst = src)     */
    int32_t delta;       /* step: smallest gap between distinct values (0 if
                            the volume is constant: nothing is done)          */
    double sigma;        /* noise estimate from the 6-neighbour Laplacian:
                            sqrt(pi / 2) sum|lap| / (N sqrt(42)) over the N
                            interior voxels (0 if a side is < 3 voxels)      */
    double rms;          /* RMS distance of dst to src                        */
} vr_mrf_info;

/* Vasculature channel, eqs. (2)-(3): each iteration moves every voxel by
 * delta in the direction sgn(sum over its in-volume face neighbours of
 * sgn(neighbour - voxel)), clamped to [0, 2^bits - 1]; the result is the last
 * image whose RMS distance to src is at most sigma (tested as
 * sum d^2 <= sigma^2 N in double), stopping early at a fixed point or after
 * max_iters (>= 0) iterations.  Runs on hip_stream and waits on it after
 * every second iteration (the stopping test reads device sums; the second
 * iteration of a pair runs before the first is judged, into the workspace,
 * and is dropped if the first stops); returns when dst holds the result.
 * src and dst must not overlap each other or the workspace. */
vr_status vr_mrf_denoise(vr_ctx* ctx, const vr_grid* grid, int32_t max_iters, const void* src,
                         void* dst, void* workspace, uint64_t workspace_bytes, void* hip_stream,
                         vr_mrf_info* info);

#ifdef __cplusplus
}
#endif

#endif /* VR_DENOISE_H */
