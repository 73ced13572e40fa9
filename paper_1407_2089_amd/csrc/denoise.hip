// Pre-render denoisers of one channel (Methods, Background Noise Removal):
// the separable integer low-pass, background subtraction and 3x3x3 median of
// eq. (1), and the sign-diffusion iteration of eqs. (2)-(3) with its
// Laplacian noise estimate.  Every voxel result is exact integer arithmetic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/vr_denoise.h"
#include "lib.h"

namespace vr {
namespace {

constexpr int kMaxTaps = 129;
constexpr int kThreads = 256;

// One axis of the low-pass, passed by value (kernel argument segment).
struct Axis1D {
    uint32_t w[kMaxTaps];
    int32_t taps;
    int32_t shift;
};

struct Dims {
    int32_t nx, ny, nz;
};

// ------------------------------------------------------------- low-pass
// Pass along x: a block filters 256 consecutive voxels of one row from an LDS
// copy of the row segment and its clamped halo.
template <typename T>
__global__ __launch_bounds__(kThreads) void lowpass_x(const T* __restrict__ src,
                                                      T* __restrict__ dst, Dims d, Axis1D k) {
    __shared__ uint32_t tile[kThreads + kMaxTaps - 1];
    __shared__ uint32_t w[kMaxTaps];
    const int tid = threadIdx.x;
    const int r = (k.taps - 1) >> 1;
    const int tiles_x = (d.nx + kThreads - 1) / kThreads;
    const int row = (int)blockIdx.x / tiles_x;
    const int x0 = ((int)blockIdx.x - row * tiles_x) * kThreads;
    const size_t base = (size_t)row * d.nx;
    for (int i = tid; i < k.taps; i += kThreads) w[i] = k.w[i];
    for (int i = tid; i < kThreads + 2 * r; i += kThreads) {
        const int x = min(max(x0 - r + i, 0), d.nx - 1);
        tile[i] = src[base + x];
    }
    __syncthreads();
    const int x = x0 + tid;
    if (x >= d.nx) return;
    uint32_t acc = 1u << (k.shift - 1);
    for (int j = 0; j < k.taps; ++j) acc += __umul24(w[j], tile[tid + j]);
    dst[base + x] = (T)(acc >> k.shift);
}

// Pass along y or z (stride sa between neighbours on the axis): a block
// filters 64 outputs along the axis for 64 consecutive x, from an LDS copy of
// the (64 + 2r) x 64 input patch (rows clamped at the axis ends).
constexpr int kLine = 64;
template <typename T>
__global__ __launch_bounds__(kThreads) void lowpass_strided(const T* __restrict__ src,
                                                            T* __restrict__ dst, Dims d, int na,
                                                            int no, long long sa, long long so,
                                                            Axis1D k) {
    __shared__ uint32_t tile[(kLine + kMaxTaps - 1) * 64];
    __shared__ uint32_t w[kMaxTaps];
    const int tid = threadIdx.x;
    const int r = (k.taps - 1) >> 1;
    const int tiles_x = (d.nx + 63) / 64;
    const int tiles_a = (na + kLine - 1) / kLine;
    int b = (int)blockIdx.x;
    const int tx = b % tiles_x;
    b /= tiles_x;
    const int ta = b % tiles_a;
    const int o = b / tiles_a;
    if (o >= no) return;
    const int x0 = tx * 64, a0 = ta * kLine;
    for (int i = tid; i < k.taps; i += kThreads) w[i] = k.w[i];
    const int rows = kLine + 2 * r;
    for (int i = tid; i < rows * 64; i += kThreads) {
        const int row = i >> 6, lane = i & 63;
        const int a = min(max(a0 - r + row, 0), na - 1);
        const int x = x0 + lane;
        tile[i] = x < d.nx ? (uint32_t)src[(size_t)(o * so + a * sa) + x] : 0u;
    }
    __syncthreads();
    const int lane = tid & 63, grp = tid >> 6;
    const int x = x0 + lane;
    if (x >= d.nx) return;
    for (int j = grp; j < kLine; j += kThreads / 64) {
        const int a = a0 + j;
        if (a >= na) break;
        uint32_t acc = 1u << (k.shift - 1);
        for (int q = 0; q < k.taps; ++q) acc += __umul24(w[q], tile[(j + q) * 64 + lane]);
        dst[(size_t)(o * so + a * sa) + x] = (T)(acc >> k.shift);
    }
}

// ------------------------------------------------------- median of 27
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void cas(u16x2& a, u16x2& b) {
    const u16x2 lo = __builtin_elementwise_min(a, b);
    b = __builtin_elementwise_max(a, b);
    a = lo;
}

// Moves the smallest of a[S .. S + M - 1] to a[S] and the largest to
// a[S + M - 1], keeping the others in between (pairs first, then one chain
// over each half; an odd middle element joins both chains).
template <int S, int M>
__device__ __forceinline__ void extremes(u16x2 (&a)[27]) {
#pragma unroll
    for (int i = 0; i < M / 2; ++i) cas(a[S + i], a[S + M - 1 - i]);
#pragma unroll
    for (int i = 1; i < (M + 1) / 2; ++i) cas(a[S], a[S + i]);
#pragma unroll
    for (int i = 1; i < (M + 1) / 2; ++i) cas(a[S + M - 1 - i], a[S + M - 1]);
}

// Forgetful selection: of 15 values the smallest and largest cannot be the
// median of 27 (14 others lie on one side), so drop both, take the next
// value, and repeat; the last value left is the 14th smallest.  Every index
// is a compile-time constant (registers only).  Two voxels per lane pair.
template <int S, int M, int Next>
__device__ __forceinline__ u16x2 forget(u16x2 (&a)[27], const u16x2 (&e)[27]) {
    extremes<S, M>(a);
    if constexpr (M - 2 == 1 && Next == 27) {
        return a[S + 1];
    } else {
        a[S + M - 1] = e[Next];
        return forget<S + 1, M - 1, Next + 1>(a, e);
    }
}

__device__ __forceinline__ u16x2 median27(const u16x2 (&e)[27]) {
    u16x2 a[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) a[i] = e[i];
    return forget<0, 15, 15>(a, e);
}

// D = max(L - B, 0) on a (64 + 2) x (8 + 2) x (4 + 2) patch (clamped), then
// pairs P[z][y][x] = D[x] | D[x + 1] << 16 so that a lane takes the windows
// of two x-neighbours with one LDS read per element.
constexpr int kMX = 64, kMY = 8, kMZ = 4;
template <typename T>
__global__ __launch_bounds__(kThreads) void subtract_median(const T* __restrict__ L,
                                                            const T* __restrict__ B,
                                                            T* __restrict__ dst, Dims d) {
    constexpr int TX = kMX + 2, TY = kMY + 2, TZ = kMZ + 2;
    constexpr int PX = kMX + 1;
    __shared__ uint16_t D[TZ * TY * TX];
    __shared__ uint32_t P[TZ * TY * PX];
    const int tid = threadIdx.x;
    const int tiles_x = (d.nx + kMX - 1) / kMX, tiles_y = (d.ny + kMY - 1) / kMY;
    int b = (int)blockIdx.x;
    const int x0 = (b % tiles_x) * kMX;
    b /= tiles_x;
    const int y0 = (b % tiles_y) * kMY;
    const int z0 = (b / tiles_y) * kMZ;
    for (int i = tid; i < TZ * TY * TX; i += kThreads) {
        const int tx = i % TX, ty = (i / TX) % TY, tz = i / (TX * TY);
        const int x = min(max(x0 - 1 + tx, 0), d.nx - 1);
        const int y = min(max(y0 - 1 + ty, 0), d.ny - 1);
        const int z = min(max(z0 - 1 + tz, 0), d.nz - 1);
        const size_t v = ((size_t)z * d.ny + y) * d.nx + x;
        const int l = (int)L[v], bb = (int)B[v];
        D[i] = (uint16_t)(l > bb ? l - bb : 0);
    }
    __syncthreads();
    for (int i = tid; i < TZ * TY * PX; i += kThreads) {
        const int px = i % PX, row = i / PX;
        P[i] = (uint32_t)D[row * TX + px] | (uint32_t)D[row * TX + px + 1] << 16;
    }
    __syncthreads();
    const int lx = tid % (kMX / 2), ly = tid / (kMX / 2);
    const int x = x0 + 2 * lx, y = y0 + ly;
    if (x >= d.nx || y >= d.ny) return;
#pragma unroll 1
    for (int lz = 0; lz < kMZ; ++lz) {
        const int z = z0 + lz;
        if (z >= d.nz) break;
        u16x2 e[27];
#pragma unroll
        for (int q = 0; q < 27; ++q) {
            const int dz = q / 9, dy = (q / 3) % 3, dx = q % 3;
            e[q] = __builtin_bit_cast(u16x2, P[((lz + dz) * TY + ly + dy) * PX + 2 * lx + dx]);
        }
        const u16x2 m = median27(e);
        const size_t v = ((size_t)z * d.ny + y) * d.nx + x;
        dst[v] = (T)m.x;
        if (x + 1 < d.nx) dst[v + 1] = (T)m.y;
    }
}

// ------------------------------------------------------ MRF iteration
__global__ void fill_u32(uint32_t* p, int n, uint32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// presence[v] = 1 for every value v in the volume (identical stores race
// harmlessly).
template <typename T>
__global__ void mark_values(const T* __restrict__ src, uint8_t* __restrict__ presence, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) presence[src[i]] = 1;
}

// Sum over the block of two unsigned 64-bit values, then one atomic add each.
__device__ __forceinline__ void block_add(unsigned long long a, unsigned long long b,
                                          unsigned long long* out) {
    __shared__ unsigned long long sa[kThreads], sb[kThreads];
    const int tid = threadIdx.x;
    sa[tid] = a;
    sb[tid] = b;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (tid < s) {
            sa[tid] += sa[tid + s];
            sb[tid] += sb[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (sa[0]) atomicAdd(&out[0], sa[0]);
        if (sb[0]) atomicAdd(&out[1], sb[0]);
    }
}

__device__ __forceinline__ void coords(int i, const Dims& d, int& x, int& y, int& z) {
    x = i % d.nx;
    const int r = i / d.nx;
    y = r % d.ny;
    z = r / d.ny;
}

// Sum of |6-neighbour Laplacian| over interior voxels -> out[0].
template <typename T>
__global__ __launch_bounds__(kThreads) void laplacian_sum(const T* __restrict__ src, Dims d, int n,
                                                          unsigned long long* out) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    unsigned long long s = 0;
    if (i < n) {
        int x, y, z;
        coords(i, d, x, y, z);
        if (x > 0 && y > 0 && z > 0 && x < d.nx - 1 && y < d.ny - 1 && z < d.nz - 1) {
            const long long sx = 1, sy = d.nx, sz = (long long)d.nx * d.ny;
            const int lap = (int)src[i - sx] + (int)src[i + sx] + (int)src[i - sy] +
                            (int)src[i + sy] + (int)src[i - sz] + (int)src[i + sz] -
                            6 * (int)src[i];
            s = (unsigned long long)(lap < 0 ? -lap : lap);
        }
    }
    block_add(s, 0, out);
}

__device__ __forceinline__ int sgn(int v) { return (v > 0) - (v < 0); }

// One iteration: out = clamp(cur + delta sgn(sum sgn(nb - cur)), 0, full);
// out[0] += sum (out - orig)^2, out[1] += voxels that changed.
template <typename T>
__global__ __launch_bounds__(kThreads) void mrf_step(const T* __restrict__ cur,
                                                     const T* __restrict__ orig,
                                                     T* __restrict__ nxt, Dims d, int n,
                                                     int delta, int full,
                                                     unsigned long long* sums) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    unsigned long long ss = 0, changed = 0;
    if (i < n) {
        int x, y, z;
        coords(i, d, x, y, z);
        const long long sy = d.nx, sz = (long long)d.nx * d.ny;
        const int c = (int)cur[i];
        int s = 0;
        if (x > 0) s += sgn((int)cur[i - 1] - c);
        if (x < d.nx - 1) s += sgn((int)cur[i + 1] - c);
        if (y > 0) s += sgn((int)cur[i - sy] - c);
        if (y < d.ny - 1) s += sgn((int)cur[i + sy] - c);
        if (z > 0) s += sgn((int)cur[i - sz] - c);
        if (z < d.nz - 1) s += sgn((int)cur[i + sz] - c);
        const int v = min(max(c + delta * sgn(s), 0), full);
        nxt[i] = (T)v;
        const long long dv = (long long)v - (long long)orig[i];
        ss = (unsigned long long)(dv * dv);
        changed = v != c;
    }
    block_add(ss, changed, sums);
}

// --------------------------------------------------------------- host
uint64_t align256(uint64_t b) { return (b + 255) & ~uint64_t(255); }

vr_status check_grid(const vr_grid* g) {
    if (!g) return fail(VR_ERR_INVALID_ARG, "grid is NULL");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1)
        return fail(VR_ERR_INVALID_ARG, "grid sides must be >= 1");
    if ((long long)g->nx * g->ny * g->nz >= (1LL << 31))
        return fail(VR_ERR_INVALID_ARG, "grid holds 2^31 voxels or more");
    if (g->dtype == VR_U8) {
        if (g->bits != 8) return fail(VR_ERR_INVALID_ARG, "uint8 volumes have 8 bits");
    } else if (g->dtype == VR_U16) {
        if (g->bits < 9 || g->bits > 16) return fail(VR_ERR_INVALID_ARG, "uint16 bits 9..16");
    } else {
        return fail(VR_ERR_INVALID_ARG, "dtype %d is unknown", g->dtype);
    }
    return VR_OK;
}

uint64_t raw_bytes(const vr_grid& g) {
    return (uint64_t)g.nx * g.ny * g.nz * (g.dtype == VR_U16 ? 2 : 1);
}

uint64_t volume_bytes(const vr_grid& g) { return align256(raw_bytes(g)); }

uint64_t workspace_need(const vr_grid& g) { return 2 * volume_bytes(g) + 256 + 65536; }

vr_status check_ctx(const vr_ctx* ctx) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    return VR_OK;
}

vr_status check_axis(const uint32_t* w, int taps, int shift, const char* name, Axis1D* out) {
    if (!w) return fail(VR_ERR_INVALID_ARG, "%s weights are NULL", name);
    if (taps < 1 || taps > kMaxTaps || taps % 2 == 0)
        return fail(VR_ERR_INVALID_ARG, "%s taps must be odd, 1..%d", name, kMaxTaps);
    uint64_t sum = 0;
    for (int i = 0; i < taps; ++i) sum += w[i];
    if (sum != (1ull << shift))
        return fail(VR_ERR_INVALID_ARG, "%s weights sum to %llu, not 2^%d", name,
                    (unsigned long long)sum, shift);
    std::memset(out, 0, sizeof *out);
    for (int i = 0; i < taps; ++i) out->w[i] = w[i];
    out->taps = taps;
    out->shift = shift;
    return VR_OK;
}

template <typename T>
hipError_t enqueue_background(const vr_grid& g, const Axis1D (&ax)[3], const T* src, T* dst,
                              T* bg, uint8_t* ws, hipStream_t s) {
    const Dims d{g.nx, g.ny, g.nz};
    T* t1 = (T*)ws;
    T* t2 = (T*)(ws + volume_bytes(g));
    T* b = bg ? bg : t1;
    const int tiles_x256 = (g.nx + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(lowpass_x<T>, dim3((unsigned)((long long)tiles_x256 * g.ny * g.nz)),
                       dim3(kThreads), 0, s, src, t1, d, ax[0]);
    const int tiles_x64 = (g.nx + 63) / 64;
    const long long plane = (long long)g.nx * g.ny;
    // y: axis stride nx, outer index z (stride nx ny)
    const int ty = (g.ny + kLine - 1) / kLine;
    hipLaunchKernelGGL(lowpass_strided<T>, dim3((unsigned)((long long)tiles_x64 * ty * g.nz)),
                       dim3(kThreads), 0, s, (const T*)t1, t2, d, g.ny, g.nz, (long long)g.nx,
                       plane, ax[1]);
    // z: axis stride nx ny, outer index y (stride nx)
    const int tz = (g.nz + kLine - 1) / kLine;
    hipLaunchKernelGGL(lowpass_strided<T>, dim3((unsigned)((long long)tiles_x64 * tz * g.ny)),
                       dim3(kThreads), 0, s, (const T*)t2, b, d, g.nz, g.ny, plane,
                       (long long)g.nx, ax[2]);
    const long long blocks = (long long)((g.nx + kMX - 1) / kMX) * ((g.ny + kMY - 1) / kMY) *
                             ((g.nz + kMZ - 1) / kMZ);
    hipLaunchKernelGGL(subtract_median<T>, dim3((unsigned)blocks), dim3(kThreads), 0, s, src,
                       (const T*)b, dst, d);
    return hipGetLastError();
}

template <typename T>
vr_status run_mrf(const vr_grid& g, int max_iters, const T* src, T* dst, uint8_t* ws,
                  hipStream_t s, vr_mrf_info* info) {
    const Dims d{g.nx, g.ny, g.nz};
    const int n = g.nx * g.ny * g.nz;
    const uint64_t vb = volume_bytes(g);
    T* spare = (T*)ws;
    unsigned long long* sums = (unsigned long long*)(ws + 2 * vb);
    uint8_t* presence = ws + 2 * vb + 256;
    const int blocks = (n + kThreads - 1) / kThreads;
    hipError_t e;
    hipLaunchKernelGGL(fill_u32, dim3(64), dim3(kThreads), 0, s, (uint32_t*)sums, 64, 0u);
    hipLaunchKernelGGL(fill_u32, dim3(64), dim3(kThreads), 0, s, (uint32_t*)presence, 16384, 0u);
    hipLaunchKernelGGL(mark_values<T>, dim3(blocks), dim3(kThreads), 0, s, src, presence, n);
    hipLaunchKernelGGL(laplacian_sum<T>, dim3(blocks), dim3(kThreads), 0, s, src, d, n, sums);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "denoise launch");
    std::vector<uint8_t> seen(65536);
    unsigned long long h[2] = {0, 0};
    if ((e = hipMemcpyAsync(seen.data(), presence, 65536, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(h, sums, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "denoise statistics");
    int delta = 0, last = -1;
    for (int v = 0; v < 65536; ++v) {
        if (!seen[v]) continue;
        if (last >= 0 && (delta == 0 || v - last < delta)) delta = v - last;
        last = v;
    }
    const long long interior = (long long)std::max(g.nx - 2, 0) * std::max(g.ny - 2, 0) *
                               std::max(g.nz - 2, 0);
    const double sigma = interior > 0 ? std::sqrt(M_PI / 2.0) * (double)h[0] /
                                            ((double)interior * std::sqrt(42.0))
                                      : 0.0;
    const int full = (1 << g.bits) - 1;
    const T* cur = src;
    int kept = 0;
    unsigned long long kept_ss = 0;
    if (delta > 0) {
        while (kept < max_iters) {
            T* out = (kept % 2 == 0) ? dst : spare;
            hipLaunchKernelGGL(fill_u32, dim3(1), dim3(64), 0, s, (uint32_t*)sums, 4, 0u);
            hipLaunchKernelGGL(mrf_step<T>, dim3(blocks), dim3(kThreads), 0, s, cur, src, out,
                               d, n, delta, full, sums);
            if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "mrf step launch");
            if ((e = hipMemcpyAsync(h, sums, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return hip_fail(e, "mrf step sums");
            if (h[1] == 0) break;  // fixed point
            if (!((double)h[0] <= sigma * sigma * (double)n)) break;
            cur = out;
            kept += 1;
            kept_ss = h[0];
        }
    }
    if (cur != dst) {
        if ((e = hipMemcpyAsync(dst, cur, (size_t)n * sizeof(T), hipMemcpyDeviceToDevice, s)) !=
            hipSuccess)
            return hip_fail(e, "mrf result copy");
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "mrf finish");
    if (info) {
        info->iterations = kept;
        info->delta = delta;
        info->sigma = sigma;
        info->rms = std::sqrt((double)kept_ss / (double)n);
    }
    return ok();
}

bool overlap(const void* a, const void* b, uint64_t na, uint64_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

}  // namespace
}  // namespace vr

using namespace vr;

extern "C" {

vr_status vr_denoise_workspace_bytes(const vr_grid* grid, uint64_t* bytes) {
    vr_status st = check_grid(grid);
    if (st != VR_OK) return st;
    if (!bytes) return fail(VR_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = workspace_need(*grid);
    return ok();
}

vr_status vr_remove_background(vr_ctx* ctx, const vr_grid* grid, const vr_lowpass* lp,
                               const void* src, void* dst, void* background, void* workspace,
                               uint64_t workspace_bytes, void* hip_stream) {
    vr_status st = check_ctx(ctx);
    if (st == VR_OK) st = check_grid(grid);
    if (st != VR_OK) return st;
    if (!lp) return fail(VR_ERR_INVALID_ARG, "low-pass is NULL");
    if (lp->shift < 1 || lp->shift > 16) return fail(VR_ERR_INVALID_ARG, "shift must be 1..16");
    Axis1D ax[3];
    const char* names[3] = {"x", "y", "z"};
    for (int a = 0; a < 3; ++a) {
        st = check_axis(lp->w[a], lp->taps[a], lp->shift, names[a], &ax[a]);
        if (st != VR_OK) return st;
    }
    if (!src || !dst || !workspace) return fail(VR_ERR_INVALID_ARG, "NULL device pointer");
    if (workspace_bytes < workspace_need(*grid))
        return fail(VR_ERR_INVALID_ARG, "workspace of %llu bytes, %llu needed",
                    (unsigned long long)workspace_bytes,
                    (unsigned long long)workspace_need(*grid));
    const uint64_t vb = raw_bytes(*grid);
    if (overlap(src, dst, vb, vb) || overlap(src, workspace, vb, workspace_bytes) ||
        overlap(dst, workspace, vb, workspace_bytes) ||
        (background && (overlap(background, src, vb, vb) || overlap(background, dst, vb, vb) ||
                        overlap(background, workspace, vb, workspace_bytes))))
        return fail(VR_ERR_INVALID_ARG, "volumes and workspace overlap");
    if (ctx->device < 0) return fail(VR_ERR_UNSUPPORTED, "validation-only context");
    DeviceGuard dg(ctx->device);
    hipError_t e;
    if (grid->dtype == VR_U8)
        e = enqueue_background<uint8_t>(*grid, ax, (const uint8_t*)src, (uint8_t*)dst,
                                        (uint8_t*)background, (uint8_t*)workspace,
                                        (hipStream_t)hip_stream);
    else
        e = enqueue_background<uint16_t>(*grid, ax, (const uint16_t*)src, (uint16_t*)dst,
                                         (uint16_t*)background, (uint8_t*)workspace,
                                         (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "background removal launch");
    return ok();
}

vr_status vr_mrf_denoise(vr_ctx* ctx, const vr_grid* grid, int32_t max_iters, const void* src,
                         void* dst, void* workspace, uint64_t workspace_bytes, void* hip_stream,
                         vr_mrf_info* info) {
    vr_status st = check_ctx(ctx);
    if (st == VR_OK) st = check_grid(grid);
    if (st != VR_OK) return st;
    if (max_iters < 0) return fail(VR_ERR_INVALID_ARG, "max_iters < 0");
    if (!src || !dst || !workspace) return fail(VR_ERR_INVALID_ARG, "NULL device pointer");
    if (workspace_bytes < workspace_need(*grid))
        return fail(VR_ERR_INVALID_ARG, "workspace of %llu bytes, %llu needed",
                    (unsigned long long)workspace_bytes,
                    (unsigned long long)workspace_need(*grid));
    const uint64_t vb = raw_bytes(*grid);
    if (overlap(src, dst, vb, vb) || overlap(src, workspace, vb, workspace_bytes) ||
        overlap(dst, workspace, vb, workspace_bytes))
        return fail(VR_ERR_INVALID_ARG, "volumes and workspace overlap");
    if (ctx->device < 0) return fail(VR_ERR_UNSUPPORTED, "validation-only context");
    DeviceGuard dg(ctx->device);
    if (grid->dtype == VR_U8)
        return run_mrf<uint8_t>(*grid, max_iters, (const uint8_t*)src, (uint8_t*)dst,
                                (uint8_t*)workspace, (hipStream_t)hip_stream, info);
    return run_mrf<uint16_t>(*grid, max_iters, (const uint16_t*)src, (uint16_t*)dst,
                             (uint8_t*)workspace, (hipStream_t)hip_stream, info);
}

}  // extern "C"
