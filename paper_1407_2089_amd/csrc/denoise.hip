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
// Each lane filters one line and produces kRun consecutive outputs along it:
// kRun x kRun multiply-adds per kRun LDS reads.  Weights are padded with
// zeros to a multiple of kRun.
constexpr int kRun = 16;
constexpr int kPadTaps = (kMaxTaps + kRun - 1) / kRun * kRun;   // 144

// One axis of the low-pass, passed by value (kernel argument segment; the
// weights are read with scalar loads).
struct Axis1D {
    uint32_t w[kPadTaps];
    int32_t taps;      // odd, <= kMaxTaps
    int32_t padded;    // taps rounded up to a multiple of kRun
    int32_t shift;
};

struct Dims {
    int32_t nx, ny, nz;
};

// ------------------------------------------------------------- low-pass
// A block filters 64 lines over 64 outputs each (4 waves x kRun outputs).
// The lines' inputs, from 64 + 2r before clamping, sit in LDS as
// tile[lane * pitch + row] (pitch odd: the 64 lanes of a read hit distinct
// banks).  Rows past the loaded span are read only against zero weights.
constexpr int kOut = (kThreads / 64) * kRun;                // 64 outputs per line
// A wave's run reads rows wave * kRun .. wave * kRun + padded + kRun - 1
// (the last chunk's final row against no weight at all).
constexpr int kRows = kOut + kPadTaps;                      // at most 208 rows
static_assert(64 * (kRows | 1) * 4 <= 65536, "the largest tile fits a block's LDS");

// acc += w * x with both factors below 2^24 (weights <= 2^16, voxels <= 2^16):
// one full-rate v_mad_u32_u24 (left to itself the compiler pairs products
// into v_add3_u32, three instructions per two multiply-adds).
__device__ __forceinline__ void mad24(uint32_t& acc, uint32_t w, uint32_t x) {
    asm("v_mad_u32_u24 %0, %1, %2, %0" : "+v"(acc) : "s"(w), "v"(x));
}

__device__ __forceinline__ void filter_run(const uint32_t* __restrict__ t, const Axis1D& k,
                                           uint32_t (&acc)[kRun]) {
    uint32_t a[kRun], b[kRun];
#pragma unroll
    for (int m = 0; m < kRun; ++m) {
        acc[m] = 1u << (k.shift - 1);
        a[m] = t[m];
    }
    for (int q0 = 0; q0 < k.padded; q0 += kRun) {
#pragma unroll
        for (int m = 0; m < kRun; ++m) b[m] = t[q0 + kRun + m];
#pragma unroll
        for (int dq = 0; dq < kRun; ++dq) {
            const uint32_t w = k.w[q0 + dq];
#pragma unroll
            for (int m = 0; m < kRun; ++m) mad24(acc[m], w, m + dq < kRun ? a[m + dq] : b[m + dq - kRun]);
        }
#pragma unroll
        for (int m = 0; m < kRun; ++m) a[m] = b[m];
    }
}

// Generic line pass.  Line l of the block is (line0 + l); element i of a line
// sits at base(line) + i * step.  For the x pass the lines are rows (step 1);
// for y and z the lines are columns at consecutive x (step nx or nx ny).
// line_base maps a line index to its first element; n_lines lines exist.
template <typename T, int AXIS>
__global__ __launch_bounds__(kThreads) void lowpass_pass(const T* __restrict__ src,
                                                         T* __restrict__ dst, Dims d, Axis1D k,
                                                         int pitch) {
    // 64 lines of `pitch` words (dynamic LDS, sized by the host to the
    // rows this filter reads: more blocks per CU for shorter filters)
    extern __shared__ uint32_t tile[];
    const int tid = threadIdx.x;
    const int r = (k.taps - 1) >> 1;
    // line geometry: length na along the axis, stride sa; lines indexed by
    // (x, y, z) with the axis coordinate removed
    const int na = AXIS == 0 ? d.nx : AXIS == 1 ? d.ny : d.nz;
    const long long sa = AXIS == 0 ? 1 : AXIS == 1 ? (long long)d.nx : (long long)d.nx * d.ny;
    const int tiles_a = (na + kOut - 1) / kOut;
    int b = (int)blockIdx.x;
    const int ta = b % tiles_a;
    b /= tiles_a;
    const int a0 = ta * kOut;
    // 64 lines per block: for x, 64 consecutive rows (y, z); for y and z,
    // 64 consecutive x of one (z) or (y) plane line
    int lines_valid;
    long long base_of_line0, line_stride;
    if (AXIS == 0) {
        const int row0 = b * 64;
        lines_valid = min(64, d.ny * d.nz - row0);
        base_of_line0 = (long long)row0 * d.nx;
        line_stride = d.nx;
    } else {
        const int tiles_x = (d.nx + 63) / 64;
        const int x0 = (b % tiles_x) * 64;
        const int o = b / tiles_x;     // z for the y pass, y for the z pass
        lines_valid = min(64, d.nx - x0);
        base_of_line0 = AXIS == 1 ? (long long)o * d.nx * d.ny + x0 : (long long)o * d.nx + x0;
        line_stride = 1;
    }
    if (lines_valid <= 0) return;
    // load rows a0 - r .. a0 + kOut + r - 1 (clamped) of every valid line
    // (unrolled so that several loads are in flight per thread)
    const int span = kOut + 2 * r;
    if (AXIS == 0) {
        // a wave loads every fourth line, its lanes consecutive x of it, in
        // three 64-voxel chunks aligned to the tile (x from a0 - 64 to
        // a0 + 127, which holds a0 - r .. a0 + kOut + r - 1 for r <= 64):
        // each wave load is one aligned 128-byte run instead of straddling
        // two; the filter then starts at tile column 64 - r
        const int lane = tid & 63, wave = tid >> 6;
#pragma unroll 4
        for (int l = wave; l < 64; l += kThreads / 64) {
            if (l >= lines_valid) break;
            const long long lb = base_of_line0 + l * line_stride;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int a = min(max(a0 - 64 + lane + 64 * j, 0), na - 1);
                tile[l * pitch + lane + 64 * j] = src[lb + a];
            }
        }
    } else {
        // coalesced across lines: consecutive threads take consecutive x
#pragma unroll 8
        for (int i = tid; i < 64 * span; i += kThreads) {
            const int row = i >> 6, l = i & 63;
            if (l >= lines_valid) continue;
            const int a = min(max(a0 - r + row, 0), na - 1);
            tile[l * pitch + row] = src[base_of_line0 + l + a * sa];
        }
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    uint32_t acc[kRun];
    filter_run(tile + lane * pitch + (AXIS == 0 ? 64 - r : 0) + wave * kRun, k, acc);
    if (AXIS == 0) {
        // The lanes hold rows: stage the results in LDS and store them row
        // by row so that consecutive threads write consecutive x.
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kRun; ++m) tile[lane * pitch + wave * kRun + m] = acc[m] >> k.shift;
        __syncthreads();
        for (int i = tid; i < 64 * kOut; i += kThreads) {
            const int l = i / kOut, o = i - l * kOut;
            const int a = a0 + o;
            if (l < lines_valid && a < na)
                dst[base_of_line0 + l * line_stride + a] = (T)tile[l * pitch + o];
        }
        return;
    }
    if (lane >= lines_valid) return;
    const long long lb = base_of_line0 + lane * line_stride;
#pragma unroll
    for (int m = 0; m < kRun; ++m) {
        const int a = a0 + wave * kRun + m;
        if (a < na) dst[lb + a * sa] = (T)(acc[m] >> k.shift);
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

// The reductions run on a grid of at most kReduceBlocks blocks that stride
// over the volume, so that only that many atomic adds meet at one address.
constexpr int kReduceBlocks = 2048;
// The iteration writes one partial pair per block instead (no contention).
constexpr int kStepBlocks = 8192;

// Sum over the block of two unsigned 64-bit values into out[0], out[1]
// (a plain store from thread 0).
__device__ __forceinline__ void block_sum(unsigned long long a, unsigned long long b,
                                          unsigned long long* out) {
    __shared__ unsigned long long ta[kThreads], tb[kThreads];
    const int tid = threadIdx.x;
    ta[tid] = a;
    tb[tid] = b;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (tid < s) {
            ta[tid] += ta[tid + s];
            tb[tid] += tb[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        out[0] = ta[0];
        out[1] = tb[0];
    }
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

// Sum of |6-neighbour Laplacian| over interior voxels -> out[0].  Blocks
// stride over rows (y, z); threads over x.
template <typename T>
__global__ __launch_bounds__(kThreads) void laplacian_sum(const T* __restrict__ src, Dims d,
                                                          unsigned long long* out) {
    unsigned long long s = 0;
    const long long sy = d.nx, sz = (long long)d.nx * d.ny;
    const int rows = d.ny * d.nz;
    for (int r = blockIdx.x; r < rows; r += gridDim.x) {
        const int y = r % d.ny, z = r / d.ny;
        if (y == 0 || z == 0 || y == d.ny - 1 || z == d.nz - 1) continue;
        const T* row = src + (size_t)r * d.nx;
        for (int x = 1 + threadIdx.x; x < d.nx - 1; x += kThreads) {
            const int lap = (int)row[x - 1] + (int)row[x + 1] + (int)row[x - sy] +
                            (int)row[x + sy] + (int)row[x - sz] + (int)row[x + sz] -
                            6 * (int)row[x];
            s += (unsigned long long)(lap < 0 ? -lap : lap);
        }
    }
    block_add(s, 0, out);
}

__device__ __forceinline__ int sgn(int v) { return (v > 0) - (v < 0); }

// One iteration: out = clamp(cur + delta sgn(sum sgn(nb - cur)), 0, full);
// the block's sum of (out - orig)^2 and count of changed voxels go to
// partial[2 b], partial[2 b + 1] (plain stores; reduce_partials adds them).
// Blocks stride over rows (y, z); a thread takes kUnroll voxels of a row at
// a time and loads all their neighbours first (clamped into the row's
// planes, so every load is in bounds; a neighbour outside the volume is then
// left out of the sum), so that those loads are in flight together.
constexpr int kUnroll = 4;
template <typename T>
__global__ __launch_bounds__(kThreads) void mrf_step(const T* __restrict__ cur,
                                                     const T* __restrict__ orig,
                                                     T* __restrict__ nxt, Dims d, int delta,
                                                     int full,
                                                     unsigned long long* __restrict__ partial) {
    unsigned long long ss = 0, changed = 0;
    const int rows = d.ny * d.nz;
    for (int r = blockIdx.x; r < rows; r += gridDim.x) {
        const int y = r % d.ny, z = r / d.ny;
        const size_t base = (size_t)r * d.nx;
        const T* c0 = cur + base;
        const T* ym = c0 - (y > 0 ? d.nx : 0);
        const T* yp = c0 + (y < d.ny - 1 ? d.nx : 0);
        const size_t plane = (size_t)d.nx * d.ny;
        const T* zm = c0 - (z > 0 ? plane : 0);
        const T* zp = c0 + (z < d.nz - 1 ? plane : 0);
        for (int x0 = 0; x0 < d.nx; x0 += kThreads * kUnroll) {
            int c[kUnroll], l[kUnroll], rr[kUnroll], a[kUnroll], b[kUnroll], e[kUnroll],
                f[kUnroll], o[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int x = min(x0 + u * kThreads + (int)threadIdx.x, d.nx - 1);
                c[u] = c0[x];
                l[u] = c0[max(x - 1, 0)];
                rr[u] = c0[min(x + 1, d.nx - 1)];
                a[u] = ym[x];
                b[u] = yp[x];
                e[u] = zm[x];
                f[u] = zp[x];
                o[u] = orig[base + x];
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int x = x0 + u * kThreads + (int)threadIdx.x;
                if (x >= d.nx) continue;
                // a clamped neighbour equals the voxel itself: sgn(0) = 0
                const int s = sgn(l[u] - c[u]) + sgn(rr[u] - c[u]) + sgn(a[u] - c[u]) +
                              sgn(b[u] - c[u]) + sgn(e[u] - c[u]) + sgn(f[u] - c[u]);
                const int v = min(max(c[u] + delta * sgn(s), 0), full);
                nxt[base + x] = (T)v;
                const long long dv = (long long)v - (long long)o[u];
                ss += (unsigned long long)(dv * dv);
                changed += v != c[u];
            }
        }
    }
    block_sum(ss, changed, partial + 2 * blockIdx.x);
}

// For rows of a multiple of 4 voxels at 4-voxel-aligned addresses a lane
// takes 4 consecutive voxels with one 4-wide load per neighbour row (and one
// voxel to each side): a quarter of the load instructions of the one-voxel
// form (0.141 -> 0.129 ms per step on 1024 x 1024 x 64 when blocks still
// strode over rows; marching along z, below, keeps the z neighbours in
// registers).
template <typename T> struct Quad4 {
    typedef T V4 __attribute__((ext_vector_type(4)));
    V4 c, a, b, e, f, o;
    int left, right;
};

template <typename T>
__device__ __forceinline__ void quad_step(const Quad4<T>& q, T* __restrict__ out, int delta,
                                          int full, unsigned long long& ss,
                                          unsigned long long& changed) {
    typedef typename Quad4<T>::V4 V4;
    const int cc[4] = {(int)q.c.x, (int)q.c.y, (int)q.c.z, (int)q.c.w};
    const int ll[4] = {q.left, (int)q.c.x, (int)q.c.y, (int)q.c.z};
    const int rr[4] = {(int)q.c.y, (int)q.c.z, (int)q.c.w, q.right};
    const int aa[4] = {(int)q.a.x, (int)q.a.y, (int)q.a.z, (int)q.a.w};
    const int bb[4] = {(int)q.b.x, (int)q.b.y, (int)q.b.z, (int)q.b.w};
    const int ee[4] = {(int)q.e.x, (int)q.e.y, (int)q.e.z, (int)q.e.w};
    const int ff[4] = {(int)q.f.x, (int)q.f.y, (int)q.f.z, (int)q.f.w};
    const int oo[4] = {(int)q.o.x, (int)q.o.y, (int)q.o.z, (int)q.o.w};
    int v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int sum = sgn(ll[u] - cc[u]) + sgn(rr[u] - cc[u]) + sgn(aa[u] - cc[u]) +
                        sgn(bb[u] - cc[u]) + sgn(ee[u] - cc[u]) + sgn(ff[u] - cc[u]);
        v[u] = min(max(cc[u] + delta * sgn(sum), 0), full);
        const long long dv = (long long)v[u] - (long long)oo[u];
        ss += (unsigned long long)(dv * dv);
        changed += v[u] != cc[u];
    }
    V4 w;
    w.x = (T)v[0];
    w.y = (T)v[1];
    w.z = (T)v[2];
    w.w = (T)v[3];
    *reinterpret_cast<V4*>(out) = w;
}

// One iteration over 4-voxel quads, marching along z: a work item is (y, a chunk of
// kZChunk planes, kThreads quads of the row); a lane keeps the rows at z - 1,
// z and z + 1 of its 4 voxels in registers as it steps through the chunk, so
// each step loads one new row of cur (z + 1), the two y neighbours, orig and
// one voxel to each side (4 vector loads instead of 6; 0.129 -> 0.106 ms
// per step on 1024 x 1024 x 64).  Work items are taken grid-stride (the grid
// is capped like the row form's, so the partial sums fit their table).
constexpr int kZChunk = 16;
template <typename T>
__global__ __launch_bounds__(kThreads) void mrf_step_zm(const T* __restrict__ cur,
                                                        const T* __restrict__ orig,
                                                        T* __restrict__ nxt, Dims d, int delta,
                                                        int full,
                                                        unsigned long long* __restrict__ partial) {
    typedef typename Quad4<T>::V4 V4;
    unsigned long long ss = 0, changed = 0;
    const int nq = d.nx >> 2;
    const int qchunks = (nq + kThreads - 1) / kThreads;
    const int zchunks = (d.nz + kZChunk - 1) / kZChunk;
    const long long items = (long long)qchunks * d.ny * zchunks;
    const size_t plane = (size_t)d.nx * d.ny;
    for (long long it = blockIdx.x; it < items; it += gridDim.x) {
        const int qc = (int)(it % qchunks);
        const long long rest = it / qchunks;
        const int y = (int)(rest % d.ny);
        const int z0 = (int)(rest / d.ny) * kZChunk;
        const int z1 = min(z0 + kZChunk, d.nz);
        const int qx = qc * kThreads + (int)threadIdx.x;
        // the wave's lanes hold consecutive quads of one row: a lane's x - 1
        // and x + 4 neighbours are the adjacent lanes' edge voxels (DPP wave
        // shifts), loaded from memory only by the wave's first and last lane
        const int lane = (int)threadIdx.x & 63;
        if (qx >= nq) continue;
        const int x = 4 * qx;
        const size_t col = (size_t)y * d.nx + x;
        const int dym = y > 0 ? d.nx : 0, dyp = y < d.ny - 1 ? d.nx : 0;
        // a neighbour outside the volume is the voxel itself: sgn(0) = 0
        V4 c = *reinterpret_cast<const V4*>(cur + (size_t)z0 * plane + col);
        V4 prev = z0 > 0 ? *reinterpret_cast<const V4*>(cur + (size_t)(z0 - 1) * plane + col) : c;
        for (int z = z0; z < z1; ++z) {
            const T* c0 = cur + (size_t)z * plane + col;
            Quad4<T> q;
            q.c = c;
            q.e = prev;
            q.f = z < d.nz - 1 ? *reinterpret_cast<const V4*>(c0 + plane) : c;
            q.a = *reinterpret_cast<const V4*>(c0 - dym);
            q.b = *reinterpret_cast<const V4*>(c0 + dyp);
            q.o = *reinterpret_cast<const V4*>(orig + (size_t)z * plane + col);
            // wave_shr:1 gives lane i the value of lane i - 1, wave_shl:1 that
            // of lane i + 1 (lanes past the row's last quad are inactive and
            // their values unused: that quad's right neighbour is itself)
            const int from_prev = __builtin_amdgcn_update_dpp(0, (int)c.w, 0x138, 0xf, 0xf, false);
            const int from_next = __builtin_amdgcn_update_dpp(0, (int)c.x, 0x130, 0xf, 0xf, false);
            q.left = x == 0 ? (int)c.x : lane == 0 ? (int)c0[-1] : from_prev;
            q.right = x + 4 >= d.nx ? (int)c.w : lane == 63 ? (int)c0[4] : from_next;
            quad_step(q, nxt + (size_t)z * plane + col, delta, full, ss, changed);
            prev = c;
            c = q.f;
        }
    }
    block_sum(ss, changed, partial + 2 * blockIdx.x);
}

// sums[0..1] = the totals of n block partials (one block).
__global__ __launch_bounds__(kThreads) void reduce_partials(
    const unsigned long long* __restrict__ partial, int n, unsigned long long* sums) {
    unsigned long long a = 0, b = 0;
#pragma unroll 8
    for (int i = threadIdx.x; i < n; i += kThreads) {
        a += partial[2 * i];
        b += partial[2 * i + 1];
    }
    block_sum(a, b, sums);
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

// Workspace: two volumes, 256 bytes of sums, 64 KiB of value presence flags,
// 1 MiB for per-block partial sums.
constexpr uint64_t kPartialBytes = 1ull << 20;
static_assert(16ull * kStepBlocks <= kPartialBytes, "partials fit their table");
uint64_t workspace_need(const vr_grid& g) {
    return 2 * volume_bytes(g) + 256 + 65536 + kPartialBytes;
}

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
    out->padded = (taps + kRun - 1) / kRun * kRun;
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
    const long long tx = (g.nx + 63) / 64;
    const long long bx = (long long)((g.nx + kOut - 1) / kOut) * ((g.ny * g.nz + 63) / 64);
    const long long by = (long long)((g.ny + kOut - 1) / kOut) * tx * g.nz;
    const long long bz = (long long)((g.nz + kOut - 1) / kOut) * tx * g.ny;
    // LDS rows per line: y and z read rows 0 .. kOut + padded - 1; x loads
    // rows 0 .. 191 (aligned chunks) and reads from 64 - r on
    int pitch[3];
    for (int a = 0; a < 3; ++a) {
        const int r = (ax[a].taps - 1) >> 1;
        const int rows = a == 0 ? std::max(192, 128 - r + ax[a].padded) : kOut + ax[a].padded;
        pitch[a] = rows | 1;
    }
    const auto lds = [&](int a) { return (unsigned)(64 * pitch[a] * sizeof(uint32_t)); };
    hipLaunchKernelGGL((lowpass_pass<T, 0>), dim3((unsigned)bx), dim3(kThreads), lds(0), s, src,
                       t1, d, ax[0], pitch[0]);
    hipLaunchKernelGGL((lowpass_pass<T, 1>), dim3((unsigned)by), dim3(kThreads), lds(1), s,
                       (const T*)t1, t2, d, ax[1], pitch[1]);
    hipLaunchKernelGGL((lowpass_pass<T, 2>), dim3((unsigned)bz), dim3(kThreads), lds(2), s,
                       (const T*)t2, b, d, ax[2], pitch[2]);
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
    unsigned long long* partial = (unsigned long long*)(ws + 2 * vb + 256 + 65536);
    const int sblocks = std::min(g.ny * g.nz, kStepBlocks);
    const int blocks = (n + kThreads - 1) / kThreads;
    const int rblocks = std::min(g.ny * g.nz, kReduceBlocks);
    hipError_t e;
    hipLaunchKernelGGL(fill_u32, dim3(64), dim3(kThreads), 0, s, (uint32_t*)sums, 64, 0u);
    hipLaunchKernelGGL(fill_u32, dim3(64), dim3(kThreads), 0, s, (uint32_t*)presence, 16384, 0u);
    hipLaunchKernelGGL(mark_values<T>, dim3(blocks), dim3(kThreads), 0, s, src, presence, n);
    hipLaunchKernelGGL(laplacian_sum<T>, dim3(rblocks), dim3(kThreads), 0, s, src, d, sums);
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
    const long long zm_items = (long long)((g.nx / 4 + kThreads - 1) / kThreads) * g.ny *
                               ((g.nz + kZChunk - 1) / kZChunk);
    // One iteration: next = step(from) with its sums (squared distance to src,
    // voxels changed) in sums[2 slot], sums[2 slot + 1].
    auto step = [&](const T* from, T* next, int slot) {
        const uintptr_t al = 4 * sizeof(T) - 1;
        int nb = sblocks;
        if (g.nx % 4 == 0 && !(((uintptr_t)from | (uintptr_t)src | (uintptr_t)next) & al)) {
            nb = (int)std::min<long long>(zm_items, kStepBlocks);
            hipLaunchKernelGGL(mrf_step_zm<T>, dim3(nb), dim3(kThreads), 0, s, from, src, next,
                               d, delta, full, partial);
        } else {
            hipLaunchKernelGGL(mrf_step<T>, dim3(sblocks), dim3(kThreads), 0, s, from, src, next,
                               d, delta, full, partial);
        }
        hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kThreads), 0, s,
                           (const unsigned long long*)partial, nb, sums + 2 * slot);
    };
    if (delta > 0) {
        // Two iterations per round trip to the host: the second runs before
        // the first is judged, into a third buffer (the workspace's second
        // volume), so the last accepted image survives a rejected second
        // step.  The images kept and the counts are those of one iteration
        // per round trip.
        T* const bufs[3] = {dst, spare, (T*)(ws + vb)};
        bool stop = false;
        while (!stop && kept < max_iters) {
            T* out[2];
            int m = 0;
            for (T* b : bufs)
                if (b != cur && m < 2) out[m++] = b;
            const int run = max_iters - kept >= 2 ? 2 : 1;
            step(cur, out[0], 0);
            if (run == 2) step(out[0], out[1], 1);
            if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "mrf step launch");
            unsigned long long hs[4] = {0, 0, 0, 0};
            if ((e = hipMemcpyAsync(hs, sums, sizeof(unsigned long long) * 2 * run,
                                    hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return hip_fail(e, "mrf step sums");
            for (int q = 0; q < run; ++q) {
                const unsigned long long ss = hs[2 * q], changed = hs[2 * q + 1];
                if (changed == 0 || !((double)ss <= sigma * sigma * (double)n)) {
                    stop = true;  // fixed point, or past the noise bound
                    break;
                }
                cur = out[q];
                kept += 1;
                kept_ss = ss;
            }
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

vr_status vr_gaussian_weights(double sigma, int32_t shift, int32_t radius, uint32_t* w,
                              int32_t capacity, int32_t* taps) {
    if (!(sigma > 0.0) || !std::isfinite(sigma))
        return fail(VR_ERR_INVALID_ARG, "sigma must be finite and > 0");
    if (shift < 1 || shift > 16) return fail(VR_ERR_INVALID_ARG, "shift must be 1..16");
    if (radius < -1 || radius > 64) return fail(VR_ERR_INVALID_ARG, "radius must be -1..64");
    if (!w || !taps) return fail(VR_ERR_INVALID_ARG, "NULL output");
    const int r = radius >= 0 ? radius : (int)std::min(64.0, std::ceil(3.0 * sigma));
    const int n = 2 * r + 1;
    if (capacity < n) return fail(VR_ERR_INVALID_ARG, "%d weights need capacity %d", n, n);
    // Samples of exp(-k^2 / (2 sigma^2)) at k = -r .. r, scaled to 2^shift
    // and rounded to nearest (ties to even); the rounding remainder goes to
    // the centre tap so that the sum is exactly 2^shift.
    double g[129], tot = 0.0;
    for (int i = 0; i < n; ++i) {
        const double k = (double)(i - r);
        g[i] = std::exp(-(k * k) / (2.0 * sigma * sigma));
        tot += g[i];
    }
    const double scale = std::ldexp(1.0, shift);
    int64_t sum = 0;
    for (int i = 0; i < n; ++i) {
        w[i] = (uint32_t)std::nearbyint(scale * g[i] / tot);
        sum += w[i];
    }
    const int64_t centre = (int64_t)w[r] + ((int64_t)1 << shift) - sum;
    if (centre < 0)
        return fail(VR_ERR_INVALID_ARG,
                    "rounded weights exceed 2^%d at sigma %g and radius %d: take a larger shift",
                    shift, sigma, r);
    w[r] = (uint32_t)centre;
    *taps = n;
    return ok();
}

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
