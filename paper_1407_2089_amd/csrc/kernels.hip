// HIP kernels for gfx950: frame relayout into bricks, the plain per-request
// render launch, the batched render launch, and the sampling test hook.
// Host-side launchers at the bottom are the only entry points the library's
// C++ code calls; the block-map test hook sits after them.
#include <hip/hip_runtime.h>

#include <array>
#include <utility>

#include "../../include/vr_test.h"
#include "kernels.h"
#include "march.h"

namespace vr {

// ------------------------------------------------------------- relayout
// Scatter form: one thread per stored position (sx, sy, sz) of the frame, stored
// coordinate s = voxel index + 1 over [0, nb B] per axis: it reads the
// voxel's channels from the linear [C][Z][Y][X] source (zero outside the
// grid; consecutive threads read consecutive x), clamps them to the declared
// bit depth, packs them into one word and writes every copy of that word.
// Per axis a position is local s mod B of brick s / B (if that brick
// exists) and, when s is a nonzero multiple of B, also the high-side halo
// (local B) of brick s / B - 1; in the row-pair layout a local row ly is the
// first word of pair row ly (ly < By) and the second of pair row ly - 1
// (ly >= 1).  Each stored word of the frame is written by exactly one
// thread.  Grid: x over positions, y and z one block row per position.
template <int C, bool U16> __device__ __forceinline__ typename WordT<C, U16>::T pack_word(
    const uint32_t (&ch)[kMaxChannels]) {
    using T = typename WordT<C, U16>::T;
    if constexpr (!U16) {
        if constexpr (C == 1) return (T)ch[0];
        else if constexpr (C == 2) return (T)(ch[0] | (ch[1] << 8));
        else if constexpr (C <= 4) return (T)(ch[0] | (ch[1] << 8) | (ch[2] << 16) | (ch[3] << 24));
        else return make_uint2(ch[0] | (ch[1] << 8) | (ch[2] << 16) | (ch[3] << 24),
                               ch[4] | (ch[5] << 8));
    } else {
        if constexpr (C == 1) return (T)ch[0];
        else if constexpr (C == 2) return (T)(ch[0] | (ch[1] << 16));
        else if constexpr (C <= 4) return make_uint2(ch[0] | (ch[1] << 16), ch[2] | (ch[3] << 16));
        else return make_uint4(ch[0] | (ch[1] << 16), ch[2] | (ch[3] << 16),
                               ch[4] | (ch[5] << 16), 0u);
    }
}

// Copies of stored position s along one axis: (brick, local) pairs.
struct AxisCopies {
    uint32_t brick[2], local[2];
    int n;
};
__device__ __forceinline__ AxisCopies axis_copies(uint32_t s, int shift, uint32_t nb) {
    AxisCopies a;
    a.n = 0;
    const uint32_t b = s >> shift, l = s & ((1u << shift) - 1u);
    if (b < nb) {
        a.brick[a.n] = b;
        a.local[a.n] = l;
        ++a.n;
    }
    if (l == 0 && b > 0) {
        a.brick[a.n] = b - 1;
        a.local[a.n] = 1u << shift;
        ++a.n;
    }
    return a;
}

// Gather form, for bricks at least 8 voxels wide: one thread per stored word
// (grid-stride), which finds its voxel and gathers the channels; a wave
// writes 64 consecutive words and reads runs of Bx + 1 voxels.  In the
// row-pair layout a word's brick-local row is its pair's row plus the word's
// parity.  (Narrower bricks take the scatter form below: runs of 5 voxels
// made the gather's reads 2.9x slower on a 4 x 16 x 8 brick frame, while
// the scatter's short write runs cost it 1.4x on 8 x 16 x 8 bricks of
// 4-byte words.)
template <int C, bool U16>
__global__ __launch_bounds__(256) void relayout_gather_kernel(BrickGeom g, const void* __restrict__ src,
                                                        uint8_t* __restrict__ dst, uint32_t maxval,
                                                        uint64_t total_words) {
    using T = typename WordT<C, U16>::T;
    using S = typename std::conditional<U16, uint16_t, uint8_t>::type;
    const S* in = reinterpret_cast<const S*>(src);
    T* out = reinterpret_cast<T*>(dst);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < total_words; w += stride) {
        const uint32_t brick = (uint32_t)(w / (uint32_t)g.brick);
        const uint32_t rem = (uint32_t)(w - (uint64_t)brick * (uint32_t)g.brick);
        const uint32_t lz = rem / (uint32_t)g.plane;
        const uint32_t r2 = rem - lz * (uint32_t)g.plane;
        const uint32_t lr = r2 / (uint32_t)g.row;
        const uint32_t e = r2 - lr * (uint32_t)g.row;
        const uint32_t ly = g.pairs ? lr + (e & 1u) : lr;
        const uint32_t lx = g.pairs ? e >> 1 : e;
        const uint32_t bx = brick % (uint32_t)g.nb[0];
        const uint32_t byz = brick / (uint32_t)g.nb[0];
        const uint32_t by = byz % (uint32_t)g.nb[1];
        const uint32_t bz = byz / (uint32_t)g.nb[1];
        // voxel index = stored coordinate - 1
        const int i = (int)((bx << g.shift[0]) + lx) - 1;
        const int j = (int)((by << g.shift[1]) + ly) - 1;
        const int k = (int)((bz << g.shift[2]) + lz) - 1;
        uint32_t ch[kMaxChannels] = {};
        if (i >= 0 && j >= 0 && k >= 0 && i < g.n[0] && j < g.n[1] && k < g.n[2]) {
            const size_t plane = (size_t)g.n[0] * g.n[1];
            const size_t vol = plane * g.n[2];
            const size_t base = (size_t)k * plane + (size_t)j * g.n[0] + i;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                uint32_t v = in[(size_t)c * vol + base];
                ch[c] = v > maxval ? maxval : v;
            }
        }
        const T word = pack_word<C, U16>(ch);
        out[w] = word;
    }
}


constexpr int kRelayoutThreads = 128;

template <int C, bool U16>
__global__ __launch_bounds__(kRelayoutThreads) void relayout_scatter_kernel(
    BrickGeom g, const void* __restrict__ src, uint8_t* __restrict__ dst, uint32_t maxval) {
    using T = typename WordT<C, U16>::T;
    using S = typename std::conditional<U16, uint16_t, uint8_t>::type;
    const uint32_t sx = blockIdx.x * kRelayoutThreads + threadIdx.x;
    const uint32_t sy = blockIdx.y, sz = blockIdx.z;
    if (sx > ((uint32_t)g.nb[0] << g.shift[0])) return;
    const int i = (int)sx - 1, j = (int)sy - 1, k = (int)sz - 1;
    uint32_t ch[kMaxChannels] = {};
    if (i >= 0 && j >= 0 && k >= 0 && i < g.n[0] && j < g.n[1] && k < g.n[2]) {
        const S* in = reinterpret_cast<const S*>(src);
        const size_t plane = (size_t)g.n[0] * g.n[1];
        const size_t vol = plane * g.n[2];
        const size_t base = (size_t)k * plane + (size_t)j * g.n[0] + i;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const uint32_t v = in[(size_t)c * vol + base];
            ch[c] = v > maxval ? maxval : v;
        }
    }
    const T word = pack_word<C, U16>(ch);
    T* out = reinterpret_cast<T*>(dst);
    const AxisCopies X = axis_copies(sx, g.shift[0], (uint32_t)g.nb[0]);
    const AxisCopies Y = axis_copies(sy, g.shift[1], (uint32_t)g.nb[1]);
    const AxisCopies Z = axis_copies(sz, g.shift[2], (uint32_t)g.nb[2]);
    const uint32_t By = 1u << g.shift[1];
    for (int zc = 0; zc < Z.n; ++zc) {
        for (int yc = 0; yc < Y.n; ++yc) {
            const uint32_t ly = Y.local[yc];
            // (row, parity) slots of local row ly within the brick plane
            uint32_t rows[2], par[2];
            int nr = 0;
            if (!g.pairs) {
                rows[0] = ly;
                par[0] = 0;
                nr = 1;
            } else {
                if (ly < By) {
                    rows[nr] = ly;
                    par[nr] = 0;
                    ++nr;
                }
                if (ly >= 1) {
                    rows[nr] = ly - 1;
                    par[nr] = 1;
                    ++nr;
                }
            }
            for (int xc = 0; xc < X.n; ++xc) {
                const uint64_t brick =
                    ((uint64_t)Z.brick[zc] * (uint32_t)g.nb[1] + Y.brick[yc]) * (uint32_t)g.nb[0] +
                    X.brick[xc];
                for (int r = 0; r < nr; ++r) {
                    const uint32_t e = g.pairs ? 2u * X.local[xc] + par[r] : X.local[xc];
                    const uint32_t local = Z.local[zc] * (uint32_t)g.plane + rows[r] * (uint32_t)g.row + e;
                    out[brick * (uint32_t)g.brick + local] = word;
                }
            }
        }
    }
}

// ------------------------------------------------------- macro-cell maxima
// The frame's macro-cell table: per cell and channel, the largest clamped
// voxel value over stored coordinates [c M, c M + M] per axis, that is voxel
// indices [c M - 1, c M + M - 1] clipped to the grid (the zero padding never
// raises a maximum), packed like a voxel word.  Built strip by strip: a block
// takes one (y, z) row of cells (cy, cz) and sweeps x in tiles of kCellTile
// voxels.  Its threads first reduce, per channel, the strip's source rows
// (up to 9 x 9) into column maxima in LDS, four consecutive columns per
// thread with one 4- or 8-byte load per row (ALIGNED: rows of a multiple of
// 4 voxels from an 8-byte aligned source), else from two or three aligned
// dword loads; then one thread per cell takes the maximum of its 9 columns
// (x from 8 cx - 1 to 8 cx + 7; columns outside the grid hold 0).  Column
// xt - 1 of a tile is the previous tile's last.
constexpr int kCellTile = 1024;
template <int C, bool U16, bool ALIGNED>
__global__ __launch_bounds__(256) void cellmax_strip_kernel(BrickGeom g,
                                                            const void* __restrict__ src,
                                                            uint8_t* __restrict__ frame,
                                                            uint32_t maxval) {
    using T = typename WordT<C, U16>::T;
    using S = typename std::conditional<U16, uint16_t, uint8_t>::type;
    __shared__ uint32_t col[C][kCellTile + 1];  // col[c][1 + i]: column xt + i
    const S* in = reinterpret_cast<const S*>(src);
    const int cy = (int)blockIdx.x, cz = (int)blockIdx.y;
    const int M = 1 << g.cshift;
    const int y0 = max(cy * M - 1, 0), y1 = min(cy * M + M - 1, g.n[1] - 1);
    const int z0 = max(cz * M - 1, 0), z1 = min(cz * M + M - 1, g.n[2] - 1);
    const size_t plane = (size_t)g.n[0] * g.n[1];
    const size_t vol = plane * g.n[2];
    T* cells = reinterpret_cast<T*>(frame + g.cell_off) + ((size_t)cz * g.nc[1] + cy) * g.nc[0];
    const int xend = g.nc[0] * M;  // the last cell starts at 8 (nc0 - 1) <= n
    const int tid = (int)threadIdx.x;
    const uint8_t* src_end = reinterpret_cast<const uint8_t*>(in + (size_t)C * vol);
    if (tid < C) col[tid][0] = 0;  // column -1
    for (int xt = 0; xt < xend; xt += kCellTile) {
        // four columns x = xt + 4 t .. xt + 4 t + 3 per thread (kCellTile = 4 x 256)
        const int x = xt + 4 * tid;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            uint32_t m[4] = {0, 0, 0, 0};
            if (x + 3 < g.n[0]) {
                for (int k = z0; k <= z1; ++k) {
                    for (int j = y0; j <= y1; ++j) {
                        const S* p = in + (size_t)c * vol + (size_t)k * plane + (size_t)j * g.n[0] + x;
                        // the four voxels' bytes: one 4- or 8-byte load where the
                        // group is aligned to its size; else from the aligned dwords
                        // around it (a row need not start on a 4-byte boundary); near
                        // the end of the source, where those dwords would reach past
                        // it, voxel by voxel
                        const uintptr_t b = (uintptr_t)p;
                        const uint32_t* a = reinterpret_cast<const uint32_t*>(b & ~(uintptr_t)3);
                        const uint32_t o = (uint32_t)(b & 3u);
                        uint32_t v[4], lo = 0, hi = 0;
                        bool packed = true;
                        if constexpr (ALIGNED) {
                            if constexpr (U16) {
                                const uint2 q = *reinterpret_cast<const uint2*>(p);
                                lo = q.x;
                                hi = q.y;
                            } else {
                                lo = *reinterpret_cast<const uint32_t*>(p);
                            }
                        } else if ((const uint8_t*)a + (U16 ? 12 : 8) <= src_end) {
                            const uint32_t d1 = a[1];
                            lo = __builtin_amdgcn_alignbyte(d1, a[0], o);
                            if constexpr (U16) hi = __builtin_amdgcn_alignbyte(a[2], d1, o);
                        } else {
                            packed = false;
#pragma unroll
                            for (int u = 0; u < 4; ++u) v[u] = (uint32_t)p[u];
                        }
                        if (packed) {
                            if constexpr (U16) {
                                v[0] = lo & 0xffffu;
                                v[1] = lo >> 16;
                                v[2] = hi & 0xffffu;
                                v[3] = hi >> 16;
                            } else {
                                v[0] = lo & 0xffu;
                                v[1] = (lo >> 8) & 0xffu;
                                v[2] = (lo >> 16) & 0xffu;
                                v[3] = lo >> 24;
                            }
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) m[u] = max(m[u], v[u]);
                    }
                }
            } else if (x < g.n[0]) {  // the row's ragged end
                for (int k = z0; k <= z1; ++k) {
                    const S* p = in + (size_t)c * vol + (size_t)k * plane;
                    for (int j = y0; j <= y1; ++j)
                        for (int u = 0; u < 4 && x + u < g.n[0]; ++u)
                            m[u] = max(m[u], (uint32_t)p[(size_t)j * g.n[0] + x + u]);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) col[c][1 + 4 * tid + u] = m[u];
        }
        __syncthreads();
        const int c_lo = xt >> g.cshift, c_hi = min(g.nc[0], (xt + kCellTile) >> g.cshift);
        for (int cx = c_lo + tid; cx < c_hi; cx += (int)blockDim.x) {
            uint32_t ch[kMaxChannels] = {};
            const int i0 = cx * M - xt;  // col index of x = 8 cx - 1
#pragma unroll
            for (int c = 0; c < C; ++c) {
                uint32_t m = 0;
                for (int i = i0; i <= i0 + M; ++i) m = max(m, col[c][i]);
                ch[c] = m > maxval ? maxval : m;
            }
            cells[cx] = pack_word<C, U16>(ch);
        }
        __syncthreads();
        if (tid < C) col[tid][0] = col[tid][kCellTile];  // column xt + kCellTile - 1
        __syncthreads();
    }
}

// ------------------------------------------------------------ plain render
// Grid: one single-wave block per (eye, wave_w x wave_h pixel tile).  Blocks
// of one wave let the dispatcher refill a SIMD as soon as any wave's rays
// end (measured: 4-wave blocks were 6 % slower on the top view and up to
// 24 % on grazing views).  kClear = false composites transparent samples in
// full (same output bits; kept to test and time the transparent-sample skip).
// Tiles of an eye run super-tile by super-tile (row-major over super-tiles of
// kSuperW x kSuperH tiles, row-major inside each); the grid covers whole
// super-tiles, and lanes past the image edge are invalid.  Unlit, a stereo
// pair's two eyes take consecutive blocks per tile (the eyes' rays of one
// tile meet nearly the same bricks, so the second often finds them in L2;
// measured 2 % faster on a 36 GB montage, 1.4 % on a 230 MB frame).  kLit:
// lit by the request's directional light; lit launches render the eyes one
// after the other (4 % faster than interleaved, measured).
// Lit kernels whose registers fit 6 waves per SIMD (80 VGPRs) without
// spilling, as compiled here; the others keep the compiler's choice.  On the
// realistic 2-channel 16-bit frame the cap gives 0.198 ms against 0.208 ms
// at the natural 88 VGPRs (5 waves).
constexpr int lit_min_waves(int v, bool lit, bool clear) {
    if (!lit || !clear) return 1;
    // variant_index(channels, u16, fp16, row pairs, large)
    switch (v) {
        case variant_index(2, true, false, false, false):
        case variant_index(2, false, false, true, false):
        case variant_index(2, true, false, true, false):
        case variant_index(2, false, true, true, false):
            return 6;
        default:
            return 1;
    }
}

template <int V, bool kClear, bool kLit>
__global__ __launch_bounds__(kWave)
__attribute__((amdgpu_waves_per_eu(lit_min_waves(V, kLit, kClear)))) void render_kernel(
    ReqParams P, TileShape ts, int supers_x, int per_eye) {
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    int eye, t;
    if constexpr (kLit) {
        eye = b / per_eye;
        t = b - eye * per_eye;
    } else {
        eye = P.eyes == 2 ? (b & 1) : 0;
        t = P.eyes == 2 ? (b >> 1) : b;
    }
    int tx, ty;
    tile_at(t, supers_x, tx, ty);
    const int lane = threadIdx.x;
    const int px = tx * ts.wave_w + lane % ts.wave_w;
    const int py = ty * ts.wave_h + lane / ts.wave_w;
    const bool valid = px < P.width && py < P.height;
    render_pixel<V, kClear, kLit>(P, eye, valid ? px : 0, valid ? py : 0, valid);
}

// -------------------------------------------------------- batched render
// Work items are (request, eye, wave tile) triples numbered request by
// request in the order the host laid the requests out (most expensive
// first); prefix[q] is the first item of request q.  Block b takes items
// b, b + grid, b + 2 grid, ... of its variant's group (after the XCD remap)
// and leaves past the group's last item; there is no shared counter.
__device__ __forceinline__ int find_req(const int32_t* __restrict__ prefix, int n, int item) {
    int lo = 0, hi = n - 1;  // largest q with prefix[q] <= item
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int V>
__device__ __forceinline__ void batch_tile(const ReqParams& P, const TileShape& ts, int local) {
    // A request's items are its tiles in super-tile order, both eyes of a
    // stereo tile in consecutive items.
    const int supers_x = (int)supers_across(P.width, ts);
    const int eye = P.eyes == 2 ? (local & 1) : 0;
    int tx, ty;
    tile_at(P.eyes == 2 ? (local >> 1) : local, supers_x, tx, ty);
    const int lane = threadIdx.x & (kWave - 1);
    const int px = tx * ts.wave_w + lane % ts.wave_w;
    const int py = ty * ts.wave_h + lane / ts.wave_w;
    const bool valid = px < P.width && py < P.height;
    render_pixel<V>(P, eye, valid ? px : 0, valid ? py : 0, valid);
}

template <int V>
__global__ __launch_bounds__(kWave) void batch_kernel(const BatchWork* __restrict__ work,
                                                      const ReqParams* __restrict__ reqs,
                                                      const int32_t* __restrict__ prefix) {
    const BatchGroup grp = work->group[V];
    const TileShape ts = work->tile;
    const int stride = (int)gridDim.x;
    // The item is uniform over the block (one wave), so the request's
    // descriptor (read-only, not aliased: restrict arguments) is read with
    // scalar loads into scalar registers.
    for (int item = xcd_remap((int)blockIdx.x, stride); item < grp.n_items; item += stride) {
        const int q = __builtin_amdgcn_readfirstlane(
            grp.first + find_req(prefix + grp.first, grp.n_req, item));
        const int local = __builtin_amdgcn_readfirstlane(item - prefix[q]);
        batch_tile<V>(reqs[q], ts, local);
    }
}

typedef void (*batch_fn)(const BatchWork*, const ReqParams*, const int32_t*);

// Kernel tables indexed by variant, null where the variant does not exist.
template <int V> constexpr batch_fn batch_entry() {
    if constexpr (variant_exists(V) && !variant_large(V)) return batch_kernel<V>;
    else return nullptr;
}
template <int... V>
constexpr std::array<batch_fn, kBatchVariants> batch_table(std::integer_sequence<int, V...>) {
    return {{batch_entry<V>()...}};
}
static const std::array<batch_fn, kBatchVariants> kBatch =
    batch_table(std::make_integer_sequence<int, kBatchVariants>{});

// ------------------------------------------------------------ test hook
template <int V>
__global__ __launch_bounds__(256) void debug_sample_kernel(ReqParams P, const float* __restrict__ pts,
                                                           int n, float* __restrict__ out) {
    constexpr int C = Variant<V>::C;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[C];
    if constexpr (Variant<V>::LARGE) {
        using T = typename WordT<C, Variant<V>::U16>::T;
        const SamplerL S = make_sampler_large(P);
        interpolate<C, Variant<V>::U16, Variant<V>::F16>(
            fetch<T, Variant<V>::PAIRS>(P.g, S, (double)pts[3 * i] + 1.0, (double)pts[3 * i + 1] + 1.0,
                            (double)pts[3 * i + 2] + 1.0), x);
    } else {
        const Sampler S = make_sampler(P.vox, P.g);
        sample<C, Variant<V>::U16, Variant<V>::F16, Variant<V>::PAIRS>(P.g, S, pts[3 * i],
                                                                        pts[3 * i + 1],
                                                                        pts[3 * i + 2], x);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) out[(size_t)i * C + c] = x[c];
}

// ------------------------------------------------------------- launchers

hipError_t launch_relayout(const BrickGeom& g, int channels, bool u16, int bits,
                           const void* src, uint8_t* dst, hipStream_t s) {
    // stored positions 0 .. nb B per axis
    const uint32_t NX = ((uint32_t)g.nb[0] << g.shift[0]) + 1u;
    const uint32_t NY = ((uint32_t)g.nb[1] << g.shift[1]) + 1u;
    const uint32_t NZ = ((uint32_t)g.nb[2] << g.shift[2]) + 1u;
    if (NY > 65535u || NZ > 65535u) return hipErrorInvalidValue;
    const uint32_t maxval = (1u << bits) - 1u;
    const dim3 grid((NX + kRelayoutThreads - 1) / kRelayoutThreads, NY, NZ);
    const uint64_t words = (uint64_t)g.nb[0] * g.nb[1] * g.nb[2] * (uint64_t)g.brick;
    const uint64_t blocks64 = (words + 255) / 256;
    const unsigned gblocks = (unsigned)(blocks64 > 65536 ? 65536 : blocks64);
    const bool gather = g.shift[0] >= 3;  // bricks at least 8 voxels wide
    if (g.nc[1] > 65535 || g.nc[2] > 65535) return hipErrorInvalidValue;
    const dim3 sgrid((unsigned)g.nc[1], (unsigned)g.nc[2]);
    // rows of a multiple of 4 voxels from an 8-byte aligned source: every
    // four-voxel group of the cell-table kernel is aligned to its own size
    const bool aligned = g.n[0] % 4 == 0 && (reinterpret_cast<uintptr_t>(src) & 7u) == 0;
#define VR_RL(C, U)                                                                       \
    if (channels == C && u16 == U) {                                                      \
        if (gather)                                                                       \
            hipLaunchKernelGGL((relayout_gather_kernel<C, U>), dim3(gblocks), dim3(256), 0, s, \
                               g, src, dst, maxval, words);                               \
        else                                                                              \
            hipLaunchKernelGGL((relayout_scatter_kernel<C, U>), grid, dim3(kRelayoutThreads), 0, s, g, \
                               src, dst, maxval);                                         \
        hipError_t e = hipGetLastError();                                                 \
        if (e != hipSuccess) return e;                                                    \
        if (aligned)                                                                      \
            hipLaunchKernelGGL((cellmax_strip_kernel<C, U, true>), sgrid, dim3(256), 0, s, g, src, \
                               dst, maxval);                                              \
        else                                                                              \
            hipLaunchKernelGGL((cellmax_strip_kernel<C, U, false>), sgrid, dim3(256), 0, s, g, \
                               src, dst, maxval);                                         \
        return hipGetLastError();                                                         \
    }
    VR_RL(1, false) VR_RL(2, false) VR_RL(3, false) VR_RL(4, false) VR_RL(5, false)
    VR_RL(6, false) VR_RL(1, true) VR_RL(2, true) VR_RL(3, true) VR_RL(4, true)
    VR_RL(5, true) VR_RL(6, true)
#undef VR_RL
    return hipErrorInvalidValue;
}

typedef void (*render_fn)(ReqParams, TileShape, int, int);
template <int V, bool kClear, bool kLit> constexpr render_fn render_entry() {
    if constexpr (variant_exists(V)) return render_kernel<V, kClear, kLit>;
    else return nullptr;
}
template <bool kClear, bool kLit, int... V>
constexpr std::array<render_fn, kVariants> render_table(std::integer_sequence<int, V...>) {
    return {{render_entry<V, kClear, kLit>()...}};
}
// [lit][clear_skip][variant]
static const std::array<render_fn, kVariants> kRender[2][2] = {
    {render_table<false, false>(std::make_integer_sequence<int, kVariants>{}),
     render_table<true, false>(std::make_integer_sequence<int, kVariants>{})},
    {render_table<false, true>(std::make_integer_sequence<int, kVariants>{}),
     render_table<true, true>(std::make_integer_sequence<int, kVariants>{})}};

hipError_t launch_render(const ReqParams& P, const TileShape& ts, bool clear_skip,
                         hipStream_t s) {
    if (P.variant < 0 || P.variant >= kVariants || !kRender[0][0][P.variant])
        return hipErrorInvalidValue;
    if (ts.wave_w <= 0 || ts.wave_h <= 0 || ts.wave_w * ts.wave_h != kWave)
        return hipErrorInvalidValue;
    const long long supers_x = supers_across(P.width, ts);
    const long long per_eye = tiles_per_eye(P.width, P.height, ts);
    const long long blocks = per_eye * P.eyes;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kRender[P.light.on ? 1 : 0][clear_skip ? 1 : 0][P.variant],
                       dim3((unsigned)blocks),
                       dim3(kWave), 0, s, P, ts, (int)supers_x, (int)per_eye);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchWork* dev_work, const ReqParams* dev_reqs,
                        const int32_t* dev_prefix, uint64_t mask, const int32_t* blocks,
                        hipStream_t s) {
    if (mask >> kBatchVariants) return hipErrorInvalidValue;
    for (int v = 0; v < kBatchVariants; ++v) {
        if (!(mask & (1ull << v))) continue;
        if (!kBatch[v] || blocks[v] <= 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL(kBatch[v], dim3(blocks[v]), dim3(kWave), 0, s, dev_work, dev_reqs,
                           dev_prefix);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t add_batch_nodes(hipGraph_t graph, const BatchWork* dev_work,
                           const ReqParams* dev_reqs, const int32_t* dev_prefix, uint64_t mask,
                           const int32_t* blocks, hipGraphNode_t* nodes) {
    if (mask >> kBatchVariants) return hipErrorInvalidValue;
    for (int v = 0; v < kBatchVariants; ++v) {
        nodes[v] = nullptr;
        if (!(mask & (1ull << v))) continue;
        if (!kBatch[v] || blocks[v] <= 0) return hipErrorInvalidValue;
        void* args[3] = {(void*)&dev_work, (void*)&dev_reqs, (void*)&dev_prefix};
        hipKernelNodeParams np{};
        np.func = (void*)kBatch[v];
        np.gridDim = dim3((unsigned)blocks[v]);
        np.blockDim = dim3(kWave);
        np.sharedMemBytes = 0;
        np.kernelParams = args;
        np.extra = nullptr;
        const hipError_t e = hipGraphAddKernelNode(&nodes[v], graph, nullptr, 0, &np);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t set_batch_node_grid(hipGraphExec_t exec, hipGraphNode_t node, int v, int blocks,
                               const BatchWork* dev_work, const ReqParams* dev_reqs,
                               const int32_t* dev_prefix) {
    if (v < 0 || v >= kBatchVariants || !kBatch[v] || blocks <= 0) return hipErrorInvalidValue;
    void* args[3] = {(void*)&dev_work, (void*)&dev_reqs, (void*)&dev_prefix};
    hipKernelNodeParams np{};
    np.func = (void*)kBatch[v];
    np.gridDim = dim3((unsigned)blocks);
    np.blockDim = dim3(kWave);
    np.sharedMemBytes = 0;
    np.kernelParams = args;
    np.extra = nullptr;
    return hipGraphExecKernelNodeSetParams(exec, node, &np);
}

typedef void (*debug_fn)(ReqParams, const float*, int, float*);
template <int V> constexpr debug_fn debug_entry() {
    if constexpr (variant_exists(V)) return debug_sample_kernel<V>;
    else return nullptr;
}
template <int... V>
constexpr std::array<debug_fn, kVariants> debug_table(std::integer_sequence<int, V...>) {
    return {{debug_entry<V>()...}};
}
static const std::array<debug_fn, kVariants> kDebug =
    debug_table(std::make_integer_sequence<int, kVariants>{});

hipError_t launch_debug_sample(const ReqParams& P, const float* pts, int n, float* out,
                               hipStream_t s) {
    if (P.variant < 0 || P.variant >= kVariants || !kDebug[P.variant])
        return hipErrorInvalidValue;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(kDebug[P.variant], dim3((n + 255) / 256), dim3(256), 0, s, P, pts, n,
                       out);
    return hipGetLastError();
}

}  // namespace vr

extern "C" vr_status vr_test_block_map(int32_t nblocks, int32_t* tiles) {
    if (nblocks < 0 || (nblocks > 0 && !tiles)) return VR_ERR_INVALID_ARG;
    for (int32_t b = 0; b < nblocks; ++b) tiles[b] = vr::xcd_remap(b, nblocks);
    return VR_OK;
}
