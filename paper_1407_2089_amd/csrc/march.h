// Device-side ray marcher: ray set-up, box clip, trilinear sampling from the
// brick-major layout, per-channel transfer functions, front-to-back
// compositing with early termination.  One lane owns one pixel of one eye.
//
// Every kernel that renders (the plain per-request launch and the batched
// launch) calls render_pixel<V>() below, so a pixel's arithmetic is the same
// instruction sequence whichever way it was scheduled.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "params.h"

namespace vr {

constexpr int kMaxSamples = 1 << 22;  // hard cap on samples per ray

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

template <int C, bool U16> struct WordT;
template <> struct WordT<1, false> { using T = uint8_t; };
template <> struct WordT<2, false> { using T = uint16_t; };
template <> struct WordT<3, false> { using T = uint32_t; };
template <> struct WordT<4, false> { using T = uint32_t; };
template <> struct WordT<1, true> { using T = uint16_t; };
template <> struct WordT<2, true> { using T = uint32_t; };
template <> struct WordT<3, true> { using T = uint2; };
template <> struct WordT<4, true> { using T = uint2; };
template <> struct WordT<5, false> { using T = uint2; };
template <> struct WordT<6, false> { using T = uint2; };
template <> struct WordT<5, true> { using T = uint4; };
template <> struct WordT<6, true> { using T = uint4; };

// 32-bit part q of a stored word (channels 4q .. 4q + 3 of uint8 words,
// 2q .. 2q + 1 of uint16 words).
template <typename T> __device__ __forceinline__ uint32_t part(T w, int q) {
    if constexpr (sizeof(T) <= 4) return (uint32_t)w;
    else if constexpr (sizeof(T) == 8) return q == 0 ? w.x : w.y;
    else return q == 0 ? w.x : q == 1 ? w.y : q == 2 ? w.z : w.w;
}

// Raw channel values of one stored word, as float.
template <int C, bool U16, typename T>
__device__ __forceinline__ void unpack_f32(T w, float (&x)[C]) {
    if constexpr (!U16) {
        if constexpr (C == 1) {
            x[0] = (float)(uint32_t)w;
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) x[c] = (float)((part(w, c >> 2) >> (8 * (c & 3))) & 0xffu);
        }
    } else {
        if constexpr (C == 1) {
            x[0] = (float)(uint32_t)w;
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) x[c] = (float)((part(w, c >> 1) >> (16 * (c & 1))) & 0xffffu);
        }
    }
}

// Raw channel values of one stored word as FP16 pairs (channel 2q, 2q + 1).
// uint8 channels convert exactly with one byte permute per pair: each byte b
// is placed under the FP16 pattern 0x64.. (the value 1024 + b), then 1024 is
// subtracted from both halves at once.  uint16 channels convert with the
// FP16 rounding of the value (exact up to 2048).
// kBiased: the values 1024 + b themselves, for a caller that subtracts the
// bias where it needs it (the difference of two such values is already exact).
constexpr half2_t kByteBias = {(_Float16)1024.0f, (_Float16)1024.0f};
template <bool kBiased = false>
__device__ __forceinline__ half2_t bytes_to_half2(uint32_t w, uint32_t sel) {
    const uint32_t v = __builtin_amdgcn_perm(0x64646464u, w, sel);
    if constexpr (kBiased) return __builtin_bit_cast(half2_t, v);
    else return __builtin_bit_cast(half2_t, v) - kByteBias;
}

typedef uint16_t u16x2_t __attribute__((ext_vector_type(2)));

// 16-bit values at or above 65520 would round to +inf in FP16; they are
// clamped to 65504, the largest finite half (a change of at most 31 raw
// units, within FP16's own rounding step of 32 at that magnitude).
// The two conversions write the halves of one register: the second converts
// the high word into the high half and keeps the low half (SDWA), which the
// compiler's own lowering does with a third instruction that packs two
// results.  Same rounding (to nearest even) and bits as the plain casts.
// kClamp = false: values known to stay below 65504 (data of at most 15 bits).
constexpr uint16_t kHalfMax = 65504;
template <bool kClamp = true>
__device__ __forceinline__ half2_t u16x2_to_half2(uint32_t w) {
    uint32_t x = w;
    if constexpr (kClamp)
        x = __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2_t, w),
                                                                   u16x2_t{kHalfMax, kHalfMax}));
    uint32_t r;
    asm("v_cvt_f16_u16_e32 %0, %1\n\t"
        "v_cvt_f16_u16_sdwa %0, %1 dst_sel:WORD_1 dst_unused:UNUSED_PRESERVE src0_sel:WORD_1"
        : "=&v"(r)
        : "v"(x));
    return __builtin_bit_cast(half2_t, r);
}

// kBiased (uint8, two channels or more): pairs of 1024 + b, see bytes_to_half2.
template <int C, bool U16, bool kClamp = true, bool kBiased = false, typename T>
__device__ __forceinline__ void unpack_f16(T w, half2_t (&h)[(C + 1) / 2]) {
    if constexpr (!U16) {
        if constexpr (C == 1) {
            h[0] = half2_t{(_Float16)(uint16_t)w, (_Float16)0.0f};
        } else {
#pragma unroll
            for (int q = 0; q < (C + 1) / 2; ++q)  // bytes 0, 1 or 2, 3 of part q / 2
                h[q] = bytes_to_half2<kBiased>(part(w, q >> 1),
                                               (q & 1) ? 0x04030402u : 0x04010400u);
        }
    } else {
        if constexpr (C == 1) {
            const uint16_t v = !kClamp || (uint16_t)w < kHalfMax ? (uint16_t)w : kHalfMax;
            h[0] = half2_t{(_Float16)v, (_Float16)0.0f};
        } else {
#pragma unroll
            for (int q = 0; q < (C + 1) / 2; ++q) h[q] = u16x2_to_half2<kClamp>(part(w, q));
        }
    }
}

// Buffer resource over one frame's storage (gfx9 family resource word 3).
// Loads through it are range-checked by the hardware against `bytes`:
// an address outside the frame reads zero instead of faulting.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t frame_rsrc(const uint8_t* vox, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)vox, (short)0, (int)bytes, 0x00020000);
}

template <typename T>
__device__ __forceinline__ T load_word(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ uint8_t load_word<uint8_t>(__amdgpu_buffer_rsrc_t r,
                                                                 uint32_t v, uint32_t s) {
    return __builtin_amdgcn_raw_buffer_load_b8(r, (int)v, (int)s, 0);
}
template <> __device__ __forceinline__ uint16_t load_word<uint16_t>(__amdgpu_buffer_rsrc_t r,
                                                                   uint32_t v, uint32_t s) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, (int)v, (int)s, 0);
}
template <> __device__ __forceinline__ uint32_t load_word<uint32_t>(__amdgpu_buffer_rsrc_t r,
                                                                   uint32_t v, uint32_t s) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)v, (int)s, 0);
}
template <> __device__ __forceinline__ uint2 load_word<uint2>(__amdgpu_buffer_rsrc_t r,
                                                             uint32_t v, uint32_t s) {
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, (int)v, (int)s, 0);
    return make_uint2(w.x, w.y);
}
template <> __device__ __forceinline__ uint4 load_word<uint4>(__amdgpu_buffer_rsrc_t r,
                                                             uint32_t v, uint32_t s) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, (int)v, (int)s, 0);
    return make_uint4(w.x, w.y, w.z, w.w);
}

// Four consecutive words (the row-pair layout's taps of one plane, which
// starts at an even word, so 4 W bytes from a 2 W-aligned byte offset): one
// 16-byte load for 4-byte words, one 8-byte load (dword-aligned) for 2-byte
// words, two 2-byte loads for 1-byte words.
template <typename T> struct Quad { T w[4]; };
template <typename T>
__device__ __forceinline__ Quad<T> load_quad(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ Quad<uint32_t> load_quad<uint32_t>(__amdgpu_buffer_rsrc_t r,
                                                                          uint32_t v, uint32_t s) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, (int)v, (int)s, 0);
    return Quad<uint32_t>{{a.x, a.y, a.z, a.w}};
}
template <> __device__ __forceinline__ Quad<uint16_t> load_quad<uint16_t>(__amdgpu_buffer_rsrc_t r,
                                                                          uint32_t v, uint32_t s) {
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 a = __builtin_amdgcn_raw_buffer_load_b64(r, (int)v, (int)s, 0);
    return Quad<uint16_t>{{(uint16_t)a.x, (uint16_t)(a.x >> 16), (uint16_t)a.y,
                           (uint16_t)(a.y >> 16)}};
}
template <> __device__ __forceinline__ Quad<uint8_t> load_quad<uint8_t>(__amdgpu_buffer_rsrc_t r,
                                                                        uint32_t v, uint32_t s) {
    const uint16_t a = __builtin_amdgcn_raw_buffer_load_b16(r, (int)v, (int)s, 0);
    const uint16_t b = __builtin_amdgcn_raw_buffer_load_b16(r, (int)(v + 2u), (int)s, 0);
    return Quad<uint8_t>{{(uint8_t)a, (uint8_t)(a >> 8), (uint8_t)b, (uint8_t)(b >> 8)}};
}
// Two consecutive words from a 2 W-aligned byte offset: one load of 2 W
// bytes.
template <typename T> struct Pair { T w[2]; };
template <typename T>
__device__ __forceinline__ Pair<T> load_pair(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ Pair<uint8_t> load_pair<uint8_t>(__amdgpu_buffer_rsrc_t r,
                                                                        uint32_t v, uint32_t s) {
    const uint16_t a = __builtin_amdgcn_raw_buffer_load_b16(r, (int)v, (int)s, 0);
    return Pair<uint8_t>{{(uint8_t)a, (uint8_t)(a >> 8)}};
}
template <> __device__ __forceinline__ Pair<uint16_t> load_pair<uint16_t>(__amdgpu_buffer_rsrc_t r,
                                                                          uint32_t v, uint32_t s) {
    const uint32_t a = __builtin_amdgcn_raw_buffer_load_b32(r, (int)v, (int)s, 0);
    return Pair<uint16_t>{{(uint16_t)a, (uint16_t)(a >> 16)}};
}
template <> __device__ __forceinline__ Pair<uint32_t> load_pair<uint32_t>(__amdgpu_buffer_rsrc_t r,
                                                                          uint32_t v, uint32_t s) {
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 a = __builtin_amdgcn_raw_buffer_load_b64(r, (int)v, (int)s, 0);
    return Pair<uint32_t>{{a.x, a.y}};
}
template <> __device__ __forceinline__ Pair<uint2> load_pair<uint2>(__amdgpu_buffer_rsrc_t r,
                                                                    uint32_t v, uint32_t s) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, (int)v, (int)s, 0);
    return Pair<uint2>{{make_uint2(a.x, a.y), make_uint2(a.z, a.w)}};
}

// floor(x) converted to int in one instruction (register-only).
__device__ __forceinline__ int cvt_floor(float x) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// Per-frame constants of the sampler, kept in scalar registers.
struct Sampler {
    __amdgpu_buffer_rsrc_t rsrc;
    float hi[3];        // largest float below n + 1 per axis (clamp bound)
    uint32_t row_b;     // bytes per brick row
    uint32_t plane_b;   // bytes per brick plane
    uint32_t diag_b;    // row_b + plane_b
    uint32_t cell_b;    // byte offset of the macro-cell table
};

__device__ __forceinline__ Sampler make_sampler(const uint8_t* vox, const BrickGeom& g) {
    Sampler S;
    S.rsrc = frame_rsrc(vox, (uint32_t)g.frame_bytes);
#pragma unroll
    for (int a = 0; a < 3; ++a) S.hi[a] = g.clamp_hi[a];  // below n + 1
    S.row_b = (uint32_t)(g.row * g.word);
    S.plane_b = (uint32_t)(g.plane * g.word);
    S.diag_b = S.row_b + S.plane_b;
    S.cell_b = (uint32_t)g.cell_off;
    return S;
}

// Large volumes (an axis above 8192 voxels, or a frame of 2^31 words or
// 4 GiB and more): plain global loads at 64-bit addresses, sample positions
// in FP64.
struct SamplerL {
    const uint8_t* vox;
    double hi[3];       // largest double below n + 1 per axis (clamp bound)
    uint32_t row_b;     // bytes per brick row
    uint32_t plane_b;   // bytes per brick plane
    uint32_t diag_b;    // row_b + plane_b
};

__device__ __forceinline__ SamplerL make_sampler_large(const ReqParams& P) {
    SamplerL S;
    S.vox = P.vox;
#pragma unroll
    for (int a = 0; a < 3; ++a) S.hi[a] = P.d64.clamp_hi[a];
    S.row_b = (uint32_t)(P.g.row * P.g.word);
    S.plane_b = (uint32_t)(P.g.plane * P.g.word);
    S.diag_b = S.row_b + S.plane_b;
    return S;
}

#define VR_GLOBAL __attribute__((address_space(1)))
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
template <typename T> __device__ __forceinline__ T load_global(const uint8_t* p) {
    if constexpr (sizeof(T) <= 4) {
        return *(const VR_GLOBAL T*)p;
    } else if constexpr (sizeof(T) == 8) {
        const u32x2_t w = *(const VR_GLOBAL u32x2_t*)p;
        return make_uint2(w.x, w.y);
    } else {
        const u32x4_t w = *(const VR_GLOBAL u32x4_t*)p;
        return make_uint4(w.x, w.y, w.z, w.w);
    }
}

// Four consecutive words of the row-pair layout through global loads (the
// first word has an even index, so the run is 2 W-aligned): two aligned loads
// of 2 W bytes each.
template <typename T> __device__ __forceinline__ Quad<T> load_quad_global(const uint8_t* p);
template <> __device__ __forceinline__ Quad<uint8_t> load_quad_global<uint8_t>(const uint8_t* p) {
    const uint16_t a = *(const VR_GLOBAL uint16_t*)p;
    const uint16_t b = *(const VR_GLOBAL uint16_t*)(p + 2);
    return Quad<uint8_t>{{(uint8_t)a, (uint8_t)(a >> 8), (uint8_t)b, (uint8_t)(b >> 8)}};
}
template <> __device__ __forceinline__ Quad<uint16_t> load_quad_global<uint16_t>(const uint8_t* p) {
    const uint32_t a = *(const VR_GLOBAL uint32_t*)p;
    const uint32_t b = *(const VR_GLOBAL uint32_t*)(p + 4);
    return Quad<uint16_t>{{(uint16_t)a, (uint16_t)(a >> 16), (uint16_t)b, (uint16_t)(b >> 16)}};
}
template <> __device__ __forceinline__ Quad<uint32_t> load_quad_global<uint32_t>(const uint8_t* p) {
    const u32x2_t a = *(const VR_GLOBAL u32x2_t*)p;
    const u32x2_t b = *(const VR_GLOBAL u32x2_t*)(p + 8);
    return Quad<uint32_t>{{a.x, a.y, b.x, b.y}};
}
template <> __device__ __forceinline__ Quad<uint2> load_quad_global<uint2>(const uint8_t* p) {
    const u32x4_t a = *(const VR_GLOBAL u32x4_t*)p;
    const u32x4_t b = *(const VR_GLOBAL u32x4_t*)(p + 16);
    return Quad<uint2>{{make_uint2(a.x, a.y), make_uint2(a.z, a.w), make_uint2(b.x, b.y),
                        make_uint2(b.z, b.w)}};
}

template <typename T> __device__ __forceinline__ Pair<T> load_pair_global(const uint8_t* p);
template <> __device__ __forceinline__ Pair<uint8_t> load_pair_global<uint8_t>(const uint8_t* p) {
    const uint16_t a = *(const VR_GLOBAL uint16_t*)p;
    return Pair<uint8_t>{{(uint8_t)a, (uint8_t)(a >> 8)}};
}
template <> __device__ __forceinline__ Pair<uint16_t> load_pair_global<uint16_t>(const uint8_t* p) {
    const uint32_t a = *(const VR_GLOBAL uint32_t*)p;
    return Pair<uint16_t>{{(uint16_t)a, (uint16_t)(a >> 16)}};
}
template <> __device__ __forceinline__ Pair<uint32_t> load_pair_global<uint32_t>(const uint8_t* p) {
    const u32x2_t a = *(const VR_GLOBAL u32x2_t*)p;
    return Pair<uint32_t>{{a.x, a.y}};
}
template <> __device__ __forceinline__ Pair<uint2> load_pair_global<uint2>(const uint8_t* p) {
    const u32x4_t a = *(const VR_GLOBAL u32x4_t*)p;
    return Pair<uint2>{{make_uint2(a.x, a.y), make_uint2(a.z, a.w)}};
}

// Low corner floor(q) of the taps of a point given in stored coordinates,
// after the clamp into [0, n + 1): the same two instructions (or FP64
// operations) the fetch below performs, so that both agree on every point.
__device__ __forceinline__ uint32_t corner(const Sampler& S, float q, int a) {
    return (uint32_t)cvt_floor(__builtin_amdgcn_fmed3f(q, 0.0f, S.hi[a]));
}
__device__ __forceinline__ uint32_t corner(const SamplerL& S, double q, int a) {
    return (uint32_t)__builtin_floor(__builtin_fmin(__builtin_fmax(q, 0.0), S.hi[a]));
}

// The word of macro cell c (cell coordinates) in the frame's cell table.  A
// 32-bit-addressed frame, table included, stays below 4 GiB, so its cell
// index and byte offset fit 32 bits; a large frame's index is formed in 64.
template <typename T>
__device__ __forceinline__ T load_cell(const BrickGeom& g, const Sampler& S,
                                       const uint32_t (&c)[3]) {
    const uint32_t idx = (c[2] * (uint32_t)g.nc[1] + c[1]) * (uint32_t)g.nc[0] + c[0];
    return load_word<T>(S.rsrc, idx * (uint32_t)sizeof(T), S.cell_b);
}
template <typename T>
__device__ __forceinline__ T load_cell(const BrickGeom& g, const SamplerL& S,
                                       const uint32_t (&c)[3]) {
    const uint64_t idx = ((uint64_t)c[2] * (uint32_t)g.nc[1] + c[1]) * (uint32_t)g.nc[0] + c[0];
    return load_global<T>(S.vox + g.cell_off + idx * sizeof(T));
}

// The 2x2x2 taps around one sample point, in flight or landed.
template <typename T> struct Taps {
    T w000, w100, w010, w110, w001, w101, w011, w111;
    float fx, fy, fz;
    uint32_t s[3];  // low corner (stored coordinates)
};

// Locate the taps around a point given in stored coordinates (index-space
// position + 1) and issue their loads (PAIRS: the row-pair layout, two quad
// loads; otherwise four x-pair loads, one per row).  The point is clamped into [0, n + 1)
// per axis (it lies in the box [0, n + 1] up to rounding; a point on the
// upper face is evaluated at the largest float below n + 1: one float step,
// about (n + 1) * 6e-8 voxels, inside the face where the field is zero).  The low corner floor(q) then
// lies in [0, n], so every tap is inside the frame; floor and fraction come
// from the same value, so they always agree.  Every factor and partial sum of
// the brick index is below 2^24 (a frame with 2^24 bricks or more takes the
// large-volume sampler), and so is every in-brick word index, so 24-bit
// multiply-adds are exact; the brick's first word, below 2^31, fits the low
// 32 bits of the 24-bit product.
template <typename T, bool PAIRS, typename Smp>
__device__ __forceinline__ void load_corner(const BrickGeom& g, const Smp& S,
                                            const uint32_t (&s)[3], Taps<T>& t);

template <typename T, bool PAIRS>
__device__ __forceinline__ Taps<T> fetch(const BrickGeom& g, const Sampler& S, float qx,
                                         float qy, float qz) {
    Taps<T> t;
    const float p[3] = {qx, qy, qz};
    float f[3];
    uint32_t s[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float q = __builtin_amdgcn_fmed3f(p[a], 0.0f, S.hi[a]);
        s[a] = (uint32_t)cvt_floor(q);
        f[a] = __builtin_amdgcn_fractf(q);
    }
    t.fx = f[0];
    t.fy = f[1];
    t.fz = f[2];
    load_corner<T, PAIRS>(g, S, s, t);
    return t;
}

// Byte offset in the frame of the first word of integer low corner s
// (stored coordinates, each in [0, n]).
template <typename T, bool PAIRS>
__device__ __forceinline__ uint32_t corner_addr(const BrickGeom& g, const Sampler& S,
                                                const uint32_t (&s)[3]) {
    const uint32_t bx = s[0] >> g.shift[0], lx = s[0] & ((1u << g.shift[0]) - 1u);
    const uint32_t by = s[1] >> g.shift[1], ly = s[1] & ((1u << g.shift[1]) - 1u);
    const uint32_t bz = s[2] >> g.shift[2], lz = s[2] & ((1u << g.shift[2]) - 1u);
    uint32_t brick = __umul24(bz, (uint32_t)g.nb[1]) + by;
    brick = __umul24(brick, (uint32_t)g.nb[0]) + bx;
    uint32_t local = __umul24(lz, (uint32_t)g.plane) + (PAIRS ? lx << 1 : lx);
    local = __umul24(ly, (uint32_t)g.row) + local;
    return (__umul24(brick, (uint32_t)g.brick) + local) * (uint32_t)sizeof(T);
}

// Loads at a corner's first word plus a per-lane byte offset v and a
// wave-uniform one u: one word, a 2 W-aligned pair of consecutive words, or
// a 2 W-aligned run of four (the row-pair layout's taps of one plane).
template <typename T>
__device__ __forceinline__ T word_at(const Sampler& S, uint32_t a, uint32_t v, uint32_t u) {
    return load_word<T>(S.rsrc, a + v, u);
}
template <typename T>
__device__ __forceinline__ Pair<T> pair_at(const Sampler& S, uint32_t a, uint32_t v, uint32_t u) {
    return load_pair<T>(S.rsrc, a + v, u);
}
template <typename T>
__device__ __forceinline__ Quad<T> quad_at(const Sampler& S, uint32_t a, uint32_t v, uint32_t u) {
    return load_quad<T>(S.rsrc, a + v, u);
}

// Large-volume fetch: the same taps, with the point, its clamp into
// [0, n + 1) and its floor in FP64 (a stored coordinate up to 16385 keeps
// 2^-38 voxel resolution) and the byte offset in 64 bits.  The brick index
// fits 32 bits (a frame holds fewer than 2^32 bricks, checked at volume
// creation), and so does the in-brick word index.  The fraction in [0, 1) is
// rounded to FP32 for the interpolation weights.
template <typename T, bool PAIRS>
__device__ __forceinline__ Taps<T> fetch(const BrickGeom& g, const SamplerL& S, double qx,
                                         double qy, double qz) {
    Taps<T> t;
    const double p[3] = {qx, qy, qz};
    float f[3];
    uint32_t s[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double q = __builtin_fmin(__builtin_fmax(p[a], 0.0), S.hi[a]);
        const double fl = __builtin_floor(q);
        s[a] = (uint32_t)fl;
        f[a] = (float)(q - fl);
    }
    t.fx = f[0];
    t.fy = f[1];
    t.fz = f[2];
    load_corner<T, PAIRS>(g, S, s, t);
    return t;
}

template <typename T, bool PAIRS>
__device__ __forceinline__ const uint8_t* corner_addr(const BrickGeom& g, const SamplerL& S,
                                                      const uint32_t (&s)[3]) {
    const uint32_t bx = s[0] >> g.shift[0], lx = s[0] & ((1u << g.shift[0]) - 1u);
    const uint32_t by = s[1] >> g.shift[1], ly = s[1] & ((1u << g.shift[1]) - 1u);
    const uint32_t bz = s[2] >> g.shift[2], lz = s[2] & ((1u << g.shift[2]) - 1u);
    const uint32_t brick = (bz * (uint32_t)g.nb[1] + by) * (uint32_t)g.nb[0] + bx;
    const uint32_t local = lz * (uint32_t)g.plane + ly * (uint32_t)g.row + (PAIRS ? lx << 1 : lx);
    return S.vox + ((uint64_t)brick * (uint32_t)g.brick + local) * sizeof(T);
}
template <typename T>
__device__ __forceinline__ T word_at(const SamplerL& S, const uint8_t* a, uint32_t v, uint32_t u) {
    return load_global<T>(a + v + u);
}
template <typename T>
__device__ __forceinline__ Pair<T> pair_at(const SamplerL& S, const uint8_t* a, uint32_t v,
                                           uint32_t u) {
    return load_pair_global<T>(a + v + u);
}
template <typename T>
__device__ __forceinline__ Quad<T> quad_at(const SamplerL& S, const uint8_t* a, uint32_t v,
                                           uint32_t u) {
    return load_quad_global<T>(a + v + u);
}

// The eight taps of integer low corner s (stored coordinates, each in
// [0, n]) into t (corner recorded in t.s).
template <typename T, bool PAIRS, typename Smp>
__device__ __forceinline__ void load_corner(const BrickGeom& g, const Smp& S,
                                            const uint32_t (&s)[3], Taps<T>& t) {
    t.s[0] = s[0];
    t.s[1] = s[1];
    t.s[2] = s[2];
    const auto a = corner_addr<T, PAIRS>(g, S, s);
    constexpr uint32_t W = sizeof(T);
    if constexpr (PAIRS) {
        // Words (x, y), (x, y + 1), (x + 1, y), (x + 1, y + 1) of each plane.
        const Quad<T> lo = quad_at<T>(S, a, 0, 0);
        const Quad<T> hi = quad_at<T>(S, a, 0, S.plane_b);
        t.w000 = lo.w[0];
        t.w010 = lo.w[1];
        t.w100 = lo.w[2];
        t.w110 = lo.w[3];
        t.w001 = hi.w[0];
        t.w011 = hi.w[1];
        t.w101 = hi.w[2];
        t.w111 = hi.w[3];
        return;
    }
    t.w000 = word_at<T>(S, a, 0, 0);
    t.w100 = word_at<T>(S, a, W, 0);
    t.w010 = word_at<T>(S, a, 0, S.row_b);
    t.w110 = word_at<T>(S, a, W, S.row_b);
    t.w001 = word_at<T>(S, a, 0, S.plane_b);
    t.w101 = word_at<T>(S, a, W, S.plane_b);
    t.w011 = word_at<T>(S, a, 0, S.diag_b);
    t.w111 = word_at<T>(S, a, W, S.diag_b);
}

// The taps one voxel layer beyond a corner's cube along axis `a`, on both
// sides: lo[m] the words at offset -1 along a, hi[m] at offset +2, where m
// indexes the other two axes' offsets (0 or 1; lower axis first).  They are
// those layers when 1 <= s[a] and s[a] + 1 <= n[a]; for a corner on a face
// the two corners are clamped into [0, n] instead (some in-frame words,
// for the caller to discard), so every address stays inside the frame even
// where an axis holds a single voxel.
template <typename T, bool PAIRS, typename Smp>
__device__ __forceinline__ void load_layers(const BrickGeom& g, const Smp& S,
                                            const uint32_t (&s)[3], int axis, T (&lo)[4],
                                            T (&hi)[4]) {
    uint32_t sl[3] = {s[0], s[1], s[2]}, sh[3] = {s[0], s[1], s[2]};
    const uint32_t n = (uint32_t)g.n[axis];
    sl[axis] = s[axis] > 0u ? s[axis] - 1u : 0u;
    sh[axis] = s[axis] < n ? s[axis] + 1u : n;
    const auto al = corner_addr<T, PAIRS>(g, S, sl);
    const auto ah = corner_addr<T, PAIRS>(g, S, sh);
    constexpr uint32_t W = sizeof(T);
    if constexpr (PAIRS) {
        // Plane words: (x, y) at 0, (x, y + 1) at W, (x + 1, y) at 2 W,
        // (x + 1, y + 1) at 3 W.
        if (axis == 0) {
            const Pair<T> l0 = pair_at<T>(S, al, 0, 0), l1 = pair_at<T>(S, al, 0, S.plane_b);
            const Pair<T> h0 = pair_at<T>(S, ah, 2 * W, 0);
            const Pair<T> h1 = pair_at<T>(S, ah, 2 * W, S.plane_b);
            lo[0] = l0.w[0]; lo[1] = l0.w[1]; lo[2] = l1.w[0]; lo[3] = l1.w[1];
            hi[0] = h0.w[0]; hi[1] = h0.w[1]; hi[2] = h1.w[0]; hi[3] = h1.w[1];
        } else if (axis == 1) {
            lo[0] = word_at<T>(S, al, 0, 0);
            lo[1] = word_at<T>(S, al, 2 * W, 0);
            lo[2] = word_at<T>(S, al, 0, S.plane_b);
            lo[3] = word_at<T>(S, al, 2 * W, S.plane_b);
            hi[0] = word_at<T>(S, ah, W, 0);
            hi[1] = word_at<T>(S, ah, 3 * W, 0);
            hi[2] = word_at<T>(S, ah, W, S.plane_b);
            hi[3] = word_at<T>(S, ah, 3 * W, S.plane_b);
        } else {
            const Quad<T> l = quad_at<T>(S, al, 0, 0);
            const Quad<T> h = quad_at<T>(S, ah, 0, S.plane_b);
            lo[0] = l.w[0]; lo[1] = l.w[2]; lo[2] = l.w[1]; lo[3] = l.w[3];
            hi[0] = h.w[0]; hi[1] = h.w[2]; hi[2] = h.w[1]; hi[3] = h.w[3];
        }
        return;
    }
    // Plain rows: (x, y) at 0, (x + 1, y) at W, rows row_b apart.
    if (axis == 0) {
        lo[0] = word_at<T>(S, al, 0, 0);
        lo[1] = word_at<T>(S, al, 0, S.row_b);
        lo[2] = word_at<T>(S, al, 0, S.plane_b);
        lo[3] = word_at<T>(S, al, 0, S.diag_b);
        hi[0] = word_at<T>(S, ah, W, 0);
        hi[1] = word_at<T>(S, ah, W, S.row_b);
        hi[2] = word_at<T>(S, ah, W, S.plane_b);
        hi[3] = word_at<T>(S, ah, W, S.diag_b);
    } else if (axis == 1) {
        lo[0] = word_at<T>(S, al, 0, 0);
        lo[1] = word_at<T>(S, al, W, 0);
        lo[2] = word_at<T>(S, al, 0, S.plane_b);
        lo[3] = word_at<T>(S, al, W, S.plane_b);
        hi[0] = word_at<T>(S, ah, 0, S.row_b);
        hi[1] = word_at<T>(S, ah, W, S.row_b);
        hi[2] = word_at<T>(S, ah, 0, S.diag_b);
        hi[3] = word_at<T>(S, ah, W, S.diag_b);
    } else {
        lo[0] = word_at<T>(S, al, 0, 0);
        lo[1] = word_at<T>(S, al, W, 0);
        lo[2] = word_at<T>(S, al, 0, S.row_b);
        lo[3] = word_at<T>(S, al, W, S.row_b);
        hi[0] = word_at<T>(S, ah, 0, S.plane_b);
        hi[1] = word_at<T>(S, ah, W, S.plane_b);
        hi[2] = word_at<T>(S, ah, 0, S.diag_b);
        hi[3] = word_at<T>(S, ah, W, S.diag_b);
    }
}

__device__ __forceinline__ float fma_r(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) {
    return __builtin_fma(a, b, c);
}

__device__ __forceinline__ float ceil_r(float x) { return ceilf(x); }
__device__ __forceinline__ double ceil_r(double x) { return __builtin_ceil(x); }

__device__ __forceinline__ float lerp(float a, float b, float f) { return fmaf(f, b - a, a); }
// An explicit fused multiply-add: left to floating-point contraction, the
// compiler may fuse the product in one kernel and round it in another, and
// kernels that must agree bit for bit (with and without the skips, plain and
// batched) would not.
__device__ __forceinline__ half2_t lerp(half2_t a, half2_t b, half2_t f) {
    return __builtin_elementwise_fma(f, b - a, a);
}

// Trilinear field (raw units) of every channel from landed taps.  kLerp
// keeps the lerp tree for any channel count: it returns a constant field
// exactly (a + f (a - a) = a), which the weighted sum does not (its FP32
// weights sum to 1 only up to rounding).
template <int C, bool U16, bool F16, bool kLerp = false, bool kClamp16 = true, typename T>
__device__ __forceinline__ void interpolate(const Taps<T>& t, float (&x)[C]) {
    const float fx = t.fx, fy = t.fy, fz = t.fz;
    if constexpr (!F16 && C >= 3 && !kLerp) {
        // Many channels: the eight trilinear weights once, then one 8-term
        // weighted sum per channel.
        const float gx = 1.0f - fx, gy = 1.0f - fy, gz = 1.0f - fz;
        const float w00 = gx * gy, w10 = fx * gy, w01 = gx * fy, w11 = fx * fy;
        const float wt[8] = {w00 * gz, w10 * gz, w01 * gz, w11 * gz,
                             w00 * fz, w10 * fz, w01 * fz, w11 * fz};
        float v[8][C];
        unpack_f32<C, U16>(t.w000, v[0]);
        unpack_f32<C, U16>(t.w100, v[1]);
        unpack_f32<C, U16>(t.w010, v[2]);
        unpack_f32<C, U16>(t.w110, v[3]);
        unpack_f32<C, U16>(t.w001, v[4]);
        unpack_f32<C, U16>(t.w101, v[5]);
        unpack_f32<C, U16>(t.w011, v[6]);
        unpack_f32<C, U16>(t.w111, v[7]);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            float acc = wt[0] * v[0][c];
#pragma unroll
            for (int q = 1; q < 8; ++q) acc = fmaf(wt[q], v[q][c], acc);
            x[c] = acc;
        }
    } else if constexpr (!F16) {
        float a000[C], a100[C], a010[C], a110[C], a001[C], a101[C], a011[C], a111[C];
        unpack_f32<C, U16>(t.w000, a000);
        unpack_f32<C, U16>(t.w100, a100);
        unpack_f32<C, U16>(t.w010, a010);
        unpack_f32<C, U16>(t.w110, a110);
        unpack_f32<C, U16>(t.w001, a001);
        unpack_f32<C, U16>(t.w101, a101);
        unpack_f32<C, U16>(t.w011, a011);
        unpack_f32<C, U16>(t.w111, a111);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            float c00 = lerp(a000[c], a100[c], fx);
            float c10 = lerp(a010[c], a110[c], fx);
            float c01 = lerp(a001[c], a101[c], fx);
            float c11 = lerp(a011[c], a111[c], fx);
            float c0 = lerp(c00, c10, fy);
            float c1 = lerp(c01, c11, fy);
            x[c] = lerp(c0, c1, fz);
        }
    } else {
        constexpr int NP = (C + 1) / 2;
        // uint8 pairs stay biased (1024 + b) into the x lerps: the difference
        // of two biased taps is the exact difference of the bytes, so only
        // each lerp's base needs the bias removed, and the lerp is the one of
        // the unbiased taps bit for bit.
        constexpr bool kB = !U16 && C >= 2;
        half2_t a000[NP], a100[NP], a010[NP], a110[NP], a001[NP], a101[NP], a011[NP], a111[NP];
        unpack_f16<C, U16, kClamp16, kB>(t.w000, a000);
        unpack_f16<C, U16, kClamp16, kB>(t.w100, a100);
        unpack_f16<C, U16, kClamp16, kB>(t.w010, a010);
        unpack_f16<C, U16, kClamp16, kB>(t.w110, a110);
        unpack_f16<C, U16, kClamp16, kB>(t.w001, a001);
        unpack_f16<C, U16, kClamp16, kB>(t.w101, a101);
        unpack_f16<C, U16, kClamp16, kB>(t.w011, a011);
        unpack_f16<C, U16, kClamp16, kB>(t.w111, a111);
        // The fractions go to FP16 through one explicit conversion (round
        // toward zero, both halves at once).  A plain cast would let the
        // compiler merge a fraction rounded from FP64 to FP32 (large volumes)
        // and then to FP16 into one direct FP64 to FP16 rounding in some
        // inlined copies and not in others: the two round differently at
        // ties, and kernels that must agree bit for bit would not.
        const half2_t hx = __builtin_bit_cast(half2_t, __builtin_amdgcn_cvt_pkrtz(fx, fx));
        const half2_t hy = __builtin_bit_cast(half2_t, __builtin_amdgcn_cvt_pkrtz(fy, fy));
        const half2_t hz = __builtin_bit_cast(half2_t, __builtin_amdgcn_cvt_pkrtz(fz, fz));
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            half2_t c00, c10, c01, c11;
            if constexpr (kB) {
                c00 = __builtin_elementwise_fma(hx, a100[q] - a000[q], a000[q] - kByteBias);
                c10 = __builtin_elementwise_fma(hx, a110[q] - a010[q], a010[q] - kByteBias);
                c01 = __builtin_elementwise_fma(hx, a101[q] - a001[q], a001[q] - kByteBias);
                c11 = __builtin_elementwise_fma(hx, a111[q] - a011[q], a011[q] - kByteBias);
            } else {
                c00 = lerp(a000[q], a100[q], hx);
                c10 = lerp(a010[q], a110[q], hx);
                c01 = lerp(a001[q], a101[q], hx);
                c11 = lerp(a011[q], a111[q], hx);
            }
            half2_t c0 = lerp(c00, c10, hy);
            half2_t c1 = lerp(c01, c11, hy);
            half2_t v = lerp(c0, c1, hz);
            x[2 * q] = (float)v.x;
            if (2 * q + 1 < C) x[2 * q + 1] = (float)v.y;
        }
    }
}

// Channel pair q of a stored word as two 16-bit lanes (channel 2q, 2q + 1).
template <int C, bool U16, typename T>
__device__ __forceinline__ u16x2_t pair16(T w, int q) {
    if constexpr (U16) {
        return __builtin_bit_cast(u16x2_t, part(w, q));
    } else {
        const uint32_t sel = (q & 1) ? 0x0c030c02u : 0x0c010c00u;  // zero-extend 2 bytes
        return __builtin_bit_cast(u16x2_t, __builtin_amdgcn_perm(0u, part(w, q >> 1), sel));
    }
}

// True when every tap of every channel c is at most tmax[c]: the sample's
// opacity is then exactly 0 (see Transparent), so its compositing can be left
// out without changing any output bit.  Costs a packed 16-bit max per word
// pair and one saturating compare per channel pair.
template <int C, bool U16, typename T>
__device__ __forceinline__ bool transparent(const Taps<T>& t, const Transparent& z) {
    if constexpr (C == 1) {
        const uint32_t m =
            max(max(max((uint32_t)t.w000, (uint32_t)t.w100), max((uint32_t)t.w010, (uint32_t)t.w110)),
                max(max((uint32_t)t.w001, (uint32_t)t.w101), max((uint32_t)t.w011, (uint32_t)t.w111)));
        return m <= z.tmax[0];
    } else if constexpr (!U16 && (C == 3 || C == 4)) {
        // Four uint8 channels: the odd channels are the high bytes of the
        // word's 16-bit lanes, the even ones become so after a shift by 8 in
        // each lane; a lane max compared with (t << 8 | 255) tests the high
        // byte (no byte unpacking).
        const u16x2_t eight = {8, 8};
        const auto hi_lo = [&](uint32_t a, uint32_t b, u16x2_t& hi, u16x2_t& lo) {
            const u16x2_t x = __builtin_bit_cast(u16x2_t, a), y = __builtin_bit_cast(u16x2_t, b);
            hi = __builtin_elementwise_max(x, y);
            lo = __builtin_elementwise_max(x << eight, y << eight);
        };
        u16x2_t h0, l0, h1, l1, h2, l2, h3, l3;
        hi_lo((uint32_t)t.w000, (uint32_t)t.w100, h0, l0);
        hi_lo((uint32_t)t.w010, (uint32_t)t.w110, h1, l1);
        hi_lo((uint32_t)t.w001, (uint32_t)t.w101, h2, l2);
        hi_lo((uint32_t)t.w011, (uint32_t)t.w111, h3, l3);
        const u16x2_t hi = __builtin_elementwise_max(__builtin_elementwise_max(h0, h1),
                                                     __builtin_elementwise_max(h2, h3));
        const u16x2_t lo = __builtin_elementwise_max(__builtin_elementwise_max(l0, l1),
                                                     __builtin_elementwise_max(l2, l3));
        const u16x2_t over_hi = __builtin_elementwise_sub_sat(hi, __builtin_bit_cast(u16x2_t, z.byte_hi));
        const u16x2_t over_lo = __builtin_elementwise_sub_sat(lo, __builtin_bit_cast(u16x2_t, z.byte_lo));
        return (__builtin_bit_cast(uint32_t, over_hi) | __builtin_bit_cast(uint32_t, over_lo)) == 0u;
    } else {
        bool clear = true;
#pragma unroll
        for (int q = 0; q < (C + 1) / 2; ++q) {
            const u16x2_t m = __builtin_elementwise_max(
                __builtin_elementwise_max(
                    __builtin_elementwise_max(pair16<C, U16>(t.w000, q), pair16<C, U16>(t.w100, q)),
                    __builtin_elementwise_max(pair16<C, U16>(t.w010, q), pair16<C, U16>(t.w110, q))),
                __builtin_elementwise_max(
                    __builtin_elementwise_max(pair16<C, U16>(t.w001, q), pair16<C, U16>(t.w101, q)),
                    __builtin_elementwise_max(pair16<C, U16>(t.w011, q), pair16<C, U16>(t.w111, q))));
            const u16x2_t over =
                __builtin_elementwise_sub_sat(m, __builtin_bit_cast(u16x2_t, z.tmax2[q]));
            clear = clear && __builtin_bit_cast(uint32_t, over) == 0u;
        }
        return clear;
    }
}

// True when a macro cell's per-channel maxima pass the transparent test:
// every sample whose low corner lies in the cell then has opacity exactly 0.
template <int C, bool U16, typename T>
__device__ __forceinline__ bool cell_clear(T w, const Transparent& z) {
    const Taps<T> t{w, w, w, w, w, w, w, w, 0.0f, 0.0f, 0.0f, {0u, 0u, 0u}};
    return transparent<C, U16>(t, z);
}

// Trilinear field (raw units) of every channel at index-space point p.
template <int C, bool U16, bool F16, bool PAIRS>
__device__ __forceinline__ void sample(const BrickGeom& g, const Sampler& S, float px, float py,
                                       float pz, float (&x)[C]) {
    using T = typename WordT<C, U16>::T;
    interpolate<C, U16, F16>(fetch<T, PAIRS>(g, S, px + 1.0f, py + 1.0f, pz + 1.0f), x);
}

template <int V> struct Variant {
    static constexpr int C = variant_channels(V);
    static constexpr bool U16 = variant_u16(V);
    static constexpr bool F16 = variant_fp16(V);
    static constexpr bool PAIRS = variant_pairs(V);
    static constexpr bool LARGE = variant_large(V);
    // Position type: FP64 for large volumes.
    using R = typename std::conditional<LARGE, double, float>::type;
    using Smp = typename std::conditional<LARGE, SamplerL, Sampler>::type;
};

template <bool LARGE> __device__ __forceinline__ auto sampler_for(const ReqParams& P) {
    if constexpr (LARGE) return make_sampler_large(P);
    else return make_sampler(P.vox, P.g);
}

// One pixel of one eye: returns nothing, writes RGBA (and the sample count).
// `valid` false lanes take part in the wave's loop structure but do no work.
// Difference, per channel, of the trilinear field at the two points one
// voxel either side of a sample along axis `a`, for a sample away from the
// faces: those points have the sample's fractions and its corner moved by
// one voxel, so the difference is one lerp tree, with the sample's
// fractions, over the eight voxel differences (exact integers).  Half of
// each neighbour's taps are the sample's own words v (index x + 2 y + 4 z
// offsets); lw and hw are the layers at -1 and +2 along a.
template <int C, bool U16, typename Word>
__device__ __forceinline__ void axis_diff(int a, const Word (&lw)[4], const Word (&hw)[4],
                                          const float (&v)[8][C], float fx, float fy, float fz,
                                          float (&diff)[C]) {
    float l[4][C], h[4][C];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        unpack_f32<C, U16>(lw[m], l[m]);
        unpack_f32<C, U16>(hw[m], h[m]);
    }
    const int bit = 1 << a;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float d[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int m = a == 0 ? i >> 1 : a == 1 ? (i & 1) | ((i >> 1) & 2) : i & 3;
            d[i] = (i & bit) ? h[m][c] - v[i & ~bit][c] : v[i | bit][c] - l[m][c];
        }
        const float c00 = lerp(d[0], d[1], fx);
        const float c10 = lerp(d[2], d[3], fx);
        const float c01 = lerp(d[4], d[5], fx);
        const float c11 = lerp(d[6], d[7], fx);
        diff[c] = lerp(lerp(c00, c10, fy), lerp(c01, c11, fy), fz);
    }
}

// Lambert shade of every channel at stored-coordinate point q: the gradient
// of each channel's trilinear field by central differences over one voxel per
// axis (FP32, also under FP16 sampling: FP16 lerps would turn a small
// gradient's direction; always the lerp tree, so that a flat neighbourhood
// has exactly zero gradient and takes ambient + diffuse), the normal against
// it, one directional light.  A sample at a face (low corner 0 or n along an
// axis) takes that axis's two neighbours as clamped trilinear samples.
template <int C, bool U16, bool PAIRS, typename Word, typename Smp, typename R>
__device__ __forceinline__ void shade_at(const ReqParams& P, const Smp& S, const R (&q)[3],
                                         const Taps<Word>& t, float (&shade)[C]) {
    float g[3][C];
    const R one = 1;
    float v[8][C];
    unpack_f32<C, U16>(t.w000, v[0]);
    unpack_f32<C, U16>(t.w100, v[1]);
    unpack_f32<C, U16>(t.w010, v[2]);
    unpack_f32<C, U16>(t.w110, v[3]);
    unpack_f32<C, U16>(t.w001, v[4]);
    unpack_f32<C, U16>(t.w101, v[5]);
    unpack_f32<C, U16>(t.w011, v[6]);
    unpack_f32<C, U16>(t.w111, v[7]);
    bool inner[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) inner[a] = t.s[a] >= 1u && t.s[a] + 1u <= (uint32_t)P.g.n[a];
    if constexpr (sizeof(Word) <= 4) {
        // Narrow words: the layers of all three axes are requested together
        // (one memory round trip instead of three, measured 5 % faster on
        // the realistic frame); a lane at a face loads clamped, in-frame
        // corners there and replaces that axis's difference below.
        Word lw[3][4], hw[3][4];
#pragma unroll
        for (int a = 0; a < 3; ++a) load_layers<Word, PAIRS>(P.g, S, t.s, a, lw[a], hw[a]);
#pragma unroll
        for (int a = 0; a < 3; ++a) axis_diff<C, U16>(a, lw[a], hw[a], v, t.fx, t.fy, t.fz, g[a]);
    } else {
        // Wide words (registers): one axis at a time.
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (inner[a]) {
                Word lw[4], hw[4];
                load_layers<Word, PAIRS>(P.g, S, t.s, a, lw, hw);
                axis_diff<C, U16>(a, lw, hw, v, t.fx, t.fy, t.fz, g[a]);
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!inner[a]) {
            const Taps<Word> hi = fetch<Word, PAIRS>(P.g, S, a == 0 ? q[0] + one : q[0],
                                                     a == 1 ? q[1] + one : q[1],
                                                     a == 2 ? q[2] + one : q[2]);
            const Taps<Word> lo = fetch<Word, PAIRS>(P.g, S, a == 0 ? q[0] - one : q[0],
                                                     a == 1 ? q[1] - one : q[1],
                                                     a == 2 ? q[2] - one : q[2]);
            float vh[C], vl[C];
            interpolate<C, U16, false, true>(hi, vh);
            interpolate<C, U16, false, true>(lo, vl);
#pragma unroll
            for (int c = 0; c < C; ++c) g[a][c] = vh[c] - vl[c];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) g[a][c] = g[a][c] * P.light.gscale[a];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const float gg = fmaf(g[0][c], g[0][c], fmaf(g[1][c], g[1][c], g[2][c] * g[2][c]));
        const float dot = -fmaf(g[0][c], P.light.dir[0],
                                fmaf(g[1][c], P.light.dir[1], g[2][c] * P.light.dir[2]));
        // gg below 2^-100 (never reached by a non-zero difference of raw
        // samples at a sane spacing ratio) counts as no gradient, keeping
        // rsqrt away from denormals.
        const float dl = gg > 0x1p-100f ? fmaxf(dot, 0.0f) * rsqrtf(gg) : 1.0f;
        shade[c] = fmaf(P.light.kd, dl, P.light.ka);
    }
}

// Ray of one pixel in index space: direction d (index units per unit of t),
// entry point pe in stored coordinates (index-space position + 1) and sample
// count n (0 for a ray that misses the box or an invalid lane).
__device__ __forceinline__ void pixel_ray(const ReqParams& P, int eye, int px, int py, bool valid,
                                          float (&d)[3], float (&pe)[3], int& n) {
    const float sx = fmaf((float)px + 0.5f, P.sx_scale, -1.0f);
    const float sy = fmaf(-((float)py + 0.5f), P.sy_scale, 1.0f);

    float p0[3];
    float w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float o = eye ? P.o0[1][a] : P.o0[0][a];
        const float bse = eye ? P.base[1][a] : P.base[0][a];
        p0[a] = fmaf(sy, P.ov[a], fmaf(sx, P.ou[a], o));
        w[a] = fmaf(sy, P.dv[a], fmaf(sx, P.du[a], bse));
    }
    const float inv_len = rsqrtf(fmaf(w[0], w[0], fmaf(w[1], w[1], w[2] * w[2])));
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = w[a] * inv_len * P.inv_sp[a];

    // Slab clip against the extended box [-1, n] per axis.
    float t_in = P.tmin, t_out = INFINITY;
    bool hit = valid;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float hi = (float)P.g.n[a];
        if (d[a] != 0.0f) {
            const float inv = 1.0f / d[a];
            const float t1 = (-1.0f - p0[a]) * inv;
            const float t2 = (hi - p0[a]) * inv;
            t_in = fmaxf(t_in, fminf(t1, t2));
            t_out = fminf(t_out, fmaxf(t1, t2));
        } else {
            hit = hit && (p0[a] >= -1.0f) && (p0[a] <= hi);
        }
    }
    n = 0;
    if (hit && t_in < t_out) {
        const float span = (t_out - t_in) / P.step - 0.5f;
        const float c = ceilf(span);
        n = c <= 0.0f ? 0 : (c >= (float)kMaxSamples ? kMaxSamples : (int)c);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) pe[a] = fmaf(n > 0 ? t_in : 0.0f, d[a], p0[a]) + 1.0f;
}

// The same ray in FP64 from the request's FP64 basis (large volumes).
__device__ __forceinline__ void pixel_ray(const ReqParams& P, int eye, int px, int py, bool valid,
                                          double (&d)[3], double (&pe)[3], int& n) {
    const auto& D = P.d64;
    const double sx = __builtin_fma((double)px + 0.5, D.sx_scale, -1.0);
    const double sy = __builtin_fma(-((double)py + 0.5), D.sy_scale, 1.0);
    double p0[3], w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double o = eye ? D.o0[1][a] : D.o0[0][a];
        const double bse = eye ? D.base[1][a] : D.base[0][a];
        p0[a] = __builtin_fma(sy, D.ov[a], __builtin_fma(sx, D.ou[a], o));
        w[a] = __builtin_fma(sy, D.dv[a], __builtin_fma(sx, D.du[a], bse));
    }
    const double inv_len =
        1.0 / __builtin_sqrt(__builtin_fma(w[0], w[0], __builtin_fma(w[1], w[1], w[2] * w[2])));
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = w[a] * inv_len * D.inv_sp[a];
    double t_in = D.tmin, t_out = __builtin_inf();
    bool hit = valid;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double hi = (double)P.g.n[a];
        if (d[a] != 0.0) {
            const double inv = 1.0 / d[a];
            const double t1 = (-1.0 - p0[a]) * inv;
            const double t2 = (hi - p0[a]) * inv;
            t_in = __builtin_fmax(t_in, __builtin_fmin(t1, t2));
            t_out = __builtin_fmin(t_out, __builtin_fmax(t1, t2));
        } else {
            hit = hit && (p0[a] >= -1.0) && (p0[a] <= hi);
        }
    }
    n = 0;
    if (hit && t_in < t_out) {
        const double c = __builtin_ceil((t_out - t_in) / D.step - 0.5);
        n = c <= 0.0 ? 0 : (c >= (double)kMaxSamples ? kMaxSamples : (int)c);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) pe[a] = __builtin_fma(n > 0 ? t_in : 0.0, d[a], p0[a]) + 1.0;
}

template <int V, bool kClear = true, bool kLit = false>
__device__ __forceinline__ void render_pixel(const ReqParams& P, int eye, int px, int py,
                                             bool valid) {
    constexpr int C = Variant<V>::C;
    constexpr bool U16 = Variant<V>::U16;
    constexpr bool F16 = Variant<V>::F16;
    constexpr bool PAIRS = Variant<V>::PAIRS;
    constexpr bool LARGE = Variant<V>::LARGE;
    using R = typename Variant<V>::R;

    R d[3], pe[3];
    int n;
    pixel_ray(P, eye, px, py, valid, d, pe, n);

    // Transfer-function coefficients (wave-uniform).
    ChanTF tf[C];
#pragma unroll
    for (int c = 0; c < C; ++c) tf[c] = P.tf[c];
    // Unlit with one or two channels, the two addends of the transfer
    // function are held in vector registers: a multiply-add reads at most
    // one scalar register, so with both its constants scalar each use would
    // first copy one into a vector register.  (Lit kernels run at a register
    // cap, and with more channels the registers would cost waves.)
    float tf_bias[C], tf_omc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        if constexpr (kLit || C > 2) {
            tf_bias[c] = tf[c].bias;
            tf_omc[c] = tf[c].one_m_curve;
        } else {
            asm("v_mov_b32 %0, %1" : "=v"(tf_bias[c]) : "v"(tf[c].bias));
            asm("v_mov_b32 %0, %1" : "=v"(tf_omc[c]) : "v"(tf[c].one_m_curve));
        }
    }

    const typename Variant<V>::Smp S = sampler_for<LARGE>(P);
    R step;
    if constexpr (LARGE) step = P.d64.step;
    else step = P.step;
    const R half_step = (R)0.5 * step;
    const float tau = P.tau;
    float Cr = 0.0f, Cg = 0.0f, Cb = 0.0f, A = 0.0f;
    int k = 0;
    // Divergent loop: a lane leaves after its last sample or once its opacity
    // reaches tau; the hardware execution mask then keeps it from
    // accumulating, and the wave leaves when the mask is empty (the wave-wide
    // ballot of the lanes' live flags).
    using Word = typename WordT<C, U16>::T;
    // Composite one sample from landed taps.  A lane leaves its state as it
    // is when `on` is false (past its last sample) or when the taps show the
    // sample to be transparent (its weight would be exactly 0); a wave skips
    // the arithmetic when that holds for all of its lanes, the common case in
    // the empty, below-floor space around stained structures.
    const bool clear_ok = kClear && P.clear.ok != 0;
    // Lit (kLit): each channel's colour term is scaled by its shade at the
    // sample point (the opacity is not).
    auto composite = [&](const Taps<Word>& t, bool on, int j) {
        if (!on || (clear_ok && transparent<C, U16>(t, P.clear))) return;
        float x[C];
        if constexpr (F16 && U16) {
            // data of at most 15 bits needs no clamp below the largest half
            if (P.half_clamp) interpolate<C, U16, F16, false, true>(t, x);
            else interpolate<C, U16, F16, false, false>(t, x);
        } else {
            interpolate<C, U16, F16>(t, x);
        }
        float shade[C];
        if constexpr (kLit) {
            const R sj = fma_r((R)j, step, half_step);
            const R q[3] = {fma_r(sj, d[0], pe[0]), fma_r(sj, d[1], pe[1]),
                            fma_r(sj, d[2], pe[2])};
            shade_at<C, U16, PAIRS, Word>(P, S, q, t, shade);
        }
        float amax = 0.0f, r = 0.0f, gg = 0.0f, bb = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float u = __builtin_amdgcn_fmed3f(fmaf(x[c], tf[c].scale, tf_bias[c]), 0.0f,
                                                   1.0f);
            const float g = u * fmaf(tf[c].curve, u, tf_omc[c]);
            amax = fmaxf(amax, tf[c].alpha_mul * g);
            const float gc = kLit ? g * shade[c] : g;
            r = fmaf(gc, tf[c].rgb[0], r);
            gg = fmaf(gc, tf[c].rgb[1], gg);
            bb = fmaf(gc, tf[c].rgb[2], bb);
        }
        const float a_s = fminf(amax, 1.0f);
        const float wgt = (1.0f - A) * a_s;
        Cr = fmaf(wgt, fminf(r, 1.0f), Cr);
        Cg = fmaf(wgt, fminf(gg, 1.0f), Cg);
        Cb = fmaf(wgt, fminf(bb, 1.0f), Cb);
        A = A + wgt;
    };
    auto fetch_at = [&](int j) -> Taps<Word> {
        const R sj = fma_r((R)j, step, half_step);
        return fetch<Word, PAIRS>(P.g, S, fma_r(sj, d[0], pe[0]), fma_r(sj, d[1], pe[1]),
                                  fma_r(sj, d[2], pe[2]));
    };
    // Empty-space skipping over macro cells (exact).  A lane marches through
    // segments: at a segment boundary (k >= kend) it looks up the macro cell
    // of sample k.  A cell shown transparent (its channel maxima all at or
    // below the thresholds) lets the lane jump past the samples whose low
    // corner lies in the cell, without loading their taps: each of them has
    // opacity exactly 0, so leaving it out changes no output bit and no
    // sample count.  Otherwise the cell's samples form the next segment,
    // composited one by one.  A cell's samples are one run of indices: per
    // axis, the clamped and floored position fma(fma(j, step, h), d, pe) is
    // monotone in j, so when samples k and jl both have their corner in the
    // cell, all between do.  jl comes from the cell's exit distance, folded
    // per axis into one multiply-add in sample-index units; it is checked
    // with the fetch's own arithmetic, and a failed check keeps sample k
    // alone.  One cell step per lane and iteration bounds the work a wave
    // spends on lanes that are between cells.
    const bool cells_on = !kLit && clear_ok && P.skip_cells != 0;
    const uint32_t cs = (uint32_t)P.g.cshift;
    R ex_mul[3], ex_add[3];  // crossing of stored coordinate b: index b ex_mul + ex_add
    {
        const R inv_step = (R)1 / step;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const R inv_d = d[a] != (R)0 ? (R)1 / d[a] : (R)0;
            ex_mul[a] = inv_d * inv_step;
            ex_add[a] = (-pe[a] * inv_d - half_step) * inv_step;
        }
    }
    auto cell_of = [&](int j, uint32_t (&c)[3]) {
        const R sj = fma_r((R)j, step, half_step);
#pragma unroll
        for (int a = 0; a < 3; ++a) c[a] = corner(S, fma_r(sj, d[a], pe[a]), a) >> cs;
    };
    // The last sample from k on whose low corner lies in cell c (the cell of
    // sample k): the exit estimate, checked with the fetch's own arithmetic.
    auto cell_last = [&](int k, const uint32_t (&c)[3]) -> int {
        R jx = (R)n;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (d[ax] != (R)0) {
                const R bound = (R)((d[ax] > (R)0 ? c[ax] + 1u : c[ax]) << cs);
                const R t = fma_r(bound, ex_mul[ax], ex_add[ax]);
                jx = t < jx ? t : jx;
            }
        }
        int jl = jx > (R)k ? (int)ceil_r(jx) - 1 : k;
        jl = jl < k ? k : (jl > n - 1 ? n - 1 : jl);
        if (jl > k) {
            uint32_t e[3];
            cell_of(jl, e);
            if (e[0] != c[0] || e[1] != c[1] || e[2] != c[2]) jl = k;
        }
        return jl;
    };
    // The first sample at or after lo, up to k, whose low corner lies in cell
    // c (the cell of sample k): the entry estimate, checked the same way (a
    // failed check keeps sample k alone).
    auto cell_first = [&](int k, const uint32_t (&c)[3], int lo) -> int {
        R jx = (R)lo;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (d[ax] != (R)0) {
                const R bound = (R)((d[ax] > (R)0 ? c[ax] : c[ax] + 1u) << cs);
                const R t = fma_r(bound, ex_mul[ax], ex_add[ax]);
                jx = t > jx ? t : jx;
            }
        }
        int jf = jx < (R)k ? (int)ceil_r(jx) : k;
        jf = jf > k ? k : (jf < lo ? lo : jf);
#pragma unroll
        for (int tries = 0; tries < 2 && jf < k; ++tries) {
            uint32_t e[3];
            cell_of(jf, e);
            if (e[0] == c[0] && e[1] == c[1] && e[2] == c[2]) return jf;
            ++jf;  // the estimate's sample lies on the cell's face, just outside
        }
        return k;
    };
    int count = n;
    int kend = cells_on ? 0 : n;  // samples below kend lie in a non-transparent cell
    if (n > 0) {
        // `count` is the sample count: n, or one past the sample at which
        // the opacity reached tau.
        if constexpr (kLit) {
            // Lit: one sample per iteration, no taps in flight across
            // iterations (the shading's loads need the registers: 6 waves
            // per SIMD instead of 4, measured 7 % faster than the pipeline
            // below), and macro cells only before the first and after the
            // last cell that is not transparent (jumps between those let the
            // lanes drift apart, and they shade in more iterations: measured
            // slower, 0.215 against 0.190 ms on the realistic frame).
            // The leading and trailing empty space is skipped over
            // transparent macro cells (exact, as below): the lane walks every
            // sample from the first cell that is not transparent to the end
            // of the last one.
            int kstop = n;
            if (clear_ok && P.skip_cells != 0) {
                bool more = true;
                while (more) {
                    uint32_t c[3];
                    cell_of(k, c);
                    const Word w = load_cell<Word>(P.g, S, c);
                    more = cell_clear<C, U16>(w, P.clear);
                    if (more) k = cell_last(k, c) + 1;
                    more = more && k < n;
                }
                more = k < n;
                while (more) {
                    uint32_t c[3];
                    cell_of(kstop - 1, c);
                    const Word w = load_cell<Word>(P.g, S, c);
                    more = cell_clear<C, U16>(w, P.clear);
                    if (more) kstop = cell_first(kstop - 1, c, k);
                    more = more && kstop > k;
                }
            }
            bool live = k < kstop;
            while (live) {
                composite(fetch_at(k), true, k);
                ++k;
                if (A >= tau) count = k;
                live = k < kstop && A < tau;
            }
        } else if (!cells_on) {
            // Without macro cells (a frame with nothing to skip, or the test
            // switched off): the same software pipeline over pairs of
            // samples, with no segment bookkeeping in the dependent chain of
            // a latency-bound launch (measured on the 256 x 256 mono frame:
            // 0.0255 ms through the segment loop below).  The pair's second
            // sample is left out on lanes that finished on its first.
            Taps<Word> a = fetch_at(k);
            bool live;
            do {
                const Taps<Word> b = fetch_at(k + 1);
                composite(a, true, k);
                ++k;
                const bool on = k < n && A < tau;
                a = fetch_at(k + 1);
                composite(b, on, k);
                k += on ? 1 : 0;
                live = on && k < n && A < tau;
            } while (live);
            count = k;
        } else {
            // Software pipeline over pairs of samples: the taps of the next
            // sample are in flight while the current one is interpolated and
            // composited, and the pair after is requested before the second is
            // composited.  A lane's last sample of a segment leaves the second
            // slot empty; the loop exits at the end of an iteration (a divergent
            // loop: finished lanes are masked off and the wave leaves when none
            // is live).  At equal sample index a wave's sample points lie on a
            // patch parallel to the face its rays entered through, which the
            // brick layout serves with few cache lines.  A fetch past a lane's
            // last sample reads a clamped, in-frame address and is unused.
            int ka = k;  // the sample whose taps `a` holds
            Taps<Word> a = fetch_at(k);
            bool live;
            do {
                if (k >= kend) {
                    uint32_t c[3];
                    cell_of(k, c);
                    const Word w = load_cell<Word>(P.g, S, c);
                    const int jl = cell_last(k, c);
                    if (cell_clear<C, U16>(w, P.clear)) k = jl + 1;
                    else kend = jl + 1;
                }
                if (k < kend) {
                    if (ka != k) {
                        a = fetch_at(k);
                        ka = k;
                    }
                    const Taps<Word> b = fetch_at(k + 1);
                    composite(a, true, k);
                    if (A >= tau) count = k + 1;
                    const bool on = A < tau && k + 1 < kend;
                    ka = on ? k + 2 : k + 1;
                    a = fetch_at(ka);
                    composite(b, on, k + 1);
                    if (on && A >= tau) count = k + 2;
                    k = ka;
                }
                live = k < n && A < tau;
            } while (live);
        }
    }

    if (valid) {
        const float T = 1.0f - A;
        float4 o;
        o.x = fmaf(T, P.bg[0], Cr);
        o.y = fmaf(T, P.bg[1], Cg);
        o.z = fmaf(T, P.bg[2], Cb);
        o.w = fmaf(T, P.bg[3], A);
        const size_t pix = ((size_t)eye * P.height + py) * P.width + px;
        reinterpret_cast<float4*>(P.out)[pix] = o;
        if (P.samples) P.samples[pix] = count;
    }
    if (P.nsamples) {
        // The request's composited samples: a wave-wide sum (every lane of
        // the wave arrives here), then one atomic add per wave with samples,
        // to the counter slot of its hardware block (device-scope atomics on
        // one address would serialise across the XCDs).
        int v = valid ? count : 0;
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0 && v != 0)
            atomicAdd(P.nsamples + (blockIdx.x % kCountSlots) * kCountStride,
                      (unsigned long long)v);
    }
}

// Blocks are dispatched round-robin over the 8 XCDs (block b to XCD b mod 8,
// as its (b / 8)-th block).  A launch orders its wave tiles by super-tiles of
// kSuperW x kSuperH tiles (32 x 32 pixels at 8 x 8 wave tiles), and the remap
// deals whole super-tiles to the XCDs in turn: an XCD's consecutive blocks
// render one compact patch whose rays share voxels in that XCD's L2.  Handing
// each XCD one contiguous eighth of the image instead leaves most XCDs idle
// (a volume seldom covers the whole image, so its rays crowd into a few
// eighths); larger super-tiles unbalance the XCDs again (measured, and
// simulated from per-pixel sample counts: 4 x 4 stays within 1-7 %).  The map
// is a bijection on [0, nblocks); blocks past the last whole round of 8 runs
// keep their index.
constexpr int kXcdRun = kSuperTiles;
__host__ __device__ __forceinline__ int xcd_remap(int b, int nblocks) {
    const int whole = nblocks - nblocks % (8 * kXcdRun);
    if (b >= whole) return b;
    const int i = b >> 3;  // the block's rank on its XCD
    return (((i / kXcdRun) << 3) + (b & 7)) * kXcdRun + i % kXcdRun;
}

// Tile (tx, ty) at position t of an eye's super-tile order.
__device__ __forceinline__ void tile_at(int t, int supers_x, int& tx, int& ty) {
    const int st = t / kSuperTiles, j = t - st * kSuperTiles;
    const int sy = st / supers_x, sx = st - sy * supers_x;
    tx = sx * kSuperW + j % kSuperW;
    ty = sy * kSuperH + j / kSuperW;
}

}  // namespace vr
