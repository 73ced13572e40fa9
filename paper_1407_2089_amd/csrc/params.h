// Plain-old-data records shared by the host library and the HIP kernels.
//
// A ReqParams holds everything one render request needs on the device: the
// frame's brick-major voxel storage, the per-channel transfer-function
// coefficients, the per-eye ray basis, the sampling parameters and the output
// pointers.  The plain path passes it as a kernel argument; the batched path
// keeps an array of them in device memory.
#pragma once
#include <stdint.h>

namespace vr {

constexpr int kMaxChannels = 6;   // the viewer's six channel colours
constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kBlockThreads = 256;

// Data variant of a request: channels (1..6), voxel width, sample precision
// and storage layout.  Index = (channels - 1) + 6 u16 + 12 fp16 + 24 pairs
// + 48 large, where large marks a large volume (an axis above 8192 voxels or
// a frame of 2^31 words or 4 GiB and more: 64-bit addresses and FP64 ray
// positions).
constexpr int kVariants = 96;
inline constexpr int variant_index(int channels, bool u16, bool fp16, bool pairs,
                                   bool large = false) {
    return (channels - 1) + (u16 ? 6 : 0) + (fp16 ? 12 : 0) + (pairs ? 24 : 0) + (large ? 48 : 0);
}
inline constexpr int variant_channels(int v) { return v % 6 + 1; }
inline constexpr bool variant_u16(int v) { return (v / 6) % 2 != 0; }
inline constexpr bool variant_fp16(int v) { return (v / 12) % 2 != 0; }
inline constexpr bool variant_pairs(int v) { return (v / 24) % 2 != 0; }
inline constexpr bool variant_large(int v) { return v >= 48; }
// Variants that the batched launch serves (large ones take plain launches).
constexpr int kBatchVariants = 48;

// Axes up to kMaxAxis voxels; above kFloatAxis the FP32 sample position no
// longer resolves a thousandth of a voxel and the large variants take over.
constexpr int kFloatAxis = 8192;
constexpr int kMaxAxis = 16384;

// Bytes of one stored voxel word: all channels of a voxel side by side, the
// channel count rounded up to 1, 2, 4 or 8.
inline constexpr int word_bytes(int channels, bool u16) {
    return (channels == 1 ? 1 : channels == 2 ? 2 : channels <= 4 ? 4 : 8) * (u16 ? 2 : 1);
}

// The row-pair layout exists for 1-, 2- and 4-byte words: a plane's four
// taps are then two aligned 2-byte loads, one 8-byte or one 16-byte load.
// 8-byte words already take 16-byte loads without pairs and lose by pairs on
// densely sampled frames (cache footprint); only large volumes, usually seen
// undersampled, where a sample's fabric traffic counts more than its cache
// footprint, offer pairs of 8-byte words too (a plane's taps: 32 bytes).
inline constexpr int max_pair_word(bool large) { return large ? 8 : 4; }
inline constexpr bool variant_exists(int v) {
    return !variant_pairs(v) ||
           word_bytes(variant_channels(v), variant_u16(v)) <= max_pair_word(variant_large(v));
}

// Brick-major layout of one frame.  Stored coordinates s = i + 1 run over
// [0, n + 1] per axis (voxel -1 and voxel n are zero padding).  A trilinear
// sample at index-space p reads the 2x2x2 words starting at s0 = floor(p + 1)
// in [0, n]; bricks tile those origins B at a time and store B + 1 words per
// axis (one-word halo on the high side) so all eight taps sit in one brick.
//
// Row pairs (optional): a brick plane stores, for each local row ly in
// [0, By), rows ly and ly + 1 interleaved word by word, (x, ly), (x, ly + 1)
// for x = 0 .. Bx.  The four taps of a sample in one plane are then four
// consecutive words (one or two wide loads per plane instead of two narrow
// ones per row), at the price of storing every inner row twice.
//
// Macro cells (empty-space skipping): the low corners s0 in [0, n] are also
// grouped into cells of M = 2^cshift per axis.  After the bricks, each frame
// stores one word per cell (same packing as a voxel word) holding, per
// channel, the largest value any tap of a sample whose low corner lies in
// the cell can read: voxels of stored coordinates [c M, c M + M] per axis.
struct BrickGeom {
    int32_t n[3];       // voxels per axis
    int32_t shift[3];   // log2 of the brick edge per axis
    int32_t nb[3];      // bricks per axis = ceil((n + 1) / B)
    int32_t row;        // words per brick row = Bx + 1 (pairs: 2 (Bx + 1))
    int32_t plane;      // words per brick plane = (By + 1) row (pairs: By row)
    int32_t brick;      // words per brick = (Bz + 1) plane
    int32_t word;       // bytes per word
    int32_t pairs;      // 1: row-pair layout
    int32_t cshift;     // log2 of the macro-cell edge
    int32_t nc[3];      // macro cells per axis = floor(n / M) + 1
    float clamp_hi[3];  // largest float below n + 1 per axis
    int32_t pad_;
    uint64_t cell_off;  // byte offset of the cell table in a frame (multiple of 256)
    uint64_t frame_bytes; // bytes per frame, multiple of 256
};

constexpr int kCellShift = 3;  // macro cells of 8 x 8 x 8 low corners

// Transfer function of one channel, folded so that u = raw * scale + bias.
struct ChanTF {
    float scale, bias;   // 1 / ((2^bits - 1)(hi - lo)),  -lo / (hi - lo)
    float one_m_curve;   // 1 - curve
    float curve;
    float alpha_mul;     // 0 for an invisible channel
    float rgb[3];        // 0 for an invisible channel
};

// Global directional light of a request.  A channel's gradient is taken in
// raw units per voxel along each axis and scaled by gscale = min spacing /
// spacing (the world-space direction, kept in range); its shade is
// ka + kd * max(0, -g . dir / |g|), or ka + kd where g = 0.
struct Light {
    float dir[3];        // unit, world space, towards the light
    float ka, kd;        // ambient and diffuse weights
    float gscale[3];
    int32_t on;
};

// Transparency thresholds of a request.  A sample whose eight taps of every
// channel c are at most tmax[c] (raw units) has opacity exactly 0 in the
// kernel's own arithmetic (FP32 or FP16 interpolation), so compositing it
// leaves the pixel bitwise unchanged.  ok = 0 when some channel can never be
// shown transparent that way (then no sample is).
struct Transparent {
    uint32_t tmax2[3];   // (tmax[2q] | tmax[2q + 1] << 16), 16-bit lanes
    uint32_t tmax[6];    // per channel, 0 .. 65535
    // 4 uint8 channels (c0 | c1 << 8 | c2 << 16 | c3 << 24) read as 16-bit
    // lanes: a lane (hi << 8 | lo) is at most (t << 8 | 255) exactly when its
    // high byte is at most t.  byte_hi tests c1, c3 on the words themselves,
    // byte_lo tests c0, c2 on the words shifted left by 8 in each lane.
    uint32_t byte_hi, byte_lo;
    int32_t ok;
    int32_t pad_;
};

struct ReqParams {
    const uint8_t* vox;     // this frame's storage
    BrickGeom g;
    int32_t channels;
    int32_t variant;
    ChanTF tf[kMaxChannels];
    Transparent clear;      // transparent-sample test of this request's TFs
    Light light;
    // Rays.  Index-space origin p0 = o0[eye] + sx * ou + sy * ov; world
    // direction w = base[eye] + sx * du + sy * dv, unit-normalised, then
    // index-space direction d = w * inv_sp.
    float o0[2][3];
    float ou[3], ov[3];
    float base[2][3];
    float du[3], dv[3];
    float inv_sp[3];
    float tmin;             // 0 for perspective, -inf for orthographic
    float step, tau;
    float bg[4];            // bg_a * bg_rgb, bg_a
    float sx_scale, sy_scale; // 2 / W, 2 / H
    int32_t width, height, eyes;
    int32_t skip_cells;     // 1: rays jump over macro cells shown transparent
    int32_t half_clamp;     // 1: uint16 words may hold values above 65503 (16-bit
                            // data), which FP16 sampling clamps to the largest half
    float* out;             // [eyes][H][W][4]
    int32_t* samples;       // [eyes][H][W] or null
    // Samples composited, or null: kCountSlots counters kCountStride words
    // apart (one per 64-byte line), a wave adding to the one its block picks,
    // so that a request's waves do not all serialise on one address.
    unsigned long long* nsamples;
    // Large variants: the same ray basis in FP64, and the clamp bound of
    // stored coordinates (largest double below n + 1 per axis).
    struct {
        double o0[2][3], ou[3], ov[3], base[2][3], du[3], dv[3], inv_sp[3];
        double tmin, step, sx_scale, sy_scale;
        double clamp_hi[3];
    } d64;
};

constexpr int kCountSlots = 64;
constexpr int kCountStride = 8;

// Work decomposition: one item = one wave's pixel tile of one eye of one
// request.  Waves take items independently (a wave whose rays end early
// does not wait for the others of its block).
struct TileShape {
    int32_t wave_w, wave_h;   // pixels per wave (wave_w * wave_h = 64)
};

// The tiles of an eye are ordered super-tile by super-tile (row-major over
// super-tiles of kSuperW x kSuperH tiles, row-major inside each), padded to
// whole super-tiles; tiles of the padding lie past the image edge.
constexpr int kSuperW = 4, kSuperH = 4;
constexpr int kSuperTiles = kSuperW * kSuperH;
inline constexpr int64_t supers_across(int32_t width, const TileShape& ts) {
    const int64_t tx = ((int64_t)width + ts.wave_w - 1) / ts.wave_w;
    return (tx + kSuperW - 1) / kSuperW;
}
inline constexpr int64_t tiles_per_eye(int32_t width, int32_t height, const TileShape& ts) {
    const int64_t ty = ((int64_t)height + ts.wave_h - 1) / ts.wave_h;
    return supers_across(width, ts) * ((ty + kSuperH - 1) / kSuperH) * kSuperTiles;
}

}  // namespace vr
