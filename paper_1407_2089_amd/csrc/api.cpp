// C ABI of libvr: contexts, resident volumes, transfer functions, the plain
// render call, validation and error reporting.  Batched launches live in
// batch.cpp, the serving loop in server.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>

#include "lib.h"

namespace vr {

static thread_local std::string t_err;

vr_status fail(vr_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return st;
}

vr_status ok() {
    t_err.clear();
    return VR_OK;
}

vr_status hip_fail(hipError_t e, const char* what) {
    return fail(VR_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

static bool finite3(const float* v) {
    return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

static int log2_exact(int v) {
    int s = 0;
    while ((1 << s) < v) ++s;
    return (1 << s) == v ? s : -1;
}

// Default brick edges by voxel-word size.  A wave's taps at one sample index
// cover a small patch parallel to the face its rays entered through; brick
// rows of about 16-36 bytes let one cache line serve several rows of that
// patch.  Measured on MI355X (2-channel uint16: 8 x 16 x 8 bricks 0.318 ms
// against 0.396 ms for 16^3 on a 1920x1080 stereo pair; 1-byte words prefer
// 16-wide rows; 8-byte words 8-wide).  The z edge of 8 keeps the halo
// overhead at 1.28-1.42x.  Large volumes (large-volume addressing) with
// 8-byte words take 4 x 16 x 8: measured on a 10173 x 3858 x 74 five-channel
// montage, 4.57 ms against 5.43 ms for 8 x 8 x 8 on a stereo overview whose
// rays lie ~7.5 voxels apart (5-word rows put a tap's y neighbour in the same
// cache line more often) and 1.46 against 1.64 ms zoomed in, for 5 % more
// storage.
static void brick_edges(const vr_volume_desc& d, int b[3], bool large) {
    const bool dflt = d.brick[0] == 0 && d.brick[1] == 0 && d.brick[2] == 0;
    if (!dflt) {
        for (int a = 0; a < 3; ++a) b[a] = d.brick[a];
        return;
    }
    const int w = word_bytes(d.channels, d.dtype == VR_U16);
    if (d.row_pairs) {  // measured per word size (layout sweep)
        b[0] = w == 1 ? 16 : w == 2 ? 8 : 4;
        b[1] = w == 2 ? 32 : 16;
        b[2] = w == 2 ? 8 : 16;
        return;
    }
    b[0] = w == 1 ? 16 : 8;
    b[1] = w >= 8 ? 8 : 16;
    b[2] = 8;
    if (large && w == 8) {
        b[0] = 4;
        b[1] = 16;
        b[2] = 8;
    }
}

static BrickGeom make_geom_with(const vr_volume_desc& d, bool large) {
    BrickGeom g{};
    int b[3];
    brick_edges(d, b, large);
    const int n[3] = {d.nx, d.ny, d.nz};
    for (int a = 0; a < 3; ++a) {
        g.n[a] = n[a];
        g.shift[a] = log2_exact(b[a]);
        g.nb[a] = (n[a] + 1 + b[a] - 1) / b[a];
        g.clamp_hi[a] = std::nextafter((float)(n[a] + 1), 0.0f);
    }
    g.pairs = d.row_pairs ? 1 : 0;
    g.row = g.pairs ? 2 * (b[0] + 1) : b[0] + 1;
    g.plane = g.pairs ? b[1] * g.row : (b[1] + 1) * g.row;
    g.brick = g.plane * (b[2] + 1);
    g.word = word_bytes(d.channels, d.dtype == VR_U16);
    const uint64_t words = (uint64_t)g.nb[0] * g.nb[1] * g.nb[2] * (uint64_t)g.brick;
    g.cell_off = (words * (uint64_t)g.word + 255u) & ~(uint64_t)255u;
    set_cell_shift(&g, kCellShift);
    return g;
}

void set_cell_shift(BrickGeom* g, int shift) {
    g->cshift = shift;
    for (int a = 0; a < 3; ++a) g->nc[a] = (g->n[a] >> shift) + 1;
    const uint64_t cells = (uint64_t)g->nc[0] * g->nc[1] * g->nc[2];
    g->frame_bytes = (g->cell_off + cells * (uint64_t)g->word + 255u) & ~(uint64_t)255u;
}

// Default bricks depend on whether the volume needs large-volume addressing
// at the regular default (the large default stores more halo, so such a
// volume still needs it at the large default).
BrickGeom make_geom(const vr_volume_desc& d) {
    const BrickGeom g = make_geom_with(d, false);
    const bool dflt = d.brick[0] == 0 && d.brick[1] == 0 && d.brick[2] == 0;
    return dflt && needs_large(d, g) ? make_geom_with(d, true) : g;
}

bool needs_large(const vr_volume_desc& d, const BrickGeom& g) {
    const uint64_t bricks = (uint64_t)g.nb[0] * g.nb[1] * g.nb[2];
    const uint64_t words = bricks * (uint64_t)g.brick;
    // The 32-bit sampler forms brick indices with 24-bit multiply-adds.
    return d.nx > kFloatAxis || d.ny > kFloatAxis || d.nz > kFloatAxis || words >= (1ull << 31) ||
           bricks >= (1ull << 24) || g.frame_bytes >= (1ull << 32);
}

vr_status check_desc(const vr_volume_desc* d) {
    if (!d) return fail(VR_ERR_INVALID_ARG, "volume description is NULL");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1 || d->nx > kMaxAxis || d->ny > kMaxAxis ||
        d->nz > kMaxAxis)
        return fail(VR_ERR_INVALID_ARG, "dimensions %d x %d x %d outside 1..%d", d->nx, d->ny,
                    d->nz, kMaxAxis);
    if (d->channels < 1 || d->channels > kMaxChannels)
        return fail(VR_ERR_INVALID_ARG, "channels = %d outside 1..%d", d->channels, kMaxChannels);
    if (d->frames < 1) return fail(VR_ERR_INVALID_ARG, "frames = %d < 1", d->frames);
    if (d->dtype == VR_U8) {
        if (d->bits != 8) return fail(VR_ERR_INVALID_ARG, "uint8 volumes need bits = 8");
    } else if (d->dtype == VR_U16) {
        if (d->bits < 9 || d->bits > 16)
            return fail(VR_ERR_INVALID_ARG, "uint16 volumes need bits in 9..16");
    } else {
        return fail(VR_ERR_INVALID_ARG, "dtype %d is neither VR_U8 nor VR_U16", d->dtype);
    }
    for (int a = 0; a < 3; ++a)
        if (!(d->spacing[a] > 0.0f) || !std::isfinite(d->spacing[a]))
            return fail(VR_ERR_INVALID_ARG, "spacing[%d] must be finite and > 0", a);
    if (!finite3(d->origin)) return fail(VR_ERR_INVALID_ARG, "origin must be finite");
    if (d->row_pairs != 0 && d->row_pairs != 1)
        return fail(VR_ERR_INVALID_ARG, "row_pairs = %d is neither 0 nor 1", d->row_pairs);
    if (d->row_pairs && word_bytes(d->channels, d->dtype == VR_U16) > max_pair_word(true))
        return fail(VR_ERR_INVALID_ARG,
                    "row pairs need voxel words of at most 8 bytes (at most 6 uint8 or 4 uint16 "
                    "channels; 8-byte words only in large volumes)");
    const bool dflt = d->brick[0] == 0 && d->brick[1] == 0 && d->brick[2] == 0;
    if (!dflt)
        for (int a = 0; a < 3; ++a)
            if (d->brick[a] != 4 && d->brick[a] != 8 && d->brick[a] != 16 && d->brick[a] != 32)
                return fail(VR_ERR_INVALID_ARG, "brick[%d] = %d is not 4, 8, 16 or 32", a,
                            d->brick[a]);
    const BrickGeom g = make_geom(*d);
    const uint64_t bricks = (uint64_t)g.nb[0] * g.nb[1] * g.nb[2];
    uint64_t total = 0;
    if (bricks >= (1ull << 32) || g.frame_bytes >= (1ull << 44) ||
        __builtin_mul_overflow(g.frame_bytes, (uint64_t)d->frames, &total))
        return fail(VR_ERR_INVALID_ARG, "one frame needs %llu bricks, %llu bytes (limits 2^32, 2^44)",
                    (unsigned long long)bricks, (unsigned long long)g.frame_bytes);
    return VR_OK;
}

static vr_status check_camera(const vr_camera& c, bool stereo) {
    if (c.projection != VR_ORTHO && c.projection != VR_PERSPECTIVE)
        return fail(VR_ERR_INVALID_ARG, "camera projection %d is unknown", c.projection);
    if (!finite3(c.center) || !finite3(c.forward) || !finite3(c.up))
        return fail(VR_ERR_INVALID_ARG, "camera vectors must be finite");
    const double f[3] = {c.forward[0], c.forward[1], c.forward[2]};
    const double u[3] = {c.up[0], c.up[1], c.up[2]};
    const double fn = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    const double un = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (!(fn > 0.0)) return fail(VR_ERR_INVALID_ARG, "camera forward is zero");
    const double x[3] = {f[1] * u[2] - f[2] * u[1], f[2] * u[0] - f[0] * u[2],
                         f[0] * u[1] - f[1] * u[0]};
    const double xn = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    if (!(un > 0.0) || !(xn > 1e-6 * fn * un))
        return fail(VR_ERR_INVALID_ARG, "camera up is zero or parallel to forward");
    if (c.projection == VR_PERSPECTIVE) {
        if (!(c.fov_y > 0.0f) || !(c.fov_y < 3.14159f))
            return fail(VR_ERR_INVALID_ARG, "fov_y must lie in (0, pi)");
        if (!(c.convergence > 0.0f) || !std::isfinite(c.convergence))
            return fail(VR_ERR_INVALID_ARG, "convergence must be finite and > 0");
        if (!(c.eye_separation >= 0.0f) || !std::isfinite(c.eye_separation))
            return fail(VR_ERR_INVALID_ARG, "eye_separation must be finite and >= 0");
    } else {
        if (stereo) return fail(VR_ERR_INVALID_ARG, "stereo needs a perspective camera");
        if (!(c.ortho_height > 0.0f) || !std::isfinite(c.ortho_height))
            return fail(VR_ERR_INVALID_ARG, "ortho_height must be finite and > 0");
    }
    return VR_OK;
}

vr_status check_request(const vr_ctx* ctx, const vr_render_req* r) {
    if (!r) return fail(VR_ERR_INVALID_ARG, "request is NULL");
    if (!r->vol) return fail(VR_ERR_INVALID_ARG, "request has no volume");
    if (r->vol->ctx != ctx) return fail(VR_ERR_INVALID_ARG, "volume belongs to another context");
    if (r->frame < 0 || r->frame >= r->vol->desc.frames)
        return fail(VR_ERR_INVALID_ARG, "frame %d outside 0..%d", r->frame,
                    r->vol->desc.frames - 1);
    if (r->width < 0 || r->height < 0 || r->width > 16384 || r->height > 16384)
        return fail(VR_ERR_INVALID_ARG, "image size %d x %d outside 0..16384", r->width,
                    r->height);
    if (r->stereo != 0 && r->stereo != 1) return fail(VR_ERR_INVALID_ARG, "stereo must be 0 or 1");
    if (!(r->step > 0.0f) || !std::isfinite(r->step))
        return fail(VR_ERR_INVALID_ARG, "step must be finite and > 0");
    if (!(r->term_alpha > 0.0f) || !(r->term_alpha <= 1.0f))
        return fail(VR_ERR_INVALID_ARG, "term_alpha must lie in (0, 1]");
    for (int q = 0; q < 4; ++q)
        if (!(r->background[q] >= 0.0f) || !(r->background[q] <= 1.0f))
            return fail(VR_ERR_INVALID_ARG, "background[%d] outside [0, 1]", q);
    if (r->precision != VR_FP32 && r->precision != VR_FP16)
        return fail(VR_ERR_INVALID_ARG, "precision %d is unknown", r->precision);
    vr_status st = check_camera(r->cam, r->stereo == 1);
    if (st != VR_OK) return st;
    const vr_light& L = r->light;
    if (L.enabled != 0 && L.enabled != 1)
        return fail(VR_ERR_INVALID_ARG, "light.enabled must be 0 or 1");
    if (L.enabled) {
        double n2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            if (!std::isfinite(L.direction[a]))
                return fail(VR_ERR_INVALID_ARG, "light.direction[%d] is not finite", a);
            n2 += (double)L.direction[a] * L.direction[a];
        }
        if (!(n2 > 0.0)) return fail(VR_ERR_INVALID_ARG, "light.direction is zero");
        if (!(L.ambient >= 0.0f) || !(L.ambient <= 1.0f))
            return fail(VR_ERR_INVALID_ARG, "light.ambient %g outside [0, 1]", L.ambient);
        if (!(L.diffuse >= 0.0f) || !(L.diffuse <= 1.0f))
            return fail(VR_ERR_INVALID_ARG, "light.diffuse %g outside [0, 1]", L.diffuse);
    }
    if ((int64_t)r->width * r->height > 0 && !r->out_rgba)
        return fail(VR_ERR_INVALID_ARG, "out_rgba is NULL");
    return VR_OK;
}

static vr_status check_transfer(const vr_transfer* t) {
    if (!t) return fail(VR_ERR_INVALID_ARG, "transfer function is NULL");
    if (!(t->lo >= 0.0f) || !(t->hi <= 1.0f) || !(t->lo < t->hi))
        return fail(VR_ERR_INVALID_ARG, "need 0 <= lo < hi <= 1 (lo %g, hi %g)", t->lo, t->hi);
    if (!(t->curve >= -1.0f) || !(t->curve <= 1.0f))
        return fail(VR_ERR_INVALID_ARG, "curve %g outside [-1, 1]", t->curve);
    if (!(t->alpha_mul >= 0.0f) || !(t->alpha_mul <= 2.0f))
        return fail(VR_ERR_INVALID_ARG, "alpha_mul %g outside [0, 2]", t->alpha_mul);
    for (int q = 0; q < 3; ++q)
        if (!(t->rgb[q] >= 0.0f) || !(t->rgb[q] <= 1.0f))
            return fail(VR_ERR_INVALID_ARG, "rgb[%d] outside [0, 1]", q);
    return VR_OK;
}

TileShape default_tile() { return TileShape{8, 8}; }

static void cross(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static void normalise(double a[3]) {
    const double n = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    for (int q = 0; q < 3; ++q) a[q] /= n;
}

// Largest raw tap value t (0 .. full) such that every field value the kernel
// can interpolate from taps that are all <= t gives u = 0 in its own FP32
// arithmetic, or -1 if there is none.  The FP32 lerp tree and weighted sum
// stay within a factor 1 + 2^-19 of the largest tap, the FP16 path (tap
// rounding, then three half-precision lerps, each adding at most three
// roundings of 2^-11 of the largest value) within 1 + 2^-7; the test allows
// 1 + 2^-6.  u_pre(x) = fma(x, scale, bias) is monotone in x, so checking the
// bound itself covers every smaller value.
static int32_t transparent_max(float scale, float bias, uint32_t full) {
    auto safe = [&](uint32_t t) {
        const double hi = (double)t * (1.0 + 1.0 / 64.0);
        float x = (float)hi;
        if ((double)x < hi) x = std::nextafter(x, INFINITY);
        return std::fma(x, scale, bias) <= 0.0f;
    };
    if (!safe(0)) return -1;
    uint32_t lo = 0, hi = full;  // safe(lo) holds
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo + 1) / 2;
        if (safe(mid)) lo = mid; else hi = mid - 1;
    }
    return (int32_t)lo;
}

// Thresholds of the transparent-sample test: a channel whose alpha
// multiplier is 0 (or that is hidden) never makes a sample opaque.  The test
// is switched off when the opaque-capable channels all have thresholds below
// 1 (floors at zero): then only all-zero taps could pass it, too rarely to
// pay for it.
static Transparent make_transparent(const ReqParams& P, uint32_t full) {
    Transparent t{};
    t.ok = 1;
    bool any = false, useful = false;
    for (int c = 0; c < kMaxChannels; ++c) {
        int32_t m = 65535;
        if (c < P.channels && P.tf[c].alpha_mul != 0.0f) {
            m = transparent_max(P.tf[c].scale, P.tf[c].bias, full);
            any = true;
            useful = useful || m >= 1;
        }
        if (m < 0) {
            t.ok = 0;
            m = 0;
        }
        t.tmax[c] = (uint32_t)m;
    }
    if (any && !useful) t.ok = 0;
    for (int q = 0; q < kMaxChannels / 2; ++q) t.tmax2[q] = t.tmax[2 * q] | t.tmax[2 * q + 1] << 16;
    auto lane = [&](int c) { return (std::min(t.tmax[c], 255u) << 8) | 255u; };
    t.byte_hi = lane(1) | lane(3) << 16;
    t.byte_lo = lane(0) | lane(2) << 16;
    return t;
}

extern "C" vr_status vr_test_transparent_max(float lo, float hi, int32_t bits, float* scale,
                                             float* bias, int32_t* tmax) {
    if (!(lo >= 0.0f) || !(hi <= 1.0f) || !(lo < hi) || bits < 8 || bits > 16 || !scale ||
        !bias || !tmax)
        return fail(VR_ERR_INVALID_ARG, "need 0 <= lo < hi <= 1, bits 8..16, outputs");
    // The same folding as make_params.
    const double full = std::ldexp(1.0, bits) - 1.0;
    const double range = (double)hi - (double)lo;
    *scale = (float)(1.0 / (full * range));
    *bias = (float)(-(double)lo / range);
    *tmax = transparent_max(*scale, *bias, (uint32_t)full);
    return ok();
}

void set_clamp_d64(const BrickGeom& g, ReqParams* P) {
    for (int a = 0; a < 3; ++a) P->d64.clamp_hi[a] = std::nextafter((double)(g.n[a] + 1), 0.0);
}

// Per-eye ray basis in double, rounded once to float.  Perspective: origin is
// the eye e_s = center + s (sep / 2) r; the unnormalised direction to pixel
// (sx, sy) is conv f - s (sep / 2) r + sx w r + sy h u.  Orthographic: the
// origin moves over the screen rectangle, the direction is f.
void make_params(const vr_render_req& r, const vr_transfer* tf_in, ReqParams* P) {
    std::memset(P, 0, sizeof *P);
    const vr_volume& v = *r.vol;
    const vr_volume_desc& d = v.desc;
    P->g = v.geom;
    P->vox = v.storage + (uint64_t)r.frame * v.geom.frame_bytes;
    P->channels = d.channels;
    P->variant = variant_index(d.channels, d.dtype == VR_U16, r.precision == VR_FP16,
                               v.geom.pairs != 0, v.large);
    set_clamp_d64(v.geom, P);

    const double full = std::ldexp(1.0, d.bits) - 1.0;
    for (int c = 0; c < d.channels; ++c) {
        const vr_transfer& t = tf_in[c];
        ChanTF& o = P->tf[c];
        const double range = (double)t.hi - (double)t.lo;
        o.scale = (float)(1.0 / (full * range));
        o.bias = (float)(-(double)t.lo / range);
        o.one_m_curve = (float)(1.0 - (double)t.curve);
        o.curve = t.curve;
        o.alpha_mul = t.visible ? t.alpha_mul : 0.0f;
        for (int q = 0; q < 3; ++q) o.rgb[q] = t.visible ? t.rgb[q] : 0.0f;
    }
    P->clear = make_transparent(*P, (uint32_t)full);

    double f[3] = {r.cam.forward[0], r.cam.forward[1], r.cam.forward[2]};
    const double up[3] = {r.cam.up[0], r.cam.up[1], r.cam.up[2]};
    normalise(f);
    double rt[3], u[3];
    cross(f, up, rt);
    normalise(rt);
    cross(rt, f, u);
    const double sp[3] = {d.spacing[0], d.spacing[1], d.spacing[2]};
    const double org[3] = {d.origin[0], d.origin[1], d.origin[2]};
    const double c[3] = {r.cam.center[0], r.cam.center[1], r.cam.center[2]};
    const double W = r.width > 0 ? r.width : 1, H = r.height > 0 ? r.height : 1;
    P->eyes = r.stereo ? 2 : 1;
    auto& D = P->d64;
    if (r.cam.projection == VR_PERSPECTIVE) {
        const double conv = r.cam.convergence;
        const double h = conv * std::tan(0.5 * (double)r.cam.fov_y);
        const double w = h * W / H;
        const double half_sep = 0.5 * (double)r.cam.eye_separation;
        for (int e = 0; e < P->eyes; ++e) {
            const double s = r.stereo ? (e == 0 ? -1.0 : 1.0) : 0.0;
            for (int a = 0; a < 3; ++a) {
                const double eye = c[a] + s * half_sep * rt[a];
                D.o0[e][a] = (eye - org[a]) / sp[a];
                D.base[e][a] = conv * f[a] - s * half_sep * rt[a];
            }
        }
        for (int a = 0; a < 3; ++a) {
            D.ou[a] = D.ov[a] = 0.0;
            D.du[a] = w * rt[a];
            D.dv[a] = h * u[a];
        }
        D.tmin = 0.0;
    } else {
        const double h = 0.5 * (double)r.cam.ortho_height;
        const double w = h * W / H;
        for (int a = 0; a < 3; ++a) {
            D.o0[0][a] = D.o0[1][a] = (c[a] - org[a]) / sp[a];
            D.ou[a] = w * rt[a] / sp[a];
            D.ov[a] = h * u[a] / sp[a];
            D.base[0][a] = D.base[1][a] = f[a];
            D.du[a] = D.dv[a] = 0.0;
        }
        D.tmin = -std::numeric_limits<double>::infinity();
    }
    for (int a = 0; a < 3; ++a) D.inv_sp[a] = 1.0 / sp[a];
    // The FP32 basis is the FP64 one rounded once.
    for (int a = 0; a < 3; ++a) {
        for (int e = 0; e < 2; ++e) {
            P->o0[e][a] = (float)D.o0[e][a];
            P->base[e][a] = (float)D.base[e][a];
        }
        P->ou[a] = (float)D.ou[a];
        P->ov[a] = (float)D.ov[a];
        P->du[a] = (float)D.du[a];
        P->dv[a] = (float)D.dv[a];
        P->inv_sp[a] = (float)D.inv_sp[a];
    }
    P->tmin = (float)D.tmin;
    if (r.light.enabled) {
        double l[3] = {r.light.direction[0], r.light.direction[1], r.light.direction[2]};
        normalise(l);
        const double smin = std::min(sp[0], std::min(sp[1], sp[2]));
        for (int a = 0; a < 3; ++a) {
            P->light.dir[a] = (float)l[a];
            P->light.gscale[a] = (float)(smin / sp[a]);
        }
        P->light.ka = r.light.ambient;
        P->light.kd = r.light.diffuse;
        P->light.on = 1;
    }
    P->step = r.step;
    D.step = (double)r.step;
    P->tau = r.term_alpha;
    const double bga = r.background[3];
    for (int q = 0; q < 3; ++q) P->bg[q] = (float)(bga * (double)r.background[q]);
    P->bg[3] = r.background[3];
    P->sx_scale = (float)(2.0 / W);
    P->sy_scale = (float)(2.0 / H);
    D.sx_scale = 2.0 / W;
    D.sy_scale = 2.0 / H;
    P->width = r.width;
    P->height = r.height;
    P->skip_cells = v.ctx->cell_skip ? 1 : 0;
    P->half_clamp = d.dtype == VR_U16 && d.bits == 16 ? 1 : 0;  // stored values <= 2^bits - 1
    P->out = r.out_rgba;
    P->samples = r.out_samples;
}

static void default_transfer(vr_transfer* t) {
    t->lo = 0.0f;
    t->hi = 1.0f;
    t->curve = 0.0f;
    t->alpha_mul = 1.0f;
    t->rgb[0] = t->rgb[1] = t->rgb[2] = 1.0f;
    t->visible = 1;
}

}  // namespace vr

using namespace vr;

extern "C" {

vr_status vr_init(int32_t device, uint64_t mem_budget_bytes, vr_ctx** out) {
    if (!out) return fail(VR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (device < -1) return fail(VR_ERR_INVALID_ARG, "device %d is invalid", device);
    vr_ctx* ctx = new vr_ctx();
    ctx->device = device;
    if (device == -1) {
        ctx->budget = mem_budget_bytes ? mem_budget_bytes : ~0ull;
        *out = ctx;
        return ok();
    }
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || device >= count) {
        delete ctx;
        return fail(VR_ERR_UNSUPPORTED, "HIP device %d is not available (hipGetDeviceCount: %s, %d devices)",
                    device, hipGetErrorString(e), count);
    }
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) {
        delete ctx;
        return hip_fail(e, "hipGetDeviceProperties");
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        delete ctx;
        return fail(VR_ERR_UNSUPPORTED, "device %d is %s; this library is built for gfx950",
                    device, prop.gcnArchName);
    }
    DeviceGuard dg(device);
    if (mem_budget_bytes == 0) {
        size_t free_b = 0, total_b = 0;
        if ((e = hipMemGetInfo(&free_b, &total_b)) != hipSuccess) {
            delete ctx;
            return hip_fail(e, "hipMemGetInfo");
        }
        const uint64_t reserve = 4ull << 30;
        mem_budget_bytes = free_b > reserve ? free_b - reserve : free_b / 2;
    }
    ctx->budget = mem_budget_bytes;
    vr_status st = noalloc_init(ctx);
    if (st != VR_OK) {
        delete ctx;
        return st;
    }
    *out = ctx;
    return ok();
}

vr_status vr_shutdown(vr_ctx* ctx) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    vr_status st = server_stop(ctx);
    if (st != VR_OK) return st;
    if (ctx->volumes.load() != 0)
        return fail(VR_ERR_BUSY, "%d volumes are still alive", ctx->volumes.load());
    DeviceGuard dg(ctx->device);
    for (auto& kv : ctx->batch_slots) batch_slot_destroy(kv.second);
    ctx->batch_slots.clear();
    if (ctx->device >= 0) noalloc_release(ctx);
    delete ctx;
    return ok();
}

vr_status vr_volume_storage_bytes(const vr_volume_desc* desc, uint64_t* bytes) {
    if (!bytes) return fail(VR_ERR_INVALID_ARG, "bytes is NULL");
    vr_status st = check_desc(desc);
    if (st != VR_OK) return st;
    const BrickGeom g = make_geom(*desc);
    *bytes = g.frame_bytes * (uint64_t)desc->frames;
    return ok();
}

vr_status vr_create_volume(vr_ctx* ctx, const vr_volume_desc* desc, void* dev_storage,
                           uint64_t storage_bytes, vr_volume** out) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    if (!out) return fail(VR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    vr_status st = check_desc(desc);
    if (st != VR_OK) return st;
    if (!dev_storage) return fail(VR_ERR_INVALID_ARG, "device storage is NULL");
    if (((uintptr_t)dev_storage & 255u) != 0)
        return fail(VR_ERR_INVALID_ARG, "device storage must be 256-byte aligned");
    BrickGeom g = make_geom(*desc);
    if (ctx->cell_shift != kCellShift) set_cell_shift(&g, ctx->cell_shift);
    const uint64_t need = g.frame_bytes * (uint64_t)desc->frames;
    if (storage_bytes < need)
        return fail(VR_ERR_OUT_OF_MEMORY, "storage holds %llu bytes, the volume needs %llu",
                    (unsigned long long)storage_bytes, (unsigned long long)need);
    const bool large = needs_large(*desc, g) || ctx->force_large;
    if (desc->row_pairs &&
        word_bytes(desc->channels, desc->dtype == VR_U16) > max_pair_word(large))
        return fail(VR_ERR_INVALID_ARG,
                    "row pairs of 8-byte voxel words need a large volume (an axis above %d "
                    "voxels, or a frame of 2^31 stored voxels or 4 GiB)",
                    kFloatAxis);
    uint64_t used = ctx->used.load();
    do {
        if (used + need > ctx->budget)
            return fail(VR_ERR_OUT_OF_MEMORY, "volume needs %llu bytes, %llu of %llu budgeted in use",
                        (unsigned long long)need, (unsigned long long)used,
                        (unsigned long long)ctx->budget);
    } while (!ctx->used.compare_exchange_weak(used, used + need));
    vr_volume* v = new vr_volume();
    v->ctx = ctx;
    v->desc = *desc;
    v->geom = g;
    v->large = large;
    v->storage = (uint8_t*)dev_storage;
    v->bytes = need;
    for (int c = 0; c < kMaxChannels; ++c) default_transfer(&v->tf[c]);
    ctx->volumes.fetch_add(1);
    *out = v;
    return ok();
}

vr_status vr_upload_frame(vr_volume* vol, int32_t frame, const void* dev_src, void* hip_stream) {
    if (!vol) return fail(VR_ERR_INVALID_ARG, "volume is NULL");
    if (frame < 0 || frame >= vol->desc.frames)
        return fail(VR_ERR_INVALID_ARG, "frame %d outside 0..%d", frame, vol->desc.frames - 1);
    if (!dev_src) return fail(VR_ERR_INVALID_ARG, "source is NULL");
    if (vol->ctx->device < 0) return fail(VR_ERR_UNSUPPORTED, "validation-only context");
    DeviceGuard dg(vol->ctx->device);
    hipError_t e = launch_relayout(vol->geom, vol->desc.channels, vol->desc.dtype == VR_U16,
                                   vol->desc.bits, dev_src,
                                   vol->storage + (uint64_t)frame * vol->geom.frame_bytes,
                                   (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "relayout launch");
    return ok();
}

vr_status vr_stream_frame(vr_volume* vol, int32_t slot, const void* host_src,
                          void* dev_staging, uint64_t staging_bytes, void* copy_stream,
                          void* render_stream) {
    if (!vol) return fail(VR_ERR_INVALID_ARG, "volume is NULL");
    if (slot < 0 || slot >= vol->desc.frames)
        return fail(VR_ERR_INVALID_ARG, "slot %d outside 0..%d", slot, vol->desc.frames - 1);
    if (!host_src || !dev_staging) return fail(VR_ERR_INVALID_ARG, "source or staging is NULL");
    const vr_volume_desc& d = vol->desc;
    const uint64_t raw = (uint64_t)d.nx * d.ny * d.nz * d.channels * (d.dtype == VR_U16 ? 2 : 1);
    if (staging_bytes < raw)
        return fail(VR_ERR_INVALID_ARG, "staging of %llu bytes, %llu needed",
                    (unsigned long long)staging_bytes, (unsigned long long)raw);
    if (copy_stream == render_stream)
        return fail(VR_ERR_INVALID_ARG, "copy and render streams must differ");
    if (vol->ctx->device < 0) return fail(VR_ERR_UNSUPPORTED, "validation-only context");
    DeviceGuard dg(vol->ctx->device);
    std::lock_guard<std::mutex> lk(vol->stream_mu);
    hipError_t e;
    if (!vol->relayout_stream) {
        if ((e = hipStreamCreateWithFlags(&vol->relayout_stream, hipStreamNonBlocking)) !=
                hipSuccess ||
            (e = hipEventCreateWithFlags(&vol->ev_before, hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "stream set-up");
        for (int h = 0; h < 2; ++h)
            if ((e = hipEventCreateWithFlags(&vol->ev_copied[h], hipEventDisableTiming)) !=
                    hipSuccess ||
                (e = hipEventCreateWithFlags(&vol->ev_free[h], hipEventDisableTiming)) !=
                    hipSuccess)
                return hip_fail(e, "stream set-up");
        vol->ev_loaded.assign((size_t)d.frames, nullptr);
    }
    if (!vol->ev_loaded[slot] &&
        (e = hipEventCreateWithFlags(&vol->ev_loaded[slot], hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "stream event");
    const hipStream_t cs = (hipStream_t)copy_stream, rs = (hipStream_t)render_stream;
    const hipStream_t ls = vol->relayout_stream;
    // Two frames of staging: alternate halves, so that a copy need not wait
    // for the previous frame's relayout.
    const int halves = staging_bytes >= 2 * raw ? 2 : 1;
    const int h = halves == 2 ? vol->next_half : 0;
    uint8_t* stage = (uint8_t*)dev_staging + (uint64_t)h * raw;
    // the copy waits until the relayout that last read this half is done
    if (vol->half_used[h] && (e = hipStreamWaitEvent(cs, vol->ev_free[h], 0)) != hipSuccess)
        return hip_fail(e, "stream ordering");
    if ((e = hipMemcpyAsync(stage, host_src, raw, hipMemcpyHostToDevice, cs)) != hipSuccess ||
        (e = hipEventRecord(vol->ev_copied[h], cs)) != hipSuccess)
        return hip_fail(e, "host to device copy");
    // the relayout writes the slot: it waits for the copy and for the renders
    // already enqueued (they may still read the slot)
    if ((e = hipEventRecord(vol->ev_before, rs)) != hipSuccess ||
        (e = hipStreamWaitEvent(ls, vol->ev_before, 0)) != hipSuccess ||
        (e = hipStreamWaitEvent(ls, vol->ev_copied[h], 0)) != hipSuccess)
        return hip_fail(e, "stream ordering");
    e = launch_relayout(vol->geom, d.channels, d.dtype == VR_U16, d.bits, stage,
                        vol->storage + (uint64_t)slot * vol->geom.frame_bytes, ls);
    if (e != hipSuccess) return hip_fail(e, "relayout launch");
    if ((e = hipEventRecord(vol->ev_free[h], ls)) != hipSuccess ||
        (e = hipEventRecord(vol->ev_loaded[slot], ls)) != hipSuccess)
        return hip_fail(e, "stream ordering");
    vol->half_used[h] = true;
    vol->next_half = halves == 2 ? 1 - h : 0;
    return ok();
}

vr_status vr_stream_ready(vr_volume* vol, int32_t slot, void* render_stream) {
    if (!vol) return fail(VR_ERR_INVALID_ARG, "volume is NULL");
    if (slot < 0 || slot >= vol->desc.frames)
        return fail(VR_ERR_INVALID_ARG, "slot %d outside 0..%d", slot, vol->desc.frames - 1);
    if (vol->ctx->device < 0) return fail(VR_ERR_UNSUPPORTED, "validation-only context");
    DeviceGuard dg(vol->ctx->device);
    std::lock_guard<std::mutex> lk(vol->stream_mu);
    if (vol->ev_loaded.empty() || !vol->ev_loaded[slot]) return ok();  // never streamed
    const hipError_t e = hipStreamWaitEvent((hipStream_t)render_stream, vol->ev_loaded[slot], 0);
    if (e != hipSuccess) return hip_fail(e, "stream ordering");
    return ok();
}

vr_status vr_destroy_volume(vr_volume* vol) {
    if (!vol) return fail(VR_ERR_INVALID_ARG, "volume is NULL");
    if (vol->in_flight.load() != 0)
        return fail(VR_ERR_BUSY, "%d served tickets still read this volume", vol->in_flight.load());
    if (vol->relayout_stream) {
        DeviceGuard dg(vol->ctx->device);
        (void)hipStreamSynchronize(vol->relayout_stream);
        (void)hipEventDestroy(vol->ev_before);
        for (int h = 0; h < 2; ++h) {
            (void)hipEventDestroy(vol->ev_copied[h]);
            (void)hipEventDestroy(vol->ev_free[h]);
        }
        for (hipEvent_t ev : vol->ev_loaded)
            if (ev) (void)hipEventDestroy(ev);
        (void)hipStreamDestroy(vol->relayout_stream);
    }
    vr_ctx* ctx = vol->ctx;
    ctx->used.fetch_sub(vol->bytes);
    ctx->volumes.fetch_sub(1);
    delete vol;
    return ok();
}

vr_status vr_set_transfer(vr_volume* vol, int32_t channel, const vr_transfer* tf) {
    if (!vol) return fail(VR_ERR_INVALID_ARG, "volume is NULL");
    if (channel < 0 || channel >= vol->desc.channels)
        return fail(VR_ERR_INVALID_ARG, "channel %d outside 0..%d", channel, vol->desc.channels - 1);
    vr_status st = check_transfer(tf);
    if (st != VR_OK) return st;
    std::lock_guard<std::mutex> lk(vol->tf_mu);
    vol->tf[channel] = *tf;
    return ok();
}

vr_status vr_render(vr_ctx* ctx, const vr_render_req* req, void* hip_stream) {
    if (!ctx) return fail(VR_ERR_INVALID_ARG, "context is NULL");
    vr_status st = check_request(ctx, req);
    if (st != VR_OK) return st;
    if (ctx->device < 0) return fail(VR_ERR_UNSUPPORTED, "validation-only context");
    if ((int64_t)req->width * req->height == 0) return ok();
    ReqParams P;
    {
        std::lock_guard<std::mutex> lk(req->vol->tf_mu);
        make_params(*req, req->vol->tf, &P);
    }
    DeviceGuard dg(ctx->device);
    hipError_t e = launch_render(P, ctx->plain_tile, ctx->clear_skip, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "render launch");
    return ok();
}

vr_status vr_debug_sample(vr_volume* vol, int32_t frame, const float* pts, int32_t n, float* out,
                          void* hip_stream) {
    if (!vol) return fail(VR_ERR_INVALID_ARG, "volume is NULL");
    if (frame < 0 || frame >= vol->desc.frames)
        return fail(VR_ERR_INVALID_ARG, "frame %d outside 0..%d", frame, vol->desc.frames - 1);
    if (n < 0) return fail(VR_ERR_INVALID_ARG, "n < 0");
    if (n > 0 && (!pts || !out)) return fail(VR_ERR_INVALID_ARG, "points or output is NULL");
    if (vol->ctx->device < 0) return fail(VR_ERR_UNSUPPORTED, "validation-only context");
    ReqParams P;
    std::memset(&P, 0, sizeof P);
    P.g = vol->geom;
    P.vox = vol->storage + (uint64_t)frame * vol->geom.frame_bytes;
    P.channels = vol->desc.channels;
    P.variant = variant_index(vol->desc.channels, vol->desc.dtype == VR_U16, false,
                              vol->geom.pairs != 0, vol->large);
    set_clamp_d64(vol->geom, &P);
    DeviceGuard dg(vol->ctx->device);
    hipError_t e = launch_debug_sample(P, pts, n, out, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "debug sample launch");
    return ok();
}

const char* vr_last_error(void) { return t_err.c_str(); }

}  // extern "C"
