/*
 * FP64 reference ray caster for multichannel direct volume rendering.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU path is
 * checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the GPU library, and it never takes an input produced by it.
 *
 * What it computes follows the paper's viewer (User Interface section):
 * multichannel voxel data (5-D x, y, z, t, channel images, Methods) sampled
 * along rays, each channel mapped through a floor / ceiling / curve / alpha-
 * multiplier transfer function, the sample's base alpha taken as the largest
 * channel value after the transfer function, and the view rendered once per
 * eye.  The paper draws view-aligned textured slices and states neither a
 * blend order nor an interpolation rule; the readings used here (ray casting,
 * trilinear interpolation with zero outside the grid, front-to-back
 * compositing with an early-termination threshold, an off-axis parallel-eye
 * stereo pair) are listed with every other reading in the design notes.
 * The optional lighting (one global directional light, normals from the
 * gradient over the 3 x 3 x 3 neighbourhood, same section) is read as
 * central differences of the trilinear field and Lambert shading of each
 * channel's colour; it leaves opacity untouched.
 *
 * Everything is IEEE double, written as the plain definition, one pixel at a
 * time.  Threads only split the pixel list; they do not change arithmetic.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_CHANNELS 8

typedef struct {
    int32_t nx, ny, nz, channels; /* channels 1 .. ORC_MAX_CHANNELS */
    int32_t bytes_per_voxel; /* 1 = uint8, 2 = uint16                         */
    int32_t bits;            /* full scale is 2^bits - 1 (8, 12 or 16)       */
    double spacing[3];       /* world units per voxel along x, y, z           */
    double origin[3];        /* world position of voxel (0, 0, 0)             */
    const void* data;        /* one frame, [channels][nz][ny][nx], row-major  */
} orc_volume;

typedef struct {
    double lo, hi;     /* floor and ceiling on normalised intensity           */
    double curve;      /* kappa in [-1, 1]; 0 is a linear ramp                */
    double alpha_mul;  /* alpha multiplier in [0, 2]; 1 is the slider centre  */
    double rgb[3];     /* channel colour                                      */
    int32_t visible;
} orc_transfer;

typedef struct {
    int32_t projection; /* 0 orthographic, 1 perspective                      */
    double center[3], forward[3], up[3];
    double fov_y;        /* radians, perspective                              */
    double ortho_height; /* world units, orthographic                         */
    double eye_separation, convergence;
} orc_camera;

typedef struct {
    int32_t width, height;
    int32_t eye;          /* -1 left, 0 centre (mono), +1 right               */
    double step;          /* world distance between samples                   */
    double term_alpha;    /* stop once accumulated opacity reaches this       */
    double band_eps;      /* width of the termination band (acceptance rule)  */
    double background[4];
    /* Global directional light (the viewer's lighting check box). */
    int32_t lit;          /* 0 off, 1 on                                      */
    double light_dir[3];  /* world space, pointing towards the light          */
    double ambient, diffuse;
} orc_view;

/* Per-pixel results. */
typedef struct {
    double* rgba;          /* [npix][4]  the ray's result                        */
    int32_t* samples;      /* [npix]     samples composited before stopping      */
    int32_t* nominal;      /* [npix]     samples in the box, ignoring stopping   */
    double* count_margin;  /* [npix]     distance of the real-valued sample count
                                         to the nearest integer (1 if no hit)    */
    double* band_lo;       /* [npix][4]  componentwise min over the band: results of
                                         the stops k with |A_k - tau| <= eps and
                                         of the stop right after each of them    */
    double* band_hi;       /* [npix][4]  componentwise max over the band         */
    int32_t* band_k;       /* [npix][2]  smallest and largest band member count,
                                         -1 when the band is empty               */
    double* lit_margin;    /* [npix]     bound on the colour change that FP32
                                         rounding of the gradients can cause
                                         (0 when unlit)                          */
    double* members;       /* NULL, or [npix][member_cap][4]: band member
                                         R_k of stop count k written at
                                         [k - smallest member count]             */
    int32_t member_cap;
} orc_result;

/* ---------------------------------------------------------------- sampling */

/* Raw voxel value of channel c at integer index (i, j, k); zero outside the
 * grid (the address mode at the volume edge). */
static double voxel(const orc_volume* v, int c, long i, long j, long k)
{
    if (i < 0 || j < 0 || k < 0 || i >= v->nx || j >= v->ny || k >= v->nz) return 0.0;
    size_t idx = (((size_t)c * (size_t)v->nz + (size_t)k) * (size_t)v->ny + (size_t)j)
                     * (size_t)v->nx + (size_t)i;
    if (v->bytes_per_voxel == 1) return (double)((const uint8_t*)v->data)[idx];
    return (double)((const uint16_t*)v->data)[idx];
}

/* Trilinear field of every channel at index-space position p: the weighted sum
 * of the eight surrounding voxels, weight = product over axes of f or (1 - f).
 * Result is in raw intensity units (not normalised). */
int orc_sample(const orc_volume* v, const double p[3], double* out)
{
    double fl[3], f[3];
    for (int a = 0; a < 3; ++a) {
        fl[a] = floor(p[a]);
        f[a] = p[a] - fl[a];
    }
    long i0 = (long)fl[0], j0 = (long)fl[1], k0 = (long)fl[2];
    for (int c = 0; c < v->channels; ++c) {
        double sum = 0.0;
        for (int dz = 0; dz <= 1; ++dz)
            for (int dy = 0; dy <= 1; ++dy)
                for (int dx = 0; dx <= 1; ++dx) {
                    double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1])
                             * (dz ? f[2] : 1.0 - f[2]);
                    sum += w * voxel(v, c, i0 + dx, j0 + dy, k0 + dz);
                }
        out[c] = sum;
    }
    return 0;
}

/* orc_sample over n points [n][3]; out is [n][channels]. */
int orc_sample_points(const orc_volume* v, const double* pts, int64_t n, double* out)
{
    for (int64_t q = 0; q < n; ++q) orc_sample(v, pts + 3 * q, out + (size_t)v->channels * q);
    return 0;
}

/* ---------------------------------------------------------------- lighting */

/* Gradient of every channel's trilinear field at index-space position p, in
 * raw intensity per world unit: the central difference over one voxel along
 * each axis, (x(p + e_a) - x(p - e_a)) / (2 spacing_a).  The six points are
 * the face neighbours of p in the 3 x 3 x 3 neighbourhood at unit offsets
 * that the viewer's lighting takes the gradient from.  g is [channels][3]. */
int orc_gradient(const orc_volume* v, const double p[3], double* g)
{
    if (v->channels < 1 || v->channels > ORC_MAX_CHANNELS) return -1;
    double hi[ORC_MAX_CHANNELS], lo[ORC_MAX_CHANNELS];
    for (int a = 0; a < 3; ++a) {
        double q[3] = {p[0], p[1], p[2]};
        q[a] = p[a] + 1.0;
        orc_sample(v, q, hi);
        q[a] = p[a] - 1.0;
        orc_sample(v, q, lo);
        for (int c = 0; c < v->channels; ++c)
            g[3 * c + a] = (hi[c] - lo[c]) / (2.0 * v->spacing[a]);
    }
    return 0;
}

/* orc_gradient over n points [n][3]; out is [n][channels][3]. */
int orc_gradient_points(const orc_volume* v, const double* pts, int64_t n, double* out)
{
    for (int64_t q = 0; q < n; ++q)
        orc_gradient(v, pts + 3 * q, out + (size_t)3 * v->channels * q);
    return 0;
}

/* Smallest and largest raw value of channel c among the eight voxels around
 * p (zero outside the grid). */
static void tap_range(const orc_volume* v, int c, const double p[3], double* mn, double* mx)
{
    long i0 = (long)floor(p[0]), j0 = (long)floor(p[1]), k0 = (long)floor(p[2]);
    *mn = INFINITY;
    *mx = -INFINITY;
    for (int dz = 0; dz <= 1; ++dz)
        for (int dy = 0; dy <= 1; ++dy)
            for (int dx = 0; dx <= 1; ++dx) {
                double w = voxel(v, c, i0 + dx, j0 + dy, k0 + dz);
                if (w < *mn) *mn = w;
                if (w > *mx) *mx = w;
            }
}

/* Lambert shading of each channel at p: the channel's surface normal is the
 * unit vector against its gradient, n = -g / |g| (pointing out of bright
 * structure), and shade = ambient + diffuse * max(0, n . l) with l the unit
 * light direction; a channel with zero gradient has no surface and takes
 * ambient + diffuse.  margin[c] bounds how far the shade can move when the
 * gradient carries an absolute error of up to 2^-19 of the largest voxel
 * value it reads per difference (FP32 lerp trees): a direction error of at
 * most 2 |dg| / |g|; zero for an axis whose sixteen voxels are all equal
 * (every lerp of equal values is exact).  shade and margin are [channels]. */
int orc_shade(const orc_volume* v, const orc_view* view, const double p[3], double* shade,
              double* margin)
{
    if (v->channels < 1 || v->channels > ORC_MAX_CHANNELS) return -1;
    double g[3 * ORC_MAX_CHANNELS];
    double l[3] = {view->light_dir[0], view->light_dir[1], view->light_dir[2]};
    double ln = sqrt(l[0] * l[0] + l[1] * l[1] + l[2] * l[2]);
    for (int a = 0; a < 3; ++a) l[a] /= ln;
    orc_gradient(v, p, g);
    for (int c = 0; c < v->channels; ++c) {
        const double* gc = g + 3 * c;
        double gn = sqrt(gc[0] * gc[0] + gc[1] * gc[1] + gc[2] * gc[2]);
        double diff = 1.0;
        if (gn > 0.0) {
            double d = -(gc[0] * l[0] + gc[1] * l[1] + gc[2] * l[2]) / gn;
            diff = d > 0.0 ? d : 0.0;
        }
        shade[c] = view->ambient + view->diffuse * diff;
        double err2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double q[3] = {p[0], p[1], p[2]}, mn1, mx1, mn2, mx2;
            q[a] = p[a] + 1.0;
            tap_range(v, c, q, &mn1, &mx1);
            q[a] = p[a] - 1.0;
            tap_range(v, c, q, &mn2, &mx2);
            double mn = mn1 < mn2 ? mn1 : mn2, mx = mx1 > mx2 ? mx1 : mx2;
            if (mn == mx) continue;
            double e = ldexp(mx, -19) / (2.0 * v->spacing[a]);
            err2 += e * e;
        }
        double rel = err2 == 0.0 ? 0.0 : (gn > 0.0 ? 2.0 * sqrt(err2) / gn : 1.0);
        margin[c] = view->diffuse * (rel < 1.0 ? rel : 1.0);
    }
    return 0;
}

/* ------------------------------------------------------- transfer function */

/* One channel's transfer function at normalised intensity x: returns g and
 * writes the channel's alpha.  u = clamp((x - lo) / (hi - lo)), curve
 * g = (1 - kappa) u + kappa u^2, alpha = multiplier * g. */
static double transfer(const orc_transfer* t, double x, double* alpha)
{
    double u = (x - t->lo) / (t->hi - t->lo);
    if (u < 0.0) u = 0.0;
    if (u > 1.0) u = 1.0;
    double g = (1.0 - t->curve) * u + t->curve * u * u;
    *alpha = t->alpha_mul * g;
    return g;
}

/* Classification of one sample: base alpha is the largest visible channel
 * alpha (capped at 1), colour is the capped sum of the channels' colours,
 * each scaled by the channel's shade when the view is lit (shade NULL:
 * unlit).  *lit_err receives the bound on the colour change that the shade
 * margins allow (sum over channels of value x largest colour component x
 * margin). */
static void classify(const orc_volume* v, const orc_transfer* tf, const double* field,
                     const double* shade, const double* margin, double* alpha_s,
                     double rgb_s[3], double* lit_err)
{
    double full_scale = ldexp(1.0, v->bits) - 1.0;
    double amax = 0.0, rgb[3] = {0.0, 0.0, 0.0}, err = 0.0;
    for (int c = 0; c < v->channels; ++c) {
        if (!tf[c].visible) continue;
        double a;
        double g = transfer(&tf[c], field[c] / full_scale, &a);
        if (a > amax) amax = a;
        double s = shade ? shade[c] : 1.0;
        for (int q = 0; q < 3; ++q) rgb[q] += g * s * tf[c].rgb[q];
        if (shade) {
            double cmax = tf[c].rgb[0];
            if (tf[c].rgb[1] > cmax) cmax = tf[c].rgb[1];
            if (tf[c].rgb[2] > cmax) cmax = tf[c].rgb[2];
            err += g * cmax * margin[c];
        }
    }
    *alpha_s = amax < 1.0 ? amax : 1.0;
    for (int q = 0; q < 3; ++q) rgb_s[q] = rgb[q] < 1.0 ? rgb[q] : 1.0;
    *lit_err = err;
}

/* ------------------------------------------------------------------ camera */

static void cross3(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static void normalise3(double a[3])
{
    double n = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    a[0] /= n;
    a[1] /= n;
    a[2] /= n;
}

/* World-space ray of pixel (i, j).  Pixel centres sit at (i + 1/2, j + 1/2)
 * and row 0 is the top of the image.  Perspective: the eye is displaced by
 * half the separation along the right vector and looks through a screen
 * shared by both eyes at the convergence distance (parallel eyes, off-axis
 * frustum).  Orthographic: parallel rays along forward, unbounded in t. */
static void pixel_ray(const orc_camera* cam, const orc_view* view, int i, int j,
                      double org[3], double dir[3], double* tmin)
{
    double f[3] = {cam->forward[0], cam->forward[1], cam->forward[2]};
    normalise3(f);
    double r[3];
    cross3(f, cam->up, r);
    normalise3(r);
    double u[3];
    cross3(r, f, u);

    double sx = 2.0 * (i + 0.5) / view->width - 1.0;
    double sy = 1.0 - 2.0 * (j + 0.5) / view->height;

    if (cam->projection == 1) {
        double h = cam->convergence * tan(0.5 * cam->fov_y);
        double w = h * view->width / view->height;
        double eye_off = view->eye * 0.5 * cam->eye_separation;
        double screen[3];
        for (int a = 0; a < 3; ++a) {
            org[a] = cam->center[a] + eye_off * r[a];
            screen[a] = cam->center[a] + cam->convergence * f[a] + sx * w * r[a] + sy * h * u[a];
            dir[a] = screen[a] - org[a];
        }
        normalise3(dir);
        *tmin = 0.0;
    } else {
        double h = 0.5 * cam->ortho_height;
        double w = h * view->width / view->height;
        for (int a = 0; a < 3; ++a) {
            org[a] = cam->center[a] + sx * w * r[a] + sy * h * u[a];
            dir[a] = f[a];
        }
        *tmin = -INFINITY;
    }
}

/* ------------------------------------------------------------------- march */

/* Output of a ray stopped after its current sample: the accumulated colour
 * plus the background seen through the remaining transparency. */
static void finish(const orc_view* view, const double C[3], double A, double out[4])
{
    const double* bg = view->background;
    for (int q = 0; q < 3; ++q) out[q] = C[q] + (1.0 - A) * bg[3] * bg[q];
    out[3] = A + (1.0 - A) * bg[3];
}

static void band_add(double lo[4], double hi[4], int32_t k_range[2], const double r[4], int k)
{
    if (k_range[0] < 0) {
        memcpy(lo, r, 4 * sizeof(double));
        memcpy(hi, r, 4 * sizeof(double));
        k_range[0] = k_range[1] = k;
        return;
    }
    for (int q = 0; q < 4; ++q) {
        if (r[q] < lo[q]) lo[q] = r[q];
        if (r[q] > hi[q]) hi[q] = r[q];
    }
    if (k < k_range[0]) k_range[0] = k;
    if (k > k_range[1]) k_range[1] = k;
}

/* Records band member R_k (the result of the ray stopped after k samples)
 * of the pixel in `slot`; the band is one run of stop counts (opacity never
 * decreases), starting at k0. */
static void member(const orc_result* res, int64_t slot, int k0, int k, const double r[4])
{
    if (!res->members || k - k0 >= res->member_cap) return;
    memcpy(res->members + 4 * ((size_t)slot * (size_t)res->member_cap + (size_t)(k - k0)), r,
           4 * sizeof(double));
}

typedef struct {
    const orc_volume* vol;
    const orc_transfer* tf;
    const orc_camera* cam;
    const orc_view* view;
    const int64_t* pixels;
    const int32_t* stop_at; /* per listed pixel: -1, or the forced stop count */
    int64_t npix;
    orc_result res;
    int64_t next; /* shared work counter */
} job_t;

static void render_pixel(const job_t* jb, int64_t slot)
{
    const orc_volume* v = jb->vol;
    const orc_view* view = jb->view;
    int64_t pix = jb->pixels ? jb->pixels[slot] : slot;
    int i = (int)(pix % view->width), j = (int)(pix / view->width);

    double org[3], dir[3], tmin;
    pixel_ray(jb->cam, view, i, j, org, dir, &tmin);

    /* Index space: p(t) = p0 + t * d_idx, t measured in world distance. */
    double p0[3], d[3];
    int n_ax[3] = {v->nx, v->ny, v->nz};
    for (int a = 0; a < 3; ++a) {
        p0[a] = (org[a] - v->origin[a]) / v->spacing[a];
        d[a] = dir[a] / v->spacing[a];
    }

    /* Slab clip against the extended box [-1, n] on each axis. */
    double t_enter = tmin, t_exit = INFINITY;
    int miss = 0;
    for (int a = 0; a < 3; ++a) {
        double lo = -1.0, hi = (double)n_ax[a];
        if (d[a] == 0.0) {
            if (p0[a] < lo || p0[a] > hi) miss = 1;
            continue;
        }
        double t1 = (lo - p0[a]) / d[a], t2 = (hi - p0[a]) / d[a];
        double tl = t1 < t2 ? t1 : t2, th = t1 < t2 ? t2 : t1;
        if (tl > t_enter) t_enter = tl;
        if (th < t_exit) t_exit = th;
    }
    if (!(t_enter < t_exit)) miss = 1;

    double C[3] = {0.0, 0.0, 0.0}, A = 0.0, out[4];
    double* rgba = jb->res.rgba + 4 * slot;
    double* blo = jb->res.band_lo + 4 * slot;
    double* bhi = jb->res.band_hi + 4 * slot;
    int32_t* bk = jb->res.band_k + 2 * slot;
    bk[0] = bk[1] = -1;

    const double tau = view->term_alpha, eps = view->band_eps;
    /* A forced stop count k >= 0 gives R_k, the result of the ray stopped
     * after exactly k samples (or after its last one), whatever its opacity:
     * the members of the termination band are such results. */
    const int32_t target = jb->stop_at ? jb->stop_at[slot] : -1;
    int stopped = 0, k_stop = 0, nominal = 0;
    double margin = 1.0, margin_lit = 0.0;

    if (!miss) {
        double span = (t_exit - t_enter) / view->step - 0.5;
        margin = fabs(span - nearbyint(span));
        finish(view, C, A, out);
        /* Band: stops k with |A_k - tau| <= eps, and the stop one sample
         * after each of them (a ray whose opacity is that close to tau may
         * decide A >= tau either way, and then stops at the next sample). */
        int prev_in = fabs(A - tau) <= eps;
        if (prev_in) {
            band_add(blo, bhi, bk, out, 0);
            member(&jb->res, slot, 0, 0, out);
        }
        if (target == 0) {
            memcpy(rgba, out, sizeof out);
            stopped = 1;
        }

        double field[ORC_MAX_CHANNELS], shade[ORC_MAX_CHANNELS], smargin[ORC_MAX_CHANNELS];
        double lit_err;
        for (int k = 0;; ++k) {
            double t = t_enter + (k + 0.5) * view->step;
            if (!(t < t_exit)) break;
            nominal = k + 1;
            if (stopped && A > tau + eps && !prev_in && target < 0) continue; /* only counting now */
            double p[3];
            for (int a = 0; a < 3; ++a) p[a] = p0[a] + t * d[a];
            orc_sample(v, p, field);
            if (view->lit) orc_shade(v, view, p, shade, smargin);
            double a_s, rgb_s[3];
            classify(v, jb->tf, field, view->lit ? shade : NULL, smargin, &a_s, rgb_s,
                     &lit_err);
            margin_lit += (1.0 - A) * a_s * lit_err;
            for (int q = 0; q < 3; ++q) C[q] += (1.0 - A) * a_s * rgb_s[q];
            A += (1.0 - A) * a_s;
            finish(view, C, A, out);
            const int in = fabs(A - tau) <= eps;
            if (in || prev_in) {
                band_add(blo, bhi, bk, out, k + 1);
                member(&jb->res, slot, bk[0], k + 1, out);
            }
            prev_in = in;
            if (!stopped) {
                memcpy(rgba, out, sizeof out);
                k_stop = k + 1;
                if (target >= 0 ? k + 1 >= target : A >= tau) stopped = 1;
            }
        }
        if (!stopped && k_stop == 0) { /* entered the box but took no sample */
            finish(view, C, 0.0, rgba);
        }
    } else {
        finish(view, C, A, rgba);
    }
    if (bk[0] < 0) {
        memcpy(blo, rgba, 4 * sizeof(double));
        memcpy(bhi, rgba, 4 * sizeof(double));
    }
    jb->res.samples[slot] = k_stop;
    jb->res.nominal[slot] = nominal;
    jb->res.count_margin[slot] = margin;
    jb->res.lit_margin[slot] = margin_lit;
}

static void* worker(void* arg)
{
    job_t* jb = (job_t*)arg;
    const int64_t chunk = 64;
    for (;;) {
        int64_t s = __atomic_fetch_add(&jb->next, chunk, __ATOMIC_RELAXED);
        if (s >= jb->npix) break;
        int64_t e = s + chunk < jb->npix ? s + chunk : jb->npix;
        for (int64_t q = s; q < e; ++q) render_pixel(jb, q);
    }
    return NULL;
}

/* Render the pixels listed in `pixels` (linear index j * width + i), or the
 * whole image in row-major order when `pixels` is NULL (npix must then be
 * width * height).  stop_at (NULL, or one entry per rendered pixel): an entry
 * k >= 0 stops that ray after exactly k samples (after its last sample if it
 * has fewer) instead of at the termination threshold, which yields the band
 * member R_k of the acceptance rule; -1 keeps the threshold.  members (NULL,
 * or [npix][member_cap][4]): every band member R_k met on the march, at
 * [k - band_k[0]] of its pixel (the first member_cap of them).  nthreads <= 1
 * runs on the calling thread.  Returns 0, or -1 on an invalid argument. */
int orc_render(const orc_volume* vol, const orc_transfer* tf, const orc_camera* cam,
               const orc_view* view, const int64_t* pixels, const int32_t* stop_at,
               int64_t npix,
               double* rgba, int32_t* samples, int32_t* nominal, double* count_margin,
               double* band_lo, double* band_hi, int32_t* band_k, double* lit_margin,
               double* members, int32_t member_cap, int nthreads)
{
    if (!vol || !tf || !cam || !view || !rgba || !samples || !nominal || !count_margin
        || !band_lo || !band_hi || !band_k || !lit_margin)
        return -1;
    if (view->width <= 0 || view->height <= 0 || !(view->step > 0.0)) return -1;
    if (vol->channels < 1 || vol->channels > ORC_MAX_CHANNELS) return -1;
    if (view->lit && !(view->light_dir[0] != 0.0 || view->light_dir[1] != 0.0
                       || view->light_dir[2] != 0.0))
        return -1;
    if (!pixels && npix != (int64_t)view->width * view->height) return -1;

    job_t jb;
    jb.vol = vol;
    jb.tf = tf;
    jb.cam = cam;
    jb.view = view;
    jb.pixels = pixels;
    jb.stop_at = stop_at;
    jb.npix = npix;
    jb.res.rgba = rgba;
    jb.res.samples = samples;
    jb.res.nominal = nominal;
    jb.res.count_margin = count_margin;
    jb.res.band_lo = band_lo;
    jb.res.band_hi = band_hi;
    jb.res.band_k = band_k;
    jb.res.lit_margin = lit_margin;
    jb.res.members = member_cap > 0 ? members : NULL;
    jb.res.member_cap = member_cap;
    jb.next = 0;

    if (nthreads <= 1) {
        worker(&jb);
        return 0;
    }
    if (nthreads > 1024) nthreads = 1024;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    if (!th) return -1;
    int started = 0;
    for (; started < nthreads; ++started)
        if (pthread_create(&th[started], NULL, worker, &jb) != 0) break;
    if (started == 0) worker(&jb);
    for (int q = 0; q < started; ++q) pthread_join(th[q], NULL);
    free(th);
    return 0;
}
