/*
 * dpvr_oracle.c -- plain FP64 CPU oracle for data-parallel volume ray casting
 * with sort-last compositing.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code with the GPU library.
 *
 * What it computes (one function per step, each the plain definition):
 *   - camera rays (perspective / orthographic)                 oc_ray
 *   - a brick's partial image: premultiplied RGBA + depth key  oc_render_brick
 *     (ray/brick ownership of a global sample lattice, trilinear
 *     reconstruction, transfer-function lookup, front-to-back
 *     emission-absorption accumulation)
 *   - sort-last compositing of partial images over a background oc_composite
 *   - gradients of a sum-of-squares image loss with respect to the
 *     transfer-function table and the stored voxels             oc_render_brick_grad
 *   - a brick's partial image with one directional light whose shadow
 *     rays run through every brick (the secondary rays that data-parallel
 *     ray tracing must send to the ranks holding the occluders)
 *                                                  oc_render_brick_shadowed
 *   - the image of a volume given as tetrahedral partitions (unstructured,
 *     possibly non-convex), marched sample by sample through the element
 *     that holds each sample                       oc_render_tets
 *     and with the directional light's shadow rays through all parts
 *                                                  oc_render_tets_shadowed
 *
 * The paper (Zellmann, "Data Parallel Visualization and Rendering on the
 * RAMSES Supercomputer with ANARI") describes data-parallel ray tracing over
 * spatially partitioned data (Sec. 2.2) and an ANARI-style frame/world/camera
 * interface whose render call is collective and whose framebuffer ends up on
 * the main rank (Sec. 3), but states no rendering mathematics.  Every
 * convention below is therefore a reading, listed in the design notes:
 *   R-grid   cell-centred voxels, half-open owned boxes, one ghost layer
 *   R-cam    pinhole camera, vertical fovy, row 0 at the top, pixel centres
 *   R-lat    samples at t_k = (k + 1/2) dt from the ray origin; sample k
 *            belongs to the brick whose half-open box contains o + t_k d
 *   R-tf     256-entry table, endpoint aligned over [vmin, vmax],
 *            piecewise linear, segment index min(floor(s), M - 2)
 *   R-ea     emission-absorption (Max 1995): sigma = scale * a,
 *            alpha = 1 - exp(-sigma dt), C += T alpha rgb, T *= (1 - alpha)
 *   R-depth  depth key = t of the first sample the brick owns (+inf if none)
 *   R-over   composite partials by ascending key with "over", then the
 *            background
 *   R-shadow one directional light (unit direction l toward the light) and
 *            an ambient fraction a0: sample k's emitted colour is scaled by
 *            a0 + (1 - a0) S(p_k), S = transmittance of the shadow ray from
 *            p_k toward the light (samples p_k + (j + 1/2) dt l, j >= 0, each
 *            evaluated in the brick whose half-open box holds it, none
 *            outside every brick); a0 = 1: no shadows
 *   R-tet    a point belongs to the tetrahedron whose four signed sub-volumes
 *            are positive, a zero one counting when a fixed direction g
 *            enters the tetrahedron across that face (so a point on shared
 *            faces, edges or vertices of a conforming mesh has exactly one
 *            owner); value = barycentric interpolation of vertex values
 * No early ray termination: every owned sample is evaluated.  The counters
 * report how many samples a renderer that stops once T < eps would evaluate.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no -ffast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t kind;          /* 0 = perspective, 1 = orthographic */
    int32_t width, height; /* image size in pixels */
    int32_t pad_;
    double eye[3];         /* perspective: eye point; orthographic: centre of the image plane */
    double target[3];      /* perspective: look-at point */
    double dir[3];         /* orthographic: viewing direction */
    double up[3];          /* up hint */
    double fovy_deg;       /* perspective: vertical field of view, degrees */
    double view_height;    /* orthographic: world-space height of the image */
} oc_camera;

typedef struct {
    int32_t dims[3];       /* owned voxels (nx, ny, nz) */
    int32_t ghost;         /* ghost layer width g on every face (0 = none) */
    double origin[3];      /* world position of the owned box's min corner */
    double spacing[3];     /* world size of one voxel */
    const void* vox;       /* (nz+2g)(ny+2g)(nx+2g) values, x fastest */
    int32_t vox_f64;       /* 0: vox holds float, 1: vox holds double */
    int32_t pad_;
} oc_brick;

typedef struct {
    const double* table;   /* n x 4 (r, g, b, a); colour non-premultiplied */
    int32_t n;             /* number of entries (>= 2) */
    int32_t pad_;
    double vmin, vmax;     /* value range mapped onto the table, endpoint aligned */
    double opacity_scale;  /* extinction per world unit = opacity_scale * a */
} oc_tf;

/* ---------------------------------------------------------------- vectors */
static void v_sub(const double a[3], const double b[3], double r[3]) {
    r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2];
}
static void v_cross(const double a[3], const double b[3], double r[3]) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
static void v_normalize(double v[3]) {
    double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] = v[0] / n; v[1] = v[1] / n; v[2] = v[2] / n;
}

/* ----------------------------------------------------------------- camera */
/* R-cam: forward f, right r = f x up, true up u = r x f (all unit).  Pixel
 * (i, j), j = 0 the top row, maps to image-plane coordinates
 *   x = (2 (i + 1/2) / W - 1) * tan(fovy / 2) * W / H
 *   y = (1 - 2 (j + 1/2) / H) * tan(fovy / 2)
 * perspective: o = eye, d = normalize(f + x r + y u)
 * orthographic: the same (x, y) scaled by view_height / 2 / tan -> offsets
 *   o = eye + x' r + y' u, d = f.                                          */
void oc_ray(const oc_camera* cam, int32_t i, int32_t j, double o[3], double d[3]) {
    double f[3], r[3], u[3];
    if (cam->kind == 0) {
        v_sub(cam->target, cam->eye, f);
    } else {
        f[0] = cam->dir[0]; f[1] = cam->dir[1]; f[2] = cam->dir[2];
    }
    v_normalize(f);
    v_cross(f, cam->up, r);
    v_normalize(r);
    v_cross(r, f, u);
    double W = (double)cam->width, H = (double)cam->height;
    double sx = (2.0 * ((double)i + 0.5)) / W - 1.0;
    double sy = 1.0 - (2.0 * ((double)j + 0.5)) / H;
    if (cam->kind == 0) {
        double th = tan(0.5 * cam->fovy_deg * (M_PI / 180.0));
        double ax = (th * W) / H, ay = th;
        double x = sx * ax, y = sy * ay;
        for (int c = 0; c < 3; ++c) { o[c] = cam->eye[c]; d[c] = (f[c] + x * r[c]) + y * u[c]; }
        v_normalize(d);
    } else {
        double hh = 0.5 * cam->view_height;
        double x = sx * ((hh * W) / H), y = sy * hh;
        for (int c = 0; c < 3; ++c) { o[c] = (cam->eye[c] + x * r[c]) + y * u[c]; d[c] = f[c]; }
    }
}

/* ------------------------------------------------------ brick primitives */
/* R-grid: owned world box is [origin, origin + dims * spacing) per axis. */
static void brick_box(const oc_brick* b, double lo[3], double hi[3]) {
    for (int c = 0; c < 3; ++c) {
        lo[c] = b->origin[c];
        hi[c] = b->origin[c] + (double)b->dims[c] * b->spacing[c];
    }
}

static int in_box(const double p[3], const double lo[3], const double hi[3]) {
    return p[0] >= lo[0] && p[0] < hi[0] && p[1] >= lo[1] && p[1] < hi[1] &&
           p[2] >= lo[2] && p[2] < hi[2];
}

/* Candidate sample indices [k0, k1] for the ray against the closed box
 * [lo, hi], widened by two samples on each side so that rounding of the slab
 * parameters can never drop a lattice point; ownership is then decided per
 * sample by in_box().  Returns 0 if the ray cannot reach the box. */
static int sample_range(const double o[3], const double d[3], const double lo[3],
                        const double hi[3], double dt, int64_t* k0, int64_t* k1) {
    double tin = 0.0, tout = INFINITY;
    for (int c = 0; c < 3; ++c) {
        if (d[c] == 0.0) {
            if (o[c] < lo[c] || o[c] > hi[c]) return 0;
            continue;
        }
        double ta = (lo[c] - o[c]) / d[c], tb = (hi[c] - o[c]) / d[c];
        double tn = ta < tb ? ta : tb, tf = ta < tb ? tb : ta;
        if (tn > tin) tin = tn;
        if (tf < tout) tout = tf;
    }
    if (tout < tin - 2.0 * dt) return 0;
    double a = floor(tin / dt - 0.5) - 2.0, bnd = ceil(tout / dt - 0.5) + 2.0;
    if (a < 0.0) a = 0.0;
    if (bnd < a) return 0;
    *k0 = (int64_t)a;
    *k1 = (int64_t)bnd;
    return 1;
}

/* Stored value at stored index (si, sj, sk), clamped to the stored array
 * (with one ghost layer the clamp never triggers for owned samples; with no
 * ghosts it is clamp-to-edge). */
static int64_t clamp_index(int64_t i, int64_t n) {
    return i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
}

static int64_t stored_offset(const oc_brick* b, int64_t si, int64_t sj, int64_t sk) {
    int64_t nx = b->dims[0] + 2 * b->ghost, ny = b->dims[1] + 2 * b->ghost,
            nz = b->dims[2] + 2 * b->ghost;
    return (clamp_index(sk, nz) * ny + clamp_index(sj, ny)) * nx + clamp_index(si, nx);
}

static double stored(const oc_brick* b, int64_t si, int64_t sj, int64_t sk) {
    int64_t off = stored_offset(b, si, sj, sk);
    return b->vox_f64 ? ((const double*)b->vox)[off] : (double)((const float*)b->vox)[off];
}

/* Trilinear reconstruction at world point p (R-grid: voxel centres at
 * origin + (i + 1/2) spacing).  Also returns the base stored index and the
 * fractional weights, which the gradient needs. */
static double sample_value(const oc_brick* b, const double p[3], int64_t base[3], double fr[3]) {
    for (int c = 0; c < 3; ++c) {
        double u = (p[c] - b->origin[c]) / b->spacing[c];   /* [0, dims) inside the box */
        double s = u - 0.5 + (double)b->ghost;               /* stored-index coordinate */
        double fl = floor(s);
        base[c] = (int64_t)fl;
        fr[c] = s - fl;
    }
    double v = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? fr[0] : 1.0 - fr[0]) * (dy ? fr[1] : 1.0 - fr[1]) *
                           (dz ? fr[2] : 1.0 - fr[2]);
                v += w * stored(b, base[0] + dx, base[1] + dy, base[2] + dz);
            }
    return v;
}

/* R-tf: x = clamp((v - vmin) / (vmax - vmin), 0, 1), s = x (M - 1),
 * i = min(floor(s), M - 2), phi = s - i, E = (1 - phi) E[i] + phi E[i+1]. */
static void classify(const oc_tf* tf, double v, double e[4], int32_t* seg, double* phi,
                     int* inside) {
    double x = (v - tf->vmin) / (tf->vmax - tf->vmin);
    *inside = (x >= 0.0 && x <= 1.0);
    if (x < 0.0) x = 0.0;
    if (x > 1.0) x = 1.0;
    double s = x * (double)(tf->n - 1);
    int32_t i = (int32_t)floor(s);
    if (i > tf->n - 2) i = tf->n - 2;
    double f = s - (double)i;
    for (int c = 0; c < 4; ++c)
        e[c] = (1.0 - f) * tf->table[4 * i + c] + f * tf->table[4 * (i + 1) + c];
    *seg = i;
    *phi = f;
}

/* ----------------------------------------------------------- one partial */
/* Partial image of one brick for pixel (i, j): premultiplied rgb in out[0..2],
 * alpha 1 - T in out[3], depth key in *depth.  counters (optional, 2 entries):
 * [0] += owned samples, [1] += samples a renderer stopping at T < ert_eps
 * would evaluate (the stopping sample included). */
static void render_pixel(const oc_camera* cam, const oc_brick* b, const oc_tf* tf, double dt,
                         double ert_eps, int32_t i, int32_t j, double out[4], double* depth,
                         int64_t* counters) {
    double o[3], d[3], lo[3], hi[3];
    oc_ray(cam, i, j, o, d);
    brick_box(b, lo, hi);
    double C[3] = {0.0, 0.0, 0.0}, T = 1.0;
    double key = INFINITY;
    int64_t nominal = 0, evaluated = 0;
    int stopped = 0;
    int64_t k0, k1;
    if (sample_range(o, d, lo, hi, dt, &k0, &k1)) {
        for (int64_t k = k0; k <= k1; ++k) {
            double t = ((double)k + 0.5) * dt;
            double p[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
            if (!in_box(p, lo, hi)) continue;
            if (key == INFINITY) key = t;
            int64_t base[3]; double fr[3], e[4], phi; int32_t seg; int inside;
            double v = sample_value(b, p, base, fr);
            classify(tf, v, e, &seg, &phi, &inside);
            double sigma = tf->opacity_scale * e[3];
            double alpha = 1.0 - exp(-sigma * dt);
            for (int c = 0; c < 3; ++c) C[c] += T * alpha * e[c];
            T = T * (1.0 - alpha);
            ++nominal;
            if (!stopped) { ++evaluated; if (T < ert_eps) stopped = 1; }
        }
    }
    out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = 1.0 - T;
    *depth = key;
    if (counters) { counters[0] += nominal; counters[1] += evaluated; }
}

/* Partial images of one brick.  If pix == NULL every pixel of the W x H image
 * is rendered into rgba[(j W + i) 4 + c] / depth[j W + i]; otherwise the npix
 * (i, j) pairs in pix are rendered into rgba[4 q + c] / depth[q].  counters
 * (2 entries, may be NULL) accumulate owned / evaluated samples. */
void oc_render_brick(const oc_camera* cam, const oc_brick* b, const oc_tf* tf, double dt,
                     double ert_eps, const int32_t* pix, int64_t npix, double* rgba,
                     double* depth, int64_t* counters) {
    int64_t n = pix ? npix : (int64_t)cam->width * cam->height;
    int64_t nom = 0, ev = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nom, ev)
    for (int64_t q = 0; q < n; ++q) {
        int32_t i = pix ? pix[2 * q] : (int32_t)(q % cam->width);
        int32_t j = pix ? pix[2 * q + 1] : (int32_t)(q / cam->width);
        int64_t cnt[2] = {0, 0};
        render_pixel(cam, b, tf, dt, ert_eps, i, j, rgba + 4 * q, depth + q, cnt);
        nom += cnt[0];
        ev += cnt[1];
    }
    if (counters) { counters[0] += nom; counters[1] += ev; }
}

/* ---------------------------------------------------------------- shadows */
/* R-shadow: transmittance from point p toward the light along unit l through
 * the nb bricks.  The shadow ray's samples are q_j = p + (j + 1/2) dt l for
 * j >= 0; each q_j inside some brick's half-open owned box is evaluated in
 * that brick exactly as a primary sample (trilinear value, table, extinction)
 * and multiplies S by 1 - alpha(q_j).  Candidates are the lattice points the
 * ray can have inside the bricks' common bounding box. */
static double shadow_transmittance(int32_t nb, const oc_brick* const* bricks, const oc_tf* tf,
                                   double dt, const double p[3], const double l[3]) {
    double LO[3] = {INFINITY, INFINITY, INFINITY}, HI[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t b = 0; b < nb; ++b) {
        double lo[3], hi[3];
        brick_box(bricks[b], lo, hi);
        for (int c = 0; c < 3; ++c) {
            if (lo[c] < LO[c]) LO[c] = lo[c];
            if (hi[c] > HI[c]) HI[c] = hi[c];
        }
    }
    int64_t j0, j1;
    if (nb == 0 || !sample_range(p, l, LO, HI, dt, &j0, &j1)) return 1.0;
    double S = 1.0;
    for (int64_t j = j0; j <= j1; ++j) {
        double t = ((double)j + 0.5) * dt;
        double q[3] = {p[0] + t * l[0], p[1] + t * l[1], p[2] + t * l[2]};
        for (int32_t b = 0; b < nb; ++b) {
            double lo[3], hi[3];
            brick_box(bricks[b], lo, hi);
            if (!in_box(q, lo, hi)) continue;
            int64_t base[3]; double fr[3], e[4], phi; int32_t seg; int inside;
            double v = sample_value(bricks[b], q, base, fr);
            classify(tf, v, e, &seg, &phi, &inside);
            double alpha = 1.0 - exp(-tf->opacity_scale * e[3] * dt);
            S = S * (1.0 - alpha);
            break;
        }
    }
    return S;
}

/* render_pixel with R-shadow: the colour of every owned sample p_k of brick b
 * is scaled by a0 + (1 - a0) S(p_k), S through all nb bricks (b among them);
 * alpha, T and the depth key are those of render_pixel. */
static void render_pixel_shadowed(const oc_camera* cam, const oc_brick* b, int32_t nb,
                                  const oc_brick* const* bricks, const oc_tf* tf, double dt,
                                  double ert_eps, const double l[3], double a0, int32_t i, int32_t j,
                                  double out[4], double* depth, int64_t* counters) {
    double o[3], d[3], lo[3], hi[3];
    oc_ray(cam, i, j, o, d);
    brick_box(b, lo, hi);
    double C[3] = {0.0, 0.0, 0.0}, T = 1.0;
    double key = INFINITY;
    int64_t nominal = 0, evaluated = 0;
    int stopped = 0;
    int64_t k0, k1;
    if (sample_range(o, d, lo, hi, dt, &k0, &k1)) {
        for (int64_t k = k0; k <= k1; ++k) {
            double t = ((double)k + 0.5) * dt;
            double p[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
            if (!in_box(p, lo, hi)) continue;
            if (key == INFINITY) key = t;
            int64_t base[3]; double fr[3], e[4], phi; int32_t seg; int inside;
            double v = sample_value(b, p, base, fr);
            classify(tf, v, e, &seg, &phi, &inside);
            double sigma = tf->opacity_scale * e[3];
            double alpha = 1.0 - exp(-sigma * dt);
            double f = a0 + (1.0 - a0) * shadow_transmittance(nb, bricks, tf, dt, p, l);
            for (int c = 0; c < 3; ++c) C[c] += T * alpha * e[c] * f;
            T = T * (1.0 - alpha);
            ++nominal;
            if (!stopped) { ++evaluated; if (T < ert_eps) stopped = 1; }
        }
    }
    out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = 1.0 - T;
    *depth = key;
    if (counters) { counters[0] += nominal; counters[1] += evaluated; }
}

/* Partial images of brick b with R-shadow (light direction l, normalised
 * here; ambient a0 in [0, 1]), shadow rays through all nb bricks; pixels,
 * outputs and counters as for oc_render_brick.  Returns -1 on bad input. */
int oc_render_brick_shadowed(const oc_camera* cam, const oc_brick* b, int32_t nb,
                             const oc_brick* const* bricks, const oc_tf* tf, double dt,
                             double ert_eps, const double light_dir[3], double a0,
                             const int32_t* pix, int64_t npix, double* rgba, double* depth,
                             int64_t* counters) {
    double l[3] = {light_dir[0], light_dir[1], light_dir[2]};
    double nl = sqrt(l[0] * l[0] + l[1] * l[1] + l[2] * l[2]);
    if (!(nl > 0.0) || !(a0 >= 0.0 && a0 <= 1.0)) return -1;
    l[0] = l[0] / nl; l[1] = l[1] / nl; l[2] = l[2] / nl;
    int64_t n = pix ? npix : (int64_t)cam->width * cam->height;
    int64_t nom = 0, ev = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : nom, ev)
    for (int64_t q = 0; q < n; ++q) {
        int32_t i = pix ? pix[2 * q] : (int32_t)(q % cam->width);
        int32_t j = pix ? pix[2 * q + 1] : (int32_t)(q / cam->width);
        int64_t cnt[2] = {0, 0};
        render_pixel_shadowed(cam, b, nb, bricks, tf, dt, ert_eps, l, a0, i, j, rgba + 4 * q,
                              depth + q, cnt);
        nom += cnt[0];
        ev += cnt[1];
    }
    if (counters) { counters[0] += nom; counters[1] += ev; }
    return 0;
}

/* ------------------------------------------------- tetrahedral partitions */
typedef struct {
    int32_t n_vertices, n_tets;
    const double* vertices;   /* n_vertices x 3 (x, y, z) */
    const float* values;      /* n_vertices */
    const int32_t* tets;      /* n_tets x 4 vertex indices, positive orientation */
} oc_tetpart;

/* Fixed direction of the face tie rule (exact binary fractions; no lattice
 * normal is orthogonal to it). */
static const double OC_TIE_G[3] = {1.0, 0.0009765625, 0.00000095367431640625};

/* orient(a, b, c, p) = (b - a) . ((c - a) x (p - a)), in this order. */
static double orient3(const double a[3], const double b[3], const double c[3], const double p[3]) {
    double bx = b[0] - a[0], by = b[1] - a[1], bz = b[2] - a[2];
    double cx = c[0] - a[0], cy = c[1] - a[1], cz = c[2] - a[2];
    double px = p[0] - a[0], py = p[1] - a[1], pz = p[2] - a[2];
    double x = cy * pz - cz * py, y = cz * px - cx * pz, z = cx * py - cy * px;
    return bx * x + by * y + bz * z;
}

static int lex_less(const double a[3], const double b[3]) {
    if (a[0] != b[0]) return a[0] < b[0];
    if (a[1] != b[1]) return a[1] < b[1];
    return a[2] < b[2];
}

/* R-tet: signed sub-volume of face i (opposite vertex i) of tetrahedron v
 * with p, computed from the face's vertices in lexicographic order (so the
 * tetrahedra sharing a face round it alike), signed positive toward v[i];
 * *owned: whether g enters the tetrahedron across that face. */
static double face_volume(const double* const v[4], int i, const double p[3], int* owned) {
    const double* f[3];
    int m = 0;
    for (int j = 0; j < 4; ++j)
        if (j != i) f[m++] = v[j];
    for (int a = 1; a < 3; ++a)
        for (int b = a; b > 0 && lex_less(f[b], f[b - 1]); --b) {
            const double* t = f[b]; f[b] = f[b - 1]; f[b - 1] = t;
        }
    double s = orient3(f[0], f[1], f[2], v[i]) > 0.0 ? 1.0 : -1.0;
    double e1[3] = {f[1][0] - f[0][0], f[1][1] - f[0][1], f[1][2] - f[0][2]};
    double e2[3] = {f[2][0] - f[0][0], f[2][1] - f[0][1], f[2][2] - f[0][2]};
    double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    *owned = s * (n[0] * OC_TIE_G[0] + n[1] * OC_TIE_G[1] + n[2] * OC_TIE_G[2]) > 0.0;
    return s * orient3(f[0], f[1], f[2], p);
}

/* Whether tetrahedron t of part P holds p (R-tet); if so its interpolated
 * value in *value. */
static int tet_holds(const oc_tetpart* P, int32_t t, const double p[3], double* value) {
    const double* v[4];
    for (int j = 0; j < 4; ++j) v[j] = P->vertices + 3 * (int64_t)P->tets[4 * (int64_t)t + j];
    double D[4];
    for (int i = 0; i < 4; ++i) {
        int owned;
        D[i] = face_volume(v, i, p, &owned);
        if (D[i] < 0.0 || (D[i] == 0.0 && !owned)) return 0;
    }
    double tot = D[0] + D[1] + D[2] + D[3];
    double val = 0.0;
    for (int i = 0; i < 4; ++i) val += (D[i] / tot) * (double)P->values[P->tets[4 * (int64_t)t + i]];
    *value = val;
    return 1;
}

/* Closed bounding box of the vertices of all parts. */
static void tets_box(int32_t n, const oc_tetpart* parts, double LO[3], double HI[3]) {
    for (int c = 0; c < 3; ++c) { LO[c] = INFINITY; HI[c] = -INFINITY; }
    for (int32_t q = 0; q < n; ++q)
        for (int32_t v = 0; v < parts[q].n_vertices; ++v)
            for (int c = 0; c < 3; ++c) {
                double x = parts[q].vertices[3 * (int64_t)v + c];
                if (x < LO[c]) LO[c] = x;
                if (x > HI[c]) HI[c] = x;
            }
}

/* R-tet: the number of tetrahedra (over all parts) that hold p; the value
 * at p from the first of them, in (part, tetrahedron) order, in *value. */
static int tets_locate(int32_t n, const oc_tetpart* parts, const double p[3], double* value) {
    int owners = 0;
    double w;
    for (int32_t a = 0; a < n; ++a)
        for (int32_t e = 0; e < parts[a].n_tets; ++e)
            if (tet_holds(&parts[a], e, p, &w)) {
                if (owners == 0) *value = w;
                ++owners;
            }
    return owners;
}

/* Image of the volume given by n tetrahedral parts (all parts together form
 * one mesh), pixels as for oc_render_brick, over bg: the ray's lattice
 * samples t_k = (k + 1/2) dt inside the parts' common bounding box, each
 * evaluated in the tetrahedron that holds it (R-tet; none: no
 * contribution), accumulated front to back (R-ea).  counters: [0] += samples
 * held by a tetrahedron, [1] += samples held by more than one (0 for a
 * conforming mesh). */
void oc_render_tets(const oc_camera* cam, int32_t n, const oc_tetpart* parts, const oc_tf* tf, double dt,
                    const double bg[4], const int32_t* pix, int64_t npix, double* rgba, int64_t* counters) {
    double LO[3], HI[3];
    tets_box(n, parts, LO, HI);
    int64_t npx = pix ? npix : (int64_t)cam->width * cam->height;
    int64_t held = 0, twice = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : held, twice)
    for (int64_t q = 0; q < npx; ++q) {
        int32_t i = pix ? pix[2 * q] : (int32_t)(q % cam->width);
        int32_t j = pix ? pix[2 * q + 1] : (int32_t)(q / cam->width);
        double o[3], d[3];
        oc_ray(cam, i, j, o, d);
        double C[3] = {0.0, 0.0, 0.0}, T = 1.0;
        int64_t k0, k1;
        if (n > 0 && sample_range(o, d, LO, HI, dt, &k0, &k1)) {
            for (int64_t k = k0; k <= k1; ++k) {
                double t = ((double)k + 0.5) * dt;
                double p[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
                double v = 0.0;
                int owners = tets_locate(n, parts, p, &v);
                if (owners == 0) continue;
                ++held;
                if (owners > 1) ++twice;
                double ev[4], phi; int32_t seg; int inside;
                classify(tf, v, ev, &seg, &phi, &inside);
                double alpha = 1.0 - exp(-tf->opacity_scale * ev[3] * dt);
                for (int c = 0; c < 3; ++c) C[c] += T * alpha * ev[c];
                T = T * (1.0 - alpha);
            }
        }
        double A = 1.0 - T;
        for (int c = 0; c < 3; ++c) rgba[4 * q + c] = C[c] + T * bg[c];
        rgba[4 * q + 3] = A + T * bg[3];
    }
    if (counters) { counters[0] += held; counters[1] += twice; }
}

/* R-shadow for tetrahedral parts: transmittance from p toward the light
 * along unit l, the shadow samples q_j = p + (j + 1/2) dt l (j >= 0) inside
 * the parts' bounding box, each held one evaluated as a primary sample and
 * multiplying S by 1 - alpha(q_j).  *held += shadow samples held. */
static double tets_shadow(int32_t n, const oc_tetpart* parts, const double LO[3], const double HI[3],
                          const oc_tf* tf, double dt, const double p[3], const double l[3], int64_t* held) {
    int64_t j0, j1;
    if (n == 0 || !sample_range(p, l, LO, HI, dt, &j0, &j1)) return 1.0;
    double S = 1.0;
    for (int64_t j = j0; j <= j1; ++j) {
        double t = ((double)j + 0.5) * dt;
        double q[3] = {p[0] + t * l[0], p[1] + t * l[1], p[2] + t * l[2]};
        double v = 0.0;
        if (tets_locate(n, parts, q, &v) == 0) continue;
        double e[4], phi; int32_t seg; int inside;
        classify(tf, v, e, &seg, &phi, &inside);
        double alpha = 1.0 - exp(-tf->opacity_scale * e[3] * dt);
        S = S * (1.0 - alpha);
        ++*held;
    }
    return S;
}

/* oc_render_tets with R-shadow (light direction normalised here, ambient a0
 * in [0, 1]): the colour of every held primary sample is scaled by
 * a0 + (1 - a0) S, S its shadow ray's transmittance through all parts;
 * alpha and T are unchanged.  counters: [0] += primary samples held,
 * [1] += primary samples held by more than one tetrahedron, [2] += shadow
 * samples held.  Returns -1 on bad input. */
int oc_render_tets_shadowed(const oc_camera* cam, int32_t n, const oc_tetpart* parts, const oc_tf* tf,
                            double dt, const double light_dir[3], double a0, const double bg[4],
                            const int32_t* pix, int64_t npix, double* rgba, int64_t* counters) {
    double l[3] = {light_dir[0], light_dir[1], light_dir[2]};
    double nl = sqrt(l[0] * l[0] + l[1] * l[1] + l[2] * l[2]);
    if (!(nl > 0.0) || !(a0 >= 0.0 && a0 <= 1.0)) return -1;
    l[0] = l[0] / nl; l[1] = l[1] / nl; l[2] = l[2] / nl;
    double LO[3], HI[3];
    tets_box(n, parts, LO, HI);
    int64_t npx = pix ? npix : (int64_t)cam->width * cam->height;
    int64_t held = 0, twice = 0, shadow = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : held, twice, shadow)
    for (int64_t q = 0; q < npx; ++q) {
        int32_t i = pix ? pix[2 * q] : (int32_t)(q % cam->width);
        int32_t j = pix ? pix[2 * q + 1] : (int32_t)(q / cam->width);
        double o[3], d[3];
        oc_ray(cam, i, j, o, d);
        double C[3] = {0.0, 0.0, 0.0}, T = 1.0;
        int64_t k0, k1;
        if (n > 0 && sample_range(o, d, LO, HI, dt, &k0, &k1)) {
            for (int64_t k = k0; k <= k1; ++k) {
                double t = ((double)k + 0.5) * dt;
                double p[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
                double v = 0.0;
                int owners = tets_locate(n, parts, p, &v);
                if (owners == 0) continue;
                ++held;
                if (owners > 1) ++twice;
                double ev[4], phi; int32_t seg; int inside;
                classify(tf, v, ev, &seg, &phi, &inside);
                double alpha = 1.0 - exp(-tf->opacity_scale * ev[3] * dt);
                double f = a0 + (1.0 - a0) * tets_shadow(n, parts, LO, HI, tf, dt, p, l, &shadow);
                for (int c = 0; c < 3; ++c) C[c] += T * alpha * ev[c] * f;
                T = T * (1.0 - alpha);
            }
        }
        double A = 1.0 - T;
        for (int c = 0; c < 3; ++c) rgba[4 * q + c] = C[c] + T * bg[c];
        rgba[4 * q + 3] = A + T * bg[3];
    }
    if (counters) { counters[0] += held; counters[1] += twice; counters[2] += shadow; }
    return 0;
}

/* -------------------------------------------------------------- composite */
/* R-over: for each of the npx pixels, sort the n partials by depth key
 * (ascending, partial index breaking ties), accumulate front to back
 *   C += (1 - A) C_i,  A += (1 - A) A_i
 * then put the result over the background: rgb = C + (1 - A) bg_rgb,
 * a = A + (1 - A) bg_a.  rgba[p] points at partial p's npx x 4 values, depth[p]
 * at its npx keys; out is npx x 4. */
#define OC_MAX_PARTIALS 256

/* Visibility order of the partials at pixel q: indices sorted by (key, index). */
static int32_t depth_order(int32_t n, const double* const* depth, int64_t q, int32_t* order) {
    int32_t m = 0;
    for (int32_t p = 0; p < n; ++p) order[m++] = p;
    for (int32_t a = 1; a < m; ++a) {
        int32_t cur = order[a];
        int32_t b = a - 1;
        while (b >= 0 && depth[order[b]][q] > depth[cur][q]) { order[b + 1] = order[b]; --b; }
        order[b + 1] = cur;
    }
    return m;
}

int oc_composite(int32_t n, const double* const* rgba, const double* const* depth, int64_t npx,
                 const double bg[4], double* out) {
    if (n < 0 || n > OC_MAX_PARTIALS) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < npx; ++q) {
        int32_t order[OC_MAX_PARTIALS];
        int32_t m = depth_order(n, depth, q, order);
        double C[3] = {0.0, 0.0, 0.0}, A = 0.0;
        for (int32_t a = 0; a < m; ++a) {
            const double* s = rgba[order[a]] + 4 * q;
            double w = 1.0 - A;
            C[0] += w * s[0]; C[1] += w * s[1]; C[2] += w * s[2];
            A += w * s[3];
        }
        double w = 1.0 - A;
        out[4 * q + 0] = C[0] + w * bg[0];
        out[4 * q + 1] = C[1] + w * bg[1];
        out[4 * q + 2] = C[2] + w * bg[2];
        out[4 * q + 3] = A + w * bg[3];
    }
    return 0;
}

/* ------------------------------------------------------------- gradients */
/* Backward of oc_composite.  With the partials in visibility order and
 * P_i = prod_{j<i} (1 - A_j) the transmittance in front of partial i, the
 * output is I = sum_i P_i X_i + P_n bg (X = C for rgb, A for alpha), so
 *   dI/dC_i = P_i (per colour channel),
 *   dI/dA_i = P_i [ e_a - S_i ],  S_i = what lies behind i composited over bg:
 *             S_{n-1} = bg, S_{i-1} = X_i + (1 - A_i) S_i,
 * where e_a contributes only to the alpha channel (A_i is also X_i there).
 * g_out: npx x 4 upstream gradient; g_parts[p]: npx x 4 output (dL/dC_rgb,
 * dL/dA) for partial p. */
int oc_composite_grad(int32_t n, const double* const* rgba, const double* const* depth,
                      int64_t npx, const double bg[4], const double* g_out, double* const* g_parts) {
    if (n < 0 || n > OC_MAX_PARTIALS) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < npx; ++q) {
        int32_t order[OC_MAX_PARTIALS];
        double P[OC_MAX_PARTIALS + 1];
        int32_t m = depth_order(n, depth, q, order);
        P[0] = 1.0;
        for (int32_t a = 0; a < m; ++a) P[a + 1] = P[a] * (1.0 - rgba[order[a]][4 * q + 3]);
        const double* g = g_out + 4 * q;
        double S[4] = {bg[0], bg[1], bg[2], bg[3]};
        for (int32_t a = m - 1; a >= 0; --a) {
            const double* x = rgba[order[a]] + 4 * q;
            double* gp = g_parts[order[a]] + 4 * q;
            gp[0] = g[0] * P[a];
            gp[1] = g[1] * P[a];
            gp[2] = g[2] * P[a];
            /* alpha enters as an opacity (attenuating S) and, on the alpha
             * channel, also as the value composited */
            gp[3] = P[a] * (g[3] * (1.0 - S[3]) - g[0] * S[0] - g[1] * S[1] - g[2] * S[2]);
            double A = x[3];
            S[0] = x[0] + (1.0 - A) * S[0];
            S[1] = x[1] + (1.0 - A) * S[1];
            S[2] = x[2] + (1.0 - A) * S[2];
            S[3] = x[3] + (1.0 - A) * S[3];
        }
    }
    return 0;
}

typedef struct {
    int64_t base[3];
    double fr[3];
    double e[4];
    double phi, alpha, T;   /* T: transmittance in front of this sample */
    int32_t seg, inside;
} oc_sample;

/* Backward of one brick's partial image.  Per ray with owned samples
 * k = 0..N-1 (T_0 = 1, T_{k+1} = T_k (1 - alpha_k)):
 *   C = sum_k T_k alpha_k rgb_k,  A = 1 - T_N.
 * With R_k = alpha_k rgb_k + (1 - alpha_k) R_{k+1} (R_N = 0) and
 * Q_k = (1 - alpha_k) Q_{k+1} (Q_N = 1):
 *   dC/drgb_k = T_k alpha_k,  dC/dalpha_k = T_k (rgb_k - R_{k+1}),
 *   dA/dalpha_k = T_k Q_{k+1},  dalpha_k/da_k = scale dt (1 - alpha_k).
 * Then through the table lerp (weights 1 - phi, phi; slope (E[i+1] - E[i])
 * (M - 1) / (vmax - vmin) inside [vmin, vmax], 0 outside) and the trilinear
 * weights onto the stored voxels (clamped stored indices, as in the forward).
 * g_part: W x H x 4 upstream gradient (dL/dC_rgb, dL/dA) of this partial;
 * grad_tf (n x 4) and grad_vox (stored array) are accumulated into. */
int oc_render_brick_grad(const oc_camera* cam, const oc_brick* b, const oc_tf* tf, double dt,
                         const double* g_part, double* grad_tf, double* grad_vox) {
    int64_t npx = (int64_t)cam->width * cam->height;
    double scale_dv = (double)(tf->n - 1) / (tf->vmax - tf->vmin);
    int status = 0;
#pragma omp parallel
    {
        double* gtf = (double*)calloc((size_t)tf->n * 4, sizeof(double));
        int64_t cap = 0;
        oc_sample* smp = NULL;
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < npx; ++q) {
            const double* g = g_part + 4 * q;
            if (g[0] == 0.0 && g[1] == 0.0 && g[2] == 0.0 && g[3] == 0.0) continue;
            int32_t i = (int32_t)(q % cam->width), j = (int32_t)(q / cam->width);
            double o[3], d[3], lo[3], hi[3];
            oc_ray(cam, i, j, o, d);
            brick_box(b, lo, hi);
            int64_t k0, k1, N = 0;
            if (!sample_range(o, d, lo, hi, dt, &k0, &k1)) continue;
            if (k1 - k0 + 1 > cap) {
                cap = k1 - k0 + 1;
                free(smp);
                smp = (oc_sample*)malloc((size_t)cap * sizeof(oc_sample));
                if (!smp) { status = -2; cap = 0; continue; }
            }
            double T = 1.0;
            for (int64_t k = k0; k <= k1; ++k) {           /* forward, storing per-sample state */
                double t = ((double)k + 0.5) * dt;
                double p[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
                if (!in_box(p, lo, hi)) continue;
                oc_sample* s = &smp[N++];
                double v = sample_value(b, p, s->base, s->fr);
                classify(tf, v, s->e, &s->seg, &s->phi, &s->inside);
                s->alpha = 1.0 - exp(-tf->opacity_scale * s->e[3] * dt);
                s->T = T;
                T = T * (1.0 - s->alpha);
            }
            double R[3] = {0.0, 0.0, 0.0}, Q = 1.0;
            for (int64_t k = N - 1; k >= 0; --k) {         /* reverse sweep */
                oc_sample* s = &smp[k];
                double dL_drgb[3], dL_dalpha = 0.0;
                for (int c = 0; c < 3; ++c) {
                    dL_drgb[c] = g[c] * s->T * s->alpha;
                    dL_dalpha += g[c] * s->T * (s->e[c] - R[c]);
                }
                dL_dalpha += g[3] * s->T * Q;
                double dL_da = dL_dalpha * tf->opacity_scale * dt * (1.0 - s->alpha);
                double gE[4] = {dL_drgb[0], dL_drgb[1], dL_drgb[2], dL_da};
                double dL_dv = 0.0;
                for (int c = 0; c < 4; ++c) {
                    gtf[4 * s->seg + c] += (1.0 - s->phi) * gE[c];
                    gtf[4 * (s->seg + 1) + c] += s->phi * gE[c];
                    if (s->inside)
                        dL_dv += gE[c] * (tf->table[4 * (s->seg + 1) + c] - tf->table[4 * s->seg + c]) *
                                 scale_dv;
                }
                for (int dz = 0; dz < 2; ++dz)
                    for (int dy = 0; dy < 2; ++dy)
                        for (int dx = 0; dx < 2; ++dx) {
                            double w = (dx ? s->fr[0] : 1.0 - s->fr[0]) *
                                       (dy ? s->fr[1] : 1.0 - s->fr[1]) *
                                       (dz ? s->fr[2] : 1.0 - s->fr[2]);
                            int64_t off = stored_offset(b, s->base[0] + dx, s->base[1] + dy,
                                                        s->base[2] + dz);
                            double add = w * dL_dv;
#pragma omp atomic
                            grad_vox[off] += add;
                        }
                for (int c = 0; c < 3; ++c) R[c] = s->alpha * s->e[c] + (1.0 - s->alpha) * R[c];
                Q = (1.0 - s->alpha) * Q;
            }
        }
#pragma omp critical
        for (int32_t e = 0; e < 4 * tf->n; ++e) grad_tf[e] += gtf[e];
        free(gtf);
        free(smp);
    }
    return status;
}

/* Threads the parallel loops above use (reported with timings). */
int oc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the thread count of the parallel loops (for a one-core timing). */
void oc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
