/*
 * CPU FP64 oracle for the spherical-grid line-integral projector.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * path.
 *
 * What it computes is the plain definition of the projector (TomoSphero,
 * Sec. 2.1, Eqs. 3-5): the object is piecewise constant on the voxels of a
 * spherical grid (Sec. 2.2) and zero outside it (Sec. 4.6), so for a ray
 * x + n l, l >= 0,
 *
 *     y = sum_v rho_v * |{ l >= 0 : x + n l lies in voxel v }|.
 *
 * It deliberately does NOT use the paper's crossing-direction bookkeeping
 * (Sec. 3.2, appendix Sec. 9.2) or the forward fill (Table 2).  Instead, per
 * ray it
 *   1. normalises the direction (distance along the ray is metric, Eq. 3);
 *   2. collects every l > 0 at which the ray meets a boundary surface
 *      (Sec. 3.1): both roots of every sphere, every root of every cone that
 *      lies on the cone's own nappe, every hit of every azimuth half-plane,
 *      plus the point where the ray crosses the polar axis when its
 *      projection on the xy-plane passes exactly through the origin (the
 *      azimuth jumps by pi there without touching any half-plane), and the
 *      start l = 0 itself, so that a ray starting inside the grid (the
 *      sunward rays from voxel centroids of Sec. 9.3) integrates from its
 *      start; for a start outside the grid the first interval lies outside
 *      and is dropped;
 *   3. sorts them (Sec. 3.3);
 *   4. classifies the midpoint of every positive-length interval by its
 *      spherical coordinates (r, colatitude, azimuth) with an upper-bound
 *      search in the boundary arrays; an index outside [0, N) is invalid
 *      (Sec. 3.3, zeroing rule of Table 2(c));
 *   5. keeps valid intervals and merges runs of the same voxel that touch in
 *      l (the canonical list: re-entering a voxel after a positive-length
 *      gap is a separate segment).
 *
 * Conventions (readings of the paper, both sides follow them):
 *   - colatitude theta is measured from +Z (Sec. 9.2 puts the principal axis
 *     on +Z; Eq. 12's sign test makes the elevation index grow with theta);
 *   - azimuth phi = atan2(y, x), counter-clockwise about +Z (Eq. 13), taken
 *     in [a_b[0], a_b[0] + 2 pi); the grid is cyclic when a_b spans 2 pi;
 *   - an azimuth boundary is a half-plane (a plane through the axis would
 *     conflate a_k with a_k + pi);
 *   - a cone with |cos e_k| < 1e-12 is the plane z = 0; cones at e = 0 or pi
 *     are the polar axis and are never crossed;
 *   - a point exactly at colatitude pi belongs to the last elevation region
 *     when e_b ends at pi.
 *
 * A ray is flagged as a "tie" when the index list near some event is not
 * decided robustly by FP64 arithmetic: two consecutive breakpoints inside
 * the grid's outer sphere closer than 1e-9 * r_max, a grazing sphere or cone
 * (normalised discriminant below 1e-9), a half-plane met at a grazing angle
 * or next to the axis, or a cone root next to the origin.  Index lists are
 * compared bit-exactly only for rays that are not ties.  A second, looser
 * flag marks rays whose segment lengths are ill-conditioned beyond FP32
 * rounding (normalised discriminant below 1e-6, breakpoints within
 * 1e-7 * r_max): a root's sensitivity to one-ulp changes of the ray grows
 * like eps * l * scale / discriminant, so lengths there are compared with a
 * conditioning-sized tolerance.  Flag byte: bit 0 tie, bit 1 sensitive.
 *
 * Build: gcc -O3 -march=native -fopenmp -shared -fPIC (see build.py here).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_TWO_PI 6.283185307179586476925286766559

typedef struct {
    int nr, ne, na;
    const double *rb, *eb, *ab;
    int cyclic;      /* azimuth boundaries span exactly 2 pi */
    double rmax;     /* outer radius */
    double tol_t;    /* 1e-9 * rmax: breakpoint closeness for ties */
} ogrid;

static void ogrid_init(ogrid *g, const double *rb, int nr, const double *eb, int ne,
                       const double *ab, int na) {
    g->nr = nr; g->ne = ne; g->na = na;
    g->rb = rb; g->eb = eb; g->ab = ab;
    g->cyclic = fabs((ab[na] - ab[0]) - ORA_TWO_PI) <= 1e-12;
    g->rmax = rb[nr];
    g->tol_t = 1e-9 * rb[nr];
}

/* number of entries of the sorted array b[0..m) that are <= v */
static int count_le(const double *b, int m, double v) {
    int lo = 0, hi = m;
    while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (b[mid] <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* Voxel that contains point p; returns -1 when p is outside the grid. */
static int64_t classify_point(const ogrid *g, const double p[3]) {
    double rxy = sqrt(p[0] * p[0] + p[1] * p[1]);
    double r = sqrt(rxy * rxy + p[2] * p[2]);
    int ir = count_le(g->rb, g->nr + 1, r) - 1;
    if (ir < 0 || ir >= g->nr) return -1;

    double th = atan2(rxy, p[2]);
    int ie = count_le(g->eb, g->ne + 1, th) - 1;
    if (ie == g->ne && g->eb[g->ne] >= M_PI && th >= g->eb[g->ne]) ie = g->ne - 1;
    if (ie < 0 || ie >= g->ne) return -1;

    double ph = atan2(p[1], p[0]) - g->ab[0];
    ph = fmod(ph, ORA_TWO_PI);
    if (ph < 0) ph += ORA_TWO_PI;
    if (ph >= ORA_TWO_PI) ph -= ORA_TWO_PI;
    /* upper-bound search on the boundaries measured from a_b[0] */
    int lo = 0, hi = g->na + 1;
    while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (g->ab[mid] - g->ab[0] <= ph) lo = mid + 1; else hi = mid;
    }
    int ia = lo - 1;
    if (ia >= g->na) {
        if (g->cyclic) ia = 0; /* sliver between a_b[Na] and a_b[0] + 2 pi */
        else return -1;
    }
    if (ia < 0) return -1;
    return ((int64_t)ir * g->ne + ie) * g->na + ia;
}

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) ? -1 : (x > y) ? 1 : 0;
}

/* Append the positive roots of  a t^2 + 2 b t + c = 0  (textbook stable form)
 * to out[]; returns how many were written (0..2).  disc_out receives the
 * discriminant b^2 - a c and norm_out the scale b^2 + |a c| it is compared to. */
static int quad_roots(double a, double b, double c, double out[2], double *disc_out,
                      double *norm_out) {
    double disc = b * b - a * c;
    *disc_out = disc;
    *norm_out = b * b + fabs(a * c);
    if (disc < 0) return 0;
    double s = sqrt(disc);
    double q = -(b + (b >= 0 ? s : -s));
    int k = 0;
    if (a != 0) out[k++] = q / a;
    if (q != 0) out[k++] = c / q;
    else if (a != 0 && k == 0) out[k++] = -b / a;
    return k;
}

typedef struct {
    double *t;      /* breakpoint buffer */
    int cap;
} obuf;

/*
 * Trace one ray.  x: start, n: direction (any length, normalised here).
 * Writes at most cap canonical segments into vox/len/t0 (when non-NULL) and
 * returns the number of canonical segments; *tie receives the tie flag.
 */
static int64_t trace_ray(const ogrid *g, const double x[3], const double nin[3], obuf *buf,
                         int32_t *vox, double *len, double *t0, int cap, uint8_t *tie) {
    double nn = sqrt(nin[0] * nin[0] + nin[1] * nin[1] + nin[2] * nin[2]);
    double n[3] = {nin[0] / nn, nin[1] / nn, nin[2] / nn};
    double xx = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    double xn = x[0] * n[0] + x[1] * n[1] + x[2] * n[2];
    int nt = 0;
    int is_tie = 0;   /* index list not decided robustly */
    int is_sens = 0;  /* lengths ill-conditioned beyond FP32 rounding */
    double *T = buf->t;
    const double tol = g->tol_t;

    /* chord of the outer sphere, used only to decide which ties matter */
    double Ro = g->rmax;
    double dsc_o = xn * xn - (xx - Ro * Ro);
    double tin = INFINITY, tout = -INFINITY;
    if (dsc_o > 0) {
        tin = -xn - sqrt(dsc_o);
        tout = -xn + sqrt(dsc_o);
    }
#define INSIDE(tt) ((tt) > tin - tol && (tt) < tout + tol)

    /* the start of the ray (l = 0) */
    T[nt++] = 0.0;

    /* spheres: |x + n t|^2 = R^2  ->  t^2 + 2 (x.n) t + (|x|^2 - R^2) = 0 */
    for (int k = 0; k <= g->nr; k++) {
        double R = g->rb[k];
        double r2[2], d, nm;
        int m = quad_roots(1.0, xn, xx - R * R, r2, &d, &nm);
        if (fabs(d) <= 1e-9 * R * R && R > 0 && INSIDE(-xn)) is_tie = 1;
        if (fabs(d) <= 1e-6 * R * R && R > 0 && INSIDE(-xn)) is_sens = 1;
        for (int i = 0; i < m; i++)
            if (r2[i] > 0) T[nt++] = r2[i];
    }

    /* cones: colatitude e_k, c = cos e_k.  (z)^2 = c^2 |p|^2 on the nappe z c >= 0 */
    for (int k = 0; k <= g->ne; k++) {
        double c = cos(g->eb[k]);
        if (fabs(c) >= 1.0) continue; /* polar axis: never crossed */
        if (fabs(c) < 1e-12) {        /* the plane z = 0 */
            if (n[2] != 0) {
                double t = -x[2] / n[2];
                if (t > 0) {
                    T[nt++] = t;
                    if (fabs(n[2]) < 1e-9 && INSIDE(t)) is_tie = 1;
                }
            }
            continue;
        }
        double c2 = c * c;
        double A = n[2] * n[2] - c2;
        double B = x[2] * n[2] - c2 * xn;
        double C = x[2] * x[2] - c2 * xx;
        double rt[2], d, nm;
        int m = quad_roots(A, B, C, rt, &d, &nm);
        if (fabs(d) <= 1e-9 * nm && A != 0) {
            /* near-double root at -B/A: a grazing pair when it lies on this
             * cone's own nappe (a near-planar cone has its two roots on
             * opposite nappes, which is no grazing) */
            double tg = -B / A;
            double zg = x[2] + n[2] * tg;
            int same = 1;
            if (m == 2) {
                double z0 = x[2] + n[2] * rt[0], z1 = x[2] + n[2] * rt[1];
                same = (z0 * c >= 0) && (z1 * c >= 0);
            } else {
                same = zg * c >= 0 || fabs(c) < 1e-6;
            }
            if (same && INSIDE(tg)) is_tie = 1;
        }
        if (fabs(d) <= 1e-6 * nm && A != 0 && INSIDE(-B / A)) is_sens = 1;
        for (int i = 0; i < m; i++) {
            double t = rt[i];
            if (!(t > 0) || !isfinite(t)) continue;
            double pz = x[2] + n[2] * t;
            if (pz * c >= 0) {
                T[nt++] = t;
                if (INSIDE(t)) {
                    double px = x[0] + n[0] * t, py = x[1] + n[1] * t;
                    if (sqrt(px * px + py * py + pz * pz) < tol) is_tie = 1;
                }
            }
        }
    }

    /* azimuth half-planes  {p : p . m_k = 0, p . (cos a_k, sin a_k, 0) > 0} */
    int nplanes = g->cyclic ? g->na : g->na + 1;
    for (int k = 0; k < nplanes; k++) {
        double ca = cos(g->ab[k]), sa = sin(g->ab[k]);
        double xm = -x[0] * sa + x[1] * ca;
        double nm = -n[0] * sa + n[1] * ca;
        if (nm == 0) continue;
        double t = -xm / nm;
        if (!(t > 0)) continue;
        double px = x[0] + n[0] * t, py = x[1] + n[1] * t;
        double side = px * ca + py * sa;
        if (INSIDE(t) && (fabs(nm) < 1e-9 || fabs(side) < tol)) is_tie = 1;
        if (side > 0) T[nt++] = t;
    }

    /* polar-axis crossing when the xy-projection of the ray passes through
     * the origin: azimuth jumps by pi with no half-plane hit */
    double L = x[0] * n[1] - x[1] * n[0];
    double nxy2 = n[0] * n[0] + n[1] * n[1];
    if (L == 0 && nxy2 > 0) {
        double t = -(x[0] * n[0] + x[1] * n[1]) / nxy2;
        if (t > 0) T[nt++] = t;
    }
#undef INSIDE

    qsort(T, (size_t)nt, sizeof(double), cmp_double);

    /* ties: two consecutive breakpoints inside the outer chord that are closer
     * than tol (different surfaces meeting, or a double root) */
    for (int j = 0; j + 1 < nt; j++) {
        double a = T[j], b = T[j + 1];
        if (a > tin - tol && b < tout + tol) {
            if (b - a < tol) is_tie = 1;
            if (b - a < 100.0 * tol) is_sens = 1;
        }
    }

    int64_t nseg = 0;
    int32_t last_v = -1;
    double last_end = -1.0, last_start = 0.0;
    for (int j = 0; j + 1 < nt; j++) {
        double ta = T[j], tb = T[j + 1];
        if (!(tb > ta)) continue;
        double tm = 0.5 * (ta + tb);
        double m[3] = {x[0] + n[0] * tm, x[1] + n[1] * tm, x[2] + n[2] * tm};
        int64_t v = classify_point(g, m);
        if (v < 0) continue;
        if (nseg > 0 && (int32_t)v == last_v && ta == last_end) {
            /* touches the previous segment of the same voxel: merge */
            last_end = tb;
            if (len && nseg - 1 < cap) len[nseg - 1] = last_end - last_start;
            continue;
        }
        if (vox && nseg < cap) {
            vox[nseg] = (int32_t)v;
            len[nseg] = tb - ta;
            if (t0) t0[nseg] = ta;
        }
        last_v = (int32_t)v;
        last_start = ta;
        last_end = tb;
        nseg++;
    }
    if (tie) *tie = (uint8_t)(is_tie | ((is_tie | is_sens) << 1));
    return nseg;
}

static int max_breakpoints(const ogrid *g) {
    return 2 * (g->nr + 1) + 2 * (g->ne + 1) + (g->na + 1) + 4;
}

/* ------------------------------------------------------------------ API -- */

int ora_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the parallel loops that follow (timing runs use 1 and all). */
void ora_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * Cone-beam rays (Sec. 4.2, detector at the cone vertex, Sec. 4.6), pinhole
 * reading: w = unit(look - pos); u = unit(w x up) (up = +X when w is
 * parallel to up); v = u x w; pixel (i, j) of an H x W detector looks along
 * unit(w + sx u + sy v) with sx = (2 (j + 1/2) / W - 1) tan(fov_w / 2),
 * sy = (2 (i + 1/2) / H - 1) tan(fov_h / 2).  Ray id = (view H + i) W + j.
 * fov_deg holds (fov_h, fov_w) per view, full angles in degrees.
 */
/* Frame of one view: w, u, v (see ora_cone_rays). */
static void cone_frame(const double *P, const double *Lk, const double *U, double w[3], double u[3],
                       double vv[3]) {
    w[0] = Lk[0] - P[0]; w[1] = Lk[1] - P[1]; w[2] = Lk[2] - P[2];
    double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    for (int i = 0; i < 3; i++) w[i] /= wn;
    double up3[3] = {U[0], U[1], U[2]};
    if (up3[0] == 0 && up3[1] == 0 && up3[2] == 0) up3[2] = 1.0;
    u[0] = w[1] * up3[2] - w[2] * up3[1];
    u[1] = w[2] * up3[0] - w[0] * up3[2];
    u[2] = w[0] * up3[1] - w[1] * up3[0];
    double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (un < 1e-12) {
        up3[0] = 1; up3[1] = 0; up3[2] = 0;
        u[0] = w[1] * up3[2] - w[2] * up3[1];
        u[1] = w[2] * up3[0] - w[0] * up3[2];
        u[2] = w[0] * up3[1] - w[1] * up3[0];
        un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    }
    for (int i = 0; i < 3; i++) u[i] /= un;
    vv[0] = u[1] * w[2] - u[2] * w[1];
    vv[1] = u[2] * w[0] - u[0] * w[2];
    vv[2] = u[0] * w[1] - u[1] * w[0];
}

/* Unit direction of pixel (i, j) of an H x W detector. */
static void cone_dir(const double w[3], const double u[3], const double vv[3], double th, double tw,
                     int i, int j, int H, int W, double d[3]) {
    double sy = (2.0 * (i + 0.5) / H - 1.0) * th;
    double sx = (2.0 * (j + 0.5) / W - 1.0) * tw;
    for (int k = 0; k < 3; k++) d[k] = w[k] + sx * u[k] + sy * vv[k];
    double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int k = 0; k < 3; k++) d[k] /= dn;
}

/*
 * Cone-beam rays (Sec. 4.2, detector at the cone vertex, Sec. 4.6), pinhole
 * reading: w = unit(look - pos); u = unit(w x up) (up = +Z when all zero,
 * +X when w is parallel to up); v = u x w; pixel (i, j) of an H x W detector
 * looks along unit(w + sx u + sy v) with sx = (2 (j + 1/2) / W - 1)
 * tan(fov_w / 2), sy = (2 (i + 1/2) / H - 1) tan(fov_h / 2).
 * Ray id = (view H + i) W + j.  fov_deg holds (fov_h, fov_w) per view, full
 * angles in degrees.
 */
void ora_cone_rays(int nv, const double *pos, const double *look, const double *up,
                   const double *fov_deg, int H, int W, double *starts, double *dirs) {
    for (int v = 0; v < nv; v++) {
        double w[3], u[3], vv[3];
        cone_frame(pos + 3 * v, look + 3 * v, up + 3 * v, w, u, vv);
        double th = tan(fov_deg[2 * v + 0] * M_PI / 360.0);
        double tw = tan(fov_deg[2 * v + 1] * M_PI / 360.0);
        for (int i = 0; i < H; i++)
            for (int j = 0; j < W; j++) {
                int64_t id = ((int64_t)v * H + i) * W + j;
                double d[3];
                cone_dir(w, u, vv, th, tw, i, j, H, W, d);
                for (int k = 0; k < 3; k++) {
                    starts[3 * id + k] = pos[3 * v + k];
                    dirs[3 * id + k] = d[k];
                }
            }
    }
}

/* The rays with the given ids only (same convention as ora_cone_rays). */
void ora_cone_ray_ids(int nv, const double *pos, const double *look, const double *up,
                      const double *fov_deg, int H, int W, const int64_t *ids, int64_t n,
                      double *starts, double *dirs) {
    for (int64_t q = 0; q < n; q++) {
        int64_t id = ids[q];
        int v = (int)(id / ((int64_t)H * W));
        int rem = (int)(id % ((int64_t)H * W));
        double w[3], u[3], vv[3], d[3];
        cone_frame(pos + 3 * v, look + 3 * v, up + 3 * v, w, u, vv);
        cone_dir(w, u, vv, tan(fov_deg[2 * v] * M_PI / 360.0),
                 tan(fov_deg[2 * v + 1] * M_PI / 360.0), rem / W, rem % W, H, W, d);
        for (int k = 0; k < 3; k++) {
            starts[3 * q + k] = pos[3 * v + k];
            dirs[3 * q + k] = d[k];
        }
    }
}

/* Per-ray canonical segment counts and tie flags. */
int ora_count(const double *rb, int nr, const double *eb, int ne, const double *ab, int na,
              const double *starts, const double *dirs, int64_t nrays, int32_t *counts,
              uint8_t *ties) {
    ogrid g;
    ogrid_init(&g, rb, nr, eb, ne, ab, na);
    int kmax = max_breakpoints(&g);
    int err = 0;
#pragma omp parallel
    {
        obuf b;
        b.cap = kmax;
        b.t = (double *)malloc(sizeof(double) * (size_t)kmax);
        if (!b.t) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 256)
            for (int64_t i = 0; i < nrays; i++) {
                uint8_t tie = 0;
                counts[i] = (int32_t)trace_ray(&g, starts + 3 * i, dirs + 3 * i, &b, NULL, NULL,
                                               NULL, 0, &tie);
                if (ties) ties[i] = tie;
            }
            free(b.t);
        }
    }
    return err;
}

/* Canonical segments of every ray at row_ptr[i] .. row_ptr[i+1]. */
int ora_fill(const double *rb, int nr, const double *eb, int ne, const double *ab, int na,
             const double *starts, const double *dirs, int64_t nrays, const int64_t *row_ptr,
             int32_t *vox, double *len, double *t0) {
    ogrid g;
    ogrid_init(&g, rb, nr, eb, ne, ab, na);
    int kmax = max_breakpoints(&g);
    int err = 0;
#pragma omp parallel
    {
        obuf b;
        b.cap = kmax;
        b.t = (double *)malloc(sizeof(double) * (size_t)kmax);
        if (!b.t) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 256)
            for (int64_t i = 0; i < nrays; i++) {
                int64_t o = row_ptr[i];
                int cap = (int)(row_ptr[i + 1] - o);
                int64_t m = trace_ray(&g, starts + 3 * i, dirs + 3 * i, &b, vox + o, len + o,
                                      t0 ? t0 + o : NULL, cap, NULL);
                if (m != cap) {
#pragma omp atomic write
                    err = 2;
                }
            }
            free(b.t);
        }
    }
    return err;
}

/* y[b, i] = sum over row i of len * rho[b, vox]   (Eq. 5), FP64. */
void ora_forward(const int64_t *row_ptr, const int32_t *vox, const double *len, int64_t nrays,
                 const double *rho, int B, int64_t V, double *y) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nrays; i++) {
        for (int b = 0; b < B; b++) {
            double s = 0;
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; k++) s += len[k] * rho[b * V + vox[k]];
            y[b * nrays + i] = s;
        }
    }
}

/* x[b, v] = sum over all segments of voxel v of len * y[b, ray]   (adjoint). */
void ora_adjoint(const int64_t *row_ptr, const int32_t *vox, const double *len, int64_t nrays,
                 const double *y, int B, int64_t V, double *x) {
    memset(x, 0, sizeof(double) * (size_t)B * (size_t)V);
    for (int64_t i = 0; i < nrays; i++)
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; k++)
            for (int b = 0; b < B; b++) x[b * V + vox[k]] += len[k] * y[b * nrays + i];
}

/* Fused trace + forward without storing segments (for bounded CPU timing of
 * large workloads); same arithmetic as ora_fill followed by ora_forward. */
int ora_project(const double *rb, int nr, const double *eb, int ne, const double *ab, int na,
                const double *starts, const double *dirs, int64_t nrays, const double *rho, int B,
                double *y, int64_t *nseg_total) {
    ogrid g;
    ogrid_init(&g, rb, nr, eb, ne, ab, na);
    int kmax = max_breakpoints(&g);
    int64_t V = (int64_t)nr * ne * na;
    int64_t total = 0;
    int err = 0;
#pragma omp parallel reduction(+ : total)
    {
        obuf b;
        b.cap = kmax;
        b.t = (double *)malloc(sizeof(double) * (size_t)kmax);
        int32_t *sv = (int32_t *)malloc(sizeof(int32_t) * (size_t)kmax);
        double *sl = (double *)malloc(sizeof(double) * (size_t)kmax);
        if (!b.t || !sv || !sl) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 256)
            for (int64_t i = 0; i < nrays; i++) {
                int64_t m = trace_ray(&g, starts + 3 * i, dirs + 3 * i, &b, sv, sl, NULL, kmax,
                                      NULL);
                total += m;
                for (int bb = 0; bb < B; bb++) {
                    double s = 0;
                    for (int64_t k = 0; k < m; k++) s += sl[k] * rho[bb * V + sv[k]];
                    y[bb * nrays + i] = s;
                }
            }
        }
        free(b.t);
        free(sv);
        free(sl);
    }
    if (nseg_total) *nseg_total = total;
    return err;
}

/*
 * Gradient of the data term ||F rho - y||^2 (Sec. 4.5, Eq. 6) at selected
 * voxels, g_v = 2 sum_i (F rho - y)_i |ray_i inside v|, for a stack of cone
 * views, without storing segment lists.  Rays are generated on the fly; a ray
 * is traced only if it passes within the bounding sphere (bsph: centre xyz,
 * radius per target) of some target voxel, which cannot change the result.
 * bound_v = 2 sum_i (sum_k |rho_k| len_k + |y_i|) |ray_i inside v| scales the
 * rounding error of an FP32 evaluation.  Returns 0 on success.
 */
int ora_cone_data_grad(const double *rb, int nr, const double *eb, int ne, const double *ab, int na,
                       int nv, const double *pos, const double *look, const double *up,
                       const double *fov_deg, int H, int W, const double *rho, const double *y,
                       int nt, const int64_t *targets, const double *bsph, double *grad,
                       double *bound, int64_t *n_traced) {
    ogrid g;
    ogrid_init(&g, rb, nr, eb, ne, ab, na);
    int kmax = max_breakpoints(&g);
    int err = 0;
    int64_t traced = 0;
    int64_t R = (int64_t)nv * H * W;
    for (int k = 0; k < nt; k++) grad[k] = bound[k] = 0.0;
#pragma omp parallel reduction(+ : traced)
    {
        obuf b;
        b.cap = kmax;
        b.t = (double *)malloc(sizeof(double) * (size_t)kmax);
        int32_t *sv = (int32_t *)malloc(sizeof(int32_t) * (size_t)kmax);
        double *sl = (double *)malloc(sizeof(double) * (size_t)kmax);
        double *gl = (double *)calloc((size_t)nt, sizeof(double));
        double *bl = (double *)calloc((size_t)nt, sizeof(double));
        if (!b.t || !sv || !sl || !gl || !bl) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 4096)
            for (int64_t id = 0; id < R; id++) {
                int v = (int)(id / ((int64_t)H * W));
                int rem = (int)(id % ((int64_t)H * W));
                int i = rem / W, j = rem % W;
                double w[3], u[3], vv[3], d[3];
                cone_frame(pos + 3 * v, look + 3 * v, up + 3 * v, w, u, vv);
                cone_dir(w, u, vv, tan(fov_deg[2 * v] * M_PI / 360.0),
                         tan(fov_deg[2 * v + 1] * M_PI / 360.0), i, j, H, W, d);
                const double *x = pos + 3 * v;
                int near = 0;
                for (int k = 0; k < nt && !near; k++) {
                    const double *c = bsph + 4 * k;
                    double cx = c[0] - x[0], cy = c[1] - x[1], cz = c[2] - x[2];
                    double tt = cx * d[0] + cy * d[1] + cz * d[2];
                    if (tt < 0) tt = 0;
                    double qx = cx - tt * d[0], qy = cy - tt * d[1], qz = cz - tt * d[2];
                    if (qx * qx + qy * qy + qz * qz <= c[3] * c[3]) near = 1;
                }
                if (!near) continue;
                traced++;
                int64_t m = trace_ray(&g, x, d, &b, sv, sl, NULL, kmax, NULL);
                double f = 0, a = 0;
                for (int64_t q = 0; q < m; q++) {
                    f += sl[q] * rho[sv[q]];
                    a += sl[q] * fabs(rho[sv[q]]);
                }
                double r = f - y[id];
                for (int64_t q = 0; q < m; q++)
                    for (int k = 0; k < nt; k++)
                        if (targets[k] == sv[q]) {
                            gl[k] += 2.0 * r * sl[q];
                            bl[k] += 2.0 * (a + fabs(y[id])) * sl[q];
                        }
            }
#pragma omp critical
            for (int k = 0; k < nt; k++) {
                grad[k] += gl[k];
                bound[k] += bl[k];
            }
        }
        free(b.t);
        free(sv);
        free(sl);
        free(gl);
        free(bl);
    }
    if (n_traced) *n_traced = traced;
    return err;
}
