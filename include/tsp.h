/*
 * tsp.h -- spherical-grid tomographic projector for MI355X (gfx950), C ABI.
 *
 * The library computes the line-integral projector of TomoSphero
 * (Sec. 2.1, Eqs. 1-5): for every detector ray x + n l, l >= 0,
 *
 *     y = F rho = sum_i rho[r_i, e_i, a_i] * dl_i                 (Eq. 5)
 *
 * over the voxels of a spherical grid (Sec. 2.2) that the ray crosses, and
 * its adjoint x = F^T y.  Per ray the HIP kernels intersect the ray with the
 * radial spheres, the colatitude cones and the azimuth half-planes
 * (Sec. 3.1), turn each crossing into a region index by its direction
 * (Sec. 3.2, Eqs. 11-13), merge the three ordered crossing streams and take
 * lengths between consecutive crossings (Sec. 3.3, Table 2), and gather-sum
 * the object (Sec. 3.4).  Steps 1-3 can be precomputed once per geometry and
 * stored (Sec. 3, Sec. 4.4): TSP_MODE_CSR stores the segment lists on the
 * device; TSP_MODE_ONTHEFLY recomputes them inside every forward/adjoint
 * launch so that nothing proportional to the number of segments is stored.
 *
 * Conventions
 *   - Grid: boundaries r_b[nr+1] (radii, strictly increasing, r_b[0] >= 0),
 *     e_b[ne+1] (colatitude from +Z in radians, strictly increasing within
 *     [0, pi]), a_b[na+1] (azimuth counter-clockwise about +Z from +X,
 *     strictly increasing, a_b[na] - a_b[0] <= 2 pi; the grid is cyclic in
 *     azimuth when the span is 2 pi within 1e-12).  The grid may be a wedge
 *     (Sec. 2.2, Fig. 3-4); the object is zero outside it (Sec. 4.6).
 *   - Voxel (ir, ie, ia) has linear index v = (ir*ne + ie)*na + ia; objects
 *     are float32 arrays [batch][nr][ne][na] (row-major, contiguous).
 *   - Rays: cone-beam views (Sec. 4.2, detector at the cone vertex, Sec. 4.6)
 *     or explicit rays (Sec. 4.2, Listing 4).  Cone view v with detector
 *     shape (H, W): w = unit(look - pos), u = unit(w x up) (up = +X if w is
 *     parallel to up), v = u x w; pixel (i, j) looks along
 *     unit(w + sx u + sy v), sx = (2 (j + 1/2)/W - 1) tan(fov_w/2),
 *     sy = (2 (i + 1/2)/H - 1) tan(fov_h/2).  Ray id = (view*H + i)*W + j.
 *     Measurements are float32 arrays [batch][n_rays].
 *   - Cone views must sit outside the outermost sphere (Sec. 4.6).  Explicit
 *     rays may start anywhere, inside the grid too: a ray integrates over
 *     l >= 0 from its start (Eq. 3), as the sunward rays from voxel
 *     centroids of Sec. 9.3 need.
 *
 * Ownership and streams
 *   - A geometry owns every device buffer it allocates (tables, view frames,
 *     explicit rays, segment stores).  The caller owns rho, y and x: plain
 *     contiguous device pointers (e.g. from PyTorch).  Outputs are
 *     overwritten, never accumulated into.
 *   - All device work is enqueued on the HIP stream passed as `stream`
 *     (hipStream_t; NULL = the legacy default stream).  Calls return once
 *     the work is enqueued, except tsp_trace, which synchronises `stream`
 *     to learn the segment count it must allocate.
 *   - After tsp_trace a geometry is immutable: tsp_forward and
 *     tsp_backproject may run concurrently on different streams.  Calls
 *     that mutate a geometry (tsp_trace, tsp_geometry_destroy) must not
 *     overlap other calls on it.
 *
 * Errors
 *   Every call returns a tsp_status; no C++ exception crosses the ABI.  On
 *   failure tsp_last_error() returns a message for the calling thread.
 *   Arguments are validated on the host before any launch.
 *
 * Launch grids
 *   One dispatch holds fewer than 2^32 work-items.  Kernels whose items can
 *   outnumber that near the size limits (4 V staged values, 64 lanes per
 *   voxel, B V elements) stride over grids of at most 2^23 workgroups; the
 *   environment variable TSP_MAX_BLOCKS (read once per process) lowers that
 *   cap, for tests of the striding.
 */
#ifndef TSP_H
#define TSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tsp_status {
    TSP_OK = 0,
    TSP_E_INVALID = 1,     /* bad argument (shape, boundaries, ray inside the grid, NULL) */
    TSP_E_NOMEM = 2,       /* device allocation failed or exceeds TSP_MAX_DEVICE_BYTES */
    TSP_E_HIP = 3,         /* a HIP runtime call failed (message carries the HIP error) */
    TSP_E_STATE = 4,       /* call not valid in the geometry's state (e.g. forward before trace) */
    TSP_E_UNSUPPORTED = 5  /* combination not implemented (e.g. object frames on explicit rays) */
} tsp_status;

/* tsp_trace modes */
#define TSP_MODE_CSR 1        /* precompute and store segment lists (Sec. 3, Sec. 4.4) */
#define TSP_MODE_ONTHEFLY 2   /* store nothing; recompute per launch */
#define TSP_TRACE_NO_CSC 0x10 /* CSR mode only: skip the voxel-major (transposed) store */

/* tsp_backproject methods */
#define TSP_ADJ_DETERMINISTIC 1 /* voxel-major store, fixed summation order, bitwise reproducible */
#define TSP_ADJ_ATOMIC 2        /* ray-major scatter with float atomics (order varies run to run) */
#define TSP_ADJ_FIXEDPOINT 3    /* traced on the fly, sums in 64-bit fixed point, bitwise reproducible */

/* Grid boundaries (Sec. 2.2, Sec. 4.1).  Host pointers, read during
 * tsp_geometry_create only. */
typedef struct tsp_grid_desc {
    int32_t nr, ne, na;
    const double *r_b; /* nr + 1 radii */
    const double *e_b; /* ne + 1 colatitudes, radians */
    const double *a_b; /* na + 1 azimuths, radians */
} tsp_grid_desc;

/* One cone-beam view (Sec. 4.2, ConeRectGeom; Sec. 4.3 stacks views). */
typedef struct tsp_cone_view {
    double pos[3];     /* detector (= cone vertex) position, outside the grid */
    double look[3];    /* point on the optical axis (the origin in the paper's examples) */
    double up[3];      /* up hint; all zero means +Z */
    double fov_deg[2]; /* full field of view along rows (H) and columns (W), degrees, in (0, 180) */
    int32_t shape[2];  /* detector (H, W); equal for every view of a geometry (Sec. 4.6) */
} tsp_cone_view;

/*
 * A view of either kind (Sec. 4.2, Listings 2-3; Sec. 4.3 stacks views of
 * any kinds with one detector shape).  Frame: w = unit(look - pos),
 * u = unit(w x up) (up = +Z when all zero, +X when w is parallel to up),
 * v = u x w; pixel (i, j) has sx = 2 (j + 1/2) / W - 1 and
 * sy = 2 (i + 1/2) / H - 1, both in (-1, 1).
 *   TSP_VIEW_CONE: as tsp_cone_view, extent = full fields of view in
 *     degrees (rows, columns), in (0, 180); the ray starts at pos and looks
 *     along unit(w + sx tan(extent[1]/2) u + sy tan(extent[0]/2) v).
 *   TSP_VIEW_PARALLEL (ParallelGeom): extent = detector height and width in
 *     grid units, > 0; the ray starts at pos + sx extent[1]/2 u +
 *     sy extent[0]/2 v and looks along w.  The detector rectangle must lie
 *     outside the outer sphere.
 */
#define TSP_VIEW_CONE 0
#define TSP_VIEW_PARALLEL 1
typedef struct tsp_view {
    int32_t kind;      /* TSP_VIEW_CONE or TSP_VIEW_PARALLEL */
    int32_t shape[2];  /* detector (H, W); equal for every view of a geometry */
    int32_t reserved;
    double pos[3];     /* cone vertex / detector centre, outside the grid */
    double look[3];    /* point on the optical axis */
    double up[3];      /* up hint; all zero means +Z */
    double extent[2];  /* cone: full FOV degrees (rows, cols); parallel: size (rows, cols) */
} tsp_view;

/* Sizes and state of a geometry. */
typedef struct tsp_info {
    int64_t n_rays;       /* R */
    int64_t n_voxels;     /* V = nr*ne*na */
    int64_t n_segments;   /* S: valid canonical segments over all rays (after tsp_trace) */
    int64_t n_stored;     /* segment slots stored in the ray-major store, padding included */
    int64_t max_per_ray;  /* longest segment list of any ray */
    int64_t device_bytes; /* device memory currently owned by the geometry */
    int32_t mode;         /* 0 before tsp_trace, else TSP_MODE_CSR or TSP_MODE_ONTHEFLY */
    int32_t has_csc;      /* voxel-major store present */
    int32_t n_obj_frames; /* F: object frames (1 for a static object) */
    int32_t reserved;
} tsp_info;

typedef struct tsp_geometry tsp_geometry;

/*
 * Create a geometry from a grid and EITHER n_views cone views (views != NULL,
 * ray_starts == ray_dirs == NULL) OR n_rays explicit rays (views == NULL;
 * ray_starts, ray_dirs: host float64 arrays [n_rays][3]; directions of any
 * non-zero length, normalised by the library; Sec. 4.2 Listing 4).
 * Validates the grid (finite, strictly increasing, ranges above), the views
 * (finite, pos outside the outer sphere, fov in (0, 180), equal shapes, pos
 * != look) and the rays (finite, non-zero direction: TSP_E_INVALID
 * otherwise).  Limits (TSP_E_INVALID beyond them):
 * fewer than 2^31 voxels and 2^31 rays (after padding cone views to 16x16
 * pixel windows), and nr + ne + 3 na <= 5627 (the boundary tables are staged
 * in workgroup-shared memory).  Uploads boundary tables and per-view
 * frames to the current HIP device.  *out receives the new geometry, owned
 * by the caller and released with tsp_geometry_destroy.
 */
tsp_status tsp_geometry_create(const tsp_grid_desc *grid, const tsp_cone_view *views,
                               int32_t n_views, const double *ray_starts, const double *ray_dirs,
                               int64_t n_rays, tsp_geometry **out);

/*
 * As tsp_geometry_create for views of any kinds (tsp_view).  Errors as
 * there, plus TSP_E_INVALID for an unknown kind, a non-positive parallel
 * size, or a parallel detector that reaches into the outer sphere.
 */
tsp_status tsp_geometry_create_views(const tsp_grid_desc *grid, const tsp_view *views,
                                     int32_t n_views, tsp_geometry **out);

/*
 * Dynamic objects (Sec. 4.4: the operator applies to a 3-D or a 4-D object;
 * Sec. 4.6: the grid stays the same for every frame).  Assigns object frame
 * frame_of_view[v] to view v (cone or parallel).  Afterwards tsp_forward reads rho as
 * [batch][n_frames][V]; every ray of view v integrates frame
 * frame_of_view[v].  tsp_backproject writes x in the same layout, and frame f
 * receives only the rays of the views assigned to it (zero if none).
 * frame_of_view: host int32 [n_views], each in [0, n_frames), read during
 * the call.  Must precede tsp_trace, because the voxel-major store is keyed
 * by frame; calling it again replaces the assignment.  Without this call a
 * geometry has one frame.
 * Errors: TSP_E_INVALID (NULL, n_frames < 1, a frame index out of range,
 * n_frames * V >= 2^31), TSP_E_STATE after tsp_trace, TSP_E_UNSUPPORTED for
 * a geometry of explicit rays.
 */
tsp_status tsp_set_object_frames(tsp_geometry *g, const int32_t *frame_of_view,
                                 int32_t n_frames);

/*
 * Precompute steps 1-3 (Sec. 3.1-3.3) for every ray.
 *   TSP_MODE_CSR: counts segments per ray, then stores the canonical segment
 *     lists in a ray-major store (a float32 length and a one-byte voxel step
 *     per segment, about 5 bytes), and unless TSP_TRACE_NO_CSC is set also
 *     a voxel-major (transposed) store for the deterministic adjoint (a
 *     float32 length and a one-byte slot increase per segment, plus escapes
 *     and padding: about 5.1 bytes).  The transposed store is built by
 *     sorting in passes whose temporary space (about 25 bytes per segment of
 *     a pass) fits the free device memory; the environment variable
 *     TSP_TRANSPOSE_MAX_ENTRIES caps the segments of one pass.  With more
 *     than one pass the segments are sorted twice (once to size the store,
 *     once to fill it).  TSP_E_NOMEM when the stores themselves exceed
 *     the device or the cap in the environment variable TSP_MAX_DEVICE_BYTES
 *     (the caller may then retry with TSP_MODE_ONTHEFLY).
 *   TSP_MODE_ONTHEFLY: only counts segments (for tsp_query) and stores no
 *     lists.
 * May be called again to switch modes; previous stores are released.
 * Synchronises `stream`.
 */
tsp_status tsp_trace(tsp_geometry *g, int32_t mode, void *stream);

/*
 * y[b][i] = sum over ray i's segments of len * rho[b][f][vox]   (Eq. 5)
 * where f is the object frame of ray i's view (0 for a static object).
 * rho: device float32 [batch][F][V] (F = n_obj_frames, usually 1);
 * y: device float32 [batch][R], overwritten.
 * batch >= 1.  TSP_E_STATE before tsp_trace.
 */
tsp_status tsp_forward(const tsp_geometry *g, const float *rho, int32_t batch, float *y,
                       void *stream);

/*
 * Adjoint (Sec. 4.4: the operator is differentiable, so reconstruction can
 * take gradients through it; F is linear, and the gradient of <g, F rho>
 * with respect to rho is F^T g, the adjoint of Eq. 5):
 * x[b][f][v] = sum over all segments in voxel v of rays of views in
 * object frame f of len * y[b][ray].
 * y: device float32 [batch][R]; x: device float32 [batch][F][V], overwritten.
 * method TSP_ADJ_DETERMINISTIC (bitwise reproducible), TSP_ADJ_ATOMIC or
 * TSP_ADJ_FIXEDPOINT (below).  The deterministic adjoint reads the transposed store when the geometry was
 * traced in CSR mode with it.  Otherwise (on the fly, or TSP_TRACE_NO_CSC) it
 * is traced within the call: the views (explicit rays: runs of whole 256-ray
 * windows) are cut into ceil(S / C) chunks of about equal segment counts
 * (C = 2^30 segments or the environment variable TSP_CHUNK_SEGMENTS; a cut
 * follows the first view or window at which the running count reaches a
 * multiple of S / chunks); each chunk is traced into stores of its own,
 * transposed, and its adjoint added into x in chunk order.  That costs about
 * a full CSR trace per call and synchronises `stream`.  The first such call
 * allocates the chunks' working memory (about 55 bytes per segment of the
 * largest chunk; TSP_E_NOMEM if it does not fit), which the geometry keeps
 * for later calls until tsp_trace or tsp_geometry_destroy; calls of this
 * kind on one geometry are serialised.  Bitwise reproducible for a given
 * geometry and C; with one chunk it equals the stored deterministic adjoint
 * bit for bit.
 * method TSP_ADJ_FIXEDPOINT (any traced geometry, stored lists or not): the
 * rays are traced within the call, as on the fly, and each term len * y is
 * rounded to an integer multiple of 2^q_b and added in 64-bit integers, so
 * that the sums do not depend on the order of addition: bitwise reproducible
 * without transposed lists or chunking, and one pass.  q_b = ilogb(M_b) + 1
 * - 62 with M_b = max |y_b| * 4 * R * r_out (R rays, r_out the outer radius),
 * which bounds every voxel's sum of |terms| by half of M_b, so no partial sum
 * overflows; a term's rounding error is at most 2^(q_b - 1), about 1e-19 M_b.
 * The result is the exact sum of the rounded terms, converted to float once;
 * it differs from TSP_ADJ_DETERMINISTIC's float sums in the last bits.
 * Allocates 8 * V * (1 or 4) bytes stream-ordered (TSP_E_NOMEM otherwise).
 */
tsp_status tsp_backproject(const tsp_geometry *g, const float *y, int32_t batch, float *x,
                           int32_t method, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * deterministic adjoint of tsp_backproject (TSP_ADJ_DETERMINISTIC, same
 * kernels, bit-identical result) with no allocation of any kind.  The
 * slot-ordered copy of y that tsp_backproject keeps in a stream-ordered
 * temporary lives here in a fixed device array of
 * TSP_NOALLOC_SCRATCH_BYTES, held by every device the library runs on
 * until the process ends (its address is looked up on the first call on a
 * device).  It needs n_stored_slots * 4 * min(batch rounded up to 2 or 4,
 * 4) bytes, where the slots are the rays padded to whole 16 x 16 pixel
 * windows: for example 1966080 slots (30 views of 256 x 256) fit up to
 * batch 4, 26214400 slots (100 views of 512 x 512) batch 1.
 * Arguments, layouts and ownership as tsp_backproject; batches above 4 are
 * taken in groups of four through the same array.
 * Every call on a device shares that device's array, so calls that overlap
 * on one device (different streams, threads) race and must be serialised by
 * the caller; nothing carries over from one call to the next.
 * Errors: TSP_E_INVALID (NULL, batch < 1), TSP_E_STATE (before tsp_trace,
 * or without the voxel-major store: on the fly or TSP_TRACE_NO_CSC),
 * TSP_E_NOMEM when the copy of y exceeds TSP_NOALLOC_SCRATCH_BYTES (use
 * tsp_backproject), TSP_E_HIP.
 */
#define TSP_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
tsp_status tsp_backproject_noalloc(const tsp_geometry *g, const float *y, int32_t batch,
                                   float *x, void *stream);

/*
 * Attenuated emission model (Sec. 9.3, Eqs. 14-18).
 *
 * Sunward geometry: one explicit ray per voxel v, starting at v's centroid
 * (mid-boundaries r_c, theta_c, phi_c of the voxel's boundaries) and running
 * along sun_dir (host double[3], finite and non-zero; normalised).  Ray v
 * belongs to voxel v, so the projection of an object along these rays is the
 * optical depth towards the Sun of every voxel (Eq. 17's F_1).  The result is
 * an ordinary explicit-ray geometry (released with tsp_geometry_destroy) to
 * be traced with tsp_trace before use; with the transposed store its adjoint
 * in tsp_atten_backward is deterministic, otherwise atomic.  Errors as for
 * tsp_geometry_create.
 */
tsp_status tsp_geometry_create_sunward(const tsp_grid_desc *grid, const double *sun_dir,
                                       tsp_geometry **out);

/*
 * Attenuated forward for batch objects (Eq. 17):
 *   s = sigma * rho, tau1 = F_sun s, w = exp(-tau1) * rho,
 *   y[b][i] = sum_k w[b][v_k] exp(-T_k) len_k,  T_k = sum_{j <= k} s[b][v_j] len_j,
 * over ray i's segments in order of distance from the detector (Eq. 18: the
 * sum includes segment k itself).  The constant g phi / 4 pi of Eq. 16 is the
 * caller's.
 * g: line-of-sight geometry traced in TSP_MODE_CSR, one object frame;
 * g_sun: traced geometry from tsp_geometry_create_sunward on the same grid.
 * rho: device float32 [batch][V]; sigma: device float32 [V], shared by the
 * batch; y: device float32 [batch][R], overwritten; tau1: device float32
 * [batch][V] receiving the sunward optical depths (keep them for
 * tsp_atten_backward), or NULL.  Temporaries (3 floats per voxel and
 * object) are stream-ordered allocations on `stream`.
 * Errors: TSP_E_INVALID (NULL, batch < 1, g_sun not one ray per voxel of
 * g's grid), TSP_E_STATE before tsp_trace, TSP_E_UNSUPPORTED (g on the fly or
 * with object frames), TSP_E_HIP.
 */
tsp_status tsp_atten_forward(const tsp_geometry *g, const tsp_geometry *g_sun, const float *rho,
                             const float *sigma, int32_t batch, float *y, float *tau1,
                             void *stream);

/*
 * Gradient of sum_b <gy[b], y[b]> with respect to rho for the attenuated
 * forward (Sec. 9.3, Eqs. 17-18 differentiated): through w (exp(-tau1) gw),
 * through T along each line of sight, and through tau1 (F_sun^T of -w gw).
 * method:
 *   TSP_ADJ_ATOMIC: the line-of-sight terms are scattered with float atomic
 *     adds (merged per voxel across a wavefront first); the summation order,
 *     and so the last bits, vary from run to run.
 *   TSP_ADJ_DETERMINISTIC: the same merged terms are rounded to integer
 *     multiples of 2^q and added as 64-bit integers (integer atomics), with
 *     q = ilogb(M) + 1 - 62 from M = 2 max|gy| R 2 r_out (1 + 2 r_out
 *     max|rho|), which bounds twice any voxel's sum of |terms|: no partial
 *     sum overflows, every order of addition gives the same sum, and the
 *     result is bitwise reproducible (each term's rounding is at most 2^-63
 *     of M); F_sun^T uses the sunward geometry's
 *     deterministic adjoint, which must have its voxel-major store
 *     (TSP_E_STATE otherwise).
 * rho, sigma as for tsp_atten_forward; tau1: [batch][V] from
 * tsp_atten_forward of the same rho; gy: device float32 [batch][R];
 * grad: device float32 [batch][V], overwritten.  Temporaries: 6 floats per
 * voxel and object (and 48 bytes per voxel for the deterministic sums),
 * stream-ordered.  Errors as for tsp_atten_forward, and TSP_E_INVALID for an
 * unknown method.
 */
tsp_status tsp_atten_backward(const tsp_geometry *g, const tsp_geometry *g_sun, const float *rho,
                              const float *sigma, const float *tau1, const float *gy,
                              int32_t batch, float *grad, int32_t method, void *stream);

/*
 * Export the canonical segment lists (the region index and length arrays of
 * Sec. 4.4, ".regs"/".lens") in ray-major CSR form into caller device
 * buffers: row_ptr int64 [R+1], vox int32 [S], len float32 [S]; ray i owns
 * entries row_ptr[i] .. row_ptr[i+1]-1 in increasing distance.  Any of
 * vox/len may be NULL.  CSR mode only (TSP_E_STATE otherwise).
 */
tsp_status tsp_segments(const tsp_geometry *g, int64_t *row_ptr, int32_t *vox, float *len,
                        void *stream);

/* Write the rays the geometry traces (start, unit direction), device
 * float64 [R][3] each; either pointer may be NULL. */
tsp_status tsp_rays(const tsp_geometry *g, double *starts, double *dirs, void *stream);

/*
 * Measurement hook (not part of the method): the next tsp_forward or
 * tsp_backproject call on g records `start` on its stream just before the
 * operation's main kernel and `stop` just after it, so that the caller's
 * hipEventElapsedTime(start, stop) is that kernel's own duration, without
 * the call's other launches.  The main kernel is the gather-sum of the
 * stored forward (Sec. 3.4) and the voxel-major sum of the deterministic
 * adjoint (the slot-ordered copy of y before it is left out); for batches
 * above four, from the first group's main kernel to the end of the last's.
 * On every other path (on the fly, atomic, fixed point, the adjoint traced
 * in chunks) the events bracket the whole operation.  One-shot: the call
 * that records them clears the setting; start = stop = NULL clears it too.
 * The events are hipEvent_t handles created by the caller on g's device
 * (with timing, i.e. without hipEventDisableTiming) and stay the caller's.
 * Setting events and calling from several threads at once on one geometry
 * leaves it open which call records them.
 * Errors: TSP_E_INVALID (g NULL, exactly one of start and stop NULL); a
 * failed record makes the forward or adjoint call return TSP_E_HIP.
 */
tsp_status tsp_set_timing_events(tsp_geometry *g, void *start, void *stop);

/* Sizes and state; valid at any time after creation. */
tsp_status tsp_query(const tsp_geometry *g, tsp_info *info);

/* Release the geometry and all its device memory (NULL is a no-op). Waits
 * for work already enqueued on the device to finish first. */
void tsp_geometry_destroy(tsp_geometry *g);

/* Message describing the last failure on the calling thread ("" if none). */
const char *tsp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TSP_H */
